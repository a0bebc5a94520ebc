// Closed-form PSD projections of the Hessians of two isotropic energies of
// the incremental potential (Eq. (3)), both over vec of a 3x3 matrix M and
// both built on a signed SVD M = U diag(s) V^T (U, V proper rotations, s3 < 0
// for an inverted M).  For an energy Psi(s) of the singular values alone the
// nine eigenpairs are known (the isotropic-energy eigensystems of Smith,
// de Goes and Kim, 2019): for each pair (p, q) with third index k, the
// matrices U (e_p e_q^T -+ e_q e_p^T) V^T / sqrt 2 carry the twist ("-")
// eigenvalue (Psi_p + Psi_q) / (s_p + s_q) and the flip ("+") eigenvalue
// (Psi_p - Psi_q) / (s_p - s_q), Psi_p = dPsi/ds_p, and U diag(a) V^T carries
// the eigenvectors a of the 3x3 block d2Psi/ds2.
//
//  * Stable Neo-Hookean, rest-stable form with lh = lambda + mu (Sec. III-C.1):
//      Psi(F) = mu/2 (|F|^2 - 3) - mu (J - 1) + lh/2 (J - 1)^2,   J = det F;
//    with sc = lh (J - 1) - mu: twist mu + sc s_k, flip mu - sc s_k, block
//    A_pp = mu + lh g_p^2, A_pq = lh g_p g_q + sc s_k, g_p = s_q s_k.
//  * Affine-body orthogonality (Sec. III-C.2), kv |A A^T - I|^2 =
//    kv sum_k (s_k^2 - 1)^2: twist 4 kv (s_p^2 - s_p s_q + s_q^2 - 1), flip
//    4 kv (s_p^2 + s_p s_q + s_q^2 - 1), block diagonal kv (12 s_k^2 - 4).
//
// A projection keeps the Hessian as formed and subtracts lambda q q^T for
// every negative eigenpair, so a matrix with no negative mode keeps its
// Hessian bit for bit.  The SVD: cyclic Jacobi on M^T M for V, columns sorted
// by decreasing norm, then Givens QR of M V for U (the triangular factor's
// diagonal is s, its last entry signed).
//
// Storage: vec index R = 3 a + i for entry (row i, column a) of M; the upper
// triangle of the symmetric 9x9 matrix packed row by row.  Plain double
// arrays only: the header is shared by the kernels and by a host build of
// the same code.
#pragma once
#include <math.h>

#ifdef __HIPCC__
#define EIG_HD __host__ __device__ __forceinline__
#else
#define EIG_HD static inline
#endif

namespace ipc {
namespace iso {

EIG_HD constexpr int pk(int r, int c) { return r <= c ? r * 9 - r * (r - 1) / 2 + (c - r) : c * 9 - c * (c - 1) / 2 + (r - c); }

// One Jacobi rotation of the symmetric 3x3 matrix A (full storage) zeroing
// A[p][q]; the rotation is accumulated into the columns of Q.
EIG_HD void jrot3(double A[3][3], double Q[3][3], int p, int q)
{
    double apq = A[p][q];
    if (apq == 0.0) return;
    double tau = (A[q][q] - A[p][p]) / (2.0 * apq);
    double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
    double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
    int r = 3 - p - q;
    double arp = A[r][p], arq = A[r][q];
    A[r][p] = A[p][r] = c * arp - s * arq;
    A[r][q] = A[q][r] = s * arp + c * arq;
    A[p][p] -= t * apq;
    A[q][q] += t * apq;
    A[p][q] = A[q][p] = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double vp = Q[k][p], vq = Q[k][q];
        Q[k][p] = c * vp - s * vq;
        Q[k][q] = s * vp + c * vq;
    }
}

// Eigen-decomposition of a symmetric 3x3 matrix in place: on return the
// diagonal of A holds the eigenvalues and the columns of Q the eigenvectors
// (Q a proper rotation).
EIG_HD void eig3(double A[3][3], double Q[3][3])
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) Q[i][j] = i == j ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 12; ++sweep) {
        double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
        double dia = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
        if (off <= 1e-36 * dia) break;
        jrot3(A, Q, 0, 1);
        jrot3(A, Q, 0, 2);
        jrot3(A, Q, 1, 2);
    }
}

// Givens rotation of rows p, q of B (3x3) zeroing B[q][j]; U <- U G^T.
EIG_HD void givens3(double B[3][3], double U[3][3], int p, int q, int j)
{
    double a = B[p][j], b = B[q][j];
    double r = sqrt(a * a + b * b);
    if (r == 0.0) return;
    double c = a / r, s = b / r;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double bp = B[p][k], bq = B[q][k];
        B[p][k] = c * bp + s * bq;
        B[q][k] = c * bq - s * bp;
        double up = U[k][p], uq = U[k][q];
        U[k][p] = c * up + s * uq;
        U[k][q] = c * uq - s * up;
    }
}

// F (F[i][a], row i, column a) = U diag(s) V^T with U, V proper rotations,
// |s0| >= |s1| >= |s2| up to rounding and s0, s1 >= 0.
EIG_HD void svd3(const double F[3][3], double U[3][3], double s[3], double V[3][3])
{
    double S[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) S[a][b] = F[0][a] * F[0][b] + F[1][a] * F[1][b] + F[2][a] * F[2][b];
    eig3(S, V);
    // sort the columns of V by decreasing eigenvalue of F^T F; every swap
    // negates one column so that V stays a proper rotation
    double e[3] = {S[0][0], S[1][1], S[2][2]};
#pragma unroll
    for (int pass = 0; pass < 3; ++pass) {
        int p = pass == 1 ? 1 : 0, q = p + 1;
        if (e[p] < e[q]) {
            double t = e[p]; e[p] = e[q]; e[q] = t;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                double vp = V[k][p];
                V[k][p] = V[k][q];
                V[k][q] = -vp;
            }
        }
    }
    double B[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int a = 0; a < 3; ++a) B[i][a] = F[i][0] * V[0][a] + F[i][1] * V[1][a] + F[i][2] * V[2][a];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) U[i][j] = i == j ? 1.0 : 0.0;
    givens3(B, U, 0, 1, 0);
    givens3(B, U, 0, 2, 0);
    givens3(B, U, 1, 2, 1);
    s[0] = B[0][0];
    s[1] = B[1][1];
    s[2] = B[2][2];
}

// Subtract the negative ones of the twist (lt) and flip (lf) eigenpairs of
// the pair (p, q) from the packed Hessian H.
EIG_HD void sub_pair(double *H, const double U[3][3], const double V[3][3], int p, int q, double lt, double lf)
{
    if (lt >= 0.0 && lf >= 0.0) return;
    const double r2 = 0.70710678118654752440;
    double X[9], Y[9];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            X[3 * a + i] = r2 * U[i][p] * V[a][q];
            Y[3 * a + i] = r2 * U[i][q] * V[a][p];
        }
    if (lt < 0.0) {
#pragma unroll
        for (int R = 0; R < 9; ++R)
#pragma unroll
            for (int C = R; C < 9; ++C) H[pk(R, C)] -= lt * (X[R] - Y[R]) * (X[C] - Y[C]);
    }
    if (lf < 0.0) {
#pragma unroll
        for (int R = 0; R < 9; ++R)
#pragma unroll
            for (int C = R; C < 9; ++C) H[pk(R, C)] -= lf * (X[R] + Y[R]) * (X[C] + Y[C]);
    }
}

// Subtract al vec(U diag(a) V^T) vec(U diag(a) V^T)^T from H.
EIG_HD void sub_scaling(double *H, const double U[3][3], const double V[3][3], const double a[3], double al)
{
    double D[9];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int i = 0; i < 3; ++i) D[3 * c + i] = U[i][0] * a[0] * V[c][0] + U[i][1] * a[1] * V[c][1] + U[i][2] * a[2] * V[c][2];
#pragma unroll
    for (int R = 0; R < 9; ++R)
#pragma unroll
        for (int C = R; C < 9; ++C) H[pk(R, C)] -= al * D[R] * D[C];
}

// H (packed Hessian of the Stable Neo-Hookean density at F) <- its
// projection onto the PSD cone; sc = lh (det F - 1) - mu.
EIG_HD void project_snh(double *H, const double F[3][3], double mu, double lh, double sc)
{
    double U[3][3], V[3][3], s[3];
    svd3(F, U, s, V);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        int p = k == 0 ? 1 : 0, q = k == 2 ? 1 : 2;
        sub_pair(H, U, V, p, q, mu + sc * s[k], mu - sc * s[k]);
    }
    // scaling block: positive definite unless a leading minor is not positive
    double g[3] = {s[1] * s[2], s[2] * s[0], s[0] * s[1]};
    double A[3][3];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int q = 0; q < 3; ++q) A[p][q] = lh * g[p] * g[q] + (p == q ? mu : sc * s[3 - p - q]);
    double m2 = A[0][0] * A[1][1] - A[0][1] * A[0][1];
    double m3 = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[1][2]) - A[0][1] * (A[0][1] * A[2][2] - A[1][2] * A[0][2]) +
                A[0][2] * (A[0][1] * A[1][2] - A[1][1] * A[0][2]);
    if (A[0][0] > 0.0 && m2 > 0.0 && m3 > 0.0) return;
    double Q[3][3];
    eig3(A, Q);
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        if (A[m][m] >= 0.0) continue;
        double a[3] = {Q[0][m], Q[1][m], Q[2][m]};
        sub_scaling(H, U, V, a, A[m][m]);
    }
}

// H (packed Hessian of kv |A A^T - I|^2 over vec A) <- its projection onto
// the PSD cone.
EIG_HD void project_ortho(double *H, const double A[3][3], double kv)
{
    double U[3][3], V[3][3], s[3];
    svd3(A, U, s, V);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        int p = k == 0 ? 1 : 0, q = k == 2 ? 1 : 2;
        double a2 = s[p] * s[p] + s[q] * s[q] - 1.0, ab = s[p] * s[q];
        sub_pair(H, U, V, p, q, 4.0 * kv * (a2 - ab), 4.0 * kv * (a2 + ab));
    }
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        double al = kv * (12.0 * s[m] * s[m] - 4.0);
        if (al >= 0.0) continue;
        double a[3] = {m == 0 ? 1.0 : 0.0, m == 1 ? 1.0 : 0.0, m == 2 ? 1.0 : 0.0};
        sub_scaling(H, U, V, a, al);
    }
}

}   // namespace iso
}   // namespace ipc
