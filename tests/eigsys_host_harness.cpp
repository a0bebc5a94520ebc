// Host build of the closed-form PSD projections used by the FEM and the
// affine-body kernels.  The Stable Neo-Hookean Hessian is formed from the
// Levi-Civita form of det (independent of the kernel's cross-product form);
// the orthogonality Hessian from G = A A^T - I.
#include "ipc_eigsys.h"
static int eps(int a, int b, int c) { return (a - b) * (b - c) * (c - a) / 2; }
/* H of Psi at F (row-major F[i][a]); packed upper triangle, R = 3a + i */
void hess(const double *Fr, double mu, double lh, double *H, int proj, double *svd)
{
    double F[3][3];
    for (int i = 0; i < 3; ++i) for (int a = 0; a < 3; ++a) F[i][a] = Fr[3 * i + a];
    double cof[3][3];
    for (int i = 0; i < 3; ++i) for (int a = 0; a < 3; ++a) {
        double v = 0;
        for (int j = 0; j < 3; ++j) for (int k = 0; k < 3; ++k) for (int b = 0; b < 3; ++b) for (int c = 0; c < 3; ++c)
            v += 0.5 * eps(i, j, k) * eps(a, b, c) * F[j][b] * F[k][c];
        cof[i][a] = v;
    }
    double J = F[0][0] * cof[0][0] + F[1][0] * cof[1][0] + F[2][0] * cof[2][0];
    double sc = lh * (J - 1.0) - mu;
    for (int a = 0; a < 3; ++a) for (int i = 0; i < 3; ++i) for (int b = 0; b < 3; ++b) for (int j = 0; j < 3; ++j) {
        int R = 3 * a + i, C = 3 * b + j;
        if (R > C) continue;
        double d2 = 0;
        for (int k = 0; k < 3; ++k) for (int c = 0; c < 3; ++c) d2 += eps(i, j, k) * eps(a, b, c) * F[k][c];
        H[ipc::iso::pk(R, C)] = lh * cof[i][a] * cof[j][b] + (R == C ? mu : 0.0) + sc * d2;
    }
    if (proj) ipc::iso::project_snh(H, F, mu, lh, sc);
    if (svd) {
        double U[3][3], V[3][3], s[3];
        ipc::iso::svd3(F, U, s, V);
        for (int i = 0; i < 9; ++i) { svd[i] = U[i / 3][i % 3]; svd[9 + i] = V[i / 3][i % 3]; }
        for (int i = 0; i < 3; ++i) svd[18 + i] = s[i];
    }
}
extern "C" void hess_c(const double *F, double mu, double lh, double *H, int proj, double *svd) { hess(F, mu, lh, H, proj, svd); }

/* Hessian of kv |A A^T - I|^2 over vec A: 4 kv (d_ac (A^T A)_db + A_ad A_cb + G_ac d_bd) */
extern "C" void ortho_c(const double *Ar, double kv, double *H, int proj)
{
    double A[3][3], G[3][3], AtA[3][3];
    for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) A[i][j] = Ar[3 * i + j];
    for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) {
        G[i][j] = -(i == j);
        AtA[i][j] = 0;
        for (int k = 0; k < 3; ++k) { G[i][j] += A[i][k] * A[j][k]; AtA[i][j] += A[k][i] * A[k][j]; }
    }
    for (int b = 0; b < 3; ++b) for (int a = 0; a < 3; ++a) for (int d = 0; d < 3; ++d) for (int c = 0; c < 3; ++c) {
        int R = 3 * b + a, C = 3 * d + c;
        if (R > C) continue;
        H[ipc::iso::pk(R, C)] = 4.0 * kv * ((a == c ? AtA[d][b] : 0.0) + A[a][d] * A[c][b] + (b == d ? G[a][c] : 0.0));
    }
    if (proj) ipc::iso::project_ortho(H, A, kv);
}
