// Device-side pointwise math: distances, barrier, Stable Neo-Hookean, PSD
// projection.  Everything here runs per thread in registers.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

namespace ipc {

struct d3 { double x, y, z; };

__device__ __forceinline__ d3 mk(double x, double y, double z) { return {x, y, z}; }
__device__ __forceinline__ d3 ld3(const double *p, int i) { return {p[3 * (size_t)i], p[3 * (size_t)i + 1], p[3 * (size_t)i + 2]}; }
__device__ __forceinline__ void st3(double *p, int i, d3 v) { p[3 * (size_t)i] = v.x; p[3 * (size_t)i + 1] = v.y; p[3 * (size_t)i + 2] = v.z; }

// ---------------------------------------------------------------------------
// Exact-order vector arithmetic.  The contact-pair predicate d^2 < dhat^2 must
// come out identical on every implementation that follows the written
// distance specification, so these helpers never fuse a*b+c.
// ---------------------------------------------------------------------------
__device__ __forceinline__ d3 xsub(d3 a, d3 b)
{
#pragma clang fp contract(off)
    return {a.x - b.x, a.y - b.y, a.z - b.z};
}
__device__ __forceinline__ double xdot(d3 a, d3 b)
{
#pragma clang fp contract(off)
    double t = a.x * b.x;
    t = t + a.y * b.y;
    t = t + a.z * b.z;
    return t;
}
__device__ __forceinline__ d3 xcross(d3 a, d3 b)
{
#pragma clang fp contract(off)
    double cx = a.y * b.z - a.z * b.y;
    double cy = a.z * b.x - a.x * b.z;
    double cz = a.x * b.y - a.y * b.x;
    return {cx, cy, cz};
}
// body point p + xb0 A0 + xb1 A1 + xb2 A2, left to right, unfused
__device__ __forceinline__ d3 xaffine(d3 p, d3 a0, d3 a1, d3 a2, d3 xb)
{
#pragma clang fp contract(off)
    double x = p.x + xb.x * a0.x; x = x + xb.y * a1.x; x = x + xb.z * a2.x;
    double y = p.y + xb.x * a0.y; y = y + xb.y * a1.y; y = y + xb.z * a2.y;
    double z = p.z + xb.x * a0.z; z = z + xb.y * a1.z; z = z + xb.z * a2.z;
    return {x, y, z};
}

__device__ __forceinline__ double d2_pp(d3 p, d3 q) { d3 u = xsub(p, q); return xdot(u, u); }
__device__ __forceinline__ double d2_pe(d3 p, d3 e0, d3 e1)
{
    d3 c = xcross(xsub(e0, p), xsub(e1, p));
    d3 e = xsub(e1, e0);
    return xdot(c, c) / xdot(e, e);
}
__device__ __forceinline__ double d2_plane(d3 p, d3 t0, d3 t1, d3 t2)
{
#pragma clang fp contract(off)
    d3 n = xcross(xsub(t1, t0), xsub(t2, t0));
    double s = xdot(n, xsub(p, t0));
    return s * s / xdot(n, n);
}
__device__ __forceinline__ double d2_line(d3 a0, d3 a1, d3 b0, d3 b1)
{
#pragma clang fp contract(off)
    d3 n = xcross(xsub(a1, a0), xsub(b1, b0));
    double s = xdot(n, xsub(b0, a0));
    return s * s / xdot(n, n);
}

// Point-triangle distance type (Voronoi regions of the closed triangle):
// 0..2 vertex t_k, 3 edge t0t1, 4 edge t1t2, 5 edge t2t0, 6 interior.
__device__ __forceinline__ int pt_type(d3 p, d3 t0, d3 t1, d3 t2)
{
#pragma clang fp contract(off)
    d3 ab = xsub(t1, t0), ac = xsub(t2, t0), ap = xsub(p, t0);
    double d1 = xdot(ab, ap), d2 = xdot(ac, ap);
    if (d1 <= 0.0 && d2 <= 0.0) return 0;
    d3 bp = xsub(p, t1);
    double d3_ = xdot(ab, bp), d4 = xdot(ac, bp);
    if (d3_ >= 0.0 && d4 <= d3_) return 1;
    double vc = d1 * d4 - d3_ * d2;
    if (vc <= 0.0 && d1 >= 0.0 && d3_ <= 0.0) return 3;
    d3 cp = xsub(p, t2);
    double d5 = xdot(ab, cp), d6 = xdot(ac, cp);
    if (d6 >= 0.0 && d5 <= d6) return 2;
    double vb = d5 * d2 - d1 * d6;
    if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) return 5;
    double va = d3_ * d6 - d5 * d4;
    if (va <= 0.0 && (d4 - d3_) >= 0.0 && (d5 - d6) >= 0.0) return 4;
    return 6;
}
__device__ __forceinline__ double pt_d2(int t, d3 p, d3 t0, d3 t1, d3 t2)
{
    switch (t) {
    case 0: return d2_pp(p, t0);
    case 1: return d2_pp(p, t1);
    case 2: return d2_pp(p, t2);
    case 3: return d2_pe(p, t0, t1);
    case 4: return d2_pe(p, t1, t2);
    case 5: return d2_pe(p, t2, t0);
    default: return d2_plane(p, t0, t1, t2);
    }
}

// Edge-edge type: 0 (a0,b0) 1 (a0,b1) 2 (a1,b0) 3 (a1,b1) point pairs,
// 4 a0-edge b, 5 a1-edge b, 6 b0-edge a, 7 b1-edge a, 8 interior of both.
__device__ __forceinline__ double ee_d2(int t, d3 a0, d3 a1, d3 b0, d3 b1)
{
    switch (t) {
    case 0: return d2_pp(a0, b0);
    case 1: return d2_pp(a0, b1);
    case 2: return d2_pp(a1, b0);
    case 3: return d2_pp(a1, b1);
    case 4: return d2_pe(a0, b0, b1);
    case 5: return d2_pe(a1, b0, b1);
    case 6: return d2_pe(b0, a0, a1);
    case 7: return d2_pe(b1, a0, a1);
    default: return d2_line(a0, a1, b0, b1);
    }
}
// closest point of segment e0e1 to p: 0 at e0, 1 at e1, 2 interior
__device__ __forceinline__ int ps_type(d3 p, d3 e0, d3 e1)
{
    d3 ev = xsub(e1, e0);
    double t = xdot(xsub(p, e0), ev), L = xdot(ev, ev);
    return t <= 0.0 ? 0 : (t >= L ? 1 : 2);
}
__device__ __forceinline__ int ee_type(d3 a0, d3 a1, d3 b0, d3 b1)
{
#pragma clang fp contract(off)
    d3 u = xsub(a1, a0), v = xsub(b1, b0), w = xsub(a0, b0);
    double A = xdot(u, u), B = xdot(u, v), C = xdot(v, v), D = xdot(u, w), E = xdot(v, w);
    double den = A * C - B * B;
    if (den > 1e-10 * A * C) {
        double sN = B * E - C * D, tN = A * E - B * D;
        if (sN > 0.0 && sN < den && tN > 0.0 && tN < den) return 8;
    }
    int k, c0, c1, c2, c3;
    k = ps_type(a0, b0, b1); c0 = k == 0 ? 0 : (k == 1 ? 1 : 4);
    k = ps_type(a1, b0, b1); c1 = k == 0 ? 2 : (k == 1 ? 3 : 5);
    k = ps_type(b0, a0, a1); c2 = k == 0 ? 0 : (k == 1 ? 2 : 6);
    k = ps_type(b1, a0, a1); c3 = k == 0 ? 1 : (k == 1 ? 3 : 7);
    int best = c0;
    double bd = ee_d2(c0, a0, a1, b0, b1), d;
    d = ee_d2(c1, a0, a1, b0, b1); if (d < bd) { bd = d; best = c1; }
    d = ee_d2(c2, a0, a1, b0, b1); if (d < bd) { bd = d; best = c2; }
    d = ee_d2(c3, a0, a1, b0, b1); if (d < bd) { bd = d; best = c3; }
    return best;
}

__device__ __forceinline__ double pair_d2(int kind, const d3 *x, int *type)
{
    if (kind == 0) { int t = pt_type(x[0], x[1], x[2], x[3]); *type = t; return pt_d2(t, x[0], x[1], x[2], x[3]); }
    int t = ee_type(x[0], x[1], x[2], x[3]); *type = t; return ee_d2(t, x[0], x[1], x[2], x[3]);
}

// ---------------------------------------------------------------------------
// Closest-point parametrisation of a distance type: r(s) = sum_k a_k(s) x_k,
// a(s) = a0 + s_0 a1 + s_1 a2, with npar free parameters at the optimum.
// ---------------------------------------------------------------------------
struct TypeParam { int npar; double a0[4], a1[4], a2[4]; };

__device__ __forceinline__ void set4(double *v, double a, double b, double c, double d) { v[0] = a; v[1] = b; v[2] = c; v[3] = d; }

__device__ __forceinline__ TypeParam type_param(int kind, int t)
{
    TypeParam P;
    P.npar = 0;
    set4(P.a1, 0, 0, 0, 0); set4(P.a2, 0, 0, 0, 0);
    if (kind == 0) {
        switch (t) {
        case 0: set4(P.a0, 1, -1, 0, 0); break;
        case 1: set4(P.a0, 1, 0, -1, 0); break;
        case 2: set4(P.a0, 1, 0, 0, -1); break;
        case 3: P.npar = 1; set4(P.a0, 1, -1, 0, 0); set4(P.a1, 0, 1, -1, 0); break;
        case 4: P.npar = 1; set4(P.a0, 1, 0, -1, 0); set4(P.a1, 0, 0, 1, -1); break;
        case 5: P.npar = 1; set4(P.a0, 1, 0, 0, -1); set4(P.a1, 0, -1, 0, 1); break;
        default: P.npar = 2; set4(P.a0, 1, -1, 0, 0); set4(P.a1, 0, 1, -1, 0); set4(P.a2, 0, 1, 0, -1); break;
        }
    } else {
        switch (t) {
        case 0: set4(P.a0, 1, 0, -1, 0); break;
        case 1: set4(P.a0, 1, 0, 0, -1); break;
        case 2: set4(P.a0, 0, 1, -1, 0); break;
        case 3: set4(P.a0, 0, 1, 0, -1); break;
        case 4: P.npar = 1; set4(P.a0, 1, 0, -1, 0); set4(P.a1, 0, 0, 1, -1); break;
        case 5: P.npar = 1; set4(P.a0, 0, 1, -1, 0); set4(P.a1, 0, 0, 1, -1); break;
        case 6: P.npar = 1; set4(P.a0, 1, 0, -1, 0); set4(P.a1, -1, 1, 0, 0); break;
        case 7: P.npar = 1; set4(P.a0, 1, 0, 0, -1); set4(P.a1, -1, 1, 0, 0); break;
        default: P.npar = 2; set4(P.a0, 1, 0, -1, 0); set4(P.a1, -1, 1, 0, 0); set4(P.a2, 0, 0, 1, -1); break;
        }
    }
    return P;
}

__device__ __forceinline__ d3 comb4(const double *a, const d3 *x)
{
    return {a[0] * x[0].x + a[1] * x[1].x + a[2] * x[2].x + a[3] * x[3].x,
            a[0] * x[0].y + a[1] * x[1].y + a[2] * x[2].y + a[3] * x[3].y,
            a[0] * x[0].z + a[1] * x[1].z + a[2] * x[2].z + a[3] * x[3].z};
}
__device__ __forceinline__ double dt(d3 a, d3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ double comp(d3 v, int c) { return c == 0 ? v.x : (c == 1 ? v.y : v.z); }

// beta = a(s*), r = sum beta_k x_k, D_m = sum a_m,k x_k
__device__ __forceinline__ void closest_point(const TypeParam &P, const d3 *x, double *beta, d3 &r, d3 &D0, d3 &D1)
{
    d3 r0 = comb4(P.a0, x);
    D0 = comb4(P.a1, x);
    D1 = comb4(P.a2, x);
    double s0 = 0.0, s1 = 0.0;
    if (P.npar == 1) {
        s0 = -dt(D0, r0) / dt(D0, D0);
    } else if (P.npar == 2) {
        double G00 = dt(D0, D0), G01 = dt(D0, D1), G11 = dt(D1, D1);
        double b0 = -dt(D0, r0), b1 = -dt(D1, r0);
        double det = G00 * G11 - G01 * G01;
        s0 = (b0 * G11 - G01 * b1) / det;
        s1 = (G00 * b1 - G01 * b0) / det;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) beta[k] = P.a0[k] + s0 * P.a1[k] + s1 * P.a2[k];
    r = comb4(beta, x);
}

// Orthonormal basis of the complement of the common translation of 4 points
// (Helmert contrasts): U[k][i], vertex k, component i.
__device__ __forceinline__ double helmert(int k, int i)
{
    const double r2 = 0.70710678118654752440, r6 = 0.40824829046386301637, r12 = 0.28867513459481288225;
    if (i == 0) return k == 0 ? r2 : (k == 1 ? -r2 : 0.0);
    if (i == 1) return k == 2 ? -2.0 * r6 : (k == 3 ? 0.0 : r6);
    return k == 3 ? -3.0 * r12 : r12;
}

// ---------------------------------------------------------------------------
// log-barrier b(d) = -(d - dh)^2 ln(d / dh) for d < dh
// ---------------------------------------------------------------------------
__device__ __forceinline__ double barrier(double d, double dh)
{
    return d >= dh ? 0.0 : -(d - dh) * (d - dh) * log(d / dh);
}
__device__ __forceinline__ double barrier1(double d, double dh)
{
    return d >= dh ? 0.0 : -2.0 * (d - dh) * log(d / dh) - (d - dh) * (d - dh) / d;
}
__device__ __forceinline__ double barrier2(double d, double dh)
{
    return d >= dh ? 0.0 : -2.0 * log(d / dh) - 4.0 * (d - dh) / d + (d - dh) * (d - dh) / (d * d);
}

// ---------------------------------------------------------------------------
// Symmetric 9x9 PSD projection by cyclic Jacobi, fully in registers.
// A is packed upper-triangular (45 values).
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int pk9(int i, int j)
{
    return i <= j ? i * 9 - (i * (i - 1)) / 2 + (j - i) : j * 9 - (j * (j - 1)) / 2 + (i - j);
}

__device__ __forceinline__ void jacobi_rot9(double *A, double *V, int p, int q)
{
    double apq = A[pk9(p, q)];
    if (apq == 0.0) return;
    double app = A[pk9(p, p)], aqq = A[pk9(q, q)];
    double theta = (aqq - app) / (2.0 * apq);
    double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(1.0 + theta * theta));
    double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        if (k == p || k == q) continue;
        double akp = A[pk9(k, p)], akq = A[pk9(k, q)];
        A[pk9(k, p)] = c * akp - s * akq;
        A[pk9(k, q)] = s * akp + c * akq;
    }
    A[pk9(p, p)] = app - t * apq;
    A[pk9(q, q)] = aqq + t * apq;
    A[pk9(p, q)] = 0.0;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        double vkp = V[k * 9 + p], vkq = V[k * 9 + q];
        V[k * 9 + p] = c * vkp - s * vkq;
        V[k * 9 + q] = s * vkp + c * vkq;
    }
}

// In place: A <- Q max(L, 0) Q^T.
__device__ __forceinline__ void psd_project9(double *A)
{
    double V[81];
#pragma unroll
    for (int i = 0; i < 81; ++i) V[i] = (i % 10 == 0) ? 1.0 : 0.0;
    double diag2 = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) diag2 += A[pk9(i, i)] * A[pk9(i, i)];
    double off2 = 0.0;
#pragma unroll
    for (int p = 0; p < 9; ++p)
#pragma unroll
        for (int q = p + 1; q < 9; ++q) off2 += A[pk9(p, q)] * A[pk9(p, q)];
    if (off2 == 0.0) {
#pragma unroll
        for (int i = 0; i < 9; ++i) A[pk9(i, i)] = fmax(A[pk9(i, i)], 0.0);
        return;
    }
    for (int sweep = 0; sweep < 20; ++sweep) {
#pragma unroll
        for (int p = 0; p < 9; ++p)
#pragma unroll
            for (int q = p + 1; q < 9; ++q) jacobi_rot9(A, V, p, q);
        off2 = 0.0;
        diag2 = 0.0;
#pragma unroll
        for (int p = 0; p < 9; ++p) {
            diag2 += A[pk9(p, p)] * A[pk9(p, p)];
#pragma unroll
            for (int q = p + 1; q < 9; ++q) off2 += A[pk9(p, q)] * A[pk9(p, q)];
        }
        if (off2 <= 1e-34 * diag2) break;
    }
    double w[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) w[i] = fmax(A[pk9(i, i)], 0.0);
#pragma unroll
    for (int i = 0; i < 9; ++i)
#pragma unroll
        for (int j = i; j < 9; ++j) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < 9; ++k) acc += V[i * 9 + k] * w[k] * V[j * 9 + k];
            A[pk9(i, j)] = acc;
        }
}

// ---------------------------------------------------------------------------
// Stable Neo-Hookean, rest-stable form with lh = lambda + mu:
//   Psi = mu/2 (|F|^2 - 3) - mu (J - 1) + lh/2 (J - 1)^2
// F given by its columns f0, f1, f2.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double cross_c(d3 a, d3 b, int c)
{
    return c == 0 ? a.y * b.z - a.z * b.y : (c == 1 ? a.z * b.x - a.x * b.z : a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ d3 cr(d3 a, d3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }

// skew matrix [v]x entry (i, j)
__device__ __forceinline__ double skew(d3 v, int i, int j)
{
    if (i == j) return 0.0;
    if (i == 0) return j == 1 ? -v.z : v.y;
    if (i == 1) return j == 0 ? v.z : -v.x;
    return j == 0 ? -v.y : v.x;
}

} // namespace ipc
