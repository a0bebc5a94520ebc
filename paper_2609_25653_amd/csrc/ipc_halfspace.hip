// Analytic half-space ground: {x : n . x >= c} with n a unit normal, met by
// every moving surface vertex (FEM or affine-body) of a scene that has one.
// It is the contact of Sec. III-C.1 (log-barrier, lagged friction, CCD) with
// a plane in place of triangulated static geometry: the distance of a vertex
// is d = n . x - c, so no broad or narrow phase is needed and every entry
// (one per moving surface vertex) is evaluated directly.
//
//  barrier   kappa b(d) for 0 < d < dhat; gradient kappa b'(d) n; Hessian
//            kappa b''(d) n n^T, positive semi-definite as it stands
//            (b'' > 0 below dhat), so it is never projected;
//  friction  lagged at the step start like the pair terms: lam = -kappa
//            b'(d^n), offset x^n, u = (I - n n^T)(x - x^n), potential
//            mu lam f0(|u|) with IPC's f0 and eps_v h;
//  CCD       along x0 + t p the distance d0 + t (n . p) is linear, so the
//            largest step keeping d >= ccd_s d0 is exact:
//            t = (1 - ccd_s) d0 / (-n . p) when n . p < 0.
//
// Entries are scattered without atomics: a contact vertex has at most one
// entry, so its gradient is added by the entry's own thread (after the pair
// terms' run sums, on the same stream), and its 3x3 Hessian goes through the
// same sorted run sums as the pair blocks (an affine body's 4x4 node blocks
// collect many vertices).
#include "ipc_device.h"
#include "ipc_internal.h"
#include "ipc_kernels.h"
#include "ipc_runsum.h"

namespace ipc {

// n . x - c, summed left to right without contraction (as the oracle does)
__device__ __forceinline__ double hs_dist(const double *__restrict__ pl, d3 x)
{
#pragma clang fp contract(off)
    return pl[0] * x.x + pl[1] * x.y + pl[2] * x.z - pl[3];
}

// IPC's friction mollifier: f0, f1(s)/s and the coefficient of u u^T in the
// Hessian of f0(|u|) (zero at s = 0)
struct FrictionCoef {
    double f0, f1s, cu;
};
__device__ __forceinline__ FrictionCoef friction_coef(double sn, double ea)
{
    FrictionCoef f;
    if (sn < ea) {
        f.f0 = -sn * sn * sn / (3.0 * ea * ea) + sn * sn / ea + ea / 3.0;
        f.f1s = 2.0 / ea - sn / (ea * ea);
        f.cu = sn > 0.0 ? -1.0 / (sn * ea * ea) : 0.0;
    } else {
        f.f0 = sn;
        f.f1s = 1.0 / sn;
        f.cu = -1.0 / (sn * sn * sn);
    }
    return f;
}

// MODE 0 energy, 1 + gradient, 2 + Hessian.  Per entry: barrier energy into
// part, friction energy into fpart (fr: friction on), gradient added into the
// contact vertex's accumulator gcv, Hessian block into H with its slot
// entries (key, code = 16 i + q for the node pair q = 4 a + b of the owner;
// a FEM vertex has one node, so only q = 0).
template <int MODE>
__global__ void __launch_bounds__(256) k_hs(int M, const int *__restrict__ hs_cv, const int *__restrict__ cv_scene,
                                            const double *__restrict__ plane, const double *__restrict__ sparam,
                                            const double *__restrict__ xw, const double *__restrict__ lam, const double *__restrict__ xn,
                                            int fr, double *__restrict__ part, double *__restrict__ fpart, double *__restrict__ gcv,
                                            double *__restrict__ H, const int *__restrict__ cv_node, const int *__restrict__ cv_body,
                                            const int *__restrict__ diag_slot, const int *__restrict__ bslot, int nnzb,
                                            int *__restrict__ key, int *__restrict__ code, int *__restrict__ inf_flag)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    const int cv = hs_cv[i], s = cv_scene[cv];
    const double *pl = plane + 4 * (size_t)s, *sp = sparam + 8 * (size_t)s;
    const double kappa = sp[P_KAPPA], dh = sp[P_DHAT];
    const d3 x = ld3(xw, cv), n = {pl[0], pl[1], pl[2]};
    const double d = hs_dist(pl, x);
    double e = 0.0, ef = 0.0, g[3] = {0.0, 0.0, 0.0}, Hl[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) Hl[q] = 0.0;
    if (!(d > 0.0)) atomicOr(inf_flag + s, 1);
    else if (d < dh) {
        e = kappa * barrier(d, dh);
        if (MODE >= 1) {
            const double b1 = kappa * barrier1(d, dh);
            g[0] = b1 * n.x; g[1] = b1 * n.y; g[2] = b1 * n.z;
        }
        if (MODE == 2) {
            const double b2 = kappa * barrier2(d, dh), nv[3] = {n.x, n.y, n.z};
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int c = 0; c < 3; ++c) Hl[3 * r + c] = b2 * nv[r] * nv[c];
        }
    }
    const double lm = fr ? lam[i] : 0.0;
    if (lm > 0.0) {
        const double ea = sp[P_EPSH], w = sp[P_MU] * lm;
        const d3 xr = ld3(xn, i);
        const double dv[3] = {x.x - xr.x, x.y - xr.y, x.z - xr.z}, nv[3] = {n.x, n.y, n.z};
        const double nd = nv[0] * dv[0] + nv[1] * dv[1] + nv[2] * dv[2];
        const double u[3] = {dv[0] - nv[0] * nd, dv[1] - nv[1] * nd, dv[2] - nv[2] * nd};
        const double sn = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        const FrictionCoef f = friction_coef(sn, ea);
        ef = w * f.f0;
        if (MODE >= 1)
#pragma unroll
            for (int q = 0; q < 3; ++q) g[q] += w * f.f1s * u[q];
        if (MODE == 2)
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int c = 0; c < 3; ++c) Hl[3 * r + c] += w * (f.cu * u[r] * u[c] + f.f1s * ((r == c ? 1.0 : 0.0) - nv[r] * nv[c]));
    }
    part[i] = e;
    fpart[i] = ef;
    if (MODE >= 1) {
        double *o = gcv + 3 * (size_t)cv;
        o[0] += g[0]; o[1] += g[1]; o[2] += g[2];
    }
    if (MODE == 2) {
#pragma unroll
        for (int q = 0; q < 9; ++q) H[9 * (size_t)i + q] = Hl[q];
        const int node = cv_node[cv], b = cv_body[cv];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            int k = nnzb;
            if (node >= 0) { if (q == 0) k = diag_slot[node]; }
            else if (b >= 0) k = bslot[16 * (size_t)b + q];
            key[16 * (size_t)i + q] = k;
            code[16 * (size_t)i + q] = 16 * i + q;
        }
    }
}

// One node-pair block of an entry: w_a w_b H with w = (1, xb) the vertex's
// weights on its body's nodes (a FEM vertex: q = 0, weight 1).
struct ValHsBlock {
    const double *H;
    const int *hs_cv, *cv_body;
    const double *cv_x;
    __device__ void operator()(int code, double *out) const
    {
        const int i = code >> 4, q = code & 15, a = q >> 2, b = q & 3, cv = hs_cv[i];
        double wa = 1.0, wb = 1.0;
        if (cv_body[cv] >= 0) {
            wa = a ? cv_x[3 * (size_t)cv + a - 1] : 1.0;
            wb = b ? cv_x[3 * (size_t)cv + b - 1] : 1.0;
        }
        const double w = wa * wb;
#pragma unroll
        for (int k = 0; k < 9; ++k) out[k] = w * H[9 * (size_t)i + k];
    }
};

// Friction lag: an entry closer than dhat (and not intersecting) at the lag
// positions xw is lagged with lam = -kappa b'(d) and offset xref (the step
// start; xw when null); others get lam = 0.  cnt: lagged entries per scene.
__global__ void k_hs_lag(int M, const int *__restrict__ hs_cv, const int *__restrict__ cv_scene, const double *__restrict__ plane,
                         const double *__restrict__ sparam, const double *__restrict__ xw, const double *__restrict__ xref,
                         double *__restrict__ lam, double *__restrict__ xn, int *__restrict__ cnt)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    const int cv = hs_cv[i], s = cv_scene[cv];
    const double *sp = sparam + 8 * (size_t)s;
    const double d = hs_dist(plane + 4 * (size_t)s, ld3(xw, cv)), dh = sp[P_DHAT];
    if (d > 0.0 && d < dh) {
        lam[i] = -sp[P_KAPPA] * barrier1(d, dh);
        st3(xn, i, ld3(xref ? xref : xw, cv));
        atomicAdd(cnt + s, 1);
    } else {
        lam[i] = 0.0;
        st3(xn, i, {0.0, 0.0, 0.0});
    }
}

// CCD bound of the scenes still searching (ls_active), as the bit pattern
// of the smallest step (non-negative doubles order as their bits).
__global__ void k_hs_ccd(int M, const int *__restrict__ hs_cv, const int *__restrict__ cv_scene, const double *__restrict__ plane,
                         const double *__restrict__ sparam, const int *__restrict__ ls_active, const double *__restrict__ xw0,
                         const double *__restrict__ xw1, unsigned long long *__restrict__ amin, int stride)
{
#pragma clang fp contract(off)
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    const int cv = hs_cv[i], s = cv_scene[cv];
    if (!ls_active[s]) return;
    const double *pl = plane + 4 * (size_t)s;
    const d3 x0 = ld3(xw0, cv), x1 = ld3(xw1, cv);
    const double p[3] = {x1.x - x0.x, x1.y - x0.y, x1.z - x0.z};
    const double d0 = hs_dist(pl, x0);
    const double np = pl[0] * p[0] + pl[1] * p[1] + pl[2] * p[2];
    if (np < 0.0) {
        const double t = (1.0 - sparam[8 * (size_t)s + P_CCDS]) * d0 / -np;
        if (t < 1.0) atomicMin(amin + (size_t)stride * s, (unsigned long long)__double_as_longlong(t));
    }
}

// Adaptive kappa: the smallest squared distance of the entries closer than
// dhat, into the scene's running minimum (bit pattern, atomic min).
__global__ void k_hs_dmin(int M, const int *__restrict__ hs_cv, const int *__restrict__ cv_scene, const double *__restrict__ plane,
                          const double *__restrict__ sparam, const double *__restrict__ xw, unsigned long long *__restrict__ dmin,
                          int stride)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    const int cv = hs_cv[i], s = cv_scene[cv];
    const double d = hs_dist(plane + 4 * (size_t)s, ld3(xw, cv));
    if (d >= sparam[8 * (size_t)s + P_DHAT]) return;
    const double d2 = d > 0.0 ? d * d : 0.0;   // sqrt(d * d) == d exactly
    atomicMin(dmin + (size_t)stride * s, (unsigned long long)__double_as_longlong(d2));
}

// Adjoint of the friction lag of the half-space entries.  For the adjoint
// vector w an entry adds phi = mu lam (f1(s)/s) (W . u) to w^T G, W the
// vertex's world-space part of w.  With the normal fixed, phi depends on
// the lag position x^n through lam = -kappa b'(n . x^n - c) (d lam / d x^n =
// -kappa b'' n) and u = (I - n n^T)(x - x^n) (d u / d x^n = -(I - n n^T)).
// -d phi / d x^n is added to the vertex's accumulator gcv (the caller adds
// it into ybar through the DOF maps), and part[i] = lam (f1/s) (W . u), the
// entry's w . dG/dmu.
__global__ void k_hs_lag_vjp(int M, const int *__restrict__ hs_cv, const int *__restrict__ cv_scene, const double *__restrict__ plane,
                             const double *__restrict__ sparam, const double *__restrict__ lam0, const double *__restrict__ xw,
                             const double *__restrict__ xwn, const int *__restrict__ cv_node, const int *__restrict__ cv_body,
                             const double *__restrict__ cv_x, const int *__restrict__ body_node0, const double *__restrict__ w,
                             double *__restrict__ gcv, double *__restrict__ part)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    part[i] = 0.0;
    if (!(lam0[i] > 0.0)) return;
    const int cv = hs_cv[i], s = cv_scene[cv];
    const double *pl = plane + 4 * (size_t)s, *sp = sparam + 8 * (size_t)s;
    const double kappa = sp[P_KAPPA], dh = sp[P_DHAT], mu = sp[P_MU], ea = sp[P_EPSH];
    const double nv[3] = {pl[0], pl[1], pl[2]};
    // W: the adjoint vector at the vertex (its node, or its body's affine map)
    d3 W;
    const int node = cv_node[cv];
    if (node >= 0) W = ld3(w, node);
    else {
        const int n0 = body_node0[cv_body[cv]];
        W = xaffine(ld3(w, n0), ld3(w, n0 + 1), ld3(w, n0 + 2), ld3(w, n0 + 3), ld3(cv_x, cv));
    }
    const double Wv[3] = {W.x, W.y, W.z};
    const d3 x = ld3(xw, cv), xn = ld3(xwn, cv);
    const double D[3] = {x.x - xn.x, x.y - xn.y, x.z - xn.z};
    const double d = hs_dist(pl, xn), b1 = barrier1(d, dh), b2 = barrier2(d, dh), lm = -kappa * b1;
    const double nD = nv[0] * D[0] + nv[1] * D[1] + nv[2] * D[2];
    const double u[3] = {D[0] - nv[0] * nD, D[1] - nv[1] * nD, D[2] - nv[2] * nD};
    const double sg = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    const double f1s = sg < ea ? 2.0 / ea - sg / (ea * ea) : 1.0 / sg;
    const double df1s = sg < ea ? -1.0 / (ea * ea) : -1.0 / (sg * sg);
    const double Wu = Wv[0] * u[0] + Wv[1] * u[1] + Wv[2] * u[2], psi = f1s * Wu;
    double dpsi_du[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) dpsi_du[c] = f1s * Wv[c] + (sg > 0.0 ? Wu * df1s * u[c] / sg : 0.0);
    part[i] = lm * psi;
    double out[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double dpsi = 0.0;
#pragma unroll
        for (int r = 0; r < 3; ++r) dpsi += dpsi_du[r] * -((r == c ? 1.0 : 0.0) - nv[r] * nv[c]);
        const double dlam = -kappa * b2 * nv[c];
        out[c] = -mu * (dlam * psi + lm * dpsi);
    }
    double *o = gcv + 3 * (size_t)cv;
    o[0] += out[0]; o[1] += out[1]; o[2] += out[2];
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
void hs_setup(ipc_ctx *c)
{
    Dev &D = c->d;
    const int64_t M = std::max<int64_t>(c->M_HS, 1);
    D.hs_part.alloc(M + 1); D.hs_fpart.alloc(M + 1);
    D.hs_w64.alloc(M / TILE + 1); D.hs_fw64.alloc(M / TILE + 1);
    D.hs_lam.alloc(M); D.hs_lam.zero(c->stream, M);
    D.hs_xn.alloc(3 * M);
    D.hs_H.alloc(9 * M);
    for (auto *b : {&D.hs_key, &D.hs_code, &D.hs_key2, &D.hs_code2}) b->alloc(16 * M);
    D.hs_nlag.alloc(c->n_scenes); D.hs_nlag.zero(c->stream, c->n_scenes);
}

void launch_hs(ipc_ctx *c, int mode, const double *xw)
{
    if (!c->M_HS) return;
    Dev &D = c->d;
    const int M = (int)c->M_HS;
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(blocks_for(M)), dim3(BLOCK), 0, c->stream, M, D.hs_cv.p, D.cv_scene.p, D.hs_plane.p,
                           D.sparam.p, xw, D.hs_lam.p, D.hs_xn.p, (int)c->fr_on, D.hs_part.p, D.hs_fpart.p, D.gcv.p, D.hs_H.p,
                           D.cv_node.p, D.cv_body.p, D.diag_slot.p, D.bslot.p, c->nnzb, D.hs_key.p, D.hs_code.p, D.inf_flag.p);
    };
    if (mode == 0) go(k_hs<0>);
    else if (mode == 1) go(k_hs<1>);
    else go(k_hs<2>);
    if (mode == 2) {
        sort_entries(c, D.hs_key.p, D.hs_key2.p, D.hs_code.p, D.hs_code2.p, 16 * (int64_t)M, bits_for(c->nnzb));
        runsum<9>(c, 16 * (int64_t)M, c->nnzb, D.hs_key2.p, D.hs_code2.p, ValHsBlock{D.hs_H.p, D.hs_cv.p, D.cv_body.p, D.cv_x.p},
                  EmitAdd9{D.val.p});
    }
    sum64(c, D.hs_part.p, M, D.hs_w64.p);
    sum64(c, D.hs_fpart.p, M, D.hs_fw64.p);
}

void launch_hs_lag(ipc_ctx *c, const double *xw, const double *xref)
{
    if (!c->M_HS) return;
    Dev &D = c->d;
    const int M = (int)c->M_HS;
    D.hs_nlag.zero(c->stream, c->n_scenes);
    hipLaunchKernelGGL(k_hs_lag, dim3(blocks_for(M)), dim3(BLOCK), 0, c->stream, M, D.hs_cv.p, D.cv_scene.p, D.hs_plane.p,
                       D.sparam.p, xw, xref, D.hs_lam.p, D.hs_xn.p, D.hs_nlag.p);
}

void launch_hs_ccd(ipc_ctx *c, const double *xw0, const double *xw1)
{
    if (!c->M_HS) return;
    Dev &D = c->d;
    const int M = (int)c->M_HS;
    hipLaunchKernelGGL(k_hs_ccd, dim3(blocks_for(M)), dim3(BLOCK), 0, c->stream, M, D.hs_cv.p, D.cv_scene.p, D.hs_plane.p,
                       D.sparam.p, D.ls_active.p, xw0, xw1, (unsigned long long *)(D.scal.p + S_CCD), NSLOT);
}

void launch_hs_dmin(ipc_ctx *c, const double *xw)
{
    if (!c->M_HS) return;
    Dev &D = c->d;
    const int M = (int)c->M_HS;
    hipLaunchKernelGGL(k_hs_dmin, dim3(blocks_for(M)), dim3(BLOCK), 0, c->stream, M, D.hs_cv.p, D.cv_scene.p, D.hs_plane.p,
                       D.sparam.p, xw, (unsigned long long *)(D.scal.p + S_DMIN), NSLOT);
}

void launch_hs_lag_vjp(ipc_ctx *c, const double *xw, const double *xwn, const double *w)
{
    if (!c->M_HS) return;
    Dev &D = c->d;
    const int M = (int)c->M_HS;
    hipLaunchKernelGGL(k_hs_lag_vjp, dim3(blocks_for(M)), dim3(BLOCK), 0, c->stream, M, D.hs_cv.p, D.cv_scene.p, D.hs_plane.p,
                       D.sparam.p, D.hs_lam.p, xw, xwn, D.cv_node.p, D.cv_body.p, D.cv_x.p, D.body_node0.p, w, D.gcv.p,
                       D.hs_fpart.p);
    sum64(c, D.hs_fpart.p, M, D.hs_fw64.p);
}

} // namespace ipc
