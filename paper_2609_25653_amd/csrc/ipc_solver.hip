// Linear algebra of the Newton step: deterministic per-scene reductions, the
// Hessian product (block-CSR FEM part + affine-body blocks + matrix-free
// springs and contacts), the block-Jacobi preconditioner (3x3 per FEM vertex,
// 12x12 per body) and a PCG that runs all scenes at once with per-scene
// scalars and convergence flags.
#include <cmath>

#include "ipc_device.h"
#include "ipc_internal.h"
#include "ipc_kernels.h"

namespace ipc {

// ---------------------------------------------------------------------------
// reductions: one workgroup per scene, fixed-order strided sums and a tree
// ---------------------------------------------------------------------------
__global__ void k_reduce(int ns, RedArgs a, double *__restrict__ scal)
{
    int s = blockIdx.x;
    __shared__ double sh[256];
    double total = a.op ? 0.0 : 0.0;
    for (int k = 0; k < a.nsrc; ++k) {
        const RedSrc &r = a.src[k];
        double part = 0.0;
        if (r.v) {
            int lo = r.seg[s] - r.base, hi = r.seg[s + 1] - r.base;
            for (int i = lo + (int)threadIdx.x; i < hi; i += 256) {
                double v = r.v[r.off + i];
                part = a.op ? fmax(part, v) : part + v;
            }
        }
        sh[threadIdx.x] = part;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) sh[threadIdx.x] = a.op ? fmax(sh[threadIdx.x], sh[threadIdx.x + o]) : sh[threadIdx.x] + sh[threadIdx.x + o];
            __syncthreads();
        }
        double v = sh[0];
        __syncthreads();
        if (threadIdx.x == 0 && a.slots[k] >= 0) scal[(size_t)s * NSLOT + a.slots[k]] = v;
        total = a.op ? fmax(total, v) : total + v;
    }
    if (threadIdx.x == 0 && a.slot >= 0) {
        double *d = scal + (size_t)s * NSLOT + a.slot;
        *d = a.acc ? (a.op ? fmax(*d, total) : *d + total) : total;
    }
}

void reduce(ipc_ctx *c, const RedArgs &a)
{
    hipLaunchKernelGGL(k_reduce, dim3(c->n_scenes), dim3(256), 0, c->stream, c->n_scenes, a, c->d.scal.p);
}

RedSrc src(const double *v, const int *seg, int off, int base)
{
    RedSrc r;
    r.v = v; r.seg = seg; r.off = off; r.base = base;
    return r;
}

int *seg_ptr(ipc_ctx *c, int region) { return c->d.segs.p + (size_t)region * (c->n_scenes + 1); }

// ---------------------------------------------------------------------------
// Hessian product
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_spmv(int N, const int *__restrict__ row_ptr, const int *__restrict__ col,
                                              const double *__restrict__ val, const double *__restrict__ v,
                                              const int *__restrict__ node_scene, const int *__restrict__ active,
                                              double *__restrict__ out, double *__restrict__ part)
{
    int n = blockIdx.x * blockDim.x + threadIdx.x;
    double qf = 0.0;
    if (n < N) {
        double ax = 0.0, ay = 0.0, az = 0.0;
        if (!active || active[node_scene[n]]) {
            int k0 = row_ptr[n], k1 = row_ptr[n + 1];
            for (int k = k0; k < k1; ++k) {
                const double *B = val + 9 * (size_t)k;
                d3 w = ld3(v, col[k]);
                ax += B[0] * w.x + B[1] * w.y + B[2] * w.z;
                ay += B[3] * w.x + B[4] * w.y + B[5] * w.z;
                az += B[6] * w.x + B[7] * w.y + B[8] * w.z;
            }
            if (k1 > k0) {
                d3 w = ld3(v, n);
                qf = w.x * ax + w.y * ay + w.z * az;
            }
        }
        st3(out, n, {ax, ay, az});
    }
    qf = wave_sum(qf);
    if (part && (threadIdx.x & (TILE - 1)) == 0 && n < N) part[n / TILE] = qf;
}

__global__ void k_body_apply(int NB, const int *__restrict__ node0, const int *__restrict__ bscene, const double *__restrict__ Hb,
                             const int *__restrict__ active, const double *__restrict__ v, double *__restrict__ out,
                             double *__restrict__ part)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= NB) return;
    if (active && !active[bscene[b]]) { if (part) part[b] = 0.0; return; }
    int n0 = node0[b];
    double w[12];
    for (int c = 0; c < 4; ++c) { d3 t = ld3(v, n0 + c); w[3 * c] = t.x; w[3 * c + 1] = t.y; w[3 * c + 2] = t.z; }
    const double *H = Hb + 144 * (size_t)b;
    double qf = 0.0;
    for (int i = 0; i < 12; ++i) {
        double acc = 0.0;
        for (int j = 0; j < 12; ++j) acc += H[12 * i + j] * w[j];
        out[3 * (size_t)n0 + i] += acc;
        qf += w[i] * acc;
    }
    if (part) part[b] = qf;
}

void hess_apply(ipc_ctx *c, const double *v, double *out, const int *active, bool partials)
{
    Dev &D = c->d;
    hipStream_t st = c->stream;
    prof_begin(c, IPC_K_SPMV);
    hipLaunchKernelGGL(k_spmv, dim3(blocks_for(c->N)), dim3(BLOCK), 0, st, c->N, D.row_ptr.p, D.col.p, D.val.p, v, D.node_scene.p,
                       active, out, partials ? D.part_node.p : nullptr);
    prof_end(c, IPC_K_SPMV, 76.0 * c->nnzb + 4.0 * (c->N + 1) + 48.0 * c->NFEM);
    if (c->NB)
        hipLaunchKernelGGL(k_body_apply, dim3(blocks_for(c->NB, 64)), dim3(64), 0, st, c->NB, D.body_node0.p, D.body_scene.p, D.Hb.p,
                           active, v, out, partials ? D.body_part.p : nullptr);
    launch_spring_apply(c, v, out, active, partials ? D.sp_part.p : nullptr, D.h2s.p);
    D.pair_part.alloc(c->n_pt + c->n_ee + 1);
    D.fr_part.alloc(c->n_lag + 1);
    prof_begin(c, IPC_K_CONTACT_APPLY);
    launch_contact_apply(c, v, out, active, partials ? D.pair_part.p : nullptr, partials ? D.fr_part.p : nullptr);
    prof_end(c, IPC_K_CONTACT_APPLY, 0.0);
    if (partials) {
        RedArgs a{};
        a.nsrc = 0;
        a.src[a.nsrc++] = src(D.part_node.p, seg_ptr(c, R_NODEW), 0, 0);
        a.src[a.nsrc++] = src(c->NB ? D.body_part.p : nullptr, seg_ptr(c, R_BODY), 0, 0);
        a.src[a.nsrc++] = src(c->NS ? D.sp_part.p : nullptr, seg_ptr(c, R_SP), 0, 0);
        a.src[a.nsrc++] = src(c->n_pt ? D.pair_part.p : nullptr, seg_ptr(c, R_PT), 0, 0);
        a.src[a.nsrc++] = src(c->n_ee ? D.pair_part.p : nullptr, seg_ptr(c, R_EE), (int)c->n_pt, 0);
        if (c->fr_on) {
            a.src[a.nsrc++] = src(c->n_lag_pt ? D.fr_part.p : nullptr, seg_ptr(c, R_LPT), 0, 0);
            a.src[a.nsrc++] = src(c->n_lag - c->n_lag_pt ? D.fr_part.p : nullptr, seg_ptr(c, R_LEE), (int)c->n_lag_pt, 0);
        }
        a.slot = S_PAP;
        a.acc = 0;
        reduce(c, a);
    }
}

// ---------------------------------------------------------------------------
// block-Jacobi preconditioner
// ---------------------------------------------------------------------------
__global__ void k_prec_fem(int N, const int *__restrict__ kind, const int *__restrict__ diag_slot, const double *__restrict__ val,
                           const double *__restrict__ spd, const double *__restrict__ diagF, double *__restrict__ dinv)
{
    int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    double *o = dinv + 9 * (size_t)n;
    if (kind[n] != 0) { for (int q = 0; q < 9; ++q) o[q] = 0.0; return; }
    double a[9];
    const double *B = val + 9 * (size_t)diag_slot[n];
    for (int q = 0; q < 9; ++q) a[q] = B[q] + spd[9 * (size_t)n + q] + diagF[9 * (size_t)n + q];
    double c0 = a[4] * a[8] - a[5] * a[7], c1 = a[5] * a[6] - a[3] * a[8], c2 = a[3] * a[7] - a[4] * a[6];
    double det = a[0] * c0 + a[1] * c1 + a[2] * c2;
    double id = 1.0 / det;
    o[0] = c0 * id; o[1] = (a[2] * a[7] - a[1] * a[8]) * id; o[2] = (a[1] * a[5] - a[2] * a[4]) * id;
    o[3] = c1 * id; o[4] = (a[0] * a[8] - a[2] * a[6]) * id; o[5] = (a[2] * a[3] - a[0] * a[5]) * id;
    o[6] = c2 * id; o[7] = (a[1] * a[6] - a[0] * a[7]) * id; o[8] = (a[0] * a[4] - a[1] * a[3]) * id;
}

// 12x12 SPD inverse by Cholesky (one thread per body)
__global__ void k_prec_body(int NB, const double *__restrict__ Hb, const double *__restrict__ spd, const double *__restrict__ diagB,
                            double *__restrict__ dinvB)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= NB) return;
    double L[144];
    for (int q = 0; q < 144; ++q) L[q] = Hb[144 * (size_t)b + q] + spd[144 * (size_t)b + q] + diagB[144 * (size_t)b + q];
    for (int j = 0; j < 12; ++j) {
        double s = L[12 * j + j];
        for (int k = 0; k < j; ++k) s -= L[12 * j + k] * L[12 * j + k];
        double dj = sqrt(fmax(s, 1e-300));
        L[12 * j + j] = dj;
        for (int i = j + 1; i < 12; ++i) {
            double t = L[12 * i + j];
            for (int k = 0; k < j; ++k) t -= L[12 * i + k] * L[12 * j + k];
            L[12 * i + j] = t / dj;
        }
    }
    // inverse = L^-T L^-1, column by column
    double *o = dinvB + 144 * (size_t)b;
    for (int cidx = 0; cidx < 12; ++cidx) {
        double y[12];
        for (int i = 0; i < 12; ++i) {
            double t = (i == cidx) ? 1.0 : 0.0;
            for (int k = 0; k < i; ++k) t -= L[12 * i + k] * y[k];
            y[i] = t / L[12 * i + i];
        }
        for (int i = 11; i >= 0; --i) {
            double t = y[i];
            for (int k = i + 1; k < 12; ++k) t -= L[12 * k + i] * y[k];
            y[i] = t / L[12 * i + i];
        }
        for (int i = 0; i < 12; ++i) o[12 * i + cidx] = y[i];
    }
}

void build_preconditioner(ipc_ctx *c)
{
    Dev &D = c->d;
    hipLaunchKernelGGL(k_prec_fem, dim3(blocks_for(c->N)), dim3(BLOCK), 0, c->stream, c->N, D.node_kind.p, D.diag_slot.p, D.val.p,
                       D.fem_sp_diag.p, D.diagF.p, D.dinv.p);
    if (c->NB)
        hipLaunchKernelGGL(k_prec_body, dim3(blocks_for(c->NB, 64)), dim3(64), 0, c->stream, c->NB, D.Hb.p, D.body_sp_diag.p, D.diagB.p,
                           D.dinvB.p);
}

// ---------------------------------------------------------------------------
// PCG kernels
// ---------------------------------------------------------------------------
// x = 0, r = b, z = M^-1 r (FEM nodes), p = z; partials of b.b and r.z
__global__ void k_pcg_init(int N, const int *__restrict__ kind, const double *__restrict__ b, const double *__restrict__ dinv,
                           double *__restrict__ x, double *__restrict__ r, double *__restrict__ z, double *__restrict__ part_bb,
                           double *__restrict__ part_rz)
{
    int n = blockIdx.x * blockDim.x + threadIdx.x;
    double bb = 0.0, rz = 0.0;
    if (n < N) {
        d3 bv = ld3(b, n);
        st3(x, n, {0.0, 0.0, 0.0});
        st3(r, n, bv);
        bb = dt(bv, bv);
        d3 zv = {0, 0, 0};
        if (kind[n] == 0) {
            const double *M = dinv + 9 * (size_t)n;
            zv = {M[0] * bv.x + M[1] * bv.y + M[2] * bv.z, M[3] * bv.x + M[4] * bv.y + M[5] * bv.z, M[6] * bv.x + M[7] * bv.y + M[8] * bv.z};
            rz = dt(bv, zv);
        }
        st3(z, n, zv);
    }
    bb = wave_sum(bb); rz = wave_sum(rz);
    if ((threadIdx.x & (TILE - 1)) == 0 && n < N) { part_bb[n / TILE] = bb; part_rz[n / TILE] = rz; }
}

// z = M^-1 r on body nodes; partial r.z per body
__global__ void k_body_prec_apply(int NB, const int *__restrict__ node0, const int *__restrict__ bscene, const double *__restrict__ dinvB,
                                  const int *__restrict__ active, const double *__restrict__ r, double *__restrict__ z,
                                  double *__restrict__ part)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= NB) return;
    if (active && !active[bscene[b]]) { part[b] = 0.0; return; }
    int n0 = node0[b];
    const double *rv = r + 3 * (size_t)n0;
    const double *M = dinvB + 144 * (size_t)b;
    double rz = 0.0;
    for (int i = 0; i < 12; ++i) {
        double acc = 0.0;
        for (int j = 0; j < 12; ++j) acc += M[12 * i + j] * rv[j];
        z[3 * (size_t)n0 + i] = acc;
        rz += rv[i] * acc;
    }
    part[b] = rz;
}

// alpha = rz / pAp; x += alpha p; r -= alpha Ap; z = M^-1 r (FEM); partials r.z, r.r
__global__ void k_pcg_update(int N, const int *__restrict__ kind, const int *__restrict__ node_scene, const int *__restrict__ active,
                             const double *__restrict__ scal, const double *__restrict__ dinv, const double *__restrict__ p,
                             const double *__restrict__ Ap, double *__restrict__ x, double *__restrict__ r, double *__restrict__ z,
                             double *__restrict__ part_rz, double *__restrict__ part_rr)
{
    int n = blockIdx.x * blockDim.x + threadIdx.x;
    double rz = 0.0, rr = 0.0;
    if (n < N) {
        int s = node_scene[n];
        if (active[s]) {
            const double *S = scal + (size_t)s * NSLOT;
            double al = S[S_RZ] / S[S_PAP];
            d3 pv = ld3(p, n), av = ld3(Ap, n), xv = ld3(x, n), rv = ld3(r, n);
            xv = {xv.x + al * pv.x, xv.y + al * pv.y, xv.z + al * pv.z};
            rv = {rv.x - al * av.x, rv.y - al * av.y, rv.z - al * av.z};
            st3(x, n, xv);
            st3(r, n, rv);
            rr = dt(rv, rv);
            if (kind[n] == 0) {
                const double *M = dinv + 9 * (size_t)n;
                d3 zv = {M[0] * rv.x + M[1] * rv.y + M[2] * rv.z, M[3] * rv.x + M[4] * rv.y + M[5] * rv.z,
                         M[6] * rv.x + M[7] * rv.y + M[8] * rv.z};
                st3(z, n, zv);
                rz = dt(rv, zv);
            }
        }
    }
    rz = wave_sum(rz); rr = wave_sum(rr);
    if ((threadIdx.x & (TILE - 1)) == 0 && n < N) { part_rz[n / TILE] = rz; part_rr[n / TILE] = rr; }
}

// per scene: convergence test and beta
__global__ void k_pcg_scalars(int ns, double *__restrict__ scal, int *__restrict__ active, int *__restrict__ iters, int maxit_dummy)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= ns || !active[s]) return;
    double *S = scal + (size_t)s * NSLOT;
    iters[s] += 1;
    if (S[S_RR] <= S[S_ALPHA] || iters[s] >= (int)S[S_ACTIVE]) { active[s] = 0; return; }   // S_ALPHA: eta^2 b.b, S_ACTIVE: cap
    S[S_BETA] = S[S_RZ_NEW] / S[S_RZ];
    S[S_RZ] = S[S_RZ_NEW];
}

__global__ void k_pcg_p(int N, const int *__restrict__ node_scene, const int *__restrict__ active, const double *__restrict__ scal,
                        const double *__restrict__ z, double *__restrict__ p)
{
    int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    int s = node_scene[n];
    if (!active[s]) return;
    double be = scal[(size_t)s * NSLOT + S_BETA];
    d3 zv = ld3(z, n), pv = ld3(p, n);
    st3(p, n, {zv.x + be * pv.x, zv.y + be * pv.y, zv.z + be * pv.z});
}

__global__ void k_pcg_start(int ns, double *__restrict__ scal, int *__restrict__ active, int *__restrict__ iters, double eta,
                            const int *__restrict__ maxit, const int *__restrict__ want)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= ns) return;
    double *S = scal + (size_t)s * NSLOT;
    iters[s] = 0;
    double e = eta > 0.0 ? eta : S[S_ETA];
    S[S_ALPHA] = e * e * S[S_BB];
    S[S_ACTIVE] = (double)maxit[s];
    active[s] = (want ? want[s] : 1) && S[S_BB] > 0.0 ? 1 : 0;
}

void pcg_solve(ipc_ctx *c, const double *b, double *x, double eta, const int *want)
{
    Dev &D = c->d;
    hipStream_t st = c->stream;
    int ns = c->n_scenes;
    int *active = D.pcg_active.p;
    int *iters = D.pcg_iters.p;
    double *r = D.r.p, *z = D.z.p, *p = D.p.p, *Ap = D.q.p;
    hipLaunchKernelGGL(k_pcg_init, dim3(blocks_for(c->N)), dim3(BLOCK), 0, st, c->N, D.node_kind.p, b, D.dinv.p, x, r, z,
                       D.part_node.p, D.part_node2.p);
    if (c->NB)
        hipLaunchKernelGGL(k_body_prec_apply, dim3(blocks_for(c->NB, 64)), dim3(64), 0, st, c->NB, D.body_node0.p, D.body_scene.p,
                           D.dinvB.p, nullptr, r, z, D.body_part.p);
    {
        RedArgs a{};
        a.src[a.nsrc++] = src(D.part_node.p, seg_ptr(c, R_NODEW), 0, 0);
        a.slot = S_BB; a.acc = 0;
        reduce(c, a);
        RedArgs b2{};
        b2.src[b2.nsrc++] = src(D.part_node2.p, seg_ptr(c, R_NODEW), 0, 0);
        b2.src[b2.nsrc++] = src(c->NB ? D.body_part.p : nullptr, seg_ptr(c, R_BODY), 0, 0);
        b2.slot = S_RZ; b2.acc = 0;
        reduce(c, b2);
    }
    IPC_HIP(hipMemcpyAsync(p, z, 3 * (size_t)c->N * sizeof(double), hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(k_pcg_start, dim3(blocks_for(ns, 64)), dim3(64), 0, st, ns, D.scal.p, active, iters, eta, D.maxpcg.p, want);
    int maxit = 0;
    for (auto &S : c->sc) maxit = std::max(maxit, S.max_pcg);
    std::vector<int> hact(ns);
    const int check_every = 8;
    for (int it = 0; it < maxit; ++it) {
        hess_apply(c, p, Ap, active, true);
        prof_begin(c, IPC_K_PCG_UPDATE);
        hipLaunchKernelGGL(k_pcg_update, dim3(blocks_for(c->N)), dim3(BLOCK), 0, st, c->N, D.node_kind.p, D.node_scene.p, active,
                           D.scal.p, D.dinv.p, p, Ap, x, r, z, D.part_node.p, D.part_node2.p);
        prof_end(c, IPC_K_PCG_UPDATE, 240.0 * c->NFEM);
        if (c->NB)
            hipLaunchKernelGGL(k_body_prec_apply, dim3(blocks_for(c->NB, 64)), dim3(64), 0, st, c->NB, D.body_node0.p, D.body_scene.p,
                               D.dinvB.p, active, r, z, D.body_part.p);
        RedArgs a{};
        a.src[a.nsrc++] = src(D.part_node.p, seg_ptr(c, R_NODEW), 0, 0);
        a.src[a.nsrc++] = src(c->NB ? D.body_part.p : nullptr, seg_ptr(c, R_BODY), 0, 0);
        a.slot = S_RZ_NEW; a.acc = 0;
        reduce(c, a);
        RedArgs b2{};
        b2.src[b2.nsrc++] = src(D.part_node2.p, seg_ptr(c, R_NODEW), 0, 0);
        b2.slot = S_RR; b2.acc = 0;
        reduce(c, b2);
        hipLaunchKernelGGL(k_pcg_scalars, dim3(blocks_for(ns, 64)), dim3(64), 0, st, ns, D.scal.p, active, iters, 0);
        hipLaunchKernelGGL(k_pcg_p, dim3(blocks_for(c->N)), dim3(BLOCK), 0, st, c->N, D.node_scene.p, active, D.scal.p, z, p);
        if ((it + 1) % check_every == 0 || it + 1 == maxit) {
            IPC_HIP(hipMemcpyAsync(hact.data(), active, ns * sizeof(int), hipMemcpyDeviceToHost, st));
            IPC_HIP(hipStreamSynchronize(st));
            bool any = false;
            for (int s = 0; s < ns; ++s) any |= hact[s] != 0;
            if (!any) break;
        }
    }
}

} // namespace ipc
