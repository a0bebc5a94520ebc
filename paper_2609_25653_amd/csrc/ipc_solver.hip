// Linear algebra of the Newton step: deterministic per-scene reductions, the
// Hessian product (one block-CSR matrix over FEM vertices and affine-body
// nodes holding elasticity, inertia, orthogonality, springs and the contact
// blocks that fit its pattern, plus pair-local contact blocks for the rest),
// the block-Jacobi preconditioner (3x3 per FEM vertex, 12x12 per body) and a
// PCG that runs all scenes at once with per-scene scalars and flags.
#include <cmath>

#include "ipc_device.h"
#include "ipc_internal.h"
#include "ipc_kernels.h"

namespace ipc {

// ---------------------------------------------------------------------------
// reductions: one workgroup per scene, fixed-order strided sums and a tree.
// The post step runs in the same workgroup once the sums are known.
// ---------------------------------------------------------------------------
enum Post { POST_NONE = 0, POST_ALPHA = 1, POST_PCG = 2 };

__global__ void k_reduce(int ns, RedArgs a, double *__restrict__ scal, int post, int *__restrict__ active, int *__restrict__ iters)
{
    int s = blockIdx.x;
    __shared__ double sh[256];
    double total = 0.0, rest = 0.0;
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
        if (a.split == 0 || k < a.split) total = a.op ? fmax(total, v) : total + v;
        else rest += v;
    }
    if (threadIdx.x != 0) return;
    double *S = scal + (size_t)s * NSLOT;
    if (a.slot >= 0) S[a.slot] = a.acc ? (a.op ? fmax(S[a.slot], total) : S[a.slot] + total) : total;
    if (post == POST_ALPHA) {
        S[S_ALPHA] = S[S_RZ] / S[S_PAP];
        if (active[s] && !(S[S_PAP] > 0.0)) {   // not positive definite along p: stop here
            S[S_INDEF] = 1.0;
            S[S_ALPHA] = 0.0;
            active[s] = 0;
        }
    } else if (post == POST_PCG && active[s]) {
        S[S_RR] = rest;   // the sources after `split` carry r.r
        iters[s] += 1;
        if (S[S_RR] <= S[S_ETA2] || iters[s] >= (int)S[S_MAXIT]) { active[s] = 0; return; }
        S[S_BETA] = S[S_RZ_NEW] / S[S_RZ];
        S[S_RZ] = S[S_RZ_NEW];
    }
}

void reduce_post(ipc_ctx *c, const RedArgs &a, int post)
{
    hipLaunchKernelGGL(k_reduce, dim3(c->n_scenes), dim3(256), 0, c->stream, c->n_scenes, a, c->d.scal.p, post, c->d.pcg_active.p,
                       c->d.pcg_iters.p);
}

void reduce(ipc_ctx *c, const RedArgs &a) { reduce_post(c, a, POST_NONE); }

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
// Rows with at most LONG_ROW blocks: one thread per row.  Longer rows (affine
// body nodes carrying many springs): one wavefront per row, lanes striding
// over the blocks, then a wavefront reduction.  Same launch.
__global__ void __launch_bounds__(256) k_spmv(int N, int nshort_blocks, int nlong, const int *__restrict__ long_rows,
                                              const int *__restrict__ row_ptr, const int *__restrict__ col,
                                              const double *__restrict__ val, const double *__restrict__ v,
                                              const int *__restrict__ node_scene, const int *__restrict__ active,
                                              double *__restrict__ out)
{
    if ((int)blockIdx.x < nshort_blocks) {
        int n = blockIdx.x * blockDim.x + threadIdx.x;
        if (n >= N) return;
        int k0 = row_ptr[n], k1 = row_ptr[n + 1];
        if (k1 - k0 > LONG_ROW) return;
        double ax = 0.0, ay = 0.0, az = 0.0;
        if (!active || active[node_scene[n]]) {
            for (int k = k0; k < k1; ++k) {
                const double *B = val + 9 * (size_t)k;
                d3 w = ld3(v, col[k]);
                ax += B[0] * w.x + B[1] * w.y + B[2] * w.z;
                ay += B[3] * w.x + B[4] * w.y + B[5] * w.z;
                az += B[6] * w.x + B[7] * w.y + B[8] * w.z;
            }
        }
        st3(out, n, {ax, ay, az});
        return;
    }
    int w = (blockIdx.x - nshort_blocks) * (blockDim.x / TILE) + threadIdx.x / TILE;
    int lane = threadIdx.x & (TILE - 1);
    if (w >= nlong) return;
    int n = long_rows[w];
    double ax = 0.0, ay = 0.0, az = 0.0;
    if (!active || active[node_scene[n]]) {
        for (int k = row_ptr[n] + lane; k < row_ptr[n + 1]; k += TILE) {
            const double *B = val + 9 * (size_t)k;
            d3 x = ld3(v, col[k]);
            ax += B[0] * x.x + B[1] * x.y + B[2] * x.z;
            ay += B[3] * x.x + B[4] * x.y + B[5] * x.z;
            az += B[6] * x.x + B[7] * x.y + B[8] * x.z;
        }
    }
    ax = wave_sum(ax); ay = wave_sum(ay); az = wave_sum(az);
    if (lane == 0) st3(out, n, {ax, ay, az});
}

// p.Ap per wavefront of nodes (the per-scene sum and alpha follow in k_reduce;
// summing in the producer's last workgroup would need a device-scope release
// fence per workgroup, which writes back the XCD's L2 and costs more than the
// extra launch)
__global__ void k_dot(int N, const int *__restrict__ node_scene, const int *__restrict__ active, const double *__restrict__ a,
                      const double *__restrict__ b, double *__restrict__ part)
{
    int n = blockIdx.x * blockDim.x + threadIdx.x;
    double s = 0.0;
    if (n < N && active[node_scene[n]]) s = dt(ld3(a, n), ld3(b, n));
    s = wave_sum(s);
    if ((threadIdx.x & (TILE - 1)) == 0 && n < N) part[n / TILE] = s;
}

// Algorithmic bytes of one block-CSR product: 76 per stored block (9 doubles
// + column index), 4 per row pointer, and 24 read plus 24 written per
// non-padding node.
double spmv_bytes(const ipc_ctx *c) { return 76.0 * c->nnzb + 4.0 * (c->N + 1) + 48.0 * (c->NFEM + 4.0 * c->NB); }

void spmv_only(ipc_ctx *c, const double *v, double *out)
{
    Dev &D = c->d;
    int nshort = blocks_for(c->N);
    int nlongb = (c->n_long + BLOCK / TILE - 1) / (BLOCK / TILE);
    hipLaunchKernelGGL(k_spmv, dim3(nshort + nlongb), dim3(BLOCK), 0, c->stream, c->N, nshort, c->n_long, D.long_rows.p, D.row_ptr.p,
                       D.col.p, D.val.p, v, D.node_scene.p, nullptr, out);
}

void hess_apply(ipc_ctx *c, const double *v, double *out, const int *active, bool pap)
{
    Dev &D = c->d;
    hipStream_t st = c->stream;
    int nshort = blocks_for(c->N);
    int nlongb = (c->n_long + BLOCK / TILE - 1) / (BLOCK / TILE);
    prof_begin(c, IPC_K_SPMV);
    hipLaunchKernelGGL(k_spmv, dim3(nshort + nlongb), dim3(BLOCK), 0, st, c->N, nshort, c->n_long, D.long_rows.p, D.row_ptr.p, D.col.p,
                       D.val.p, v, D.node_scene.p, active, out);
    prof_end(c, IPC_K_SPMV, spmv_bytes(c));
    prof_begin(c, IPC_K_CONTACT_APPLY);
    launch_contact_apply(c, v, out, active, nullptr, nullptr);
    prof_end(c, IPC_K_CONTACT_APPLY, 0.0);
    if (pap) {
        hipLaunchKernelGGL(k_dot, dim3(blocks_for(c->N)), dim3(BLOCK), 0, st, c->N, D.node_scene.p, active, v, out, D.part_node.p);
        RedArgs a{};
        a.src[a.nsrc++] = src(D.part_node.p, seg_ptr(c, R_NODEW), 0, 0);
        a.slot = S_PAP;
        reduce_post(c, a, POST_ALPHA);
    }
}

// ---------------------------------------------------------------------------
// block-Jacobi preconditioner: diagonal blocks of the matrix plus the
// diagonal blocks of the pair-local contact terms
// ---------------------------------------------------------------------------
__global__ void k_prec_fem(int N, const int *__restrict__ kind, const int *__restrict__ diag_slot, const double *__restrict__ val,
                           const double *__restrict__ diagF, double *__restrict__ dinv)
{
    int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    double *o = dinv + 9 * (size_t)n;
    if (kind[n] != 0) { for (int q = 0; q < 9; ++q) o[q] = 0.0; return; }
    double a[9];
    const double *B = val + 9 * (size_t)diag_slot[n];
    for (int q = 0; q < 9; ++q) a[q] = B[q] + diagF[9 * (size_t)n + q];
    double c0 = a[4] * a[8] - a[5] * a[7], c1 = a[5] * a[6] - a[3] * a[8], c2 = a[3] * a[7] - a[4] * a[6];
    double det = a[0] * c0 + a[1] * c1 + a[2] * c2;
    double id = 1.0 / det;
    o[0] = c0 * id; o[1] = (a[2] * a[7] - a[1] * a[8]) * id; o[2] = (a[1] * a[5] - a[2] * a[4]) * id;
    o[3] = c1 * id; o[4] = (a[0] * a[8] - a[2] * a[6]) * id; o[5] = (a[2] * a[3] - a[0] * a[5]) * id;
    o[6] = c2 * id; o[7] = (a[1] * a[6] - a[0] * a[7]) * id; o[8] = (a[0] * a[4] - a[1] * a[3]) * id;
}

// 12x12 SPD inverse by Cholesky (one thread per body)
__global__ void k_prec_body(int NB, const int *__restrict__ bslot, const double *__restrict__ val, const double *__restrict__ diagB,
                            double *__restrict__ dinvB)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= NB) return;
    double L[144];
    for (int ca = 0; ca < 4; ++ca)
        for (int cb = 0; cb < 4; ++cb) {
            const double *B = val + 9 * (size_t)bslot[16 * (size_t)b + 4 * ca + cb];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    int r = 3 * ca + i, cc = 3 * cb + j;
                    L[12 * r + cc] = B[3 * i + j] + diagB[144 * (size_t)b + 12 * r + cc];
                }
        }
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
                       D.diagF.p, D.dinv.p);
    if (c->NB)
        hipLaunchKernelGGL(k_prec_body, dim3(blocks_for(c->NB, 64)), dim3(64), 0, c->stream, c->NB, D.bslot.p, D.val.p, D.diagB.p,
                           D.dinvB.p);
}

// ---------------------------------------------------------------------------
// PCG kernels
// ---------------------------------------------------------------------------
// x = 0, r = b, z = M^-1 r (FEM nodes); partials of b.b and r.z
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

// x += alpha p; r -= alpha Ap; z = M^-1 r with partials of r.z and r.r.
// Workgroups [0, nnode_blocks) take FEM and padding nodes, one thread per
// node; the rest take one affine body per thread (its 4 nodes and its 12x12
// inverse block).  The last workgroup tests convergence and forms beta.
__global__ void k_pcg_update2(int N, int nnode_blocks, int NB, const int *__restrict__ kind, const int *__restrict__ node_scene,
                              int *__restrict__ active, double *__restrict__ scal, const double *__restrict__ dinv,
                              const double *__restrict__ dinvB, const int *__restrict__ body_node0, const int *__restrict__ body_scene,
                              const double *__restrict__ p, const double *__restrict__ Ap, double *__restrict__ x, double *__restrict__ r,
                              double *__restrict__ z, double *__restrict__ part_rz, double *__restrict__ part_rr,
                              double *__restrict__ bpart_rz, double *__restrict__ bpart_rr)
{
    if ((int)blockIdx.x < nnode_blocks) {
        int n = blockIdx.x * blockDim.x + threadIdx.x;
        double rz = 0.0, rr = 0.0;
        if (n < N && kind[n] != 1) {
            int s = node_scene[n];
            if (active[s]) {
                double al = scal[(size_t)s * NSLOT + S_ALPHA];
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
    } else {
        int b = (blockIdx.x - nnode_blocks) * blockDim.x + threadIdx.x;
        if (b < NB) {
            double rz = 0.0, rr = 0.0;
            int s = body_scene[b];
            if (active[s]) {
                double al = scal[(size_t)s * NSLOT + S_ALPHA];
                int n0 = body_node0[b];
                double rv[12];
                for (int i = 0; i < 12; ++i) {
                    size_t q = 3 * (size_t)n0 + i;
                    x[q] += al * p[q];
                    rv[i] = r[q] - al * Ap[q];
                    r[q] = rv[i];
                    rr += rv[i] * rv[i];
                }
                const double *M = dinvB + 144 * (size_t)b;
                for (int i = 0; i < 12; ++i) {
                    double acc = 0.0;
                    for (int j = 0; j < 12; ++j) acc += M[12 * i + j] * rv[j];
                    z[3 * (size_t)n0 + i] = acc;
                    rz += rv[i] * acc;
                }
            }
            bpart_rz[b] = rz;
            bpart_rr[b] = rr;
        }
    }
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
    S[S_ETA2] = e * e * S[S_BB];
    S[S_MAXIT] = (double)maxit[s];
    S[S_INDEF] = 0.0;
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
        a.src[a.nsrc] = src(D.part_node.p, seg_ptr(c, R_NODEW), 0, 0); a.slots[a.nsrc++] = S_BB;
        reduce(c, a);
        RedArgs b2{};
        b2.src[b2.nsrc++] = src(D.part_node2.p, seg_ptr(c, R_NODEW), 0, 0);
        b2.src[b2.nsrc++] = src(c->NB ? D.body_part.p : nullptr, seg_ptr(c, R_BODY), 0, 0);
        b2.slot = S_RZ;
        reduce(c, b2);
    }
    IPC_HIP(hipMemcpyAsync(p, z, 3 * (size_t)c->N * sizeof(double), hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(k_pcg_start, dim3(blocks_for(ns, 64)), dim3(64), 0, st, ns, D.scal.p, active, iters, eta, D.maxpcg.p, want);
    int maxit = 0;
    for (auto &S : c->sc) maxit = std::max(maxit, S.max_pcg);
    std::vector<int> hact(ns);
    // one PCG iteration; every kernel skips scenes whose flag is down, so extra
    // iterations after convergence change nothing
    auto iteration = [&]() {
        hipStream_t s2 = c->stream;
        hess_apply(c, p, Ap, active, true);
        int nnb = blocks_for(c->N), nbb = blocks_for(c->NB);
        prof_begin(c, IPC_K_PCG_UPDATE);
        hipLaunchKernelGGL(k_pcg_update2, dim3(nnb + nbb), dim3(BLOCK), 0, s2, c->N, nnb, c->NB, D.node_kind.p, D.node_scene.p, active,
                           D.scal.p, D.dinv.p, D.dinvB.p, D.body_node0.p, D.body_scene.p, p, Ap, x, r, z, D.part_node.p,
                           D.part_node2.p, D.body_part.p, D.body_part2.p);
        prof_end(c, IPC_K_PCG_UPDATE, 240.0 * c->NFEM);
        RedArgs a{};
        a.src[a.nsrc] = src(D.part_node.p, seg_ptr(c, R_NODEW), 0, 0); a.slots[a.nsrc++] = -1;
        a.src[a.nsrc] = src(c->NB ? D.body_part.p : nullptr, seg_ptr(c, R_BODY), 0, 0); a.slots[a.nsrc++] = -1;
        a.slot = S_RZ_NEW;
        a.split = 2;   // r.z = the first two sources; r.r = the last two
        a.src[a.nsrc] = src(D.part_node2.p, seg_ptr(c, R_NODEW), 0, 0); a.slots[a.nsrc++] = -1;
        a.src[a.nsrc] = src(c->NB ? D.body_part2.p : nullptr, seg_ptr(c, R_BODY), 0, 0); a.slots[a.nsrc++] = -1;
        reduce_post(c, a, POST_PCG);
        hipLaunchKernelGGL(k_pcg_p, dim3(blocks_for(c->N)), dim3(BLOCK), 0, s2, c->N, D.node_scene.p, active, D.scal.p, z, p);
    };
    auto any_active = [&]() {
        IPC_HIP(hipMemcpyAsync(hact.data(), active, ns * sizeof(int), hipMemcpyDeviceToHost, st));
        IPC_HIP(hipStreamSynchronize(st));
        bool any = false;
        for (int s = 0; s < ns; ++s) any |= hact[s] != 0;
        return any;
    };
    const int K = 8;   // iterations per convergence check
    if (c->use_graphs && !c->prof) {
        // Capture K iterations once per solve on the context's capture stream
        // (the caller's stream may be the null stream, which cannot capture)
        // and replay the graph on the context's stream.
        IPC_HIP(hipStreamSynchronize(st));
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        c->stream = c->cap_stream;
        hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            for (int k = 0; k < K; ++k) iteration();
            e = hipStreamEndCapture(c->cap_stream, &graph);
        }
        c->stream = st;
        IPC_HIP(e);
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        IPC_HIP(e);
        hipError_t le = hipSuccess;
        for (int it = 0; it < maxit; it += K) {
            le = hipGraphLaunch(exec, st);
            if (le != hipSuccess) break;
            if (!any_active()) break;
        }
        (void)hipGraphExecDestroy(exec);
        IPC_HIP(le);
        return;
    }
    for (int it = 0; it < maxit; ++it) {
        iteration();
        if (((it + 1) % K == 0 || it + 1 == maxit) && !any_active()) break;
    }
}

} // namespace ipc
