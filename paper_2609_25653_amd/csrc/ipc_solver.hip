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
// reductions: one workgroup per scene.  Each thread sums a fixed strided
// subset of a source's partials, wavefront shuffles and a 4-entry LDS step
// combine them in a fixed order, and the post step runs in the same
// workgroup once the sums are known.
// ---------------------------------------------------------------------------
enum Post { POST_NONE = 0, POST_CG_FIRST = 1, POST_CG = 2 };

__global__ void __launch_bounds__(256) k_reduce(int ns, RedArgs a, double *__restrict__ scal, int post, int *__restrict__ active,
                                                int *__restrict__ iters)
{
    int s = blockIdx.x;
    __shared__ double sh[8][BLOCK / TILE];
    int wave = threadIdx.x / TILE, lane = threadIdx.x & (TILE - 1);
    // all loads first (independent, in flight together), then the shuffles:
    // the first 4 strided partials of every source are loaded unconditionally
    // (predicated), the rest (scenes with more than 1024 partials) in a loop
    double part[8];
    // the post step's inputs, fetched while the partials are in flight
    double S0 = 0.0, S1 = 0.0, Sg = 0.0, Se = 0.0, Sm = 0.0;
    int act = 0, it0 = 0;
    if (threadIdx.x == 0 && post != POST_NONE) {
        const double *Sp = scal + (size_t)s * NSLOT;
        S0 = Sp[S_RZ]; S1 = Sp[S_ALPHA]; Sg = Sp[S_RZ_NEW]; Se = Sp[S_ETA2]; Sm = Sp[S_MAXIT];
        act = active[s]; it0 = iters[s];
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        part[k] = 0.0;
        if (k >= a.nsrc) continue;
        const RedSrc &r = a.src[k];
        if (!r.v) continue;
        int lo = r.seg[s] - r.base, hi = r.seg[s + 1] - r.base;
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            int i = lo + (int)threadIdx.x + u * BLOCK;
            v[u] = i < hi ? r.v[r.off + i] : (a.op ? -INFINITY : 0.0);
        }
        double acc = a.op ? fmax(fmax(v[0], v[1]), fmax(v[2], v[3])) : (v[0] + v[1]) + (v[2] + v[3]);
        for (int i = lo + (int)threadIdx.x + 4 * BLOCK; i < hi; i += BLOCK) {
            double x = r.v[r.off + i];
            acc = a.op ? fmax(acc, x) : acc + x;
        }
        part[k] = a.op ? fmax(acc, 0.0) : acc;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        if (k >= a.nsrc) break;
        double v = a.op ? wave_max(part[k]) : wave_sum(part[k]);
        if (lane == 0) sh[k][wave] = v;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double *S = scal + (size_t)s * NSLOT;
    double tot[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < a.nsrc; ++k) {
        double v = sh[k][0];
        for (int w = 1; w < BLOCK / TILE; ++w) v = a.op ? fmax(v, sh[k][w]) : v + sh[k][w];
        if (a.slots[k] >= 0) S[a.slots[k]] = v;
        int g = a.grp[k];
        if (g >= 0) tot[g] = a.op ? fmax(tot[g], v) : tot[g] + v;
    }
    if (a.slot >= 0) S[a.slot] = a.acc ? (a.op ? fmax(S[a.slot], tot[0]) : S[a.slot] + tot[0]) : tot[0];
    if (a.slot1 >= 0) S[a.slot1] = tot[1];
    if (a.slot2 >= 0) S[a.slot2] = tot[2];
    if (post == POST_NONE || !act) return;
    // Conjugate gradients with one reduction per iteration (Chronopoulos and
    // Gear): with gamma = r.z and delta = z.Az of the current residual,
    //   beta = gamma / gamma_old,  p.Ap = delta - beta gamma / alpha_old,
    //   alpha = gamma / p.Ap.
    // POST_CG: group 0 = gamma, 1 = delta, 2 = r.r; POST_CG_FIRST: group 1 =
    // delta, gamma from the set-up reduction.
    double gam = post == POST_CG ? tot[0] : Sg, del = tot[1], be = 0.0;
    if (post == POST_CG) {
        iters[s] = it0 + 1;
        if (tot[2] <= Se || it0 + 1 >= (int)Sm) { active[s] = 0; return; }
        be = gam / S0;
        del -= be * gam / S1;
    }
    if (!(del > 0.0)) {   // not positive definite along the search direction: stop here
        S[S_INDEF] = 1.0;
        active[s] = 0;
        return;
    }
    S[S_BETA] = be;
    S[S_ALPHA] = gam / del;
    S[S_RZ] = gam;
}

void reduce_post(ipc_ctx *c, const RedArgs &a, int post)
{
    hipLaunchKernelGGL(k_reduce, dim3(c->n_scenes), dim3(BLOCK), 0, c->stream, c->n_scenes, a, c->d.scal.p, post, c->d.pcg_active.p,
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
// Hessian product out = H v: the block-CSR matrix (elasticity, inertia,
// orthogonality, springs and the contact blocks merged at assembly) plus the
// row-sorted pair-local contact blocks.
//
// One workgroup per tile of 64 rows, L lanes per row (workgroup 64 L): the L
// lanes of a row read consecutive blocks (coalesced 72 B runs), and a 44k-row
// matrix still yields L x 700 wavefronts, enough to hide the gather latency
// of v.  The row's partial sums meet through shuffles inside the lane group.
// Rows with more than LONG_ROW blocks in all (affine-body nodes with many
// springs or contacts) go to extra workgroups, one workgroup per row.  With
// `part`, also v . out per tile (long rows into part_long): the dot product
// the conjugate-gradient step needs, in the same pass.  L is chosen by the
// autotuner among 1, 2, 4, 8 and 16.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void acc_block(const double *__restrict__ B, d3 w, double &ax, double &ay, double &az)
{
    ax += B[0] * w.x + B[1] * w.y + B[2] * w.z;
    ay += B[3] * w.x + B[4] * w.y + B[5] * w.z;
    az += B[6] * w.x + B[7] * w.y + B[8] * w.z;
}

template <int L>
__global__ void __launch_bounds__(64 * L) k_spmv(int N, int ntiles, int nlong, const int *__restrict__ long_rows,
                                                 const int *__restrict__ row_ptr, const int *__restrict__ col,
                                                 const double *__restrict__ val, const int *__restrict__ dptr,
                                                 const int *__restrict__ dcol, const double *__restrict__ dval,
                                                 const double *__restrict__ v, const int *__restrict__ node_scene,
                                                 const int *__restrict__ active, double *__restrict__ out,
                                                 double *__restrict__ part, double *__restrict__ part_long)
{
    constexpr int NW = L;   // wavefronts per workgroup
    int lane = threadIdx.x & (TILE - 1);
    if ((int)blockIdx.x < ntiles) {
        __shared__ double sh[NW];
        int sub = threadIdx.x % L;
        int n = blockIdx.x * TILE + threadIdx.x / L;
        double ax = 0.0, ay = 0.0, az = 0.0;
        bool mine = false, on = false;
        if (n < N) {
            int k0 = row_ptr[n], k1 = row_ptr[n + 1], d0 = dptr[n], d1 = dptr[n + 1];
            if ((k1 - k0) + (d1 - d0) <= LONG_ROW) {
                mine = true;
                on = !active || active[node_scene[n]];
                if (on) {
                    for (int k = k0 + sub; k < k1; k += L) acc_block(val + 9 * (size_t)k, ld3(v, col[k]), ax, ay, az);
                    for (int k = d0 + sub; k < d1; k += L) acc_block(dval + 9 * (size_t)k, ld3(v, dcol[k]), ax, ay, az);
                }
            }
        }
#pragma unroll
        for (int o = L / 2; o > 0; o >>= 1) {
            ax += __shfl_xor(ax, o, TILE);
            ay += __shfl_xor(ay, o, TILE);
            az += __shfl_xor(az, o, TILE);
        }
        double dot = 0.0;
        if (mine && sub == 0) {
            st3(out, n, {ax, ay, az});
            if (part && on) dot = dt(ld3(v, n), {ax, ay, az});
        }
        if (part) {
            dot = wave_sum(dot);
            if (lane == 0) sh[threadIdx.x / TILE] = dot;
            __syncthreads();
            if (threadIdx.x == 0) {
                double t = sh[0];
                for (int q = 1; q < NW; ++q) t += sh[q];
                part[blockIdx.x] = t;
            }
        }
        return;
    }
    // one workgroup per long row: all 64 L lanes stride over its blocks
    __shared__ double shl[3][NW];
    int w = (int)blockIdx.x - ntiles;
    if (w >= nlong) return;
    int n = long_rows[w];
    double ax = 0.0, ay = 0.0, az = 0.0;
    bool on = !active || active[node_scene[n]];
    if (on) {
        for (int k = row_ptr[n] + (int)threadIdx.x; k < row_ptr[n + 1]; k += 64 * L) acc_block(val + 9 * (size_t)k, ld3(v, col[k]), ax, ay, az);
        for (int k = dptr[n] + (int)threadIdx.x; k < dptr[n + 1]; k += 64 * L) acc_block(dval + 9 * (size_t)k, ld3(v, dcol[k]), ax, ay, az);
    }
    ax = wave_sum(ax); ay = wave_sum(ay); az = wave_sum(az);
    if (lane == 0) { shl[0][threadIdx.x / TILE] = ax; shl[1][threadIdx.x / TILE] = ay; shl[2][threadIdx.x / TILE] = az; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < NW; ++q) { ax += shl[0][q]; ay += shl[1][q]; az += shl[2][q]; }
        st3(out, n, {ax, ay, az});
        if (part_long) part_long[w] = on ? dt(ld3(v, n), {ax, ay, az}) : 0.0;
    }
}

// Algorithmic bytes of one product: 76 per stored block (9 doubles + column
// index) of the matrix and of the pair-local list, 4 per row pointer of each,
// and 24 read plus 24 written per non-padding node.
double spmv_bytes(const ipc_ctx *c)
{
    return 76.0 * ((double)c->nnzb + (double)c->n_dyn) + 8.0 * (c->N + 1) + 48.0 * (c->NFEM + 4.0 * c->NB);
}

static void spmv_launch(ipc_ctx *c, int L, const double *v, double *out, const int *active, double *part)
{
    Dev &D = c->d;
    int ntiles = (c->N + TILE - 1) / TILE;
    dim3 grid(ntiles + c->n_long), blk(64 * L);
    double *pl = part ? D.part_long.p : nullptr;
#define IPC_SPMV(LL) hipLaunchKernelGGL(k_spmv<LL>, grid, blk, 0, c->stream, c->N, ntiles, c->n_long, D.long_rows.p, D.row_ptr.p, D.col.p, \
                                        D.val.p, D.dyn_ptr.p, D.dyn_col.p, D.dyn_val.p, v, D.node_scene.p, active, out, part, pl)
    switch (L) {
    case 1: IPC_SPMV(1); break;
    case 2: IPC_SPMV(2); break;
    case 4: IPC_SPMV(4); break;
    case 8: IPC_SPMV(8); break;
    default: IPC_SPMV(16); break;
    }
#undef IPC_SPMV
}

void hess_apply(ipc_ctx *c, const double *v, double *out, const int *active, double *part)
{
    prof_begin(c, IPC_K_SPMV);
    spmv_launch(c, c->spmv_lanes, v, out, active, part);
    prof_end(c, IPC_K_SPMV, spmv_bytes(c));
}

// Time every lane count on the current matrix (reps back-to-back launches
// each, HIP events on the context's stream) and keep the fastest.
void autotune_spmv(ipc_ctx *c, int reps, double *us)
{
    Dev &D = c->d;
    const int Ls[5] = {1, 2, 4, 8, 16};
    hipEvent_t e0, e1;
    IPC_HIP(hipEventCreate(&e0));
    IPC_HIP(hipEventCreate(&e1));
    double best = 1e300;
    int bestL = c->spmv_lanes;
    for (int i = 0; i < 5; ++i) {
        spmv_launch(c, Ls[i], D.p.p, D.q.p, nullptr, nullptr);
        IPC_HIP(hipEventRecord(e0, c->stream));
        for (int k = 0; k < reps; ++k) spmv_launch(c, Ls[i], D.p.p, D.q.p, nullptr, nullptr);
        IPC_HIP(hipEventRecord(e1, c->stream));
        IPC_HIP(hipEventSynchronize(e1));
        float ms = 0.0f;
        IPC_HIP(hipEventElapsedTime(&ms, e0, e1));
        double t = 1e3 * ms / reps;
        if (us) us[i] = t;
        if (t < best) { best = t; bestL = Ls[i]; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->spmv_lanes = bestL;
}

// ---------------------------------------------------------------------------
// block-Jacobi preconditioner: diagonal blocks of the matrix plus the
// pair-local contact blocks on the diagonal (found in the row-sorted list)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int dyn_find(const int *__restrict__ dptr, const int *__restrict__ dcol, int r, int cc)
{
    int lo = dptr[r], hi = dptr[r + 1];
    while (lo < hi) {
        int m = (lo + hi) >> 1;
        if (dcol[m] < cc) lo = m + 1; else hi = m;
    }
    return (lo < dptr[r + 1] && dcol[lo] == cc) ? lo : -1;
}

__global__ void k_prec_fem(int N, const int *__restrict__ kind, const int *__restrict__ diag_slot, const double *__restrict__ val,
                           const int *__restrict__ dptr, const int *__restrict__ dcol, const double *__restrict__ dval,
                           double *__restrict__ dinv)
{
    int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    double *o = dinv + 9 * (size_t)n;
    if (kind[n] != 0) { for (int q = 0; q < 9; ++q) o[q] = 0.0; return; }
    double a[9];
    const double *B = val + 9 * (size_t)diag_slot[n];
    for (int q = 0; q < 9; ++q) a[q] = B[q];
    int k = dyn_find(dptr, dcol, n, n);
    if (k >= 0) for (int q = 0; q < 9; ++q) a[q] += dval[9 * (size_t)k + q];
    double c0 = a[4] * a[8] - a[5] * a[7], c1 = a[5] * a[6] - a[3] * a[8], c2 = a[3] * a[7] - a[4] * a[6];
    double det = a[0] * c0 + a[1] * c1 + a[2] * c2;
    double id = 1.0 / det;
    o[0] = c0 * id; o[1] = (a[2] * a[7] - a[1] * a[8]) * id; o[2] = (a[1] * a[5] - a[2] * a[4]) * id;
    o[3] = c1 * id; o[4] = (a[0] * a[8] - a[2] * a[6]) * id; o[5] = (a[2] * a[3] - a[0] * a[5]) * id;
    o[6] = c2 * id; o[7] = (a[1] * a[6] - a[0] * a[7]) * id; o[8] = (a[0] * a[4] - a[1] * a[3]) * id;
}

// 12x12 SPD inverse by Cholesky (one thread per body)
__global__ void k_prec_body(int NB, const int *__restrict__ bslot, const int *__restrict__ node0, const double *__restrict__ val,
                            const int *__restrict__ dptr, const int *__restrict__ dcol, const double *__restrict__ dval,
                            double *__restrict__ dinvB)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= NB) return;
    double L[144];
    int n0 = node0[b];
    for (int ca = 0; ca < 4; ++ca)
        for (int cb = 0; cb < 4; ++cb) {
            const double *B = val + 9 * (size_t)bslot[16 * (size_t)b + 4 * ca + cb];
            int k = dyn_find(dptr, dcol, n0 + ca, n0 + cb);
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    double v = B[3 * i + j];
                    if (k >= 0) v += dval[9 * (size_t)k + 3 * i + j];
                    L[12 * (3 * ca + i) + 3 * cb + j] = v;
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
                       D.dyn_ptr.p, D.dyn_col.p, D.dyn_val.p, D.dinv.p);
    if (c->NB)
        hipLaunchKernelGGL(k_prec_body, dim3(blocks_for(c->NB, 64)), dim3(64), 0, c->stream, c->NB, D.bslot.p, D.body_node0.p, D.val.p,
                           D.dyn_ptr.p, D.dyn_col.p, D.dyn_val.p,
                           D.dinvB.p);
}

// ---------------------------------------------------------------------------
// PCG kernels (preconditioned conjugate gradients in the single-reduction
// form of Chronopoulos and Gear: besides p it carries s = A p, so that one
// product w = A z and one per-scene reduction per iteration suffice)
// ---------------------------------------------------------------------------
// x = 0, r = b, p = s = 0, z = M^-1 r (FEM nodes); partials of b.b and r.z
__global__ void k_pcg_init(int N, const int *__restrict__ kind, const double *__restrict__ b, const double *__restrict__ dinv,
                           double *__restrict__ x, double *__restrict__ r, double *__restrict__ z, double *__restrict__ p,
                           double *__restrict__ s, double *__restrict__ part_bb, double *__restrict__ part_rz)
{
    int n = blockIdx.x * blockDim.x + threadIdx.x;
    double bb = 0.0, rz = 0.0;
    if (n < N) {
        d3 bv = ld3(b, n);
        st3(x, n, {0.0, 0.0, 0.0});
        st3(p, n, {0.0, 0.0, 0.0});
        st3(s, n, {0.0, 0.0, 0.0});
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
__global__ void k_body_prec_apply(int NB, const int *__restrict__ node0, const double *__restrict__ dinvB, const double *__restrict__ r,
                                  double *__restrict__ z, double *__restrict__ part)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= NB) return;
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

// p = z + beta p; s = w + beta s; x += alpha p; r -= alpha s; z = M^-1 r,
// with partials of r.z and r.r.  Workgroups [0, nnode_blocks) take FEM and
// padding nodes, one thread per node; the rest take one affine body per
// thread (its 4 nodes and its 12x12 inverse block).
__global__ void k_pcg_update(int N, int nnode_blocks, int NB, const int *__restrict__ kind, const int *__restrict__ node_scene,
                             const int *__restrict__ active, const double *__restrict__ scal, const double *__restrict__ dinv,
                             const double *__restrict__ dinvB, const int *__restrict__ body_node0, const int *__restrict__ body_scene,
                             const double *__restrict__ w, double *__restrict__ p, double *__restrict__ s, double *__restrict__ x,
                             double *__restrict__ r, double *__restrict__ z, double *__restrict__ part_rz, double *__restrict__ part_rr,
                             double *__restrict__ bpart_rz, double *__restrict__ bpart_rr)
{
    if ((int)blockIdx.x < nnode_blocks) {
        int n = blockIdx.x * blockDim.x + threadIdx.x;
        double rz = 0.0, rr = 0.0;
        if (n < N && kind[n] == 0) {
            int sc = node_scene[n];
            if (active[sc]) {
                const double *S = scal + (size_t)sc * NSLOT;
                double al = S[S_ALPHA], be = S[S_BETA];
                d3 zv = ld3(z, n), pv = ld3(p, n), wv = ld3(w, n), sv = ld3(s, n), xv = ld3(x, n), rv = ld3(r, n);
                pv = {zv.x + be * pv.x, zv.y + be * pv.y, zv.z + be * pv.z};
                sv = {wv.x + be * sv.x, wv.y + be * sv.y, wv.z + be * sv.z};
                xv = {xv.x + al * pv.x, xv.y + al * pv.y, xv.z + al * pv.z};
                rv = {rv.x - al * sv.x, rv.y - al * sv.y, rv.z - al * sv.z};
                const double *M = dinv + 9 * (size_t)n;
                zv = {M[0] * rv.x + M[1] * rv.y + M[2] * rv.z, M[3] * rv.x + M[4] * rv.y + M[5] * rv.z, M[6] * rv.x + M[7] * rv.y + M[8] * rv.z};
                st3(p, n, pv); st3(s, n, sv); st3(x, n, xv); st3(r, n, rv); st3(z, n, zv);
                rr = dt(rv, rv);
                rz = dt(rv, zv);
            }
        }
        rz = wave_sum(rz); rr = wave_sum(rr);
        if ((threadIdx.x & (TILE - 1)) == 0 && n < N) { part_rz[n / TILE] = rz; part_rr[n / TILE] = rr; }
    } else {
        int b = (blockIdx.x - nnode_blocks) * blockDim.x + threadIdx.x;
        if (b >= NB) return;
        double rz = 0.0, rr = 0.0;
        int sc = body_scene[b];
        if (active[sc]) {
            const double *S = scal + (size_t)sc * NSLOT;
            double al = S[S_ALPHA], be = S[S_BETA];
            size_t o = 3 * (size_t)body_node0[b];
            double rv[12];
            for (int i = 0; i < 12; ++i) {
                double pi = z[o + i] + be * p[o + i];
                double si = w[o + i] + be * s[o + i];
                p[o + i] = pi;
                s[o + i] = si;
                x[o + i] += al * pi;
                rv[i] = r[o + i] - al * si;
                r[o + i] = rv[i];
                rr += rv[i] * rv[i];
            }
            const double *M = dinvB + 144 * (size_t)b;
            for (int i = 0; i < 12; ++i) {
                double acc = 0.0;
                for (int j = 0; j < 12; ++j) acc += M[12 * i + j] * rv[j];
                z[o + i] = acc;
                rz += rv[i] * acc;
            }
        }
        bpart_rz[b] = rz;
        bpart_rr[b] = rr;
    }
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

// Bytes one update pass moves: 6 node vectors read and 5 written (24 B
// each) plus the 3x3 inverse block per FEM vertex; 12x12 blocks per body.
static double update_bytes(const ipc_ctx *c) { return (264.0 + 72.0) * c->NFEM + (4 * 264.0 + 1152.0) * c->NB; }

void pcg_solve(ipc_ctx *c, const double *b, double *x, double eta, const int *want)
{
    Dev &D = c->d;
    hipStream_t st = c->stream;
    int ns = c->n_scenes;
    int *active = D.pcg_active.p;
    double *r = D.r.p, *z = D.z.p, *p = D.p.p, *s = D.q.p, *w = D.w.p;
    D.part_node3.alloc(c->N / TILE + 1);
    D.part_long.alloc(c->n_long + 1);
    hipLaunchKernelGGL(k_pcg_init, dim3(blocks_for(c->N)), dim3(BLOCK), 0, st, c->N, D.node_kind.p, b, D.dinv.p, x, r, z, p, s,
                       D.part_node.p, D.part_node2.p);
    if (c->NB)
        hipLaunchKernelGGL(k_body_prec_apply, dim3(blocks_for(c->NB, 64)), dim3(64), 0, st, c->NB, D.body_node0.p, D.dinvB.p, r, z,
                           D.body_part.p);
    {
        RedArgs a{};
        a.src[a.nsrc] = src(D.part_node.p, seg_ptr(c, R_NODEW), 0, 0); a.grp[a.nsrc++] = 0;
        a.src[a.nsrc] = src(D.part_node2.p, seg_ptr(c, R_NODEW), 0, 0); a.grp[a.nsrc++] = 1;
        a.src[a.nsrc] = src(c->NB ? D.body_part.p : nullptr, seg_ptr(c, R_BODY), 0, 0); a.grp[a.nsrc++] = 1;
        a.slot = S_BB;
        a.slot1 = S_RZ_NEW;
        reduce(c, a);
    }
    hipLaunchKernelGGL(k_pcg_start, dim3(blocks_for(ns, 64)), dim3(64), 0, st, ns, D.scal.p, active, D.pcg_iters.p, eta, D.maxpcg.p,
                       want);
    // first product and step length
    auto product = [&](int post) {
        hess_apply(c, z, w, active, D.part_node3.p);
        RedArgs a{};
        if (post == POST_CG) {
            a.src[a.nsrc] = src(D.part_node.p, seg_ptr(c, R_NODEW), 0, 0); a.grp[a.nsrc++] = 0;
            a.src[a.nsrc] = src(c->NB ? D.body_part.p : nullptr, seg_ptr(c, R_BODY), 0, 0); a.grp[a.nsrc++] = 0;
            a.src[a.nsrc] = src(D.part_node2.p, seg_ptr(c, R_NODEW), 0, 0); a.grp[a.nsrc++] = 2;
            a.src[a.nsrc] = src(c->NB ? D.body_part2.p : nullptr, seg_ptr(c, R_BODY), 0, 0); a.grp[a.nsrc++] = 2;
            a.slot = S_RZ_NEW;
            a.slot2 = S_RR;
        }
        a.src[a.nsrc] = src(D.part_node3.p, seg_ptr(c, R_NODEW), 0, 0); a.grp[a.nsrc++] = 1;
        a.src[a.nsrc] = src(c->n_long ? D.part_long.p : nullptr, seg_ptr(c, R_LONG), 0, 0); a.grp[a.nsrc++] = 1;
        a.slot1 = S_PAP;
        reduce_post(c, a, post);
    };
    product(POST_CG_FIRST);
    int maxit = 0;
    for (auto &S : c->sc) maxit = std::max(maxit, S.max_pcg);
    std::vector<int> hact(ns);
    // one iteration; every kernel skips scenes whose flag is down, so extra
    // iterations after convergence change nothing
    auto iteration = [&]() {
        int nnb = blocks_for(c->N), nbb = blocks_for(c->NB);
        prof_begin(c, IPC_K_PCG_UPDATE);
        hipLaunchKernelGGL(k_pcg_update, dim3(nnb + nbb), dim3(BLOCK), 0, c->stream, c->N, nnb, c->NB, D.node_kind.p, D.node_scene.p,
                           active, D.scal.p, D.dinv.p, D.dinvB.p, D.body_node0.p, D.body_scene.p, w, p, s, x, r, z, D.part_node.p,
                           D.part_node2.p, D.body_part.p, D.body_part2.p);
        prof_end(c, IPC_K_PCG_UPDATE, update_bytes(c));
        product(POST_CG);
    };
    // Host view after a batch: the active flags and, per active scene, an
    // estimate of the iterations left from the residual's geometric decay
    // since the previous check (capped; unknown on the first check).
    std::vector<double> hs((size_t)ns * NSLOT), prev_rr(ns, -1.0);
    auto check = [&](int done_since) {
        IPC_HIP(hipMemcpyAsync(hact.data(), active, ns * sizeof(int), hipMemcpyDeviceToHost, st));
        IPC_HIP(hipMemcpyAsync(hs.data(), D.scal.p, hs.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        IPC_HIP(hipStreamSynchronize(st));
        int left = 0;
        bool any = false;
        for (int q = 0; q < ns; ++q) {
            if (!hact[q]) continue;
            any = true;
            double rr = hs[(size_t)q * NSLOT + S_RR], e2 = hs[(size_t)q * NSLOT + S_ETA2];
            int est = 1 << 20;
            if (prev_rr[q] > 0.0 && rr > 0.0 && rr < prev_rr[q] && done_since > 0) {
                double rate = std::log(prev_rr[q] / rr) / done_since;
                est = (int)std::ceil(std::log(rr / e2) / rate);
            }
            prev_rr[q] = rr;
            left = std::max(left, est);
        }
        return any ? std::max(left, 1) : 0;
    };
    const int KB = 16, KS = 4;   // iterations per batch: far from and near convergence
    if (c->use_graphs && !c->prof) {
        // Capture a long and a short batch of iterations once per solve on the
        // context's capture stream (the caller's stream may be the null
        // stream, which cannot capture) and replay them on the context's
        // stream, the short one once few iterations are predicted to remain.
        IPC_HIP(hipStreamSynchronize(st));
        hipGraphExec_t exec[2] = {nullptr, nullptr};
        const int Ks[2] = {KB, KS};
        hipError_t e = hipSuccess;
        for (int g = 0; g < 2 && e == hipSuccess; ++g) {
            hipGraph_t graph = nullptr;
            c->stream = c->cap_stream;
            e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                for (int k = 0; k < Ks[g]; ++k) iteration();
                e = hipStreamEndCapture(c->cap_stream, &graph);
            }
            c->stream = st;
            if (e == hipSuccess) {
                e = hipGraphInstantiate(&exec[g], graph, nullptr, nullptr, 0);
                (void)hipGraphDestroy(graph);
            }
        }
        hipError_t le = e;
        int it = 0, left = 1 << 20;
        while (le == hipSuccess && it < maxit && left > 0) {
            int g = left > KB ? 0 : 1;
            le = hipGraphLaunch(exec[g], st);
            if (le != hipSuccess) break;
            it += Ks[g];
            left = check(Ks[g]);
        }
        for (auto &x : exec) if (x) (void)hipGraphExecDestroy(x);
        IPC_HIP(le);
        return;
    }
    for (int it = 0, since = 0; it < maxit; ++it) {
        iteration();
        ++since;
        if ((since == KS || it + 1 == maxit) && !check(since)) break;
        if (since == KS) since = 0;
    }
}

} // namespace ipc
