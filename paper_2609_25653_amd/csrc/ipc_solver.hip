// Linear algebra of the Newton step: deterministic per-scene reductions, the
// Hessian product (one block-CSR matrix over FEM vertices and affine-body
// nodes holding elasticity, inertia, orthogonality, springs and the contact
// blocks that fit its pattern, plus pair-local contact blocks for the rest),
// the block-Jacobi preconditioner (3x3 per FEM vertex, 12x12 per body) and a
// PCG that runs all scenes at once with per-scene scalars and flags.
#include <hip/hip_ext.h>

#include <chrono>
#include <cmath>

#include "ipc_device.h"
#include "ipc_internal.h"
#include "ipc_kernels.h"
#include "ipc_pcgdev.h"

namespace ipc {

// ---------------------------------------------------------------------------
// reductions: one workgroup per scene.  Each thread sums a fixed strided
// subset of a source's partials, and wavefront shuffles and a 4-entry LDS
// step combine them in a fixed order.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_reduce(int ns, RedArgs a, double *__restrict__ scal)
{
    int s = blockIdx.x;
    __shared__ double sh[RED_MAX][BLOCK / TILE];
    int wave = threadIdx.x / TILE, lane = threadIdx.x & (TILE - 1);
    // all loads first (independent, in flight together), then the shuffles:
    // the first 4 strided partials of every source are loaded unconditionally
    // (predicated), the rest (scenes with more than 1024 partials) in a loop
    double part[RED_MAX];
#pragma unroll
    for (int k = 0; k < RED_MAX; ++k) {
        part[k] = 0.0;
        if (k >= a.nsrc) continue;
        const RedSrc &r = a.src[k];
        if (!r.v) continue;
        int lo = r.seg[s] - r.base, hi = r.seg[s + 1] - r.base;
        if (r.w64 && !a.op) {
            // positions [off + lo, off + hi): the unaligned head and tail
            // entries, the whole 64-entry chunks between them from w64
            int plo = r.off + lo, phi = r.off + hi, c0 = (plo + 63) >> 6, c1 = phi >> 6;
            if (c0 < c1) {
                double acc = 0.0;
                if ((int)threadIdx.x < 64 * c0 - plo) acc += r.v[plo + threadIdx.x];
                for (int q = c0 + (int)threadIdx.x; q < c1; q += BLOCK) acc += r.w64[q];
                if (64 * c1 + (int)threadIdx.x < phi) acc += r.v[64 * c1 + threadIdx.x];
                part[k] = acc;
                continue;
            }
        }
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
    for (int k = 0; k < RED_MAX; ++k) {
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
    if (a.total >= 0) {
        double t = 0.0;
        for (int k = 0; k < a.nsrc; ++k) {
            double v = sh[k][0];
            for (int w = 1; w < BLOCK / TILE; ++w) v = a.op ? fmax(v, sh[k][w]) : v + sh[k][w];
            t = a.op ? fmax(t, v) : t + v;
        }
        S[a.total] = t;
    }
}

__global__ void k_sum64(int64_t n, const double *__restrict__ v, double *__restrict__ w)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double x = i < n ? v[i] : 0.0;
    x = wave_sum(x);
    if ((threadIdx.x & (TILE - 1)) == 0 && i < n) w[i / TILE] = x;
}

void sum64(ipc_ctx *c, const double *v, int64_t n, double *w)
{
    if (n > 0) hipLaunchKernelGGL(k_sum64, dim3(blocks_for(n)), dim3(BLOCK), 0, c->stream, n, v, w);
}

void reduce(ipc_ctx *c, const RedArgs &a)
{
    hipLaunchKernelGGL(k_reduce, dim3(c->n_scenes), dim3(BLOCK), 0, c->stream, c->n_scenes, a, c->d.scal.p);
}

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

// Workgroup b of a grid of n tiles -> tile, so that the b's one XCD runs
// (b = x + 8 j for XCD x) cover a contiguous range of tiles: XCD x takes
// tiles [x q + min(x, rem), ...) of length q (+1 for the first rem XCDs).
__device__ __forceinline__ int tile_of(int b, int n)
{
    constexpr int NX = 8;
    int x = b % NX, j = b / NX, q = n / NX, rem = n % NX;
    return x * q + min(x, rem) + j;
}

#ifndef IPC_SPMV_U
#define IPC_SPMV_U 2
#endif
constexpr int SPMV_U = IPC_SPMV_U;   // blocks per lane fetched together

template <int L>
__global__ void __launch_bounds__(64 * L) k_spmv(int N, int ntiles, const int *__restrict__ nlong, const int *__restrict__ long_rows,
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
        // Workgroups are dealt to the 8 XCDs round-robin; tile_of gives each
        // XCD one contiguous run of tiles, whose rows share most of their
        // columns, so the gathered vector entries are reused in that XCD's L2.
        const int tile = tile_of(blockIdx.x, ntiles);
        int sub = threadIdx.x % L;
        int n = tile * TILE + threadIdx.x / L;
        double ax = 0.0, ay = 0.0, az = 0.0;
        bool mine = false, on = false;
        if (n < N) {
            int k0 = row_ptr[n], k1 = row_ptr[n + 1], d0 = dptr[n], d1 = dptr[n + 1];
            const int sc = node_scene[n];
            if ((k1 - k0) + (d1 - d0) <= LONG_ROW) {
                mine = true;
                // The lane's first SPMV_U blocks are fetched together: their
                // columns before the scene's flag is known, then every block
                // and vector entry at once, so that a row costs two round
                // trips to memory instead of two per block.  Lanes past the
                // row's end read slot 0 and column 0 and add nothing.
                int ks[SPMV_U], cs[SPMV_U];
#pragma unroll
                for (int u = 0; u < SPMV_U; ++u) {
                    const int k = k0 + sub + u * L;
                    ks[u] = k < k1 ? k : 0;
                    cs[u] = k < k1 ? col[k] : 0;
                }
                on = !active || active[sc];
                if (on) {
                    d3 w[SPMV_U];
                    double B[SPMV_U][9];
#pragma unroll
                    for (int u = 0; u < SPMV_U; ++u) {
                        w[u] = ld3(v, cs[u]);
#pragma unroll
                        for (int q = 0; q < 9; ++q) B[u][q] = val[9 * (size_t)ks[u] + q];
                    }
#pragma unroll
                    for (int u = 0; u < SPMV_U; ++u) {
                        if (k0 + sub + u * L >= k1) w[u] = {0.0, 0.0, 0.0};
                        acc_block(B[u], w[u], ax, ay, az);
                    }
                    for (int k = k0 + sub + SPMV_U * L; k < k1; k += L) acc_block(val + 9 * (size_t)k, ld3(v, col[k]), ax, ay, az);
                    for (int k = d0 + sub; k < d1; k += L) acc_block(dval + 9 * (size_t)k, ld3(v, dcol[k]), ax, ay, az);
                }
            }
        }
        // the row's L lanes are aligned lanes of one wavefront: DPP sums
        ax = lane_sum<L>(ax); ay = lane_sum<L>(ay); az = lane_sum<L>(az);
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
                part[tile] = t;
            }
        }
        return;
    }
    // one workgroup per long row: all 64 L lanes stride over its blocks
    __shared__ double shl[3][NW];
    int w = (int)blockIdx.x - ntiles;
    if (w >= nlong[0]) {   // unused: a zero partial, so that a reduction may span all of them
        if (part_long && threadIdx.x == 0) part_long[w] = 0.0;
        return;
    }
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

// ev0 / ev1 (nullable): HIP events stamped by the dispatch itself at the
// kernel's start and end, so that no marker packet enters the interval
static void spmv_launch(ipc_ctx *c, int L, const double *v, double *out, const int *active, double *part,
                        hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr)
{
    Dev &D = c->d;
    int ntiles = (c->N + TILE - 1) / TILE;
    dim3 grid(ntiles + c->long_cap), blk(64 * L);   // extra workgroups beyond the long-row count exit at once
    double *pl = part ? D.part_long.p : nullptr;
    // plain launches otherwise (they are the ones captured into graphs)
#define IPC_SPMV_ARGS c->N, ntiles, D.long_count.p, D.long_rows.p, D.row_ptr.p, D.col.p, D.val.p, D.dyn_ptr.p, D.dyn_col.p, D.dyn_val.p, \
                      v, D.node_scene.p, active, out, part, pl
#define IPC_SPMV(LL) do { \
        if (ev0) hipExtLaunchKernelGGL(k_spmv<LL>, grid, blk, 0, c->stream, ev0, ev1, 0, IPC_SPMV_ARGS); \
        else hipLaunchKernelGGL(k_spmv<LL>, grid, blk, 0, c->stream, IPC_SPMV_ARGS); \
    } while (0)
    switch (L) {
    case 1: IPC_SPMV(1); break;
    case 2: IPC_SPMV(2); break;
    case 4: IPC_SPMV(4); break;
    case 8: IPC_SPMV(8); break;
    default: IPC_SPMV(16); break;
    }
#undef IPC_SPMV
#undef IPC_SPMV_ARGS
}

// Profiled products: the algorithmic bytes of one launch from the scenes it
// did not skip, added to a counter by a small launch after the product (its
// HIP events bracket the product alone): per scene 8 B per row, and for a
// scene still iterating 76 B per block of its rows (matrix and pair-local)
// and 48 B per real node.  With every scene on this is spmv_bytes.
__global__ void __launch_bounds__(BLOCK) k_spmv_bytes(int ns, const int *__restrict__ rng, const int *__restrict__ row_ptr,
                                                      const int *__restrict__ dptr, const int *__restrict__ active,
                                                      double *__restrict__ total)
{
    __shared__ double sh[BLOCK / TILE];
    double b = 0.0;
    for (int s = threadIdx.x; s < ns; s += BLOCK) {
        const int n0 = rng[3 * (size_t)s], n1 = rng[3 * (size_t)s + 1];
        b += 8.0 * (n1 - n0);
        if (!active || active[s]) b += 76.0 * ((row_ptr[n1] - row_ptr[n0]) + (dptr[n1] - dptr[n0])) + 48.0 * rng[3 * (size_t)s + 2];
    }
    b = wave_sum(b);
    if ((threadIdx.x & (TILE - 1)) == 0) sh[threadIdx.x / TILE] = b;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = sh[0];
        for (int q = 1; q < BLOCK / TILE; ++q) t += sh[q];
        total[0] += t;
    }
}

void hess_apply(ipc_ctx *c, const double *v, double *out, const int *active, double *part)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    prof_dispatch_events(c, IPC_K_SPMV, &e0, &e1, spmv_bytes(c));
    spmv_launch(c, c->spmv_lanes, v, out, active, part, e0, e1);
    if (e0 && c->d.prof_bytes.p)
        hipLaunchKernelGGL(k_spmv_bytes, dim3(1), dim3(BLOCK), 0, c->stream, c->n_scenes, c->d.prof_scene.p, c->d.row_ptr.p,
                           c->d.dyn_ptr.p, active, c->d.prof_bytes.p);
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
    double best = 1e300, t8 = 1e300;
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
        if (Ls[i] == 8) t8 = t;
        if (t < best) { best = t; bestL = Ls[i]; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // Back-to-back launches on one matrix favour the variants whose working
    // set stays in L2; inside PCG the update kernel runs in between.  8 lanes
    // is kept unless another count is more than 3 % faster here.
    c->spmv_lanes = t8 <= 1.03 * best ? 8 : bestL;
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
                           double *__restrict__ dinv, const int *__restrict__ node_scene, const int *__restrict__ active)
{
    int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    if (active && !active[node_scene[n]]) return;
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
// One thread per body (launched with 64 threads, so the register file holds
// the 12x12 factor); every loop is unrolled, so no array needs scratch memory.
__global__ void __launch_bounds__(64) k_prec_body(int NB, const int *__restrict__ bslot, const int *__restrict__ node0,
                                                  const double *__restrict__ val, const int *__restrict__ dptr,
                                                  const int *__restrict__ dcol, const double *__restrict__ dval,
                                                  double *__restrict__ dinvB, const int *__restrict__ body_scene,
                                                  const int *__restrict__ active)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= NB) return;
    if (active && !active[body_scene[b]]) return;
    double L[144];
    int n0 = node0[b];
#pragma unroll
    for (int ca = 0; ca < 4; ++ca)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            const double *B = val + 9 * (size_t)bslot[16 * (size_t)b + 4 * ca + cb];
            int k = dyn_find(dptr, dcol, n0 + ca, n0 + cb);
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    double v = B[3 * i + j];
                    if (k >= 0) v += dval[9 * (size_t)k + 3 * i + j];
                    L[12 * (3 * ca + i) + 3 * cb + j] = v;
                }
        }
    // Cholesky factor L L^T (lower triangle of L)
#pragma unroll
    for (int j = 0; j < 12; ++j) {
        double s = L[12 * j + j];
#pragma unroll
        for (int k = 0; k < j; ++k) s -= L[12 * j + k] * L[12 * j + k];
        double dj = sqrt(fmax(s, 1e-300));
        L[12 * j + j] = dj;
#pragma unroll
        for (int i = j + 1; i < 12; ++i) {
            double t = L[12 * i + j];
#pragma unroll
            for (int k = 0; k < j; ++k) t -= L[12 * i + k] * L[12 * j + k];
            L[12 * i + j] = t / dj;
        }
    }
    // the inverse, one column at a time by forward and back substitution
    double *o = dinvB + 144 * (size_t)b;
#pragma unroll
    for (int cidx = 0; cidx < 12; ++cidx) {
        double y[12];
#pragma unroll
        for (int i = 0; i < 12; ++i) {
            double t = (i == cidx) ? 1.0 : 0.0;
#pragma unroll
            for (int k = 0; k < i; ++k) t -= L[12 * i + k] * y[k];
            y[i] = t / L[12 * i + i];
        }
#pragma unroll
        for (int i = 11; i >= 0; --i) {
            double t = y[i];
#pragma unroll
            for (int k = i + 1; k < 12; ++k) t -= L[12 * k + i] * y[k];
            y[i] = t / L[12 * i + i];
        }
#pragma unroll
        for (int i = 0; i < 12; ++i) o[12 * i + cidx] = y[i];
    }
}

void build_preconditioner(ipc_ctx *c)
{
    Dev &D = c->d;
    hipLaunchKernelGGL(k_prec_fem, dim3(blocks_for(c->N)), dim3(BLOCK), 0, c->stream, c->N, D.node_kind.p, D.diag_slot.p, D.val.p,
                       D.dyn_ptr.p, D.dyn_col.p, D.dyn_val.p, D.dinv.p, D.node_scene.p, c->assemble_only);
    if (c->NB)
        hipLaunchKernelGGL(k_prec_body, dim3(blocks_for(c->NB, 64)), dim3(64), 0, c->stream, c->NB, D.bslot.p, D.body_node0.p, D.val.p,
                           D.dyn_ptr.p, D.dyn_col.p, D.dyn_val.p, D.dinvB.p, D.body_scene.p, c->assemble_only);
    coarse_build(c);
}

// ---------------------------------------------------------------------------
// PCG (preconditioned conjugate gradients in the single-reduction form of
// Chronopoulos and Gear: besides p it carries s = A p, so that one product
// w = A z and one per-scene reduction per iteration suffice).
//
// An iteration is two launches: k_pcg_step, whose workgroups first reduce
// their scenes' partials of the previous iteration themselves (every
// workgroup of a scene sums the same partials in the same order, so all of
// them obtain bit-identical scalars) and then update p, s, x, r, z; and the
// product w = A z with its partials of z . w.  The per-scene state (gamma,
// alpha, eta^2 b.b, r.r, running flag, update count) and the partials of
// r.z and r.r are double-buffered by iteration parity: the step of
// iteration k reads buffer k & 1, and the workgroup holding the scene's
// first tile writes buffer (k + 1) & 1, so no launch reads what it writes.
// ---------------------------------------------------------------------------
constexpr int WG_TILES = BLOCK / TILE;   // node tiles per step workgroup

// Sums of up to three per-tile sources and one per-long-row source over a
// scene's ranges; every thread of the workgroup returns the same totals.
// (ca: per-domain partials added to the first sum, over [clo, chi))
// The first 4 strided entries of every source (scenes of up to 1024 tiles,
// 64k nodes), the long rows' first and the domains' first entry are loaded
// predicated, all before the first add, so their latencies overlap instead
// of following each other; longer ranges finish in loops.  bs_issue makes
// those first loads (a caller may issue them early), bs_finish the rest.
struct BsFirst {
    double ea[4], eb[4], ec[4], el, ec0;
};
__device__ __forceinline__ void bs_issue(int lo, int hi, int llo, int lhi, int clo, int chi, const double *__restrict__ a,
                                         const double *__restrict__ b, const double *__restrict__ c,
                                         const double *__restrict__ cl, const double *__restrict__ ca, BsFirst &f)
{
    const int t = (int)threadIdx.x;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int i = lo + t + u * BLOCK;
        const bool in = i < hi;
        f.ea[u] = in ? a[i] : 0.0;
        f.eb[u] = in ? b[i] : 0.0;
        f.ec[u] = in && c ? c[i] : 0.0;
    }
    f.el = cl && llo + t < lhi ? cl[llo + t] : 0.0;
    f.ec0 = ca && clo + t < chi ? ca[clo + t] : 0.0;
}
__device__ __forceinline__ void bs_finish(int lo, int hi, int llo, int lhi, int clo, int chi, const double *__restrict__ a,
                                          const double *__restrict__ b, const double *__restrict__ c,
                                          const double *__restrict__ cl, const double *__restrict__ ca, const BsFirst &f,
                                          double (*sh)[WG_TILES], double &ta, double &tb, double &tc)
{
    const int t = (int)threadIdx.x;
    double va = (f.ea[0] + f.ea[1]) + (f.ea[2] + f.ea[3]), vb = (f.eb[0] + f.eb[1]) + (f.eb[2] + f.eb[3]),
           vc = (f.ec[0] + f.ec[1]) + (f.ec[2] + f.ec[3]);
    for (int i = lo + t + 4 * BLOCK; i < hi; i += BLOCK) {
        va += a[i];
        vb += b[i];
        if (c) vc += c[i];
    }
    vc += f.el;
    if (cl)
        for (int i = llo + t + BLOCK; i < lhi; i += BLOCK) vc += cl[i];
    va += f.ec0;
    if (ca)
        for (int i = clo + t + BLOCK; i < chi; i += BLOCK) va += ca[i];
    va = wave_sum(va); vb = wave_sum(vb); vc = wave_sum(vc);
    int wave = threadIdx.x / TILE;
    if ((threadIdx.x & (TILE - 1)) == 0) { sh[0][wave] = va; sh[1][wave] = vb; sh[2][wave] = vc; }
    __syncthreads();
    ta = (sh[0][0] + sh[0][1]) + (sh[0][2] + sh[0][3]);
    tb = (sh[1][0] + sh[1][1]) + (sh[1][2] + sh[1][3]);
    tc = (sh[2][0] + sh[2][1]) + (sh[2][2] + sh[2][3]);
    __syncthreads();
}
__device__ __forceinline__ void block_sums(int lo, int hi, int llo, int lhi, int clo, int chi, const double *__restrict__ a,
                                           const double *__restrict__ b, const double *__restrict__ c,
                                           const double *__restrict__ cl, const double *__restrict__ ca, double (*sh)[WG_TILES],
                                           double &ta, double &tb, double &tc)
{
    BsFirst f;
    bs_issue(lo, hi, llo, lhi, clo, chi, a, b, c, cl, ca, f);
    bs_finish(lo, hi, llo, lhi, clo, chi, a, b, c, cl, ca, f, sh, ta, tb, tc);
}

__device__ __forceinline__ d3 mat3v(const double *__restrict__ M, d3 v)
{
    return {M[0] * v.x + M[1] * v.y + M[2] * v.z, M[3] * v.x + M[4] * v.y + M[5] * v.z, M[6] * v.x + M[7] * v.y + M[8] * v.z};
}

// Per step workgroup: its first and last scene and the first scene's tile,
// long-row and coarse-domain ranges (refreshed whenever the long rows change).
constexpr int WGI = 8;
__global__ void k_pcg_wginfo(int nwg, int ntile, const int *__restrict__ tile_scene, const int *__restrict__ seg_nodew,
                             const int *__restrict__ seg_long, const int *__restrict__ seg_cdom, int *__restrict__ info)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nwg) return;
    int t0 = b * WG_TILES, lo = tile_scene[t0], hi = tile_scene[min(t0 + WG_TILES, ntile) - 1];
    int *o = info + WGI * (size_t)b;
    o[0] = lo; o[1] = hi;
    o[2] = seg_nodew[lo]; o[3] = seg_nodew[lo + 1];
    o[4] = seg_long[lo]; o[5] = seg_long[lo + 1];
    o[6] = seg_cdom[lo]; o[7] = seg_cdom[lo + 1];
}

void pcg_wginfo(ipc_ctx *c)
{
    int ntile = c->N / TILE, nwg = blocks_for(c->N);
    c->d.pcg_wginfo.alloc(WGI * (size_t)nwg);
    hipLaunchKernelGGL(k_pcg_wginfo, dim3(blocks_for(nwg)), dim3(BLOCK), 0, c->stream, nwg, ntile, c->d.tile_scene_node.p,
                       seg_ptr(c, R_NODEW), seg_ptr(c, R_LONG), seg_ptr(c, R_CDOM), c->d.pcg_wginfo.p);
}

// x = 0, r = b, p = s = 0, z = M^-1 r; partials of r.z and r.r per tile
// (affine bodies: the thread of the body's first node applies its 12x12
// block); each scene's first-tile thread sets the parity-0 state, with the
// relative tolerance (eta, or the scene's own when eta <= 0) in the eta^2
// b.b entry until the first step.
__global__ void __launch_bounds__(BLOCK) k_pcg_init(int N, int ns, const int *__restrict__ kind, const int *__restrict__ node_body,
                                                    const int *__restrict__ tile_scene, const int *__restrict__ seg_nodew,
                                                    const double *__restrict__ b, const double *__restrict__ dinv,
                                                    const double *__restrict__ dinvB, double *__restrict__ x, double *__restrict__ r,
                                                    double *__restrict__ z, double *__restrict__ p, double *__restrict__ s,
                                                    double *__restrict__ part, int ntile, const int *__restrict__ want,
                                                    double eta, const double *__restrict__ sparam, double *__restrict__ st,
                                                    double *__restrict__ prev_rr,
                                                    int *__restrict__ act, int *__restrict__ it, int *__restrict__ iters,
                                                    double *__restrict__ scal)
{
    int n = blockIdx.x * blockDim.x + threadIdx.x;
    double rz = 0.0, rr = 0.0;
    if (n < N) {
        d3 bv = ld3(b, n);
        st3(x, n, {0.0, 0.0, 0.0});
        st3(p, n, {0.0, 0.0, 0.0});
        st3(s, n, {0.0, 0.0, 0.0});
        st3(r, n, bv);
        int k = kind[n];
        if (k == 0) {
            d3 zv = mat3v(dinv + 9 * (size_t)n, bv);
            st3(z, n, zv);
            rz = dt(bv, zv);
            rr = dt(bv, bv);
        } else if (k == 2) {
            st3(z, n, {0.0, 0.0, 0.0});
        } else if (node_body[n] >= 0) {
            const double *bb = b + 3 * (size_t)n;
            const double *M = dinvB + 144 * (size_t)node_body[n];
            for (int i = 0; i < 12; ++i) {
                double acc = 0.0;
                for (int j = 0; j < 12; ++j) acc += M[12 * i + j] * bb[j];
                z[3 * (size_t)n + i] = acc;
                rz += bb[i] * acc;
                rr += bb[i] * bb[i];
            }
        }
    }
    rz = wave_sum(rz); rr = wave_sum(rr);
    if ((threadIdx.x & (TILE - 1)) == 0 && n < N) {
        int t = n / TILE;
        part[t] = rz;
        part[ntile + t] = rr;
        int sc = tile_scene[t];
        if (seg_nodew[sc] == t) {
            act[sc] = (!want || want[sc]) ? 2 : 0;
            it[sc] = 0;
            st[4 * (size_t)sc + 2] = eta > 0.0 ? eta : sparam[8 * (size_t)sc + P_ETA];   // the first step squares it and scales by b.b
            prev_rr[sc] = -1.0;
            iters[sc] = 0;
            scal[(size_t)sc * NSLOT + S_INDEF] = 0.0;
        }
    }
}

// One iteration, parity q.  State per scene and parity: st[4] = {gamma,
// alpha, eta^2 b.b, r.r}, act (0 stopped, 1 running, 2 first iteration), it
// (updates done).  part holds [r.z | r.r] for parity 0 then parity 1.
//
// FUSED (one scene whose coarse domains are contiguous node ranges, see
// coarse_setup): the workgroup of slice sl of domain d takes that slice's
// 256 nodes and also applies the slice's part of the coarse correction, so
// that no second launch is needed.  Workgroups number (domain, slice) so
// that a domain's slices share an XCD.  Restricting the new residual over
// the whole domain needs r of the other slices' nodes, which their own
// workgroups are updating: r and s are read from the parity-q buffers
// (r_in, s_in), the update is recomputed for the foreign entries with the
// same arithmetic, and r, s and z are written to the other parity's buffers.
// An entry whose slot holds a body's translation node gets its
// block-Jacobi value recomputed here too (the same rows of the body's
// inverse as its own workgroup, which does not store that node's z).  The
// bits come out as those of the step followed by k_coarse_apply.  Without
// FUSED the in and out buffers are the same and the correction follows in
// its own launch.
template <bool FUSED>
__global__ void __launch_bounds__(BLOCK) k_pcg_step(int N, int ns, int q, const int *__restrict__ kind, const int *__restrict__ node_body,
                                                    const int *__restrict__ tile_scene, const int *__restrict__ seg_nodew,
                                                    const int *__restrict__ seg_long, const int *__restrict__ seg_cdom,
                                                    const int *__restrict__ wginfo, int single, int lcap,
                                                    const double *__restrict__ cg_part, int ncdom,
                                                    const int *__restrict__ maxit, const double *__restrict__ dinv,
                                                    const double *__restrict__ dinvB, const double *__restrict__ w, double *__restrict__ p,
                                                    const double *s_in, double *s, double *__restrict__ x, const double *r_in,
                                                    double *r, const double *z_in, double *z, const double *__restrict__ part_zw,
                                                    const double *__restrict__ part_long, double *__restrict__ part, int ntile,
                                                    double *__restrict__ st, int *__restrict__ act, int *__restrict__ it,
                                                    const double *__restrict__ st_in, const int *__restrict__ act_in,
                                                    const int *__restrict__ it_in, double *__restrict__ scal, int ndom, int nwin, int nfr, int bnode0, const int *__restrict__ ph_ptr,
                                                    const int *__restrict__ ph_e, const int *__restrict__ ph_n,
                                                    const int *__restrict__ node_da, const double *__restrict__ inv, double *cg_out)
{
    __shared__ double sh[3][WG_TILES];
    const int wave = threadIdx.x / TILE, lane = threadIdx.x & (TILE - 1), tid = threadIdx.x;
    int L = blockIdx.x, d = 0, sl = 0;   // L: the workgroup's place in node order
    if (FUSED) {
        const int k = blockIdx.x / NXCD;
        sl = k % CG_SPLIT;
        d = blockIdx.x % NXCD + NXCD * (k / CG_SPLIT);
        if (d >= nwin) return;   // the grid is rounded up to whole XCD rounds
        L = CG_SPLIT * d + sl;
    }
    const bool cg = FUSED && d < ndom;   // uniform: this workgroup applies a slice of domain d
    const int t0 = L * WG_TILES, t = t0 + wave;
    const int n = t * TILE + lane;
    const double *rz_in = part + (size_t)(2 * q) * ntile, *rr_in = rz_in + ntile;
    const double *cz_in = ncdom ? cg_part + (size_t)q * ncdom : nullptr;   // r . z of the coarse correction (CG_SPLIT per domain)
    // The first scene's partials are the first loads, so that the loads
    // below do not hold back its reduction.  Its ranges: for a single scene
    // all tiles, every long-row partial (unused ones are 0) and every coarse
    // domain; otherwise the workgroup's record.
    const int *wi = wginfo + WGI * (size_t)L;
    const int r0t = single ? 0 : wi[2], r1t = single ? ntile : wi[3], r0l = single ? 0 : wi[4], r1l = single ? lcap : wi[5],
              r0c = single ? 0 : CG_SPLIT * wi[6], r1c = single ? ncdom : CG_SPLIT * wi[7];
    BsFirst pre;
    bs_issue(r0t, r1t, r0l, r1l, r0c, r1c, rz_in, rr_in, part_zw, part_long, cz_in, pre);
    // FUSED: the domain's entries.  Entry e of domain d is node
    // CG_AGG CG_DOM d + e, entries end at nfr, and the few slots that stand
    // for a body's translation node come from a per-domain list read through
    // scalar loads, so no vector load waits for another.
    int nd[CG_PASSES];
#pragma unroll
    for (int j = 0; j < CG_PASSES; ++j) {
        const int slot = CG_AGG * CG_DOM * d + CG_APPLY * j + tid;
        nd[j] = cg && slot < nfr ? slot : -1;
    }
    if (cg)
        for (int u = ph_ptr[d]; u < ph_ptr[d + 1]; ++u) {   // uniform
            const int e = ph_e[u], node = ph_n[u];
#pragma unroll
            for (int j = 0; j < CG_PASSES; ++j)
                if (e == CG_APPLY * j + tid) nd[j] = node;
        }
    // this node's operands, without waiting for its kind: their loads
    // overlap the reductions below
    // (a lane past the last node reads the last node, so that no branch
    // joins values whose loads are still in flight; its kind counts as 2)
    const bool live = n < N;
    const int nc = live ? n : N - 1;
    const int kraw = kind[nc];
    const int da = FUSED ? node_da[nc] : -1;   // FUSED: the node's coarse group (a grouped body node's z comes from its entry's workgroup)
    d3 zv = ld3(z_in, nc), pv = ld3(p, nc), wv = ld3(w, nc), sv = ld3(s_in, nc), xv = ld3(x, nc), rv = ld3(r_in, nc);
    double Mi[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) Mi[q] = dinv[9 * (size_t)nc + q];
    // FUSED: the slice's inverse rows and the other entries' operands, also
    // before the reductions
    const int i = tid / CG_CLANES, cl = tid % CG_CLANES;
    double m[CG_CPL];
    d3 fr[CG_PASSES], fs[CG_PASSES], fw[CG_PASSES];
    // (none of these loads is predicated: the waits for the partials count
    // the loads issued after them, and a load that may be skipped would make
    // them wait for more; a lane or workgroup without a use reads a valid
    // address and discards the value)
    if (FUSED) {
        const double *M = inv + (size_t)(cg ? d : ndom - 1) * CG_N * CG_N + (size_t)(CG_ROWS * sl + min(i, CG_ROWS - 1)) * CG_N + cl;
#pragma unroll
        for (int j = 0; j < CG_CPL; ++j) m[j] = M[CG_CLANES * j];
#pragma unroll
        for (int j = 0; j < CG_PASSES; ++j) {
            const int f = nd[j] >= 0 ? nd[j] : nc;
            fr[j] = ld3(r_in, f); fs[j] = ld3(s_in, f); fw[j] = ld3(w, f);
        }
    }
    double *rz_out = part + (size_t)(2 * (q ^ 1)) * ntile, *rr_out = rz_out + ntile;
    // the workgroup's scenes and the first one's tile and long-row ranges in
    // one record, so the partials' loads wait for a single load
    // (a single scene needs no record: its ranges are all tiles, every
    // long-row partial, unused ones being 0, and every coarse domain)
    const int sc_lo = single ? 0 : wi[0], sc_hi = single ? 0 : wi[1];
    const int my_sc = t < ntile ? (single ? 0 : tile_scene[t]) : -1;
    double al = 0.0, be = 0.0;
    bool on = false;
    for (int sc = sc_lo; sc <= sc_hi; ++sc) {   // uniform over the workgroup
        const bool first = sc == sc_lo;
        const int tlo = single ? 0 : first ? wi[2] : seg_nodew[sc], thi = single ? ntile : first ? wi[3] : seg_nodew[sc + 1];
        const int llo = single ? 0 : first ? wi[4] : seg_long[sc], lhi = single ? lcap : first ? wi[5] : seg_long[sc + 1];
        const int clo = single ? 0 : first ? wi[6] : seg_cdom[sc], chi = single ? ncdom / CG_SPLIT : first ? wi[7] : seg_cdom[sc + 1];
        const int a = act_in[q * ns + sc], itc = it_in[q * ns + sc];
        const double *S = st_in + ((size_t)q * ns + sc) * 4;
        const bool writer = tlo / WG_TILES == L && threadIdx.x == 0;
        double *So = st + ((size_t)(q ^ 1) * ns + sc) * 4;
        if (!a) {
            if (writer) {
                So[0] = S[0]; So[1] = S[1]; So[2] = S[2]; So[3] = S[3];
                act[(q ^ 1) * ns + sc] = 0;
                it[(q ^ 1) * ns + sc] = itc;
            }
            continue;
        }
        double gam, rr, del;
        if (first) bs_finish(r0t, r1t, r0l, r1l, r0c, r1c, rz_in, rr_in, part_zw, part_long, cz_in, pre, sh, gam, rr, del);
        else block_sums(tlo, thi, llo, lhi, CG_SPLIT * clo, CG_SPLIT * chi, rz_in, rr_in, part_zw, part_long, cz_in, sh, gam, rr, del);
        // gamma = r.z, delta = z.Az of the current residual:
        //   beta = gamma / gamma_old,  p.Ap = delta - beta gamma / alpha_old,
        //   alpha = gamma / p.Ap
        double eta2, bs = 0.0;
        int na = 1;
        bool indef = false;
        if (a == 2) {
            eta2 = S[2] * S[2] * rr;
            if (!(rr > 0.0)) na = 0;
        } else {
            eta2 = S[2];
            if (rr <= eta2 || itc >= maxit[sc]) na = 0;
            else {
                bs = gam / S[0];
                del -= bs * gam / S[1];
            }
        }
        if (na && !(del > 0.0)) { na = 0; indef = true; }   // not positive definite along p: stop
        const double as = na ? gam / del : 0.0;
        if (writer) {
            So[0] = gam; So[1] = as; So[2] = eta2; So[3] = rr;
            act[(q ^ 1) * ns + sc] = na;
            it[(q ^ 1) * ns + sc] = itc + na;
            if (indef) scal[(size_t)sc * NSLOT + S_INDEF] = 1.0;
        }
        if (sc == my_sc || (FUSED && sc == 0)) { on = na; al = as; be = bs; }
    }
    const int k = live ? kraw : 2;
    double rz = 0.0, rr = 0.0;
    // z of this node from its block-Jacobi part; the coarse correction is
    // added before it is stored when the node is an entry of this slice
    bool store_z = false;
    if (on && k == 0) {
        pv = {zv.x + be * pv.x, zv.y + be * pv.y, zv.z + be * pv.z};
        xv = {xv.x + al * pv.x, xv.y + al * pv.y, xv.z + al * pv.z};
        pcg_sr(wv, al, be, sv, rv);
        zv = mat3v(Mi, rv);
        st3(p, n, pv); st3(s, n, sv); st3(x, n, xv); st3(r, n, rv);
        store_z = true;
        rr = dt(rv, rv);
        rz = dt(rv, zv);
    } else if (on && k == 1) {
        // An affine body's 4 nodes are 4 consecutive lanes of this wavefront
        // (its first node is a multiple of 4).  Each lane updates its own
        // node, gathers the body's 12 residual entries from the 4 lanes and
        // forms 3 rows of the body's 12x12 inverse block times them.
        pv = {zv.x + be * pv.x, zv.y + be * pv.y, zv.z + be * pv.z};
        xv = {xv.x + al * pv.x, xv.y + al * pv.y, xv.z + al * pv.z};
        pcg_sr(wv, al, be, sv, rv);
        st3(p, n, pv); st3(s, n, sv); st3(x, n, xv); st3(r, n, rv);
        const int a = n & 3, first = lane - a;
        double rb[12];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            rb[3 * q] = __shfl(rv.x, first + q);
            rb[3 * q + 1] = __shfl(rv.y, first + q);
            rb[3 * q + 2] = __shfl(rv.z, first + q);
        }
        zv = body_rows(dinvB + 144 * (size_t)node_body[n - a] + 36 * a, rb);
        store_z = !(FUSED && da >= 0);
        rr = dt(rv, rv);
        rz = dt(rv, zv);
    }
    if (cg && on) {   // uniform: FUSED has one scene
        __shared__ double rc[CG_N], zl[CG_ROWS];
        // the new residual on every entry of the domain: this node's own,
        // or recomputed from the parity-q operands
        d3 rn[CG_PASSES];
#pragma unroll
        for (int j = 0; j < CG_PASSES; ++j) {
            rn[j] = d3{0.0, 0.0, 0.0};
            if (nd[j] == n) rn[j] = rv;
            else if (nd[j] >= 0) {
                d3 sj = fs[j], rj = fr[j];
                pcg_sr(fw[j], al, be, sj, rj);
                rn[j] = rj;
            }
        }
#pragma unroll
        for (int j = 0; j < CG_PASSES; ++j) {
            const d3 v = cg_group_sum(rn[j]);
            const int g = (tid + j * CG_APPLY) / CG_AGG;
            if ((lane & (CG_AGG - 1)) == CG_AGG - 1) { rc[3 * g] = v.x; rc[3 * g + 1] = v.y; rc[3 * g + 2] = v.z; }
        }
        __syncthreads();
        if (tid < 192) {
            const double a = cg_row(m, rc, cl);
            if (cl == 0) zl[i] = a;   // rows past a short domain's end: rc and the inverse are 0 there
        }
        __syncthreads();
        int me = -1;
#pragma unroll
        for (int j = 0; j < CG_PASSES; ++j)
            if (j == sl) me = nd[j];
        const int g = tid / CG_AGG;
        if (me == n) {
            zv = {zv.x + zl[3 * g], zv.y + zl[3 * g + 1], zv.z + zl[3 * g + 2]};
        } else if (me >= 0) {
            // an entry that stands for a body's translation node: the body's
            // 4 nodes' new residual and the first 3 rows of its inverse block
            // (read here, with the block, to keep registers for the loads
            // every workgroup waits for)
            double rb[12];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                d3 sc = ld3(s_in, me + c), rc4 = ld3(r_in, me + c);
                pcg_sr(ld3(w, me + c), al, be, sc, rc4);
                rb[3 * c] = rc4.x; rb[3 * c + 1] = rc4.y; rb[3 * c + 2] = rc4.z;
            }
            const d3 zb = body_rows(dinvB + 144 * (size_t)((me - bnode0) / 4), rb);   // one scene: body b at bnode0 + 4 b
            st3(z, me, {zb.x + zl[3 * g], zb.y + zl[3 * g + 1], zb.z + zl[3 * g + 2]});
        }
        if (tid < TILE) {
            double dot = tid < CG_ROWS ? rc[CG_ROWS * sl + tid] * zl[tid] : 0.0;
            dot = wave_sum(dot);
            if (tid == 0) cg_out[(size_t)CG_SPLIT * d + sl] = dot;
        }
    }
    if (store_z) st3(z, n, zv);
    rz = wave_sum(rz); rr = wave_sum(rr);
    if (lane == 0 && t < ntile) { rz_out[t] = rz; rr_out[t] = rr; }
}

// After a batch of iterations (parity q): per scene, whether the next step
// would still iterate (the same sums and test as the step) and, if so, an
// estimate of the iterations left from the residual's geometric decay over
// the batch (n_since iterations; 2^20 when unknown), published to host memory
// as one 64-bit word (seq << 32 | estimate, 0 = stopped) that the host polls;
// also the update count.
constexpr int PCG_EST_UNKNOWN = 1 << 20;
__global__ void __launch_bounds__(BLOCK) k_pcg_peek(int ns, int q, const int *__restrict__ seg_nodew, const int *__restrict__ maxit,
                                                    const double *__restrict__ part, int ntile, const double *__restrict__ st,
                                                    const int *__restrict__ act, const int *__restrict__ it,
                                                    double *__restrict__ prev_rr, int n_since, unsigned int seq,
                                                    unsigned long long *__restrict__ out, int *__restrict__ iters)
{
    __shared__ double sh[3][WG_TILES];
    int sc = blockIdx.x;
    int a = act[q * ns + sc], itc = it[q * ns + sc];
    double rr = 0.0;
    bool live = false;
    if (a) {
        const double *rz_in = part + (size_t)(2 * q) * ntile;
        double g, d;
        block_sums(seg_nodew[sc], seg_nodew[sc + 1], 0, 0, 0, 0, rz_in, rz_in + ntile, nullptr, nullptr, nullptr, sh, g, rr, d);
        live = a == 2 || !(rr <= st[((size_t)q * ns + sc) * 4 + 2] || itc >= maxit[sc]);
    }
    if (threadIdx.x != 0) return;
    iters[sc] = itc;
    int est = 0;
    if (live) {
        est = PCG_EST_UNKNOWN;
        double pr = prev_rr[sc], e2 = a == 2 ? 0.0 : st[((size_t)q * ns + sc) * 4 + 2];
        if (pr > 0.0 && rr > 0.0 && e2 > 0.0 && rr < pr && n_since > 0) {
            double rate = log(pr / rr) / n_since, k = ceil(log(rr / e2) / rate);
            est = k < (double)PCG_EST_UNKNOWN ? (int)fmax(k, 1.0) : PCG_EST_UNKNOWN;
        }
        prev_rr[sc] = rr;
    }
    out[sc] = ((unsigned long long)seq << 32) | (unsigned int)est;
}

// Bytes one step pass moves: 6 node vectors read and 5 written (24 B each)
// plus the 3x3 inverse block per FEM vertex; 12x12 blocks per body.
static double update_bytes(const ipc_ctx *c) { return (264.0 + 72.0) * c->NFEM + (4 * 264.0 + 1152.0) * c->NB; }

void pcg_solve(ipc_ctx *c, const double *b, double *x, double eta, const int *want)
{
    Dev &D = c->d;
    hipStream_t st = c->stream;
    const int ns = c->n_scenes, ntile = c->N / TILE;
    double *r = D.r.p, *z = D.z.p, *p = D.p.p, *s = D.q.p, *w = D.w.p;
    // the one-launch step keeps r, z and s of odd iterations in buffers of
    // their own; otherwise the step updates them in place
    const bool fused = c->cg_fusable && c->coarse_on && c->pcg_fused && c->n_cdom > 0;
    double *rb[2] = {r, fused ? D.r2.p : r}, *zb[2] = {z, fused ? D.z2.p : z}, *sb[2] = {s, fused ? D.q2.p : s};
    const int nwin = fused ? std::max(c->n_cdom, (ntile + CG_SPLIT * WG_TILES - 1) / (CG_SPLIT * WG_TILES)) : 0;
    D.part_node3.alloc(ntile + 1);
    D.part_long.alloc(c->long_cap + 1);
    D.pcg_part.alloc(4 * (size_t)ntile + 1);
    D.pcg_st.alloc(8 * (size_t)ns);
    D.pcg_act.alloc(2 * (size_t)ns);
    D.pcg_it.alloc(2 * (size_t)ns);
    D.pcg_prev.alloc(ns);
    int *act = D.pcg_act.p;
    hipLaunchKernelGGL(k_pcg_init, dim3(blocks_for(c->N)), dim3(BLOCK), 0, st, c->N, ns, D.node_kind.p, D.node_body.p,
                       D.tile_scene_node.p, seg_ptr(c, R_NODEW), b, D.dinv.p, D.dinvB.p, x, r, z, p, s, D.pcg_part.p, ntile, want, eta,
                       D.sparam.p, D.pcg_st.p, D.pcg_prev.p, act, D.pcg_it.p, D.pcg_iters.p, D.scal.p);
    coarse_apply(c, act, r, z, 0);              // z += the coarse correction of r, its r . z partials
    hess_apply(c, z, w, act, D.part_node3.p);   // w = A z and z . w for the first step
    int maxit = 0;
    for (auto &S : c->sc) maxit = std::max(maxit, S.max_pcg);
    // one iteration of parity q; every kernel skips scenes that stopped, so
    // extra iterations after convergence change nothing
    auto iteration = [&](int q) {
        prof_begin(c, IPC_K_PCG_UPDATE);
        const int ncd = c->coarse_on ? CG_SPLIT * c->n_cdom : 0;
        double *cg_out = D.cg_part.p + (size_t)(q ^ 1) * ncd;
        if (fused)
            hipLaunchKernelGGL(k_pcg_step<true>, dim3(NXCD * CG_SPLIT * ((nwin + NXCD - 1) / NXCD)), dim3(BLOCK), 0, c->stream, c->N, ns,
                               q, D.node_kind.p, D.node_body.p, D.tile_scene_node.p, seg_ptr(c, R_NODEW), seg_ptr(c, R_LONG),
                               seg_ptr(c, R_CDOM), D.pcg_wginfo.p, 1, c->long_cap, D.cg_part.p, ncd, D.maxpcg.p, D.dinv.p, D.dinvB.p,
                               w, p, sb[q], sb[q ^ 1], x, rb[q], rb[q ^ 1], zb[q], zb[q ^ 1], D.part_node3.p, D.part_long.p,
                               D.pcg_part.p, ntile, D.pcg_st.p, act, D.pcg_it.p, D.pcg_st.p, act, D.pcg_it.p, D.scal.p, c->n_cdom,
                               nwin, c->cg_nfr, c->sc[0].bnode0,
                               D.cg_ph_ptr.p, D.cg_ph_e.p, D.cg_ph_n.p, D.cg_node_da.p, D.cg_inv.p, cg_out);
        else
            hipLaunchKernelGGL(k_pcg_step<false>, dim3(blocks_for(c->N)), dim3(BLOCK), 0, c->stream, c->N, ns, q, D.node_kind.p,
                               D.node_body.p, D.tile_scene_node.p, seg_ptr(c, R_NODEW), seg_ptr(c, R_LONG), seg_ptr(c, R_CDOM),
                               D.pcg_wginfo.p, (int)(ns == 1), c->long_cap, D.cg_part.p, ncd, D.maxpcg.p, D.dinv.p, D.dinvB.p, w, p,
                               s, s, x, r, r, z, z, D.part_node3.p, D.part_long.p, D.pcg_part.p, ntile, D.pcg_st.p, act, D.pcg_it.p,
                               D.pcg_st.p, act, D.pcg_it.p, D.scal.p, 0, 0, 0, 0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
        prof_end(c, IPC_K_PCG_UPDATE, update_bytes(c));
        if (!fused) coarse_apply(c, act + (q ^ 1) * ns, r, z, q ^ 1);
        hess_apply(c, zb[q ^ 1], w, act + (q ^ 1) * ns, D.part_node3.p);
    };
    // The peek kernel publishes one word per scene into pinned, coherent host
    // memory, which the host polls: no event and no stream synchronisation
    // per batch.  If the words do not appear within a second the host
    // synchronises the stream (which also reports a failed launch) and reads
    // them again.
    if (!c->h_peek) {
        IPC_HIP(hipHostMalloc((void **)&c->h_peek, 2 * (size_t)ns * sizeof(unsigned long long), hipHostMallocMapped | hipHostMallocCoherent));
        IPC_HIP(hipHostGetDevicePointer((void **)&c->h_peek_dev, c->h_peek, 0));
        for (size_t i = 0; i < 2 * (size_t)ns; ++i) c->h_peek[i] = 0;
    }
    auto peek = [&](int q, int slot, int n_since) {
        unsigned int seq = ++c->peek_seq;
        if (seq == 0) seq = ++c->peek_seq;   // 0 never names a peek
        hipLaunchKernelGGL(k_pcg_peek, dim3(ns), dim3(BLOCK), 0, st, ns, q, seg_ptr(c, R_NODEW), D.maxpcg.p, D.pcg_part.p, ntile,
                           D.pcg_st.p, act, D.pcg_it.p, D.pcg_prev.p, n_since, seq, c->h_peek_dev + (size_t)ns * slot,
                           D.pcg_iters.p);
        return seq;
    };
    // 0 when no scene iterates any more, else the largest estimate
    auto await = [&](int slot, unsigned int seq) {
        volatile unsigned long long *wv = c->h_peek + (size_t)ns * slot;
        auto ready = [&]() {
            for (int k = 0; k < ns; ++k)
                if ((unsigned int)(wv[k] >> 32) != seq) return false;
            return true;
        };
        auto t0 = std::chrono::steady_clock::now();
        while (!ready()) {
            if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(1)) {
                IPC_HIP(hipStreamSynchronize(st));
                if (!ready()) throw Error(IPC_E_DEVICE, "PCG progress words did not reach host memory");
                break;
            }
        }
        int left = 0;
        for (int k = 0; k < ns; ++k) left = std::max(left, (int)(unsigned int)(wv[k] & 0xffffffffull));
        return left;
    };
    const int KB = 16, KS = 4;   // iterations per batch (even): far from and near convergence
    const int Ks[2] = {KB, KS};
    // Two copies of a long and of a short batch of iterations, captured on
    // the context's capture stream (the caller's stream may be the null
    // stream, which cannot capture) and kept while the arguments they were
    // captured with stay the same; consecutive replays of one batch length
    // alternate between the copies, so a replay never waits for the previous
    // replay of the same executable.  Both lengths are even, so every replay
    // starts at parity 0.
    const bool graphs = c->use_graphs && !c->prof;
    if (graphs) {
        std::vector<uintptr_t> key = {(uintptr_t)c->N, (uintptr_t)ns, (uintptr_t)c->spmv_lanes, (uintptr_t)c->long_cap,
                                      (uintptr_t)D.node_kind.p, (uintptr_t)D.node_body.p, (uintptr_t)D.tile_scene_node.p,
                                      (uintptr_t)D.segs.p, (uintptr_t)D.maxpcg.p, (uintptr_t)D.dinv.p, (uintptr_t)D.dinvB.p, (uintptr_t)w,
                                      (uintptr_t)p, (uintptr_t)s, (uintptr_t)x, (uintptr_t)r, (uintptr_t)z, (uintptr_t)D.part_node3.p,
                                      (uintptr_t)D.part_long.p, (uintptr_t)D.pcg_part.p, (uintptr_t)D.pcg_st.p, (uintptr_t)act,
                                      (uintptr_t)D.pcg_it.p, (uintptr_t)D.scal.p, (uintptr_t)D.long_count.p, (uintptr_t)D.long_rows.p,
                                      (uintptr_t)D.row_ptr.p, (uintptr_t)D.col.p, (uintptr_t)D.val.p, (uintptr_t)D.dyn_ptr.p,
                                      (uintptr_t)D.dyn_col.p, (uintptr_t)D.dyn_val.p, (uintptr_t)D.node_scene.p,
                                      (uintptr_t)D.pcg_wginfo.p, (uintptr_t)(c->coarse_on ? c->n_cdom : 0), (uintptr_t)D.cg_ent.p, (uintptr_t)D.cg_nodes.p,
                                      (uintptr_t)D.cg_dom_scene.p, (uintptr_t)D.cg_inv.p, (uintptr_t)D.cg_part.p, (uintptr_t)D.cg_pnodes.p,
                                      (uintptr_t)fused, (uintptr_t)D.r2.p, (uintptr_t)D.z2.p, (uintptr_t)D.q2.p, (uintptr_t)D.cg_node_da.p,
                                      (uintptr_t)c->cg_nfr, (uintptr_t)D.cg_ph_ptr.p, (uintptr_t)D.cg_ph_e.p, (uintptr_t)D.cg_ph_n.p};
        bool have = key == c->pcg_key;
        for (auto xg : c->pcg_exec) have = have && xg;
        if (!have) {
            for (auto &xg : c->pcg_exec) if (xg) { (void)hipGraphExecDestroy(xg); xg = nullptr; }
            c->pcg_key.clear();
            hipError_t e = hipSuccess;
            for (int g = 0; g < 4 && e == hipSuccess; ++g) {
                hipGraph_t graph = nullptr;
                c->stream = c->cap_stream;
                e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
                if (e == hipSuccess) {
                    for (int k = 0; k < Ks[g / 2]; ++k) iteration(k & 1);
                    e = hipStreamEndCapture(c->cap_stream, &graph);
                }
                c->stream = st;
                if (e == hipSuccess) {
                    e = hipGraphInstantiate(&c->pcg_exec[g], graph, nullptr, nullptr, 0);
                    (void)hipGraphDestroy(graph);
                }
            }
            IPC_HIP(e);
            c->pcg_key = key;
        }
    }
    // Batches are pipelined: each batch is followed by a peek whose result
    // lands in host memory behind an event, and while the estimate asks for
    // more iterations than are already in flight, a second batch is queued
    // before the host waits for the first one's peek.  A batch queued past
    // convergence does nothing.
    int launched = 0, nb = 0, k_done = 0, inflight = 0, size_of[2] = {0, 0}, replays[2] = {0, 0};
    unsigned int seq_of[2] = {0, 0};
    int left = PCG_EST_UNKNOWN;
    auto launch_batch = [&](int g) {
        if (graphs) IPC_HIP(hipGraphLaunch(c->pcg_exec[2 * g + (replays[g]++ & 1)], st));
        else for (int k = 0; k < Ks[g]; ++k) iteration(k & 1);
        int slot = nb & 1;
        seq_of[slot] = peek(0, slot, Ks[g]);
        size_of[slot] = Ks[g];
        launched += Ks[g];
        inflight += Ks[g];
        ++nb;
    };
    while (true) {
        if (nb - k_done < 2 && launched < maxit && left > inflight) launch_batch(left - inflight > KB ? 0 : 1);
        if (k_done == nb) break;   // nothing in flight: the iteration cap is reached
        int slot = k_done & 1;
        left = await(slot, seq_of[slot]);
        inflight -= size_of[slot];
        ++k_done;
        if (left == 0) break;
    }
}

} // namespace ipc
