// Contact: world positions, LBVH broad phase, narrow phase, IPC log-barrier,
// lagged friction, contact Hessian products and additive CCD
// (Sec. III-C.1, "barrier potentials together with continuous collision
// detection"; Eq. (3) E_barrier and E_friction).
//
// Broad phase: one linear BVH per scene and primitive kind (triangles for
// point-triangle queries, edges for edge-edge queries), built in a single
// launch sequence over all scenes: Morton keys carry the scene id in their
// high bits so one radix sort groups the scenes; the Karras hierarchy is
// built per scene segment; boxes are refitted bottom-up with arrival
// counters; queries traverse only their own scene's tree.  Candidates are
// compacted with count / exclusive-scan / write passes, which keeps their
// order deterministic.  The narrow phase keeps a candidate when d^2 < dhat^2
// and compacts the survivors with a wavefront ballot and a scan over
// per-wavefront counts.
#include <hipcub/hipcub.hpp>
#include <rocprim/device/device_radix_sort.hpp>

#include "ipc_device.h"
#include "ipc_internal.h"
#include "ipc_runsum.h"
#include "ipc_kernels.h"

namespace ipc {

// ---------------------------------------------------------------------------
// world positions of contact vertices (exact operation order)
// ---------------------------------------------------------------------------
__global__ void k_world(int CV, const double *__restrict__ y, const int *__restrict__ cv_node, const int *__restrict__ cv_body,
                        const double *__restrict__ cv_x, const int *__restrict__ body_node0, double *__restrict__ xw)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= CV) return;
    int n = cv_node[i];
    d3 x;
    if (n >= 0) x = ld3(y, n);
    else {
        int b = cv_body[i];
        d3 xb = ld3(cv_x, i);
        if (b >= 0) {
            int n0 = body_node0[b];
            x = xaffine(ld3(y, n0), ld3(y, n0 + 1), ld3(y, n0 + 2), ld3(y, n0 + 3), xb);
        } else x = xb;
    }
    st3(xw, i, x);
}

void launch_world(ipc_ctx *c, const double *y, double *xw)
{
    if (c->CV == 0) return;
    hipLaunchKernelGGL(k_world, dim3(blocks_for(c->CV)), dim3(BLOCK), 0, c->stream, c->CV, y, c->d.cv_node.p, c->d.cv_body.p,
                       c->d.cv_x.p, c->d.body_node0.p, xw);
}

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ void box_of(const double *xw0, const double *xw1, const int *v, int nv, double r, double *b)
{
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int k = 0; k < nv; ++k) {
        d3 p = ld3(xw0, v[k]);
        lo[0] = fmin(lo[0], p.x); lo[1] = fmin(lo[1], p.y); lo[2] = fmin(lo[2], p.z);
        hi[0] = fmax(hi[0], p.x); hi[1] = fmax(hi[1], p.y); hi[2] = fmax(hi[2], p.z);
        if (xw1) {
            d3 q = ld3(xw1, v[k]);
            lo[0] = fmin(lo[0], q.x); lo[1] = fmin(lo[1], q.y); lo[2] = fmin(lo[2], q.z);
            hi[0] = fmax(hi[0], q.x); hi[1] = fmax(hi[1], q.y); hi[2] = fmax(hi[2], q.z);
        }
    }
    for (int k = 0; k < 3; ++k) { b[k] = lo[k] - r; b[3 + k] = hi[k] + r; }
}

__device__ __forceinline__ bool overlap(const double *a, const double *b)
{
    return a[0] <= b[3] && b[0] <= a[3] && a[1] <= b[4] && b[1] <= a[4] && a[2] <= b[5] && b[2] <= a[5];
}

__device__ __forceinline__ bool allowed(int oa, int ob, const int *okind, const int *excl, int nex)
{
    int ka = oa >= 0 ? okind[oa] : 2, kb = ob >= 0 ? okind[ob] : 2;
    if (ka == 2 && kb == 2) return false;
    if (oa == ob && ka == 1) return false;
    for (int i = 0; i < nex; ++i) {
        int a = excl[2 * i], b = excl[2 * i + 1];
        if ((a == oa && b == ob) || (a == ob && b == oa)) return false;
    }
    return true;
}

__device__ __forceinline__ unsigned int expand_bits(unsigned int v)
{
    v = (v * 0x00010001u) & 0xFF0000FFu;
    v = (v * 0x00000101u) & 0x0F00F00Fu;
    v = (v * 0x00000011u) & 0xC30C30C3u;
    v = (v * 0x00000005u) & 0x49249249u;
    return v;
}

// ---------------------------------------------------------------------------
// LBVH
// ---------------------------------------------------------------------------
// primitive boxes + Morton keys.  kind 0: triangles, 1: edges.
__global__ void k_prim_box(int P, int kind, const int4 *__restrict__ tri, const int2 *__restrict__ edge, const int *__restrict__ cv_scene,
                           const double *__restrict__ xw0, const double *__restrict__ xw1, const double *__restrict__ sparam,
                           const double *__restrict__ sbox, double *__restrict__ box, unsigned long long *__restrict__ key,
                           int *__restrict__ id)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    int v[3], nv, s;
    if (kind == 0) { int4 t = tri[i]; v[0] = t.x; v[1] = t.y; v[2] = t.z; nv = 3; s = t.w; }
    else { int2 e = edge[i]; v[0] = e.x; v[1] = e.y; nv = 2; s = cv_scene[e.x]; }
    double r = kind == 0 ? 0.0 : 0.5 * 1.01 * sparam[8 * s + 2];
    double b[6];
    box_of(xw0, xw1, v, nv, r, b);
#pragma unroll
    for (int k = 0; k < 6; ++k) box[6 * (size_t)i + k] = b[k];
    const double *sb = sbox + 6 * (size_t)s;
    unsigned int q[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double cc = (0.5 * (b[k] + b[3 + k]) - sb[k]) * sb[3 + k];
        cc = fmin(fmax(cc, 0.0), 1023.0);
        q[k] = (unsigned int)cc;
    }
    unsigned int m = (expand_bits(q[0]) << 2) | (expand_bits(q[1]) << 1) | expand_bits(q[2]);
    key[i] = ((unsigned long long)s << 32) | m;
    id[i] = i;
}

// Morton keys of the surface-vertex queries (centre of the swept point, or the
// point itself when there is no end position: xw1 = nullptr), so that
// neighbouring lanes of a wavefront traverse neighbouring parts of the tree;
// the scene id sits above the code as for the leaves.
__global__ void k_query_keys(int Q, const int *__restrict__ cv_scene, const double *__restrict__ xw0, const double *__restrict__ xw1,
                             const double *__restrict__ sbox, unsigned long long *__restrict__ key, int *__restrict__ id)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Q) return;
    int s = cv_scene[i];
    const double *sb = sbox + 6 * (size_t)s;
    unsigned int q[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double x0 = xw0[3 * (size_t)i + k], x1 = xw1 ? xw1[3 * (size_t)i + k] : x0;
        double cc = (0.5 * (x0 + x1) - sb[k]) * sb[3 + k];
        cc = fmin(fmax(cc, 0.0), 1023.0);
        q[k] = (unsigned int)cc;
    }
    unsigned int m = (expand_bits(q[0]) << 2) | (expand_bits(q[1]) << 1) | expand_bits(q[2]);
    key[i] = ((unsigned long long)s << 32) | m;
    id[i] = i;
}

__device__ __forceinline__ int lcp(const unsigned long long *key, int base, int n, int a, int b)
{
    if (b < 0 || b >= n) return -1;
    unsigned long long ka = key[base + a], kb = key[base + b];
    if (ka == kb) return 64 + __clz((unsigned int)(a ^ b));
    return __clzll(ka ^ kb);
}

// Karras (2012) internal nodes per scene segment [seg[s], seg[s+1]).
// Internal node ids share the leaf numbering: node seg[s]+j, j < n-1.
// Child encoding: >= 0 internal node, < 0 leaf -1-k (k = sorted position).
__global__ void k_karras(int P, const int *__restrict__ prim_scene_of_sorted, const int *__restrict__ seg,
                         const unsigned long long *__restrict__ key, int *__restrict__ left, int *__restrict__ right,
                         int2 *__restrict__ range)
{
    int gi = blockIdx.x * blockDim.x + threadIdx.x;
    if (gi >= P) return;
    int s = prim_scene_of_sorted[gi];
    int base = seg[s], n = seg[s + 1] - base;
    int i = gi - base;
    if (i >= n - 1) { range[gi] = make_int2(-1, -1); return; }
    int d = (lcp(key, base, n, i, i + 1) - lcp(key, base, n, i, i - 1)) >= 0 ? 1 : -1;
    int dmin = lcp(key, base, n, i, i - d);
    int lmax = 2;
    while (lcp(key, base, n, i, i + lmax * d) > dmin) lmax *= 2;
    int l = 0;
    for (int t = lmax / 2; t >= 1; t /= 2)
        if (lcp(key, base, n, i, i + (l + t) * d) > dmin) l += t;
    int j = i + l * d;
    int dnode = lcp(key, base, n, i, j);
    int sp = 0, t = l;
    do {
        t = (t + 1) >> 1;
        if (lcp(key, base, n, i, i + (sp + t) * d) > dnode) sp += t;
    } while (t > 1);
    int gamma = i + sp * d + min(d, 0);
    int lo = min(i, j), hi = max(i, j);
    int L = (lo == gamma) ? -1 - (base + gamma) : base + gamma;
    int R = (hi == gamma + 1) ? -1 - (base + gamma + 1) : base + gamma + 1;
    left[gi] = L;
    right[gi] = R;
    range[gi] = make_int2(base + lo, base + hi);   // sorted leaves covered by the node
}

// Node boxes.  A Karras node covers a contiguous range of sorted leaves, so
// its box is a range union.  A perfect binary tree of unions over the sorted
// leaf boxes (levels built 8 at a time in LDS, one workgroup per 256 inputs)
// answers every node's range with O(log P) independent loads, and no
// workgroup waits on another (a bottom-up refit would need device-scope
// fences, which write back the XCD's L2 at every level).
struct SegLevels { int n; int off[32]; int size[32]; };

__device__ __forceinline__ void box_union(double *a, const double *b)
{
    for (int m = 0; m < 3; ++m) { a[m] = fmin(a[m], b[m]); a[3 + m] = fmax(a[3 + m], b[3 + m]); }
}
__device__ __forceinline__ void box_empty(double *a)
{
    for (int m = 0; m < 3; ++m) { a[m] = INFINITY; a[3 + m] = -INFINITY; }
}

// level 0: the leaf boxes in sorted order, and 1 for every sorted leaf whose
// primitive is not static (its object moves)
__global__ void k_seg_leaves(int P, int kind, const int *__restrict__ sorted_id, const double *__restrict__ pbox,
                             const int4 *__restrict__ tri, const int2 *__restrict__ edge, const int *__restrict__ cv_obj,
                             const int *__restrict__ okind, double *__restrict__ lev, int *__restrict__ moving)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    int pid = sorted_id[i];
    const double *b = pbox + 6 * (size_t)pid;
    for (int m = 0; m < 6; ++m) lev[6 * (size_t)i + m] = b[m];
    int o = cv_obj[kind == 0 ? tri[pid].x : edge[pid].x];
    moving[i] = (o >= 0 ? okind[o] : 2) != 2 ? 1 : 0;
}

// levels j0+1 .. j0+8 from level j0 (256 inputs per workgroup)
__global__ void __launch_bounds__(256) k_seg_up(SegLevels L, int j0, double *__restrict__ lev)
{
    __shared__ double sh[256][6];
    int t = threadIdx.x, i = blockIdx.x * 256 + t;
    if (i < L.size[j0]) for (int m = 0; m < 6; ++m) sh[t][m] = lev[6 * ((size_t)L.off[j0] + i) + m];
    else box_empty(sh[t]);
    __syncthreads();
    for (int step = 1; step <= 8 && j0 + step < L.n; ++step) {
        int w = 256 >> step;
        double b[6];
        if (t < w) {
            for (int m = 0; m < 6; ++m) b[m] = sh[2 * t][m];
            box_union(b, sh[2 * t + 1]);
        }
        __syncthreads();
        if (t < w) {
            for (int m = 0; m < 6; ++m) sh[t][m] = b[m];
            int j = j0 + step, k = blockIdx.x * w + t;
            if (k < L.size[j]) for (int m = 0; m < 6; ++m) lev[6 * ((size_t)L.off[j] + k) + m] = b[m];
        }
        __syncthreads();
    }
}

// every internal node: the union over its leaf range [lo, hi], and whether
// the range holds a moving primitive (from the exclusive scan of the flags)
__global__ void k_node_box(int P, SegLevels L, const double *__restrict__ lev, const int2 *__restrict__ range,
                           const int *__restrict__ moving_scan, double *__restrict__ nbox, int *__restrict__ nmoving)
{
    int gi = blockIdx.x * blockDim.x + threadIdx.x;
    if (gi >= P) return;
    int2 rg = range[gi];
    if (rg.x < 0) return;
    nmoving[gi] = moving_scan[rg.y + 1] - moving_scan[rg.x] > 0 ? 1 : 0;
    double acc[6];
    box_empty(acc);
    int l = rg.x, r = rg.y + 1;
    for (int j = 0; j < L.n && l < r; ++j, l >>= 1, r >>= 1) {
        if (l & 1) { box_union(acc, lev + 6 * ((size_t)L.off[j] + l)); ++l; }
        if (r & 1) { --r; box_union(acc, lev + 6 * ((size_t)L.off[j] + r)); }
    }
    for (int m = 0; m < 6; ++m) nbox[6 * (size_t)gi + m] = acc[m];
}

// Queries.  kind 0: surface vertex vs triangle tree; kind 1: edge vs edge tree.
// Thread t takes query perm[t] (Morton order).  WRITE = false counts and
// stashes the first TRAV_STASH candidates of each query; WRITE = true writes
// every candidate at off[q]: from the stash when it held them all, else by
// traversing again (with stash = nullptr: always traversing).
constexpr int TRAV_BLOCK = 128, TRAV_DEPTH = 64;
template <bool WRITE>
__global__ void __launch_bounds__(TRAV_BLOCK) k_traverse(int Q, int kind, const int2 *__restrict__ qedge, const int *__restrict__ cv_scene,
                           const int4 *__restrict__ tri, const int2 *__restrict__ edge, const int *__restrict__ cv_obj,
                           const int *__restrict__ okind, const int *__restrict__ excl, int nex, const double *__restrict__ xw0,
                           const double *__restrict__ xw1, const double *__restrict__ sparam, const int *__restrict__ seg,
                           const int *__restrict__ sorted_id, const double *__restrict__ pbox, const int *__restrict__ left,
                           const int *__restrict__ right, const double *__restrict__ nbox, const int *__restrict__ nmoving,
                           double grow, const int *__restrict__ perm,
                           int *__restrict__ count, const int *__restrict__ off, int2 *__restrict__ out, int *__restrict__ overflow,
                           int2 *__restrict__ stash)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= Q) return;
    int qi = perm[t];
    if (WRITE && stash) {
        int n = count[qi];
        if (n <= TRAV_STASH) {
            int o = off[qi];
            for (int c = 0; c < n; ++c) out[o + c] = stash[(size_t)qi * TRAV_STASH + c];
            return;
        }
    }
    int qv[2], nq, s;
    if (kind == 0) { qv[0] = qi; nq = 1; s = cv_scene[qi]; }
    else { int2 e = qedge[qi]; qv[0] = e.x; qv[1] = e.y; nq = 2; s = cv_scene[e.x]; }
    double r = 1.01 * sparam[8 * s + 2] * (kind == 0 ? 1.0 : 0.5) + grow * sparam[8 * s + 2];
    double qb[6];
    box_of(xw0, xw1, qv, nq, r, qb);
    int oq = cv_obj[qv[0]];
    // a static query pairs only with moving primitives: subtrees without one are skipped
    const bool qstatic = (oq >= 0 ? okind[oq] : 2) == 2;
    int base = seg[s], n = seg[s + 1] - base;
    int cnt = 0, w = WRITE ? off[qi] : 0;
    // traversal stack in LDS, one column per thread (a private array would
    // live in scratch memory); children are tested before they are pushed
    __shared__ int stk[TRAV_DEPTH * TRAV_BLOCK];
    int *my = stk + threadIdx.x;
    auto leaf = [&](int pid) {
        if (!overlap(qb, pbox + 6 * (size_t)pid)) return;
        bool ok;
        int ob;
        if (kind == 0) {
            int4 t = tri[pid];
            ok = qi != t.x && qi != t.y && qi != t.z;
            ob = cv_obj[t.x];
        } else {
            int2 f = edge[pid];
            ok = pid > qi && qv[0] != f.x && qv[0] != f.y && qv[1] != f.x && qv[1] != f.y;
            ob = cv_obj[f.x];
        }
        if (ok && allowed(oq, ob, okind, excl, nex)) {
            if (WRITE) out[w + cnt] = make_int2(qi, pid);
            else if (cnt < TRAV_STASH) stash[(size_t)qi * TRAV_STASH + cnt] = make_int2(qi, pid);
            ++cnt;
        }
    };
    if (n == 1) leaf(sorted_id[base]);
    else if (n > 1 && !(qstatic && !nmoving[base]) && overlap(qb, nbox + 6 * (size_t)base)) {
        int sp = 0;
        my[0] = base;
        sp = 1;
        while (sp > 0) {
            int node = my[TRAV_BLOCK * --sp];
            int ch[2] = {left[node], right[node]};
            for (int c2 = 0; c2 < 2; ++c2) {
                int x = ch[c2];
                if (x < 0) { leaf(sorted_id[-1 - x]); continue; }
                if (qstatic && !nmoving[x]) continue;
                if (!overlap(qb, nbox + 6 * (size_t)x)) continue;
                if (sp >= TRAV_DEPTH) { atomicOr(overflow, 1); continue; }
                my[TRAV_BLOCK * sp++] = x;
            }
        }
    }
    if (!WRITE) {
        count[qi] = cnt;
        if (cnt > TRAV_STASH) atomicOr(overflow + 1, 1);
    }
}

// candidates of every query from its stash, at its scanned offset
__global__ void k_unstash(int Q, const int *__restrict__ count, const int *__restrict__ off, const int2 *__restrict__ stash,
                          int2 *__restrict__ out)
{
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= Q) return;
    int n = count[q], o = off[q];
    for (int c = 0; c < n; ++c) out[o + c] = stash[(size_t)q * TRAV_STASH + c];
}

__global__ void k_scene_of_sorted(int P, const unsigned long long *__restrict__ key, int *__restrict__ sc)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < P) sc[i] = (int)(key[i] >> 32);
}

__global__ void k_fill_int(int n, int *p, int v)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// per-scene segment offsets of a query-ordered output from its exclusive
// scan (qseg[n_scenes] = number of queries, off[that] = total)
__global__ void k_seg_from_scan(int n_scenes, const int *__restrict__ qseg, const int *__restrict__ off, int *__restrict__ seg)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s > n_scenes) return;
    seg[s] = off[qseg[s]];
}

// per-scene segments of a ballot-compacted list: survivors before each
// scene's first candidate (cseg), from the wavefront masks and their scan
__global__ void k_compact_seg(int n_scenes, int ncand, const int *__restrict__ cseg, const unsigned long long *__restrict__ mask,
                              const int *__restrict__ woff, int nw, int *__restrict__ seg)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s > n_scenes) return;
    int q = cseg[s];
    if (q >= ncand) { seg[s] = woff[nw]; return; }
    int w = q / TILE, l = q % TILE;
    seg[s] = woff[w] + (l ? __popcll(mask[w] & ((1ull << l) - 1ull)) : 0);
}

void exclusive_scan_int(ipc_ctx *c, const int *in, int *out, int n)
{
    size_t bytes = 0;
    IPC_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, in, out, n + 1, c->stream));
    c->d.sort_tmp.alloc(bytes + 16);
    IPC_HIP(hipcub::DeviceScan::ExclusiveSum(c->d.sort_tmp.p, bytes, in, out, n + 1, c->stream));
}

// exclusive scan helper (count[n] -> off[n + 1], off[n] = total)
static void exclusive_scan(ipc_ctx *c, const int *in, int *out, int n)
{
    size_t bytes = 0;
    IPC_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, in, out, n + 1, c->stream));
    c->d.sort_tmp.alloc(bytes + 16);
    IPC_HIP(hipcub::DeviceScan::ExclusiveSum(c->d.sort_tmp.p, bytes, in, out, n + 1, c->stream));
}

// Build the tree over one primitive kind and run one query kind against it.
static void bvh_query(ipc_ctx *c, int kind, const double *xw0, const double *xw1, double grow, DBuf<int2> &outbuf, int64_t &cap,
                      int64_t &count, std::vector<int> &hseg)
{
    Dev &D = c->d;
    hipStream_t st = c->stream;
    int P = kind == 0 ? c->TRI : c->EDGE;
    int Q = kind == 0 ? c->NSURF : c->EDGE;
    int ns = c->n_scenes;
    hseg.assign(ns + 1, 0);
    count = 0;
    if (P == 0 || Q == 0) {
        hipLaunchKernelGGL(k_fill_int, dim3(blocks_for(ns + 1)), dim3(BLOCK), 0, st, ns + 1, seg_ptr(c, kind == 0 ? R_CPT : R_CEE), 0);
        return;
    }
    D.box.alloc(6 * (size_t)P); D.mkey.alloc(P); D.mkey2.alloc(P); D.mid.alloc(P); D.mid2.alloc(P);
    D.bvh_left.alloc(P); D.bvh_right.alloc(P); D.bvh_range.alloc(P); D.bvh_flag.alloc(P); D.bvh_box.alloc(6 * (size_t)P);
    D.qcount.alloc(Q + 1); D.qoff.alloc(Q + 1); D.qstash.alloc((size_t)Q * TRAV_STASH);
    hipLaunchKernelGGL(k_prim_box, dim3(blocks_for(P)), dim3(BLOCK), 0, st, P, kind, D.tri.p, D.edge.p, D.cv_scene.p, xw0, xw1,
                       D.sparam.p, D.scene_lo.p, D.box.p, D.mkey.p, D.mid.p);
    size_t bytes = 0;
    int end_bit = 32;
    while ((1 << (end_bit - 32)) < ns) ++end_bit;
    IPC_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, D.mkey.p, D.mkey2.p, D.mid.p, D.mid2.p, P, 0, end_bit, st));
    D.sort_tmp.alloc(bytes + 16);
    IPC_HIP(hipcub::DeviceRadixSort::SortPairs(D.sort_tmp.p, bytes, D.mkey.p, D.mkey2.p, D.mid.p, D.mid2.p, P, 0, end_bit, st));
    int *pseg_d = seg_ptr(c, kind == 0 ? R_TRI : R_EDGE);
    int *qseg_d = seg_ptr(c, kind == 0 ? R_SURF : R_EDGE);
    int *sseg = seg_ptr(c, kind == 0 ? R_CPT : R_CEE);
    int *scene_sorted = D.bvh_flag.p;   // scratch: scene of each sorted leaf
    hipLaunchKernelGGL(k_scene_of_sorted, dim3(blocks_for(P)), dim3(BLOCK), 0, st, P, D.mkey2.p, scene_sorted);
    hipLaunchKernelGGL(k_karras, dim3(blocks_for(P)), dim3(BLOCK), 0, st, P, scene_sorted, pseg_d, D.mkey2.p, D.bvh_left.p,
                       D.bvh_right.p, D.bvh_range.p);
    // node boxes from the union tree over the sorted leaf boxes
    SegLevels SL{};
    {
        int64_t total = 0;
        int sz = P;
        for (SL.n = 0; SL.n < 32; ++SL.n) {
            SL.off[SL.n] = (int)total;
            SL.size[SL.n] = sz;
            total += sz;
            if (sz == 1) { ++SL.n; break; }
            sz = (sz + 1) / 2;
        }
        D.bvh_lev.alloc(6 * (size_t)total);
    }
    D.bvh_moving.alloc(P + 1); D.bvh_mscan.alloc(P + 1); D.bvh_nmoving.alloc(P);
    hipLaunchKernelGGL(k_seg_leaves, dim3(blocks_for(P)), dim3(BLOCK), 0, st, P, kind, D.mid2.p, D.box.p, D.tri.p, D.edge.p, D.cv_obj.p,
                       D.obj_kind.p, D.bvh_lev.p, D.bvh_moving.p);
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, st, 1, D.bvh_moving.p + P, 0);
    exclusive_scan(c, D.bvh_moving.p, D.bvh_mscan.p, P);
    for (int j0 = 0; j0 + 1 < SL.n; j0 += 8)
        hipLaunchKernelGGL(k_seg_up, dim3(blocks_for(SL.size[j0], 256)), dim3(256), 0, st, SL, j0, D.bvh_lev.p);
    hipLaunchKernelGGL(k_node_box, dim3(blocks_for(P)), dim3(BLOCK), 0, st, P, SL, D.bvh_lev.p, D.bvh_range.p, D.bvh_mscan.p,
                       D.bvh_box.p, D.bvh_nmoving.p);
    DBuf<int> &ovf = D.woff;
    ovf.alloc(2);
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, st, 2, ovf.p, 0);
    const int2 *qedge = D.edge.p;
    // query order: edges in their own tree's sorted order; surface vertices by their own Morton keys
    const int *perm = D.mid2.p;
    if (kind == 0) {
        D.qkey.alloc(Q); D.qkey2.alloc(Q); D.qid.alloc(Q); D.qperm.alloc(Q);
        hipLaunchKernelGGL(k_query_keys, dim3(blocks_for(Q)), dim3(BLOCK), 0, st, Q, D.cv_scene.p, xw0, xw1, D.scene_lo.p, D.qkey.p, D.qid.p);
        size_t qb = 0;
        IPC_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, qb, D.qkey.p, D.qkey2.p, D.qid.p, D.qperm.p, Q, 0, end_bit, st));
        D.sort_tmp.alloc(qb + 16);
        IPC_HIP(hipcub::DeviceRadixSort::SortPairs(D.sort_tmp.p, qb, D.qkey.p, D.qkey2.p, D.qid.p, D.qperm.p, Q, 0, end_bit, st));
        perm = D.qperm.p;
    }
    hipLaunchKernelGGL(k_traverse<false>, dim3(blocks_for(Q, TRAV_BLOCK)), dim3(TRAV_BLOCK), 0, st, Q, kind, qedge, D.cv_scene.p, D.tri.p, D.edge.p,
                       D.cv_obj.p, D.obj_kind.p, D.excl.p, c->NEX, xw0, xw1, D.sparam.p, pseg_d, D.mid2.p, D.box.p, D.bvh_left.p,
                       D.bvh_right.p, D.bvh_box.p, D.bvh_nmoving.p, grow, perm, D.qcount.p, nullptr, nullptr, ovf.p, D.qstash.p);
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, st, 1, D.qcount.p + Q, 0);
    exclusive_scan(c, D.qcount.p, D.qoff.p, Q);
    // the candidates' per-scene segments go straight to the device table
    hipLaunchKernelGGL(k_seg_from_scan, dim3(blocks_for(ns + 1)), dim3(BLOCK), 0, st, ns, qseg_d, D.qoff.p, sseg);
    int total = 0, of[2] = {0, 0};
    {
        HostReads r(c);
        r.add(&total, D.qoff.p + Q, sizeof(int));
        r.add(of, ovf.p, 2 * sizeof(int));
        r.add(hseg.data(), sseg, (ns + 1) * sizeof(int));
        r.wait();
    }
    if (of[0]) throw Error(IPC_E_CAPACITY, "BVH traversal stack overflow");
    if (total > cap) {
        if (c->ws.base)
            throw Error(IPC_E_CAPACITY, std::to_string(total) + (kind == 0 ? " point-triangle" : " edge-edge") +
                                            " candidates exceed the planned capacity of " + std::to_string(cap));
        cap = (int64_t)(total * 1.5) + 1024;
        outbuf.alloc(cap);
    }
    count = total;
    if (!of[1])
        hipLaunchKernelGGL(k_unstash, dim3(blocks_for(Q)), dim3(BLOCK), 0, st, Q, D.qcount.p, D.qoff.p, D.qstash.p, outbuf.p);
    else   // queries whose candidates did not fit the stash traverse again
        hipLaunchKernelGGL(k_traverse<true>, dim3(blocks_for(Q, TRAV_BLOCK)), dim3(TRAV_BLOCK), 0, st, Q, kind, qedge, D.cv_scene.p,
                           D.tri.p, D.edge.p, D.cv_obj.p, D.obj_kind.p, D.excl.p, c->NEX, xw0, xw1, D.sparam.p, pseg_d, D.mid2.p,
                           D.box.p, D.bvh_left.p, D.bvh_right.p, D.bvh_box.p, D.bvh_nmoving.p, grow, perm, D.qcount.p, D.qoff.p, outbuf.p, ovf.p, D.qstash.p);
}

void broad_phase(ipc_ctx *c, const double *xw0, const double *xw1, double grow)
{
    prof_begin(c, IPC_K_BROAD);
    c->cand_cached = false;
    bvh_query(c, 0, xw0, xw1, grow, c->d.cand_pt, c->cap_cand_pt, c->n_cand_pt, c->h_cand_pt_seg);
    bvh_query(c, 1, xw0, xw1, grow, c->d.cand_ee, c->cap_cand_ee, c->n_cand_ee, c->h_cand_ee_seg);
    prof_end(c, IPC_K_BROAD, 0.0);
}

// ---------------------------------------------------------------------------
// Candidates kept across Newton iterations.  The swept-box candidates are
// built with query boxes grown by CAND_GROW dhat, and every contact vertex
// keeps its swept box [min, max] of the two end positions.  Later sweeps
// may reuse the list while no vertex's swept box leaves its kept box by more
// than half the growth: each primitive box then grows by at most that much,
// so every pair whose exact boxes overlap is still on the list (a
// superset).  CCD skips listed pairs whose exact boxes do not overlap, so the
// step bound is the one of the exact candidates; the pair set is exact for
// any superset.
// ---------------------------------------------------------------------------
constexpr double CAND_GROW = 1.0;

__global__ void k_cand_ref(int CV, const double *__restrict__ xw0, const double *__restrict__ xw1, double *__restrict__ ref)
{
    int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= CV) return;
    for (int k = 0; k < 3; ++k) {
        double a = xw0[3 * (size_t)v + k], b = xw1[3 * (size_t)v + k];
        ref[6 * (size_t)v + k] = fmin(a, b);
        ref[6 * (size_t)v + 3 + k] = fmax(a, b);
    }
}

__global__ void k_cand_check(int CV, const double *__restrict__ xw0, const double *__restrict__ xw1, const double *__restrict__ ref,
                             const int *__restrict__ cv_scene, const double *__restrict__ sparam, double grow, int *__restrict__ flag)
{
    int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= CV) return;
    int s = cv_scene[v];
    double m = 0.5 * grow * sparam[8 * (size_t)s + P_DHAT], ex = 0.0;
    for (int k = 0; k < 3; ++k) {
        double a = xw0[3 * (size_t)v + k], b = xw1[3 * (size_t)v + k];
        ex = fmax(ex, fmax(ref[6 * (size_t)v + k] - fmin(a, b), fmax(a, b) - ref[6 * (size_t)v + 3 + k]));
    }
    if (ex > m) atomicOr(flag + s, 1);
}

void broad_phase_cached(ipc_ctx *c, const double *xw0, const double *xw1)
{
    broad_phase(c, xw0, xw1, CAND_GROW);
    c->d.cand_ref.alloc(6 * (size_t)c->CV + 1);
    if (c->CV)
        hipLaunchKernelGGL(k_cand_ref, dim3(blocks_for(c->CV)), dim3(BLOCK), 0, c->stream, c->CV, xw0, xw1, c->d.cand_ref.p);
    c->cand_cached = true;
}

void cand_check(ipc_ctx *c, const double *xw0, const double *xw1, int *flag)
{
    hipLaunchKernelGGL(k_fill_int, dim3(blocks_for(c->n_scenes)), dim3(BLOCK), 0, c->stream, c->n_scenes, flag, 0);
    if (c->CV)
        hipLaunchKernelGGL(k_cand_check, dim3(blocks_for(c->CV)), dim3(BLOCK), 0, c->stream, c->CV, xw0, xw1, c->d.cand_ref.p,
                           c->d.cv_scene.p, c->d.sparam.p, CAND_GROW, flag);
}

// ---------------------------------------------------------------------------
// narrow phase: keep candidates with d^2 < dhat^2 (ballot compaction)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void pair_vertices(int kind, int2 p, const int4 *tri, const int2 *edge, int *cv)
{
    if (kind == 0) { int4 t = tri[p.y]; cv[0] = p.x; cv[1] = t.x; cv[2] = t.y; cv[3] = t.z; }
    else { int2 a = edge[p.x], b = edge[p.y]; cv[0] = a.x; cv[1] = a.y; cv[2] = b.x; cv[3] = b.y; }
}

template <bool WRITE>
__global__ void k_narrow(int n, int kind, const int2 *__restrict__ cand, const int4 *__restrict__ tri, const int2 *__restrict__ edge,
                         const int *__restrict__ cv_scene, const double *__restrict__ xw, const double *__restrict__ sparam,
                         unsigned long long *__restrict__ mask, int *__restrict__ wcount, const int *__restrict__ woff,
                         int2 *__restrict__ out)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int wave = i / TILE, lane = threadIdx.x & (TILE - 1);
    if (!WRITE) {
        bool act = false;
        if (i < n) {
            int cv[4];
            pair_vertices(kind, cand[i], tri, edge, cv);
            d3 x[4] = {ld3(xw, cv[0]), ld3(xw, cv[1]), ld3(xw, cv[2]), ld3(xw, cv[3])};
            int t;
            double d2 = pair_d2(kind, x, &t);
            double dh = sparam[8 * cv_scene[cv[0]] + 2];
            act = d2 < dh * dh;
        }
        unsigned long long m = __ballot(act);
        if (lane == 0 && wave * TILE < n) { mask[wave] = m; wcount[wave] = __popcll(m); }
    } else {
        if (i >= n) return;
        unsigned long long m = mask[wave];
        if ((m >> lane) & 1ull) {
            int pos = woff[wave] + __popcll(m & ((1ull << lane) - 1ull));
            out[pos] = cand[i];
        }
    }
}

static void compact(ipc_ctx *c, int kind, const double *xw, const DBuf<int2> &cand, int64_t ncand, int cseg_region, int pseg_region,
                    DBuf<int2> &out, int64_t &cap, int64_t &count, std::vector<int> &hseg)
{
    Dev &D = c->d;
    hipStream_t st = c->stream;
    int ns = c->n_scenes;
    hseg.assign(ns + 1, 0);
    count = 0;
    int *sseg = seg_ptr(c, pseg_region);
    if (ncand == 0) {
        hipLaunchKernelGGL(k_fill_int, dim3(blocks_for(ns + 1)), dim3(BLOCK), 0, st, ns + 1, sseg, 0);
        return;
    }
    int nw = (int)((ncand + TILE - 1) / TILE);
    DBuf<unsigned long long> &mask = D.mkey;   // scratch reuse
    mask.alloc(nw);
    D.wcount.alloc(nw + 1); D.woff.alloc(nw + 1);
    hipLaunchKernelGGL(k_narrow<false>, dim3(blocks_for(ncand)), dim3(BLOCK), 0, st, (int)ncand, kind, cand.p, D.tri.p, D.edge.p,
                       D.cv_scene.p, xw, D.sparam.p, mask.p, D.wcount.p, nullptr, nullptr);
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, st, 1, D.wcount.p + nw, 0);
    exclusive_scan(c, D.wcount.p, D.woff.p, nw);
    // candidates are grouped by scene and the order is kept, so each scene's
    // first survivor is the number of survivors before its first candidate
    hipLaunchKernelGGL(k_compact_seg, dim3(blocks_for(ns + 1)), dim3(BLOCK), 0, st, ns, (int)ncand, seg_ptr(c, cseg_region), mask.p,
                       D.woff.p, nw, sseg);
    int total = 0;
    {
        HostReads r(c);
        r.add(&total, D.woff.p + nw, sizeof(int));
        r.add(hseg.data(), sseg, (ns + 1) * sizeof(int));
        r.wait();
    }
    if (total > cap) {
        if (c->ws.base)
            throw Error(IPC_E_CAPACITY, std::to_string(total) + (kind == 0 ? " point-triangle" : " edge-edge") +
                                            " pairs exceed the planned capacity of " + std::to_string(cap));
        cap = (int64_t)(total * 1.5) + 1024;
        out.alloc(cap);
    }
    count = total;
    hipLaunchKernelGGL(k_narrow<true>, dim3(blocks_for(ncand)), dim3(BLOCK), 0, st, (int)ncand, kind, cand.p, D.tri.p, D.edge.p,
                       D.cv_scene.p, xw, D.sparam.p, mask.p, D.wcount.p, D.woff.p, out.p);
}

void narrow_phase(ipc_ctx *c, const double *xw)
{
    compact(c, 0, xw, c->d.cand_pt, c->n_cand_pt, R_CPT, R_PT, c->d.pt, c->cap_pt, c->n_pt, c->h_pt_seg);
    compact(c, 1, xw, c->d.cand_ee, c->n_cand_ee, R_CEE, R_EE, c->d.ee, c->cap_ee, c->n_ee, c->h_ee_seg);
}

// ---------------------------------------------------------------------------
// barrier: energy / gradient / projected Hessian of one pair
// ---------------------------------------------------------------------------
struct Map {   // contact vertex -> DOFs
    int node;  // FEM node or -1
    int body;  // body node0 or -1
    d3 xb;
};
__device__ __forceinline__ Map cv_map(int cv, const int *cv_node, const int *cv_body, const double *cv_x, const int *body_node0)
{
    Map m;
    m.node = cv_node[cv];
    int b = cv_body[cv];
    m.body = b >= 0 ? body_node0[b] : -1;
    m.xb = (b >= 0) ? ld3(cv_x, cv) : mk(0, 0, 0);
    return m;
}
__device__ __forceinline__ d3 gather_cv(const Map &m, const double *v)
{
    if (m.node >= 0) return ld3(v, m.node);
    if (m.body >= 0) {
        d3 p = ld3(v, m.body), a0 = ld3(v, m.body + 1), a1 = ld3(v, m.body + 2), a2 = ld3(v, m.body + 3);
        return {p.x + m.xb.x * a0.x + m.xb.y * a1.x + m.xb.z * a2.x, p.y + m.xb.x * a0.y + m.xb.y * a1.y + m.xb.z * a2.y,
                p.z + m.xb.x * a0.z + m.xb.y * a1.z + m.xb.z * a2.z};
    }
    return {0.0, 0.0, 0.0};
}

// When every dynamic vertex of a pair is a FEM node and each pair of them
// already shares a block of the matrix (same tetrahedral mesh, adjacent - as
// for a surface triangle or edge against static geometry), add the pair's
// world-vertex blocks straight into the block-CSR values and report true; the
// pair then costs nothing in the PCG products.
//
// bsr_slots finds the blocks (slot -1 where a vertex is static); the up to
// 16 look-ups are branchless lower-bound searches over the rows' sorted columns, advanced one halving step at a time all together, so
// that a step issues all of its loads at once: a pair waits for about
// log2(row length) + 1 rounds of loads instead of one round per probe.
__device__ __forceinline__ bool bsr_slots(const Map *m, const int *row_ptr, const int *col, int slot[4][4])
{
    int nd[4], lo[4], len[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (m[k].body >= 0) return false;
        nd[k] = m[k].node;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        lo[k] = 0;
        len[k] = 0;
        if (nd[k] >= 0) {
            lo[k] = row_ptr[nd[k]];
            len[k] = row_ptr[nd[k] + 1] - lo[k];
            if (len[k] <= 0) return false;
        }
    }
    int base[4][4], n[4][4], most = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            bool on = nd[k] >= 0 && nd[l] >= 0;
            base[k][l] = lo[k];
            n[k][l] = on ? len[k] : 0;
            most = max(most, n[k][l]);
        }
    // invariant: the first column >= nd[l] of row k lies in [base, base + n]
    while (most > 1) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int l = 0; l < 4; ++l) {
                int h = n[k][l] >> 1;
                if (h > 0) {
                    if (col[base[k][l] + h] < nd[l]) base[k][l] += h;
                    n[k][l] -= h;
                }
            }
        most -= most >> 1;
    }
    bool all = true;
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            slot[k][l] = -1;
            if (n[k][l] == 0) continue;
            int b = base[k][l], end = lo[k] + len[k];
            int c0 = col[b], c1 = b + 1 < end ? col[b + 1] : -1;
            slot[k][l] = c0 == nd[l] ? b : (c0 < nd[l] && c1 == nd[l] ? b + 1 : -1);
            all = all && slot[k][l] >= 0;
        }
    return all;
}
// The pair's 16 (k, l) entries for the slot-sorted merge: the block's slot
// when every block of the pair is in the pattern (nnzb for a static
// vertex's blocks), else nnzb for all and false (the pair stays pair-local).
__device__ __forceinline__ bool pair_slot_keys(const Map *m, const int *row_ptr, const int *col, int nnzb, int i,
                                               int *__restrict__ key, int *__restrict__ code)
{
    int slot[4][4];
    bool on = bsr_slots(m, row_ptr, col, slot);
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            size_t o = 16 * (size_t)i + 4 * k + l;
            key[o] = on && slot[k][l] >= 0 ? slot[k][l] : nnzb;
            code[o] = (int)o;
        }
    return on;
}

template <int MODE>   // 0 energy, 1 energy + gradient, 2 gradient + projected Hessian
__global__ void __launch_bounds__(256) k_barrier(int npt, int nee, const int2 *__restrict__ pt, const int2 *__restrict__ ee,
    const int4 *__restrict__ tri, const int2 *__restrict__ edge, const double *__restrict__ xw, const int *__restrict__ cv_scene,
    const double *__restrict__ sparam, const double *__restrict__ rest2, const int *__restrict__ cv_node,
    const int *__restrict__ cv_body, const double *__restrict__ cv_x, const int *__restrict__ body_node0, double *__restrict__ pg,
    int *__restrict__ gkey, int *__restrict__ gcode, int ncv, int4 *__restrict__ pair_cv, double *__restrict__ pair_H,
    double *__restrict__ pe, int project, int *__restrict__ inf_flag, const int *__restrict__ row_ptr, const int *__restrict__ col,
    int nnzb, int *__restrict__ bkey, int *__restrict__ bcode, int *__restrict__ pair_flag, const int *__restrict__ active)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npt + nee) return;
    int kind = i < npt ? 0 : 1;
    int2 pr = kind == 0 ? pt[i] : ee[i - npt];
    int cv[4];
    pair_vertices(kind, pr, tri, edge, cv);
    d3 x[4] = {ld3(xw, cv[0]), ld3(xw, cv[1]), ld3(xw, cv[2]), ld3(xw, cv[3])};
    int s = cv_scene[cv[0]];
    double kappa = sparam[8 * s + 1], dh = sparam[8 * s + 2];
    int type;
    double d2 = pair_d2(kind, x, &type);
    if (MODE == 2) pair_cv[i] = make_int4(cv[0], cv[1], cv[2], cv[3]);
    // a pair with no contribution: no gradient entries and no blocks
    auto none = [&]() {
        if (pe) pe[i] = 0.0;
        if (MODE >= 1)
            for (int k = 0; k < 4; ++k) { gkey[4 * (size_t)i + k] = ncv; gcode[4 * (size_t)i + k] = 4 * i + k; }
        if (MODE == 2) {
            pair_flag[i] = 1;
            for (int q = 0; q < 16; ++q) { bkey[16 * (size_t)i + q] = nnzb; bcode[16 * (size_t)i + q] = 16 * i + q; }
        }
    };
    if (!(d2 > 0.0)) {
        atomicOr(inf_flag + s, 1);
        none();
        return;
    }
    if (d2 >= dh * dh || (MODE == 2 && active && !active[s])) {   // beyond dhat, or a scene not being assembled
        none();
        return;
    }
    double d = sqrt(d2);
    double b = barrier(d, dh);
    double m = 1.0, m1 = 0.0, m2 = 0.0, ex = 1.0, cval = 0.0;
    d3 u, v, nn;
    if (kind == 1) {
        u = {x[1].x - x[0].x, x[1].y - x[0].y, x[1].z - x[0].z};
        v = {x[3].x - x[2].x, x[3].y - x[2].y, x[3].z - x[2].z};
        nn = cr(u, v);
        cval = dt(nn, nn);
        ex = 1e-3 * rest2[pr.x] * rest2[pr.y];
        if (cval < ex) {
            double rr = cval / ex;
            m = (2.0 - rr) * rr;
            m1 = 2.0 / ex - 2.0 * cval / (ex * ex);
            m2 = -2.0 / (ex * ex);
        }
    }
    if (pe) pe[i] = kappa * m * b;
    if (MODE == 0) return;
    TypeParam P = type_param(kind, type);
    double beta[4];
    d3 r, D0, D1;
    closest_point(P, x, beta, r, D0, D1);
    double b1 = barrier1(d, dh), b2 = barrier2(d, dh);
    double Bq1 = b1 / (2.0 * d), Bq2 = (b2 - b1 / d) / (4.0 * d2);
    bool moll = kind == 1 && cval < ex;
    d3 cu = {0, 0, 0}, cvv = {0, 0, 0};
    if (moll) {
        d3 t1 = cr(v, nn), t2 = cr(nn, u);
        cu = {2.0 * t1.x, 2.0 * t1.y, 2.0 * t1.z};
        cvv = {2.0 * t2.x, 2.0 * t2.y, 2.0 * t2.z};
    }
    Map mp[4];
    for (int k = 0; k < 4; ++k) mp[k] = cv_map(cv[k], cv_node, cv_body, cv_x, body_node0);
    // gradient in world coordinates
    const double su[4] = {-1.0, 1.0, 0.0, 0.0}, sv[4] = {0.0, 0.0, -1.0, 1.0};
    for (int k = 0; k < 4; ++k) {
        double cq = kappa * m * Bq1 * 2.0 * beta[k];
        d3 gk = {cq * r.x, cq * r.y, cq * r.z};
        if (moll) {
            double cb = kappa * b * m1;
            gk.x += cb * (su[k] * cu.x + sv[k] * cvv.x);
            gk.y += cb * (su[k] * cu.y + sv[k] * cvv.y);
            gk.z += cb * (su[k] * cu.z + sv[k] * cvv.z);
        }
        // summed per contact vertex by the slot-ordered gather (static: none)
        st3(pg, 4 * i + k, gk);
        gkey[4 * (size_t)i + k] = (mp[k].node >= 0 || mp[k].body >= 0) ? cv[k] : ncv;
        gcode[4 * (size_t)i + k] = 4 * i + k;
    }
    if (MODE < 2) return;
    // reduced (translation-free) 9x9 Hessian, index 3*i + c
    double gam[3], al0[3], al1[3], etu[3], etv[3];
    for (int ii = 0; ii < 3; ++ii) {
        gam[ii] = al0[ii] = al1[ii] = 0.0;
        for (int k = 0; k < 4; ++k) {
            double U = helmert(k, ii);
            gam[ii] += U * beta[k]; al0[ii] += U * P.a1[k]; al1[ii] += U * P.a2[k];
        }
        etu[ii] = helmert(1, ii) - helmert(0, ii);
        etv[ii] = helmert(3, ii) - helmert(2, ii);
    }
    double gq[9], F0[9], F1[9], gc[9];
    for (int ii = 0; ii < 3; ++ii)
        for (int cc = 0; cc < 3; ++cc) {
            double rc = comp(r, cc);
            gq[3 * ii + cc] = 2.0 * gam[ii] * rc;
            F0[3 * ii + cc] = 2.0 * al0[ii] * rc + 2.0 * gam[ii] * comp(D0, cc);
            F1[3 * ii + cc] = 2.0 * al1[ii] * rc + 2.0 * gam[ii] * comp(D1, cc);
            gc[3 * ii + cc] = etu[ii] * comp(cu, cc) + etv[ii] * comp(cvv, cc);
        }
    double Fi00 = 0, Fi01 = 0, Fi11 = 0;
    if (P.npar == 1) Fi00 = 1.0 / (2.0 * dt(D0, D0));
    else if (P.npar == 2) {
        double s00 = 2.0 * dt(D0, D0), s01 = 2.0 * dt(D0, D1), s11 = 2.0 * dt(D1, D1);
        double det = s00 * s11 - s01 * s01;
        Fi00 = s11 / det; Fi11 = s00 / det; Fi01 = -s01 / det;
    }
    double H[45];   // every index below is a compile-time constant, so H stays in registers
#pragma unroll
    for (int R = 0; R < 9; ++R)
#pragma unroll
        for (int C = R; C < 9; ++C) {
            int iR = R / 3, cR = R % 3, iC = C / 3, cC = C % 3;
            double hq = (cR == cC ? 2.0 * gam[iR] * gam[iC] : 0.0)
                      - (F0[R] * Fi00 * F0[C] + F0[R] * Fi01 * F1[C] + F1[R] * Fi01 * F0[C] + F1[R] * Fi11 * F1[C]);
            double hv = kappa * m * (Bq2 * gq[R] * gq[C] + Bq1 * hq);
            if (moll) {
                // Hessian of c = |u x v|^2 in (u, v): Huu = 2[v]x^T[v]x, Hvv = 2[u]x^T[u]x, Huv = 2[v]x[u]x - 2[n]x
                double huu = 0, hvv = 0, huv = 0, hvu = 0;
                for (int k = 0; k < 3; ++k) {
                    huu += skew(v, k, cR) * skew(v, k, cC);
                    hvv += skew(u, k, cR) * skew(u, k, cC);
                    huv += skew(v, cR, k) * skew(u, k, cC);
                    hvu += skew(v, cC, k) * skew(u, k, cR);
                }
                huu *= 2.0; hvv *= 2.0;
                huv = 2.0 * huv - 2.0 * skew(nn, cR, cC);
                hvu = 2.0 * hvu - 2.0 * skew(nn, cC, cR);   // (Huv)^T entry (cR, cC)
                double hc = etu[iR] * etu[iC] * huu + etv[iR] * etv[iC] * hvv + etu[iR] * etv[iC] * huv + etv[iR] * etu[iC] * hvu;
                hv += kappa * (b * (m2 * gc[R] * gc[C] + m1 * hc) + m1 * Bq1 * (gc[R] * gq[C] + gq[R] * gc[C]));
            }
            H[pk9(R, C)] = hv;
        }
    if (project) psd_project9(H);
    // The reduced Hessian of every pair is kept.  A pair whose blocks are all
    // in the matrix pattern is added into the matrix values by the
    // slot-sorted gather (flag 1); the others stay pair-local blocks of the
    // product (flag 0).
    double *out = pair_H + 45 * (size_t)i;
#pragma unroll
    for (int q = 0; q < 45; ++q) out[q] = H[q];
    pair_flag[i] = pair_slot_keys(mp, row_ptr, col, nnzb, i, bkey, bcode) ? 1 : 0;
}

// ---- run-sum values (ipc_runsum.h) ------------------------------------------
// world-vertex block (k, l) of a barrier pair from its reduced Hessian
struct ValBarrierBlock {
    const double *pH;
    __device__ void operator()(int code, double *B) const
    {
        const int i = code >> 4, k = (code >> 2) & 3, l = code & 3;
        const double *H = pH + 45 * (size_t)i;
        double uk[3], ul[3];
#pragma unroll
        for (int ii = 0; ii < 3; ++ii) { uk[ii] = helmert(k, ii); ul[ii] = helmert(l, ii); }
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                double acc = 0.0;
#pragma unroll
                for (int ii = 0; ii < 3; ++ii)
#pragma unroll
                    for (int jj = 0; jj < 3; ++jj) acc += uk[ii] * ul[jj] * H[pk9(3 * ii + a, 3 * jj + b)];
                B[3 * a + b] = acc;
            }
    }
};
// friction block (k, l) of a lag pair: beta_k beta_l M
struct ValLagBlock {
    const double *lbeta, *lM;
    __device__ void operator()(int code, double *B) const
    {
        const int i = code >> 4, k = (code >> 2) & 3, l = code & 3;
        const double w = lbeta[4 * (size_t)i + k] * lbeta[4 * (size_t)i + l];
        const double *M = lM + 6 * (size_t)i;
        B[0] = w * M[0]; B[1] = w * M[1]; B[2] = w * M[2];
        B[3] = w * M[1]; B[4] = w * M[3]; B[5] = w * M[4];
        B[6] = w * M[2]; B[7] = w * M[4]; B[8] = w * M[5];
    }
};

// stable sort of m (key, code) int pairs by the low end_bit bits of the key
// Stable sort of (key, code) entries by key, for the run sums.  rocPRIM's
// radix sort picks a block sort with merge passes below a million entries
// (about 20 launches for the barrier's entries); a merge limit of 0 makes it
// use the onesweep radix passes at every size, a handful of launches.  A
// stable sort has one result, so the choice does not change any sum.
using EntrySortConfig = rocprim::radix_sort_config<rocprim::default_config, rocprim::default_config, rocprim::default_config, 0>;

size_t sort_entries_bytes(ipc_ctx *c, int64_t m, int end_bit)
{
    size_t bytes = 0;
    IPC_HIP(rocprim::radix_sort_pairs<EntrySortConfig>(nullptr, bytes, (const int *)nullptr, (int *)nullptr, (const int *)nullptr,
                                                       (int *)nullptr, (unsigned int)std::max<int64_t>(m, 1), 0u,
                                                       (unsigned int)end_bit, c->stream));
    return bytes;
}

void sort_entries(ipc_ctx *c, const int *key, int *key2, const int *code, int *code2, int64_t m, int end_bit)
{
    if (m <= 0) return;
    size_t bytes = sort_entries_bytes(c, m, end_bit);
    c->d.sort_tmp.alloc(bytes + 16);
    IPC_HIP(rocprim::radix_sort_pairs<EntrySortConfig>(c->d.sort_tmp.p, bytes, key, key2, code, code2, (unsigned int)m, 0u,
                                                       (unsigned int)end_bit, c->stream));
}

int bits_for(int64_t n)   // bits that hold every value in [0, n]
{
    int b = 1;
    while (b < 31 && (1ll << b) <= n) ++b;
    return b;
}

// Barrier pairs.  Gradients (mode >= 1) are summed per contact vertex into
// D.gcv; projected or plain blocks (mode 2) whose slots exist are summed per
// matrix slot into the values, both through sorted run sums.
void launch_barrier(ipc_ctx *c, int mode, bool candidates, const double *xw, bool project)
{
    Dev &D = c->d;
    int64_t npt = candidates ? c->n_cand_pt : c->n_pt, nee = candidates ? c->n_cand_ee : c->n_ee;
    const int2 *pt = candidates ? D.cand_pt.p : D.pt.p, *ee = candidates ? D.cand_ee.p : D.ee.p;
    int64_t n = npt + nee;
    D.pair_part.alloc(n + 1);
    if (mode >= 1) {
        D.pair_g.alloc(12 * (size_t)n + 3);
        for (auto *b : {&D.pg_key, &D.pg_code, &D.pg_key2, &D.pg_code2}) b->alloc(4 * (size_t)n + 1);
    }
    if (mode == 2) {
        D.pair_cv.alloc(n + 1); D.pair_H.alloc(45 * (size_t)(n + 1)); D.pair_flag.alloc(n + 1);
        for (auto *b : {&D.pb_key, &D.pb_code, &D.pb_key2, &D.pb_code2}) b->alloc(16 * (size_t)n + 1);
    }
    if (n == 0) return;
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(blocks_for(n)), dim3(BLOCK), 0, c->stream, (int)npt, (int)nee, pt, ee, D.tri.p, D.edge.p, xw,
                           D.cv_scene.p, D.sparam.p, D.edge_rest2.p, D.cv_node.p, D.cv_body.p, D.cv_x.p, D.body_node0.p, D.pair_g.p,
                           D.pg_key.p, D.pg_code.p, c->CV, D.pair_cv.p, D.pair_H.p, D.pair_part.p, (int)project, D.inf_flag.p,
                           D.row_ptr.p, D.col.p, c->nnzb, D.pb_key.p, D.pb_code.p, D.pair_flag.p, mode == 2 ? c->assemble_only : nullptr);
    };
    if (mode == 2) prof_begin(c, IPC_K_BARRIER_HESS);
    if (mode == 0) go(k_barrier<0>);
    else if (mode == 1) go(k_barrier<1>);
    else go(k_barrier<2>);
    if (mode >= 1) {
        sort_entries(c, D.pg_key.p, D.pg_key2.p, D.pg_code.p, D.pg_code2.p, 4 * n, bits_for(c->CV));
        runsum<3>(c, 4 * n, c->CV, D.pg_key2.p, D.pg_code2.p, ValVec3{D.pair_g.p}, EmitAdd3{D.gcv.p});
    }
    if (mode == 2) {
        sort_entries(c, D.pb_key.p, D.pb_key2.p, D.pb_code.p, D.pb_code2.p, 16 * n, bits_for(c->nnzb));
        runsum<9>(c, 16 * n, c->nnzb, D.pb_key2.p, D.pb_code2.p, ValBarrierBlock{D.pair_H.p}, EmitAdd9{D.val.p});
    }
    if (mode == 2) prof_end(c, IPC_K_BARRIER_HESS, 0.0);
}

// The contact-vertex sums into DOF gradients: a FEM contact vertex is its
// node's only contact vertex; a body's contact vertices are summed over the
// body in their listed order (one wavefront per body, fixed-order shuffle
// reduction) into its 4 nodes with weights (1, xb).
__global__ void k_cv_fem(int CV, const int *__restrict__ cv_node, const double *__restrict__ gcv, double *__restrict__ g)
{
    int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= CV) return;
    int n = cv_node[v];
    if (n < 0) return;
    d3 a = ld3(gcv, v), b = ld3(g, n);
    st3(g, n, {b.x + a.x, b.y + a.y, b.z + a.z});
}

__global__ void __launch_bounds__(64) k_cv_bodies(const int *__restrict__ ptr, const int *__restrict__ list,
                                                  const double *__restrict__ cv_x, const int *__restrict__ body_node0,
                                                  const double *__restrict__ gcv, double *__restrict__ g)
{
    const int b = blockIdx.x, lane = threadIdx.x;
    double a[12];
#pragma unroll
    for (int q = 0; q < 12; ++q) a[q] = 0.0;
    for (int e = ptr[b] + lane; e < ptr[b + 1]; e += 64) {
        int v = list[e];
        d3 f = ld3(gcv, v), xb = ld3(cv_x, v);
        a[0] += f.x; a[1] += f.y; a[2] += f.z;
        a[3] += xb.x * f.x; a[4] += xb.x * f.y; a[5] += xb.x * f.z;
        a[6] += xb.y * f.x; a[7] += xb.y * f.y; a[8] += xb.y * f.z;
        a[9] += xb.z * f.x; a[10] += xb.z * f.y; a[11] += xb.z * f.z;
    }
#pragma unroll
    for (int q = 0; q < 12; ++q) a[q] = wave_sum(a[q]);
    if (lane != 0) return;
    double *o = g + 3 * (size_t)body_node0[b];
#pragma unroll
    for (int q = 0; q < 12; ++q) o[q] += a[q];
}

void contact_grad_begin(ipc_ctx *c)
{
    c->d.gcv.alloc(3 * (size_t)c->CV + 3);
    c->d.gcv.zero(c->stream, 3 * (size_t)c->CV + 3);
}

void contact_grad_end(ipc_ctx *c, double *g)
{
    Dev &D = c->d;
    if (c->CV == 0) return;
    hipLaunchKernelGGL(k_cv_fem, dim3(blocks_for(c->CV)), dim3(BLOCK), 0, c->stream, c->CV, D.cv_node.p, D.gcv.p, g);
    if (c->NB) hipLaunchKernelGGL(k_cv_bodies, dim3(c->NB), dim3(64), 0, c->stream, D.body_cv_ptr.p, D.body_cv.p, D.cv_x.p,
                                  D.body_node0.p, D.gcv.p, g);
}

// ---------------------------------------------------------------------------
// friction, lagged at the step start (closest-point weights beta, normal n,
// normal force lambda = -kappa m b'(d)); a later lag pass takes them at the
// current solution but keeps measuring slip from the step start: lrn is the
// weighted closest-point sum at the reference positions xref
// ---------------------------------------------------------------------------
__global__ void k_lag(int npt, int nee, const int2 *__restrict__ pt, const int2 *__restrict__ ee, const int4 *__restrict__ tri,
                      const int2 *__restrict__ edge, const double *__restrict__ xw, const int *__restrict__ cv_scene,
                      const double *__restrict__ sparam, const double *__restrict__ rest2, int4 *__restrict__ lcv,
                      double *__restrict__ lbeta, double *__restrict__ lnrm, double *__restrict__ llam, double *__restrict__ lrn,
                      int *__restrict__ ltype, double *__restrict__ lex, const double *__restrict__ xref)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npt + nee) return;
    int kind = i < npt ? 0 : 1;
    int2 pr = kind == 0 ? pt[i] : ee[i - npt];
    int cv[4];
    pair_vertices(kind, pr, tri, edge, cv);
    d3 x[4] = {ld3(xw, cv[0]), ld3(xw, cv[1]), ld3(xw, cv[2]), ld3(xw, cv[3])};
    int s = cv_scene[cv[0]];
    double kappa = sparam[8 * s + 1], dh = sparam[8 * s + 2];
    int type;
    double d2 = pair_d2(kind, x, &type);
    double d = sqrt(d2);
    TypeParam P = type_param(kind, type);
    double beta[4];
    d3 r, D0, D1;
    closest_point(P, x, beta, r, D0, D1);
    double rn = sqrt(dt(r, r));
    double m = 1.0, ex = 0.0;
    if (kind == 1) {
        d3 u = {x[1].x - x[0].x, x[1].y - x[0].y, x[1].z - x[0].z}, v = {x[3].x - x[2].x, x[3].y - x[2].y, x[3].z - x[2].z};
        d3 nn = cr(u, v);
        double cval = dt(nn, nn);
        ex = 1e-3 * rest2[pr.x] * rest2[pr.y];
        if (cval < ex) m = (2.0 - cval / ex) * (cval / ex);
    }
    ltype[i] = type;
    lex[i] = ex;
    lcv[i] = make_int4(cv[0], cv[1], cv[2], cv[3]);
    for (int k = 0; k < 4; ++k) lbeta[4 * (size_t)i + k] = beta[k];
    lnrm[3 * (size_t)i] = r.x / rn; lnrm[3 * (size_t)i + 1] = r.y / rn; lnrm[3 * (size_t)i + 2] = r.z / rn;
    if (xref) {   // the same weights on the reference positions
        r = {0.0, 0.0, 0.0};
        for (int k = 0; k < 4; ++k) {
            d3 p = ld3(xref, cv[k]);
            r.x += beta[k] * p.x; r.y += beta[k] * p.y; r.z += beta[k] * p.z;
        }
    }
    lrn[3 * (size_t)i] = r.x; lrn[3 * (size_t)i + 1] = r.y; lrn[3 * (size_t)i + 2] = r.z;
    llam[i] = -kappa * m * barrier1(d, dh);
}

// Per lag: the matrix block of every (k, l) of a lag pair whose blocks are
// all in the pattern (key nnzb: none), for the slot-sorted gather below.
// Also the pair's 4 gradient entries keyed by contact vertex (CV: static).
__global__ void k_lag_slots(int n, int nnzb, int ncv, const int4 *__restrict__ lcv, const int *__restrict__ cv_node,
                            const int *__restrict__ cv_body, const double *__restrict__ cv_x, const int *__restrict__ body_node0,
                            const int *__restrict__ row_ptr, const int *__restrict__ col, int *__restrict__ lmerge,
                            int *__restrict__ key, int *__restrict__ code, int *__restrict__ gkey, int *__restrict__ gcode)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int4 c4 = lcv[i];
    int cv[4] = {c4.x, c4.y, c4.z, c4.w};
    Map mp[4];
    for (int k = 0; k < 4; ++k) mp[k] = cv_map(cv[k], cv_node, cv_body, cv_x, body_node0);
    lmerge[i] = pair_slot_keys(mp, row_ptr, col, nnzb, i, key, code) ? 1 : 0;
    for (int k = 0; k < 4; ++k) {
        gkey[4 * (size_t)i + k] = (mp[k].node >= 0 || mp[k].body >= 0) ? cv[k] : ncv;
        gcode[4 * (size_t)i + k] = 4 * i + k;
    }
}

void launch_lag(ipc_ctx *c, const double *xw, const double *xref)
{
    Dev &D = c->d;
    launch_hs_lag(c, xw, xref);
    int64_t n = c->n_pt + c->n_ee;
    if (n > c->cap_lag) {
        if (c->ws.base)
            throw Error(IPC_E_CAPACITY, std::to_string(n) + " friction pairs exceed the planned capacity of " + std::to_string(c->cap_lag));
        c->cap_lag = (int64_t)(n * 1.5) + 1024;
        D.lag_cv.alloc(c->cap_lag); D.lag_beta.alloc(4 * c->cap_lag); D.lag_nrm.alloc(3 * c->cap_lag);
        D.lag_lam.alloc(c->cap_lag); D.lag_rn.alloc(3 * c->cap_lag); D.lag_M.alloc(6 * c->cap_lag);
        D.lag_flag.alloc(c->cap_lag); D.lag_type.alloc(c->cap_lag); D.lag_ex.alloc(c->cap_lag);
        D.lag_merge.alloc(c->cap_lag);
        D.lag_key.alloc(16 * c->cap_lag); D.lag_code.alloc(16 * c->cap_lag);
        D.lag_key2.alloc(16 * c->cap_lag); D.lag_code2.alloc(16 * c->cap_lag);
        D.lag_g.alloc(12 * c->cap_lag);
        for (auto *b : {&D.lg_key, &D.lg_code, &D.lg_key2, &D.lg_code2}) b->alloc(4 * c->cap_lag);
    }
    c->n_lag = n;
    c->h_lag_seg.assign(c->n_scenes + 1, 0);
    for (int s = 0; s <= c->n_scenes; ++s) c->h_lag_seg[s] = c->h_pt_seg[s] + c->h_ee_seg[s];
    if (n == 0) return;
    hipLaunchKernelGGL(k_lag, dim3(blocks_for(n)), dim3(BLOCK), 0, c->stream, (int)c->n_pt, (int)c->n_ee, D.pt.p, D.ee.p, D.tri.p,
                       D.edge.p, xw, D.cv_scene.p, D.sparam.p, D.edge_rest2.p, D.lag_cv.p, D.lag_beta.p, D.lag_nrm.p, D.lag_lam.p,
                       D.lag_rn.p, D.lag_type.p, D.lag_ex.p, xref);
    // slot lists of the merged friction blocks and the gradient entries by
    // contact vertex, sorted once per lag
    hipLaunchKernelGGL(k_lag_slots, dim3(blocks_for(n)), dim3(BLOCK), 0, c->stream, (int)n, c->nnzb, c->CV, D.lag_cv.p, D.cv_node.p,
                       D.cv_body.p, D.cv_x.p, D.body_node0.p, D.row_ptr.p, D.col.p, D.lag_merge.p, D.lag_key.p, D.lag_code.p,
                       D.lg_key.p, D.lg_code.p);
    sort_entries(c, D.lag_key.p, D.lag_key2.p, D.lag_code.p, D.lag_code2.p, 16 * n, bits_for(c->nnzb));
    sort_entries(c, D.lg_key.p, D.lg_key2.p, D.lg_code.p, D.lg_code2.p, 4 * n, bits_for(c->CV));
}

template <int MODE>
__global__ void k_friction(int n, const int4 *__restrict__ lcv, const double *__restrict__ lbeta, const double *__restrict__ lnrm,
                           const double *__restrict__ llam, const double *__restrict__ lrn, const double *__restrict__ xw,
                           const int *__restrict__ cv_scene, const double *__restrict__ sparam, const int *__restrict__ cv_node,
                           const int *__restrict__ cv_body, const double *__restrict__ cv_x, const int *__restrict__ body_node0,
                           double *__restrict__ lg, double *__restrict__ lM,
                           double *__restrict__ pe, const int *__restrict__ lmerge, int *__restrict__ lflag)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int4 c4 = lcv[i];
    int cv[4] = {c4.x, c4.y, c4.z, c4.w};
    int s = cv_scene[cv[0]];
    double mu = sparam[8 * s + 3], ea = sparam[8 * s + 4];
    double beta[4];
    for (int k = 0; k < 4; ++k) beta[k] = lbeta[4 * (size_t)i + k];
    d3 sx = {0, 0, 0};
    for (int k = 0; k < 4; ++k) {
        d3 p = ld3(xw, cv[k]);
        sx.x += beta[k] * p.x; sx.y += beta[k] * p.y; sx.z += beta[k] * p.z;
    }
    d3 rn = ld3(lrn, i), nr = ld3(lnrm, i);
    d3 dv = {sx.x - rn.x, sx.y - rn.y, sx.z - rn.z};
    double nd = dt(nr, dv);
    d3 u = {dv.x - nr.x * nd, dv.y - nr.y * nd, dv.z - nr.z * nd};
    double sn = sqrt(dt(u, u));
    double f0 = sn < ea ? -sn * sn * sn / (3.0 * ea * ea) + sn * sn / ea + ea / 3.0 : sn;
    double w = mu * llam[i];
    if (pe) pe[i] = w * f0;
    if (MODE == 0) return;
    double f1s = sn < ea ? 2.0 / ea - sn / (ea * ea) : 1.0 / sn;
    // per-vertex gradients, summed per contact vertex by the sorted run sums
    for (int k = 0; k < 4; ++k) {
        double cc = w * f1s * beta[k];
        st3(lg, 4 * i + k, {cc * u.x, cc * u.y, cc * u.z});
    }
    if (MODE < 2) return;
    double cu = sn < ea ? (sn > 0.0 ? -1.0 / (sn * ea * ea) : 0.0) : -1.0 / (sn * sn * sn);
    double M[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            M[3 * a + b] = w * (cu * comp(u, a) * comp(u, b) + f1s * ((a == b ? 1.0 : 0.0) - comp(nr, a) * comp(nr, b)));
    // a pair whose blocks are all in the pattern is added into the matrix
    // values by k_fric_gather; the others stay pair-local in the products
    lflag[i] = lmerge[i];
    double *o = lM + 6 * (size_t)i;
    o[0] = M[0]; o[1] = M[1]; o[2] = M[2]; o[3] = M[4]; o[4] = M[5]; o[5] = M[8];
}

// Lagged friction.  Gradients (mode >= 1) are summed per contact vertex into
// D.gcv; the blocks of the merged lag pairs (mode 2) per matrix slot into the
// values, both through the lists sorted once per lag.
void launch_friction(ipc_ctx *c, int mode, const double *xw)
{
    Dev &D = c->d;
    int64_t n = c->n_lag;
    D.pair_part.alloc(std::max<int64_t>(n, c->n_pt + c->n_ee) + 1);
    if (n == 0) return;
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(blocks_for(n)), dim3(BLOCK), 0, c->stream, (int)n, D.lag_cv.p, D.lag_beta.p, D.lag_nrm.p,
                           D.lag_lam.p, D.lag_rn.p, xw, D.cv_scene.p, D.sparam.p, D.cv_node.p, D.cv_body.p, D.cv_x.p, D.body_node0.p,
                           D.lag_g.p, D.lag_M.p, D.fr_part.p, D.lag_merge.p, D.lag_flag.p);
    };
    D.fr_part.alloc(n + 1);
    if (mode == 0) go(k_friction<0>);
    else if (mode == 1) go(k_friction<1>);
    else go(k_friction<2>);
    if (mode >= 1) runsum<3>(c, 4 * n, c->CV, D.lg_key2.p, D.lg_code2.p, ValVec3{D.lag_g.p}, EmitAdd3{D.gcv.p});
    if (mode == 2) runsum<9>(c, 16 * n, c->nnzb, D.lag_key2.p, D.lag_code2.p, ValLagBlock{D.lag_beta.p, D.lag_M.p}, EmitAdd9{D.val.p});
}

// ---------------------------------------------------------------------------
// adjoint of the friction lag.  For the adjoint vector w, a lagged pair adds
// phi = mu lam (f1(s)/s) (W . u) to w^T G, with W = sum_k beta_k w_k and u the
// tangential relative displacement.  phi depends on the lag positions x^n of
// its four vertices through beta (the closest-point parameters s* minimise
// |r(s)|^2, so ds* = -F_ss^-1 F_sx dx^n), the offset r, the normal n = r/|r|,
// the normal force lam = -kappa m(c) b'(|r|) and the -x^n inside u.  One
// thread per pair: ybar -= d phi / d y^n (through the contact-vertex maps) and
// part[i] = lam (f1/s) (W . u), the pair's w . dG/dmu.
// ---------------------------------------------------------------------------
__global__ void k_lag_vjp(int n, int npt, const int4 *__restrict__ lcv, const int *__restrict__ ltype, const double *__restrict__ lex,
                          const double *__restrict__ xw, const double *__restrict__ xwn, const int *__restrict__ cv_scene,
                          const double *__restrict__ sparam, const int *__restrict__ cv_node, const int *__restrict__ cv_body,
                          const double *__restrict__ cv_x, const int *__restrict__ body_node0, const double *__restrict__ w,
                          double *__restrict__ lg, double *__restrict__ part)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int kind = i < npt ? 0 : 1;
    int4 c4 = lcv[i];
    int cv[4] = {c4.x, c4.y, c4.z, c4.w};
    int s = cv_scene[cv[0]];
    const double *sp = sparam + 8 * (size_t)s;
    double kappa = sp[P_KAPPA], dh = sp[P_DHAT], mu = sp[P_MU], ea = sp[P_EPSH];
    Map mp[4];
    d3 x[4], xn[4], wv[4];
    for (int k = 0; k < 4; ++k) {
        mp[k] = cv_map(cv[k], cv_node, cv_body, cv_x, body_node0);
        x[k] = ld3(xw, cv[k]);
        xn[k] = ld3(xwn, cv[k]);
        wv[k] = gather_cv(mp[k], w);
    }
    TypeParam P = type_param(kind, ltype[i]);
    double beta[4];
    d3 r, D0, D1;
    closest_point(P, xn, beta, r, D0, D1);
    double d = sqrt(dt(r, r));
    d3 nr = {r.x / d, r.y / d, r.z / d};
    // normal force with the edge-edge mollifier m(c), c = |u x v|^2 at x^n
    double m = 1.0, m1 = 0.0;
    d3 gu = {0, 0, 0}, gv = {0, 0, 0};
    if (kind == 1) {
        d3 ue = {xn[1].x - xn[0].x, xn[1].y - xn[0].y, xn[1].z - xn[0].z}, ve = {xn[3].x - xn[2].x, xn[3].y - xn[2].y, xn[3].z - xn[2].z};
        d3 nn = cr(ue, ve);
        double cval = dt(nn, nn), ex = lex[i];
        if (cval < ex) {
            m = (2.0 - cval / ex) * (cval / ex);
            m1 = 2.0 / ex - 2.0 * cval / (ex * ex);
            gu = cr(ve, nn); gu = {2.0 * gu.x, 2.0 * gu.y, 2.0 * gu.z};   // dc/du
            gv = cr(nn, ue); gv = {2.0 * gv.x, 2.0 * gv.y, 2.0 * gv.z};   // dc/dv
        }
    }
    double b1 = barrier1(d, dh), b2 = barrier2(d, dh);
    double lam = -kappa * m * b1;
    d3 Dv = {0, 0, 0}, W = {0, 0, 0}, dx[4];
    for (int k = 0; k < 4; ++k) {
        dx[k] = {x[k].x - xn[k].x, x[k].y - xn[k].y, x[k].z - xn[k].z};
        Dv.x += beta[k] * dx[k].x; Dv.y += beta[k] * dx[k].y; Dv.z += beta[k] * dx[k].z;
        W.x += beta[k] * wv[k].x; W.y += beta[k] * wv[k].y; W.z += beta[k] * wv[k].z;
    }
    double nD = dt(nr, Dv);
    d3 u = {Dv.x - nr.x * nD, Dv.y - nr.y * nD, Dv.z - nr.z * nD};
    double sg = sqrt(dt(u, u));
    double f1s = sg < ea ? 2.0 / ea - sg / (ea * ea) : 1.0 / sg;
    double df1s = sg < ea ? -1.0 / (ea * ea) : -1.0 / (sg * sg);
    double Wu = dt(W, u), psi = f1s * Wu;
    double cq = sg > 0.0 ? Wu * df1s / sg : 0.0;
    d3 gpsi = {f1s * W.x + cq * u.x, f1s * W.y + cq * u.y, f1s * W.z + cq * u.z};   // d psi / d u
    part[i] = lam * psi;
    double wu[4];
    for (int k = 0; k < 4; ++k) wu[k] = dt(wv[k], u);
    // inverse of F_ss = 2 [D_a . D_b]
    double i00 = 0.0, i01 = 0.0, i11 = 0.0;
    if (P.npar == 1) i00 = 1.0 / (2.0 * dt(D0, D0));
    else if (P.npar == 2) {
        double a00 = 2.0 * dt(D0, D0), a01 = 2.0 * dt(D0, D1), a11 = 2.0 * dt(D1, D1), det = a00 * a11 - a01 * a01;
        i00 = a11 / det; i01 = -a01 / det; i11 = a00 / det;
    }
    const double su[4] = {-1.0, 1.0, 0.0, 0.0}, sv[4] = {0.0, 0.0, -1.0, 1.0};
    for (int j = 0; j < 4; ++j) {
        if (mp[j].node < 0 && mp[j].body < 0) continue;
        double res[3];
        for (int c = 0; c < 3; ++c) {
            double rc = comp(r, c);
            double F0 = 2.0 * P.a1[j] * rc + 2.0 * beta[j] * comp(D0, c);
            double F1 = 2.0 * P.a2[j] * rc + 2.0 * beta[j] * comp(D1, c);
            double ds0 = -(i00 * F0 + i01 * F1), ds1 = -(i01 * F0 + i11 * F1);
            double db[4];
            for (int k = 0; k < 4; ++k) db[k] = P.a1[k] * ds0 + P.a2[k] * ds1;
            d3 dr = {D0.x * ds0 + D1.x * ds1, D0.y * ds0 + D1.y * ds1, D0.z * ds0 + D1.z * ds1};
            d3 dD = {0, 0, 0};
            for (int k = 0; k < 4; ++k) { dD.x += db[k] * dx[k].x; dD.y += db[k] * dx[k].y; dD.z += db[k] * dx[k].z; }
            if (c == 0) { dr.x += beta[j]; dD.x -= beta[j]; }
            else if (c == 1) { dr.y += beta[j]; dD.y -= beta[j]; }
            else { dr.z += beta[j]; dD.z -= beta[j]; }
            double dd = dt(nr, dr);
            d3 dn = {(dr.x - nr.x * dd) / d, (dr.y - nr.y * dd) / d, (dr.z - nr.z * dd) / d};
            double dnD = dt(dn, Dv) + dt(nr, dD);
            d3 du = {dD.x - dn.x * nD - nr.x * dnD, dD.y - dn.y * nD - nr.y * dnD, dD.z - dn.z * nD - nr.z * dnD};
            double dWu = 0.0;
            for (int k = 0; k < 4; ++k) dWu += db[k] * wu[k];
            double dc = su[j] * comp(gu, c) + sv[j] * comp(gv, c);
            double dlam = -kappa * (m1 * dc * b1 + m * b2 * dd);
            double dpsi = dt(gpsi, du) + f1s * dWu;
            res[c] = -mu * (dlam * psi + lam * dpsi);
        }
        st3(lg, 4 * i + j, {res[0], res[1], res[2]});
    }
}

void launch_lag_vjp(ipc_ctx *c, const double *xw, const double *xwn, const double *w, double *ybar)
{
    Dev &D = c->d;
    int64_t n = c->n_lag;
    D.fr_part.alloc(n + 1);
    if (n == 0 && !c->M_HS) return;
    // per-vertex values summed per contact vertex (the pairs' through run
    // sums, then the half-space entries'), then into ybar
    contact_grad_begin(c);
    if (n) {
        hipLaunchKernelGGL(k_lag_vjp, dim3(blocks_for(n)), dim3(BLOCK), 0, c->stream, (int)n, (int)c->n_lag_pt, D.lag_cv.p, D.lag_type.p,
                           D.lag_ex.p, xw, xwn, D.cv_scene.p, D.sparam.p, D.cv_node.p, D.cv_body.p, D.cv_x.p, D.body_node0.p, w,
                           D.lag_g.p, D.fr_part.p);
        runsum<3>(c, 4 * n, c->CV, D.lg_key2.p, D.lg_code2.p, ValVec3{D.lag_g.p}, EmitAdd3{D.gcv.p});
    }
    launch_hs_lag_vjp(c, xw, xwn, w);
    contact_grad_end(c, ybar);
}

// ---------------------------------------------------------------------------
// Pair-local contact blocks as extra rows of the product.  A barrier or
// friction pair whose blocks did not fit the matrix pattern couples the DOF
// nodes of its vertices: a FEM vertex is one node, and the vertices of one
// affine body share that body's 4 nodes with weights (1, xb).  The pair's
// vertices are grouped by owner, and the pair emits one 3x3 block per
// (node, node) of its groups, B = sum_{k in g, l in h} w_k w_l H_kl with H_kl
// the world-vertex blocks.  Blocks are written per pair in a fixed order,
// stably radix-sorted by row and gathered, so the product reads them per row
// without atomics and in a run-to-run fixed order.
// ---------------------------------------------------------------------------
struct PairNodes {
    int ng;          // owner groups (distinct FEM nodes / bodies)
    int first[4];    // first DOF node of each group
    int nn[4];       // nodes per group (1 FEM, 4 body)
    int g[4];        // group of each vertex (-1: static)
    int total;       // sum of nn
};

__device__ __forceinline__ PairNodes pair_nodes(const Map *mp)
{
    PairNodes P;
    P.ng = 0; P.total = 0;
    for (int k = 0; k < 4; ++k) {
        P.g[k] = -1;
        int f = mp[k].node >= 0 ? mp[k].node : mp[k].body;
        if (f < 0) continue;
        int gi = -1;
        for (int q = 0; q < P.ng; ++q) if (P.first[q] == f) gi = q;
        if (gi < 0) {
            gi = P.ng++;
            P.first[gi] = f;
            P.nn[gi] = mp[k].node >= 0 ? 1 : 4;
            P.total += P.nn[gi];
        }
        P.g[k] = gi;
    }
    return P;
}

__device__ __forceinline__ double map_weight(const Map &m, int q)
{
    if (m.node >= 0) return 1.0;
    return q == 0 ? 1.0 : (q == 1 ? m.xb.x : (q == 2 ? m.xb.y : m.xb.z));
}

// world-vertex block (k, l) of pair entry i: barrier pairs (i < nb) from the
// reduced 9x9 Hessian through the Helmert basis, friction pairs from beta and M
__device__ __forceinline__ void pair_block(int i, int nb, const double *pH, const double *lbeta, const double *lM, int k, int l,
                                           double *B)
{
    if (i < nb) {
        const double *H = pH + 45 * (size_t)i;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double acc = 0.0;
                for (int ii = 0; ii < 3; ++ii)
                    for (int jj = 0; jj < 3; ++jj) acc += helmert(k, ii) * helmert(l, jj) * H[pk9(3 * ii + a, 3 * jj + b)];
                B[3 * a + b] = acc;
            }
    } else {
        int j = i - nb;
        const double *M = lM + 6 * (size_t)j;
        double bb = lbeta[4 * (size_t)j + k] * lbeta[4 * (size_t)j + l];
        double Mf[9] = {M[0], M[1], M[2], M[1], M[3], M[4], M[2], M[4], M[5]};
        for (int q = 0; q < 9; ++q) B[q] = bb * Mf[q];
    }
}

__device__ __forceinline__ void pair_maps(int i, int nb, const int4 *pcv, const int4 *lcv, const int *cv_node, const int *cv_body,
                                          const double *cv_x, const int *body_node0, Map *mp)
{
    int4 c4 = i < nb ? pcv[i] : lcv[i - nb];
    int cv[4] = {c4.x, c4.y, c4.z, c4.w};
    for (int k = 0; k < 4; ++k) mp[k] = cv_map(cv[k], cv_node, cv_body, cv_x, body_node0);
}

// blocks per pair entry (0 when merged into the matrix)
__global__ void k_dyn_count(int nb, int nf, const int *__restrict__ pflag, const int *__restrict__ lflag, const int4 *__restrict__ pcv,
                            const int4 *__restrict__ lcv, const int *__restrict__ cv_node, const int *__restrict__ cv_body,
                            const double *__restrict__ cv_x, const int *__restrict__ body_node0, int *__restrict__ cnt,
                            int *__restrict__ nlocal, const int *__restrict__ cv_scene, const int *__restrict__ active)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb + nf) return;
    bool local = (i < nb ? pflag[i] : lflag[i - nb]) == 0;
    // active (nullable): the pairs of scenes whose flag is clear get no
    // blocks (their rows are not used until they are assembled again)
    if (local && active && !active[cv_scene[i < nb ? pcv[i].x : lcv[i - nb].x]]) local = false;
    int n = 0;
    if (local) {
        Map mp[4];
        pair_maps(i, nb, pcv, lcv, cv_node, cv_body, cv_x, body_node0, mp);
        PairNodes P = pair_nodes(mp);
        n = P.total * P.total;
        atomicAdd(nlocal, 1);
    }
    cnt[i] = n;
}

// DYN_LANES lanes per pair entry: lane j writes output blocks j, j +
// DYN_LANES, ... of the entry, block b at row node b / total and column node
// b % total in the owner groups' order (a pair touches at most two bodies, so
// at most 8 nodes and 64 blocks; one between FEM vertices at most 16).  A
// thread per entry walked up to 64 blocks one after another, which took
// 0.26 ms per assembly where a body met the pads; a wavefront per entry left
// most lanes idle on FEM pairs (40 -> 72 us on the 200k-tet squeeze).
constexpr int DYN_LANES = 16;
__global__ void k_dyn_write(int nb, int nf, const int *__restrict__ off, const int4 *__restrict__ pcv, const int4 *__restrict__ lcv,
                            const double *__restrict__ pH, const double *__restrict__ lbeta, const double *__restrict__ lM,
                            const int *__restrict__ cv_node, const int *__restrict__ cv_body, const double *__restrict__ cv_x,
                            const int *__restrict__ body_node0, unsigned long long *__restrict__ key, int *__restrict__ idx,
                            double *__restrict__ valc)
{
    const int i = (int)((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / DYN_LANES), lane = threadIdx.x & (DYN_LANES - 1);
    if (i >= nb + nf) return;
    const int o0 = off[i], n = off[i + 1] - o0;
    if (n == 0) return;
    Map mp[4];
    pair_maps(i, nb, pcv, lcv, cv_node, cv_body, cv_x, body_node0, mp);
    const PairNodes P = pair_nodes(mp);
    for (int j = lane; j < n; j += DYN_LANES) {
        int ga = 0, qa = j / P.total, gb = 0, qb = j % P.total;
        while (qa >= P.nn[ga]) qa -= P.nn[ga++];
        while (qb >= P.nn[gb]) qb -= P.nn[gb++];
        double B[9], S[9];
        for (int q = 0; q < 9; ++q) S[q] = 0.0;
        for (int k = 0; k < 4; ++k) {
            if (P.g[k] != ga) continue;
            double wk = map_weight(mp[k], qa);
            for (int l = 0; l < 4; ++l) {
                if (P.g[l] != gb) continue;
                double w = wk * map_weight(mp[l], qb);
                pair_block(i, nb, pH, lbeta, lM, k, l, B);
                for (int q = 0; q < 9; ++q) S[q] += w * B[q];
            }
        }
        const int o = o0 + j;
        key[o] = ((unsigned long long)(P.first[ga] + qa) << 32) | (unsigned)(P.first[gb] + qb);
        idx[o] = o;
        for (int q = 0; q < 9; ++q) valc[9 * (size_t)o + q] = S[q];
    }
}

// entries with the same (row, column) after the sort: one head per run
__global__ void k_dyn_heads(int n, const unsigned long long *__restrict__ key, int *__restrict__ head)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > n) return;
    head[p] = (p < n && (p == 0 || key[p] != key[p - 1])) ? 1 : 0;
}

// first sorted position of every run (and n after the last)
__global__ void k_dyn_starts(int n, const int *__restrict__ head, const int *__restrict__ pos, int *__restrict__ start)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > n) return;
    if (p == n || head[p]) start[pos[p]] = p;
}

// one wavefront per run (a body's node blocks can collect thousands of
// entries): lanes stride over the run's blocks, then shuffle-sum in a fixed
// order into one block
__global__ void k_dyn_merge(const int *__restrict__ nruns, const unsigned long long *__restrict__ key, const int *__restrict__ idx,
                            const int *__restrict__ start, const double *__restrict__ valc, int *__restrict__ row,
                            int *__restrict__ col, double *__restrict__ val)
{
    int w = (blockIdx.x * blockDim.x + threadIdx.x) / TILE, lane = threadIdx.x & (TILE - 1);
    if (w >= *nruns) return;
    int lo = start[w], hi = start[w + 1];
    double acc[9];
    for (int q = 0; q < 9; ++q) acc[q] = 0.0;
    // four entries per lane in flight, added in the order of the plain
    // strided loop (a body's blocks collect thousands of entries)
    int r = lo + lane;
    for (; r + 3 * TILE < hi; r += 4 * TILE) {
        const int e0 = idx[r], e1 = idx[r + TILE], e2 = idx[r + 2 * TILE], e3 = idx[r + 3 * TILE];
        double v[4][9];
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            v[0][q] = valc[9 * (size_t)e0 + q];
            v[1][q] = valc[9 * (size_t)e1 + q];
            v[2][q] = valc[9 * (size_t)e2 + q];
            v[3][q] = valc[9 * (size_t)e3 + q];
        }
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int q = 0; q < 9; ++q) acc[q] += v[m][q];
    }
    for (; r < hi; r += TILE) {
        const double *B = valc + 9 * (size_t)idx[r];
        for (int q = 0; q < 9; ++q) acc[q] += B[q];
    }
    for (int q = 0; q < 9; ++q) acc[q] = wave_sum(acc[q]);
    if (lane == 0) {
        unsigned long long k = key[lo];
        row[w] = (int)(k >> 32);
        col[w] = (int)(k & 0xffffffffull);
        for (int q = 0; q < 9; ++q) val[9 * (size_t)w + q] = acc[q];
    }
}

// row pointers from the sorted rows of the *count entries: ptr[n] = first
// position with row >= n
__global__ void k_dyn_ptr(const int *__restrict__ count, int N, const int *__restrict__ key, int *__restrict__ ptr)
{
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r > N) return;
    int lo = 0, hi = *count;
    while (lo < hi) {
        int m = (lo + hi) >> 1;
        if (key[m] < r) lo = m + 1; else hi = m;
    }
    ptr[r] = lo;
}

// rows whose static plus pair-local blocks exceed LONG_ROW, in node order
template <bool WRITE>
__global__ void k_long(int N, const int *__restrict__ row_ptr, const int *__restrict__ dyn_ptr, unsigned long long *__restrict__ mask,
                       int *__restrict__ wcount, const int *__restrict__ woff, int *__restrict__ out)
{
    int n = blockIdx.x * blockDim.x + threadIdx.x;
    int wave = n / TILE, lane = threadIdx.x & (TILE - 1);
    if (!WRITE) {
        bool lg = n < N && (row_ptr[n + 1] - row_ptr[n]) + (dyn_ptr[n + 1] - dyn_ptr[n]) > LONG_ROW;
        unsigned long long m = __ballot(lg);
        if (lane == 0 && wave * TILE < N) { mask[wave] = m; wcount[wave] = __popcll(m); }
    } else {
        if (n >= N) return;
        unsigned long long m = mask[wave];
        if ((m >> lane) & 1ull) out[woff[wave] + __popcll(m & ((1ull << lane) - 1ull))] = n;
    }
}

// per-scene segments of the long-row list (node ranges of scenes are tiles)
__global__ void k_long_seg(int ns, const int *__restrict__ nodew, const int *__restrict__ rows, int nlong, int *__restrict__ seg,
                           int *__restrict__ count)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s == 0) count[0] = nlong;
    if (s > ns) return;
    int start = nodew[s] * TILE, lo = 0, hi = nlong;
    while (lo < hi) {
        int m = (lo + hi) >> 1;
        if (rows[m] < start) lo = m + 1; else hi = m;
    }
    seg[s] = lo;
}

void build_dyn_blocks(ipc_ctx *c)
{
    Dev &D = c->d;
    hipStream_t st = c->stream;
    int64_t nb = c->n_pt + c->n_ee, nf = c->fr_on ? c->n_lag : 0, n = nb + nf;
    int N = c->N;
    D.dyn_ptr.alloc(N + 1);
    c->n_local = 0;
    c->n_dyn = 0;
    if (n > 0) {
        D.dyn_cnt.alloc(n + 1); D.dyn_off.alloc(n + 1);
        D.tickets.alloc(4);
        hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, st, 1, D.tickets.p, 0);
        hipLaunchKernelGGL(k_dyn_count, dim3(blocks_for(n)), dim3(BLOCK), 0, st, (int)nb, (int)nf, D.pair_flag.p, D.lag_flag.p,
                           D.pair_cv.p, D.lag_cv.p, D.cv_node.p, D.cv_body.p, D.cv_x.p, D.body_node0.p, D.dyn_cnt.p, D.tickets.p,
                           D.cv_scene.p, c->assemble_only);
        hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, st, 1, D.dyn_cnt.p + n, 0);
        exclusive_scan(c, D.dyn_cnt.p, D.dyn_off.p, (int)n);
        int hv[2];
        HostReads rd(c);
        rd.add(&hv[0], D.dyn_off.p + n, sizeof(int));
        rd.add(&hv[1], D.tickets.p, sizeof(int));
        rd.wait();
        c->n_dyn = hv[0];
        c->n_local = hv[1];
    }
    int64_t E = c->n_dyn;
    if (E > 0) {
        if (E > c->cap_dyn) {
            if (c->ws.base)
                throw Error(IPC_E_CAPACITY, std::to_string(E) + " pair-local blocks exceed the planned capacity of " +
                                                std::to_string(c->cap_dyn));
            c->cap_dyn = E + E / 2 + 1024;
            D.dyn_key64.alloc(c->cap_dyn); D.dyn_key64b.alloc(c->cap_dyn);
            for (auto *b : {&D.dyn_idx, &D.dyn_idx2, &D.dyn_head, &D.dyn_pos, &D.dyn_start, &D.dyn_row, &D.dyn_col}) b->alloc(c->cap_dyn + 1);
            D.dyn_val.alloc(9 * (size_t)c->cap_dyn); D.dyn_val_coo.alloc(9 * (size_t)c->cap_dyn);
        }
        hipLaunchKernelGGL(k_dyn_write, dim3(blocks_for(n * DYN_LANES)), dim3(BLOCK), 0, st, (int)nb, (int)nf, D.dyn_off.p, D.pair_cv.p, D.lag_cv.p,
                           D.pair_H.p, D.lag_beta.p, D.lag_M.p, D.cv_node.p, D.cv_body.p, D.cv_x.p, D.body_node0.p, D.dyn_key64.p,
                           D.dyn_idx.p, D.dyn_val_coo.p);
        int end_bit = 33;
        while ((1ll << (end_bit - 32)) <= N) ++end_bit;
        size_t bytes = 0;
        IPC_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, D.dyn_key64.p, D.dyn_key64b.p, D.dyn_idx.p, D.dyn_idx2.p, (int)E,
                                                   0, end_bit, st));
        D.sort_tmp.alloc(bytes + 16);
        IPC_HIP(hipcub::DeviceRadixSort::SortPairs(D.sort_tmp.p, bytes, D.dyn_key64.p, D.dyn_key64b.p, D.dyn_idx.p, D.dyn_idx2.p,
                                                   (int)E, 0, end_bit, st));
        hipLaunchKernelGGL(k_dyn_heads, dim3(blocks_for(E + 1)), dim3(BLOCK), 0, st, (int)E, D.dyn_key64b.p, D.dyn_head.p);
        exclusive_scan(c, D.dyn_head.p, D.dyn_pos.p, (int)E);
        hipLaunchKernelGGL(k_dyn_starts, dim3(blocks_for(E + 1)), dim3(BLOCK), 0, st, (int)E, D.dyn_head.p, D.dyn_pos.p, D.dyn_start.p);
        hipLaunchKernelGGL(k_dyn_merge, dim3(blocks_for(E * TILE)), dim3(BLOCK), 0, st, D.dyn_pos.p + E, D.dyn_key64b.p, D.dyn_idx2.p,
                           D.dyn_start.p, D.dyn_val_coo.p, D.dyn_row.p, D.dyn_col.p, D.dyn_val.p);
        // unique count: dyn_pos[E]; the row pointers search the sorted rows of
        // the first dyn_pos[E] entries, read on the device
        hipLaunchKernelGGL(k_dyn_ptr, dim3(blocks_for(N + 1)), dim3(BLOCK), 0, st, D.dyn_pos.p + E, N, D.dyn_row.p, D.dyn_ptr.p);
    } else {
        hipLaunchKernelGGL(k_fill_int, dim3(blocks_for(N + 1)), dim3(BLOCK), 0, st, N + 1, D.dyn_ptr.p, 0);
    }
    // long rows of the product
    int nw = (N + TILE - 1) / TILE;
    D.mkey.alloc(nw); D.wcount.alloc(nw + 1); D.woff.alloc(nw + 1); D.long_rows.alloc(N + 1);
    hipLaunchKernelGGL(k_long<false>, dim3(blocks_for(N)), dim3(BLOCK), 0, st, N, D.row_ptr.p, D.dyn_ptr.p, D.mkey.p, D.wcount.p,
                       nullptr, nullptr);
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, st, 1, D.wcount.p + nw, 0);
    exclusive_scan(c, D.wcount.p, D.woff.p, nw);
    {
        int hv[2] = {0, 0};
        HostReads rd(c);
        rd.add(&hv[0], D.woff.p + nw, sizeof(int));
        if (c->n_dyn > 0) rd.add(&hv[1], D.dyn_pos.p + c->n_dyn, sizeof(int));
        rd.wait();
        c->n_long = hv[0];
        c->n_dyn = hv[1];   // blocks after merging equal (row, column) entries
    }
    if (c->n_long)
        hipLaunchKernelGGL(k_long<true>, dim3(blocks_for(N)), dim3(BLOCK), 0, st, N, D.row_ptr.p, D.dyn_ptr.p, D.mkey.p, D.wcount.p,
                           D.woff.p, D.long_rows.p);
    if (c->n_long > c->long_cap) c->long_cap = (c->n_long + 63) / 64 * 64;
    D.part_long.alloc(c->long_cap + 1);
    D.long_count.alloc(1);
    hipLaunchKernelGGL(k_long_seg, dim3(blocks_for(c->n_scenes + 1)), dim3(BLOCK), 0, st, c->n_scenes, seg_ptr(c, R_NODEW),
                       D.long_rows.p, c->n_long, seg_ptr(c, R_LONG), D.long_count.p);
    pcg_wginfo(c);
}

// ---------------------------------------------------------------------------
// additive CCD over swept candidates; per-scene minimum through the bit
// pattern of non-negative doubles (monotone as unsigned integers)
// ---------------------------------------------------------------------------
__device__ double accd(int kind, const d3 *x0, const d3 *p, double s)
{
    // every operation in its written order, unfused: the bound of each
    // candidate is the same double on any implementation of this recipe
#pragma clang fp contract(off)
    d3 pm = {0.25 * (p[0].x + p[1].x + p[2].x + p[3].x), 0.25 * (p[0].y + p[1].y + p[2].y + p[3].y),
             0.25 * (p[0].z + p[1].z + p[2].z + p[3].z)};
    d3 dp[4];
    double nrm[4];
    for (int k = 0; k < 4; ++k) {
        dp[k] = {p[k].x - pm.x, p[k].y - pm.y, p[k].z - pm.z};
        nrm[k] = sqrt(xdot(dp[k], dp[k]));
    }
    double lp = kind == 0 ? nrm[0] + fmax(nrm[1], fmax(nrm[2], nrm[3])) : fmax(nrm[0], nrm[1]) + fmax(nrm[2], nrm[3]);
    if (lp == 0.0) return 1.0;
    d3 xx[4] = {x0[0], x0[1], x0[2], x0[3]};
    int ty;
    double d = sqrt(pair_d2(kind, xx, &ty));
    double gap = s * d;
    double t = 0.0, tl = (1.0 - s) * d / lp;
    for (int it = 0; it < 10000; ++it) {
        for (int k = 0; k < 4; ++k) { xx[k].x += tl * dp[k].x; xx[k].y += tl * dp[k].y; xx[k].z += tl * dp[k].z; }
        d = sqrt(pair_d2(kind, xx, &ty));
        if (t > 0.0 && d < gap) return t;
        t += tl;
        if (t > 1.0) return 1.0;
        tl = 0.9 * d / lp;
    }
    return t;
}

__global__ void k_ccd(int npt, int nee, const int2 *__restrict__ pt, const int2 *__restrict__ ee, const int4 *__restrict__ tri,
                      const int2 *__restrict__ edge, const double *__restrict__ xw0, const double *__restrict__ xw1,
                      const int *__restrict__ cv_scene, const double *__restrict__ sparam, const int *__restrict__ active,
                      unsigned long long *__restrict__ amin, int stride)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npt + nee) return;
    int kind = i < npt ? 0 : 1;
    int2 pr = kind == 0 ? pt[i] : ee[i - npt];
    int cv[4];
    pair_vertices(kind, pr, tri, edge, cv);
    int s = cv_scene[cv[0]];
    if (active && !active[s]) return;
    d3 x0[4], x1[4], p[4];
    for (int k = 0; k < 4; ++k) {
        x0[k] = ld3(xw0, cv[k]);
        x1[k] = ld3(xw1, cv[k]);
        p[k] = {x1[k].x - x0[k].x, x1[k].y - x0[k].y, x1[k].z - x0[k].z};
    }
    // exact swept candidates only (the list may be a kept superset): the
    // boxes of the two sides over both end positions, inflated as in the
    // broad phase (vertex 1.01 dhat, triangle 0; each edge half of that)
    {
        double r = 1.01 * sparam[8 * s + 2];
        double ra = kind == 0 ? r : 0.5 * r, rb = kind == 0 ? 0.0 : 0.5 * r;
        int na = kind == 0 ? 1 : 2;
        double A[6], B[6];
        for (int k = 0; k < 3; ++k) { A[k] = B[k] = INFINITY; A[3 + k] = B[3 + k] = -INFINITY; }
        for (int q = 0; q < 4; ++q) {
            double *T = q < na ? A : B;
            T[0] = fmin(T[0], fmin(x0[q].x, x1[q].x)); T[3] = fmax(T[3], fmax(x0[q].x, x1[q].x));
            T[1] = fmin(T[1], fmin(x0[q].y, x1[q].y)); T[4] = fmax(T[4], fmax(x0[q].y, x1[q].y));
            T[2] = fmin(T[2], fmin(x0[q].z, x1[q].z)); T[5] = fmax(T[5], fmax(x0[q].z, x1[q].z));
        }
        for (int k = 0; k < 3; ++k) { A[k] -= ra; A[3 + k] += ra; B[k] -= rb; B[3 + k] += rb; }
        if (!overlap(A, B)) return;
    }
    double t = accd(kind, x0, p, sparam[8 * s + 5]);
    if (t < 1.0) atomicMin(amin + (size_t)stride * s, (unsigned long long)__double_as_longlong(t));
}

void launch_ccd(ipc_ctx *c, const double *xw0, const double *xw1)
{
    Dev &D = c->d;
    launch_hs_ccd(c, xw0, xw1);
    int64_t n = c->n_cand_pt + c->n_cand_ee;
    if (n == 0) return;
    prof_begin(c, IPC_K_CCD);
    hipLaunchKernelGGL(k_ccd, dim3(blocks_for(n, 64)), dim3(64), 0, c->stream, (int)c->n_cand_pt, (int)c->n_cand_ee, D.cand_pt.p,
                       D.cand_ee.p, D.tri.p, D.edge.p, xw0, xw1, D.cv_scene.p, D.sparam.p, D.ls_active.p,
                       (unsigned long long *)(D.scal.p + S_CCD), NSLOT);
    prof_end(c, IPC_K_CCD, 0.0);
}

// Adaptive barrier stiffness (IPC's doubling rule, applied to the barrier
// term of Eq. (3)).  k_pair_dmin: the smallest squared distance over each
// scene's active pairs, an atomic min on the bit pattern (non-negative
// doubles order as their bits; the result does not depend on the order).
static __global__ void k_set_slot_c(int ns, double *scal, int slot, double v)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < ns) scal[(size_t)s * NSLOT + slot] = v;
}

__global__ void k_pair_dmin(int npt, int nee, const int2 *__restrict__ pt, const int2 *__restrict__ ee, const int4 *__restrict__ tri,
                            const int2 *__restrict__ edge, const double *__restrict__ xw, const int *__restrict__ cv_scene,
                            unsigned long long *__restrict__ dmin, int stride)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npt + nee) return;
    int kind = i < npt ? 0 : 1;
    int2 pr = kind == 0 ? pt[i] : ee[i - npt];
    int cv[4];
    pair_vertices(kind, pr, tri, edge, cv);
    d3 x[4] = {ld3(xw, cv[0]), ld3(xw, cv[1]), ld3(xw, cv[2]), ld3(xw, cv[3])};
    int type;
    double d2 = pair_d2(kind, x, &type);
    if (!(d2 > 0.0)) d2 = 0.0;
    atomicMin(dmin + (size_t)stride * cv_scene[cv[0]], (unsigned long long)__double_as_longlong(d2));
}

// Per scene, from its smallest active distance d (infinite without pairs):
// at an accepted update (S_LS_ON set), kappa doubles when d < frac dhat and d
// is below the previous iterate's, capped at factor kappa0; the previous
// distance then becomes d.  first: the step start only records d.
__global__ void k_kappa_update(int ns, double frac, double factor, int first, double *__restrict__ sparam, double *__restrict__ scal)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= ns) return;
    double *S = scal + (size_t)s * NSLOT;
    double d = sqrt(S[S_DMIN]);
    bool accepted = S[S_LS_ON] != 0.0;
    if (!first && accepted) {
        double *sp = sparam + 8 * (size_t)s;
        if (d < frac * sp[P_DHAT] && d < S[S_DPREV]) {
            double k2 = 2.0 * sp[P_KAPPA], kmax = factor * S[S_KAPPA0];
            sp[P_KAPPA] = k2 < kmax ? k2 : kmax;
        }
    }
    if (first || accepted) S[S_DPREV] = d;
}

void launch_kappa_update(ipc_ctx *c, const double *xw, bool first)
{
    Dev &D = c->d;
    hipStream_t st = c->stream;
    hipLaunchKernelGGL(k_set_slot_c, dim3(blocks_for(c->n_scenes, 64)), dim3(64), 0, st, c->n_scenes, D.scal.p, S_DMIN, INFINITY);
    launch_hs_dmin(c, xw);
    int64_t n = c->n_pt + c->n_ee;
    if (n)
        hipLaunchKernelGGL(k_pair_dmin, dim3(blocks_for(n)), dim3(BLOCK), 0, st, (int)c->n_pt, (int)c->n_ee, D.pt.p, D.ee.p, D.tri.p,
                           D.edge.p, xw, D.cv_scene.p, (unsigned long long *)(D.scal.p + S_DMIN), NSLOT);
    hipLaunchKernelGGL(k_kappa_update, dim3(blocks_for(c->n_scenes, 64)), dim3(64), 0, st, c->n_scenes, c->kappa_frac,
                       c->kappa_factor, (int)first, D.sparam.p, D.scal.p);
}

} // namespace ipc

namespace ipc {

// Sizes every buffer whose length depends on the contact state for the given
// capacity, once, at creation over a caller's workspace: later calls then
// take no memory, and a state beyond the capacity ends with IPC_E_CAPACITY.
void reserve_capacity(ipc_ctx *c, int64_t P, int64_t C, int64_t B)
{
    Dev &D = c->d;
    hipStream_t st = c->stream;
    P = std::max<int64_t>(P, 1); C = std::max<int64_t>(C, 1); B = std::max<int64_t>(B, 1);
    const int64_t Pp = std::max<int64_t>(std::max(c->TRI, c->EDGE), 1), Q = std::max<int64_t>(std::max(c->NSURF, c->EDGE), 1);
    // broad phase over the larger kind of primitive and of query
    D.box.alloc(6 * Pp); D.mid.alloc(Pp); D.mid2.alloc(Pp);
    D.bvh_left.alloc(Pp); D.bvh_right.alloc(Pp); D.bvh_range.alloc(Pp); D.bvh_flag.alloc(Pp); D.bvh_box.alloc(6 * Pp);
    D.bvh_lev.alloc(6 * (2 * Pp + 64)); D.bvh_moving.alloc(Pp + 1); D.bvh_mscan.alloc(Pp + 1); D.bvh_nmoving.alloc(Pp);
    D.qcount.alloc(Q + 1); D.qoff.alloc(Q + 1); D.qstash.alloc(Q * TRAV_STASH);
    D.qkey.alloc(Q); D.qkey2.alloc(Q); D.qid.alloc(Q); D.qperm.alloc(Q);
    // scratch words shared by the Morton keys, the narrow phase's masks and the long rows' masks
    const int64_t nw = std::max<int64_t>(C, c->N) / TILE + 1;
    D.mkey.alloc(std::max<int64_t>(Pp, nw)); D.mkey2.alloc(Pp);
    D.wcount.alloc(nw + 1); D.woff.alloc(nw + 1);
    c->cap_cand_pt = c->cap_cand_ee = C;
    D.cand_pt.alloc(C); D.cand_ee.alloc(C);
    D.cand_ref.alloc(6 * (size_t)c->CV + 1);
    c->cap_pt = c->cap_ee = P;
    D.pt.alloc(P); D.ee.alloc(P);
    // barrier: per-pair values over pairs or candidates, gradients and blocks over pairs
    const int64_t PC = std::max(P, C);
    D.pair_part.alloc(PC + 1); D.pair_w64.alloc(PC / TILE + 1);
    D.pair_g.alloc(12 * P + 3);
    for (auto *b : {&D.pg_key, &D.pg_code, &D.pg_key2, &D.pg_code2}) b->alloc(4 * P + 1);
    D.pair_cv.alloc(P + 1); D.pair_H.alloc(45 * (P + 1)); D.pair_flag.alloc(P + 1);
    for (auto *b : {&D.pb_key, &D.pb_code, &D.pb_key2, &D.pb_code2}) b->alloc(16 * P + 1);
    // friction lag
    c->cap_lag = P;
    D.lag_cv.alloc(P); D.lag_beta.alloc(4 * P); D.lag_nrm.alloc(3 * P); D.lag_lam.alloc(P); D.lag_rn.alloc(3 * P);
    D.lag_M.alloc(6 * P); D.lag_flag.alloc(P); D.lag_type.alloc(P); D.lag_ex.alloc(P); D.lag_merge.alloc(P);
    for (auto *b : {&D.lag_key, &D.lag_code, &D.lag_key2, &D.lag_code2}) b->alloc(16 * P);
    D.lag_g.alloc(12 * P);
    for (auto *b : {&D.lg_key, &D.lg_code, &D.lg_key2, &D.lg_code2}) b->alloc(4 * P);
    D.fr_part.alloc(P + 1); D.fr_w64.alloc(P / TILE + 1);
    D.gcv.alloc(3 * (size_t)c->CV + 3);
    // pair-local blocks
    D.dyn_cnt.alloc(2 * P + 1); D.dyn_off.alloc(2 * P + 1);
    c->cap_dyn = B;
    D.dyn_key64.alloc(B); D.dyn_key64b.alloc(B);
    for (auto *b : {&D.dyn_idx, &D.dyn_idx2, &D.dyn_head, &D.dyn_pos, &D.dyn_start, &D.dyn_row, &D.dyn_col}) b->alloc(B + 1);
    D.dyn_val.alloc(9 * B); D.dyn_val_coo.alloc(9 * B);
    // run sums: the largest has 16 entries of 9 doubles per pair
    D.rs_first.alloc(9 * (16 * P / TILE + 1) + 1); D.rs_last.alloc(9 * (16 * P / TILE + 1) + 1);
    // PCG: long rows at most every row
    c->long_cap = std::max(c->long_cap, (c->N + 63) / 64 * 64);
    D.part_long.alloc(c->long_cap + 1);
    D.part_node3.alloc(c->N / TILE + 1); D.pcg_part.alloc(4 * (size_t)(c->N / TILE) + 1);
    D.pcg_st.alloc(8 * (size_t)c->n_scenes); D.pcg_act.alloc(2 * (size_t)c->n_scenes); D.pcg_it.alloc(2 * (size_t)c->n_scenes);
    D.pcg_prev.alloc(c->n_scenes); D.cand_flag.alloc(c->n_scenes);
    // the sorts' temporary storage at these sizes
    size_t tmp = 0, b = 0;
    auto upd = [&]() { tmp = std::max(tmp, b); };
    b = sort_entries_bytes(c, 16 * std::max(P, std::max<int64_t>(c->M_HS, 1)), 31); upd();   // the run sums' entry sorts
    IPC_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, b, D.dyn_key64.p, D.dyn_key64b.p, D.dyn_idx.p, D.dyn_idx2.p, (int)B, 0, 64, st)); upd();
    IPC_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, b, D.mkey.p, D.mkey2.p, D.mid.p, D.mid2.p, (int)Pp, 0, 64, st)); upd();
    IPC_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, b, D.qkey.p, D.qkey2.p, D.qid.p, D.qperm.p, (int)Q, 0, 64, st)); upd();
    IPC_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, b, D.dyn_cnt.p, D.dyn_off.p, (int)std::max<int64_t>(std::max(B, 2 * P + 1), std::max(nw, Q + 1)), st)); upd();
    D.sort_tmp.alloc(tmp + 16);
}

} // namespace ipc
