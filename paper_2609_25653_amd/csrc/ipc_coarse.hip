// Coarse correction of the PCG preconditioner.  The paper names no linear
// solver (Sec. III-C); block-Jacobi alone leaves the smooth, low-frequency
// error of soft bodies to be removed one neighbourhood per iteration.  The
// preconditioner used by the PCG is the additive two-level operator
//
//     M^-1 = D^-1 + P C^-1 P^T
//
// with D the 3x3 (FEM vertex) and 12x12 (affine body) diagonal blocks and P
// the aggregation of nodes into groups of CG_AGG that share one translation:
// FEM vertices and the translation node of every affine body, taken in the
// Morton order of their positions at creation, so that a group is a compact
// patch of one object.  That order is also the order of a scene's first
// nodes (a body's translation is represented there by an unused slot), so a
// domain is one contiguous range of nodes.  C is block diagonal over domains of CG_DOM
// consecutive groups: each block is the domain's part of P^T A P (the sum of
// the 3x3 blocks of A between the nodes of two groups), a dense SPD matrix
// of at most 96 x 96 that is inverted after every assembly.  Nothing crosses
// scenes: groups and domains are per scene.
//
// Per PCG iteration one launch (CG_SPLIT workgroups per domain) restricts
// the new residual to its groups, multiplies by the domain's inverse, adds
// the result to z on every node of the group and writes r . z of the
// correction, which the next step's reduction adds to r . z of the
// block-Jacobi part.  For a context of one scene the PCG step does the same
// inside its own launch (k_pcg_step<true>); this kernel then runs once per
// solve, for the first z.
#include <algorithm>
#include <cstdlib>
#include <numeric>

#include "ipc_device.h"
#include "ipc_internal.h"
#include "ipc_kernels.h"
#include "ipc_pcgdev.h"

namespace ipc {

void coarse_setup(ipc_ctx *c)
{
    const int ns = c->n_scenes;
    c->seg_cdom.assign(ns + 1, 0);
    std::vector<int> ent, nodes, dom_scene, grp, node_da(c->N, -1);
    int ndom = 0;
    bool windows = ns == 1;
    for (int s = 0; s < ns; ++s) {
        c->seg_cdom[s] = ndom;
        if (!c->coarse) continue;
        const SceneInfo &S = c->sc[s];
        // groups of CG_AGG consecutive entries of the scene's Morton order,
        // domains of CG_DOM consecutive groups; a scene's last group and
        // domain may be short
        const int per_dom = CG_AGG * CG_DOM;
        for (int m = 0; m < (int)S.entry.size(); ++m) {
            if (m % per_dom == 0) {
                ent.push_back((int)nodes.size());
                dom_scene.push_back(s);
                ++ndom;
            }
            const int g = (ndom - 1) * CG_DOM + (m % per_dom) / CG_AGG;
            if (m % CG_AGG == 0) grp.push_back(g);
            const int node = S.entry[m] >= 0 ? S.node0 + m : S.bnode0 + 4 * (-1 - S.entry[m]);
            node_da[node] = g;
            nodes.push_back(node);
        }
        // one scene at node 0: entry e of domain d is node CG_AGG CG_DOM d + e
        // or stands in that slot for a body's translation node
        windows = windows && S.node0 == 0;
    }
    c->cg_fusable = windows && ndom > 0;
    c->seg_cdom[ns] = ndom;
    ent.push_back((int)nodes.size());   // ndom + 1 offsets
    c->n_cdom = ndom;
    // a fixed cost per iteration (a few dependent stages): it pays on large contexts
    c->coarse_on = ndom > 0 && (c->coarse_forced || c->N >= CG_MIN_NODES);
    c->n_cgrp = (int)grp.size();
    Dev &D = c->d;
    D.cg_grp.upload(grp.empty() ? std::vector<int>(1, 0) : grp, c->stream);
    D.cg_ent.upload(ent, c->stream);
    D.cg_nodes.upload(nodes.empty() ? std::vector<int>(1, 0) : nodes, c->stream);
    {   // the same lists padded to CG_AGG * CG_DOM entries per domain (-1 after the end)
        std::vector<int> pn((size_t)std::max(ndom, 1) * CG_AGG * CG_DOM, -1);
        for (int d = 0; d < ndom; ++d)
            for (int e = ent[d]; e < ent[d + 1]; ++e) pn[(size_t)d * CG_AGG * CG_DOM + (e - ent[d])] = nodes[e];
        D.cg_pnodes.upload(pn, c->stream);
    }
    {   // one scene: per domain the entries whose slot stands for a body's translation node
        std::vector<int> ph_ptr(ndom + 1, 0), ph_e, ph_n;
        if (c->cg_fusable) {
            const SceneInfo &S = c->sc[0];
            c->cg_nfr = (int)S.entry.size();
            for (int m = 0; m < c->cg_nfr; ++m)
                if (S.entry[m] < 0) {
                    ph_ptr[m / (CG_AGG * CG_DOM) + 1]++;
                    ph_e.push_back(m % (CG_AGG * CG_DOM));
                    ph_n.push_back(S.bnode0 + 4 * (-1 - S.entry[m]));
                }
            for (int d = 0; d < ndom; ++d) ph_ptr[d + 1] += ph_ptr[d];
        }
        D.cg_ph_ptr.upload(ph_ptr, c->stream);
        D.cg_ph_e.upload(ph_e.empty() ? std::vector<int>(1, 0) : ph_e, c->stream);
        D.cg_ph_n.upload(ph_n.empty() ? std::vector<int>(1, 0) : ph_n, c->stream);
    }
    D.cg_node_da.upload(node_da, c->stream);
    D.cg_dom_scene.upload(dom_scene.empty() ? std::vector<int>(1, 0) : dom_scene, c->stream);
    // zero once: the entries past a short domain's n are never written and
    // are read as 0 by the product with the inverse
    D.cg_inv.alloc((size_t)std::max(ndom, 1) * CG_N * CG_N);
    D.cg_inv.zero(c->stream, (size_t)std::max(ndom, 1) * CG_N * CG_N);
    D.cg_part.alloc(2 * (size_t)CG_SPLIT * std::max(ndom, 1));
}

// The domains' blocks of P^T A P: one workgroup per group (32 rows of 8
// lanes) sums the 3x3 blocks of its nodes' rows (block-CSR and pair-local)
// whose column node lies in a group of the same domain, then stores the
// group's 3 rows of its domain's block (all CG_N columns; a group owns its
// rows, so no other workgroup writes them).  The sums come out the same on
// every run: each row adds into a strip of its own in LDS, its 8 lanes take
// turns in lane order (blocks loaded ahead into registers, CG_PRE at a time),
// and the 32 strips are then summed in row order.
constexpr int CG_ASM = 256, CG_LPR = CG_ASM / CG_AGG, CG_PRE = 4;   // lanes per row; blocks per lane per round
__global__ void __launch_bounds__(CG_ASM) k_coarse_assemble(const int *__restrict__ grp, const int *__restrict__ ent,
                                                            const int *__restrict__ nodes, const int *__restrict__ node_da,
                                                            const int *__restrict__ row_ptr, const int *__restrict__ col,
                                                            const double *__restrict__ val, const int *__restrict__ dptr,
                                                            const int *__restrict__ dcol, const double *__restrict__ dval,
                                                            double *__restrict__ mat, const int *__restrict__ dom_scene,
                                                            const int *__restrict__ active)
{
    __shared__ double P[CG_AGG][3 * CG_N];   // 72 KB: one strip per row
    const int g = grp[blockIdx.x], d = g / CG_DOM, a = g % CG_DOM;
    if (active && !active[dom_scene[d]]) return;   // uniform over the workgroup
    for (int q = threadIdx.x; q < CG_AGG * 3 * CG_N; q += CG_ASM) (&P[0][0])[q] = 0.0;
    __syncthreads();
    const int row = (int)threadIdx.x / CG_LPR, sub = threadIdx.x % CG_LPR, e = ent[d] + a * CG_AGG + row;
    const bool live = e < ent[d + 1];
    const int i = live ? nodes[e] : 0;
    const int n0 = live ? row_ptr[i + 1] - row_ptr[i] : 0, n1 = live ? dptr[i + 1] - dptr[i] : 0;
    // the lane's blocks: k = sub, sub + 8, ... over the row's static then
    // pair-local blocks; every lane runs the same number of rounds
    int mine = n0 + n1 > sub ? (n0 + n1 - sub + CG_LPR - 1) / CG_LPR : 0;
    int most = mine;
    for (int o = 32; o > 0; o >>= 1) most = max(most, __shfl_xor(most, o, 64));
    __shared__ int wmost[CG_ASM / 64];
    if ((threadIdx.x & 63) == 0) wmost[threadIdx.x / 64] = most;
    __syncthreads();
    most = 0;
    for (int w = 0; w < CG_ASM / 64; ++w) most = max(most, wmost[w]);
    for (int r0 = 0; r0 < most; r0 += CG_PRE) {
        double B[CG_PRE][9];
        int dst[CG_PRE];
#pragma unroll
        for (int u = 0; u < CG_PRE; ++u) {
            dst[u] = -1;
            const int kk = sub + CG_LPR * (r0 + u);
            if (r0 + u >= mine) continue;
            const bool dyn = kk >= n0;
            const int j = dyn ? dcol[dptr[i] + kk - n0] : col[row_ptr[i] + kk];
            const double *src = dyn ? dval + 9 * (size_t)(dptr[i] + kk - n0) : val + 9 * (size_t)(row_ptr[i] + kk);
            const int tj = node_da[j];
            if (tj < 0 || tj / CG_DOM != d) continue;
            dst[u] = 3 * (tj % CG_DOM);
#pragma unroll
            for (int q = 0; q < 9; ++q) B[u][q] = src[q];
        }
        for (int turn = 0; turn < CG_LPR; ++turn) {
            if (sub == turn) {
#pragma unroll
                for (int u = 0; u < CG_PRE; ++u) {
                    if (dst[u] < 0) continue;
                    double *o = &P[row][dst[u]];
#pragma unroll
                    for (int r = 0; r < 3; ++r)
#pragma unroll
                        for (int k = 0; k < 3; ++k) o[r * CG_N + k] += B[u][3 * r + k];
                }
            }
            __syncthreads();
        }
    }
    double *G = mat + (size_t)d * CG_N * CG_N + (size_t)(3 * a) * CG_N;   // rows 3a .. 3a + 2, contiguous
    for (int q = threadIdx.x; q < 3 * CG_N; q += CG_ASM) {
        double t = 0.0;
        for (int r = 0; r < CG_AGG; ++r) t += P[r][q];
        G[q] = t;
    }
}

// One workgroup per domain: Gauss-Jordan on the 3x3 diagonal pivot blocks
// K of the domain's block of P^T A P (n is a multiple of 3; the matrix is SPD,
// so every pivot block is and no exchanges are needed):
//     A_IJ -= A_IK P^-1 A_KJ off row and column K,
//     A_KJ <- P^-1 A_KJ,  A_IK <- -A_IK P^-1,  A_KK <- P^-1,  P = A_KK.
// Thread t keeps the 3x3 tile (I, J) = (t / 32, t % 32) of the 96 x 96
// matrix in registers for the whole inversion; at each step the 63 tiles of
// row and column K are published to LDS, every thread reads the pivot and
// the two tiles it needs, and updates its own tile.  (The first version kept
// the whole matrix in LDS and updated 9 scattered entries per thread, each
// with six LDS reads and a read-modify-write: 97 us per assembly.)  Rows and
// columns past a short domain's n stay the identity.  A pivot that is not
// positive definite (the adjoint's unprojected Hessian can be indefinite)
// gives the domain a zero inverse: there the preconditioner is block-Jacobi
// alone.  n / 3 steps of two barriers each.
constexpr int CG_INV = 1024, CG_T = CG_N / 3;   // threads; tiles per row
static_assert(CG_T * CG_T == CG_INV, "one 3x3 tile per thread");
__global__ void __launch_bounds__(CG_INV) k_coarse_invert(const int *__restrict__ ent, double *__restrict__ mat,
                                                          const int *__restrict__ dom_scene, const int *__restrict__ active)
{
    __shared__ double rowK[CG_T][9], colK[CG_T][9];   // the tiles of pivot row and column K
    const int d = blockIdx.x, ne = ent[d + 1] - ent[d], n = 3 * ((ne + CG_AGG - 1) / CG_AGG);
    if (active && !active[dom_scene[d]]) return;   // uniform over the workgroup
    double *G = mat + (size_t)d * CG_N * CG_N;
    const int I = threadIdx.x / CG_T, J = threadIdx.x % CG_T;
    double a[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int i = 3 * I + r, j = 3 * J + c;
            a[r][c] = (i < n && j < n) ? G[(size_t)i * CG_N + j] : (i == j ? 1.0 : 0.0);
        }
    bool bad = false;
    for (int K = 0; 3 * K < n; ++K) {
        if (I == K) {
#pragma unroll
            for (int q = 0; q < 9; ++q) rowK[J][q] = a[q / 3][q % 3];
        }
        if (J == K) {
#pragma unroll
            for (int q = 0; q < 9; ++q) colK[I][q] = a[q / 3][q % 3];
        }
        __syncthreads();
        double p[3][3];   // every thread reads the same pivot block
#pragma unroll
        for (int q = 0; q < 9; ++q) p[q / 3][q % 3] = rowK[K][q];
        const double c00 = p[1][1] * p[2][2] - p[1][2] * p[2][1], c01 = p[1][2] * p[2][0] - p[1][0] * p[2][2],
                     c02 = p[1][0] * p[2][1] - p[1][1] * p[2][0], c10 = p[0][2] * p[2][1] - p[0][1] * p[2][2],
                     c11 = p[0][0] * p[2][2] - p[0][2] * p[2][0], c12 = p[0][1] * p[2][0] - p[0][0] * p[2][1],
                     c20 = p[0][1] * p[1][2] - p[0][2] * p[1][1], c21 = p[0][2] * p[1][0] - p[0][0] * p[1][2],
                     c22 = p[0][0] * p[1][1] - p[0][1] * p[1][0];
        const double det = p[0][0] * c00 + p[0][1] * c01 + p[0][2] * c02;
        if (!(p[0][0] > 0.0 && c22 > 0.0 && det > 0.0)) { bad = true; break; }   // uniform
        const double id = 1.0 / det;
        const double qi[3][3] = {{c00 * id, c10 * id, c20 * id}, {c01 * id, c11 * id, c21 * id}, {c02 * id, c12 * id, c22 * id}};
        if (I != K && J != K) {
            // w = P^-1 A_KJ, column by column, then A_IJ -= A_IK w
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double b0 = rowK[J][c], b1 = rowK[J][3 + c], b2 = rowK[J][6 + c];
                const double w0 = qi[0][0] * b0 + qi[0][1] * b1 + qi[0][2] * b2, w1 = qi[1][0] * b0 + qi[1][1] * b1 + qi[1][2] * b2,
                             w2 = qi[2][0] * b0 + qi[2][1] * b1 + qi[2][2] * b2;
#pragma unroll
                for (int r = 0; r < 3; ++r) a[r][c] -= colK[I][3 * r] * w0 + colK[I][3 * r + 1] * w1 + colK[I][3 * r + 2] * w2;
            }
        } else if (I == K && J != K) {
            double b[3][3];
#pragma unroll
            for (int q = 0; q < 9; ++q) b[q / 3][q % 3] = a[q / 3][q % 3];
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int c = 0; c < 3; ++c) a[r][c] = qi[r][0] * b[0][c] + qi[r][1] * b[1][c] + qi[r][2] * b[2][c];
        } else if (J == K && I != K) {
            double b[3][3];
#pragma unroll
            for (int q = 0; q < 9; ++q) b[q / 3][q % 3] = a[q / 3][q % 3];
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int c = 0; c < 3; ++c) a[r][c] = -(b[r][0] * qi[0][c] + b[r][1] * qi[1][c] + b[r][2] * qi[2][c]);
        } else {
#pragma unroll
            for (int q = 0; q < 9; ++q) a[q / 3][q % 3] = qi[q / 3][q % 3];
        }
        __syncthreads();   // the tiles of row and column K are read before the next step publishes its own
    }
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int i = 3 * I + r, j = 3 * J + c;
            if (i < n && j < n) G[(size_t)i * CG_N + j] = bad ? 0.0 : a[r][c];
        }
}

// CG_SPLIT workgroups per domain of a scene that updated its residual
// (act != 0).  Each one restricts the whole residual, rc = P^T r over the
// domain's groups, multiplies its slice of CG_N / CG_SPLIT rows of the
// domain's inverse by rc, adds the result to z on the nodes of its slice's
// groups, and writes the partial of rc . zc (= r . P zc) over its rows into
// part[CG_SPLIT d + slice].  The stages are latency-bound and one workgroup
// per domain left most CUs idle while each of the few busy ones streamed a
// 74 KB inverse; a slice reads a quarter of it.  Every load that does not
// wait for another is issued first: the inverse's rows (entries past a short
// domain's n are 0), the scene's flag, then the entries' r and z.  A group is
// 32 consecutive entries, i.e. half a wavefront of one pass over the entries.
// The slices of a domain are numbered so that they share an XCD (workgroups
// go round-robin over the 8 XCDs): the residual's repeated reads hit its L2.
__global__ void __launch_bounds__(CG_APPLY) k_coarse_apply(int ndom, int single, const int *__restrict__ pnodes,
                                                           const int *__restrict__ dom_scene, const int *__restrict__ act,
                                                           const double *__restrict__ inv, const double *__restrict__ r,
                                                           double *__restrict__ z, double *__restrict__ part)
{
    __shared__ double rc[CG_N], zl[CG_ROWS];
    const int b = blockIdx.x, k = b / NXCD;
    const int sl = k % CG_SPLIT, d = b % NXCD + NXCD * (k / CG_SPLIT);
    if (d >= ndom) return;   // the grid is rounded up to whole XCD rounds
    const int t = threadIdx.x, lane = t & (TILE - 1);
    // product lanes: row i of the slice, columns cl + CG_CLANES j (the
    // inverse is symmetric, so its row is read for the row of the product)
    const int i = t / CG_CLANES, cl = t % CG_CLANES, row = CG_ROWS * sl + i;
    double m[CG_CPL];
    if (t < 192) {
        const double *M = inv + (size_t)d * CG_N * CG_N + (size_t)row * CG_N + cl;
#pragma unroll
        for (int j = 0; j < CG_CPL; ++j) m[j] = M[CG_CLANES * j];
    }
    const int on = act[single ? 0 : dom_scene[d]];
    // the domain's entries from its padded list (-1 past a short domain's
    // end): no wait for the entry offsets
    int nd[CG_PASSES];
#pragma unroll
    for (int j = 0; j < CG_PASSES; ++j) nd[j] = pnodes[(size_t)d * (CG_AGG * CG_DOM) + t + j * CG_APPLY];
    // the slice's entries are those of pass jp on a contiguous range of threads
    constexpr int PER_PASS = CG_APPLY / CG_SNODES;
    const int jp = sl / PER_PASS, eo = t + jp * CG_APPLY - CG_SNODES * sl;
    const bool mine = eo >= 0 && eo < CG_SNODES;
    int ndp = -1;
#pragma unroll
    for (int j = 0; j < CG_PASSES; ++j)
        if (j == jp) ndp = mine ? nd[j] : -1;
    d3 rv[CG_PASSES], zv{0.0, 0.0, 0.0};
#pragma unroll
    for (int j = 0; j < CG_PASSES; ++j) rv[j] = nd[j] >= 0 ? ld3(r, nd[j]) : d3{0.0, 0.0, 0.0};
    if (ndp >= 0) zv = ld3(z, ndp);
    if (!on) return;   // uniform over the workgroup; nothing written yet
    // every group of the domain is one half wavefront of one pass, so each
    // rc entry is written exactly once (0 for groups past the domain's end)
#pragma unroll
    for (int j = 0; j < CG_PASSES; ++j) {
        const d3 v = cg_group_sum(rv[j]);
        const int g = (t + j * CG_APPLY) / CG_AGG;
        if ((lane & (CG_AGG - 1)) == CG_AGG - 1) { rc[3 * g] = v.x; rc[3 * g + 1] = v.y; rc[3 * g + 2] = v.z; }
    }
    __syncthreads();
    if (t < 192) {
        const double a = cg_row(m, rc, cl);
        if (cl == 0) zl[i] = a;   // rows past a short domain's end: rc and the inverse are 0 there
    }
    __syncthreads();
    if (ndp >= 0) {
        const int g = eo / CG_AGG;
        st3(z, ndp, {zv.x + zl[3 * g], zv.y + zl[3 * g + 1], zv.z + zl[3 * g + 2]});
    }
    if (t < TILE) {
        double dot = t < CG_ROWS ? rc[CG_ROWS * sl + t] * zl[t] : 0.0;
        dot = wave_sum(dot);
        if (t == 0) part[(size_t)CG_SPLIT * d + sl] = dot;
    }
}

void coarse_build(ipc_ctx *c)
{
    if (!c->n_cdom || !c->coarse_on) return;
    Dev &D = c->d;
    hipLaunchKernelGGL(k_coarse_assemble, dim3(c->n_cgrp), dim3(CG_ASM), 0, c->stream, D.cg_grp.p, D.cg_ent.p, D.cg_nodes.p,
                       D.cg_node_da.p, D.row_ptr.p, D.col.p, D.val.p, D.dyn_ptr.p, D.dyn_col.p, D.dyn_val.p, D.cg_inv.p,
                       D.cg_dom_scene.p, c->assemble_only);
    hipLaunchKernelGGL(k_coarse_invert, dim3(c->n_cdom), dim3(CG_INV), 0, c->stream, D.cg_ent.p, D.cg_inv.p, D.cg_dom_scene.p,
                       c->assemble_only);
}

void coarse_apply(ipc_ctx *c, const int *act, const double *r, double *z, int parity)
{
    if (!c->n_cdom || !c->coarse_on) return;
    Dev &D = c->d;
    const int rounds = (c->n_cdom + NXCD - 1) / NXCD;
    hipLaunchKernelGGL(k_coarse_apply, dim3(NXCD * CG_SPLIT * rounds), dim3(CG_APPLY), 0, c->stream, c->n_cdom,
                       (int)(c->n_scenes == 1), D.cg_pnodes.p, D.cg_dom_scene.p, act, D.cg_inv.p, r, z,
                       D.cg_part.p + (size_t)parity * CG_SPLIT * c->n_cdom);
}

} // namespace ipc
