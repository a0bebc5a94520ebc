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
// patch of one object.  C is block diagonal over domains of CG_DOM
// consecutive groups: each block is the domain's part of P^T A P (the sum of
// the 3x3 blocks of A between the nodes of two groups), a dense SPD matrix
// of at most 96 x 96 that is inverted after every assembly.  Nothing crosses
// scenes: groups and domains are per scene.
//
// Per PCG iteration one launch (a workgroup per domain) restricts the new
// residual to its groups, multiplies by the domain's inverse, adds the
// result to z on every node of the group and writes r . z of the correction,
// which the next step's reduction adds to r . z of the block-Jacobi part.
#include <algorithm>
#include <cstdlib>
#include <numeric>

#include "ipc_device.h"
#include "ipc_internal.h"
#include "ipc_kernels.h"

namespace ipc {

namespace {

unsigned int spread10(unsigned int v)
{
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

} // namespace

void coarse_setup(ipc_ctx *c, const std::vector<double> &X)
{
    const int ns = c->n_scenes;
    c->seg_cdom.assign(ns + 1, 0);
    std::vector<int> ent, nodes, dom_scene, node_da(c->N, -1);
    int ndom = 0;
    for (int s = 0; s < ns; ++s) {
        c->seg_cdom[s] = ndom;
        if (!c->coarse) continue;
        const SceneInfo &S = c->sc[s];
        std::vector<int> part;
        for (int i = 0; i < S.nv; ++i) part.push_back(S.node0 + i);
        for (int b = 0; b < S.nb; ++b) part.push_back(S.node0 + S.nv + 4 * b);   // translation node
        if (part.empty()) continue;
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
        for (int n : part)
            for (int k = 0; k < 3; ++k) { lo[k] = std::min(lo[k], X[3 * (size_t)n + k]); hi[k] = std::max(hi[k], X[3 * (size_t)n + k]); }
        double ext = std::max(hi[0] - lo[0], std::max(hi[1] - lo[1], hi[2] - lo[2]));
        double sc = ext > 0.0 ? 1023.0 / ext : 0.0;
        std::vector<unsigned int> key(part.size());
        for (size_t m = 0; m < part.size(); ++m) {
            unsigned int q[3];
            for (int k = 0; k < 3; ++k)
                q[k] = (unsigned int)std::min(1023.0, std::max(0.0, (X[3 * (size_t)part[m] + k] - lo[k]) * sc));
            key[m] = (spread10(q[0]) << 2) | (spread10(q[1]) << 1) | spread10(q[2]);
        }
        std::vector<size_t> ord(part.size());
        std::iota(ord.begin(), ord.end(), (size_t)0);
        std::stable_sort(ord.begin(), ord.end(), [&](size_t a, size_t b) { return key[a] < key[b]; });
        // groups of CG_AGG consecutive nodes, domains of CG_DOM consecutive
        // groups; a scene's last group and domain may be short
        const int per_dom = CG_AGG * CG_DOM;
        for (size_t m = 0; m < ord.size(); ++m) {
            if (m % per_dom == 0) {
                ent.push_back((int)nodes.size());
                dom_scene.push_back(s);
                ++ndom;
            }
            node_da[part[ord[m]]] = (ndom - 1) * CG_DOM + (int)(m % per_dom) / CG_AGG;
            nodes.push_back(part[ord[m]]);
        }
    }
    c->seg_cdom[ns] = ndom;
    ent.push_back((int)nodes.size());   // ndom + 1 offsets
    c->n_cdom = ndom;
    Dev &D = c->d;
    D.cg_ent.upload(ent, c->stream);
    D.cg_nodes.upload(nodes.empty() ? std::vector<int>(1, 0) : nodes, c->stream);
    D.cg_node_da.upload(node_da, c->stream);
    D.cg_dom_scene.upload(dom_scene.empty() ? std::vector<int>(1, 0) : dom_scene, c->stream);
    D.cg_inv.alloc((size_t)std::max(ndom, 1) * CG_N * CG_N);
    D.cg_part.alloc(2 * (size_t)std::max(ndom, 1));
}

// The domains' blocks of P^T A P, summed into cg_mat (zeroed before): one
// thread per matrix row of a grouped node adds the 3x3 blocks whose column
// node lies in a group of the same domain (block-CSR row and pair-local row).
__global__ void k_coarse_assemble(int N, const int *__restrict__ node_da, const int *__restrict__ row_ptr,
                                  const int *__restrict__ col, const double *__restrict__ val, const int *__restrict__ dptr,
                                  const int *__restrict__ dcol, const double *__restrict__ dval, double *__restrict__ mat)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int ti = node_da[i];
    if (ti < 0) return;
    const int d = ti / CG_DOM, a = ti % CG_DOM;
    double *M = mat + (size_t)d * CG_N * CG_N + 3 * a * CG_N;
    auto add = [&](int j, const double *__restrict__ B) {
        const int tj = node_da[j];
        if (tj < 0 || tj / CG_DOM != d) return;
        double *o = M + 3 * (tj % CG_DOM);
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int k = 0; k < 3; ++k) atomicAdd(&o[r * CG_N + k], B[3 * r + k]);
    };
    for (int k = row_ptr[i]; k < row_ptr[i + 1]; ++k) add(col[k], val + 9 * (size_t)k);
    for (int k = dptr[i]; k < dptr[i + 1]; ++k) add(dcol[k], dval + 9 * (size_t)k);
}

// One workgroup per domain: the inverse of its n x n block (n = 3 x groups)
// by Gauss-Jordan elimination without pivoting in LDS (the pivots of an SPD
// matrix are positive), written over the block.  A domain whose block shows
// a pivot that is not positive (the unprojected Hessian of the adjoint can
// be indefinite) gets a zero inverse: there the preconditioner is block-
// Jacobi alone.
constexpr int CG_INV = 512;
__global__ void __launch_bounds__(CG_INV) k_coarse_invert(const int *__restrict__ ent, double *__restrict__ mat)
{
    __shared__ double A[CG_N * CG_N];
    const int d = blockIdx.x, ne = ent[d + 1] - ent[d], n = 3 * ((ne + CG_AGG - 1) / CG_AGG);
    double *G = mat + (size_t)d * CG_N * CG_N;
    for (int q = threadIdx.x; q < n * n; q += CG_INV) A[(q / n) * CG_N + q % n] = G[(q / n) * CG_N + q % n];
    __syncthreads();
    bool bad = false;
    for (int k = 0; k < n; ++k) {
        const double piv = A[k * CG_N + k];
        if (!(piv > 0.0)) { bad = true; break; }   // uniform: every thread reads the same pivot
        const double ip = 1.0 / piv;
        // A[i][j] -= A[i][k] A[k][j] / piv for i, j != k (row and column k are only read)
        for (int q = threadIdx.x; q < n * n; q += CG_INV) {
            const int i = q / n, j = q % n;
            if (i != k && j != k) A[i * CG_N + j] -= A[i * CG_N + k] * A[k * CG_N + j] * ip;
        }
        __syncthreads();
        if (threadIdx.x < n && (int)threadIdx.x != k) {
            A[k * CG_N + threadIdx.x] *= ip;
            A[threadIdx.x * CG_N + k] *= -ip;
        } else if ((int)threadIdx.x == k) {
            A[k * CG_N + k] = ip;
        }
        __syncthreads();
    }
    for (int q = threadIdx.x; q < n * n; q += CG_INV) {
        const int i = q / n, j = q % n;
        G[i * CG_N + j] = bad ? 0.0 : A[i * CG_N + j];
    }
}

// One workgroup per domain of a scene that updated its residual (act != 0):
// rc = P^T r over the domain's groups, zc = C^-1 rc, z += P zc, and the
// partial rc . zc (= r . P zc) into part[d].  Every stage spreads over the
// whole workgroup: a group is 32 consecutive entries, i.e. half a wavefront
// of one pass over the entries.
constexpr int CG_APPLY = 256;
constexpr int CG_PASSES = CG_AGG * CG_DOM / CG_APPLY;
__global__ void __launch_bounds__(CG_APPLY) k_coarse_apply(const int *__restrict__ ent, const int *__restrict__ nodes,
                                                           const int *__restrict__ dom_scene, const int *__restrict__ act,
                                                           const double *__restrict__ inv, const double *__restrict__ r,
                                                           double *__restrict__ z, double *__restrict__ part)
{
    static_assert(CG_APPLY == 4 * TILE && CG_N == 96, "four wavefronts of 24 columns");
    __shared__ double rc[CG_N], zc[CG_N], zp[CG_APPLY / TILE][CG_N], sh[CG_APPLY / TILE];
    const int d = blockIdx.x;
    if (!act[dom_scene[d]]) return;   // uniform over the workgroup
    const int e0 = ent[d], ne = ent[d + 1] - e0, n = 3 * ((ne + CG_AGG - 1) / CG_AGG);
    const int t = threadIdx.x, lane = t & (TILE - 1), wave = t / TILE;
    // restriction: all entries' residuals in flight at once
    int nd[CG_PASSES];
    d3 rv[CG_PASSES];
#pragma unroll
    for (int j = 0; j < CG_PASSES; ++j) {
        const int e = t + j * CG_APPLY;
        nd[j] = e < ne ? nodes[e0 + e] : -1;
    }
#pragma unroll
    for (int j = 0; j < CG_PASSES; ++j) rv[j] = nd[j] >= 0 ? ld3(r, nd[j]) : d3{0.0, 0.0, 0.0};
#pragma unroll
    for (int j = 0; j < CG_PASSES; ++j) {
        double x = rv[j].x, y = rv[j].y, zz = rv[j].z;
#pragma unroll
        for (int o = CG_AGG / 2; o > 0; o >>= 1) {
            x += __shfl_xor(x, o, TILE);
            y += __shfl_xor(y, o, TILE);
            zz += __shfl_xor(zz, o, TILE);
        }
        const int g = (t + j * CG_APPLY) / CG_AGG;   // group of this half wavefront
        if ((lane & (CG_AGG - 1)) == 0 && 3 * g < n) { rc[3 * g] = x; rc[3 * g + 1] = y; rc[3 * g + 2] = zz; }
    }
    __syncthreads();
    // zc = C^-1 rc: wavefront w sums the columns k in [KW w, KW w + KW) for
    // the rows i = lane and lane + 64; all its loads are issued before the
    // sums (the inverse is symmetric: row k is column k, read coalesced)
    {
        constexpr int KW = CG_N / (CG_APPLY / TILE);   // 24 columns per wavefront
        const double *M = inv + (size_t)d * CG_N * CG_N;
        const int i0 = lane, i1 = lane + TILE;
        double m0[KW], m1[KW];
#pragma unroll
        for (int j = 0; j < KW; ++j) {
            const int k = wave * KW + j;
            m0[j] = (k < n && i0 < n) ? M[(size_t)k * CG_N + i0] : 0.0;
            m1[j] = (k < n && i1 < n) ? M[(size_t)k * CG_N + i1] : 0.0;
        }
        double a0 = 0.0, a1 = 0.0;
#pragma unroll
        for (int j = 0; j < KW; ++j) {
            const int k = wave * KW + j;
            const double rk = k < n ? rc[k] : 0.0;
            a0 += m0[j] * rk;
            a1 += m1[j] * rk;
        }
        zp[wave][i0] = a0;
        if (i1 < CG_N) zp[wave][i1] = a1;
    }
    __syncthreads();
    if (t < n) zc[t] = (zp[0][t] + zp[1][t]) + (zp[2][t] + zp[3][t]);
    __syncthreads();
    double dot = t < n ? rc[t] * zc[t] : 0.0;
    dot = wave_sum(dot);
    if (lane == 0) sh[wave] = dot;
    // prolongation
#pragma unroll
    for (int j = 0; j < CG_PASSES; ++j) {
        if (nd[j] < 0) continue;
        const int g = (t + j * CG_APPLY) / CG_AGG;
        d3 zv = ld3(z, nd[j]);
        st3(z, nd[j], {zv.x + zc[3 * g], zv.y + zc[3 * g + 1], zv.z + zc[3 * g + 2]});
    }
    __syncthreads();
    if (t == 0) {
        double s2 = 0.0;
        for (int w = 0; w < CG_APPLY / TILE; ++w) s2 += sh[w];
        part[d] = s2;
    }
}

void coarse_build(ipc_ctx *c)
{
    if (!c->n_cdom) return;
    Dev &D = c->d;
    D.cg_inv.zero(c->stream, (size_t)c->n_cdom * CG_N * CG_N);
    hipLaunchKernelGGL(k_coarse_assemble, dim3(blocks_for(c->N)), dim3(BLOCK), 0, c->stream, c->N, D.cg_node_da.p, D.row_ptr.p,
                       D.col.p, D.val.p, D.dyn_ptr.p, D.dyn_col.p, D.dyn_val.p, D.cg_inv.p);
    hipLaunchKernelGGL(k_coarse_invert, dim3(c->n_cdom), dim3(CG_INV), 0, c->stream, D.cg_ent.p, D.cg_inv.p);
}

void coarse_apply(ipc_ctx *c, const int *act, const double *r, double *z, int parity)
{
    if (!c->n_cdom) return;
    Dev &D = c->d;
    hipLaunchKernelGGL(k_coarse_apply, dim3(c->n_cdom), dim3(CG_APPLY), 0, c->stream, D.cg_ent.p, D.cg_nodes.p, D.cg_dom_scene.p,
                       act, D.cg_inv.p, r, z, D.cg_part.p + (size_t)parity * c->n_cdom);
}

} // namespace ipc
