// Device arithmetic shared by the PCG step and the coarse correction.  The
// one-launch step (the update and the coarse correction of a domain in one
// kernel) must produce the same bits as the step followed by the apply
// kernel, so each piece of arithmetic they have in common is written once,
// here: the update of s and r, a body's block-Jacobi rows, the restriction's
// group sums and a row of the product with a domain's inverse.
#pragma once
#include <hip/hip_runtime.h>

#include "ipc_device.h"
#include "ipc_internal.h"
#include "ipc_kernels.h"

namespace ipc {

constexpr int CG_APPLY = 256;                          // threads per apply workgroup (and per step workgroup)
constexpr int CG_PASSES = CG_AGG * CG_DOM / CG_APPLY;  // passes over a domain's entries
constexpr int CG_ROWS = CG_N / CG_SPLIT;               // inverse rows per slice
constexpr int CG_SNODES = CG_AGG * CG_DOM / CG_SPLIT;  // entries per slice
constexpr int CG_CLANES = 192 / CG_ROWS;               // lanes per row in the product
constexpr int CG_CPL = CG_N / CG_CLANES;               // columns per lane
constexpr int NXCD = 8;                                // XCDs; workgroups go round-robin over them
static_assert(CG_N % CG_SPLIT == 0 && CG_ROWS * CG_CLANES == 192 && CG_N % CG_CLANES == 0, "whole rows and columns per lane");
static_assert(TILE % CG_CLANES == 0 && CG_SNODES <= CG_APPLY && CG_APPLY % CG_SNODES == 0, "lane groups inside a wavefront");
static_assert(CG_SNODES == CG_APPLY && CG_APPLY == BLOCK, "a slice is one step workgroup's nodes");

// s <- w + beta s, r <- r - alpha s (the PCG's update of s = A p and r)
__device__ __forceinline__ void pcg_sr(d3 w, double al, double be, d3 &s, d3 &r)
{
    s = {w.x + be * s.x, w.y + be * s.y, w.z + be * s.z};
    r = {r.x - al * s.x, r.y - al * s.y, r.z - al * s.z};
}

// three rows of a body's 12x12 inverse block (row-major, 12 apart) times the
// body's 12 residual entries
__device__ __forceinline__ d3 body_rows(const double *__restrict__ M, const double (&rb)[12])
{
    double zz[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < 12; ++j) acc += M[12 * c + j] * rb[j];
        zz[c] = acc;
    }
    return {zz[0], zz[1], zz[2]};
}

// sum over the CG_AGG lanes of a group (aligned lanes of one wavefront),
// held by the group's last lane (lane & (CG_AGG - 1)) == CG_AGG - 1
static_assert(CG_AGG == 32 && CG_CLANES == 8, "the DPP sums below are for groups of 32 and rows of 8 lanes");
__device__ __forceinline__ d3 cg_group_sum(d3 v) { return {sum32_hi(v.x), sum32_hi(v.y), sum32_hi(v.z)}; }

// one row of the product with a domain's inverse: this lane's CG_CPL columns
// cl + CG_CLANES j, then the sum over the row's CG_CLANES lanes (in each)
__device__ __forceinline__ double cg_row(const double (&m)[CG_CPL], const double *rc, int cl)
{
    double a = 0.0;
#pragma unroll
    for (int j = 0; j < CG_CPL; ++j) a += m[j] * rc[cl + CG_CLANES * j];
    return sum8(a);
}

} // namespace ipc
