// Kernel launch wrappers shared between the translation units.
#pragma once
#include "ipc_internal.h"

namespace ipc {

// Cross-lane moves through DPP (a VALU operand modifier, no LDS round trip).
// A double moves as its two 32-bit halves; lanes whose row is not in ROWS
// (or whose source lane does not exist) receive 0.  Callers keep the whole
// wavefront active.
enum DppCtrl {
    DPP_XOR1 = 0xB1,         // quad_perm [1,0,3,2]: lane ^ 1
    DPP_XOR2 = 0x4E,         // quad_perm [2,3,0,1]: lane ^ 2
    DPP_HALF_MIRROR = 0x141, // lane 7 - i within each 8
    DPP_MIRROR = 0x140,      // lane 15 - i within each 16
    DPP_BCAST15 = 0x142,     // lane 15 of the previous row of 16
    DPP_BCAST31 = 0x143,     // lane 31, into rows 2 and 3
};
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ double dpp_d(double v)
{
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u & 0xffffffffull), CTRL, ROWS, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, ROWS, 0xf, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
// sum over each aligned group of 8 lanes, in every lane of the group
__device__ __forceinline__ double sum8(double v)
{
    v += dpp_d<DPP_XOR1>(v);
    v += dpp_d<DPP_XOR2>(v);
    return v + dpp_d<DPP_HALF_MIRROR>(v);
}
// sum over each aligned group of L lanes (L = 1, 2, 4, 8 or 16), in every
// lane of the group
template <int L>
__device__ __forceinline__ double lane_sum(double v)
{
    static_assert(L == 1 || L == 2 || L == 4 || L == 8 || L == 16, "groups of 1 to 16 lanes");
    if (L >= 2) v += dpp_d<DPP_XOR1>(v);
    if (L >= 4) v += dpp_d<DPP_XOR2>(v);
    if (L >= 8) v += dpp_d<DPP_HALF_MIRROR>(v);
    if (L >= 16) v += dpp_d<DPP_MIRROR>(v);
    return v;
}
// sum over each aligned group of 16 lanes, in every lane of the group
__device__ __forceinline__ double sum16(double v) { v = sum8(v); return v + dpp_d<DPP_MIRROR>(v); }
// sum over each aligned group of 32 lanes, in its upper 16 lanes (lanes
// 16-31 and 48-63; the lower 16 keep their 16-lane sums)
__device__ __forceinline__ double sum32_hi(double v) { v = sum16(v); return v + dpp_d<DPP_BCAST15, 0xA>(v); }
// sum over the wavefront, in every lane (the same order in every call)
__device__ __forceinline__ double wave_sum(double v)
{
    v = sum32_hi(v);
    v += dpp_d<DPP_BCAST31, 0xC>(v);
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u & 0xffffffffull), 63);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), 63);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// elastic terms (ipc_elastic.hip)
void launch_node_inertia(ipc_ctx *c, const double *y, double *g, double *part);
void autotune_fem(ipc_ctx *c, int reps);
void launch_fem(ipc_ctx *c, int mode, const double *y, double *g, bool project, double *part, const double *h2s);
void launch_body(ipc_ctx *c, int mode, const double *y, double *g, bool project, double *part, const double *h2s);
void launch_spring(ipc_ctx *c, int mode, const double *y, double *g, double *part, const double *h2s);

// contact (ipc_contact.hip)
void launch_world(ipc_ctx *c, const double *y, double *xw);
// candidates from the LBVH over boxes at xw0 (and xw1 when swept)
void broad_phase(ipc_ctx *c, const double *xw0, const double *xw1, double grow = 0.0);
// swept candidates kept across Newton iterations (see ipc_contact.hip) and
// the per-scene test (flag 1: rebuild) of whether they still cover [xw0, xw1]
void broad_phase_cached(ipc_ctx *c, const double *xw0, const double *xw1);
void cand_check(ipc_ctx *c, const double *xw0, const double *xw1, int *flag);
// narrow phase: active pairs from the candidate lists at xw
void narrow_phase(ipc_ctx *c, const double *xw);
// barrier (mode 0 energy, 1 + gradient, 2 + Hessian blocks) and friction:
// gradients are summed per contact vertex into D.gcv, between
// contact_grad_begin (zeroes it) and contact_grad_end (adds it into g)
void launch_barrier(ipc_ctx *c, int mode, bool candidates, const double *xw, bool project);
// the lag at world positions xw; slips measured from xref (nullptr: xw)
void launch_lag(ipc_ctx *c, const double *xw, const double *xref = nullptr);
void launch_friction(ipc_ctx *c, int mode, const double *xw);
void contact_grad_begin(ipc_ctx *c);
void contact_grad_end(ipc_ctx *c, double *g);
// stable sort of m (key, code) pairs by the low end_bit bits of the key, and
// the bits that hold every value in [0, n]
void sort_entries(ipc_ctx *c, const int *key, int *key2, const int *code, int *code2, int64_t m, int end_bit);
size_t sort_entries_bytes(ipc_ctx *c, int64_t m, int end_bit);
int bits_for(int64_t n);
// pair-local contact blocks as row-sorted extra blocks of the product, and the
// rows the product takes one wavefront per row
void build_dyn_blocks(ipc_ctx *c);
void launch_ccd(ipc_ctx *c, const double *xw0, const double *xw1);
void launch_kappa_update(ipc_ctx *c, const double *xw, bool first);
// half-space ground
void hs_setup(ipc_ctx *c);
void launch_hs(ipc_ctx *c, int mode, const double *xw);
void launch_hs_lag(ipc_ctx *c, const double *xw, const double *xref);
void launch_hs_ccd(ipc_ctx *c, const double *xw0, const double *xw1);
void launch_hs_dmin(ipc_ctx *c, const double *xw);
void launch_hs_lag_vjp(ipc_ctx *c, const double *xw, const double *xwn, const double *w);

// adjoint of the friction lag: ybar -= (dG_F/dy^n)^T w; per-pair w . dG/dmu into fr_part
void launch_lag_vjp(ipc_ctx *c, const double *xw, const double *xwn, const double *w, double *ybar);

// adjoint of one step (ipc_adjoint.hip)
void launch_set_E(ipc_ctx *c, const double *E_ext);
void launch_adj_rhs(ipc_ctx *c, const double *ybar_next, const double *vbar_next, double *rhs);
void launch_adj_mass(ipc_ctx *c, const double *w, const double *vbar_next, double *ybar_prev, double *vbar_prev);
void launch_adj_E(ipc_ctx *c, const double *y, const double *w, double *Ebar_ext);


} // namespace ipc
