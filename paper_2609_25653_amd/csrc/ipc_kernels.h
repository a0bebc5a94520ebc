// Kernel launch wrappers shared between the translation units.
#pragma once
#include "ipc_internal.h"

namespace ipc {

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// elastic terms (ipc_elastic.hip)
void launch_node_inertia(ipc_ctx *c, const double *y, double *g, double *part);
void launch_fem(ipc_ctx *c, int mode, const double *y, double *g, bool project, double *part, const double *h2s);
void launch_bsr_init(ipc_ctx *c);
void launch_body(ipc_ctx *c, int mode, const double *y, double *g, bool project, double *part, const double *h2s);
void launch_spring(ipc_ctx *c, int mode, const double *y, double *g, double *part, const double *h2s);

// contact (ipc_contact.hip)
void launch_world(ipc_ctx *c, const double *y, double *xw);
// candidates from the LBVH over boxes at xw0 (and xw1 when swept)
void broad_phase(ipc_ctx *c, const double *xw0, const double *xw1);
// narrow phase: active pairs from the candidate lists at xw
void narrow_phase(ipc_ctx *c, const double *xw);
void launch_barrier(ipc_ctx *c, int mode, bool candidates, const double *xw, double *g, bool project);
void launch_lag(ipc_ctx *c, const double *xw);
void launch_friction(ipc_ctx *c, int mode, const double *xw, double *g);
void launch_contact_apply(ipc_ctx *c, const double *v, double *out, const int *active, double *part_b, double *part_f);
void build_local_list(ipc_ctx *c);
void launch_ccd(ipc_ctx *c, const double *xw0, const double *xw1);

// per-scene scalars (ipc_solver.hip)
const double *scene_h2(ipc_ctx *c);
const double *scene_param(ipc_ctx *c, int which);   // 0 kappa, 1 dhat, 2 mu, 3 eps_v*h, 4 ccd_s
void seg_sum(ipc_ctx *c, const double *vals, const int *seg_dev, int slot, bool accumulate);
void node_seg_sum(ipc_ctx *c, const double *part, int slot, bool accumulate);
void tet_seg_sum(ipc_ctx *c, const double *part, int slot, bool accumulate);
int *upload_seg(ipc_ctx *c, const std::vector<int> &seg, int which);

} // namespace ipc
