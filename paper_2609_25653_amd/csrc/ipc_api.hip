// C-ABI entry points and the host orchestration of the Newton step
// (PhyVisGen Sec. III-C.2: all degrees of freedom advanced jointly by
// minimising one incremental potential per step, Eq. (3)).
//
// Stream-ordered on the context's stream.  Host synchronisation happens only
// at control decisions: PCG convergence (every few iterations), candidate and
// pair counts (to size buffers), the Newton measure and line-search energies.
#include <algorithm>
#include <array>
#include <climits>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <cstdio>
#include <map>
#include <mutex>

#include "ipc_device.h"
#include "ipc_internal.h"
#include "ipc_kernels.h"

namespace ipc {

namespace {

thread_local std::string g_create_error;

// ---- node-vector kernels -----------------------------------------------------
__global__ void k_to_internal(int64_t NE, const int *__restrict__ ext2node, const double *__restrict__ ext, double *__restrict__ v)
{
    int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= NE) return;
    int n = ext2node[e];
    v[3 * (size_t)n] = ext[3 * e]; v[3 * (size_t)n + 1] = ext[3 * e + 1]; v[3 * (size_t)n + 2] = ext[3 * e + 2];
}
__global__ void k_to_external(int64_t NE, const int *__restrict__ ext2node, const double *__restrict__ v, double *__restrict__ ext)
{
    int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= NE) return;
    int n = ext2node[e];
    ext[3 * e] = v[3 * (size_t)n]; ext[3 * e + 1] = v[3 * (size_t)n + 1]; ext[3 * e + 2] = v[3 * (size_t)n + 2];
}
__global__ void k_zero(int64_t n, double *p)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}
// x~ = y + h ydot + h^2 g on FEM nodes and body translation nodes; y + h ydot on A nodes
__global__ void k_predict(int N, const int *__restrict__ kind, const int *__restrict__ node_scene, const int *__restrict__ is_trans,
                          const double *__restrict__ sparam, const double *__restrict__ grav, const double *__restrict__ y,
                          const double *__restrict__ yd, double *__restrict__ xt)
{
    int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    int s = node_scene[n];
    double h = sparam[8 * s + P_H];
    bool gv = kind[n] == 0 || (kind[n] == 1 && is_trans[n]);
    for (int k = 0; k < 3; ++k) {
        double v = y[3 * (size_t)n + k] + h * yd[3 * (size_t)n + k];
        if (gv) v += h * h * grav[3 * s + k];
        xt[3 * (size_t)n + k] = v;
    }
}
__global__ void k_negate(int64_t n, const double *__restrict__ a, double *__restrict__ b)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) b[i] = -a[i];
}
// joint slot j: the b-side body-frame point of spring joint_sp[j]
__global__ void k_joint_points(int nj, const double *__restrict__ pts, const int *__restrict__ joint_sp, double *__restrict__ sp_xb)
{
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nj) return;
    for (int k = 0; k < 3; ++k) sp_xb[3 * (size_t)joint_sp[j] + k] = pts[3 * (size_t)j + k];
}
// line search set-up: the scene takes part when on[s]; step 1; CCD bound 1
__global__ void k_ls_begin(int ns, const int *__restrict__ on, double *__restrict__ scal)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= ns) return;
    double *S = scal + (size_t)s * NSLOT;
    S[S_LS_ON] = on[s] ? 1.0 : 0.0;
    S[S_LS_ALPHA] = 1.0;
    S[S_CCD] = 1.0;
}
// the first line-search trial of each scene still iterating: min(1, CCD bound)
__global__ void k_ls_first(int ns, double *__restrict__ scal)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= ns) return;
    double *S = scal + (size_t)s * NSLOT;
    const double a = S[S_CCD];
    S[S_LS_ALPHA] = S[S_LS_ON] != 0.0 ? (a < 1.0 ? a : 1.0) : 0.0;
}
__global__ void k_copy_slot(int ns, double *__restrict__ scal, int from, int to)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < ns) scal[(size_t)s * NSLOT + to] = scal[(size_t)s * NSLOT + from];
}
// yt = y + alpha_s p (alpha from the scene's line-search slot, 0 when off)
__global__ void k_trial(int N, const int *__restrict__ node_scene, const double *__restrict__ scal, const double *__restrict__ y,
                        const double *__restrict__ p, double *__restrict__ yt)
{
    int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    int s = node_scene[n];
    const double *S = scal + (size_t)s * NSLOT;
    double a = S[S_LS_ON] != 0.0 ? S[S_LS_ALPHA] : 0.0;
    for (int k = 0; k < 3; ++k) yt[3 * (size_t)n + k] = y[3 * (size_t)n + k] + a * p[3 * (size_t)n + k];
}
__global__ void k_velocity(int N, const int *__restrict__ node_scene, const double *__restrict__ sparam, const double *__restrict__ y,
                           const double *__restrict__ y0, double *__restrict__ yd)
{
    int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    double h = sparam[8 * node_scene[n] + P_H];
    for (int k = 0; k < 3; ++k) yd[3 * (size_t)n + k] = (y[3 * (size_t)n + k] - y0[3 * (size_t)n + k]) / h;
}
// Newton measure: largest world displacement of p (FEM DOFs; bodies through
// their box corners), one partial max per wavefront / per body
__global__ void k_measure_nodes(int N, const int *__restrict__ kind, const double *__restrict__ p, double *__restrict__ part)
{
    int n = blockIdx.x * blockDim.x + threadIdx.x;
    double m = 0.0;
    if (n < N && kind[n] == 0) m = fmax(fabs(p[3 * (size_t)n]), fmax(fabs(p[3 * (size_t)n + 1]), fabs(p[3 * (size_t)n + 2])));
    m = wave_max(m);
    if ((threadIdx.x & (TILE - 1)) == 0 && n < N) part[n / TILE] = m;
}
__global__ void k_measure_bodies(int NB, const int *__restrict__ node0, const double *__restrict__ ext, const double *__restrict__ p,
                                 double *__restrict__ part)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= NB) return;
    const double *q = p + 3 * (size_t)node0[b], *e = ext + 3 * (size_t)b;
    double m = 0.0;
    for (int k = 0; k < 3; ++k) m = fmax(m, fabs(q[k]) + e[0] * fabs(q[3 + k]) + e[1] * fabs(q[6 + k]) + e[2] * fabs(q[9 + k]));
    part[b] = m;
}
__global__ void k_set_slot(int ns, double *scal, int slot, double v)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < ns) scal[(size_t)s * NSLOT + slot] = v;
}
__global__ void k_gather_slot(int ns, const double *scal, int slot, double *out)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < ns) out[s] = scal[(size_t)s * NSLOT + slot];
}
__global__ void k_copy_int(int n, const int *a, int *b)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}
__global__ void k_sub_slot(int ns, const double *scal, int slot, double *out)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < ns) out[s] -= scal[(size_t)s * NSLOT + slot];
}
__global__ void k_inf_to_scal(int ns, int *flag, double *scal)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= ns) return;
    scal[(size_t)s * NSLOT + S_INF] = flag[s] ? 1.0 : 0.0;
    if (flag[s]) scal[(size_t)s * NSLOT + S_E] = INFINITY;
}

// ---- host helpers --------------------------------------------------------------
void sync(ipc_ctx *c) { IPC_HIP(hipStreamSynchronize(c->stream)); }

std::vector<double> read_scal(ipc_ctx *c)
{
    std::vector<double> h((size_t)c->n_scenes * NSLOT);
    HostReads r(c);
    r.add(h.data(), c->d.scal.p, h.size() * sizeof(double));
    r.wait();
    return h;
}

void write_scal(ipc_ctx *c, const std::vector<double> &h) { upload_async(c, c->d.scal.p, h.data(), h.size() * sizeof(double)); }

void upload_seg_region(ipc_ctx *c, int region, const std::vector<int> &h)
{
    c->h_seg_stage = h;
    IPC_HIP(hipMemcpyAsync(seg_ptr(c, region), c->h_seg_stage.data(), h.size() * sizeof(int), hipMemcpyHostToDevice, c->stream));
    sync(c);
}

// per-scene parameters (8 per scene) from the host scene records
void upload_sparam(ipc_ctx *c)
{
    int ns = c->n_scenes;
    std::vector<double> &sp = c->h_scal_stage;
    sp.assign(8 * (size_t)ns, 0.0);
    for (int s = 0; s < ns; ++s) {
        SceneInfo &S = c->sc[s];
        sp[8 * s + P_H2] = S.h * S.h; sp[8 * s + P_KAPPA] = S.kappa; sp[8 * s + P_DHAT] = S.dhat; sp[8 * s + P_MU] = S.mu;
        sp[8 * s + P_EPSH] = S.eps_v * S.h; sp[8 * s + P_CCDS] = S.ccd_s; sp[8 * s + P_H] = S.h;
        sp[8 * s + P_ETA] = S.pcg_tol;
    }
    c->d.sparam.upload(sp, c->stream);
    sync(c);
}

void setup_after_create(ipc_ctx *c)
{
    Dev &D = c->d;
    int ns = c->n_scenes;
    std::vector<double> h2(ns), grav(3 * (size_t)ns), lo(6 * (size_t)ns);
    std::vector<int> maxpcg(ns);
    for (int s = 0; s < ns; ++s) {
        SceneInfo &S = c->sc[s];
        h2[s] = S.h * S.h;
        for (int k = 0; k < 3; ++k) grav[3 * s + k] = S.g[k];
        maxpcg[s] = S.max_pcg;
    }
    upload_sparam(c);
    D.h2s.upload(h2, c->stream); D.grav.upload(grav, c->stream); D.maxpcg.upload(maxpcg, c->stream);
    // Morton boxes: initial world bounds of each scene's moving contact
    // vertices (FEM and body surfaces; all of them if there are none),
    // enlarged.  Static geometry is left out: a large ground would otherwise
    // set the quantisation and crowd the moving primitives into few codes
    // (its primitives get codes clamped to the box, which any tree allows).
    {
        launch_world(c, D.y.p, D.xw.p);
        std::vector<double> xw(3 * (size_t)c->CV);
        std::vector<int> cvn(c->CV), cvb(c->CV);
        if (c->CV) {
            IPC_HIP(hipMemcpyAsync(xw.data(), D.xw.p, xw.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
            IPC_HIP(hipMemcpyAsync(cvn.data(), D.cv_node.p, cvn.size() * sizeof(int), hipMemcpyDeviceToHost, c->stream));
            IPC_HIP(hipMemcpyAsync(cvb.data(), D.cv_body.p, cvb.size() * sizeof(int), hipMemcpyDeviceToHost, c->stream));
        }
        sync(c);
        for (int s = 0; s < ns; ++s) {
            SceneInfo &S = c->sc[s];
            double l[3] = {INFINITY, INFINITY, INFINITY}, h[3] = {-INFINITY, -INFINITY, -INFINITY};
            bool any_moving = false;
            for (int i = S.cv0; i < S.cv0 + S.ncv; ++i) any_moving = any_moving || cvn[i] >= 0 || cvb[i] >= 0;
            for (int i = S.cv0; i < S.cv0 + S.ncv; ++i) {
                if (any_moving && cvn[i] < 0 && cvb[i] < 0) continue;
                for (int k = 0; k < 3; ++k) { l[k] = std::min(l[k], xw[3 * i + k]); h[k] = std::max(h[k], xw[3 * i + k]); }
            }
            for (int k = 0; k < 3; ++k) {
                if (!(h[k] >= l[k])) { l[k] = 0.0; h[k] = 1.0; }
                double ext = std::max(h[k] - l[k], 1e-3), m = 0.25 * ext;
                lo[6 * s + k] = l[k] - m;
                lo[6 * s + 3 + k] = 1023.0 / (ext + 2.0 * m);
            }
        }
        D.scene_lo.upload(lo, c->stream);
    }
    std::vector<int> is_trans(c->N, 0), node_body(c->N, -1);
    for (int s = 0; s < ns; ++s) {
        SceneInfo &S = c->sc[s];
        for (int b = 0; b < S.nb; ++b) {
            is_trans[S.bnode0 + 4 * b] = 1;
            node_body[S.bnode0 + 4 * b] = S.body0 + b;
        }
    }
    D.is_trans.upload(is_trans, c->stream);
    D.node_body.upload(node_body, c->stream);
    for (auto *b : {&D.inf_flag, &D.ls_active, &D.pcg_iters, &D.newton_on}) b->alloc(ns);
    D.tickets.alloc(4);
    D.tickets.zero(c->stream, 4);
    D.segs.alloc((size_t)NREGION * (ns + 1));
    D.segs.zero(c->stream, (size_t)NREGION * (ns + 1));
    std::vector<int> nodew(ns + 1), tetw(ns + 1);
    for (int s = 0; s < ns; ++s) { nodew[s] = c->sc[s].node0 / TILE; tetw[s] = c->sc[s].tet0 / TILE; }
    nodew[ns] = c->N / TILE; tetw[ns] = c->T / TILE;
    upload_seg_region(c, R_NODEW, nodew);
    upload_seg_region(c, R_TETW, tetw);
    upload_seg_region(c, R_BODY, c->seg_body);
    upload_seg_region(c, R_SP, c->seg_sp);
    upload_seg_region(c, R_SURF, c->seg_surf);
    upload_seg_region(c, R_TRI, c->seg_tri);
    upload_seg_region(c, R_EDGE, c->seg_edge);
    upload_seg_region(c, R_CDOM, c->seg_cdom);
    upload_seg_region(c, R_HS, c->seg_hs);
    build_dyn_blocks(c);   // no pairs yet: row pointers and the long rows of the static pattern
    sync(c);
}

// ---- potential evaluation --------------------------------------------------------
// Energy per scene into S_E (and the per-term slots).  The barrier runs over
// the candidate lists (from_candidates) or over the active pairs.
void eval_energy(ipc_ctx *c, const double *y, bool from_candidates)
{
    Dev &D = c->d;
    hipStream_t st = c->stream;
    launch_world(c, y, D.xw.p);
    hipLaunchKernelGGL(k_fill_int_api, dim3(blocks_for(c->n_scenes)), dim3(BLOCK), 0, st, c->n_scenes, D.inf_flag.p, 0);
    launch_node_inertia(c, y, nullptr, D.part_node.p);
    launch_fem(c, 0, y, nullptr, false, D.part_tet.p, D.h2s.p);
    launch_body(c, 0, y, nullptr, false, D.body_part.p, D.h2s.p);
    launch_spring(c, 0, y, nullptr, D.sp_part.p, D.h2s.p);
    launch_barrier(c, 0, from_candidates, D.xw.p, false);
    if (c->fr_on) launch_friction(c, 0, D.xw.p);
    launch_hs(c, 0, D.xw.p);
    int64_t npt = from_candidates ? c->n_cand_pt : c->n_pt, nee = from_candidates ? c->n_cand_ee : c->n_ee;
    // the per-pair values are pre-summed in chunks of 64, so that a scene's
    // reduction reads its chunk sums and at most 126 single entries
    int64_t nlag = c->fr_on ? c->n_lag : 0;
    D.pair_w64.alloc((npt + nee) / TILE + 1);
    D.fr_w64.alloc(nlag / TILE + 1);
    sum64(c, D.pair_part.p, npt + nee, D.pair_w64.p);
    sum64(c, D.fr_part.p, nlag, D.fr_w64.p);
    // one pass: every term in its slot, the barrier (group 1) and friction
    // (group 2) totals, and the energy as the sum of all sources in order
    RedArgs a{};
    auto add = [&](RedSrc r, int slot, int grp) { a.src[a.nsrc] = r; a.slots[a.nsrc] = slot; a.grp[a.nsrc++] = grp; };
    add(src(D.part_node.p, seg_ptr(c, R_NODEW), 0, 0), S_E_IN, -1);
    add(src(c->T ? D.part_tet.p : nullptr, seg_ptr(c, R_TETW), 0, 0), S_E_FEM, -1);
    add(src(c->NB ? D.body_part.p : nullptr, seg_ptr(c, R_BODY), 0, 0), S_E_ABD, -1);
    add(src(c->NS ? D.sp_part.p : nullptr, seg_ptr(c, R_SP), 0, 0), S_E_SP, -1);
    RedSrc bp = src(npt ? D.pair_part.p : nullptr, seg_ptr(c, from_candidates ? R_CPT : R_PT), 0, 0);
    RedSrc be = src(nee ? D.pair_part.p : nullptr, seg_ptr(c, from_candidates ? R_CEE : R_EE), (int)npt, 0);
    bp.w64 = be.w64 = D.pair_w64.p;
    add(bp, -1, 1);
    add(be, -1, 1);
    RedSrc fp = src(c->fr_on && c->n_lag_pt ? D.fr_part.p : nullptr, seg_ptr(c, R_LPT), 0, 0);
    RedSrc fe = src(c->fr_on && c->n_lag - c->n_lag_pt ? D.fr_part.p : nullptr, seg_ptr(c, R_LEE), (int)c->n_lag_pt, 0);
    fp.w64 = fe.w64 = D.fr_w64.p;
    add(fp, -1, 2);
    add(fe, -1, 2);
    if (c->M_HS) {   // the half-space's barrier and friction
        RedSrc hb = src(D.hs_part.p, seg_ptr(c, R_HS), 0, 0), hf = src(c->fr_on ? D.hs_fpart.p : nullptr, seg_ptr(c, R_HS), 0, 0);
        hb.w64 = D.hs_w64.p;
        hf.w64 = D.hs_fw64.p;
        add(hb, -1, 1);
        add(hf, -1, 2);
    }
    a.slot1 = S_E_BAR;
    a.slot2 = S_E_FR;
    a.total = S_E;
    reduce(c, a);
    hipLaunchKernelGGL(k_inf_to_scal, dim3(blocks_for(c->n_scenes, 64)), dim3(64), 0, st, c->n_scenes, D.inf_flag.p, D.scal.p);
}

// Gradient into g (internal layout) and, with hess, the projected (or not)
// Hessian: FEM block-CSR values, body blocks, contact blocks, friction blocks
// and the diagonal accumulators of the preconditioner.  Pairs must be current.
void eval_grad_hess(ipc_ctx *c, const double *y, double *g, bool hess, bool project)
{
    Dev &D = c->d;
    hipStream_t st = c->stream;
    launch_world(c, y, D.xw.p);
    hipLaunchKernelGGL(k_fill_int_api, dim3(blocks_for(c->n_scenes)), dim3(BLOCK), 0, st, c->n_scenes, D.inf_flag.p, 0);
    // inertia writes g; the FEM gathers then write the matrix values (constant
    // part + tets) and add the tets' gradients; the bodies add their own
    // nodes; springs, barrier and friction pairs add through sorted run sums
    // (one writer per destination, in an order fixed by the inputs), so the
    // gradient and the matrix are the same bit for bit on every run
    launch_node_inertia(c, y, g, D.part_node.p);
    launch_fem(c, hess ? 2 : 1, y, g, project, D.part_tet.p, D.h2s.p);
    launch_body(c, hess ? 2 : 1, y, g, project, D.body_part.p, D.h2s.p);
    launch_spring(c, 1, y, g, D.sp_part.p, D.h2s.p);
    contact_grad_begin(c);
    launch_barrier(c, hess ? 2 : 1, false, D.xw.p, project);
    if (c->fr_on) launch_friction(c, hess ? 2 : 1, D.xw.p);
    launch_hs(c, hess ? 2 : 1, D.xw.p);
    contact_grad_end(c, g);
    if (hess) build_dyn_blocks(c);
}

// Active pairs at internal y from a static broad phase.
void pairs_from_scratch(ipc_ctx *c, const double *y)
{
    launch_world(c, y, c->d.xw.p);
    broad_phase(c, c->d.xw.p, nullptr);
    narrow_phase(c, c->d.xw.p);
}

void begin_step_impl(ipc_ctx *c, const double *targets_dev)
{
    Dev &D = c->d;
    hipStream_t st = c->stream;
    if (targets_dev && c->ND)
        IPC_HIP(hipMemcpyAsync(D.targets.p, targets_dev, 12 * (size_t)c->ND * sizeof(double), hipMemcpyDeviceToDevice, st));
    if (targets_dev && c->NJ) {
        // joint references: the b-side body-frame point of every joint
        // spring, then the constant matrix part for the new points
        hipLaunchKernelGGL(k_joint_points, dim3(blocks_for(c->NJ)), dim3(BLOCK), 0, st, c->NJ, targets_dev + 12 * (size_t)c->ND,
                           D.joint_sp.p, D.sp_xb.p);
        build_const_part(c, D.h2s.p);
    }
    hipLaunchKernelGGL(k_predict, dim3(blocks_for(c->N)), dim3(BLOCK), 0, st, c->N, D.node_kind.p, D.node_scene.p, D.is_trans.p,
                       D.sparam.p, D.grav.p, D.y.p, D.ydot.p, D.xt.p);
    pairs_from_scratch(c, D.y.p);
    launch_lag(c, D.xw.p);
    c->n_lag_pt = c->n_pt;
    hipLaunchKernelGGL(k_copy_int, dim3(blocks_for(c->n_scenes + 1)), dim3(BLOCK), 0, st, c->n_scenes + 1, seg_ptr(c, R_PT), seg_ptr(c, R_LPT));
    hipLaunchKernelGGL(k_copy_int, dim3(blocks_for(c->n_scenes + 1)), dim3(BLOCK), 0, st, c->n_scenes + 1, seg_ptr(c, R_EE), seg_ptr(c, R_LEE));
    c->step_ready = true;
}

} // namespace

// pinned staging areas of the context (allocated on first use)
constexpr size_t PIN_RD_BYTES = 1 << 20, PIN_WR_BYTES = 1 << 20;
static void ensure_pinned(ipc_ctx *c)
{
    if (c->pin_rd) return;
    IPC_HIP(hipHostMalloc((void **)&c->pin_rd, PIN_RD_BYTES, hipHostMallocDefault));
    IPC_HIP(hipHostMalloc((void **)&c->pin_wr, PIN_WR_BYTES, hipHostMallocDefault));
    c->pin_wr_off = 0;
}

HostReads::HostReads(ipc_ctx *cc) : c(cc) { ensure_pinned(c); }

void HostReads::add(void *dst, const void *src, size_t bytes)
{
    if (!bytes) return;
    size_t off = (used + 63) & ~(size_t)63;
    if (off + bytes > PIN_RD_BYTES) {
        IPC_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, c->stream));
        return;
    }
    IPC_HIP(hipMemcpyAsync(c->pin_rd + off, src, bytes, hipMemcpyDeviceToHost, c->stream));
    items.push_back({dst, off, bytes});
    used = off + bytes;
}

void HostReads::wait()
{
    IPC_HIP(hipStreamSynchronize(c->stream));
    for (auto &it : items) std::memcpy(it.dst, c->pin_rd + it.off, it.bytes);
    items.clear();
    used = 0;
}

// The ring wraps after a stream synchronisation, so no pending copy still
// reads the part that is overwritten.
void upload_async(ipc_ctx *c, void *dst_dev, const void *src, size_t bytes)
{
    if (!bytes) return;
    ensure_pinned(c);
    if (bytes > PIN_WR_BYTES) {
        IPC_HIP(hipMemcpyAsync(dst_dev, src, bytes, hipMemcpyHostToDevice, c->stream));
        sync(c);
        return;
    }
    size_t off = (c->pin_wr_off + 255) & ~(size_t)255;
    if (off + bytes > PIN_WR_BYTES) {
        sync(c);
        off = 0;
    }
    std::memcpy(c->pin_wr + off, src, bytes);
    IPC_HIP(hipMemcpyAsync(dst_dev, c->pin_wr + off, bytes, hipMemcpyHostToDevice, c->stream));
    c->pin_wr_off = off + bytes;
}


__global__ void k_fill_int_api(int n, int *p, int v)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

} // namespace ipc

using namespace ipc;

// ---------------------------------------------------------------------------------
// C-ABI
// ---------------------------------------------------------------------------------
namespace ipc {
thread_local Arena *g_arena = nullptr;
}

template <class F>
static int guard(ipc_ctx *c, F f)
{
    // device buffers of a workspace context come from its workspace
    ArenaScope scope(c && c->ws.base ? &c->ws : nullptr);
    try {
        f();
        return IPC_OK;
    } catch (const Error &e) {
        if (c) c->err = e.msg;
        return e.code;
    } catch (const std::exception &e) {
        if (c) c->err = e.what();
        return IPC_E_DEVICE;
    } catch (...) {
        if (c) c->err = "unknown error";
        return IPC_E_DEVICE;
    }
}

// run-time options of a new context (environment variables read at creation)
static void read_options(ipc_ctx *c)
{
    const char *ng = std::getenv("IPC_NO_GRAPH");
    c->use_graphs = !(ng && ng[0] == '1');
    const char *nl = std::getenv("IPC_SPMV_LANES");
    if (nl) {
        int L = std::atoi(nl);
        if (L == 1 || L == 2 || L == 4 || L == 8 || L == 16) {
            c->spmv_lanes = L;
            c->spmv_lanes_forced = true;
        }
    }
    const char *nc = std::getenv("IPC_PCG_COARSE");   // 0: never, 1: always, else by size and the autotuner
    c->coarse = !(nc && nc[0] == '0');
    c->coarse_forced = nc && nc[0] == '1';
    const char *nfp = std::getenv("IPC_NO_FUSED_PCG");   // 1: the coarse correction in a launch of its own
    c->pcg_fused = !(nfp && nfp[0] == '1');
    const char *nf = std::getenv("IPC_NO_FLOOR_STOP");   // 1: no stop at the energy's rounding floor
    c->floor_stop = !(nf && nf[0] == '1');
    const char *tr = std::getenv("IPC_TRACE_NEWTON");   // a scene index: its Newton iterations on stderr
    c->trace_scene = tr ? std::atoi(tr) : -1;
    if (hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) c->use_graphs = false;
}

// scene checks on the host, before any HIP call
static int precheck(const ipc_scene_desc *scenes, int n_scenes)
{
    try {
        validate_scenes(scenes, n_scenes);
    } catch (const Error &e) {
        g_create_error = e.msg;
        return e.code;
    }
    return IPC_OK;
}

// The autotuner's choices, kept for the process and keyed by the size
// bucket of the context: powers of two of the block count of the static
// matrix pattern and of the node count, and whether it holds several scenes.
// A new context of a known bucket starts with the product's tuned lane count.
struct Tuned {
    int lanes, fem_block, asm_block, grad_block;
};
static std::mutex g_tune_mu;
static std::map<uint32_t, Tuned> g_tuned;

static uint32_t tune_key(const ipc_ctx *c)
{
    auto lg = [](int64_t n) { uint32_t b = 0; while (b < 40 && (int64_t(1) << b) < n) ++b; return b; };
    return (lg(c->nnzb) << 16) | (lg(c->N) << 1) | (c->n_scenes > 1 ? 1u : 0u);
}

static void adopt_tuned(ipc_ctx *c)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(tune_key(c));
    if (it == g_tuned.end()) return;
    if (!c->spmv_lanes_forced) c->spmv_lanes = it->second.lanes;
    c->fem_block = it->second.fem_block;
    c->asm_block = it->second.asm_block;
    c->grad_block = it->second.grad_block;
}

extern "C" int ipc_create(const ipc_scene_desc *scenes, int n_scenes, void *hip_stream, ipc_ctx **out)
{
    if (!out) return IPC_E_INVALID;
    *out = nullptr;
    if (int rc = precheck(scenes, n_scenes)) return rc;
    ipc_ctx *c = new ipc_ctx;
    c->stream = (hipStream_t)hip_stream;
    read_options(c);
    int rc = guard(c, [&] {
        create_context(c, scenes, n_scenes);
        setup_after_create(c);
        adopt_tuned(c);
    });
    if (rc != IPC_OK) {
        g_create_error = c->err;
        delete c;
        return rc;
    }
    *out = c;
    return IPC_OK;
}

static bool caps_ok(const ipc_capacity *cap)
{
    return cap && cap->max_pairs >= 0 && cap->max_candidates >= 0 && cap->max_local_blocks >= 0 &&
           16 * std::max(cap->max_pairs, cap->max_candidates) < (int64_t)INT32_MAX && cap->max_local_blocks < (int64_t)INT32_MAX;
}

extern "C" int ipc_plan(const ipc_scene_desc *scenes, int n_scenes, const ipc_capacity *cap, size_t *workspace_bytes)
{
    if (!workspace_bytes) return IPC_E_INVALID;
    *workspace_bytes = 0;
    if (!caps_ok(cap)) { g_create_error = "invalid capacity"; return IPC_E_INVALID; }
    if (int rc = precheck(scenes, n_scenes)) return rc;
    try {
        ipc_ctx tmp;   // the host half of the creation only: no HIP call
        const int64_t caps[3] = {cap->max_pairs, cap->max_candidates, cap->max_local_blocks};
        create_context(&tmp, scenes, n_scenes, caps, workspace_bytes);
    } catch (const Error &e) {
        g_create_error = e.msg;
        return e.code;
    } catch (const std::exception &e) {
        g_create_error = e.what();
        return IPC_E_INVALID;
    }
    return IPC_OK;
}

extern "C" int ipc_create_ws(const ipc_scene_desc *scenes, int n_scenes, const ipc_capacity *cap, void *workspace_dev,
                             size_t workspace_bytes, void *hip_stream, ipc_ctx **out)
{
    if (!out) return IPC_E_INVALID;
    *out = nullptr;
    if (!caps_ok(cap)) { g_create_error = "invalid capacity"; return IPC_E_INVALID; }
    if (!workspace_dev || workspace_bytes == 0 || ((uintptr_t)workspace_dev & 255)) {
        g_create_error = "need a workspace of nonzero size aligned to 256 bytes";
        return IPC_E_INVALID;
    }
    if (int rc = precheck(scenes, n_scenes)) return rc;
    ipc_ctx *c = new ipc_ctx;
    c->stream = (hipStream_t)hip_stream;
    c->ws.init(workspace_dev, workspace_bytes);
    read_options(c);
    int rc = guard(c, [&] {
        create_context(c, scenes, n_scenes);
        setup_after_create(c);
        adopt_tuned(c);
        reserve_capacity(c, cap->max_pairs, cap->max_candidates, cap->max_local_blocks);
        IPC_HIP(hipStreamSynchronize(c->stream));
    });
    if (rc != IPC_OK) {
        g_create_error = c->err;
        delete c;
        return rc;
    }
    *out = c;
    return IPC_OK;
}

extern "C" int ipc_destroy(ipc_ctx *c)
{
    if (!c) return IPC_E_INVALID;
    (void)hipStreamSynchronize(c->stream);
    delete c;
    return IPC_OK;
}

extern "C" const char *ipc_last_error(const ipc_ctx *c) { return c ? c->err.c_str() : g_create_error.c_str(); }

extern "C" int ipc_query(const ipc_ctx *c, int what, int64_t *v)
{
    if (!c || !v) return IPC_E_INVALID;
    switch (what) {
    case IPC_Q_NDOF: *v = c->ndof; return IPC_OK;
    case IPC_Q_NSCENES: *v = c->n_scenes; return IPC_OK;
    case IPC_Q_NDRIVEN: *v = c->ND; return IPC_OK;
    case IPC_Q_NTRI: *v = c->TRI; return IPC_OK;
    case IPC_Q_NEDGE: *v = c->EDGE; return IPC_OK;
    case IPC_Q_NNODES: *v = c->N; return IPC_OK;
    case IPC_Q_NTETS: *v = c->T; return IPC_OK;
    case IPC_Q_NLOCAL: *v = c->n_local; return IPC_OK;
    case IPC_Q_NPAIRS: *v = c->n_pt + c->n_ee; return IPC_OK;
    case IPC_Q_NTETS_EXT: *v = c->ext_tets; return IPC_OK;
    case IPC_Q_COARSE: *v = c->coarse_on ? 1 : 0; return IPC_OK;
    case IPC_Q_WS_BYTES: *v = (int64_t)c->ws.size; return IPC_OK;
    case IPC_Q_WS_PEAK: *v = (int64_t)c->ws.peak; return IPC_OK;
    case IPC_Q_SPMV_LANES: *v = c->spmv_lanes; return IPC_OK;
    case IPC_Q_FEM_BLOCKS: *v = ((int64_t)c->fem_block << 32) | ((int64_t)c->asm_block << 16) | c->grad_block; return IPC_OK;
    case IPC_Q_PCG_FUSED: *v = c->cg_fusable && c->coarse_on && c->pcg_fused && c->n_cdom > 0 ? 1 : 0; return IPC_OK;
    }
    return IPC_E_INVALID;
}

extern "C" int ipc_set_timestep(ipc_ctx *c, const double *h_host)
{
    if (!c || !h_host) return IPC_E_INVALID;
    for (int s = 0; s < c->n_scenes; ++s)
        if (!std::isfinite(h_host[s])) { c->err = "time step must be finite"; return IPC_E_INVALID; }
    return guard(c, [&] {
        std::vector<double> h2(c->n_scenes);
        for (int s = 0; s < c->n_scenes; ++s) {
            SceneInfo &S = c->sc[s];
            if (h_host[s] > 0.0) {
                S.h = h_host[s];
                S.thr = S.newton_tol * S.h * S.L;   // the Newton stop scales with h
            }
            h2[s] = S.h * S.h;
        }
        upload_sparam(c);                 // h, h^2, eps_v h (kappa keeps its creation value)
        c->d.h2s.upload(h2, c->stream);
        build_const_part(c, c->d.h2s.p);  // the h^2-weighted spring blocks
        sync(c);
        c->step_ready = false;            // the predictor and the friction lag use h
    });
}

extern "C" int ipc_set_friction_lag(ipc_ctx *c, int passes)
{
    if (!c) return IPC_E_INVALID;
    if (passes < 1 || passes > 16) { c->err = "friction lag passes must lie in [1, 16]"; return IPC_E_INVALID; }
    c->lag_passes = passes;
    return IPC_OK;
}

extern "C" int ipc_set_kappa_adaptive(ipc_ctx *c, double frac, double factor)
{
    if (!c) return IPC_E_INVALID;
    if (!(frac >= 0.0) || !std::isfinite(frac) || !(factor >= 1.0) || !std::isfinite(factor)) {
        c->err = "adaptive kappa needs a finite frac >= 0 and factor >= 1";
        return IPC_E_INVALID;
    }
    return guard(c, [&] {
        std::vector<double> sc = read_scal(c);
        for (int s = 0; s < c->n_scenes; ++s) sc[(size_t)s * NSLOT + S_KAPPA0] = c->sc[s].kappa;
        write_scal(c, sc);
        c->kappa_frac = frac;
        c->kappa_factor = factor;
        sync(c);
    });
}

extern "C" int ipc_scene_scalars(const ipc_ctx *c, int s, double *kappa, double *L, double *thr)
{
    if (!c || s < 0 || s >= c->n_scenes) return IPC_E_INVALID;
    if (kappa) *kappa = c->sc[s].kappa;
    if (L) *L = c->sc[s].L;
    if (thr) *thr = c->sc[s].thr;
    return IPC_OK;
}

extern "C" int ipc_get_state(ipc_ctx *c, double *y_dev, double *ydot_dev)
{
    if (!c || !y_dev) return IPC_E_INVALID;
    return guard(c, [&] {
        hipLaunchKernelGGL(k_to_external, dim3(blocks_for(c->ext_nodes)), dim3(BLOCK), 0, c->stream, c->ext_nodes, c->d.ext2node.p,
                           c->d.y.p, y_dev);
        if (ydot_dev)
            hipLaunchKernelGGL(k_to_external, dim3(blocks_for(c->ext_nodes)), dim3(BLOCK), 0, c->stream, c->ext_nodes,
                               c->d.ext2node.p, c->d.ydot.p, ydot_dev);
        IPC_HIP(hipGetLastError());
    });
}

extern "C" int ipc_set_state(ipc_ctx *c, const double *y_dev, const double *ydot_dev)
{
    if (!c || !y_dev || !ydot_dev) return IPC_E_INVALID;
    return guard(c, [&] {
        hipLaunchKernelGGL(k_to_internal, dim3(blocks_for(c->ext_nodes)), dim3(BLOCK), 0, c->stream, c->ext_nodes, c->d.ext2node.p,
                           y_dev, c->d.y.p);
        hipLaunchKernelGGL(k_to_internal, dim3(blocks_for(c->ext_nodes)), dim3(BLOCK), 0, c->stream, c->ext_nodes, c->d.ext2node.p,
                           ydot_dev, c->d.ydot.p);
        IPC_HIP(hipGetLastError());
        c->step_ready = false;
    });
}

extern "C" int ipc_begin_step(ipc_ctx *c, const double *targets_dev)
{
    if (!c) return IPC_E_INVALID;
    if ((c->ND || c->NJ) && !targets_dev) { c->err = "targets required: the scenes have driven links or joint springs"; return IPC_E_INVALID; }
    return guard(c, [&] { begin_step_impl(c, targets_dev); });
}

extern "C" int ipc_energy_grad_hess(ipc_ctx *c, const double *y_dev, double *E_dev, double *g_dev, const double *v_dev, double *Hv_dev,
                                    uint32_t flags)
{
    if (!c || !y_dev) return IPC_E_INVALID;
    if (!c->step_ready) { c->err = "call ipc_begin_step first"; return IPC_E_INVALID; }
    int status = IPC_OK;
    int rc = guard(c, [&] {
        Dev &D = c->d;
        hipStream_t st = c->stream;
        c->fr_on = (flags & IPC_WITH_FRICTION) != 0;
        double *y = D.v2.p;
        hipLaunchKernelGGL(k_zero, dim3(blocks_for(3 * (int64_t)c->N)), dim3(BLOCK), 0, st, 3 * (int64_t)c->N, y);
        hipLaunchKernelGGL(k_to_internal, dim3(blocks_for(c->ext_nodes)), dim3(BLOCK), 0, st, c->ext_nodes, D.ext2node.p, y_dev, y);
        pairs_from_scratch(c, y);
        if (E_dev) {
            eval_energy(c, y, false);
            hipLaunchKernelGGL(k_gather_slot, dim3(blocks_for(c->n_scenes, 64)), dim3(64), 0, st, c->n_scenes, D.scal.p, S_E, E_dev);
        }
        bool hv = v_dev && Hv_dev;
        if (g_dev || hv) {
            eval_grad_hess(c, y, D.g.p, hv, (flags & IPC_PSD_PROJECT) != 0);
            if (g_dev)
                hipLaunchKernelGGL(k_to_external, dim3(blocks_for(c->ext_nodes)), dim3(BLOCK), 0, st, c->ext_nodes, D.ext2node.p, D.g.p,
                                   g_dev);
        }
        if (hv) {
            hipLaunchKernelGGL(k_zero, dim3(blocks_for(3 * (int64_t)c->N)), dim3(BLOCK), 0, st, 3 * (int64_t)c->N, D.v1.p);
            hipLaunchKernelGGL(k_to_internal, dim3(blocks_for(c->ext_nodes)), dim3(BLOCK), 0, st, c->ext_nodes, D.ext2node.p, v_dev, D.v1.p);
            hess_apply(c, D.v1.p, D.q.p, nullptr, nullptr);
            hipLaunchKernelGGL(k_to_external, dim3(blocks_for(c->ext_nodes)), dim3(BLOCK), 0, st, c->ext_nodes, D.ext2node.p, D.q.p, Hv_dev);
        }
        std::vector<int> inf(c->n_scenes);
        IPC_HIP(hipMemcpyAsync(inf.data(), D.inf_flag.p, c->n_scenes * sizeof(int), hipMemcpyDeviceToHost, st));
        IPC_HIP(hipStreamSynchronize(st));
        for (int s = 0; s < c->n_scenes; ++s) if (inf[s]) status = IPC_E_INTERSECTING;
        c->fr_on = true;
    });
    return rc != IPC_OK ? rc : status;
}

namespace ipc {
// internal node -> external node (-1: padding)
__global__ void k_int2ext(int64_t NE, const int *__restrict__ ext2node, int *__restrict__ int2ext)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < NE) int2ext[ext2node[i]] = (int)i;
}
// Export of the assembled matrix in the external numbering: row i of the
// result is internal row ext2node[i], the union of its block-CSR columns and
// its pair-local columns (both ascending internally), equal columns summed,
// then ordered by external column.
template <bool WRITE>
__global__ void k_bsr_export(int64_t NE, const int *__restrict__ ext2node, const int *__restrict__ int2ext,
                             const int *__restrict__ rp, const int *__restrict__ col, const double *__restrict__ val,
                             const int *__restrict__ dp, const int *__restrict__ dcol, const double *__restrict__ dval,
                             int *__restrict__ cnt, const int *__restrict__ off, int *__restrict__ ocol, double *__restrict__ oval)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= NE) return;
    const int r = ext2node[i];
    int a = rp[r], ae = rp[r + 1], b = dp[r], be = dp[r + 1], n = 0;
    int o = WRITE ? off[i] : 0;
    while (a < ae || b < be) {
        const int ca = a < ae ? col[a] : INT_MAX, cb = b < be ? dcol[b] : INT_MAX;
        const int cc = min(ca, cb);
        if (WRITE) {
            double blk[9];
#pragma unroll
            for (int q = 0; q < 9; ++q) blk[q] = 0.0;
            if (ca == cc) for (int q = 0; q < 9; ++q) blk[q] += val[9 * (size_t)a + q];
            if (cb == cc) for (int q = 0; q < 9; ++q) blk[q] += dval[9 * (size_t)b + q];
            ocol[o + n] = int2ext[cc];
            for (int q = 0; q < 9; ++q) oval[9 * (size_t)(o + n) + q] = blk[q];
        }
        if (ca == cc) ++a;
        if (cb == cc) ++b;
        ++n;
    }
    if (!WRITE) {
        cnt[i] = n;
        return;
    }
    // the internal node order is not the external one: sort the row's blocks
    // by external column (insertion sort; rows hold a few dozen blocks)
    for (int u = 1; u < n; ++u) {
        const int key = ocol[o + u];
        double blk[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) blk[q] = oval[9 * (size_t)(o + u) + q];
        int v = u - 1;
        for (; v >= 0 && ocol[o + v] > key; --v) {
            ocol[o + v + 1] = ocol[o + v];
#pragma unroll
            for (int q = 0; q < 9; ++q) oval[9 * (size_t)(o + v + 1) + q] = oval[9 * (size_t)(o + v) + q];
        }
        ocol[o + v + 1] = key;
#pragma unroll
        for (int q = 0; q < 9; ++q) oval[9 * (size_t)(o + v + 1) + q] = blk[q];
    }
}
} // namespace ipc

extern "C" int ipc_hessian_bsr(ipc_ctx *c, const double *y_dev, uint32_t flags, int32_t *row_ptr_dev, int32_t *col_dev,
                               double *val_dev, int64_t cap_blocks, int64_t *nnzb_out)
{
    if (!c || !y_dev || !row_ptr_dev || !nnzb_out || cap_blocks < 0) return IPC_E_INVALID;
    if (!c->step_ready) { c->err = "call ipc_begin_step first"; return IPC_E_INVALID; }
    int status = IPC_OK;
    int rc = guard(c, [&] {
        Dev &D = c->d;
        hipStream_t st = c->stream;
        c->fr_on = (flags & IPC_WITH_FRICTION) != 0;
        double *y = D.v2.p;
        hipLaunchKernelGGL(k_zero, dim3(blocks_for(3 * (int64_t)c->N)), dim3(BLOCK), 0, st, 3 * (int64_t)c->N, y);
        hipLaunchKernelGGL(k_to_internal, dim3(blocks_for(c->ext_nodes)), dim3(BLOCK), 0, st, c->ext_nodes, D.ext2node.p, y_dev, y);
        pairs_from_scratch(c, y);
        eval_grad_hess(c, y, D.g.p, true, (flags & IPC_PSD_PROJECT) != 0);
        c->fr_on = true;
        const int64_t NE = c->ext_nodes;
        D.int2ext.alloc(c->N);
        hipLaunchKernelGGL(k_int2ext, dim3(blocks_for(NE)), dim3(BLOCK), 0, st, NE, D.ext2node.p, D.int2ext.p);
        D.bsr_cnt.alloc(NE + 1);
        hipLaunchKernelGGL(k_bsr_export<false>, dim3(blocks_for(NE)), dim3(BLOCK), 0, st, NE, D.ext2node.p, D.int2ext.p, D.row_ptr.p,
                           D.col.p, D.val.p, D.dyn_ptr.p, D.dyn_col.p, D.dyn_val.p, D.bsr_cnt.p, nullptr, nullptr, nullptr);
        hipLaunchKernelGGL(k_fill_int_api, dim3(1), dim3(64), 0, st, 1, D.bsr_cnt.p + NE, 0);
        exclusive_scan_int(c, D.bsr_cnt.p, row_ptr_dev, (int)NE);
        int total = 0;
        std::vector<int> inf(c->n_scenes);
        IPC_HIP(hipMemcpyAsync(&total, row_ptr_dev + NE, sizeof(int), hipMemcpyDeviceToHost, st));
        IPC_HIP(hipMemcpyAsync(inf.data(), D.inf_flag.p, c->n_scenes * sizeof(int), hipMemcpyDeviceToHost, st));
        IPC_HIP(hipStreamSynchronize(st));
        *nnzb_out = total;
        for (int s = 0; s < c->n_scenes; ++s) if (inf[s]) status = IPC_E_INTERSECTING;
        if (total > cap_blocks || !col_dev || !val_dev) {
            if (status == IPC_OK) status = IPC_E_CAPACITY;
            c->err = "the matrix has " + std::to_string(total) + " blocks";
            return;
        }
        hipLaunchKernelGGL(k_bsr_export<true>, dim3(blocks_for(NE)), dim3(BLOCK), 0, st, NE, D.ext2node.p, D.int2ext.p, D.row_ptr.p,
                           D.col.p, D.val.p, D.dyn_ptr.p, D.dyn_col.p, D.dyn_val.p, nullptr, row_ptr_dev, col_dev, val_dev);
        IPC_HIP(hipGetLastError());
        IPC_HIP(hipStreamSynchronize(st));
    });
    return rc != IPC_OK ? rc : status;
}

extern "C" int ipc_get_pairs(ipc_ctx *c, const double *y_dev, int scene, int32_t *pt_host, int32_t *ee_host, int64_t cap, int64_t *n_pt,
                             int64_t *n_ee)
{
    if (!c || !y_dev || scene < 0 || scene >= c->n_scenes || !n_pt || !n_ee) return IPC_E_INVALID;
    int status = IPC_OK;
    int rc = guard(c, [&] {
        Dev &D = c->d;
        hipStream_t st = c->stream;
        double *y = D.v2.p;
        hipLaunchKernelGGL(k_zero, dim3(blocks_for(3 * (int64_t)c->N)), dim3(BLOCK), 0, st, 3 * (int64_t)c->N, y);
        hipLaunchKernelGGL(k_to_internal, dim3(blocks_for(c->ext_nodes)), dim3(BLOCK), 0, st, c->ext_nodes, D.ext2node.p, y_dev, y);
        pairs_from_scratch(c, y);
        SceneInfo &S = c->sc[scene];
        int a0 = c->h_pt_seg[scene], a1 = c->h_pt_seg[scene + 1], b0 = c->h_ee_seg[scene], b1 = c->h_ee_seg[scene + 1];
        *n_pt = a1 - a0; *n_ee = b1 - b0;
        if (*n_pt > cap || *n_ee > cap) { status = IPC_E_CAPACITY; return; }
        std::vector<int2> hp(a1 - a0), he(b1 - b0);
        if (a1 > a0) IPC_HIP(hipMemcpyAsync(hp.data(), D.pt.p + a0, hp.size() * sizeof(int2), hipMemcpyDeviceToHost, st));
        if (b1 > b0) IPC_HIP(hipMemcpyAsync(he.data(), D.ee.p + b0, he.size() * sizeof(int2), hipMemcpyDeviceToHost, st));
        IPC_HIP(hipStreamSynchronize(st));
        std::vector<std::array<int, 4>> P, E;
        for (auto &q : hp) {
            int t = q.y - S.tri0;
            P.push_back({S.surf_ext[q.x - S.cv0], S.tri_ext[3 * t], S.tri_ext[3 * t + 1], S.tri_ext[3 * t + 2]});
        }
        for (auto &q : he) {
            int e = q.x - S.edge0, f = q.y - S.edge0;
            E.push_back({S.edge_ext[2 * e], S.edge_ext[2 * e + 1], S.edge_ext[2 * f], S.edge_ext[2 * f + 1]});
        }
        std::sort(P.begin(), P.end());
        std::sort(E.begin(), E.end());
        for (size_t k = 0; k < P.size(); ++k) for (int m = 0; m < 4; ++m) pt_host[4 * k + m] = P[k][m];
        for (size_t k = 0; k < E.size(); ++k) for (int m = 0; m < 4; ++m) ee_host[4 * k + m] = E[k][m];
    });
    return rc != IPC_OK ? rc : status;
}

extern "C" int ipc_ccd(ipc_ctx *c, const double *y_dev, const double *p_dev, double *alpha_dev)
{
    if (!c || !y_dev || !p_dev || !alpha_dev) return IPC_E_INVALID;
    return guard(c, [&] {
        Dev &D = c->d;
        hipStream_t st = c->stream;
        hipLaunchKernelGGL(k_zero, dim3(blocks_for(3 * (int64_t)c->N)), dim3(BLOCK), 0, st, 3 * (int64_t)c->N, D.v2.p);
        hipLaunchKernelGGL(k_zero, dim3(blocks_for(3 * (int64_t)c->N)), dim3(BLOCK), 0, st, 3 * (int64_t)c->N, D.v1.p);
        hipLaunchKernelGGL(k_to_internal, dim3(blocks_for(c->ext_nodes)), dim3(BLOCK), 0, st, c->ext_nodes, D.ext2node.p, y_dev, D.v2.p);
        hipLaunchKernelGGL(k_to_internal, dim3(blocks_for(c->ext_nodes)), dim3(BLOCK), 0, st, c->ext_nodes, D.ext2node.p, p_dev, D.v1.p);
        hipLaunchKernelGGL(k_set_slot, dim3(blocks_for(c->n_scenes, 64)), dim3(64), 0, st, c->n_scenes, D.scal.p, S_LS_ON, 1.0);
        hipLaunchKernelGGL(k_set_slot, dim3(blocks_for(c->n_scenes, 64)), dim3(64), 0, st, c->n_scenes, D.scal.p, S_LS_ALPHA, 1.0);
        hipLaunchKernelGGL(k_trial, dim3(blocks_for(c->N)), dim3(BLOCK), 0, st, c->N, D.node_scene.p, D.scal.p, D.v2.p, D.v1.p, D.yt.p);
        launch_world(c, D.v2.p, D.xw.p);
        launch_world(c, D.yt.p, D.xw1.p);
        broad_phase(c, D.xw.p, D.xw1.p);
        hipLaunchKernelGGL(k_set_slot, dim3(blocks_for(c->n_scenes, 64)), dim3(64), 0, st, c->n_scenes, D.scal.p, S_CCD, 1.0);
        hipLaunchKernelGGL(k_fill_int_api, dim3(blocks_for(c->n_scenes)), dim3(BLOCK), 0, st, c->n_scenes, D.ls_active.p, 1);
        launch_ccd(c, D.xw.p, D.xw1.p);
        hipLaunchKernelGGL(k_gather_slot, dim3(blocks_for(c->n_scenes, 64)), dim3(64), 0, st, c->n_scenes, D.scal.p, S_CCD, alpha_dev);
        IPC_HIP(hipStreamSynchronize(st));
    });
}

extern "C" int ipc_pcg(ipc_ctx *c, const double *y_dev, const double *b_dev, double *x_dev, double eta, int32_t *iters_host)
{
    if (!c || !y_dev || !b_dev || !x_dev) return IPC_E_INVALID;
    if (!c->step_ready) { c->err = "call ipc_begin_step first"; return IPC_E_INVALID; }
    return guard(c, [&] {
        Dev &D = c->d;
        hipStream_t st = c->stream;
        double *y = D.y0.p;   // y0 is free outside ipc_step
        hipLaunchKernelGGL(k_zero, dim3(blocks_for(3 * (int64_t)c->N)), dim3(BLOCK), 0, st, 3 * (int64_t)c->N, y);
        hipLaunchKernelGGL(k_to_internal, dim3(blocks_for(c->ext_nodes)), dim3(BLOCK), 0, st, c->ext_nodes, D.ext2node.p, y_dev, y);
        pairs_from_scratch(c, y);
        eval_grad_hess(c, y, D.g.p, true, true);
        build_preconditioner(c);
        hipLaunchKernelGGL(k_zero, dim3(blocks_for(3 * (int64_t)c->N)), dim3(BLOCK), 0, st, 3 * (int64_t)c->N, D.v1.p);
        hipLaunchKernelGGL(k_to_internal, dim3(blocks_for(c->ext_nodes)), dim3(BLOCK), 0, st, c->ext_nodes, D.ext2node.p, b_dev, D.v1.p);
        pcg_solve(c, D.v1.p, D.x.p, eta, nullptr);
        hipLaunchKernelGGL(k_to_external, dim3(blocks_for(c->ext_nodes)), dim3(BLOCK), 0, st, c->ext_nodes, D.ext2node.p, D.x.p, x_dev);
        if (iters_host) IPC_HIP(hipMemcpyAsync(iters_host, D.pcg_iters.p, c->n_scenes * sizeof(int), hipMemcpyDeviceToHost, st));
        IPC_HIP(hipStreamSynchronize(st));
    });
}

extern "C" int ipc_set_params(ipc_ctx *c, const double *tet_E_dev, const double *mu_host)
{
    if (!c) return IPC_E_INVALID;
    if (mu_host)
        for (int s = 0; s < c->n_scenes; ++s)
            if (!(mu_host[s] >= 0.0) || !std::isfinite(mu_host[s])) { c->err = "mu must be finite and >= 0"; return IPC_E_INVALID; }
    return guard(c, [&] {
        hipStream_t st = c->stream;
        if (tet_E_dev && c->ext_tets) {
            std::vector<double> E((size_t)c->ext_tets);
            IPC_HIP(hipMemcpyAsync(E.data(), tet_E_dev, E.size() * sizeof(double), hipMemcpyDeviceToHost, st));
            sync(c);
            for (size_t i = 0; i < E.size(); ++i)
                if (!(E[i] > 0.0) || !std::isfinite(E[i])) throw Error(IPC_E_INVALID, "Young's modulus must be finite and > 0 (tet " + std::to_string(i) + ")");
            launch_set_E(c, tet_E_dev);
        }
        if (mu_host) {
            for (int s = 0; s < c->n_scenes; ++s) c->sc[s].mu = mu_host[s];
            upload_sparam(c);
        }
        IPC_HIP(hipGetLastError());
        sync(c);
    });
}

extern "C" int ipc_step_vjp(ipc_ctx *c, const double *y_prev_dev, const double *ydot_prev_dev, const double *targets_dev,
                            const double *y_next_dev, const double *ybar_next_dev, const double *vbar_next_dev, double *ybar_prev_dev,
                            double *vbar_prev_dev, double *Ebar_dev, double *mubar_dev, double eta, int32_t *iters_host)
{
    if (!c || !y_prev_dev || !ydot_prev_dev || !y_next_dev || !ybar_next_dev || !vbar_next_dev || !ybar_prev_dev || !vbar_prev_dev)
        return IPC_E_INVALID;
    if ((c->ND || c->NJ) && !targets_dev) { c->err = "targets required: the scenes have driven links or joint springs"; return IPC_E_INVALID; }
    if (!(eta > 0.0)) { c->err = "eta must be > 0"; return IPC_E_INVALID; }
    if (c->lag_passes != 1) { c->err = "the adjoint differentiates steps lagged once at their start (ipc_set_friction_lag(ctx, 1))"; return IPC_E_INVALID; }
    if (c->kappa_frac > 0.0) { c->err = "the adjoint holds kappa fixed: switch adaptive kappa off (ipc_set_kappa_adaptive(ctx, 0, ...))"; return IPC_E_INVALID; }
    int status = IPC_OK;
    int rc = guard(c, [&] {
        Dev &D = c->d;
        hipStream_t st = c->stream;
        int64_t n3 = 3 * (int64_t)c->N;
        auto to_int = [&](const double *ext, double *v) {
            hipLaunchKernelGGL(k_zero, dim3(blocks_for(n3)), dim3(BLOCK), 0, st, n3, v);
            hipLaunchKernelGGL(k_to_internal, dim3(blocks_for(c->ext_nodes)), dim3(BLOCK), 0, st, c->ext_nodes, D.ext2node.p, ext, v);
        };
        // the step's set-up at (y^n, ydot^n): predictor and friction lag
        hipLaunchKernelGGL(k_to_internal, dim3(blocks_for(c->ext_nodes)), dim3(BLOCK), 0, st, c->ext_nodes, D.ext2node.p, y_prev_dev,
                           D.y.p);
        hipLaunchKernelGGL(k_to_internal, dim3(blocks_for(c->ext_nodes)), dim3(BLOCK), 0, st, c->ext_nodes, D.ext2node.p,
                           ydot_prev_dev, D.ydot.p);
        begin_step_impl(c, targets_dev);
        if (c->CV) IPC_HIP(hipMemcpyAsync(D.xw1.p, D.xw.p, 3 * (size_t)c->CV * sizeof(double), hipMemcpyDeviceToDevice, st));
        // y^{n+1}, the upstream adjoints and the right-hand side
        to_int(y_next_dev, D.yt.p);
        to_int(vbar_next_dev, D.y0.p);
        to_int(ybar_next_dev, D.v2.p);
        launch_adj_rhs(c, D.v2.p, D.y0.p, D.v1.p);
        // unprojected Hessian at y^{n+1} and H w = rhs
        c->fr_on = true;
        pairs_from_scratch(c, D.yt.p);
        eval_grad_hess(c, D.yt.p, D.g.p, true, false);
        build_preconditioner(c);
        pcg_solve(c, D.v1.p, D.x.p, eta, nullptr);
        std::vector<double> sc = read_scal(c);
        for (int s = 0; s < c->n_scenes; ++s)
            if (sc[(size_t)s * NSLOT + S_INDEF] != 0.0) status = IPC_E_INDEFINITE;
        if (iters_host) IPC_HIP(hipMemcpyAsync(iters_host, D.pcg_iters.p, c->n_scenes * sizeof(int), hipMemcpyDeviceToHost, st));
        if (status != IPC_OK) {
            c->err = "the Hessian at y_next is not positive definite along a PCG direction";
            sync(c);
            return;
        }
        // state adjoints: inertia, then the friction lag at x^n (D.xw1) and x^{n+1}
        launch_adj_mass(c, D.x.p, D.y0.p, D.v2.p, D.r.p);
        launch_world(c, D.yt.p, D.xw.p);
        launch_lag_vjp(c, D.xw.p, D.xw1.p, D.x.p, D.v2.p);
        D.fr_w64.alloc(c->n_lag / TILE + 1);
        sum64(c, D.fr_part.p, c->n_lag, D.fr_w64.p);
        RedArgs f{};
        f.src[f.nsrc++] = src(c->n_lag_pt ? D.fr_part.p : nullptr, seg_ptr(c, R_LPT), 0, 0);
        f.src[f.nsrc++] = src(c->n_lag - c->n_lag_pt ? D.fr_part.p : nullptr, seg_ptr(c, R_LEE), (int)c->n_lag_pt, 0);
        f.src[0].w64 = f.src[1].w64 = D.fr_w64.p;
        if (c->M_HS) {
            f.src[f.nsrc] = src(D.hs_fpart.p, seg_ptr(c, R_HS), 0, 0);
            f.src[f.nsrc++].w64 = D.hs_fw64.p;
        }
        f.slot = S_MUBAR;
        reduce(c, f);
        if (mubar_dev)
            hipLaunchKernelGGL(k_sub_slot, dim3(blocks_for(c->n_scenes, 64)), dim3(64), 0, st, c->n_scenes, D.scal.p, S_MUBAR, mubar_dev);
        if (Ebar_dev) launch_adj_E(c, D.yt.p, D.x.p, Ebar_dev);
        hipLaunchKernelGGL(k_to_external, dim3(blocks_for(c->ext_nodes)), dim3(BLOCK), 0, st, c->ext_nodes, D.ext2node.p, D.v2.p,
                           ybar_prev_dev);
        hipLaunchKernelGGL(k_to_external, dim3(blocks_for(c->ext_nodes)), dim3(BLOCK), 0, st, c->ext_nodes, D.ext2node.p, D.r.p,
                           vbar_prev_dev);
        IPC_HIP(hipGetLastError());
        sync(c);
    });
    return rc != IPC_OK ? rc : status;
}

// ---------------------------------------------------------------------------------
// the Newton step
// ---------------------------------------------------------------------------------
namespace ipc {

// Sets the context's assembly flags for a scope; cleared on exit, also when
// a device error unwinds it, so no later call assembles a subset.
struct AssembleOnly {
    ipc_ctx *c;
    AssembleOnly(ipc_ctx *cc, const int *flags) : c(cc) { c->assemble_only = flags; }
    ~AssembleOnly() { c->assemble_only = nullptr; }
};

// The stop at the energy's rounding floor (see the line search below).
constexpr double FLOOR_ALPHA = 1.0 / 1024.0, FLOOR_MEASURE = 10.0, FLOOR_ENERGY = 1e-13;

void newton_step(ipc_ctx *c, const double *targets_dev, ipc_stats *stats)
{
    Dev &D = c->d;
    hipStream_t st = c->stream;
    int ns = c->n_scenes;
    begin_step_impl(c, targets_dev);
    c->fr_on = true;
    IPC_HIP(hipMemcpyAsync(D.y0.p, D.y.p, 3 * (size_t)c->N * sizeof(double), hipMemcpyDeviceToDevice, st));
    std::vector<ipc_stats> S(ns);
    for (int s = 0; s < ns; ++s) {
        std::memset(&S[s], 0, sizeof(ipc_stats));
        S[s].status = IPC_E_NOT_CONVERGED;
        S[s].alpha_min = 1.0;
        S[s].n_lag = 0;
    }
    std::vector<int> on(ns, 1);
    const bool kappa_adapt = c->kappa_frac > 0.0;
    if (kappa_adapt) launch_kappa_update(c, D.xw.p, true);   // pairs and world positions at y^n
    // energy at the start
    eval_energy(c, D.y.p, false);
    std::vector<double> sc((size_t)ns * NSLOT);
    std::vector<int> hs_nlag(ns, 0);
    {
        HostReads rd(c);
        rd.add(sc.data(), D.scal.p, sc.size() * sizeof(double));
        if (c->M_HS) rd.add(hs_nlag.data(), D.hs_nlag.p, ns * sizeof(int));
        rd.wait();
    }
    std::vector<double> E0(ns), meas(ns, 0.0);
    for (int s = 0; s < ns; ++s) {
        E0[s] = sc[(size_t)s * NSLOT + S_E];
        if (sc[(size_t)s * NSLOT + S_INF] != 0.0) { S[s].status = IPC_E_INTERSECTING; on[s] = 0; }
        S[s].energy = E0[s];
        S[s].n_lag = (c->h_pt_seg[s + 1] - c->h_pt_seg[s]) + (c->h_ee_seg[s + 1] - c->h_ee_seg[s]) + hs_nlag[s];
    }
    int max_newton = 0;
    for (auto &si : c->sc) max_newton = std::max(max_newton, si.max_newton);
    std::vector<int> want(ns);
    // E0 holds each scene's energy at its iterate.  The trials are summed over
    // the swept candidate list; E0 is compared with them only when it was
    // summed over the same list in the same order (after an accepted trial),
    // and is evaluated again over the list whenever the list is rebuilt: a
    // decrease smaller than the rounding of the sums must not be lost to a
    // change of summation order (rebuilds follow any scene's sweep, so in a
    // batch they come far more often than a scene's own sweep asks for).
    bool e0_on_list = false;
    // friction lag passes: after a converged pass the lag is taken again at
    // the solution (slips still measured from the step start) and Newton
    // runs again from there, for the scenes that converged
    for (int pass = 0; pass < c->lag_passes; ++pass) {
    if (pass > 0) {
        bool again = false;
        for (int s = 0; s < ns; ++s) {
            on[s] = S[s].status == IPC_OK;
            if (on[s]) { S[s].status = IPC_E_NOT_CONVERGED; again = true; }
        }
        if (!again) break;
        pairs_from_scratch(c, D.y.p);          // pairs and world positions at the solution
        launch_world(c, D.y0.p, D.xw1.p);      // the step start
        launch_lag(c, D.xw.p, D.xw1.p);
        c->n_lag_pt = c->n_pt;
        hipLaunchKernelGGL(k_copy_int, dim3(blocks_for(c->n_scenes + 1)), dim3(BLOCK), 0, st, c->n_scenes + 1, seg_ptr(c, R_PT), seg_ptr(c, R_LPT));
        hipLaunchKernelGGL(k_copy_int, dim3(blocks_for(c->n_scenes + 1)), dim3(BLOCK), 0, st, c->n_scenes + 1, seg_ptr(c, R_EE), seg_ptr(c, R_LEE));
        eval_energy(c, D.y.p, false);
        sc = read_scal(c);
        for (int s = 0; s < ns; ++s)
            if (on[s]) { E0[s] = sc[(size_t)s * NSLOT + S_E]; S[s].energy = E0[s]; }
        e0_on_list = false;
    }
    for (int j = 0; j < max_newton; ++j) {
        bool any = false;
        for (int s = 0; s < ns; ++s) {
            if (on[s] && j >= c->sc[s].max_newton) on[s] = 0;
            any |= on[s] != 0;
        }
        if (!any) break;
        for (int s = 0; s < ns; ++s) {
            S[s].n_pt_max = std::max(S[s].n_pt_max, c->h_pt_seg[s + 1] - c->h_pt_seg[s]);
            S[s].n_ee_max = std::max(S[s].n_ee_max, c->h_ee_seg[s + 1] - c->h_ee_seg[s]);
        }
        // assemble and solve H p = -g for the scenes still iterating (in a
        // batch, the FEM, matrix, preconditioner and coarse blocks of scenes
        // that have converged are not formed again)
        upload_async(c, D.newton_on.p, on.data(), ns * sizeof(int));
        bool all_on = true;
        for (int s = 0; s < ns; ++s) all_on = all_on && on[s];
        {
            AssembleOnly only(c, all_on ? nullptr : D.newton_on.p);
            eval_grad_hess(c, D.y.p, D.g.p, true, true);
            build_preconditioner(c);
        }
        hipLaunchKernelGGL(k_negate, dim3(blocks_for(3 * (int64_t)c->N)), dim3(BLOCK), 0, st, 3 * (int64_t)c->N, D.g.p, D.v1.p);
        pcg_solve(c, D.v1.p, D.x.p, -1.0, D.newton_on.p);
        std::vector<int> it(ns);
        // the trial point y + p (step 1) and world positions at both ends,
        // and whether the kept candidates still cover that sweep; read
        // together with the Newton measure
        upload_async(c, D.ls_active.p, on.data(), ns * sizeof(int));
        hipLaunchKernelGGL(k_ls_begin, dim3(blocks_for(ns, 64)), dim3(64), 0, st, ns, D.ls_active.p, D.scal.p);
        hipLaunchKernelGGL(k_trial, dim3(blocks_for(c->N)), dim3(BLOCK), 0, st, c->N, D.node_scene.p, D.scal.p, D.y.p, D.x.p, D.yt.p);
        launch_world(c, D.y.p, D.xw.p);
        launch_world(c, D.yt.p, D.xw1.p);
        const bool cached = c->cand_cached;
        std::vector<int> stale(ns, 1);
        D.cand_flag.alloc(ns);
        if (cached) cand_check(c, D.xw.p, D.xw1.p, D.cand_flag.p);
        // Newton measure
        hipLaunchKernelGGL(k_measure_nodes, dim3(blocks_for(c->N)), dim3(BLOCK), 0, st, c->N, D.node_kind.p, D.x.p, D.part_node.p);
        if (c->NB)
            hipLaunchKernelGGL(k_measure_bodies, dim3(blocks_for(c->NB, 64)), dim3(64), 0, st, c->NB, D.body_node0.p, D.bext.p, D.x.p,
                               D.body_part.p);
        {
            RedArgs a{};
            a.op = 1;
            a.src[a.nsrc++] = src(D.part_node.p, seg_ptr(c, R_NODEW), 0, 0);
            a.src[a.nsrc++] = src(c->NB ? D.body_part.p : nullptr, seg_ptr(c, R_BODY), 0, 0);
            a.slot = S_NEWTON_MAX;
            reduce(c, a);
        }
        {
            HostReads rd(c);
            rd.add(it.data(), D.pcg_iters.p, ns * sizeof(int));
            rd.add(sc.data(), D.scal.p, sc.size() * sizeof(double));
            if (cached) rd.add(stale.data(), D.cand_flag.p, ns * sizeof(int));
            rd.wait();
        }
        any = false;
        for (int s = 0; s < ns; ++s) {
            if (!on[s]) continue;
            S[s].newton_iters += 1;
            S[s].pcg_iters_total += it[s];
            S[s].pcg_iters_max = std::max(S[s].pcg_iters_max, it[s]);
            if (s == c->trace_scene)
                std::fprintf(stderr, "ipc trace: scene %d newton %d: measure %.6g (stop %.6g), pcg %d\n", s, S[s].newton_iters,
                             sc[(size_t)s * NSLOT + S_NEWTON_MAX], c->sc[s].thr, it[s]);
            meas[s] = sc[(size_t)s * NSLOT + S_NEWTON_MAX];
            if (meas[s] <= c->sc[s].thr) { on[s] = 0; S[s].status = IPC_OK; }
            any |= on[s] != 0;
        }
        if (!any) break;
        // CCD over the swept candidates of [y, y + p]: the kept list while it
        // still covers every iterating scene's sweep, else a new one
        bool rebuild = !cached;
        for (int s = 0; s < ns; ++s) rebuild = rebuild || (on[s] && stale[s]);
        if (rebuild) {
            broad_phase_cached(c, D.xw.p, D.xw1.p);
            e0_on_list = false;
        }
        for (int s = 0; s < ns; ++s) S[s].n_cand_max = std::max(S[s].n_cand_max, (c->h_cand_pt_seg[s + 1] - c->h_cand_pt_seg[s]) +
                                                                             (c->h_cand_ee_seg[s + 1] - c->h_cand_ee_seg[s]));
        launch_ccd(c, D.xw.p, D.xw1.p);
        // The first trial is queued behind the CCD without a host read: the
        // step min(1, CCD bound) is set on the device, E(y) over the list the
        // trials use is evaluated first when that list is new (kept in S_E0),
        // then E(y + alpha p).  One read returns the bound, E(y) and the
        // first trial's energy.
        hipLaunchKernelGGL(k_ls_first, dim3(blocks_for(ns, 64)), dim3(64), 0, st, ns, D.scal.p);
        const bool new_e0 = !e0_on_list;
        if (new_e0) {
            eval_energy(c, D.y.p, true);
            hipLaunchKernelGGL(k_copy_slot, dim3(blocks_for(ns, 64)), dim3(64), 0, st, ns, D.scal.p, S_E, S_E0);
            e0_on_list = true;
        }
        hipLaunchKernelGGL(k_trial, dim3(blocks_for(c->N)), dim3(BLOCK), 0, st, c->N, D.node_scene.p, D.scal.p, D.y.p, D.x.p, D.yt.p);
        eval_energy(c, D.yt.p, true);
        sc = read_scal(c);
        std::vector<double> alpha(ns, 0.0);
        std::vector<int> ls(ns, 0);
        for (int s = 0; s < ns; ++s) {
            if (!on[s]) continue;
            alpha[s] = std::min(1.0, sc[(size_t)s * NSLOT + S_CCD]);
            ls[s] = 1;
            if (new_e0) E0[s] = sc[(size_t)s * NSLOT + S_E0];
        }
        // backtracking: halve each scene's step until its energy does not increase
        std::vector<double> Eacc(ns, 0.0);
        for (int h = 0; h <= 40; ++h) {
            bool pending = false;
            for (int s = 0; s < ns; ++s) {
                sc[(size_t)s * NSLOT + S_LS_ON] = on[s] ? 1.0 : 0.0;
                sc[(size_t)s * NSLOT + S_LS_ALPHA] = alpha[s];
                pending |= ls[s] != 0;
            }
            if (!pending) break;
            if (h > 0) {   // the first trial is already evaluated
                write_scal(c, sc);
                hipLaunchKernelGGL(k_trial, dim3(blocks_for(c->N)), dim3(BLOCK), 0, st, c->N, D.node_scene.p, D.scal.p, D.y.p, D.x.p,
                                   D.yt.p);
                eval_energy(c, D.yt.p, true);
                sc = read_scal(c);
            }
            for (int s = 0; s < ns; ++s) {
                if (!ls[s]) continue;
                double E1 = sc[(size_t)s * NSLOT + S_E];
                if (E1 <= E0[s]) { ls[s] = 0; Eacc[s] = E1; }
                else if (h == 40) { ls[s] = 0; on[s] = 0; S[s].status = IPC_E_LINESEARCH; alpha[s] = 0.0; }
                else alpha[s] *= 0.5;
            }
        }
        // accept: y <- y + alpha p (alpha = 0 for scenes that stopped)
        for (int s = 0; s < ns; ++s) {
            sc[(size_t)s * NSLOT + S_LS_ON] = alpha[s] > 0.0 ? 1.0 : 0.0;
            sc[(size_t)s * NSLOT + S_LS_ALPHA] = alpha[s];
            if (s == c->trace_scene)
                std::fprintf(stderr, "ipc trace: scene %d line search: alpha %.6g (CCD bound %.6g), E %.17g -> %.17g\n", s, alpha[s],
                             sc[(size_t)s * NSLOT + S_CCD], E0[s], Eacc[s]);
            if (alpha[s] > 0.0) {
                // The rounding floor: a direction whose measure is within
                // FLOOR_MEASURE of the stop, cut below FLOOR_ALPHA before the
                // energy stopped increasing, and whose step changed the
                // energy by no more than its rounding, cannot be resolved
                // further by the energy: the step is taken and the scene
                // stops as converged.
                if (c->floor_stop && alpha[s] <= FLOOR_ALPHA && meas[s] <= FLOOR_MEASURE * c->sc[s].thr &&
                    std::fabs(Eacc[s] - E0[s]) <= FLOOR_ENERGY * std::fabs(E0[s])) {
                    on[s] = 0;
                    S[s].status = IPC_OK;
                }
                E0[s] = Eacc[s];
                S[s].energy = Eacc[s];
                S[s].alpha_min = std::min(S[s].alpha_min, alpha[s]);
            }
        }
        write_scal(c, sc);
        hipLaunchKernelGGL(k_trial, dim3(blocks_for(c->N)), dim3(BLOCK), 0, st, c->N, D.node_scene.p, D.scal.p, D.y.p, D.x.p, D.yt.p);
        IPC_HIP(hipMemcpyAsync(D.y.p, D.yt.p, 3 * (size_t)c->N * sizeof(double), hipMemcpyDeviceToDevice, st));
        // pairs at the new iterate from the swept candidates (a superset)
        launch_world(c, D.y.p, D.xw.p);
        narrow_phase(c, D.xw.p);
        if (kappa_adapt) {
            // kappa may have changed: the next comparison energy is evaluated afresh
            launch_kappa_update(c, D.xw.p, false);
            e0_on_list = false;
        }
    }
    }
    if (kappa_adapt) {
        std::vector<double> sp(8 * (size_t)ns);
        IPC_HIP(hipMemcpyAsync(sp.data(), D.sparam.p, sp.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        IPC_HIP(hipStreamSynchronize(st));
        for (int s = 0; s < ns; ++s) c->sc[s].kappa = sp[8 * (size_t)s + P_KAPPA];
    }
    hipLaunchKernelGGL(k_velocity, dim3(blocks_for(c->N)), dim3(BLOCK), 0, st, c->N, D.node_scene.p, D.sparam.p, D.y.p, D.y0.p, D.ydot.p);
    IPC_HIP(hipStreamSynchronize(st));
    c->step_ready = false;
    if (stats) for (int s = 0; s < ns; ++s) stats[s] = S[s];
    c->last_status = IPC_OK;
    for (int s = 0; s < ns; ++s) if (S[s].status != IPC_OK) { c->last_status = S[s].status; break; }
}

} // namespace ipc

extern "C" int ipc_step(ipc_ctx *c, const double *targets_dev, ipc_stats *stats_host)
{
    if (!c) return IPC_E_INVALID;
    if ((c->ND || c->NJ) && !targets_dev) { c->err = "targets required: the scenes have driven links or joint springs"; return IPC_E_INVALID; }
    int rc = guard(c, [&] { newton_step(c, targets_dev, stats_host); });
    if (rc != IPC_OK) return rc;
    if (c->last_status != IPC_OK) c->err = "a scene did not finish its step cleanly (see ipc_stats.status)";
    return c->last_status;
}

// ---------------------------------------------------------------------------------
// kernel timing
// ---------------------------------------------------------------------------------
namespace ipc {

static void prof_flush(ipc_ctx *c, int k)
{
    auto &T = c->timers[k];
    if (T.ev.empty()) return;
    IPC_HIP(hipStreamSynchronize(c->stream));
    for (size_t i = 0; i + 1 < T.ev.size(); i += 2) {
        float ms = 0.0f;
        IPC_HIP(hipEventElapsedTime(&ms, T.ev[i], T.ev[i + 1]));
        T.total_ms += ms;
    }
    for (auto e : T.ev) T.pool.push_back(e);
    T.ev.clear();
}

static hipEvent_t prof_event(ipc_ctx *c, int k)
{
    auto &T = c->timers[k];
    if (T.pool.empty()) {
        hipEvent_t e;
        IPC_HIP(hipEventCreate(&e));
        return e;
    }
    hipEvent_t e = T.pool.back();
    T.pool.pop_back();
    return e;
}

void prof_begin(ipc_ctx *c, int k)
{
    if (!c->prof) return;
    hipEvent_t e = prof_event(c, k);
    IPC_HIP(hipEventRecord(e, c->stream));
    c->timers[k].ev.push_back(e);
}

void prof_dispatch_events(ipc_ctx *c, int k, hipEvent_t *start, hipEvent_t *stop, double bytes)
{
    *start = *stop = nullptr;
    if (!c->prof) return;
    auto &T = c->timers[k];
    // read the pending pairs first: the new pair is stamped only once its
    // launch has been issued
    if (T.ev.size() >= 2048) prof_flush(c, k);
    *start = prof_event(c, k);
    *stop = prof_event(c, k);
    T.ev.push_back(*start);
    T.ev.push_back(*stop);
    T.launches += 1;
    T.bytes += bytes;
}

void prof_end(ipc_ctx *c, int k, double bytes)
{
    if (!c->prof) return;
    hipEvent_t e = prof_event(c, k);
    IPC_HIP(hipEventRecord(e, c->stream));
    auto &T = c->timers[k];
    T.ev.push_back(e);
    T.launches += 1;
    T.bytes += bytes;
    if (T.ev.size() >= 2048) prof_flush(c, k);
}

} // namespace ipc

ipc_ctx::~ipc_ctx()
{
    for (auto &T : timers) {
        for (auto e : T.ev) (void)hipEventDestroy(e);
        for (auto e : T.pool) (void)hipEventDestroy(e);
    }
    for (auto &x : pcg_exec) if (x) (void)hipGraphExecDestroy(x);
    if (h_peek) (void)hipHostFree(h_peek);
    if (pin_rd) (void)hipHostFree(pin_rd);
    if (pin_wr) (void)hipHostFree(pin_wr);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
}

extern "C" int ipc_profile(ipc_ctx *c, int enable)
{
    if (!c) return IPC_E_INVALID;
    return guard(c, [&] {
        for (int k = 0; k < IPC_K_COUNT; ++k) {
            prof_flush(c, k);
            if (enable) { c->timers[k].total_ms = 0.0; c->timers[k].launches = 0; c->timers[k].bytes = 0.0; }
        }
        if (enable) {
            c->d.prof_bytes.alloc(1);
            c->d.prof_bytes.zero(c->stream, 1);
            std::vector<int> rng(3 * (size_t)c->n_scenes);
            for (int k = 0; k < c->n_scenes; ++k) {
                rng[3 * (size_t)k] = c->sc[k].node0;
                rng[3 * (size_t)k + 1] = c->sc[k].node0 + c->sc[k].nnode_pad;
                rng[3 * (size_t)k + 2] = c->sc[k].nnode;
            }
            c->d.prof_scene.upload(rng, c->stream);
        }
        c->prof = enable != 0;
    });
}

extern "C" int ipc_kernel_time(ipc_ctx *c, int kernel, double *total_ms, int64_t *launches, double *bytes)
{
    if (!c || kernel < 0 || kernel >= IPC_K_COUNT) return IPC_E_INVALID;
    return guard(c, [&] {
        prof_flush(c, kernel);
        if (total_ms) *total_ms = c->timers[kernel].total_ms;
        if (launches) *launches = c->timers[kernel].launches;
        if (bytes) *bytes = c->timers[kernel].bytes;
        if (bytes && kernel == IPC_K_SPMV && c->d.prof_bytes.p) {
            // counted per launch on the device: rows of stopped scenes are skipped
            double nb = 0.0;
            IPC_HIP(hipMemcpyAsync(&nb, c->d.prof_bytes.p, sizeof(nb), hipMemcpyDeviceToHost, c->stream));
            IPC_HIP(hipStreamSynchronize(c->stream));
            *bytes = nb;
        }
    });
}

extern "C" int ipc_autotune(ipc_ctx *c, int reps, double *us_host, int32_t *lanes_host)
{
    if (!c || reps < 1) return IPC_E_INVALID;
    return guard(c, [&] {
        bool prof = c->prof;
        c->prof = false;
        int keep = c->spmv_lanes;
        autotune_spmv(c, reps, us_host);
        if (c->spmv_lanes_forced) c->spmv_lanes = keep;
        autotune_fem(c, reps);
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            auto it = g_tuned.find(tune_key(c));
            Tuned t = it != g_tuned.end() ? it->second : Tuned{8, BLOCK, BLOCK, BLOCK};
            if (!c->spmv_lanes_forced) t.lanes = c->spmv_lanes;   // a fixed lane count is not a choice
            t.fem_block = c->fem_block;
            t.asm_block = c->asm_block;
            t.grad_block = c->grad_block;
            g_tuned[tune_key(c)] = t;
        }
        c->prof = prof;
        if (lanes_host) *lanes_host = c->spmv_lanes;
    });
}

extern "C" int ipc_time_kernel(ipc_ctx *c, int kernel, int reps, double *avg_us, double *bytes)
{
    if (!c || reps < 1 || !avg_us || kernel != IPC_K_SPMV) return IPC_E_INVALID;
    return guard(c, [&] {
        Dev &D = c->d;
        hipEvent_t e0, e1;
        IPC_HIP(hipEventCreate(&e0));
        IPC_HIP(hipEventCreate(&e1));
        bool prof = c->prof;
        c->prof = false;
        // one warm launch, then the timed batch: q = H p on the current matrix
        hess_apply(c, D.p.p, D.q.p, nullptr, nullptr);
        IPC_HIP(hipEventRecord(e0, c->stream));
        for (int k = 0; k < reps; ++k) hess_apply(c, D.p.p, D.q.p, nullptr, nullptr);
        IPC_HIP(hipEventRecord(e1, c->stream));
        IPC_HIP(hipEventSynchronize(e1));
        c->prof = prof;
        float ms = 0.0f;
        IPC_HIP(hipEventElapsedTime(&ms, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        *avg_us = 1e3 * ms / reps;
        if (bytes) *bytes = spmv_bytes(c);
    });
}
