// Internal declarations of the IPC Newton-step library (gfx950).
//
// Device data is laid out structure-of-arrays over all scenes.  Node ranges
// (FEM vertices, then 4 pseudo-nodes per affine body) and tetrahedron ranges
// of every scene are padded to a multiple of TILE = 64 (one wavefront), so a
// wavefront never straddles two scenes: reductions write one partial per
// wavefront and a per-scene pass sums a scene's partials in a fixed order,
// which keeps energies and dot products bit-reproducible run to run.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "../../include/ipc.h"

namespace ipc {

constexpr int TILE = 64;      // wavefront size on CDNA
constexpr int BLOCK = 256;    // default workgroup: 4 wavefronts
constexpr int CG_AGG = 32;    // coarse preconditioner: nodes per group
constexpr int CG_DOM = 32;    // groups per coarse domain
constexpr int CG_N = 3 * CG_DOM;   // coarse unknowns per domain
constexpr int CG_SPLIT = 4;   // workgroups (row slices of the inverse) per domain in the apply
constexpr int CG_MIN_NODES = 32768;  // contexts from this size apply it by default
constexpr int LONG_ROW = 64;  // rows with more blocks go to the wavefront-per-row path
constexpr int TRAV_STASH = 16;   // broad phase: candidates a query keeps from its counting pass

// per-scene device scalar slots
enum Slot {
    S_E = 0,        // energy (sum over terms)
    S_NEWTON_MAX,   // Newton measure (max world displacement of p)
    S_CCD,          // CCD step bound (stored through its bit pattern, atomic min)
    S_LS_ALPHA,     // line-search step of the scene
    S_LS_ON,        // 1 while the scene takes part in the current Newton iteration
    S_INF,          // 1 when some pair has d <= 0
    S_E_IN, S_E_FEM, S_E_ABD, S_E_SP, S_E_BAR, S_E_FR,
    S_E0,           // line search: energy at the current iterate
    S_NEWTON_ON,    // 1 while the scene's Newton loop runs
    S_INDEF,        // 1 when the scene's PCG met p.Ap <= 0
    S_MUBAR,        // adjoint: w . dG/dmu of the last step
    S_DMIN,         // adaptive kappa: smallest squared distance over the active pairs (bit pattern, atomic min)
    S_DPREV,        // adaptive kappa: smallest distance at the previous iterate
    S_KAPPA0,       // adaptive kappa: the scene's kappa when the rule was switched on
    NSLOT
};

// per-scene segment tables (device, n_scenes + 1 entries each)
enum Region {
    R_NODEW = 0,    // wavefront tiles of nodes
    R_TETW,         // wavefront tiles of tetrahedra
    R_BODY, R_SP, R_SURF, R_TRI, R_EDGE,
    R_CPT, R_CEE,   // candidates
    R_PT, R_EE,     // active pairs
    R_LPT, R_LEE,   // friction lag lists
    R_LONG,         // rows of the product handled one wavefront per row
    R_CDOM,         // domains of the coarse preconditioner
    R_HS,           // vertices that meet the scene's half-space
    NREGION
};

// per-scene parameters (device, 8 per scene)
enum Param { P_H2 = 0, P_KAPPA = 1, P_DHAT = 2, P_MU = 3, P_EPSH = 4, P_CCDS = 5, P_H = 6, P_ETA = 7 };

struct RedSrc {
    const double *v;
    const int *seg;
    int off;
    int base;
    const double *w64 = nullptr;   // optional sums of v[64 k .. 64 k + 63] (whole chunks are read from here)
};
constexpr int RED_MAX = 10;
// Per-scene reduction of up to RED_MAX sources.  Each source's sum can be stored in
// its own slot; the sources of group g (grp[k] = g) are combined in source
// order into the slot of that group (slot, slot1, slot2).
struct RedArgs {
    RedSrc src[RED_MAX];
    int nsrc = 0;
    int slot = -1;          // total of group 0 (-1: none)
    int slot1 = -1;         // total of group 1
    int slot2 = -1;         // total of group 2
    int acc = 0;            // accumulate into the group-0 slot
    int slots[RED_MAX] = {-1, -1, -1, -1, -1, -1, -1, -1, -1, -1};   // per-source sums (-1: none)
    int grp[RED_MAX] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};             // group of each source (-1: none)
    int op = 0;             // 0 sum, 1 max
    int total = -1;         // slot of the combination of every source in source order (-1: none)
};

#define IPC_HIP(call)                                                           \
    do {                                                                        \
        hipError_t e_ = (call);                                                 \
        if (e_ != hipSuccess) throw ipc::Error(IPC_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

struct Error {
    int code;
    std::string msg;
    Error(int c, std::string m) : code(c), msg(std::move(m)) {}
};

// Device memory of a context created over a caller's workspace
// (ipc_create_ws): sub-ranges handed out first fit from a free list, with
// neighbours merged on release, so that no hipMalloc is made.  Every use of a
// range is ordered on the context's stream, so a released range can be handed
// out again at once.
struct Arena {
    char *base = nullptr;
    size_t size = 0, used = 0, peak = 0;
    std::map<size_t, size_t> free;   // offset -> bytes
    void init(void *b, size_t bytes)
    {
        base = (char *)b; size = bytes; used = peak = 0;
        free.clear();
        if (bytes) free[0] = bytes;
    }
    static size_t round(size_t bytes) { return (bytes + 255) & ~(size_t)255; }
    void *take(size_t bytes)
    {
        bytes = round(bytes);
        for (auto it = free.begin(); it != free.end(); ++it) {
            if (it->second < bytes) continue;
            size_t off = it->first, sz = it->second;
            free.erase(it);
            if (sz > bytes) free[off + bytes] = sz - bytes;
            used += bytes;
            peak = std::max(peak, used);
            return base + off;
        }
        return nullptr;
    }
    void give(void *p, size_t bytes)
    {
        bytes = round(bytes);
        size_t off = (size_t)((char *)p - base);
        used -= bytes;
        auto nx = free.lower_bound(off);
        if (nx != free.end() && off + bytes == nx->first) { bytes += nx->second; nx = free.erase(nx); }
        if (nx != free.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == off) { pv->second += bytes; return; }
        }
        free[off] = bytes;
    }
};
// The arena of the context whose call is running on this thread (null: the
// context allocates with hipMalloc).
extern thread_local Arena *g_arena;
struct ArenaScope {
    Arena *prev;
    explicit ArenaScope(Arena *a) : prev(g_arena) { g_arena = a; }
    ~ArenaScope() { g_arena = prev; }
};

template <class T>
struct DBuf {
    T *p = nullptr;
    size_t n = 0;
    Arena *from = nullptr;   // the arena the range came from (null: hipMalloc)
    DBuf() = default;
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    ~DBuf() { release(); }
    void release()
    {
        if (p) {
            if (from) from->give(p, n * sizeof(T));
            else (void)hipFree(p);
        }
        p = nullptr;
        n = 0;
        from = nullptr;
    }
    void alloc(size_t count)
    {
        if (count <= n && p) return;
        release();
        if (count == 0) count = 1;
        if (g_arena) {
            p = (T *)g_arena->take(count * sizeof(T));
            if (!p)
                throw Error(IPC_E_CAPACITY, "workspace exhausted: " + std::to_string(Arena::round(count * sizeof(T))) +
                                                " more bytes needed (" + std::to_string(g_arena->used) + " of " +
                                                std::to_string(g_arena->size) + " in use); plan a larger capacity");
            from = g_arena;
        } else {
            IPC_HIP(hipMalloc(&p, count * sizeof(T)));
        }
        n = count;
    }
    void upload(const std::vector<T> &h, hipStream_t s)
    {
        alloc(h.size());
        if (!h.empty()) IPC_HIP(hipMemcpyAsync(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
    }
    void zero(hipStream_t s, size_t count)
    {
        if (count) IPC_HIP(hipMemsetAsync(p, 0, count * sizeof(T), s));
    }
};

struct SceneInfo {
    // sizes
    int nv, nt, nb, nbv, nbt, nsv, nst, nobj, nex, ns, nd, nj;
    // offsets into the concatenated device arrays
    int node0, nnode, nnode_pad;     // nodes: FEM region then 4 per body (nnode: without padding)
    int bnode0;                      // first body node: node0 + nv + nb rounded up to 4, so that a
                                     // body's 4 nodes are 4 lanes of one wavefront
    std::vector<int> entry;          // the FEM region's nv + nb slots in Morton order: FEM vertex
                                     // entry[m] at node0 + m, or -1 - b for body b's translation
    int tet0, nt_pad;
    int body0, drv0, sp0, jt0;       // bodies, driven slots, springs, joint springs
    int cv0, ncv, nsurf;             // contact vertices; the first nsurf are PT query points
    int tri0, ntri, edge0, nedge;
    int obj0;
    int64_t dof0;                    // external DOF offset
    // parameters
    double h, g[3], dhat, kappa, mu, eps_v, newton_tol, pcg_tol, ccd_s;
    int max_newton, max_pcg;
    double L, thr, mbar;
    double hs[4];                    // half-space (n, c); hs_on when n != 0
    bool hs_on;
    // host topology in the scene's vertex numbering (for the pair export)
    std::vector<int> tri_ext, edge_ext, surf_ext;
};

struct Dev {
    // nodes
    DBuf<double> y, ydot, xt, y0, yt, g, p, r, z, q, w, x, v1, v2;
    DBuf<double> r2, z2, q2;               // the PCG's r, z and s of odd iterations (one-launch step)
    DBuf<int> node_scene, node_kind;       // kind: 0 FEM, 1 body node, 2 padding
    DBuf<int> slot_scene;                  // scene of each block-CSR block (its row's)
    DBuf<double> mass;                     // lumped FEM vertex mass (0 elsewhere)
    DBuf<double> dinv;                     // 3x3 inverse diagonal block per node
    DBuf<int> ext2node;                    // external node -> internal node
    // tetrahedra (SoA over the padded tet range)
    DBuf<int4> tv;
    DBuf<double> Bm;                       // 9 arrays of nT
    DBuf<double> vol, tmu, tlam;
    DBuf<double> tE, tnu;                  // Young's modulus and Poisson ratio per tet
    DBuf<int> ext2tet;                     // external tet (scenes concatenated) -> internal tet
    // FEM assembly by gathering: each tet writes its gradient ([a][tet][3]) and
    // its 16 3x3 blocks ([a*4+b][tet][9]); nodes and matrix slots then sum
    // their contributions in a fixed order
    DBuf<double> tgrad, telem;
    DBuf<int> fadj_ptr, fadj;              // node -> incident (tet, local vertex) codes 4 tet + a
    DBuf<int> sc_ptr, sc_list;             // matrix slot -> contributing codes 16 tet + 4 a + b
    // FEM matrix (block CSR, 3x3 blocks, rows = nodes)
    DBuf<int> row_ptr, col, diag_slot;
    DBuf<double> val, val_const;           // assembled values; constant part (mass, springs)
    DBuf<int> bslot, long_rows;            // 16 body-block slots per body; rows with > LONG_ROW blocks in all
    DBuf<int> long_count;                  // number of long rows (read by the product's extra workgroups)
    // pair-local contact blocks, sorted by row: extra blocks of the product
    DBuf<int> dyn_ptr, dyn_row, dyn_col, dyn_cnt, dyn_off, dyn_idx, dyn_idx2, dyn_head, dyn_pos, dyn_start;
    DBuf<unsigned long long> dyn_key64, dyn_key64b;   // (row << 32 | column) before / after the sort
    DBuf<double> dyn_val, dyn_val_coo;
    DBuf<double> part_node3, part_long;    // product dot partials (per wavefront of nodes / per long row)
    // bodies
    DBuf<double> bM;                       // 4x4 mass matrix per body
    DBuf<double> bvol, bkappa, bext;
    DBuf<int> body_node0, body_scene;
    DBuf<double> dinvB;
    // springs
    DBuf<int> sp_ka, sp_ia, sp_kb, sp_ib, sp_scene;
    DBuf<double> sp_xa, sp_xb, sp_k;
    DBuf<double> targets;                  // 12 per driven slot
    DBuf<int> joint_sp;                    // spring of every joint slot (its b-side point follows the joint reference)
    DBuf<int> driven_body;
    DBuf<double> sp_part;                  // per-spring values for reductions
    DBuf<double> body_part;
    // contact vertices, triangles, edges
    DBuf<int> cv_node, cv_body, cv_obj, cv_scene;
    DBuf<double> cv_x;                     // body-frame point or static world point
    DBuf<double> xw, xw1;                  // world positions at y and at y + p
    DBuf<int4> tri;                        // (cv0, cv1, cv2, scene)
    DBuf<int2> edge;
    DBuf<double> edge_rest2;
    DBuf<int> obj_kind, excl;              // global object ids
    // broad phase (LBVH per scene and primitive kind)
    DBuf<double> box;                      // 6 per primitive (lo, hi)
    DBuf<unsigned long long> mkey, mkey2;
    DBuf<int> mid, mid2;
    DBuf<int> bvh_left, bvh_right, bvh_flag;
    DBuf<int2> bvh_range;                  // sorted-leaf range of every internal node
    DBuf<double> bvh_box, bvh_lev;         // node boxes; union tree over the sorted leaf boxes
    DBuf<int> bvh_moving, bvh_mscan, bvh_nmoving;   // moving-primitive flag per sorted leaf, its scan; per node
    DBuf<int> qcount, qoff;                // per-query candidate counts and offsets
    DBuf<int2> qstash;                     // first candidates of every query from the counting pass
    DBuf<unsigned long long> qkey, qkey2;  // surface-vertex query keys before / after the sort
    DBuf<int> qid, qperm;                  // query order (Morton-sorted surface vertices)
    DBuf<unsigned char> sort_tmp;
    DBuf<double> scene_lo;                 // Morton quantisation box per scene (6)
    // candidates and active pairs
    DBuf<int2> cand_pt, cand_ee;
    DBuf<double> cand_ref;                 // kept candidates: swept box of every contact vertex (lo, hi)
    DBuf<int> cand_flag;                   // per scene: 1 when the kept candidates no longer cover the sweep
    DBuf<int2> pt, ee;
    DBuf<int> wcount, woff;
    DBuf<double> pair_part;                // per-pair reduction values
    DBuf<double> pair_w64, fr_w64;         // their sums over chunks of 64 (pairs; friction lag pairs)
    DBuf<int4> pair_cv;                    // 4 contact vertices per active pair (PT then EE)
    DBuf<double> pair_H;                   // 45 per pair: projected reduced Hessian
    // friction lag
    DBuf<int4> lag_cv;
    DBuf<double> lag_beta, lag_nrm, lag_lam, lag_rn;
    DBuf<double> lag_M;                    // 6 (symmetric 3x3) per lag pair, scaled
    DBuf<int> lag_type;                    // distance type at the lag state
    DBuf<double> lag_ex;                   // edge-edge mollifier threshold (0 for PT)
    DBuf<int> lag_merge;                   // 1: all blocks of the lag pair are in the block-CSR pattern
    DBuf<int> lag_key, lag_code;           // 16 per lag pair: block slot (nnzb: none) and 16 i + 4 k + l
    DBuf<int> lag_key2, lag_code2;         // the same sorted by slot (stable)
    DBuf<unsigned char> lag_sort_tmp;
    // scalars and partials
    // half-space ground: entries (moving surface vertices of scenes with
    // one), the planes, per-entry energies, lag data, Hessian blocks and
    // their sorted slot entries, lagged contacts per scene
    DBuf<int> hs_cv, hs_key, hs_code, hs_key2, hs_code2, hs_nlag;
    DBuf<double> hs_plane, hs_part, hs_fpart, hs_w64, hs_fw64, hs_lam, hs_xn, hs_H;
    DBuf<double> scal;                     // n_scenes x NSLOT
    DBuf<double> part_node, part_tet;      // one partial per wavefront
    DBuf<int> seg;                         // scratch segment offsets (broad phase)
    DBuf<int> segs;                        // NREGION tables of n_scenes + 1
    DBuf<int> tile_scene_node, tile_scene_tet;
    DBuf<double> fr_part;
    DBuf<double> sparam, h2s;              // per-scene parameters
    DBuf<int> inf_flag, ls_active, pcg_iters, maxpcg, newton_on;
    DBuf<int> is_trans, node_body;         // first node of an affine body: 1 / the body's index (else 0 / -1)
    // conjugate-gradient state, two parity buffers: per scene {gamma, alpha,
    // eta^2 b.b, r.r}, running flag and update count; per-tile partials of
    // r.z and r.r
    DBuf<double> pcg_st, pcg_part, pcg_prev;   // pcg_prev: r.r at the previous peek
    DBuf<double> prof_bytes;               // profiled products: the algorithmic bytes they moved (1 counter)
    DBuf<int> prof_scene;                  // per scene: first row, end row, real nodes (for that count)
    DBuf<int> pcg_wginfo;                  // per step workgroup: scenes and the first scene's ranges (8 ints)
    // coarse preconditioner: per domain its entry range (ent, n_cdom + 1) into
    // the node list (groups of CG_AGG consecutive entries), its scene, its
    // inverse (CG_N x CG_N) and r . z partials of both parities; per node
    // domain * CG_DOM + group, or -1 for nodes outside every group
    DBuf<int> cg_ent, cg_nodes, cg_node_da, cg_dom_scene;
    DBuf<int> cg_grp;                      // per group: domain * CG_DOM + group in the domain
    DBuf<int> cg_pnodes;                   // per domain its node list padded to CG_AGG * CG_DOM entries (-1 after the end)
    DBuf<int> cg_ph_ptr, cg_ph_e, cg_ph_n; // one-launch step: per domain its entries that stand for a body (entry, node)
    DBuf<double> cg_inv, cg_part;
    DBuf<int> pcg_act, pcg_it;
    DBuf<int> pair_flag, lag_flag;         // 1: the pair's blocks were merged into the matrix
    DBuf<int> tickets;                     // small device counters
    DBuf<double> grav;
    DBuf<double> red_tmp;
    // deterministic scatters: sorted (key, code) entries summed per run of
    // equal keys (ipc_runsum.h) instead of floating-point atomics
    DBuf<double> rs_first, rs_last;        // per-wavefront pieces of runs crossing wavefront boundaries
    DBuf<double> pair_g;                   // barrier: world gradient of each pair vertex (12 per pair)
    DBuf<int> pg_key, pg_code, pg_key2, pg_code2;   // 4 per pair: contact vertex (CV: static) / 4 i + k, unsorted and sorted
    DBuf<int> pb_key, pb_code, pb_key2, pb_code2;   // 16 per pair: matrix slot (nnzb: none) / 16 i + 4 k + l
    DBuf<double> lag_g;                    // friction (and its adjoint): per lag-pair vertex values (12 per pair)
    DBuf<int> lg_key, lg_code, lg_key2, lg_code2;   // 4 per lag pair, sorted by contact vertex once per lag
    DBuf<double> gcv;                      // contact-vertex sums (3 per contact vertex)
    DBuf<int> body_cv_ptr, body_cv;        // contact vertices of every body (CSR over bodies)
    DBuf<double> sp_f;                     // spring force h^2 k (a - b) per spring
    DBuf<int> spg_key, spg_code;           // spring gradient entries sorted by node: code 8 s + 4 side + q
    int64_t n_spg = 0;
    DBuf<int> spc_key, spc_code;           // constant spring blocks sorted by slot: code 64 s + 8 i + j
    int64_t n_spc = 0;
    DBuf<int> int2ext, bsr_cnt;            // matrix export: internal -> external node, blocks per exported row
};

} // namespace ipc

struct ipc_ctx {
    hipStream_t stream = nullptr;
    int n_scenes = 0;
    std::vector<ipc::SceneInfo> sc;
    int64_t ndof = 0;
    int N = 0, T = 0, NB = 0, NS = 0, ND = 0, NJ = 0, CV = 0, NSURF = 0, TRI = 0, EDGE = 0, NOBJ = 0, NEX = 0;
    int64_t NFEM = 0, TREAL = 0;   // real FEM vertices and tetrahedra over all scenes
    int nnzb = 0, nnzb_fem = 0, n_long = 0;
    int long_cap = 0;                     // long-row workgroups the product launches (grows, multiple of 64)
    int64_t n_dyn = 0, cap_dyn = 0;       // pair-local blocks of the last assembly (merged), capacity
    int spmv_lanes = 8;                   // lanes per row of the product (autotuned)
    bool spmv_lanes_forced = false;       // set by IPC_SPMV_LANES: the autotuner times but keeps it
    int fem_block = ipc::BLOCK, asm_block = ipc::BLOCK, grad_block = ipc::BLOCK;   // workgroups of k_fem, k_bsr_assemble, k_fem_grad_gather (autotuned)
    bool coarse = true;                   // coarse domains built (the PCG preconditioner's correction)
    bool coarse_on = false;               // the PCG applies the coarse correction
    bool coarse_forced = false;           // on by request, whatever the size
    bool cg_fusable = false;              // one scene whose domains match the step's workgroups (see coarse_setup)
    int cg_nfr = 0;                       // its entries (FEM vertices and body translations)
    bool pcg_fused = true;                // IPC_NO_FUSED_PCG unset: a fusable context applies its coarse
                                          // correction inside the PCG step
    int lag_passes = 1;                   // friction lag passes per step
    double kappa_frac = 0.0;              // adaptive kappa: distance threshold / dhat (0: off)
    double kappa_factor = 100.0;          // adaptive kappa: cap / kappa0
    int n_cdom = 0, n_cgrp = 0;           // its domains and groups over all scenes
    std::vector<int> seg_cdom;            // per scene: first domain (n_scenes + 1)
    int64_t ext_nodes = 0;
    int64_t ext_tets = 0;
    // host copies of segment tables
    std::vector<int> seg_surf, seg_tri, seg_edge, seg_sp, seg_body, seg_hs;
    int64_t M_HS = 0;                      // half-space entries: moving surface vertices of scenes with one
    // dynamic counts
    int64_t cap_cand_pt = 0, cap_cand_ee = 0, n_cand_pt = 0, n_cand_ee = 0;
    int64_t cap_pt = 0, cap_ee = 0, n_pt = 0, n_ee = 0, cap_lag = 0, n_lag = 0;
    std::vector<int> h_cand_pt_seg, h_cand_ee_seg, h_pt_seg, h_ee_seg, h_lag_seg;
    ipc::Arena ws;                        // the caller's workspace (ipc_create_ws); empty: hipMalloc
    ipc::Dev d;                           // (declared after ws: released into it before it goes)
    bool step_ready = false;
    bool fr_on = true;
    // per-scene flags (device, nullable): while set, the FEM assembly, the
    // block-CSR values, the preconditioner blocks and the coarse blocks are
    // formed for the flagged scenes only (a batch's Newton iterations after
    // some scenes have converged); the others keep stale values they never use
    const int *assemble_only = nullptr;
    bool use_graphs = true;              // PCG iterations replayed from a captured graph
    int trace_scene = -1;                // IPC_TRACE_NEWTON: the scene whose Newton iterations go to stderr
    bool floor_stop = true;              // the Newton stop at the energy's rounding floor (IPC_NO_FLOOR_STOP=1: off)
    hipStream_t cap_stream = nullptr;    // private stream used only for graph capture
    // PCG batch graphs, reused while every launch argument they captured is unchanged
    std::vector<uintptr_t> pcg_key;
    hipGraphExec_t pcg_exec[4] = {nullptr, nullptr, nullptr, nullptr};   // [batch length][copy]
    unsigned long long *h_peek = nullptr;       // pinned, coherent host memory: 2 slots of one word per scene
    unsigned long long *h_peek_dev = nullptr;   // its device address
    unsigned int peek_seq = 0;
    // pinned host staging: a readback arena (one HostReads at a time) and an upload ring
    char *pin_rd = nullptr, *pin_wr = nullptr;
    size_t pin_wr_off = 0;
    int64_t n_lag_pt = 0, n_local = 0;
    bool cand_cached = false;            // the candidate lists are a kept superset (valid while cand_check passes)
    int last_status = 0;
    // host staging for small uploads (kept alive until the copy has completed)
    std::vector<double> h_scal_stage;
    std::vector<int> h_seg_stage, h_int_stage;
    // kernel timing (HIP events on the context's stream, only while enabled)
    struct Timer {
        std::vector<hipEvent_t> ev;      // start/stop pairs not yet read
        std::vector<hipEvent_t> pool;
        double total_ms = 0.0;
        int64_t launches = 0;
        double bytes = 0.0;              // algorithmic bytes of the launches counted
    };
    bool prof = false;
    Timer timers[IPC_K_COUNT];
    ~ipc_ctx();
    std::string err;
};

namespace ipc {

// ---- helpers implemented in the .hip files ---------------------------------
// plan (non-null): only the host half; *plan = the device bytes a workspace
// context takes for the capacity caps = {pairs, candidates, pair-local blocks}
void create_context(ipc_ctx *c, const ipc_scene_desc *scenes, int n, const int64_t *caps = nullptr, size_t *plan = nullptr);
// size every contact-state buffer for that capacity (workspace contexts)
void reserve_capacity(ipc_ctx *c, int64_t max_pairs, int64_t max_candidates, int64_t max_local_blocks);
// host checks of the scene data (throws Error(IPC_E_INVALID, ...)); no HIP call
void validate_scenes(const ipc_scene_desc *scenes, int n);
void reduce(ipc_ctx *c, const RedArgs &a);
// w[k] = sum of v[64 k .. 64 k + 63] (entries past n count as 0), k < ceil(n / 64)
void sum64(ipc_ctx *c, const double *v, int64_t n, double *w);
RedSrc src(const double *v, const int *seg, int off, int base);
int *seg_ptr(ipc_ctx *c, int region);
void prof_begin(ipc_ctx *c, int k);
void prof_end(ipc_ctx *c, int k, double bytes);
// While timing is enabled: two events for a launch that stamps them itself at
// its start and end (hipExtLaunchKernelGGL), counted as one launch of kernel
// k with the given algorithmic bytes; both stay null when timing is off.
void prof_dispatch_events(ipc_ctx *c, int k, hipEvent_t *start, hipEvent_t *stop, double bytes);
__global__ void k_fill_int_api(int n, int *p, int v);
void hess_apply(ipc_ctx *c, const double *v, double *out, const int *active, double *part);
void autotune_spmv(ipc_ctx *c, int reps, double *us);
double spmv_bytes(const ipc_ctx *c);
void build_preconditioner(ipc_ctx *c);
// coarse correction of the preconditioner: groups and domains from node
// positions at creation; the domains' inverses after an assembly; z += its
// correction of r for the scenes whose act entry is set, r . z partials into
// the given parity
void coarse_setup(ipc_ctx *c);
void coarse_build(ipc_ctx *c);
void coarse_apply(ipc_ctx *c, const int *act, const double *r, double *z, int parity);

void pcg_solve(ipc_ctx *c, const double *b, double *x, double eta, const int *want);
// exclusive scan of n ints into out[0..n] (out[n] = total), on the context's stream
void exclusive_scan_int(ipc_ctx *c, const int *in, int *out, int n);
void pcg_wginfo(ipc_ctx *c);
// constant part of the matrix (lumped mass, spring blocks) from the current
// spring points; h2s: h^2 per scene
void build_const_part(ipc_ctx *c, const double *h2s);   // refresh the step workgroups' scene records (after the long rows change)

// Several device values to the host with one synchronisation, staged in the
// context's pinned readback arena (asynchronous copies); reads that do not
// fit go straight to their destination.  One instance at a time per context.
struct HostReads {
    ipc_ctx *c;
    size_t used = 0;
    struct Item { void *dst; size_t off, bytes; };
    std::vector<Item> items;
    explicit HostReads(ipc_ctx *cc);
    void add(void *dst, const void *src, size_t bytes);
    void wait();
};
// host -> device copy through the context's pinned upload ring (asynchronous;
// the host data may be reused as soon as the call returns)
void upload_async(ipc_ctx *c, void *dst_dev, const void *src, size_t bytes);

// launch helper
inline int blocks_for(int64_t n, int bs = BLOCK) { return (int)((n + bs - 1) / bs); }

} // namespace ipc
