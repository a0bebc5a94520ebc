/*
 * ipc.h - C-ABI of the MI355X (gfx950) IPC Newton-step library.
 *
 * The library advances one or more independent scenes by one implicit step
 * each call, minimising the incremental potential of PhyVisGen Eq. (3)
 * (Sec. III-C.2):
 *     E = E_inertia + E_barrier + E_friction + E_FEM + E_ABD
 *       + E_joint(q_ref) + E_couple,         E_couple = E_fixed + E_stitch (Eq. (1)),
 * with E_stitch the attachment springs of Eq. (2), over all degrees of freedom
 * jointly (the arm links, the rigid gripper parts, the soft fingertips and the
 * manipulated objects).  The state a call returns is the physical record of
 * Eq. (4): FEM vertex positions and affine-body states.
 *
 * Conventions shared by every entry point
 *  - Units SI, FP64 throughout.
 *  - DOF vector layout ("external layout"): scenes concatenated in creation
 *    order; within a scene, the FEM vertices (x, y, z each) followed by the
 *    affine bodies, 12 numbers per body: translation p, then the three columns
 *    of the affine matrix A.  A body point with body-frame coordinates xb sits
 *    at p + xb0 A[:,0] + xb1 A[:,1] + xb2 A[:,2].
 *  - Pointers named *_dev are device pointers (HIP global memory of the device
 *    the context was created on); *_host are host pointers.  The caller owns
 *    every buffer it passes; the library reads or writes it only during the
 *    call, stream-ordered on the context's stream.
 *  - Every call returns an int status.  On error the context keeps a message
 *    readable through ipc_last_error().  No C++ exception crosses the ABI.
 */
#ifndef IPC_H
#define IPC_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    IPC_OK = 0,
    IPC_E_INVALID = 1,        /* bad argument or scene data (checked on the host)      */
    IPC_E_CAPACITY = 2,       /* a size limit was exceeded                              */
    IPC_E_NOT_CONVERGED = 3,  /* Newton hit max_newton; the state holds the last iterate */
    IPC_E_LINESEARCH = 4,     /* no decrease after 40 halvings                           */
    IPC_E_INTERSECTING = 5,   /* a contact pair has zero distance                        */
    IPC_E_INDEFINITE = 6,     /* adjoint PCG met p^T H p <= 0                            */
    IPC_E_DEVICE = 7          /* a HIP runtime call failed                               */
};

/* Host description of one scene.  Arrays are host pointers with the layouts
 * below; they are copied by ipc_create() and may be freed afterwards.
 *
 *  FEM tetrahedra (Sec. III-C.1, Stable Neo-Hookean material)
 *    X[nv*3], V[nv*3]      rest (= initial) positions and initial velocities
 *    tets[nt*4]            vertex indices, det[X1-X0,X2-X0,X3-X0] > 0 required
 *    tet_E, tet_nu, tet_rho[nt]  Young's modulus (> 0), Poisson ratio in (0, 0.5),
 *                          density (> 0)
 *    vobj[nv]              object id of each FEM vertex
 *  Affine bodies (rigid parts, arm links, rigid objects; affine body dynamics)
 *    body_q, body_qdot[nb*12]  state (p, A[:,0..2]) and its rate
 *    body_mass[nb], body_S[nb*9]  mass and second moment of mass (row-major
 *                          3x3) about the frame origin, which must be the centroid
 *    body_vol, body_kappa[nb]  volume and orthogonality stiffness
 *    body_ext[nb*3]        half extents of the body box (convergence measure)
 *    body_obj[nb]          object id
 *  Contact geometry
 *    bv_xbar[nbv*3], bv_body[nbv], btri[nbt*3]  body-frame surface vertices of
 *                          bodies and their outward triangles (body-vertex indices)
 *    sv_x[nsv*3], stri[nst*3]  static world geometry
 *    obj_kind[nobj]        0 FEM mesh, 1 affine body, 2 static
 *    excl[nex*2]           object pairs that never collide
 *  Springs E = h^2 k/2 |a - b|^2: stitch springs (Eq. (2)), fixed joints and
 *  joint drives toward per-step link targets
 *    sp_ka, sp_kb[ns]      side kind: 0 FEM vertex, 1 body point, 2 drive target
 *    sp_ia, sp_ib[ns]      FEM vertex / body / driven-link slot
 *    sp_xa, sp_xb[ns*3]    body-frame point (kind 1) or link-frame anchor (kind 2)
 *    sp_k[ns]              stiffness (N/m)
 *    driven_body[nd]       body driven by slot d
 *  Parameters
 *    h time step; g gravity; dhat barrier threshold; kappa barrier stiffness
 *    (<= 0: 10 * mean FEM vertex mass * |g| * h^2 / dhat); mu friction;
 *    eps_v friction velocity threshold; newton_tol (stop when the largest world
 *    displacement of the Newton direction is below newton_tol * h * L, L the
 *    initial bounding-box diagonal); pcg_tol (relative residual); ccd_s (CCD
 *    gap fraction); max_newton, max_pcg iteration caps. */
typedef struct ipc_scene_desc {
    int32_t nv, nt, nb, nbv, nbt, nsv, nst, nobj, nex, ns, nd;
    const double *X, *V;
    const int32_t *tets;
    const double *tet_E, *tet_nu, *tet_rho;
    const int32_t *vobj;
    const double *body_q, *body_qdot, *body_mass, *body_S, *body_vol, *body_kappa, *body_ext;
    const int32_t *body_obj;
    const double *bv_xbar;
    const int32_t *bv_body, *btri;
    const double *sv_x;
    const int32_t *stri, *obj_kind, *excl;
    const int32_t *sp_ka, *sp_ia;
    const double *sp_xa;
    const int32_t *sp_kb, *sp_ib;
    const double *sp_xb, *sp_k;
    const int32_t *driven_body;
    double h, g[3], dhat, kappa, mu, eps_v, newton_tol, pcg_tol, ccd_s;
    int32_t max_newton, max_pcg;
    /* joint-space drives (E_joint of Eq. (3)): nj springs whose b side is a
     * body point that follows the joint reference; their b-side body-frame
     * points arrive with every step's targets (see ipc_begin_step) */
    int32_t nj;
    const int32_t *joint_spring;   /* nj spring indices (b side of kind 1) */
    /* an analytic half-space ground {x : n . x >= c}, half_space = (n, c) with
     * n a unit normal (|n|^2 within 1e-12 of 1), or n = 0 for none.  Every
     * moving surface vertex (FEM or body) meets it with the barrier of
     * Sec. III-C.1 on d = n . x - c, its lagged friction (normal n, tangent
     * displacement (I - n n^T)(x - x^n)) and an exact CCD bound (the step at
     * which d reaches ccd_s times its start value on the straight path). */
    double half_space[4];
} ipc_scene_desc;

/* Per-scene statistics of the last ipc_step(). */
typedef struct ipc_stats {
    int32_t status;            /* IPC_OK or the scene's error code                 */
    int32_t newton_iters;
    int32_t pcg_iters_total;
    int32_t pcg_iters_max;
    int32_t n_pt_max, n_ee_max;  /* active pairs, max over Newton iterations    */
    int32_t n_lag;             /* friction pairs lagged at the step start         */
    int32_t n_cand_max;        /* CCD candidates, max over Newton iterations      */
    double alpha_min;          /* smallest accepted line-search step              */
    double energy;             /* potential at the final iterate                  */
} ipc_stats;

typedef struct ipc_ctx ipc_ctx;

/* Size queries (ipc_query). */
enum {
    IPC_Q_NDOF = 0,       /* DOFs of all scenes (external layout)             */
    IPC_Q_NSCENES = 1,
    IPC_Q_NDRIVEN = 2,    /* driven-link slots of all scenes                  */
    IPC_Q_NTRI = 3,       /* contact triangles of all scenes                   */
    IPC_Q_NEDGE = 4,
    IPC_Q_NNODES = 5,     /* internal padded node count                        */
    IPC_Q_NTETS = 6,      /* internal padded tetrahedron count                 */
    IPC_Q_NLOCAL = 7,     /* contact entries (barrier + friction) of the last
                             assembly that stay pair-local, i.e. whose blocks
                             did not fit the matrix pattern                      */
    IPC_Q_NPAIRS = 8,     /* active barrier pairs of the last assembly         */
    IPC_Q_NTETS_EXT = 9,  /* tetrahedra of all scenes (external numbering)     */
    IPC_Q_COARSE = 10,    /* 1 when the PCG preconditioner applies its coarse
                             correction: for contexts of at least 32768 nodes
                             (its cost per iteration is a fixed few
                             microseconds); the environment variable
                             IPC_PCG_COARSE = 0 or 1, read at ipc_create,
                             switches it off or on whatever the size       */
    IPC_Q_WS_BYTES = 11,  /* workspace size of an ipc_create_ws context (0: the
                             context allocates its own memory)                */
    IPC_Q_WS_PEAK = 12,   /* the most workspace bytes in use at once so far    */
    IPC_Q_SPMV_LANES = 13, /* lanes per row the Hessian product uses            */
    IPC_Q_FEM_BLOCKS = 14, /* workgroup sizes of the FEM assembly's kernels:
                              (k_fem << 32) | (k_bsr_assemble << 16) | k_fem_grad_gather */
    IPC_Q_PCG_FUSED = 15   /* 1 when a PCG iteration applies the coarse correction
                              inside its update launch (one scene, correction on;
                              the environment variable IPC_NO_FUSED_PCG = 1, read
                              at ipc_create, keeps it in a launch of its own).
                              Both forms give the same bits.                  */
};

/* Flags of ipc_energy_grad_hess. */
enum { IPC_PSD_PROJECT = 1u, IPC_WITH_FRICTION = 2u };

/* Create a context over n_scenes >= 1 scenes (batching uses the same API:
 * all scenes are stepped together, each with its own Newton, PCG and line
 * search decisions).  hip_stream is a hipStream_t (NULL = default stream) on
 * the current device.  Validates the scene data on the host; allocates the
 * device memory the context needs (released by ipc_destroy). */
int ipc_create(const ipc_scene_desc *scenes, int n_scenes, void *hip_stream, ipc_ctx **out);

/* Capacity of a context over a caller's workspace (ipc_create_ws): the most
 * active contact pairs (point-triangle plus edge-edge, all scenes together)
 * any evaluation meets, the most swept candidates of one broad phase (per
 * kind), and the most pair-local contact blocks of one assembly (the blocks
 * of pairs whose vertices do not all share one mesh's pattern, before equal
 * blocks are merged; up to 16 per pair of FEM vertices and 64 or more when
 * affine bodies are involved). */
typedef struct ipc_capacity {
    int64_t max_pairs, max_candidates, max_local_blocks;
} ipc_capacity;

/* The device bytes a context over these scenes takes at this capacity (an
 * upper bound from the scenes' sizes), after the host checks of ipc_create
 * (IPC_E_INVALID with a message from ipc_last_error(NULL)).  Host work only:
 * no HIP call. */
int ipc_plan(const ipc_scene_desc *scenes, int n_scenes, const ipc_capacity *cap, size_t *workspace_bytes);

/* ipc_create over a caller-owned device workspace of workspace_bytes (256-byte
 * aligned, at least what ipc_plan returned): every device buffer of the
 * context is a range of it, and neither creation nor any later call makes a
 * hipMalloc (the library still creates a private stream for graph capture
 * and pinned host staging).  The workspace must outlive the context.  A call
 * whose contact state exceeds the capacity returns IPC_E_CAPACITY with the
 * count it met (the context is then left in the state of that call's start
 * for a step, and should be recreated with a larger capacity). */
int ipc_create_ws(const ipc_scene_desc *scenes, int n_scenes, const ipc_capacity *cap, void *workspace_dev,
                  size_t workspace_bytes, void *hip_stream, ipc_ctx **out);
int ipc_destroy(ipc_ctx *ctx);
const char *ipc_last_error(const ipc_ctx *ctx);
int ipc_query(const ipc_ctx *ctx, int what, int64_t *value);
/* Per-scene scalars: kappa (as used), L, Newton threshold (newton_tol*h*L). */
int ipc_scene_scalars(const ipc_ctx *ctx, int scene, double *kappa, double *L, double *newton_thr);
/* Change the time step of every scene s with h_host[s] > 0 (entries <= 0
 * keep the scene's step; a non-finite entry is IPC_E_INVALID).  The
 * implicit step of Eq. (3) scales the elastic, spring and orthogonality
 * terms by h^2, predicts y + h ydot + h^2 g and regularises friction by
 * eps_v h; all of these follow, as does the Newton stop newton_tol h L.
 * kappa keeps its creation value.  For retries of a step that did not
 * converge: take it again as two steps of h/2 (host arrays; synchronous). */
int ipc_set_timestep(ipc_ctx *ctx, const double *h_host);
/* Friction lag passes per step, 1 <= passes <= 16 (default 1: friction
 * lagged once at the step start, Sec. III-C).  With more, each scene whose
 * Newton pass converged takes the lag again at its solution (closest-point
 * weights, normals, normal forces and active pairs there; slips still
 * measured from the step start) and runs Newton again from it; the stats
 * count the iterations of all passes.  ipc_step_vjp needs 1 pass. */
int ipc_set_friction_lag(ipc_ctx *ctx, int passes);
/* Adaptive barrier stiffness (a robustness variant of the barrier term of
 * Eq. (3), whose contact model Sec. III-C.1 takes from IPC; the doubling rule
 * is IPC's).  Off by default.  With frac > 0: after every accepted Newton
 * update of a scene, its kappa doubles when the smallest distance d over its
 * active pairs is below frac * dhat and below that of its previous iterate
 * (the step start for a step's first update), capped at factor * kappa0,
 * kappa0 being the scene's kappa at this call.  kappa carries over to later
 * steps (ipc_scene_scalars reports it after each step) and enters the
 * friction lag from the next step on.  frac = 0 switches the rule off; kappa
 * keeps its value.  IPC_E_INVALID for frac < 0, factor < 1 or non-finite
 * values.  ipc_step_vjp refuses contexts with the rule on.  Synchronous. */
int ipc_set_kappa_adaptive(ipc_ctx *ctx, double frac, double factor);

/* State in the external layout (ndof doubles each).  ydot may be NULL on get. */
int ipc_get_state(ipc_ctx *ctx, double *y_dev, double *ydot_dev);
int ipc_set_state(ipc_ctx *ctx, const double *y_dev, const double *ydot_dev);

/* Step set-up at the current state: predictive positions x~ = x + h v + h^2 g
 * (bodies: q + h qdot + h^2 (g, 0, 0, 0)), the drive targets of this step
 * (targets_dev: 12 doubles per driven slot, all scenes concatenated, then 3
 * per joint spring, all scenes concatenated: the spring's b-side body-frame
 * point for this step; may be NULL when there are neither driven links nor
 * joint springs) and the friction data lagged at the current state.
 * ipc_step() calls it itself. */
int ipc_begin_step(ipc_ctx *ctx, const double *targets_dev);

/* Evaluate the potential of the step set up by ipc_begin_step() at any y_dev
 * (external layout): E_dev[n_scenes] (nullable), the gradient g_dev[ndof]
 * (nullable) and, when both v_dev and Hv_dev are given, Hv_dev = H(y) v_dev.
 * flags: IPC_PSD_PROJECT projects the element / body / contact Hessians to PSD
 * (what the Newton solve uses); IPC_WITH_FRICTION includes the lagged friction.
 * Returns IPC_E_INTERSECTING (and E = +inf) when a pair has zero distance. */
int ipc_energy_grad_hess(ipc_ctx *ctx, const double *y_dev, double *E_dev, double *g_dev,
                         const double *v_dev, double *Hv_dev, uint32_t flags);

/* The Hessian of the potential of the step set up by ipc_begin_step(), at any
 * y_dev (external layout), as one block-CSR matrix over external nodes (a node
 * is 3 consecutive DOFs: a FEM vertex, or one of a body's p, A[:,0], A[:,1],
 * A[:,2]): row_ptr_dev[nodes + 1], col_dev[nnzb], val_dev[9 nnzb] (each 3x3
 * block row-major), columns ascending in every row.  It is the matrix the
 * Newton step solves with: inertia, elasticity, orthogonality, springs,
 * barrier and (with IPC_WITH_FRICTION) lagged friction, each term's block
 * projected to PSD with IPC_PSD_PROJECT; the contact blocks that the
 * product keeps pair-local are merged in.  All arrays are device arrays the
 * caller owns; *nnzb_out receives the block count.  With cap_blocks below it
 * (or col_dev / val_dev NULL) only row_ptr_dev is written and the call
 * returns IPC_E_CAPACITY; IPC_E_INTERSECTING as ipc_energy_grad_hess. */
int ipc_hessian_bsr(ipc_ctx *ctx, const double *y_dev, uint32_t flags, int32_t *row_ptr_dev, int32_t *col_dev, double *val_dev,
                    int64_t cap_blocks, int64_t *nnzb_out);

/* Active contact pairs at y_dev for one scene, as vertex tuples in the scene's
 * own vertex numbering (FEM vertices, then body surface vertices, then static
 * vertices): point-triangle (v, t0, t1, t2) and edge-edge (a0, a1, b0, b1),
 * sorted lexicographically.  n_pt / n_ee receive the counts; returns
 * IPC_E_CAPACITY (with the counts set) when cap is too small. */
int ipc_get_pairs(ipc_ctx *ctx, const double *y_dev, int scene, int32_t *pt_host, int32_t *ee_host,
                  int64_t cap, int64_t *n_pt, int64_t *n_ee);

/* Largest safe step alpha_dev[n_scenes] in [0, 1] from additive CCD over the
 * swept candidates of [y, y + p] (external layout). */
int ipc_ccd(ipc_ctx *ctx, const double *y_dev, const double *p_dev, double *alpha_dev);

/* Solve H(y) x = b with the PCG of the Newton step (projected Hessian at y,
 * relative tolerance eta; block-Jacobi preconditioner, plus the coarse
 * correction of IPC_Q_COARSE); iters_host[n_scenes] (nullable). */
int ipc_pcg(ipc_ctx *ctx, const double *y_dev, const double *b_dev, double *x_dev, double eta,
            int32_t *iters_host);

/* Advance every scene by one step: ipc_begin_step(targets_dev), then projected
 * Newton iterations with PCG directions, CCD step bounds and backtracking line
 * search until each scene's Newton measure is below its threshold.  stats_host
 * (nullable) receives n_scenes records.  Returns IPC_OK, or the first non-OK
 * scene status (IPC_E_NOT_CONVERGED leaves that scene at its last iterate).
 * A scene also stops as converged at the energy's rounding floor: when its
 * measure is within 10x its threshold and the line search had to cut the
 * step below 1/1024 before the energy stopped increasing, with the accepted
 * step changing the energy by at most 1e-13 of its value (the environment
 * variable IPC_NO_FLOOR_STOP=1, read at create, turns this off).
 * IPC_TRACE_NEWTON=<scene index>, read at create, prints that scene's
 * Newton measures and line-search steps to stderr. */
int ipc_step(ipc_ctx *ctx, const double *targets_dev, ipc_stats *stats_host);

/* Differentiable parameters theta: the Young's modulus of every tetrahedron
 * (tet_E_dev: all scenes' tets concatenated in creation order, > 0; NULL
 * keeps them) and the friction coefficient of every scene (mu_host[n_scenes],
 * >= 0; NULL keeps them).  Lame parameters follow from E with the scene's
 * Poisson ratios.  The barrier stiffness does not depend on theta. */
int ipc_set_params(ipc_ctx *ctx, const double *tet_E_dev, const double *mu_host);

/* Adjoint of one converged step (the implicit function theorem applied to
 * the stationarity of Eq. (3)'s incremental potential).  The step went from
 * (y_prev, ydot_prev) with drive targets targets_dev (as for ipc_step) to
 * y_next; ybar_next and vbar_next are the adjoints of the loss with respect
 * to y_next and ydot_next = (y_next - y_prev)/h (all external layout, ndof).
 * The call sets the context's state to (y_prev, ydot_prev), redoes the step
 * set-up there (predictor, friction lag), assembles the Hessian at y_next
 * WITHOUT PSD projection, solves H w = ybar_next + vbar_next/h by the Newton
 * step's PCG to relative residual eta (each scene's max_pcg caps it), and writes
 *   vbar_prev = h M w,
 *   ybar_prev = M w - (dG_F/dy_prev)^T w - vbar_next/h
 * (G_F: friction gradient, whose lagged normals, weights and normal forces are
 * functions of y_prev).  It accumulates the parameter adjoints
 *   Ebar_dev[e] -= w . dG/dE_e   (external tets, nullable),
 *   mubar_dev[s] -= w . dG/dmu_s (n_scenes, nullable).
 * iters_host[n_scenes] (nullable) receives the PCG iterations.  Returns
 * IPC_E_INDEFINITE when the PCG met p^T H p <= 0 in some scene (outputs are
 * then not written). */
int ipc_step_vjp(ipc_ctx *ctx, const double *y_prev_dev, const double *ydot_prev_dev, const double *targets_dev,
                 const double *y_next_dev, const double *ybar_next_dev, const double *vbar_next_dev, double *ybar_prev_dev,
                 double *vbar_prev_dev, double *Ebar_dev, double *mubar_dev, double eta, int32_t *iters_host);

/* Kernel timing for measurement.  ipc_profile(ctx, 1) resets the counters
 * and starts recording HIP events on the context's stream around the timed
 * kernels (ipc_profile(ctx, 0) stops).  ipc_kernel_time() returns, for one
 * timed kernel, the summed duration of its launches since the reset, the
 * launch count and the summed algorithmic bytes of those launches (the bytes
 * the operation must move at minimum for its storage format: for IPC_K_SPMV,
 * 76 per stored 3x3 block (9 doubles + column index) of the matrix and of the
 * row-sorted pair-local contact blocks, 4 per row pointer of each, and 24 read
 * plus 24 written per FEM vertex and per body node).  The products count
 * these bytes themselves on the device, row by row: a row of a scene whose
 * PCG has stopped adds only its row pointers, so a product launched past a
 * scene's convergence is not credited with that scene's matrix. */
enum {
    IPC_K_SPMV = 0,          /* Hessian product (block CSR + pair-local blocks) */
    IPC_K_FEM_HESS = 1,      /* FEM gradient + projected Hessian assembly        */
    IPC_K_BARRIER_HESS = 2,  /* barrier gradient + projected Hessian per pair    */
    IPC_K_CONTACT_APPLY = 3, /* unused: pair-local contact blocks are part of
                                the IPC_K_SPMV product (records nothing)         */
    IPC_K_PCG_UPDATE = 4,    /* PCG vector update + preconditioner               */
    IPC_K_BROAD = 5,         /* LBVH build + traversal (both primitive kinds)    */
    IPC_K_CCD = 6,           /* additive CCD over candidates                     */
    IPC_K_FEM_ENERGY = 7,    /* FEM energy for the line search                    */
    IPC_K_COUNT = 8
};
int ipc_profile(ipc_ctx *ctx, int enable);
int ipc_kernel_time(ipc_ctx *ctx, int kernel, double *total_ms, int64_t *launches, double *bytes);
/* Duration of one launch of a timed kernel on the matrix of the last
 * assembly, from `reps` back-to-back launches between two HIP events on the
 * context's stream (so no host gap enters the figure).  Supported kernels:
 * IPC_K_SPMV.  avg_us and bytes (algorithmic bytes of one launch) are
 * written on success.  Uses the context's solver scratch vectors. */
int ipc_time_kernel(ipc_ctx *ctx, int kernel, int reps, double *avg_us, double *bytes);
/* Autotuner: times the Hessian product on the matrix of the last assembly
 * with 1, 2, 4, 8 and 16 lanes per row (reps back-to-back launches each,
 * HIP events on the context's stream) and keeps the fastest for all later
 * products (8 lanes unless another count is more than 3 % faster).
 * us_host[5] (nullable) receives the five times in microseconds, lanes_host
 * (nullable) the choice.  The default before any call is 8 lanes; the
 * environment variable IPC_SPMV_LANES (1, 2, 4, 8 or 16), read at
 * ipc_create, fixes the count instead: the autotuner still times every
 * count but keeps that one.  Otherwise the choice is also kept for the
 * process, keyed by the context's size bucket (the powers of two of the
 * static pattern's block count and of the node count, and whether it holds
 * several scenes); a context created later in the same bucket starts with
 * it (IPC_Q_SPMV_LANES).  The same call then times the three kernels of the
 * FEM assembly (element blocks and gradients, matrix-slot gather, node
 * gradient gather) alone with 64, 128 and 256 threads per workgroup on the
 * current state and keeps the fastest of each (256 unless another is more
 * than 3 % faster; IPC_Q_FEM_BLOCKS), in the same per-bucket record.  No
 * result depends on these choices.  The matrix values are left without the
 * contact and body blocks until the next assembly (every step and
 * ipc_energy_grad_hess assemble first).  Uses the context's solver scratch
 * vectors. */
int ipc_autotune(ipc_ctx *ctx, int reps, double *us_host, int32_t *lanes_host);

#ifdef __cplusplus
}
#endif
#endif
