/*
 * Oracle for one IPC Newton step (PhyVisGen, Sec. III-C, Eq. (1)-(3)).
 *
 * TEST INFRASTRUCTURE ONLY.  A plain, slow FP64 CPU implementation that the
 * tests, the smoke check and the benchmark's CPU-baseline leg use to check and
 * time the HIP library.  It shares no code with the library.  Nothing in the
 * product path may link or call it.
 *
 * Marshalling: or_create() takes three arrays.
 *   sizes[12]  = nv, nt, nb, nbv, nbt, nsv, nst, nobj, nex, ns, nd, nj
 *   ptrs[31]   = X, V, tets, tet_E, tet_nu, tet_rho, vobj,
 *                body_q, body_qdot, body_mass, body_S, body_vol, body_kappa,
 *                body_ext, body_obj, bv_xbar, bv_body, btri, sv_x, stri,
 *                obj_kind, excl, sp_ka, sp_ia, sp_xa, sp_kb, sp_ib, sp_xb,
 *                sp_k, driven_body, joint_spring (layouts as in the scene dict)
 *   params[17] = h, gx, gy, gz, dhat, kappa(0 = automatic), mu, eps_v,
 *                newton_tol, max_newton, pcg_tol, max_pcg, ccd_s,
 *                nx, ny, nz, c: an analytic half-space ground {x : n . x >= c}
 *                (n unit) against every moving surface vertex; n = 0: none
 * All inputs are copied.  The DOF vector is y = [FEM vertices xyz ; per body
 * (p, A[:,0], A[:,1], A[:,2])], i.e. node n owns y[3n..3n+2], body b owns the
 * four nodes nv+4b .. nv+4b+3.
 */
#ifndef IPC_ORACLE_H
#define IPC_ORACLE_H
#ifdef __cplusplus
extern "C" {
#endif

typedef struct OScene OScene;

typedef struct {
    int newton_iters;
    int pcg_iters_total;
    int pcg_iters_max;
    int n_pt_max, n_ee_max;     /* active pairs, max over Newton iterations */
    int n_lag;                  /* friction pairs lagged at the step start   */
    int status;                 /* 0 ok, 3 not converged, 4 line search      */
    double alpha_min;           /* smallest accepted step                    */
    double energy;              /* incremental potential at the final iterate */
} OStats;

OScene *or_create(const int *sizes, const void *const *ptrs, const double *params);
void    or_destroy(OScene *s);

/* scalars: 0 ndof, 1 n_nodes, 2 ncv, 3 ntri, 4 nedge, 5 n_surface_vertices */
int     or_count(const OScene *s, int which);
/* 0 kappa, 1 L (bbox diagonal), 2 mean FEM vertex mass, 3 newton threshold */
double  or_scalar(const OScene *s, int which);
void    or_get_mass(const OScene *s, double *m_nv);
void    or_get_tris(const OScene *s, int *tri3);
void    or_get_edges(const OScene *s, int *edge2);
void    or_get_state(const OScene *s, double *y, double *ydot);
void    or_set_state(OScene *s, const double *y, const double *ydot);
/* contact-vertex world positions at y: ncv x 3 */
void    or_world(const OScene *s, const double *y, double *xw);

/* Step set-up at the current state: predictive positions, drive targets
 * (nd x 12, then nj x 3 joint-spring points: the b-side body-frame point of
 * each joint spring for this step; may be NULL when nd == nj == 0) and the
 * friction lag at y^n. */
void    or_begin_step(OScene *s, const double *targets);
/* Incremental potential at y; terms[7] = inertia, fem, abd, spring,
 * barrier, friction, total.  Returns the total (inf if some pair has d <= 0). */
double  or_energy(OScene *s, const double *y, double *terms);
/* Gradient; gabs (nullable) receives the sum of absolute contributions. */
void    or_gradient(OScene *s, const double *y, double *g, double *gabs);
/* out = H(y) v, with PSD projection when project != 0. */
void    or_hessian_matvec(OScene *s, const double *y, int project, const double *v, double *out);
/* The same product, with or without the lagged friction terms; outabs
 * (nullable) receives, per entry, the sum over all terms of |P|^T |H| |P| |v|
 * (absolute values of every factor), the scale of the operands whose sums
 * and cancellations form that entry. */
void    or_hessian_matvec_abs(OScene *s, const double *y, int project, int with_friction, const double *v, double *out,
                              double *outabs);
/* The Hessian as a dense ndof x ndof row-major matrix (small scenes), and in
 * Habs (nullable) the same sum with every factor's absolute value. */
void    or_hessian_dense(OScene *s, const double *y, int project, int with_friction, double *H, double *Habs);
/* Active pair set at y as vertex tuples (PT: v,t0,t1,t2 ; EE: a0,a1,b0,b1),
 * canonical order.  Returns 0, or -1 when a capacity is too small. */
int     or_pairs(OScene *s, const double *y, int *pt, int cap_pt, int *ee, int cap_ee,
                 int *n_pt, int *n_ee);
/* Largest safe step from additive CCD over the swept candidates of [y, y+p]. */
double  or_ccd(OScene *s, const double *y, const double *p);
/* Block-Jacobi PCG on H(y) x = b (projected).  Returns iterations. */
int     or_pcg(OScene *s, const double *y, const double *b, double *x, double eta);
/* One full step; advances the state.  targets as in or_begin_step. */
int     or_step(OScene *s, const double *targets, OStats *st);

/* Single-pair kernels for unit pins (positions x: 12 doubles). */
double  or_dist2_pt(const double *x, int *type);
double  or_dist2_ee(const double *x, int *type);
/* d^2 with its gradient (12) and Hessian (144) for the given pair kind (0 PT, 1 EE). */
double  or_dist2_derivs(int kind, const double *x, double *g, double *H);
double  or_accd(int kind, const double *x, const double *p, double s);
/* Stable Neo-Hookean density, first Piola stress (9, column-major) and
 * dPsi/dF^2 (81) at F (9, column-major). */
double  or_snh(const double *F, double mu, double lam, double *P, double *HF);
/* b(d), b'(d), b''(d) of the log-barrier with threshold dh */
void    or_barrier3(double d, double dh, double *b3);
/* Symmetric PSD projection of an n x n matrix in place (n <= 12). */
void    or_psd_project(double *A, int n);

/* Adjoint of one converged step (Eq. (3) by the implicit function theorem).
 * Parameters theta = (E per tet, mu): or_set_params replaces them (E may be
 * NULL; mu < 0 keeps mu).  The calls below set the state to (y_prev, yd_prev)
 * and redo the step set-up there (predictor, lag) with the given drive
 * targets, so that the lag data are the functions of y_prev they are in the
 * forward step.
 *   or_dG_dyn_T:    out = (dG/dy^n)^T w  (inertia and the friction lag).
 *   or_dG_dtheta_T: Ebar[e] = w . dG/dE_e; returns w . dG/dmu.
 *   or_step_vjp:    solves H w = ybar_next + vbar_next/h (H unprojected at
 *                   y_next, PCG to relative residual eta) and writes
 *                   ybar_prev, vbar_prev; Ebar (nt) and *mubar are
 *                   accumulated (-=) when non-NULL.  Returns 0, or 6 when the
 *                   PCG met p^T H p <= 0. */
void    or_set_params(OScene *s, const double *E, double mu);
/* New time step h > 0 (every use of h follows; kappa keeps its value). */
void    or_set_timestep(OScene *s, double h);
/* Friction lag passes per step (default 1): after a converged pass the lag
 * is retaken at the solution, displacements still from the step start. */
void    or_set_friction_lag(OScene *s, int passes);
/* Adaptive barrier stiffness (off by default): after every accepted Newton
 * update, kappa doubles when the smallest active-pair distance d is below
 * frac dhat and below that of the previous iterate (the step start for the
 * first update), up to factor kappa0; kappa0 is kappa when this is called,
 * and kappa carries over to later steps.  frac = 0 switches it off. */
void    or_set_kappa_adaptive(OScene *s, double frac, double factor);
/* Set kappa (> 0) and kappa0 to a value. */
void    or_set_kappa(OScene *s, double kappa);
void    or_dG_dyn_T(OScene *s, const double *y_prev, const double *yd_prev, const double *targets,
                    const double *y_next, const double *w, double *out);
double  or_dG_dtheta_T(OScene *s, const double *y_prev, const double *yd_prev, const double *targets,
                       const double *y_next, const double *w, double *Ebar);
int     or_step_vjp(OScene *s, const double *y_prev, const double *yd_prev, const double *targets,
                    const double *y_next, const double *ybar_next, const double *vbar_next,
                    double *ybar_prev, double *vbar_prev, double *Ebar, double *mubar, double eta,
                    int *pcg_iters);

#ifdef __cplusplus
}
#endif
#endif
