/*
 * Oracle for one IPC Newton step of the PhyVisGen arm-gripper system
 * (Sec. III-C.1-2, Eq. (1)-(3)): inertia + Stable Neo-Hookean FEM + affine-body
 * orthogonality + point springs (stitch Eq. (2), fixed joint, joint drives) +
 * IPC log-barrier + lagged friction, minimised by projected Newton with a
 * block-Jacobi PCG solve and an additive-CCD-filtered backtracking line search.
 *
 * TEST INFRASTRUCTURE ONLY: plain, slow FP64 code used to check and time the
 * HIP library; it shares no code with it.  Where the paper is silent the
 * formulas follow the published mathematics of the works it cites (IPC,
 * Stable Neo-Hookean, affine body dynamics, additive CCD); every such reading
 * is listed with the design notes of the repository.
 *
 * Compile with -ffp-contract=off: the contact-pair predicate d^2 < dhat^2 is
 * evaluated with a fixed operation order so that it is reproducible bit for bit.
 */
#include "ipc_oracle.h"

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* small helpers                                                             */
/* ------------------------------------------------------------------------ */
static void *xmalloc(size_t n) { void *p = malloc(n ? n : 1); if (!p) abort(); return p; }
static void *xcalloc(size_t n, size_t k) { void *p = calloc(n ? n : 1, k ? k : 1); if (!p) abort(); return p; }
static void *dupmem(const void *src, size_t n) { void *p = xmalloc(n); if (n) memcpy(p, src, n); return p; }

static inline void sub3(const double *a, const double *b, double *o) { o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2]; }
static inline double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static inline void cross3(const double *a, const double *b, double *o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

typedef struct { int *v; size_t n, cap; } IVec;
static void iv_push(IVec *a, int x)
{
    if (a->n == a->cap) { a->cap = a->cap ? 2 * a->cap : 64; a->v = realloc(a->v, a->cap * sizeof(int)); if (!a->v) abort(); }
    a->v[a->n++] = x;
}

/* ------------------------------------------------------------------------ */
/* symmetric eigen-decomposition (cyclic Jacobi) and PSD projection (C11)    */
/* ------------------------------------------------------------------------ */
/* A (n x n, row-major, symmetric) -> eigenvalues w, eigenvectors in the
 * columns of V.  Plain cyclic Jacobi iterated to full double precision. */
static void jacobi_eig(const double *Ain, int n, double *w, double *V)
{
    double A[144];
    memcpy(A, Ain, sizeof(double) * n * n);
    for (int i = 0; i < n * n; ++i) V[i] = 0.0;
    for (int i = 0; i < n; ++i) V[i * n + i] = 1.0;
    double fro = 0.0;
    for (int i = 0; i < n * n; ++i) fro += A[i] * A[i];
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) off += 2.0 * A[p * n + q] * A[p * n + q];
        if (off <= 1e-36 * fro || off == 0.0) break;
        for (int p = 0; p < n; ++p) {
            for (int q = p + 1; q < n; ++q) {
                double apq = A[p * n + q];
                if (apq == 0.0) continue;
                double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
                double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(1.0 + theta * theta));
                double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
                for (int k = 0; k < n; ++k) {          /* A <- A J */
                    double akp = A[k * n + p], akq = A[k * n + q];
                    A[k * n + p] = c * akp - s * akq;
                    A[k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {          /* A <- J^T A */
                    double apk = A[p * n + k], aqk = A[q * n + k];
                    A[p * n + k] = c * apk - s * aqk;
                    A[q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {          /* V <- V J */
                    double vkp = V[k * n + p], vkq = V[k * n + q];
                    V[k * n + p] = c * vkp - s * vkq;
                    V[k * n + q] = s * vkp + c * vkq;
                }
            }
        }
    }
    for (int i = 0; i < n; ++i) w[i] = A[i * n + i];
}

/* [A]+ = Q max(L, 0) Q^T, the Frobenius-nearest PSD matrix. */
void or_psd_project(double *A, int n)
{
    double w[12], V[144];
    jacobi_eig(A, n, w, V);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double acc = 0.0;
            for (int k = 0; k < n; ++k)
                if (w[k] > 0.0) acc += V[i * n + k] * w[k] * V[j * n + k];
            A[i * n + j] = acc;
        }
}

/* plain Gauss-Jordan inverse with partial pivoting (n <= 12) */
static int invert(const double *Ain, int n, double *Inv)
{
    double A[144];
    memcpy(A, Ain, sizeof(double) * n * n);
    for (int i = 0; i < n * n; ++i) Inv[i] = 0.0;
    for (int i = 0; i < n; ++i) Inv[i * n + i] = 1.0;
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r) if (fabs(A[r * n + c]) > fabs(A[piv * n + c])) piv = r;
        if (A[piv * n + c] == 0.0) return -1;
        if (piv != c)
            for (int k = 0; k < n; ++k) {
                double t = A[c * n + k]; A[c * n + k] = A[piv * n + k]; A[piv * n + k] = t;
                t = Inv[c * n + k]; Inv[c * n + k] = Inv[piv * n + k]; Inv[piv * n + k] = t;
            }
        double d = A[c * n + c];
        for (int k = 0; k < n; ++k) { A[c * n + k] /= d; Inv[c * n + k] /= d; }
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            double f = A[r * n + c];
            if (f == 0.0) continue;
            for (int k = 0; k < n; ++k) { A[r * n + k] -= f * A[c * n + k]; Inv[r * n + k] -= f * Inv[c * n + k]; }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* scene                                                                    */
/* ------------------------------------------------------------------------ */
/* A "point" is a world position that is a linear map of up to four nodes. */
typedef struct { int n; int node[4]; double w[4]; } OPt;
/* A local Hessian term over np points; H is (3np x 3np), row-major. */
typedef struct { int np; OPt pt[4]; double H[144]; } OTerm;
typedef struct { OTerm *t; size_t n, cap; } Terms;

typedef struct {       /* friction data lagged at y^n (C10) */
    int cv[4];
    double beta[4];
    double nrm[3];
    double lam;
    double rn[3];      /* sum_i beta_i x_i^n */
    int kind;          /* 0 point-triangle, 1 edge-edge */
    int type;          /* distance type at y^n */
    double ex;         /* edge-edge mollifier threshold */
} OLag;

struct OScene {
    int nv, nt, nb, nbv, nbt, nsv, nst, nobj, nex, ns, nd, nj;
    double *X, *V, *E, *nu, *rho;
    int *tets, *vobj;
    double *bq, *bqd, *bmass, *bS, *bvol, *bkappa, *bext;
    int *bobj;
    double *bv_xbar, *sv_x;
    int *bv_body, *btri, *stri, *obj_kind, *excl;
    int *sp_ka, *sp_ia, *sp_kb, *sp_ib;
    double *sp_xa, *sp_xb, *sp_k;
    int *driven;
    int *joint_spring;           /* joint slot -> spring whose b-side point follows the joint reference */
    int lag_passes;              /* friction lag passes per step (>= 1) */
    /* adaptive barrier stiffness: kappa doubles after an accepted Newton
     * update whose smallest active-pair distance is below kappa_frac dhat and
     * below the previous iterate's, up to kappa_factor kappa0 (off when
     * kappa_frac is 0) */
    double kappa_frac, kappa_factor, kappa0, dmin_prev;
    /* analytic half-space ground {x : n . x >= c} (n unit) against every
     * dynamic surface vertex; hs_on = 0 when the scene has none */
    int hs_on;
    double hs_n[3], hs_c;
    double h, g[3], dhat, kappa, mu, eps_v, newton_tol, pcg_tol, ccd_s;
    int max_newton, max_pcg;
    /* precompute (C1) */
    double *Bm, *vol, *lmu, *llam, *mass;
    int nnodes, ndof, ncv;
    int ntri, nedge;
    int *tri, *edge;
    double *edge_rest2;
    int *cv_obj;
    int nsurf;
    int *surf_v;                 /* contact vertices referenced by triangles */
    double L, mbar;
    /* state */
    double *y, *ydot, *xtilde, *targets;
    OLag *lag;
    int nlag;
};

static const double *P3(const double *a, int i) { return a + 3 * (size_t)i; }

/* world position of contact vertex c at DOF vector y (C0) */
static void cv_pos(const OScene *s, const double *y, int c, double *x)
{
    if (c < s->nv) { x[0] = y[3 * c]; x[1] = y[3 * c + 1]; x[2] = y[3 * c + 2]; return; }
    c -= s->nv;
    if (c < s->nbv) {
        int b = s->bv_body[c];
        const double *q = y + 3 * (size_t)(s->nv + 4 * b), *xb = P3(s->bv_xbar, c);
        for (int k = 0; k < 3; ++k) x[k] = q[k] + xb[0] * q[3 + k] + xb[1] * q[6 + k] + xb[2] * q[9 + k];
        return;
    }
    c -= s->nbv;
    memcpy(x, P3(s->sv_x, c), 3 * sizeof(double));
}

static OPt cv_point(const OScene *s, int c)
{
    OPt p; memset(&p, 0, sizeof p);
    if (c < s->nv) { p.n = 1; p.node[0] = c; p.w[0] = 1.0; return p; }
    c -= s->nv;
    if (c < s->nbv) {
        int b = s->bv_body[c];
        const double *xb = P3(s->bv_xbar, c);
        p.n = 4;
        for (int k = 0; k < 4; ++k) p.node[k] = s->nv + 4 * b + k;
        p.w[0] = 1.0; p.w[1] = xb[0]; p.w[2] = xb[1]; p.w[3] = xb[2];
        return p;
    }
    p.n = 0;
    return p;
}

static OPt body_point(const OScene *s, int b, const double *xb)
{
    OPt p; p.n = 4;
    for (int k = 0; k < 4; ++k) p.node[k] = s->nv + 4 * b + k;
    p.w[0] = 1.0; p.w[1] = xb[0]; p.w[2] = xb[1]; p.w[3] = xb[2];
    return p;
}

static int cmp_int3(const void *a, const void *b)
{
    const int *x = a, *y = b;
    for (int k = 0; k < 3; ++k) if (x[k] != y[k]) return x[k] < y[k] ? -1 : 1;
    return 0;
}
static int cmp_int2(const void *a, const void *b)
{
    const int *x = a, *y = b;
    for (int k = 0; k < 2; ++k) if (x[k] != y[k]) return x[k] < y[k] ? -1 : 1;
    return 0;
}
static int cmp_int4(const void *a, const void *b)
{
    const int *x = a, *y = b;
    for (int k = 0; k < 4; ++k) if (x[k] != y[k]) return x[k] < y[k] ? -1 : 1;
    return 0;
}

/* rest position of a contact vertex (for the EE mollifier) */
static void cv_rest(const OScene *s, int c, double *x)
{
    if (c < s->nv) { memcpy(x, P3(s->X, c), 3 * sizeof(double)); return; }
    c -= s->nv;
    if (c < s->nbv) { memcpy(x, P3(s->bv_xbar, c), 3 * sizeof(double)); return; }
    memcpy(x, P3(s->sv_x, c - s->nbv), 3 * sizeof(double));
}

OScene *or_create(const int *sz, const void *const *pp, const double *prm)
{
    OScene *s = xcalloc(1, sizeof(OScene));
    s->nv = sz[0]; s->nt = sz[1]; s->nb = sz[2]; s->nbv = sz[3]; s->nbt = sz[4];
    s->nsv = sz[5]; s->nst = sz[6]; s->nobj = sz[7]; s->nex = sz[8]; s->ns = sz[9]; s->nd = sz[10]; s->nj = sz[11];
    size_t D = sizeof(double), I = sizeof(int);
    s->X = dupmem(pp[0], D * 3 * s->nv);      s->V = dupmem(pp[1], D * 3 * s->nv);
    s->tets = dupmem(pp[2], I * 4 * s->nt);
    s->E = dupmem(pp[3], D * s->nt); s->nu = dupmem(pp[4], D * s->nt); s->rho = dupmem(pp[5], D * s->nt);
    s->vobj = dupmem(pp[6], I * s->nv);
    s->bq = dupmem(pp[7], D * 12 * s->nb);     s->bqd = dupmem(pp[8], D * 12 * s->nb);
    s->bmass = dupmem(pp[9], D * s->nb);       s->bS = dupmem(pp[10], D * 9 * s->nb);
    s->bvol = dupmem(pp[11], D * s->nb);       s->bkappa = dupmem(pp[12], D * s->nb);
    s->bext = dupmem(pp[13], D * 3 * s->nb);   s->bobj = dupmem(pp[14], I * s->nb);
    s->bv_xbar = dupmem(pp[15], D * 3 * s->nbv); s->bv_body = dupmem(pp[16], I * s->nbv);
    s->btri = dupmem(pp[17], I * 3 * s->nbt);
    s->sv_x = dupmem(pp[18], D * 3 * s->nsv);  s->stri = dupmem(pp[19], I * 3 * s->nst);
    s->obj_kind = dupmem(pp[20], I * s->nobj); s->excl = dupmem(pp[21], I * 2 * s->nex);
    s->sp_ka = dupmem(pp[22], I * s->ns); s->sp_ia = dupmem(pp[23], I * s->ns); s->sp_xa = dupmem(pp[24], D * 3 * s->ns);
    s->sp_kb = dupmem(pp[25], I * s->ns); s->sp_ib = dupmem(pp[26], I * s->ns); s->sp_xb = dupmem(pp[27], D * 3 * s->ns);
    s->sp_k = dupmem(pp[28], D * s->ns);
    s->driven = dupmem(pp[29], I * s->nd);
    s->joint_spring = dupmem(pp[30], I * s->nj);
    s->h = prm[0]; s->g[0] = prm[1]; s->g[1] = prm[2]; s->g[2] = prm[3];
    s->dhat = prm[4]; s->kappa = prm[5]; s->mu = prm[6]; s->eps_v = prm[7];
    s->newton_tol = prm[8]; s->max_newton = (int)prm[9]; s->pcg_tol = prm[10];
    s->lag_passes = 1;
    s->kappa_frac = 0.0; s->kappa_factor = 100.0; s->dmin_prev = INFINITY;
    s->max_pcg = (int)prm[11]; s->ccd_s = prm[12];
    s->hs_n[0] = prm[13]; s->hs_n[1] = prm[14]; s->hs_n[2] = prm[15]; s->hs_c = prm[16];
    s->hs_on = s->hs_n[0] != 0.0 || s->hs_n[1] != 0.0 || s->hs_n[2] != 0.0;

    /* C1: per-tet inverse rest shape matrix, volume, Lame parameters, lumped mass */
    s->Bm = xmalloc(D * 9 * s->nt); s->vol = xmalloc(D * s->nt);
    s->lmu = xmalloc(D * s->nt); s->llam = xmalloc(D * s->nt);
    s->mass = xcalloc(s->nv, D);
    for (int e = 0; e < s->nt; ++e) {
        const int *t = s->tets + 4 * e;
        double Dm[9]; /* Dm[r*3+c] = (X_{c+1} - X_0)_r */
        for (int c = 0; c < 3; ++c)
            for (int r = 0; r < 3; ++r) Dm[r * 3 + c] = s->X[3 * t[c + 1] + r] - s->X[3 * t[0] + r];
        double det = Dm[0] * (Dm[4] * Dm[8] - Dm[5] * Dm[7]) - Dm[1] * (Dm[3] * Dm[8] - Dm[5] * Dm[6])
                   + Dm[2] * (Dm[3] * Dm[7] - Dm[4] * Dm[6]);
        invert(Dm, 3, s->Bm + 9 * e);
        s->vol[e] = det / 6.0;
        double E = s->E[e], nu = s->nu[e];
        s->lmu[e] = E / (2.0 * (1.0 + nu));
        s->llam[e] = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
        for (int k = 0; k < 4; ++k) s->mass[t[k]] += s->rho[e] * s->vol[e] / 4.0;
    }
    s->nnodes = s->nv + 4 * s->nb;
    s->ndof = 3 * s->nnodes;
    s->ncv = s->nv + s->nbv + s->nsv;

    /* surface: faces owned by exactly one tet, outward (C1) */
    int nf = 4 * s->nt;
    int *faces = xmalloc(I * 4 * (size_t)nf); /* sorted key (3) + oriented index */
    int *ofaces = xmalloc(I * 3 * (size_t)nf);
    static const int fl[4][3] = {{0, 2, 1}, {0, 1, 3}, {0, 3, 2}, {1, 2, 3}};
    for (int e = 0; e < s->nt; ++e)
        for (int f = 0; f < 4; ++f) {
            int *o = ofaces + 3 * (4 * e + f);
            for (int k = 0; k < 3; ++k) o[k] = s->tets[4 * e + fl[f][k]];
            int a = o[0], b = o[1], c = o[2], t;
            if (a > b) { t = a; a = b; b = t; }
            if (b > c) { t = b; b = c; c = t; }
            if (a > b) { t = a; a = b; b = t; }
            int *k4 = faces + 4 * (4 * e + f);
            k4[0] = a; k4[1] = b; k4[2] = c; k4[3] = 4 * e + f;
        }
    qsort(faces, nf, 4 * I, cmp_int3);
    IVec tris = {0};
    for (int i = 0; i < nf;) {
        int j = i + 1;
        while (j < nf && cmp_int3(faces + 4 * i, faces + 4 * j) == 0) ++j;
        if (j - i == 1) {
            const int *o = ofaces + 3 * faces[4 * i + 3];
            for (int k = 0; k < 3; ++k) iv_push(&tris, o[k]);
        }
        i = j;
    }
    free(faces); free(ofaces);
    for (int t = 0; t < s->nbt; ++t) for (int k = 0; k < 3; ++k) iv_push(&tris, s->nv + s->btri[3 * t + k]);
    for (int t = 0; t < s->nst; ++t) for (int k = 0; k < 3; ++k) iv_push(&tris, s->nv + s->nbv + s->stri[3 * t + k]);
    s->ntri = (int)(tris.n / 3);
    /* canonical triangle: rotate so the smallest index comes first; sort */
    for (int t = 0; t < s->ntri; ++t) {
        int *v = tris.v + 3 * t;
        while (v[0] > v[1] || v[0] > v[2]) { int a = v[0]; v[0] = v[1]; v[1] = v[2]; v[2] = a; }
    }
    qsort(tris.v, s->ntri, 3 * I, cmp_int3);
    s->tri = tris.v;
    /* unique edges (min, max), sorted */
    int *ed = xmalloc(I * 6 * (size_t)s->ntri);
    for (int t = 0; t < s->ntri; ++t)
        for (int k = 0; k < 3; ++k) {
            int a = s->tri[3 * t + k], b = s->tri[3 * t + (k + 1) % 3];
            ed[6 * t + 2 * k] = a < b ? a : b;
            ed[6 * t + 2 * k + 1] = a < b ? b : a;
        }
    qsort(ed, 3 * (size_t)s->ntri, 2 * I, cmp_int2);
    int ne = 0;
    for (int i = 0; i < 3 * s->ntri; ++i)
        if (ne == 0 || cmp_int2(ed + 2 * i, ed + 2 * (ne - 1)) != 0) { ed[2 * ne] = ed[2 * i]; ed[2 * ne + 1] = ed[2 * i + 1]; ++ne; }
    s->nedge = ne;
    s->edge = ed;
    s->edge_rest2 = xmalloc(D * (ne ? ne : 1));
    for (int i = 0; i < ne; ++i) {
        double a[3], b[3], d[3];
        cv_rest(s, ed[2 * i], a); cv_rest(s, ed[2 * i + 1], b); sub3(b, a, d);
        s->edge_rest2[i] = dot3(d, d);
    }
    /* objects and surface vertices */
    s->cv_obj = xmalloc(I * (size_t)(s->ncv ? s->ncv : 1));
    int static_obj = -1;
    for (int o = 0; o < s->nobj; ++o) if (s->obj_kind[o] == 2) { static_obj = o; break; }
    for (int c = 0; c < s->ncv; ++c) {
        if (c < s->nv) s->cv_obj[c] = s->vobj[c];
        else if (c < s->nv + s->nbv) s->cv_obj[c] = s->bobj[s->bv_body[c - s->nv]];
        else s->cv_obj[c] = static_obj;
    }
    char *on = xcalloc(s->ncv ? s->ncv : 1, 1);
    for (int t = 0; t < 3 * s->ntri; ++t) on[s->tri[t]] = 1;
    s->surf_v = xmalloc(I * (size_t)(s->ncv ? s->ncv : 1));
    s->nsurf = 0;
    for (int c = 0; c < s->ncv; ++c) if (on[c]) s->surf_v[s->nsurf++] = c;
    free(on);

    /* kappa (C9), characteristic length L (C13) */
    double msum = 0.0;
    for (int i = 0; i < s->nv; ++i) msum += s->mass[i];
    if (s->nv > 0) s->mbar = msum / s->nv;
    else {
        double bm = 0.0; int nbs = 0;
        for (int b = 0; b < s->nb; ++b) bm += s->bmass[b];
        nbs = s->nbv;
        s->mbar = nbs ? bm / nbs : 0.0;
    }
    double gn = sqrt(dot3(s->g, s->g));
    if (s->kappa <= 0.0) s->kappa = 10.0 * s->mbar * gn * s->h * s->h / s->dhat;
    s->kappa0 = s->kappa;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int i = 0; i < s->nv; ++i)
        for (int k = 0; k < 3; ++k) { double x = s->X[3 * i + k]; if (x < lo[k]) lo[k] = x; if (x > hi[k]) hi[k] = x; }
    for (int b = 0; b < s->nb; ++b)
        for (int k = 0; k < 3; ++k) {
            double a = s->bq[12 * b + k] - s->bext[3 * b + k], c = s->bq[12 * b + k] + s->bext[3 * b + k];
            if (a < lo[k]) lo[k] = a; if (c > hi[k]) hi[k] = c;
        }
    double dd = 0.0;
    for (int k = 0; k < 3; ++k) if (hi[k] > lo[k]) dd += (hi[k] - lo[k]) * (hi[k] - lo[k]);
    s->L = sqrt(dd);

    /* state */
    s->y = xmalloc(D * (size_t)s->ndof); s->ydot = xmalloc(D * (size_t)s->ndof);
    s->xtilde = xmalloc(D * (size_t)s->ndof);
    memcpy(s->y, s->X, D * 3 * s->nv); memcpy(s->ydot, s->V, D * 3 * s->nv);
    memcpy(s->y + 3 * s->nv, s->bq, D * 12 * s->nb); memcpy(s->ydot + 3 * s->nv, s->bqd, D * 12 * s->nb);
    memcpy(s->xtilde, s->y, D * (size_t)s->ndof);
    s->targets = xcalloc(12 * (size_t)(s->nd ? s->nd : 1), D);
    for (int d = 0; d < s->nd; ++d) memcpy(s->targets + 12 * d, s->bq + 12 * s->driven[d], 12 * D);
    s->lag = NULL; s->nlag = 0;
    return s;
}

void or_destroy(OScene *s)
{
    if (!s) return;
    void *p[] = {s->X, s->V, s->E, s->nu, s->rho, s->tets, s->vobj, s->bq, s->bqd, s->bmass, s->bS, s->bvol,
                 s->bkappa, s->bext, s->bobj, s->bv_xbar, s->sv_x, s->bv_body, s->btri, s->stri, s->obj_kind,
                 s->excl, s->sp_ka, s->sp_ia, s->sp_kb, s->sp_ib, s->sp_xa, s->sp_xb, s->sp_k, s->driven, s->joint_spring,
                 s->Bm, s->vol, s->lmu, s->llam, s->mass, s->tri, s->edge, s->edge_rest2, s->cv_obj,
                 s->surf_v, s->y, s->ydot, s->xtilde, s->targets, s->lag};
    for (size_t i = 0; i < sizeof p / sizeof p[0]; ++i) free(p[i]);
    free(s);
}

int or_count(const OScene *s, int w)
{
    switch (w) {
    case 0: return s->ndof; case 1: return s->nnodes; case 2: return s->ncv;
    case 3: return s->ntri; case 4: return s->nedge; case 5: return s->nsurf;
    }
    return -1;
}
double or_scalar(const OScene *s, int w)
{
    switch (w) {
    case 0: return s->kappa; case 1: return s->L; case 2: return s->mbar;
    case 3: return s->newton_tol * s->h * s->L;
    }
    return NAN;
}
void or_get_mass(const OScene *s, double *m) { memcpy(m, s->mass, sizeof(double) * s->nv); }
void or_get_tris(const OScene *s, int *t) { memcpy(t, s->tri, sizeof(int) * 3 * s->ntri); }
void or_get_edges(const OScene *s, int *e) { memcpy(e, s->edge, sizeof(int) * 2 * s->nedge); }
void or_get_state(const OScene *s, double *y, double *yd)
{
    memcpy(y, s->y, sizeof(double) * s->ndof);
    if (yd) memcpy(yd, s->ydot, sizeof(double) * s->ndof);
}
void or_set_state(OScene *s, const double *y, const double *yd)
{
    memcpy(s->y, y, sizeof(double) * s->ndof);
    memcpy(s->ydot, yd, sizeof(double) * s->ndof);
}
void or_world(const OScene *s, const double *y, double *xw)
{
    for (int c = 0; c < s->ncv; ++c) cv_pos(s, y, c, xw + 3 * (size_t)c);
}

/* ------------------------------------------------------------------------ */
/* distances (C7); fixed operation order, see the distance specification     */
/* ------------------------------------------------------------------------ */
static double d2_pp(const double *p, const double *q) { double u[3]; sub3(p, q, u); return dot3(u, u); }
static double d2_pe(const double *p, const double *e0, const double *e1)
{
    double a[3], b[3], c[3], e[3];
    sub3(e0, p, a); sub3(e1, p, b); cross3(a, b, c); sub3(e1, e0, e);
    return dot3(c, c) / dot3(e, e);
}
static double d2_plane(const double *p, const double *t0, const double *t1, const double *t2)
{
    double e1[3], e2[3], n[3], w[3];
    sub3(t1, t0, e1); sub3(t2, t0, e2); cross3(e1, e2, n); sub3(p, t0, w);
    double s = dot3(n, w);
    return s * s / dot3(n, n);
}
static double d2_line(const double *a0, const double *a1, const double *b0, const double *b1)
{
    double u[3], v[3], n[3], w[3];
    sub3(a1, a0, u); sub3(b1, b0, v); cross3(u, v, n); sub3(b0, a0, w);
    double s = dot3(n, w);
    return s * s / dot3(n, n);
}

/* PT types: 0..2 PP(p,t_k), 3 PE(t0,t1), 4 PE(t1,t2), 5 PE(t2,t0), 6 plane */
static int pt_type(const double *p, const double *t0, const double *t1, const double *t2)
{
    double ab[3], ac[3], ap[3], bp[3], cp[3];
    sub3(t1, t0, ab); sub3(t2, t0, ac); sub3(p, t0, ap);
    double d1 = dot3(ab, ap), d2 = dot3(ac, ap);
    if (d1 <= 0.0 && d2 <= 0.0) return 0;
    sub3(p, t1, bp);
    double d3 = dot3(ab, bp), d4 = dot3(ac, bp);
    if (d3 >= 0.0 && d4 <= d3) return 1;
    double vc = d1 * d4 - d3 * d2;
    if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) return 3;
    sub3(p, t2, cp);
    double d5 = dot3(ab, cp), d6 = dot3(ac, cp);
    if (d6 >= 0.0 && d5 <= d6) return 2;
    double vb = d5 * d2 - d1 * d6;
    if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) return 5;
    double va = d3 * d6 - d5 * d4;
    if (va <= 0.0 && (d4 - d3) >= 0.0 && (d5 - d6) >= 0.0) return 4;
    return 6;
}
static double pt_d2_of_type(int t, const double *p, const double *t0, const double *t1, const double *t2)
{
    switch (t) {
    case 0: return d2_pp(p, t0);
    case 1: return d2_pp(p, t1);
    case 2: return d2_pp(p, t2);
    case 3: return d2_pe(p, t0, t1);
    case 4: return d2_pe(p, t1, t2);
    case 5: return d2_pe(p, t2, t0);
    default: return d2_plane(p, t0, t1, t2);
    }
}

/* point-segment sub-case: 0 PP(p,e0), 1 PP(p,e1), 2 PE */
static int ps_type(const double *p, const double *e0, const double *e1)
{
    double ev[3], w[3];
    sub3(e1, e0, ev); sub3(p, e0, w);
    double t = dot3(w, ev), L = dot3(ev, ev);
    if (t <= 0.0) return 0;
    if (t >= L) return 1;
    return 2;
}

/* EE types: 0 PP(a0,b0) 1 PP(a0,b1) 2 PP(a1,b0) 3 PP(a1,b1)
 *           4 PE(a0;b) 5 PE(a1;b) 6 PE(b0;a) 7 PE(b1;a) 8 line-line */
static double ee_d2_of_type(int t, const double *a0, const double *a1, const double *b0, const double *b1)
{
    switch (t) {
    case 0: return d2_pp(a0, b0);
    case 1: return d2_pp(a0, b1);
    case 2: return d2_pp(a1, b0);
    case 3: return d2_pp(a1, b1);
    case 4: return d2_pe(a0, b0, b1);
    case 5: return d2_pe(a1, b0, b1);
    case 6: return d2_pe(b0, a0, a1);
    case 7: return d2_pe(b1, a0, a1);
    default: return d2_line(a0, a1, b0, b1);
    }
}
static int ee_type(const double *a0, const double *a1, const double *b0, const double *b1)
{
    double u[3], v[3], w[3];
    sub3(a1, a0, u); sub3(b1, b0, v); sub3(a0, b0, w);
    double A = dot3(u, u), B = dot3(u, v), C = dot3(v, v), D = dot3(u, w), E = dot3(v, w);
    double den = A * C - B * B;
    if (den > 1e-10 * A * C) {
        double sN = B * E - C * D, tN = A * E - B * D;
        if (sN > 0.0 && sN < den && tN > 0.0 && tN < den) return 8;
    }
    /* the minimum lies on the boundary of the parameter square */
    int cand[4];
    int k;
    k = ps_type(a0, b0, b1); cand[0] = k == 0 ? 0 : k == 1 ? 1 : 4;
    k = ps_type(a1, b0, b1); cand[1] = k == 0 ? 2 : k == 1 ? 3 : 5;
    k = ps_type(b0, a0, a1); cand[2] = k == 0 ? 0 : k == 1 ? 2 : 6;
    k = ps_type(b1, a0, a1); cand[3] = k == 0 ? 1 : k == 1 ? 3 : 7;
    int best = cand[0];
    double bd = ee_d2_of_type(cand[0], a0, a1, b0, b1);
    for (int i = 1; i < 4; ++i) {
        double d = ee_d2_of_type(cand[i], a0, a1, b0, b1);
        if (d < bd) { bd = d; best = cand[i]; }
    }
    return best;
}

double or_dist2_pt(const double *x, int *type)
{
    int t = pt_type(x, x + 3, x + 6, x + 9);
    if (type) *type = t;
    return pt_d2_of_type(t, x, x + 3, x + 6, x + 9);
}
double or_dist2_ee(const double *x, int *type)
{
    int t = ee_type(x, x + 3, x + 6, x + 9);
    if (type) *type = t;
    return ee_d2_of_type(t, x, x + 3, x + 6, x + 9);
}
static double dist2_kind(int kind, const double *x, int *type)
{
    return kind == 0 ? or_dist2_pt(x, type) : or_dist2_ee(x, type);
}

/* Affine parametrisation of the closest-point difference for a distance type:
 * r(s) = sum_k (a0_k + sum_m s_m am_k) x_k, m < npar. */
typedef struct { int npar; double a0[4], a[2][4]; } Param;
static Param type_param(int kind, int t)
{
    Param P; memset(&P, 0, sizeof P);
#define SET4(v, A, B, C, D) do { (v)[0] = A; (v)[1] = B; (v)[2] = C; (v)[3] = D; } while (0)
    if (kind == 0) {
        switch (t) {
        case 0: SET4(P.a0, 1, -1, 0, 0); break;
        case 1: SET4(P.a0, 1, 0, -1, 0); break;
        case 2: SET4(P.a0, 1, 0, 0, -1); break;
        case 3: P.npar = 1; SET4(P.a0, 1, -1, 0, 0); SET4(P.a[0], 0, 1, -1, 0); break;
        case 4: P.npar = 1; SET4(P.a0, 1, 0, -1, 0); SET4(P.a[0], 0, 0, 1, -1); break;
        case 5: P.npar = 1; SET4(P.a0, 1, 0, 0, -1); SET4(P.a[0], 0, -1, 0, 1); break;
        default: P.npar = 2; SET4(P.a0, 1, -1, 0, 0); SET4(P.a[0], 0, 1, -1, 0); SET4(P.a[1], 0, 1, 0, -1); break;
        }
    } else {
        switch (t) {
        case 0: SET4(P.a0, 1, 0, -1, 0); break;
        case 1: SET4(P.a0, 1, 0, 0, -1); break;
        case 2: SET4(P.a0, 0, 1, -1, 0); break;
        case 3: SET4(P.a0, 0, 1, 0, -1); break;
        case 4: P.npar = 1; SET4(P.a0, 1, 0, -1, 0); SET4(P.a[0], 0, 0, 1, -1); break;
        case 5: P.npar = 1; SET4(P.a0, 0, 1, -1, 0); SET4(P.a[0], 0, 0, 1, -1); break;
        case 6: P.npar = 1; SET4(P.a0, 1, 0, -1, 0); SET4(P.a[0], -1, 1, 0, 0); break;
        case 7: P.npar = 1; SET4(P.a0, 1, 0, 0, -1); SET4(P.a[0], -1, 1, 0, 0); break;
        default: P.npar = 2; SET4(P.a0, 1, 0, -1, 0); SET4(P.a[0], -1, 1, 0, 0); SET4(P.a[1], 0, 0, 1, -1); break;
        }
    }
#undef SET4
    return P;
}

/* Closest-point coefficients beta = a(s*) and r = sum beta_k x_k. */
static void closest(const Param *P, const double *x, double *beta, double *r, double *Dm /* 3 x npar */)
{
    double r0[3] = {0, 0, 0};
    for (int k = 0; k < 4; ++k) for (int c = 0; c < 3; ++c) r0[c] += P->a0[k] * x[3 * k + c];
    for (int m = 0; m < P->npar; ++m)
        for (int c = 0; c < 3; ++c) {
            double acc = 0.0;
            for (int k = 0; k < 4; ++k) acc += P->a[m][k] * x[3 * k + c];
            Dm[3 * m + c] = acc;
        }
    double sv[2] = {0, 0};
    if (P->npar == 1) {
        sv[0] = -dot3(Dm, r0) / dot3(Dm, Dm);
    } else if (P->npar == 2) {
        double G00 = dot3(Dm, Dm), G01 = dot3(Dm, Dm + 3), G11 = dot3(Dm + 3, Dm + 3);
        double b0 = -dot3(Dm, r0), b1 = -dot3(Dm + 3, r0);
        double det = G00 * G11 - G01 * G01;
        sv[0] = (b0 * G11 - G01 * b1) / det;
        sv[1] = (G00 * b1 - G01 * b0) / det;
    }
    for (int k = 0; k < 4; ++k) {
        beta[k] = P->a0[k];
        for (int m = 0; m < P->npar; ++m) beta[k] += sv[m] * P->a[m][k];
    }
    for (int c = 0; c < 3; ++c) {
        double acc = 0.0;
        for (int k = 0; k < 4; ++k) acc += beta[k] * x[3 * k + c];
        r[c] = acc;
    }
}

/* Gradient and Hessian of d^2 = min_s |r(s)|^2 (envelope theorem):
 *   g = 2 beta (x) r,  H = 2 (beta beta^T) (x) I - F_xs F_ss^{-1} F_sx. */
static void d2_derivs_type(int kind, int t, const double *x, double *g, double *H)
{
    Param P = type_param(kind, t);
    double beta[4], r[3], Dm[6];
    closest(&P, x, beta, r, Dm);
    for (int k = 0; k < 4; ++k) for (int c = 0; c < 3; ++c) g[3 * k + c] = 2.0 * beta[k] * r[c];
    for (int i = 0; i < 144; ++i) H[i] = 0.0;
    for (int k = 0; k < 4; ++k)
        for (int l = 0; l < 4; ++l)
            for (int c = 0; c < 3; ++c) H[(3 * k + c) * 12 + 3 * l + c] = 2.0 * beta[k] * beta[l];
    if (P.npar == 0) return;
    double Fxs[12][2], Fss[2][2], Fi[2][2];
    for (int m = 0; m < P.npar; ++m) {
        for (int n = 0; n < P.npar; ++n) Fss[m][n] = 2.0 * dot3(Dm + 3 * m, Dm + 3 * n);
        for (int k = 0; k < 4; ++k)
            for (int c = 0; c < 3; ++c) Fxs[3 * k + c][m] = 2.0 * P.a[m][k] * r[c] + 2.0 * beta[k] * Dm[3 * m + c];
    }
    if (P.npar == 1) Fi[0][0] = 1.0 / Fss[0][0];
    else {
        double det = Fss[0][0] * Fss[1][1] - Fss[0][1] * Fss[1][0];
        Fi[0][0] = Fss[1][1] / det; Fi[1][1] = Fss[0][0] / det;
        Fi[0][1] = -Fss[0][1] / det; Fi[1][0] = -Fss[1][0] / det;
    }
    for (int i = 0; i < 12; ++i)
        for (int j = 0; j < 12; ++j) {
            double acc = 0.0;
            for (int m = 0; m < P.npar; ++m)
                for (int n = 0; n < P.npar; ++n) acc += Fxs[i][m] * Fi[m][n] * Fxs[j][n];
            H[i * 12 + j] -= acc;
        }
}

double or_dist2_derivs(int kind, const double *x, double *g, double *H)
{
    int t;
    double d2 = dist2_kind(kind, x, &t);
    d2_derivs_type(kind, t, x, g, H);
    return d2;
}

/* ------------------------------------------------------------------------ */
/* barrier (C8), mollifier, friction mollifier (C10)                        */
/* ------------------------------------------------------------------------ */
static double barrier(double d, double dh)
{
    if (d >= dh) return 0.0;
    return -(d - dh) * (d - dh) * log(d / dh);
}
static double barrier_d1(double d, double dh)
{
    if (d >= dh) return 0.0;
    return -2.0 * (d - dh) * log(d / dh) - (d - dh) * (d - dh) / d;
}
static double barrier_d2(double d, double dh)
{
    if (d >= dh) return 0.0;
    return -2.0 * log(d / dh) - 4.0 * (d - dh) / d + (d - dh) * (d - dh) / (d * d);
}

/* The signed distance of a point to the half-space's boundary plane,
 * n . x - c (n unit), summed left to right. */
static double hs_dist(const OScene *s, const double *x)
{
    return s->hs_n[0] * x[0] + s->hs_n[1] * x[1] + s->hs_n[2] * x[2] - s->hs_c;
}

/* Whether contact vertex c moves (a FEM or body vertex, not static). */
static int cv_dynamic(const OScene *s, int c) { return c < s->nv + s->nbv; }

void or_barrier3(double d, double dh, double *b3)
{
    b3[0] = barrier(d, dh); b3[1] = barrier_d1(d, dh); b3[2] = barrier_d2(d, dh);
}

/* c = |u x v|^2 with u = a1 - a0, v = b1 - b0: value, gradient (12), Hessian (144) */
static double cross2_derivs(const double *x, double *g, double *H)
{
    double u[3], v[3], n[3];
    sub3(x + 3, x, u); sub3(x + 9, x + 6, v); cross3(u, v, n);
    double c = dot3(n, n);
    if (!g) return c;
    double cu[3], cv[3];
    cross3(v, n, cu); cross3(n, u, cv);
    for (int k = 0; k < 3; ++k) {
        cu[k] *= 2.0; cv[k] *= 2.0;
        g[k] = -cu[k]; g[3 + k] = cu[k]; g[6 + k] = -cv[k]; g[9 + k] = cv[k];
    }
    /* 6x6 Hessian in (u, v): Huu = 2 [v]x^T [v]x, Hvv = 2 [u]x^T [u]x,
     * Huv = 2 [v]x [u]x - 2 [n]x */
    double Vx[9] = {0, -v[2], v[1], v[2], 0, -v[0], -v[1], v[0], 0};
    double Ux[9] = {0, -u[2], u[1], u[2], 0, -u[0], -u[1], u[0], 0};
    double Nx[9] = {0, -n[2], n[1], n[2], 0, -n[0], -n[1], n[0], 0};
    double Huu[9], Hvv[9], Huv[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double a = 0, b = 0, c2 = 0;
            for (int k = 0; k < 3; ++k) { a += Vx[k * 3 + i] * Vx[k * 3 + j]; b += Ux[k * 3 + i] * Ux[k * 3 + j]; c2 += Vx[i * 3 + k] * Ux[k * 3 + j]; }
            Huu[i * 3 + j] = 2.0 * a; Hvv[i * 3 + j] = 2.0 * b; Huv[i * 3 + j] = 2.0 * c2 - 2.0 * Nx[i * 3 + j];
        }
    /* map: a0 = -u, a1 = +u, b0 = -v, b1 = +v */
    static const double su[4] = {-1, 1, 0, 0}, sv[4] = {0, 0, -1, 1};
    for (int k = 0; k < 4; ++k)
        for (int l = 0; l < 4; ++l)
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j)
                    H[(3 * k + i) * 12 + 3 * l + j] = su[k] * su[l] * Huu[i * 3 + j] + sv[k] * sv[l] * Hvv[i * 3 + j]
                                                    + su[k] * sv[l] * Huv[i * 3 + j] + sv[k] * su[l] * Huv[j * 3 + i];
    return c;
}

/* ------------------------------------------------------------------------ */
/* candidate search: sweep-and-prune on x over axis-aligned boxes            */
/* ------------------------------------------------------------------------ */
typedef struct { double lo[3], hi[3]; int set, idx; } Box;
static int cmp_box(const void *a, const void *b)
{
    const Box *x = a, *y = b;
    if (x->lo[0] != y->lo[0]) return x->lo[0] < y->lo[0] ? -1 : 1;
    if (x->set != y->set) return x->set - y->set;
    return x->idx - y->idx;
}
static void box_add(Box *b, const double *p)
{
    for (int k = 0; k < 3; ++k) { if (p[k] < b->lo[k]) b->lo[k] = p[k]; if (p[k] > b->hi[k]) b->hi[k] = p[k]; }
}
static void box_init(Box *b, int set, int idx)
{
    for (int k = 0; k < 3; ++k) { b->lo[k] = INFINITY; b->hi[k] = -INFINITY; }
    b->set = set; b->idx = idx;
}
static void box_inflate(Box *b, double r) { for (int k = 0; k < 3; ++k) { b->lo[k] -= r; b->hi[k] += r; } }

static int obj_allowed(const OScene *s, int oa, int ob)
{
    int ka = oa >= 0 ? s->obj_kind[oa] : 2, kb = ob >= 0 ? s->obj_kind[ob] : 2;
    if (ka == 2 && kb == 2) return 0;
    if (oa == ob && ka == 1) return 0;
    for (int i = 0; i < s->nex; ++i) {
        int a = s->excl[2 * i], b = s->excl[2 * i + 1];
        if ((a == oa && b == ob) || (a == ob && b == oa)) return 0;
    }
    return 1;
}

/* Candidates whose boxes over positions x0 and x1 (ncv x 3 each), inflated
 * by 1.01 dhat, overlap.  PT: (surface vertex, triangle); EE: (e < e'). */
static void candidates(const OScene *s, const double *x0, const double *x1, IVec *pt, IVec *ee)
{
    double r = 1.01 * s->dhat;
    int nbx = s->nsurf + s->ntri;
    Box *bx = xmalloc(sizeof(Box) * (size_t)(nbx ? nbx : 1));
    for (int i = 0; i < s->nsurf; ++i) {
        int c = s->surf_v[i];
        box_init(bx + i, 0, c); box_add(bx + i, P3(x0, c)); box_add(bx + i, P3(x1, c)); box_inflate(bx + i, r);
    }
    for (int t = 0; t < s->ntri; ++t) {
        Box *b = bx + s->nsurf + t;
        box_init(b, 1, t);
        for (int k = 0; k < 3; ++k) { box_add(b, P3(x0, s->tri[3 * t + k])); box_add(b, P3(x1, s->tri[3 * t + k])); }
    }
    qsort(bx, nbx, sizeof(Box), cmp_box);
    for (int i = 0; i < nbx; ++i)
        for (int j = i + 1; j < nbx && bx[j].lo[0] <= bx[i].hi[0]; ++j) {
            if (bx[i].set == bx[j].set) continue;
            if (bx[i].lo[1] > bx[j].hi[1] || bx[j].lo[1] > bx[i].hi[1]) continue;
            if (bx[i].lo[2] > bx[j].hi[2] || bx[j].lo[2] > bx[i].hi[2]) continue;
            int v = bx[i].set == 0 ? bx[i].idx : bx[j].idx;
            int t = bx[i].set == 0 ? bx[j].idx : bx[i].idx;
            const int *tv = s->tri + 3 * t;
            if (v == tv[0] || v == tv[1] || v == tv[2]) continue;
            if (!obj_allowed(s, s->cv_obj[v], s->cv_obj[tv[0]])) continue;
            iv_push(pt, v); iv_push(pt, t);
        }
    free(bx);
    bx = xmalloc(sizeof(Box) * (size_t)(s->nedge ? s->nedge : 1));
    for (int e = 0; e < s->nedge; ++e) {
        box_init(bx + e, 0, e);
        for (int k = 0; k < 2; ++k) { box_add(bx + e, P3(x0, s->edge[2 * e + k])); box_add(bx + e, P3(x1, s->edge[2 * e + k])); }
        box_inflate(bx + e, 0.5 * r);
    }
    qsort(bx, s->nedge, sizeof(Box), cmp_box);
    for (int i = 0; i < s->nedge; ++i)
        for (int j = i + 1; j < s->nedge && bx[j].lo[0] <= bx[i].hi[0]; ++j) {
            if (bx[i].lo[1] > bx[j].hi[1] || bx[j].lo[1] > bx[i].hi[1]) continue;
            if (bx[i].lo[2] > bx[j].hi[2] || bx[j].lo[2] > bx[i].hi[2]) continue;
            int e = bx[i].idx < bx[j].idx ? bx[i].idx : bx[j].idx;
            int f = bx[i].idx < bx[j].idx ? bx[j].idx : bx[i].idx;
            const int *a = s->edge + 2 * e, *b = s->edge + 2 * f;
            if (a[0] == b[0] || a[0] == b[1] || a[1] == b[0] || a[1] == b[1]) continue;
            if (!obj_allowed(s, s->cv_obj[a[0]], s->cv_obj[b[0]])) continue;
            iv_push(ee, e); iv_push(ee, f);
        }
    free(bx);
}

/* positions of the 4 vertices of a candidate */
static void pair_x(const OScene *s, const double *xw, int kind, int i, int j, int *cv, double *x)
{
    if (kind == 0) {
        cv[0] = i; cv[1] = s->tri[3 * j]; cv[2] = s->tri[3 * j + 1]; cv[3] = s->tri[3 * j + 2];
    } else {
        cv[0] = s->edge[2 * i]; cv[1] = s->edge[2 * i + 1]; cv[2] = s->edge[2 * j]; cv[3] = s->edge[2 * j + 1];
    }
    for (int k = 0; k < 4; ++k) memcpy(x + 3 * k, P3(xw, cv[k]), 3 * sizeof(double));
}

/* the active pair set C(y) (C6) from a candidate superset */
static void active_pairs(const OScene *s, const double *xw, const IVec *cpt, const IVec *cee, IVec *apt, IVec *aee)
{
    double dh2 = s->dhat * s->dhat;
    for (size_t k = 0; k < cpt->n / 2; ++k) {
        int cv[4]; double x[12];
        pair_x(s, xw, 0, cpt->v[2 * k], cpt->v[2 * k + 1], cv, x);
        if (or_dist2_pt(x, NULL) < dh2) { iv_push(apt, cpt->v[2 * k]); iv_push(apt, cpt->v[2 * k + 1]); }
    }
    for (size_t k = 0; k < cee->n / 2; ++k) {
        int cv[4]; double x[12];
        pair_x(s, xw, 1, cee->v[2 * k], cee->v[2 * k + 1], cv, x);
        if (or_dist2_ee(x, NULL) < dh2) { iv_push(aee, cee->v[2 * k]); iv_push(aee, cee->v[2 * k + 1]); }
    }
}

static double *world_alloc(const OScene *s, const double *y)
{
    double *xw = xmalloc(sizeof(double) * 3 * (size_t)(s->ncv ? s->ncv : 1));
    or_world(s, y, xw);
    return xw;
}

int or_pairs(OScene *s, const double *y, int *pt, int cap_pt, int *ee, int cap_ee, int *n_pt, int *n_ee)
{
    double *xw = world_alloc(s, y);
    IVec cpt = {0}, cee = {0}, apt = {0}, aee = {0};
    candidates(s, xw, xw, &cpt, &cee);
    active_pairs(s, xw, &cpt, &cee, &apt, &aee);
    int np = (int)(apt.n / 2), ne = (int)(aee.n / 2);
    *n_pt = np; *n_ee = ne;
    int rc = 0;
    if (np > cap_pt || ne > cap_ee) rc = -1;
    else {
        for (int k = 0; k < np; ++k) {
            int t = apt.v[2 * k + 1];
            pt[4 * k] = apt.v[2 * k];
            for (int m = 0; m < 3; ++m) pt[4 * k + 1 + m] = s->tri[3 * t + m];
        }
        for (int k = 0; k < ne; ++k) {
            const int *a = s->edge + 2 * aee.v[2 * k], *b = s->edge + 2 * aee.v[2 * k + 1];
            ee[4 * k] = a[0]; ee[4 * k + 1] = a[1]; ee[4 * k + 2] = b[0]; ee[4 * k + 3] = b[1];
        }
        qsort(pt, np, 4 * sizeof(int), cmp_int4);
        qsort(ee, ne, 4 * sizeof(int), cmp_int4);
    }
    free(cpt.v); free(cee.v); free(apt.v); free(aee.v); free(xw);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Stable Neo-Hookean (C3)                                                  */
/* ------------------------------------------------------------------------ */
/* F, P column-major (F[3*c + r] = F_rc).  The rest-stable form
 *   Psi = mu/2 (|F|^2 - 3) - mu (J - 1) + lh/2 (J - 1)^2,  lh = lam + mu,
 * whose small-strain limit is mu eps:eps + lam/2 tr(eps)^2. */
double or_snh(const double *F, double mu, double lam, double *P, double *HF)
{
    double lh = lam + mu;
    const double *f0 = F, *f1 = F + 3, *f2 = F + 6;
    double cof[9];
    cross3(f1, f2, cof); cross3(f2, f0, cof + 3); cross3(f0, f1, cof + 6);
    double J = dot3(f0, cof);
    double I2 = 0.0;
    for (int i = 0; i < 9; ++i) I2 += F[i] * F[i];
    double psi = 0.5 * mu * (I2 - 3.0) - mu * (J - 1.0) + 0.5 * lh * (J - 1.0) * (J - 1.0);
    double sc = lh * (J - 1.0) - mu;
    if (P) for (int i = 0; i < 9; ++i) P[i] = mu * F[i] + sc * cof[i];
    if (HF) {
        for (int i = 0; i < 81; ++i) HF[i] = 0.0;
        for (int i = 0; i < 9; ++i) {
            HF[i * 9 + i] += mu;
            for (int j = 0; j < 9; ++j) HF[i * 9 + j] += lh * cof[i] * cof[j];
        }
        /* d^2 J / dF^2: block (a,b) over columns = +-[f_c]x */
        const double *fc[3] = {f0, f1, f2};
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                if (a == b) continue;
                int c = 3 - a - b;
                /* d(f_{a+1} x f_{a+2})/d f_b : sign +1 when b == a+2 (mod 3), else -1 */
                double sg = (b == (a + 2) % 3) ? 1.0 : -1.0;
                const double *v = fc[c];
                double Xm[9] = {0, -v[2], v[1], v[2], 0, -v[0], -v[1], v[0], 0};
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) HF[(3 * a + i) * 9 + 3 * b + j] += sc * sg * Xm[i * 3 + j];
            }
    }
    return psi;
}

/* dF/dx coefficients: f_j depends on x_a through c[a][j] */
static void dFdx_coef(const double *B, double c[4][3])
{
    for (int j = 0; j < 3; ++j) {
        c[1][j] = B[0 * 3 + j]; c[2][j] = B[1 * 3 + j]; c[3][j] = B[2 * 3 + j];
        c[0][j] = -(c[1][j] + c[2][j] + c[3][j]);
    }
}
static void tet_F(const OScene *s, const double *y, int e, double *F, double c[4][3])
{
    const int *t = s->tets + 4 * e;
    const double *B = s->Bm + 9 * e;
    dFdx_coef(B, c);
    for (int j = 0; j < 3; ++j)
        for (int r = 0; r < 3; ++r) {
            double acc = 0.0;
            for (int a = 0; a < 4; ++a) acc += c[a][j] * y[3 * t[a] + r];
            F[3 * j + r] = acc;
        }
}

/* ------------------------------------------------------------------------ */
/* affine-body orthogonality (C4): E = kappa V |A A^T - I|^2                 */
/* ------------------------------------------------------------------------ */
static double abd_energy(const double *q, double kv, double *g /*9*/, double *H /*81*/)
{
    double A[3][3]; /* A[r][c] = column c, row r = q[3 + 3c + r] */
    for (int c = 0; c < 3; ++c) for (int r = 0; r < 3; ++r) A[r][c] = q[3 + 3 * c + r];
    double C[3][3], AtA[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double a = 0, b = 0;
            for (int k = 0; k < 3; ++k) { a += A[i][k] * A[j][k]; b += A[k][i] * A[k][j]; }
            C[i][j] = a - (i == j ? 1.0 : 0.0);
            AtA[i][j] = b;
        }
    double E = 0.0;
    for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) E += C[i][j] * C[i][j];
    E *= kv;
    if (g)
        for (int b = 0; b < 3; ++b)
            for (int a = 0; a < 3; ++a) {
                double acc = 0.0;
                for (int k = 0; k < 3; ++k) acc += C[a][k] * A[k][b];
                g[3 * b + a] = 4.0 * kv * acc;
            }
    if (H)
        for (int b = 0; b < 3; ++b)
            for (int a = 0; a < 3; ++a)
                for (int d = 0; d < 3; ++d)
                    for (int c = 0; c < 3; ++c)
                        H[(3 * b + a) * 9 + 3 * d + c] = 4.0 * kv * ((a == c ? AtA[b][d] : 0.0) + A[a][d] * A[c][b]
                                                                    + (b == d ? C[a][c] : 0.0));
    return E;
}

/* ------------------------------------------------------------------------ */
/* springs (C5)                                                             */
/* ------------------------------------------------------------------------ */
static void spring_side(const OScene *s, const double *y, int kind, int idx, const double *xb, double *x, OPt *pt)
{
    pt->n = 0;
    if (kind == 0) { memcpy(x, y + 3 * (size_t)idx, 3 * sizeof(double)); pt->n = 1; pt->node[0] = idx; pt->w[0] = 1.0; return; }
    const double *q = kind == 1 ? y + 3 * (size_t)(s->nv + 4 * idx) : s->targets + 12 * idx;
    for (int k = 0; k < 3; ++k) x[k] = q[k] + xb[0] * q[3 + k] + xb[1] * q[6 + k] + xb[2] * q[9 + k];
    if (kind == 1) *pt = body_point(s, idx, xb);
}

/* ------------------------------------------------------------------------ */
/* the incremental potential                                                */
/* ------------------------------------------------------------------------ */
static void terms_push(Terms *T, const OTerm *t)
{
    if (T->n == T->cap) { T->cap = T->cap ? 2 * T->cap : 1024; T->t = realloc(T->t, T->cap * sizeof(OTerm)); if (!T->t) abort(); }
    T->t[T->n++] = *t;
}

/* accumulate a point-space gradient into the DOF gradient */
static void scatter_grad(const OPt *p, const double *gp, double *g, double *gabs)
{
    for (int c = 0; c < p->n; ++c)
        for (int k = 0; k < 3; ++k) {
            double v = p->w[c] * gp[k];
            g[3 * (size_t)p->node[c] + k] += v;
            if (gabs) gabs[3 * (size_t)p->node[c] + k] += fabs(v);
        }
}

/* Barrier contribution of one pair at positions x (12): energy, and optionally
 * the gradient (12) and Hessian (144) in world-vertex coordinates. */
static double pair_barrier(const OScene *s, int kind, const double *x, double eps_x, double *g, double *H)
{
    int t;
    double d2 = dist2_kind(kind, x, &t);
    double dh = s->dhat;
    if (d2 >= dh * dh) { if (g) { memset(g, 0, 12 * sizeof(double)); memset(H, 0, 144 * sizeof(double)); } return 0.0; }
    double d = sqrt(d2);
    double b = barrier(d, dh);
    double m = 1.0, m1 = 0.0, m2 = 0.0, cval = 0.0;
    if (kind == 1) {
        cval = cross2_derivs(x, NULL, NULL);
        if (cval < eps_x) {
            double r = cval / eps_x;
            m = (2.0 - r) * r;
            m1 = 2.0 / eps_x - 2.0 * cval / (eps_x * eps_x);
            m2 = -2.0 / (eps_x * eps_x);
        }
    }
    double E = s->kappa * m * b;
    if (!g) return E;
    double gd2[12], Hd2[144];
    d2_derivs_type(kind, t, x, gd2, Hd2);
    double b1 = barrier_d1(d, dh), b2 = barrier_d2(d, dh);
    /* b as a function of q = d^2: B' = b'/(2d), B'' = (b'' - b'/d)/(4 d^2) */
    double Bq1 = b1 / (2.0 * d), Bq2 = (b2 - b1 / d) / (4.0 * d2);
    for (int i = 0; i < 12; ++i) g[i] = s->kappa * m * Bq1 * gd2[i];
    for (int i = 0; i < 12; ++i)
        for (int j = 0; j < 12; ++j) H[i * 12 + j] = s->kappa * m * (Bq2 * gd2[i] * gd2[j] + Bq1 * Hd2[i * 12 + j]);
    if (kind == 1 && cval < eps_x) {
        double gc[12], Hc[144];
        cross2_derivs(x, gc, Hc);
        for (int i = 0; i < 12; ++i) g[i] += s->kappa * b * m1 * gc[i];
        for (int i = 0; i < 12; ++i)
            for (int j = 0; j < 12; ++j)
                H[i * 12 + j] += s->kappa * (b * (m2 * gc[i] * gc[j] + m1 * Hc[i * 12 + j])
                                             + m1 * Bq1 * (gc[i] * gd2[j] + gd2[i] * gc[j]));
    }
    return E;
}

static double pair_eps_x(const OScene *s, int e, int f) { return 1e-3 * s->edge_rest2[e] * s->edge_rest2[f]; }

/* friction of one lagged pair at positions x (12) */
static double pair_friction(const OScene *s, const OLag *L, const double *x, double *g, double *H)
{
    double ea = s->eps_v * s->h;
    double sumx[3] = {0, 0, 0};
    for (int k = 0; k < 4; ++k) for (int c = 0; c < 3; ++c) sumx[c] += L->beta[k] * x[3 * k + c];
    double dv[3], u[3];
    sub3(sumx, L->rn, dv);
    double nd = dot3(L->nrm, dv);
    for (int c = 0; c < 3; ++c) u[c] = dv[c] - L->nrm[c] * nd;
    double sn = sqrt(dot3(u, u));
    double f0 = sn < ea ? -sn * sn * sn / (3.0 * ea * ea) + sn * sn / ea + ea / 3.0 : sn;
    double w = s->mu * L->lam;
    double E = w * f0;
    if (!g) return E;
    double f1s = sn < ea ? 2.0 / ea - sn / (ea * ea) : 1.0 / sn;   /* f1(s)/s */
    for (int k = 0; k < 4; ++k) for (int c = 0; c < 3; ++c) g[3 * k + c] = w * f1s * L->beta[k] * u[c];
    /* H = w beta beta^T (x) [ (f1' - f1/s)/s^2 u u^T + (f1/s) P ] */
    double cu;
    if (sn < ea) cu = sn > 0.0 ? -1.0 / (sn * ea * ea) : 0.0;
    else cu = -1.0 / (sn * sn * sn);
    double M[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            M[i * 3 + j] = cu * u[i] * u[j] + f1s * ((i == j ? 1.0 : 0.0) - L->nrm[i] * L->nrm[j]);
    for (int k = 0; k < 4; ++k)
        for (int l = 0; l < 4; ++l)
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) H[(3 * k + i) * 12 + 3 * l + j] = w * L->beta[k] * L->beta[l] * M[i * 3 + j];
    return E;
}

/* Evaluate the potential at y; with g (and T) also its gradient (and Hessian terms).
 * pair lists give the active pairs; the lag list gives friction. */
static double eval_ip(OScene *s, const double *y, const IVec *apt, const IVec *aee,
                      double *terms, double *g, double *gabs, Terms *T, int project, int with_friction)
{
    double h2 = s->h * s->h;
    double Ein = 0, Efem = 0, Eabd = 0, Esp = 0, Ebar = 0, Efr = 0;
    int inf = 0;
    if (g) memset(g, 0, sizeof(double) * s->ndof);
    if (gabs) memset(gabs, 0, sizeof(double) * s->ndof);
    OTerm tm;
    /* inertia (C2) */
    for (int i = 0; i < s->nv; ++i) {
        double d[3]; sub3(y + 3 * i, s->xtilde + 3 * i, d);
        Ein += 0.5 * s->mass[i] * dot3(d, d);
        if (g) { OPt p = {1, {i}, {1.0}}; double gp[3] = {s->mass[i] * d[0], s->mass[i] * d[1], s->mass[i] * d[2]}; scatter_grad(&p, gp, g, gabs); }
        if (T) {
            memset(&tm, 0, sizeof tm); tm.np = 1; tm.pt[0].n = 1; tm.pt[0].node[0] = i; tm.pt[0].w[0] = 1.0;
            for (int k = 0; k < 3; ++k) tm.H[k * 3 + k] = s->mass[i];
            terms_push(T, &tm);
        }
    }
    for (int b = 0; b < s->nb; ++b) {
        int n0 = s->nv + 4 * b;
        double Mh[4][4] = {{0}};
        Mh[0][0] = s->bmass[b];
        for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) Mh[1 + i][1 + j] = s->bS[9 * b + 3 * i + j];
        double d[4][3];
        for (int c = 0; c < 4; ++c) sub3(y + 3 * (n0 + c), s->xtilde + 3 * (n0 + c), d[c]);
        for (int c = 0; c < 4; ++c)
            for (int c2 = 0; c2 < 4; ++c2) Ein += 0.5 * Mh[c][c2] * dot3(d[c], d[c2]);
        if (g)
            for (int c = 0; c < 4; ++c) {
                double gp[3] = {0, 0, 0};
                for (int c2 = 0; c2 < 4; ++c2) for (int k = 0; k < 3; ++k) gp[k] += Mh[c][c2] * d[c2][k];
                OPt p = {1, {n0 + c}, {1.0}};
                scatter_grad(&p, gp, g, gabs);
            }
        if (T) {
            memset(&tm, 0, sizeof tm); tm.np = 4;
            for (int c = 0; c < 4; ++c) { tm.pt[c].n = 1; tm.pt[c].node[0] = n0 + c; tm.pt[c].w[0] = 1.0; }
            for (int c = 0; c < 4; ++c) for (int c2 = 0; c2 < 4; ++c2) for (int k = 0; k < 3; ++k)
                tm.H[(3 * c + k) * 12 + 3 * c2 + k] = Mh[c][c2];
            terms_push(T, &tm);
        }
    }
    /* FEM (C3) */
    size_t t_fem0 = T ? T->n : 0;
    if (T) {
        for (int e = 0; e < s->nt; ++e) { memset(&tm, 0, sizeof tm); terms_push(T, &tm); }
    }
    double *pe = xmalloc(sizeof(double) * (size_t)(s->nt ? s->nt : 1));
    double *ge = g ? xmalloc(sizeof(double) * 12 * (size_t)(s->nt ? s->nt : 1)) : NULL;
    /* gradient scale of each tet: the stress terms mu F and (lh (J-1) - mu) cof F
     * before they cancel (near rest they do, and rounding follows their size) */
    double *gs = gabs ? xmalloc(sizeof(double) * 12 * (size_t)(s->nt ? s->nt : 1)) : NULL;
    #pragma omp parallel for schedule(static)
    for (int e = 0; e < s->nt; ++e) {
        double F[9], c[4][3], P[9], HF[81];
        tet_F(s, y, e, F, c);
        double w = h2 * s->vol[e];
        pe[e] = w * or_snh(F, s->lmu[e], s->llam[e], g ? P : NULL, T ? HF : NULL);
        if (g)
            for (int a = 0; a < 4; ++a)
                for (int r = 0; r < 3; ++r) {
                    double acc = 0.0;
                    for (int j = 0; j < 3; ++j) acc += c[a][j] * P[3 * j + r];
                    ge[12 * e + 3 * a + r] = w * acc;
                }
        if (gs) {
            double cof[9];
            cross3(F + 3, F + 6, cof); cross3(F + 6, F, cof + 3); cross3(F, F + 3, cof + 6);
            double J = dot3(F, cof), mu = s->lmu[e], sc = (s->llam[e] + mu) * (J - 1.0) - mu;
            for (int a = 0; a < 4; ++a)
                for (int r = 0; r < 3; ++r) {
                    double acc = 0.0;
                    for (int j = 0; j < 3; ++j) acc += fabs(c[a][j]) * (fabs(mu * F[3 * j + r]) + fabs(sc * cof[3 * j + r]));
                    gs[12 * e + 3 * a + r] = w * acc;
                }
        }
        if (T) {
            if (project) or_psd_project(HF, 9);
            OTerm *tt = T->t + t_fem0 + e;
            tt->np = 4;
            for (int a = 0; a < 4; ++a) { tt->pt[a].n = 1; tt->pt[a].node[0] = s->tets[4 * e + a]; tt->pt[a].w[0] = 1.0; }
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b)
                    for (int r = 0; r < 3; ++r)
                        for (int q = 0; q < 3; ++q) {
                            double acc = 0.0;
                            for (int j = 0; j < 3; ++j)
                                for (int l = 0; l < 3; ++l) acc += c[a][j] * c[b][l] * HF[(3 * j + r) * 9 + 3 * l + q];
                            tt->H[(3 * a + r) * 12 + 3 * b + q] = w * acc;
                        }
        }
    }
    for (int e = 0; e < s->nt; ++e) {
        Efem += pe[e];
        if (g)
            for (int a = 0; a < 4; ++a) {
                OPt p = {1, {s->tets[4 * e + a]}, {1.0}};
                scatter_grad(&p, ge + 12 * e + 3 * a, g, NULL);
                if (gabs) for (int r = 0; r < 3; ++r) gabs[3 * (size_t)s->tets[4 * e + a] + r] += gs[12 * e + 3 * a + r];
            }
    }
    free(pe); free(ge); free(gs);
    /* affine bodies (C4) */
    for (int b = 0; b < s->nb; ++b) {
        int n0 = s->nv + 4 * b;
        double gA[9], HA[81];
        double kv = h2 * s->bkappa[b] * s->bvol[b];
        Eabd += abd_energy(y + 3 * n0, kv, g ? gA : NULL, T ? HA : NULL);
        if (g) for (int c = 0; c < 3; ++c) { OPt p = {1, {n0 + 1 + c}, {1.0}}; scatter_grad(&p, gA + 3 * c, g, NULL); }
        if (gabs) {
            /* scale: 4 kappa V (|A A^T| + I) |A|, the operands of A A^T - I before they cancel */
            const double *q = y + 3 * (size_t)n0;
            for (int bcol = 0; bcol < 3; ++bcol)
                for (int a = 0; a < 3; ++a) {
                    double acc = 0.0;
                    for (int k = 0; k < 3; ++k) {
                        double aat = 0.0;
                        for (int m = 0; m < 3; ++m) aat += fabs(q[3 + 3 * m + a] * q[3 + 3 * m + k]);
                        acc += (aat + (a == k ? 1.0 : 0.0)) * fabs(q[3 + 3 * bcol + k]);
                    }
                    gabs[3 * (size_t)(n0 + 1 + bcol) + a] += 4.0 * kv * acc;
                }
        }
        if (T) {
            if (project) or_psd_project(HA, 9);
            memset(&tm, 0, sizeof tm); tm.np = 3;
            for (int c = 0; c < 3; ++c) { tm.pt[c].n = 1; tm.pt[c].node[0] = n0 + 1 + c; tm.pt[c].w[0] = 1.0; }
            for (int i = 0; i < 9; ++i) for (int j = 0; j < 9; ++j) tm.H[i * 9 + j] = HA[i * 9 + j];
            terms_push(T, &tm);
        }
    }
    /* springs (C5) */
    for (int k = 0; k < s->ns; ++k) {
        double xa[3], xb[3], d[3];
        OPt pa, pb;
        spring_side(s, y, s->sp_ka[k], s->sp_ia[k], s->sp_xa + 3 * k, xa, &pa);
        spring_side(s, y, s->sp_kb[k], s->sp_ib[k], s->sp_xb + 3 * k, xb, &pb);
        sub3(xa, xb, d);
        double kk = h2 * s->sp_k[k];
        Esp += 0.5 * kk * dot3(d, d);
        if (g) {
            double ga[3] = {kk * d[0], kk * d[1], kk * d[2]}, gb[3] = {-ga[0], -ga[1], -ga[2]};
            scatter_grad(&pa, ga, g, NULL); scatter_grad(&pb, gb, g, NULL);
            if (gabs) {
                /* scale: h^2 k (|a| + |b|), the operands of a - b before they cancel */
                double sa[3] = {kk * (fabs(xa[0]) + fabs(xb[0])), kk * (fabs(xa[1]) + fabs(xb[1])), kk * (fabs(xa[2]) + fabs(xb[2]))};
                for (int side = 0; side < 2; ++side) {
                    const OPt *pp = side ? &pb : &pa;
                    for (int c = 0; c < pp->n; ++c)
                        for (int k2 = 0; k2 < 3; ++k2) gabs[3 * (size_t)pp->node[c] + k2] += fabs(pp->w[c]) * sa[k2];
                }
            }
        }
        if (T) {
            memset(&tm, 0, sizeof tm); tm.np = 2; tm.pt[0] = pa; tm.pt[1] = pb;
            for (int a = 0; a < 2; ++a) for (int b2 = 0; b2 < 2; ++b2) for (int i = 0; i < 3; ++i)
                tm.H[(3 * a + i) * 6 + 3 * b2 + i] = (a == b2 ? kk : -kk);
            terms_push(T, &tm);
        }
    }
    /* barrier (C8) */
    double *xw = world_alloc(s, y);
    for (int kind = 0; kind < 2; ++kind) {
        const IVec *L = kind == 0 ? apt : aee;
        if (!L) continue;
        for (size_t k = 0; k < L->n / 2; ++k) {
            int cv[4]; double x[12], gp[12], Hp[144];
            int i = L->v[2 * k], j = L->v[2 * k + 1];
            pair_x(s, xw, kind, i, j, cv, x);
            double ex = kind == 1 ? pair_eps_x(s, i, j) : 0.0;
            double d2 = dist2_kind(kind, x, NULL);
            if (d2 <= 0.0) { inf = 1; continue; }
            Ebar += pair_barrier(s, kind, x, ex, g ? gp : NULL, g ? Hp : NULL);
            if (g) for (int a = 0; a < 4; ++a) { OPt p = cv_point(s, cv[a]); scatter_grad(&p, gp + 3 * a, g, gabs); }
            if (T) {
                if (project) or_psd_project(Hp, 12);
                memset(&tm, 0, sizeof tm); tm.np = 4;
                for (int a = 0; a < 4; ++a) tm.pt[a] = cv_point(s, cv[a]);
                memcpy(tm.H, Hp, sizeof Hp);
                terms_push(T, &tm);
            }
        }
    }
    /* the half-space: kappa b(d) per dynamic surface vertex, d = n . x - c;
     * gradient kappa b'(d) n, Hessian kappa b''(d) n n^T (b'' > 0 below
     * dhat, so the term is convex and needs no projection) */
    if (s->hs_on)
        for (int k = 0; k < s->nsurf; ++k) {
            int c = s->surf_v[k];
            if (!cv_dynamic(s, c)) continue;
            double d = hs_dist(s, P3(xw, c));
            if (d <= 0.0) { inf = 1; continue; }
            if (d >= s->dhat) continue;
            Ebar += s->kappa * barrier(d, s->dhat);
            OPt p = cv_point(s, c);
            if (g) {
                double b1 = s->kappa * barrier_d1(d, s->dhat), gp[3];
                for (int q = 0; q < 3; ++q) gp[q] = b1 * s->hs_n[q];
                scatter_grad(&p, gp, g, gabs);
            }
            if (T) {
                double b2 = s->kappa * barrier_d2(d, s->dhat);
                memset(&tm, 0, sizeof tm); tm.np = 1; tm.pt[0] = p;
                for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) tm.H[3 * i + j] = b2 * s->hs_n[i] * s->hs_n[j];
                terms_push(T, &tm);
            }
        }
    /* friction (C10) */
    if (with_friction)
        for (int k = 0; k < s->nlag; ++k) {
            const OLag *L = s->lag + k;
            double x[12], gp[12], Hp[144];
            for (int a = 0; a < 4; ++a) memcpy(x + 3 * a, P3(xw, L->cv[a]), 3 * sizeof(double));
            Efr += pair_friction(s, L, x, g ? gp : NULL, g ? Hp : NULL);
            if (g) for (int a = 0; a < 4; ++a) { OPt p = cv_point(s, L->cv[a]); scatter_grad(&p, gp + 3 * a, g, gabs); }
            if (T) {
                memset(&tm, 0, sizeof tm); tm.np = 4;
                for (int a = 0; a < 4; ++a) tm.pt[a] = cv_point(s, L->cv[a]);
                memcpy(tm.H, Hp, sizeof Hp);
                terms_push(T, &tm);
            }
        }
    free(xw);
    double tot = Ein + Efem + Eabd + Esp + Ebar + Efr;
    if (inf) tot = INFINITY;
    if (terms) { terms[0] = Ein; terms[1] = Efem; terms[2] = Eabd; terms[3] = Esp; terms[4] = Ebar; terms[5] = Efr; terms[6] = tot; }
    return tot;
}

/* out = sum over terms of P^T H P v; outabs (nullable) receives the same sum
 * with every factor replaced by its absolute value, |P|^T |H| |P| |v|: the
 * size of the operands whose rounding forms each entry of out. */
static void terms_matvec(const OScene *s, const Terms *T, const double *v, double *out, double *outabs)
{
    memset(out, 0, sizeof(double) * s->ndof);
    if (outabs) memset(outabs, 0, sizeof(double) * s->ndof);
    for (size_t k = 0; k < T->n; ++k) {
        const OTerm *t = T->t + k;
        int m = 3 * t->np;
        double vl[12], yl[12], va[12], ya[12];
        for (int a = 0; a < t->np; ++a)
            for (int c = 0; c < 3; ++c) {
                double acc = 0.0, aa = 0.0;
                for (int q = 0; q < t->pt[a].n; ++q) {
                    double vq = v[3 * (size_t)t->pt[a].node[q] + c];
                    acc += t->pt[a].w[q] * vq;
                    aa += fabs(t->pt[a].w[q]) * fabs(vq);
                }
                vl[3 * a + c] = acc;
                va[3 * a + c] = aa;
            }
        for (int i = 0; i < m; ++i) {
            double acc = 0.0, aa = 0.0;
            for (int j = 0; j < m; ++j) { acc += t->H[i * m + j] * vl[j]; aa += fabs(t->H[i * m + j]) * va[j]; }
            yl[i] = acc;
            ya[i] = aa;
        }
        for (int a = 0; a < t->np; ++a)
            for (int q = 0; q < t->pt[a].n; ++q)
                for (int c = 0; c < 3; ++c) {
                    size_t o = 3 * (size_t)t->pt[a].node[q] + c;
                    out[o] += t->pt[a].w[q] * yl[3 * a + c];
                    if (outabs) outabs[o] += fabs(t->pt[a].w[q]) * ya[3 * a + c];
                }
    }
}

/* The dense Hessian (ndof x ndof, row-major) of the terms T, P^T H P summed
 * over terms; Habs (nullable) the same sum of |P|^T |H| |P|. */
static void terms_dense(const OScene *s, const Terms *T, double *H, double *Habs)
{
    size_t n = (size_t)s->ndof;
    memset(H, 0, sizeof(double) * n * n);
    if (Habs) memset(Habs, 0, sizeof(double) * n * n);
    for (size_t k = 0; k < T->n; ++k) {
        const OTerm *t = T->t + k;
        int m = 3 * t->np;
        for (int a = 0; a < t->np; ++a)
            for (int qa = 0; qa < t->pt[a].n; ++qa)
                for (int b = 0; b < t->np; ++b)
                    for (int qb = 0; qb < t->pt[b].n; ++qb) {
                        double w = t->pt[a].w[qa] * t->pt[b].w[qb];
                        size_t r0 = 3 * (size_t)t->pt[a].node[qa], c0 = 3 * (size_t)t->pt[b].node[qb];
                        for (int i = 0; i < 3; ++i)
                            for (int j = 0; j < 3; ++j) {
                                double h = t->H[(3 * a + i) * m + 3 * b + j];
                                H[(r0 + i) * n + c0 + j] += w * h;
                                if (Habs) Habs[(r0 + i) * n + c0 + j] += fabs(w) * fabs(h);
                            }
                    }
    }
}

/* ------------------------------------------------------------------------ */
/* friction lag (C10)                                                        */
/* ------------------------------------------------------------------------ */
/* The lag at state ylag (active pairs, closest-point weights, normals and
 * normal forces there); the tangential displacement of a pair is measured
 * from its weighted closest-point sum at state yref (NULL: ylag), i.e. from
 * the step start whatever the state the lag was taken at. */
static void compute_lag_at(OScene *s, const double *ylag, const double *yref)
{
    free(s->lag); s->lag = NULL; s->nlag = 0;
    double *xw = world_alloc(s, ylag);
    double *xr = yref ? world_alloc(s, yref) : NULL;
    IVec cpt = {0}, cee = {0}, apt = {0}, aee = {0};
    candidates(s, xw, xw, &cpt, &cee);
    active_pairs(s, xw, &cpt, &cee, &apt, &aee);
    int n = (int)(apt.n / 2 + aee.n / 2) + (s->hs_on ? s->nsurf : 0);
    s->lag = xmalloc(sizeof(OLag) * (size_t)(n ? n : 1));
    for (int kind = 0; kind < 2; ++kind) {
        const IVec *L = kind == 0 ? &apt : &aee;
        for (size_t k = 0; k < L->n / 2; ++k) {
            OLag *lg = s->lag + s->nlag;
            double x[12], Dm[6];
            int i = L->v[2 * k], j = L->v[2 * k + 1], t;
            pair_x(s, xw, kind, i, j, lg->cv, x);
            double d2 = dist2_kind(kind, x, &t);
            double d = sqrt(d2);
            Param P = type_param(kind, t);
            double r[3];
            closest(&P, x, lg->beta, r, Dm);
            double rn = sqrt(dot3(r, r));
            for (int c = 0; c < 3; ++c) { lg->nrm[c] = r[c] / rn; lg->rn[c] = r[c]; }
            if (xr) {   /* the same weights on the reference positions */
                double xref[12];
                int cvr[4];
                pair_x(s, xr, kind, i, j, cvr, xref);
                for (int c = 0; c < 3; ++c) {
                    double acc = 0.0;
                    for (int q = 0; q < 4; ++q) acc += lg->beta[q] * xref[3 * q + c];
                    lg->rn[c] = acc;
                }
            }
            double m = 1.0;
            lg->kind = kind;
            lg->type = t;
            lg->ex = 0.0;
            if (kind == 1) {
                double ex = pair_eps_x(s, i, j), c = cross2_derivs(x, NULL, NULL);
                lg->ex = ex;
                if (c < ex) m = (2.0 - c / ex) * (c / ex);
            }
            lg->lam = -s->kappa * m * barrier_d1(d, s->dhat);
            s->nlag++;
        }
    }
    /* the half-space: a vertex closer than dhat at the lag state is one
     * lagged contact with normal n, weights (1, 0, 0, 0) on the vertex itself
     * and offset its reference position */
    if (s->hs_on)
        for (int k = 0; k < s->nsurf; ++k) {
            int c = s->surf_v[k];
            if (!cv_dynamic(s, c)) continue;
            double d = hs_dist(s, P3(xw, c));
            if (!(d > 0.0) || d >= s->dhat) continue;
            OLag *lg = s->lag + s->nlag;
            for (int q = 0; q < 4; ++q) { lg->cv[q] = c; lg->beta[q] = q == 0 ? 1.0 : 0.0; }
            memcpy(lg->nrm, s->hs_n, 3 * sizeof(double));
            memcpy(lg->rn, P3(xr ? xr : xw, c), 3 * sizeof(double));
            lg->kind = 2;
            lg->type = 0;
            lg->ex = 0.0;
            lg->lam = -s->kappa * barrier_d1(d, s->dhat);
            s->nlag++;
        }
    free(cpt.v); free(cee.v); free(apt.v); free(aee.v); free(xw); free(xr);
}

static void compute_lag(OScene *s) { compute_lag_at(s, s->y, NULL); }

void or_begin_step(OScene *s, const double *targets)
{
    double h = s->h;
    for (int i = 0; i < s->nv; ++i)
        for (int k = 0; k < 3; ++k) s->xtilde[3 * i + k] = s->y[3 * i + k] + h * s->ydot[3 * i + k] + h * h * s->g[k];
    for (int b = 0; b < s->nb; ++b) {
        size_t o = 3 * (size_t)(s->nv + 4 * b);
        for (int i = 0; i < 12; ++i) s->xtilde[o + i] = s->y[o + i] + h * s->ydot[o + i] + (i < 3 ? h * h * s->g[i] : 0.0);
    }
    if (targets && s->nd) memcpy(s->targets, targets, sizeof(double) * 12 * s->nd);
    /* joint references: the b-side body-frame point of every joint spring */
    if (targets)
        for (int j = 0; j < s->nj; ++j) memcpy(s->sp_xb + 3 * (size_t)s->joint_spring[j], targets + 12 * (size_t)s->nd + 3 * j, 3 * sizeof(double));
    compute_lag(s);
}

/* ------------------------------------------------------------------------ */
/* public evaluation entry points                                           */
/* ------------------------------------------------------------------------ */
static void pairs_at(OScene *s, const double *y, IVec *apt, IVec *aee)
{
    double *xw = world_alloc(s, y);
    IVec cpt = {0}, cee = {0};
    candidates(s, xw, xw, &cpt, &cee);
    active_pairs(s, xw, &cpt, &cee, apt, aee);
    free(cpt.v); free(cee.v); free(xw);
}

double or_energy(OScene *s, const double *y, double *terms)
{
    IVec apt = {0}, aee = {0};
    pairs_at(s, y, &apt, &aee);
    double E = eval_ip(s, y, &apt, &aee, terms, NULL, NULL, NULL, 0, 1);
    free(apt.v); free(aee.v);
    return E;
}

void or_gradient(OScene *s, const double *y, double *g, double *gabs)
{
    IVec apt = {0}, aee = {0};
    pairs_at(s, y, &apt, &aee);
    eval_ip(s, y, &apt, &aee, NULL, g, gabs, NULL, 0, 1);
    free(apt.v); free(aee.v);
}

void or_hessian_matvec(OScene *s, const double *y, int project, const double *v, double *out)
{
    or_hessian_matvec_abs(s, y, project, 1, v, out, NULL);
}

void or_hessian_matvec_abs(OScene *s, const double *y, int project, int with_friction, const double *v, double *out,
                           double *outabs)
{
    IVec apt = {0}, aee = {0};
    pairs_at(s, y, &apt, &aee);
    Terms T = {0};
    double *g = xmalloc(sizeof(double) * s->ndof);
    eval_ip(s, y, &apt, &aee, NULL, g, NULL, &T, project, with_friction);
    terms_matvec(s, &T, v, out, outabs);
    free(g); free(T.t); free(apt.v); free(aee.v);
}

void or_hessian_dense(OScene *s, const double *y, int project, int with_friction, double *H, double *Habs)
{
    IVec apt = {0}, aee = {0};
    pairs_at(s, y, &apt, &aee);
    Terms T = {0};
    double *g = xmalloc(sizeof(double) * s->ndof);
    eval_ip(s, y, &apt, &aee, NULL, g, NULL, &T, project, with_friction);
    terms_dense(s, &T, H, Habs);
    free(g); free(T.t); free(apt.v); free(aee.v);
}

/* ------------------------------------------------------------------------ */
/* block-Jacobi PCG (C12)                                                   */
/* ------------------------------------------------------------------------ */
static int group_of(const OScene *s, int node, int *local)
{
    if (node < s->nv) { *local = 0; return node; }
    *local = (node - s->nv) % 4;
    return s->nv + (node - s->nv) / 4;
}

/* PCG on the terms T with their block-Jacobi preconditioner.  Returns the
 * iterations; *indef (nullable) is set when some p^T A p <= 0 stopped it. */
static int pcg_terms(OScene *s, const Terms *T, const double *b, double *x, double eta, int maxit, int *indef)
{
    int n = s->ndof;
    /* block diagonal: 3x3 per FEM vertex, 12x12 per body */
    double *Dv = xcalloc(9 * (size_t)(s->nv ? s->nv : 1), sizeof(double));
    double *Db = xcalloc(144 * (size_t)(s->nb ? s->nb : 1), sizeof(double));
    for (size_t k = 0; k < T->n; ++k) {
        const OTerm *t = T->t + k;
        int m = 3 * t->np;
        for (int a = 0; a < t->np; ++a)
            for (int b2 = 0; b2 < t->np; ++b2)
                for (int qa = 0; qa < t->pt[a].n; ++qa)
                    for (int qb = 0; qb < t->pt[b2].n; ++qb) {
                        int la, lb;
                        int ga = group_of(s, t->pt[a].node[qa], &la), gb = group_of(s, t->pt[b2].node[qb], &lb);
                        if (ga != gb) continue;
                        double w = t->pt[a].w[qa] * t->pt[b2].w[qb];
                        for (int i = 0; i < 3; ++i)
                            for (int j = 0; j < 3; ++j) {
                                double v = w * t->H[(3 * a + i) * m + 3 * b2 + j];
                                if (ga < s->nv) Dv[9 * (size_t)ga + 3 * i + j] += v;
                                else Db[144 * (size_t)(ga - s->nv) + (3 * la + i) * 12 + 3 * lb + j] += v;
                            }
                    }
    }
    double *Iv = xmalloc(sizeof(double) * 9 * (size_t)(s->nv ? s->nv : 1));
    double *Ib = xmalloc(sizeof(double) * 144 * (size_t)(s->nb ? s->nb : 1));
    for (int i = 0; i < s->nv; ++i) invert(Dv + 9 * (size_t)i, 3, Iv + 9 * (size_t)i);
    for (int b2 = 0; b2 < s->nb; ++b2) invert(Db + 144 * (size_t)b2, 12, Ib + 144 * (size_t)b2);
    double *r = xmalloc(sizeof(double) * n), *z = xmalloc(sizeof(double) * n), *p = xmalloc(sizeof(double) * n),
           *Ap = xmalloc(sizeof(double) * n);
#define PREC(src, dst) do { \
        for (int i_ = 0; i_ < s->nv; ++i_) for (int a_ = 0; a_ < 3; ++a_) { double acc_ = 0; \
            for (int b_ = 0; b_ < 3; ++b_) acc_ += Iv[9 * (size_t)i_ + 3 * a_ + b_] * (src)[3 * i_ + b_]; (dst)[3 * i_ + a_] = acc_; } \
        for (int q_ = 0; q_ < s->nb; ++q_) { size_t o_ = 3 * (size_t)s->nv + 12 * (size_t)q_; \
            for (int a_ = 0; a_ < 12; ++a_) { double acc_ = 0; \
                for (int b_ = 0; b_ < 12; ++b_) acc_ += Ib[144 * (size_t)q_ + 12 * a_ + b_] * (src)[o_ + b_]; (dst)[o_ + a_] = acc_; } } \
    } while (0)
    double bn = 0.0;
    for (int i = 0; i < n; ++i) { x[i] = 0.0; r[i] = b[i]; bn += b[i] * b[i]; }
    bn = sqrt(bn);
    int it = 0;
    if (indef) *indef = 0;
    if (bn > 0.0) {
        PREC(r, z);
        double rz = 0.0;
        for (int i = 0; i < n; ++i) { p[i] = z[i]; rz += r[i] * z[i]; }
        for (it = 1; it <= maxit; ++it) {
            terms_matvec(s, T, p, Ap, NULL);
            double pAp = 0.0;
            for (int i = 0; i < n; ++i) pAp += p[i] * Ap[i];
            if (!(pAp > 0.0)) { if (indef) *indef = 1; break; }
            double al = rz / pAp, rn = 0.0;
            for (int i = 0; i < n; ++i) { x[i] += al * p[i]; r[i] -= al * Ap[i]; rn += r[i] * r[i]; }
            if (sqrt(rn) <= eta * bn) break;
            PREC(r, z);
            double rz2 = 0.0;
            for (int i = 0; i < n; ++i) rz2 += r[i] * z[i];
            double be = rz2 / rz;
            rz = rz2;
            for (int i = 0; i < n; ++i) p[i] = z[i] + be * p[i];
        }
        if (it > maxit) it = maxit;
    }
#undef PREC
    free(Dv); free(Db); free(Iv); free(Ib); free(r); free(z); free(p); free(Ap);
    return it;
}

int or_pcg(OScene *s, const double *y, const double *b, double *x, double eta)
{
    IVec apt = {0}, aee = {0};
    pairs_at(s, y, &apt, &aee);
    Terms T = {0};
    double *g = xmalloc(sizeof(double) * s->ndof);
    eval_ip(s, y, &apt, &aee, NULL, g, NULL, &T, 1, 1);
    int it = pcg_terms(s, &T, b, x, eta, s->max_pcg, NULL);
    free(g); free(T.t); free(apt.v); free(aee.v);
    return it;
}

/* ------------------------------------------------------------------------ */
/* additive CCD (C13)                                                       */
/* ------------------------------------------------------------------------ */
double or_accd(int kind, const double *x, const double *p, double s)
{
    double dp[12], xx[12], pm[3] = {0, 0, 0};
    for (int k = 0; k < 4; ++k) for (int c = 0; c < 3; ++c) pm[c] += p[3 * k + c];
    for (int c = 0; c < 3; ++c) pm[c] /= 4.0;
    for (int k = 0; k < 4; ++k) for (int c = 0; c < 3; ++c) dp[3 * k + c] = p[3 * k + c] - pm[c];
    double nrm[4];
    for (int k = 0; k < 4; ++k) nrm[k] = sqrt(dot3(dp + 3 * k, dp + 3 * k));
    double lp;
    if (kind == 0) {
        double mb = nrm[1]; if (nrm[2] > mb) mb = nrm[2]; if (nrm[3] > mb) mb = nrm[3];
        lp = nrm[0] + mb;
    } else {
        lp = (nrm[0] > nrm[1] ? nrm[0] : nrm[1]) + (nrm[2] > nrm[3] ? nrm[2] : nrm[3]);
    }
    if (lp == 0.0) return 1.0;
    memcpy(xx, x, sizeof xx);
    double d = sqrt(dist2_kind(kind, xx, NULL));
    double gap = s * d;
    double t = 0.0, tl = (1.0 - s) * d / lp;
    for (int it = 0; it < 10000; ++it) {
        for (int i = 0; i < 12; ++i) xx[i] += tl * dp[i];
        d = sqrt(dist2_kind(kind, xx, NULL));
        if (t > 0.0 && d < gap) return t;
        t += tl;
        if (t > 1.0) return 1.0;
        tl = 0.9 * d / lp;
    }
    return t;
}

static double ccd_alpha(const OScene *s, const double *xw0, const double *xw1, const IVec *cpt, const IVec *cee)
{
    double a = 1.0;
    for (int kind = 0; kind < 2; ++kind) {
        const IVec *L = kind == 0 ? cpt : cee;
        for (size_t k = 0; k < L->n / 2; ++k) {
            int cv[4]; double x0[12], x1[12], p[12];
            pair_x(s, xw0, kind, L->v[2 * k], L->v[2 * k + 1], cv, x0);
            pair_x(s, xw1, kind, L->v[2 * k], L->v[2 * k + 1], cv, x1);
            for (int i = 0; i < 12; ++i) p[i] = x1[i] - x0[i];
            double t = or_accd(kind, x0, p, s->ccd_s);
            if (t < a) a = t;
        }
    }
    /* the half-space: along x0 + t p the distance d0 + t (n . p) is linear,
     * so the step at which it reaches the additive CCD's gap s d0 is exact */
    if (s->hs_on)
        for (int k = 0; k < s->nsurf; ++k) {
            int c = s->surf_v[k];
            if (!cv_dynamic(s, c)) continue;
            const double *x0 = P3(xw0, c), *x1 = P3(xw1, c);
            double p[3] = {x1[0] - x0[0], x1[1] - x0[1], x1[2] - x0[2]};
            double d0 = hs_dist(s, x0);
            double np = s->hs_n[0] * p[0] + s->hs_n[1] * p[1] + s->hs_n[2] * p[2];
            if (np < 0.0) {
                double t = (1.0 - s->ccd_s) * d0 / -np;
                if (t < a) a = t;
            }
        }
    return a;
}

double or_ccd(OScene *s, const double *y, const double *p)
{
    double *y1 = xmalloc(sizeof(double) * s->ndof);
    for (int i = 0; i < s->ndof; ++i) y1[i] = y[i] + p[i];
    double *xw0 = world_alloc(s, y), *xw1 = world_alloc(s, y1);
    IVec cpt = {0}, cee = {0};
    candidates(s, xw0, xw1, &cpt, &cee);
    double a = ccd_alpha(s, xw0, xw1, &cpt, &cee);
    free(cpt.v); free(cee.v); free(xw0); free(xw1); free(y1);
    return a;
}

/* ------------------------------------------------------------------------ */
/* the Newton step (C13)                                                    */
/* ------------------------------------------------------------------------ */
static double newton_measure(const OScene *s, const double *p)
{
    double m = 0.0;
    for (int i = 0; i < 3 * s->nv; ++i) if (fabs(p[i]) > m) m = fabs(p[i]);
    for (int b = 0; b < s->nb; ++b) {
        const double *q = p + 3 * (size_t)(s->nv + 4 * b), *e = s->bext + 3 * b;
        for (int k = 0; k < 3; ++k) {
            double v = fabs(q[k]) + e[0] * fabs(q[3 + k]) + e[1] * fabs(q[6 + k]) + e[2] * fabs(q[9 + k]);
            if (v > m) m = v;
        }
    }
    return m;
}

/* A new time step h > 0: every use of h (predictor, h^2 weights, friction
 * regularisation eps_v h, Newton stop) reads s->h; kappa keeps its value. */
void or_set_timestep(OScene *s, double h)
{
    if (h > 0.0) s->h = h;
}

/* Friction lag passes per step (1: lagged once at the step start). */
void or_set_friction_lag(OScene *s, int passes)
{
    if (passes >= 1) s->lag_passes = passes;
}

/* The smallest distance over the pairs active at y (closer than dhat);
 * INFINITY when none is. */
static double min_active_distance(OScene *s, const double *y)
{
    IVec apt = {0}, aee = {0};
    pairs_at(s, y, &apt, &aee);
    double *xw = world_alloc(s, y);
    double m2 = INFINITY;
    for (int kind = 0; kind < 2; ++kind) {
        const IVec *L = kind == 0 ? &apt : &aee;
        for (size_t k = 0; k < L->n / 2; ++k) {
            int cv[4]; double x[12];
            pair_x(s, xw, kind, L->v[2 * k], L->v[2 * k + 1], cv, x);
            double d2 = dist2_kind(kind, x, NULL);
            if (d2 < m2) m2 = d2;
        }
    }
    double m = sqrt(m2);
    if (s->hs_on)   /* vertices closer than dhat to the half-space */
        for (int k = 0; k < s->nsurf; ++k) {
            int c = s->surf_v[k];
            if (!cv_dynamic(s, c)) continue;
            double d = hs_dist(s, P3(xw, c));
            if (d < s->dhat && d < m) m = d > 0.0 ? d : 0.0;
        }
    free(xw); free(apt.v); free(aee.v);
    return m;
}

/* Adaptive barrier stiffness (IPC's rule; a robustness variant of the
 * barrier term of Eq. (3)): frac > 0 switches it on with kappa0 = the
 * current kappa, frac = 0 off (kappa keeps its value); factor >= 1 caps
 * kappa at factor kappa0. */
void or_set_kappa_adaptive(OScene *s, double frac, double factor)
{
    if (frac >= 0.0) s->kappa_frac = frac;
    if (factor >= 1.0) s->kappa_factor = factor;
    s->kappa0 = s->kappa;
}

void or_set_kappa(OScene *s, double kappa)
{
    if (kappa > 0.0) s->kappa = s->kappa0 = kappa;
}

int or_step(OScene *s, const double *targets, OStats *st)
{
    OStats loc; memset(&loc, 0, sizeof loc);
    loc.alpha_min = 1.0;
    or_begin_step(s, targets);
    loc.n_lag = s->nlag;
    int n = s->ndof;
    double *y = xmalloc(sizeof(double) * n), *g = xmalloc(sizeof(double) * n), *p = xmalloc(sizeof(double) * n),
           *b = xmalloc(sizeof(double) * n), *yt = xmalloc(sizeof(double) * n);
    memcpy(y, s->y, sizeof(double) * n);
    double thr = s->newton_tol * s->h * s->L;
    int status = 3;
    if (s->kappa_frac > 0.0) s->dmin_prev = min_active_distance(s, y);
    /* friction lag passes: after a converged pass, the lag is taken again at
     * the solution (displacements still from the step start) and Newton
     * runs again from there */
    for (int pass = 0; pass < s->lag_passes; ++pass) {
    if (pass > 0) {
        if (status != 0) break;
        compute_lag_at(s, y, s->y);
        status = 3;
    }
    for (int j = 0; j < s->max_newton; ++j) {
        IVec apt = {0}, aee = {0};
        pairs_at(s, y, &apt, &aee);
        if ((int)(apt.n / 2) > loc.n_pt_max) loc.n_pt_max = (int)(apt.n / 2);
        if ((int)(aee.n / 2) > loc.n_ee_max) loc.n_ee_max = (int)(aee.n / 2);
        Terms T = {0};
        double E0 = eval_ip(s, y, &apt, &aee, NULL, g, NULL, &T, 1, 1);
        for (int i = 0; i < n; ++i) b[i] = -g[i];
        int it = pcg_terms(s, &T, b, p, s->pcg_tol, s->max_pcg, NULL);
        free(T.t); free(apt.v); free(aee.v);
        loc.pcg_iters_total += it;
        if (it > loc.pcg_iters_max) loc.pcg_iters_max = it;
        loc.newton_iters++;
        loc.energy = E0;
        if (newton_measure(s, p) <= thr) { status = 0; break; }
        /* CCD over the swept candidates, then backtracking on the energy */
        for (int i = 0; i < n; ++i) yt[i] = y[i] + p[i];
        double *xw0 = world_alloc(s, y), *xw1 = world_alloc(s, yt);
        IVec cpt = {0}, cee = {0};
        candidates(s, xw0, xw1, &cpt, &cee);
        double alpha = ccd_alpha(s, xw0, xw1, &cpt, &cee);
        /* the energy the trials are compared with: E(y) over the active pairs
         * taken from the same candidate list as the trials', summed in the
         * same order, so that a decrease smaller than the sums' rounding is
         * not lost to a change of summation order */
        {
            IVec cp0 = {0}, ce0 = {0};
            active_pairs(s, xw0, &cpt, &cee, &cp0, &ce0);
            E0 = eval_ip(s, y, &cp0, &ce0, NULL, NULL, NULL, NULL, 0, 1);
            free(cp0.v); free(ce0.v);
        }
        free(xw0); free(xw1);
        int h;
        double E1 = INFINITY;
        for (h = 0; h <= 40; ++h) {
            for (int i = 0; i < n; ++i) yt[i] = y[i] + alpha * p[i];
            double *xw = world_alloc(s, yt);
            IVec tpt = {0}, tee = {0};
            active_pairs(s, xw, &cpt, &cee, &tpt, &tee);
            free(xw);
            E1 = eval_ip(s, yt, &tpt, &tee, NULL, NULL, NULL, NULL, 0, 1);
            free(tpt.v); free(tee.v);
            if (E1 <= E0) break;
            alpha *= 0.5;
        }
        free(cpt.v); free(cee.v);
        if (h > 40) { status = 4; break; }
        if (alpha < loc.alpha_min) loc.alpha_min = alpha;
        memcpy(y, yt, sizeof(double) * n);
        loc.energy = E1;
        if (s->kappa_frac > 0.0) {
            double d = min_active_distance(s, y);
            if (d < s->kappa_frac * s->dhat && d < s->dmin_prev) {
                double k2 = 2.0 * s->kappa, kmax = s->kappa_factor * s->kappa0;
                s->kappa = k2 < kmax ? k2 : kmax;
            }
            s->dmin_prev = d;
        }
    }
    }
    for (int i = 0; i < n; ++i) s->ydot[i] = (y[i] - s->y[i]) / s->h;
    memcpy(s->y, y, sizeof(double) * n);
    loc.status = status;
    if (st) *st = loc;
    free(y); free(g); free(p); free(b); free(yt);
    return status;
}

/* ------------------------------------------------------------------------ */
/* adjoint of one converged step (C15)                                      */
/* ------------------------------------------------------------------------ */
/* The step solves G(y^{n+1}; y^n, ydot^n, theta) = grad E_n = 0 with
 * theta = (E_e per tet, mu).  By the implicit function theorem, for an
 * upstream adjoint a = dL/dy^{n+1} the sensitivities are -(dG/dq)^T w with
 * H w = a, H the unprojected Hessian at y^{n+1} and the lagged friction data
 * held as functions of y^n. */
void or_set_params(OScene *s, const double *E, double mu)
{
    if (E)
        for (int e = 0; e < s->nt; ++e) {
            double nu = s->nu[e];
            s->E[e] = E[e];
            s->lmu[e] = E[e] / (2.0 * (1.0 + nu));
            s->llam[e] = E[e] * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
        }
    if (mu >= 0.0) s->mu = mu;
}

/* out = M v with M the mass matrix of the inertia term (lumped FEM masses,
 * per body the 4x4 generalised mass [m 0; 0 S] times I3) */
static void mass_apply(const OScene *s, const double *v, double *out)
{
    for (int i = 0; i < s->nv; ++i)
        for (int k = 0; k < 3; ++k) out[3 * i + k] = s->mass[i] * v[3 * i + k];
    for (int b = 0; b < s->nb; ++b) {
        int n0 = s->nv + 4 * b;
        double Mh[4][4] = {{0}};
        Mh[0][0] = s->bmass[b];
        for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) Mh[1 + i][1 + j] = s->bS[9 * b + 3 * i + j];
        for (int c = 0; c < 4; ++c)
            for (int k = 0; k < 3; ++k) {
                double acc = 0.0;
                for (int c2 = 0; c2 < 4; ++c2) acc += Mh[c][c2] * v[3 * (size_t)(n0 + c2) + k];
                out[3 * (size_t)(n0 + c) + k] = acc;
            }
    }
}

/* Friction part of (dG/dy^n)^T w, accumulated into out.  Each lagged pair
 * contributes phi = mu lam f1(|u|)/|u| (W . u), W = sum_a beta_a w_a, and
 * phi depends on the positions x^n of the pair's vertices through the
 * closest-point weights beta (the minimiser s* of |r(s)|^2 moves with x^n),
 * the offset r = sum beta x^n, the normal n = r/|r|, the normal force
 * lam = -kappa m(c) b'(|r|), and the -x^n inside u = P (sum beta (x - x^n)).
 * Returns sum_k lam_k f1_k/|u_k| (W_k . u_k) = w^T dG/dmu. */
static double friction_lag_vjp(const OScene *s, const double *xw, const double *xwn, const double *w, double *out)
{
    double ea = s->eps_v * s->h, dh = s->dhat, wgf = 0.0;
    for (int k = 0; k < s->nlag; ++k) {
        const OLag *L = s->lag + k;
        if (L->kind == 2) {
            /* the half-space: the normal is fixed, lam = -kappa b'(n . x^n - c)
             * and u = P (x - x^n), so d lam / d x^n = -kappa b'' n and
             * d u / d x^n = -P */
            const double *xv = P3(xw, L->cv[0]), *xnv = P3(xwn, L->cv[0]), *n = s->hs_n;
            OPt pt = cv_point(s, L->cv[0]);
            double W[3], D[3], u[3];
            for (int c = 0; c < 3; ++c) {
                double acc = 0.0;
                for (int q = 0; q < pt.n; ++q) acc += pt.w[q] * w[3 * (size_t)pt.node[q] + c];
                W[c] = acc;
                D[c] = xv[c] - xnv[c];
            }
            double d = hs_dist(s, xnv), b1 = barrier_d1(d, dh), b2 = barrier_d2(d, dh), lam = -s->kappa * b1;
            double nD = dot3(n, D);
            for (int c = 0; c < 3; ++c) u[c] = D[c] - n[c] * nD;
            double sg = sqrt(dot3(u, u));
            double f1s = sg < ea ? 2.0 / ea - sg / (ea * ea) : 1.0 / sg;
            double df1s = sg < ea ? -1.0 / (ea * ea) : -1.0 / (sg * sg);
            double Wu = dot3(W, u), psi = f1s * Wu, dpsi_du[3];
            for (int c = 0; c < 3; ++c) dpsi_du[c] = f1s * W[c] + (sg > 0.0 ? Wu * df1s * u[c] / sg : 0.0);
            wgf += lam * psi;
            for (int c = 0; c < 3; ++c) {
                double du[3];
                for (int i = 0; i < 3; ++i) du[i] = -((i == c ? 1.0 : 0.0) - n[i] * n[c]);
                double dlam = -s->kappa * b2 * n[c];
                double dphi = s->mu * (dlam * psi + lam * dot3(dpsi_du, du));
                for (int q = 0; q < pt.n; ++q) out[3 * (size_t)pt.node[q] + c] += pt.w[q] * dphi;
            }
            continue;
        }
        double x[12], xn[12], wv[12];
        OPt pts[4];
        for (int a = 0; a < 4; ++a) {
            memcpy(x + 3 * a, P3(xw, L->cv[a]), 3 * sizeof(double));
            memcpy(xn + 3 * a, P3(xwn, L->cv[a]), 3 * sizeof(double));
            pts[a] = cv_point(s, L->cv[a]);
            for (int c = 0; c < 3; ++c) {
                double acc = 0.0;
                for (int q = 0; q < pts[a].n; ++q) acc += pts[a].w[q] * w[3 * (size_t)pts[a].node[q] + c];
                wv[3 * a + c] = acc;
            }
        }
        Param P = type_param(L->kind, L->type);
        double beta[4], r[3], Dm[6];
        closest(&P, xn, beta, r, Dm);
        double d = sqrt(dot3(r, r)), n[3] = {r[0] / d, r[1] / d, r[2] / d};
        double m = 1.0, m1 = 0.0, gc[12] = {0}, Hc[144];
        if (L->kind == 1) {
            double c = cross2_derivs(xn, gc, Hc);
            if (c < L->ex) { m = (2.0 - c / L->ex) * (c / L->ex); m1 = 2.0 / L->ex - 2.0 * c / (L->ex * L->ex); }
        }
        double b1 = barrier_d1(d, dh), b2 = barrier_d2(d, dh);
        double lam = -s->kappa * m * b1;
        double D[3] = {0, 0, 0}, W[3] = {0, 0, 0};
        for (int a = 0; a < 4; ++a)
            for (int c = 0; c < 3; ++c) { D[c] += beta[a] * (x[3 * a + c] - xn[3 * a + c]); W[c] += beta[a] * wv[3 * a + c]; }
        double nD = dot3(n, D), u[3];
        for (int c = 0; c < 3; ++c) u[c] = D[c] - n[c] * nD;
        double sg = sqrt(dot3(u, u));
        double f1s = sg < ea ? 2.0 / ea - sg / (ea * ea) : 1.0 / sg;
        double df1s = sg < ea ? -1.0 / (ea * ea) : -1.0 / (sg * sg);   /* d(f1/s)/ds */
        double Wu = dot3(W, u), psi = f1s * Wu, dpsi_du[3];
        for (int c = 0; c < 3; ++c) dpsi_du[c] = f1s * W[c] + (sg > 0.0 ? Wu * df1s * u[c] / sg : 0.0);
        wgf += lam * psi;
        /* s* sensitivity: ds = -F_ss^{-1} F_sx, F = |r(s)|^2 */
        double Fi[2][2] = {{0, 0}, {0, 0}};
        if (P.npar == 1) Fi[0][0] = 1.0 / (2.0 * dot3(Dm, Dm));
        else if (P.npar == 2) {
            double a00 = 2.0 * dot3(Dm, Dm), a01 = 2.0 * dot3(Dm, Dm + 3), a11 = 2.0 * dot3(Dm + 3, Dm + 3);
            double det = a00 * a11 - a01 * a01;
            Fi[0][0] = a11 / det; Fi[1][1] = a00 / det; Fi[0][1] = Fi[1][0] = -a01 / det;
        }
        for (int j = 0; j < 4; ++j) {
            if (pts[j].n == 0) continue;
            for (int c = 0; c < 3; ++c) {
                double Fsx[2] = {0, 0}, ds[2] = {0, 0};
                for (int q = 0; q < P.npar; ++q) Fsx[q] = 2.0 * P.a[q][j] * r[c] + 2.0 * beta[j] * Dm[3 * q + c];
                for (int q = 0; q < P.npar; ++q)
                    for (int q2 = 0; q2 < P.npar; ++q2) ds[q] -= Fi[q][q2] * Fsx[q2];
                double db[4], dr[3], dn[3], dD[3], du[3];
                for (int a = 0; a < 4; ++a) {
                    db[a] = 0.0;
                    for (int q = 0; q < P.npar; ++q) db[a] += P.a[q][a] * ds[q];
                }
                for (int i = 0; i < 3; ++i) {
                    dr[i] = (i == c ? beta[j] : 0.0);
                    for (int q = 0; q < P.npar; ++q) dr[i] += Dm[3 * q + i] * ds[q];
                }
                double dd = dot3(n, dr);
                for (int i = 0; i < 3; ++i) dn[i] = (dr[i] - n[i] * dd) / d;
                for (int i = 0; i < 3; ++i) {
                    dD[i] = -(i == c ? beta[j] : 0.0);
                    for (int a = 0; a < 4; ++a) dD[i] += db[a] * (x[3 * a + i] - xn[3 * a + i]);
                }
                double dnD = dot3(dn, D) + dot3(n, dD);
                for (int i = 0; i < 3; ++i) du[i] = dD[i] - dn[i] * nD - n[i] * dnD;
                double dWu = 0.0;
                for (int a = 0; a < 4; ++a) dWu += db[a] * dot3(wv + 3 * a, u);
                double dlam = -s->kappa * (m1 * gc[3 * j + c] * b1 + m * b2 * dd);
                double dpsi = dot3(dpsi_du, du) + f1s * dWu;
                double dphi = s->mu * (dlam * psi + lam * dpsi);
                for (int q = 0; q < pts[j].n; ++q) out[3 * (size_t)pts[j].node[q] + c] += pts[j].w[q] * dphi;
            }
        }
    }
    return wgf;
}

/* Set up step n at (y_prev, yd_prev, targets): state, predictor, lag. */
static void adjoint_setup(OScene *s, const double *y_prev, const double *yd_prev, const double *targets)
{
    or_set_state(s, y_prev, yd_prev);
    or_begin_step(s, targets);
}

void or_dG_dyn_T(OScene *s, const double *y_prev, const double *yd_prev, const double *targets,
                 const double *y_next, const double *w, double *out)
{
    adjoint_setup(s, y_prev, yd_prev, targets);
    int n = s->ndof;
    mass_apply(s, w, out);
    for (int i = 0; i < n; ++i) out[i] = -out[i];
    double *xw = world_alloc(s, y_next), *xwn = world_alloc(s, y_prev);
    friction_lag_vjp(s, xw, xwn, w, out);
    free(xw); free(xwn);
}

/* Ebar[e] = w . dG/dE_e = (w_e . g_e)/E_e, g_e the tet's own gradient
 * contribution (Psi_e is linear in E_e at fixed nu); returns w . dG/dmu. */
double or_dG_dtheta_T(OScene *s, const double *y_prev, const double *yd_prev, const double *targets,
                      const double *y_next, const double *w, double *Ebar)
{
    adjoint_setup(s, y_prev, yd_prev, targets);
    double h2 = s->h * s->h;
    if (Ebar)
        for (int e = 0; e < s->nt; ++e) {
            double F[9], c[4][3], P[9];
            tet_F(s, y_next, e, F, c);
            or_snh(F, s->lmu[e], s->llam[e], P, NULL);
            double acc = 0.0;
            for (int a = 0; a < 4; ++a)
                for (int r = 0; r < 3; ++r) {
                    double ga = 0.0;
                    for (int j = 0; j < 3; ++j) ga += c[a][j] * P[3 * j + r];
                    acc += h2 * s->vol[e] * ga * w[3 * (size_t)s->tets[4 * e + a] + r];
                }
            Ebar[e] = acc / s->E[e];
        }
    double *xw = world_alloc(s, y_next), *xwn = world_alloc(s, y_prev);
    double *tmp = xcalloc((size_t)s->ndof, sizeof(double));
    double wgf = friction_lag_vjp(s, xw, xwn, w, tmp);
    free(tmp); free(xw); free(xwn);
    return wgf;
}

int or_step_vjp(OScene *s, const double *y_prev, const double *yd_prev, const double *targets,
                const double *y_next, const double *ybar_next, const double *vbar_next,
                double *ybar_prev, double *vbar_prev, double *Ebar, double *mubar, double eta, int *pcg_iters)
{
    int n = s->ndof;
    double h = s->h;
    adjoint_setup(s, y_prev, yd_prev, targets);
    IVec apt = {0}, aee = {0};
    pairs_at(s, y_next, &apt, &aee);
    Terms T = {0};
    double *g = xmalloc(sizeof(double) * n), *a = xmalloc(sizeof(double) * n), *w = xmalloc(sizeof(double) * n),
           *Mw = xmalloc(sizeof(double) * n), *lv = xcalloc((size_t)n, sizeof(double));
    eval_ip(s, y_next, &apt, &aee, NULL, g, NULL, &T, 0, 1);
    for (int i = 0; i < n; ++i) a[i] = ybar_next[i] + vbar_next[i] / h;
    int indef = 0;
    int it = pcg_terms(s, &T, a, w, eta, s->max_pcg, &indef);
    if (pcg_iters) *pcg_iters = it;
    free(T.t); free(apt.v); free(aee.v);
    int status = indef ? 6 : 0;
    if (!indef) {
        mass_apply(s, w, Mw);
        double *xw = world_alloc(s, y_next), *xwn = world_alloc(s, y_prev);
        double wgf = friction_lag_vjp(s, xw, xwn, w, lv);
        free(xw); free(xwn);
        for (int i = 0; i < n; ++i) {
            vbar_prev[i] = h * Mw[i];
            ybar_prev[i] = Mw[i] - lv[i] - vbar_next[i] / h;
        }
        if (mubar) *mubar -= wgf;
        if (Ebar) {
            double *eb = xmalloc(sizeof(double) * (size_t)(s->nt ? s->nt : 1));
            or_dG_dtheta_T(s, y_prev, yd_prev, targets, y_next, w, eb);
            for (int e = 0; e < s->nt; ++e) Ebar[e] -= eb[e];
            free(eb);
        }
    }
    free(g); free(a); free(w); free(Mw); free(lv);
    return status;
}
