// Adjoint of one converged step of the incremental potential (Eq. (3)).
//
// The step ends at G(y^{n+1}; y^n, ydot^n, theta) = grad E = 0 with
// theta = (Young's modulus per tet, friction coefficient).  For upstream
// adjoints (ybar^{n+1}, vbar^{n+1}) of the step's outputs y^{n+1} and
// ydot^{n+1} = (y^{n+1} - y^n)/h, the implicit function theorem gives
//   H w = ybar^{n+1} + vbar^{n+1}/h          (H: unprojected Hessian at y^{n+1})
//   vbar^n = h M w                           (dG/dydot^n = -h M)
//   ybar^n = M w - (dG_F/dy^n)^T w - vbar^{n+1}/h
//   Ebar_e -= w . dG/dE_e = (w_e . g_e)/E_e (the tet's energy is linear in E_e)
//   mubar  -= w . dG/dmu  = w . grad E_F / mu
// The kernels below cover the node-wise terms and the per-tet parameter term;
// the friction-lag term runs with the other contact kernels.
#include "ipc_device.h"
#include "ipc_internal.h"
#include "ipc_kernels.h"

namespace ipc {

// new Young's moduli (external tet order) and the Lame parameters from them
__global__ void k_set_E(int64_t n, const int *__restrict__ ext2tet, const double *__restrict__ E, const double *__restrict__ nu,
                        double *__restrict__ tE, double *__restrict__ tmu, double *__restrict__ tlam)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    int e = ext2tet[i];
    double Ee = E[i], v = nu[e];
    tE[e] = Ee;
    tmu[e] = Ee / (2.0 * (1.0 + v));
    tlam[e] = Ee * v / ((1.0 + v) * (1.0 - 2.0 * v));
}

// rhs = ybar^{n+1} + vbar^{n+1} / h (internal layout; zero on padding nodes)
__global__ void k_adj_rhs(int N, const int *__restrict__ kind, const int *__restrict__ node_scene, const double *__restrict__ sparam,
                          const double *__restrict__ yb, const double *__restrict__ vb, double *__restrict__ rhs)
{
    int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    d3 o = {0.0, 0.0, 0.0};
    if (kind[n] != 2) {
        double ih = 1.0 / sparam[8 * (size_t)node_scene[n] + P_H];
        d3 a = ld3(yb, n), b = ld3(vb, n);
        o = {a.x + b.x * ih, a.y + b.y * ih, a.z + b.z * ih};
    }
    st3(rhs, n, o);
}

// FEM and padding nodes: vbar^n = h m w, ybar^n = m w - vbar^{n+1}/h
__global__ void k_adj_nodes(int N, const int *__restrict__ kind, const int *__restrict__ node_scene, const double *__restrict__ sparam,
                            const double *__restrict__ mass, const double *__restrict__ w, const double *__restrict__ vbn,
                            double *__restrict__ ybp, double *__restrict__ vbp)
{
    int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N || kind[n] == 1) return;
    if (kind[n] == 2) { st3(ybp, n, {0.0, 0.0, 0.0}); st3(vbp, n, {0.0, 0.0, 0.0}); return; }
    double h = sparam[8 * (size_t)node_scene[n] + P_H], m = mass[n], ih = 1.0 / h;
    d3 wv = ld3(w, n), b = ld3(vbn, n);
    st3(vbp, n, {h * m * wv.x, h * m * wv.y, h * m * wv.z});
    st3(ybp, n, {m * wv.x - b.x * ih, m * wv.y - b.y * ih, m * wv.z - b.z * ih});
}

// affine bodies: the same with the 4x4 generalised mass [m 0; 0 S] (x) I3
__global__ void k_adj_bodies(int NB, const int *__restrict__ node0, const int *__restrict__ bscene, const double *__restrict__ sparam,
                             const double *__restrict__ bM, const double *__restrict__ w, const double *__restrict__ vbn,
                             double *__restrict__ ybp, double *__restrict__ vbp)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= NB) return;
    int n0 = node0[b];
    double h = sparam[8 * (size_t)bscene[b] + P_H], ih = 1.0 / h;
    const double *M = bM + 16 * (size_t)b;
    d3 wv[4] = {ld3(w, n0), ld3(w, n0 + 1), ld3(w, n0 + 2), ld3(w, n0 + 3)};
    for (int c = 0; c < 4; ++c) {
        d3 mw = {0.0, 0.0, 0.0};
        for (int c2 = 0; c2 < 4; ++c2) {
            double mm = M[4 * c + c2];
            mw.x += mm * wv[c2].x; mw.y += mm * wv[c2].y; mw.z += mm * wv[c2].z;
        }
        d3 vb = ld3(vbn, n0 + c);
        st3(vbp, n0 + c, {h * mw.x, h * mw.y, h * mw.z});
        st3(ybp, n0 + c, {mw.x - vb.x * ih, mw.y - vb.y * ih, mw.z - vb.z * ih});
    }
}

// Ebar[i] -= (w_e . g_e) / E_e for external tet i, g_e the tet's gradient at y
__global__ void k_adj_E(int64_t n, const int *__restrict__ ext2tet, int T, const int4 *__restrict__ tv, const double *__restrict__ Bm,
                        const double *__restrict__ vol, const double *__restrict__ tmu, const double *__restrict__ tlam,
                        const double *__restrict__ tE, const double *__restrict__ y, const double *__restrict__ w,
                        const int *__restrict__ tile_scene, const double *__restrict__ h2s, double *__restrict__ Ebar)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    int e = ext2tet[i];
    int4 t = tv[e];
    int vi[4] = {t.x, t.y, t.z, t.w};
    d3 x[4];
    for (int a = 0; a < 4; ++a) x[a] = ld3(y, vi[a]);
    double c[4][3];
    for (int j = 0; j < 3; ++j) {
        c[1][j] = Bm[(size_t)j * T + e];
        c[2][j] = Bm[(size_t)(3 + j) * T + e];
        c[3][j] = Bm[(size_t)(6 + j) * T + e];
        c[0][j] = -(c[1][j] + c[2][j] + c[3][j]);
    }
    d3 f[3];
    for (int j = 0; j < 3; ++j)
        f[j] = {c[0][j] * x[0].x + c[1][j] * x[1].x + c[2][j] * x[2].x + c[3][j] * x[3].x,
                c[0][j] * x[0].y + c[1][j] * x[1].y + c[2][j] * x[2].y + c[3][j] * x[3].y,
                c[0][j] * x[0].z + c[1][j] * x[1].z + c[2][j] * x[2].z + c[3][j] * x[3].z};
    double mu = tmu[e], lh = tlam[e] + mu;
    d3 cof[3] = {cr(f[1], f[2]), cr(f[2], f[0]), cr(f[0], f[1])};
    double J = dt(f[0], cof[0]);
    double sc = lh * (J - 1.0) - mu;
    d3 P[3];
    for (int j = 0; j < 3; ++j) P[j] = {mu * f[j].x + sc * cof[j].x, mu * f[j].y + sc * cof[j].y, mu * f[j].z + sc * cof[j].z};
    // w_e . g_e = wt sum_a w_a . (sum_j c[a][j] P_j) = wt sum_j P_j . (sum_a c[a][j] w_a)
    d3 wv[4];
    for (int a = 0; a < 4; ++a) wv[a] = ld3(w, vi[a]);
    double acc = 0.0;
    for (int j = 0; j < 3; ++j) {
        d3 q = {c[0][j] * wv[0].x + c[1][j] * wv[1].x + c[2][j] * wv[2].x + c[3][j] * wv[3].x,
                c[0][j] * wv[0].y + c[1][j] * wv[1].y + c[2][j] * wv[2].y + c[3][j] * wv[3].y,
                c[0][j] * wv[0].z + c[1][j] * wv[1].z + c[2][j] * wv[2].z + c[3][j] * wv[3].z};
        acc += dt(P[j], q);
    }
    double wt = h2s[tile_scene[e / TILE]] * vol[e];
    Ebar[i] -= wt * acc / tE[e];
}

void launch_set_E(ipc_ctx *c, const double *E_ext)
{
    Dev &D = c->d;
    if (c->ext_tets == 0) return;
    hipLaunchKernelGGL(k_set_E, dim3(blocks_for(c->ext_tets)), dim3(BLOCK), 0, c->stream, c->ext_tets, D.ext2tet.p, E_ext, D.tnu.p,
                       D.tE.p, D.tmu.p, D.tlam.p);
}

void launch_adj_rhs(ipc_ctx *c, const double *ybar_next, const double *vbar_next, double *rhs)
{
    Dev &D = c->d;
    hipLaunchKernelGGL(k_adj_rhs, dim3(blocks_for(c->N)), dim3(BLOCK), 0, c->stream, c->N, D.node_kind.p, D.node_scene.p, D.sparam.p,
                       ybar_next, vbar_next, rhs);
}

void launch_adj_mass(ipc_ctx *c, const double *w, const double *vbar_next, double *ybar_prev, double *vbar_prev)
{
    Dev &D = c->d;
    hipLaunchKernelGGL(k_adj_nodes, dim3(blocks_for(c->N)), dim3(BLOCK), 0, c->stream, c->N, D.node_kind.p, D.node_scene.p, D.sparam.p,
                       D.mass.p, w, vbar_next, ybar_prev, vbar_prev);
    if (c->NB)
        hipLaunchKernelGGL(k_adj_bodies, dim3(blocks_for(c->NB, 64)), dim3(64), 0, c->stream, c->NB, D.body_node0.p, D.body_scene.p,
                           D.sparam.p, D.bM.p, w, vbar_next, ybar_prev, vbar_prev);
}

void launch_adj_E(ipc_ctx *c, const double *y, const double *w, double *Ebar_ext)
{
    Dev &D = c->d;
    if (c->ext_tets == 0) return;
    hipLaunchKernelGGL(k_adj_E, dim3(blocks_for(c->ext_tets)), dim3(BLOCK), 0, c->stream, c->ext_tets, D.ext2tet.p, c->T, D.tv.p,
                       D.Bm.p, D.vol.p, D.tmu.p, D.tlam.p, D.tE.p, y, w, D.tile_scene_tet.p, D.h2s.p, Ebar_ext);
}

} // namespace ipc
