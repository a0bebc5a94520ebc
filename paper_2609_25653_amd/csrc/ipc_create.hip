// Context creation: host validation and topology, device precompute.
//
// Host side (once per scene): surface extraction (faces owned by exactly one
// tetrahedron, outward, canonical rotation, sorted), unique surface edges,
// contact-vertex numbering, block-CSR pattern of the FEM matrix and the
// per-tetrahedron scatter slots.  Device side: inverse rest shape matrices,
// volumes, Lame parameters, lumped masses and the constant spring diagonals.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <numeric>

#include "ipc_device.h"
#include "ipc_internal.h"
#include "ipc_kernels.h"
#include "ipc_runsum.h"

namespace ipc {

namespace {

// ---- device precompute kernels ---------------------------------------------
__global__ void k_tet_precompute(int T, const int4 *__restrict__ tv, const double *__restrict__ X, const double *__restrict__ E,
                                 const double *__restrict__ nu, double *__restrict__ Bm, double *__restrict__ vol,
                                 double *__restrict__ tmu, double *__restrict__ tlam, const int *__restrict__ valid)
{
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= T) return;
    if (!valid[e]) {
#pragma unroll
        for (int k = 0; k < 9; ++k) Bm[(size_t)k * T + e] = 0.0;
        vol[e] = 0.0; tmu[e] = 0.0; tlam[e] = 0.0;
        return;
    }
    int4 t = tv[e];
    d3 x0 = ld3(X, t.x), x1 = ld3(X, t.y), x2 = ld3(X, t.z), x3 = ld3(X, t.w);
    // Dm columns: x1-x0, x2-x0, x3-x0
    double m[3][3] = {{x1.x - x0.x, x2.x - x0.x, x3.x - x0.x},
                      {x1.y - x0.y, x2.y - x0.y, x3.y - x0.y},
                      {x1.z - x0.z, x2.z - x0.z, x3.z - x0.z}};
    double c00 = m[1][1] * m[2][2] - m[1][2] * m[2][1];
    double c01 = m[1][2] * m[2][0] - m[1][0] * m[2][2];
    double c02 = m[1][0] * m[2][1] - m[1][1] * m[2][0];
    double det = m[0][0] * c00 + m[0][1] * c01 + m[0][2] * c02;
    double id = 1.0 / det;
    // inverse = adj^T / det, row-major B[r][c]
    double B[9];
    B[0] = c00 * id;
    B[1] = (m[0][2] * m[2][1] - m[0][1] * m[2][2]) * id;
    B[2] = (m[0][1] * m[1][2] - m[0][2] * m[1][1]) * id;
    B[3] = c01 * id;
    B[4] = (m[0][0] * m[2][2] - m[0][2] * m[2][0]) * id;
    B[5] = (m[0][2] * m[1][0] - m[0][0] * m[1][2]) * id;
    B[6] = c02 * id;
    B[7] = (m[0][1] * m[2][0] - m[0][0] * m[2][1]) * id;
    B[8] = (m[0][0] * m[1][1] - m[0][1] * m[1][0]) * id;
#pragma unroll
    for (int k = 0; k < 9; ++k) Bm[(size_t)k * T + e] = B[k];
    vol[e] = det / 6.0;
    double Ee = E[e], n = nu[e];
    tmu[e] = Ee / (2.0 * (1.0 + n));
    tlam[e] = Ee * n / ((1.0 + n) * (1.0 - 2.0 * n));
}

// lumped mass by gathering incident tetrahedra in a fixed order
__global__ void k_node_mass(int N, const int *__restrict__ adj_ptr, const int *__restrict__ adj, const double *__restrict__ vol,
                            const double *__restrict__ rho, double *__restrict__ mass)
{
    int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    double m = 0.0;
    for (int k = adj_ptr[n]; k < adj_ptr[n + 1]; ++k) {
        int e = adj[k] >> 2;
        m += rho[e] * vol[e] / 4.0;
    }
    mass[n] = m;
}

// constant part of the matrix: lumped FEM mass on the diagonal blocks
__global__ void k_const_mass(int N, const int *__restrict__ kind, const int *__restrict__ diag_slot, const double *__restrict__ mass,
                             double *__restrict__ vc)
{
    int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N || kind[n] != 0) return;
    double *b = vc + 9 * (size_t)diag_slot[n];
    b[0] += mass[n]; b[4] += mass[n]; b[8] += mass[n];
}

// constant part of the matrix: spring Hessians h^2 k (u u^T) (x) I3 where u
// lists the side nodes with weights +w (side a) and -w (side b).  Entry code
// 64 s + 8 i + j of the slot-sorted list is h^2 k u_i u_j; the run sums add
// it to the three diagonal entries of the slot's block.
__device__ __forceinline__ double spring_u(int s, int i, const int *ka, const double *xa, const int *kb, const double *xb)
{
    for (int side = 0; side < 2; ++side) {
        int kind = side ? kb[s] : ka[s];
        int n = kind == 0 ? 1 : (kind == 1 ? 4 : 0);
        if (i < n) {
            double sg = side ? -1.0 : 1.0;
            return (kind == 0 || i == 0) ? sg : sg * (side ? xb : xa)[3 * (size_t)s + i - 1];
        }
        i -= n;
    }
    return 0.0;
}
struct ValConstSpring {
    const int *ka, *kb, *sscene;
    const double *xa, *xb, *k, *h2s;
    __device__ void operator()(int code, double *a) const
    {
        const int s = code >> 6, i = (code >> 3) & 7, j = code & 7;
        a[0] = h2s[sscene[s]] * k[s] * spring_u(s, i, ka, xa, kb, xb) * spring_u(s, j, ka, xa, kb, xb);
    }
};
struct EmitDiag {   // the scalar onto the diagonal of a 3x3 block
    double *out;
    __device__ void operator()(int key, const double *a) const
    {
        double *b = out + 9 * (size_t)key;
        b[0] += a[0]; b[4] += a[0]; b[8] += a[0];
    }
};

__global__ void k_zero_vals(int64_t n, double *__restrict__ v)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) v[i] = 0.0;
}

__global__ void k_sum_mass(int nv, const double *__restrict__ mass, int node0, double *out)
{
    // one block; fixed-order strided sums then a tree
    __shared__ double sh[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nv; i += 256) acc += mass[node0 + i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

// ---- host helpers -----------------------------------------------------------
void fail(const std::string &m) { throw Error(IPC_E_INVALID, m); }

bool finite_all(const double *p, size_t n)
{
    for (size_t i = 0; i < n; ++i) if (!std::isfinite(p[i])) return false;
    return true;
}

void validate(const ipc_scene_desc &s, int si)
{
    auto pre = "scene " + std::to_string(si) + ": ";
    if (s.nv < 0 || s.nt < 0 || s.nb < 0 || s.nbv < 0 || s.nbt < 0 || s.nsv < 0 || s.nst < 0 || s.nobj < 0 || s.nex < 0 ||
        s.ns < 0 || s.nd < 0)
        fail(pre + "negative size");
    // every array that a nonzero count asks for must be there
    auto need = [&](bool cond, const void *p, const char *what) { if (cond && !p) fail(pre + "missing array " + what); };
    need(s.nv > 0, s.X, "X"); need(s.nv > 0, s.V, "V"); need(s.nv > 0, s.vobj, "vobj");
    need(s.nt > 0, s.tets, "tets"); need(s.nt > 0, s.tet_E, "tet_E"); need(s.nt > 0, s.tet_nu, "tet_nu");
    need(s.nt > 0, s.tet_rho, "tet_rho");
    for (const void *p : {(const void *)s.body_q, (const void *)s.body_qdot, (const void *)s.body_mass, (const void *)s.body_S,
                          (const void *)s.body_vol, (const void *)s.body_kappa, (const void *)s.body_ext, (const void *)s.body_obj})
        need(s.nb > 0, p, "body arrays");
    need(s.nbv > 0, s.bv_xbar, "bv_xbar"); need(s.nbv > 0, s.bv_body, "bv_body"); need(s.nbt > 0, s.btri, "btri");
    need(s.nsv > 0, s.sv_x, "sv_x"); need(s.nst > 0, s.stri, "stri"); need(s.nobj > 0, s.obj_kind, "obj_kind");
    need(s.nex > 0, s.excl, "excl");
    for (const void *p : {(const void *)s.sp_ka, (const void *)s.sp_ia, (const void *)s.sp_xa, (const void *)s.sp_kb,
                          (const void *)s.sp_ib, (const void *)s.sp_xb, (const void *)s.sp_k})
        need(s.ns > 0, p, "spring arrays");
    need(s.nd > 0, s.driven_body, "driven_body");
    if (s.nv + s.nb == 0) fail(pre + "no degrees of freedom");
    if (!(s.h > 0) || !(s.dhat > 0) || !(s.mu >= 0) || !(s.eps_v > 0) || !(s.newton_tol > 0) || !(s.pcg_tol > 0) ||
        !(s.ccd_s > 0 && s.ccd_s < 1) || s.max_newton < 1 || s.max_pcg < 1)
        fail(pre + "invalid parameters");
    {
        const double *q = s.half_space, n2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2];
        for (int k = 0; k < 4; ++k)
            if (!std::isfinite(q[k])) fail(pre + "invalid half-space");
        if (n2 != 0.0 && !(std::fabs(n2 - 1.0) <= 1e-12)) fail(pre + "half-space normal is not a unit vector");
    }
    if (!finite_all(s.X, 3 * (size_t)s.nv) || !finite_all(s.V, 3 * (size_t)s.nv)) fail(pre + "non-finite FEM state");
    for (int e = 0; e < s.nt; ++e) {
        for (int k = 0; k < 4; ++k)
            if (s.tets[4 * e + k] < 0 || s.tets[4 * e + k] >= s.nv) fail(pre + "tet index out of range");
        if (!(s.tet_E[e] > 0) || !(s.tet_nu[e] > 0 && s.tet_nu[e] < 0.5) || !(s.tet_rho[e] > 0))
            fail(pre + "invalid material at tet " + std::to_string(e));
        const double *x0 = s.X + 3 * s.tets[4 * e], *x1 = s.X + 3 * s.tets[4 * e + 1], *x2 = s.X + 3 * s.tets[4 * e + 2],
                     *x3 = s.X + 3 * s.tets[4 * e + 3];
        double a[3], b[3], c[3];
        for (int k = 0; k < 3; ++k) { a[k] = x1[k] - x0[k]; b[k] = x2[k] - x0[k]; c[k] = x3[k] - x0[k]; }
        double det = a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0]) + a[2] * (b[0] * c[1] - b[1] * c[0]);
        if (!(det > 0)) fail(pre + "tet " + std::to_string(e) + " is inverted or degenerate");
    }
    for (int i = 0; i < s.nv; ++i)
        if (s.vobj[i] < 0 || s.vobj[i] >= s.nobj || s.obj_kind[s.vobj[i]] != 0) fail(pre + "bad FEM vertex object");
    for (int b = 0; b < s.nb; ++b) {
        if (!(s.body_mass[b] > 0) || !(s.body_vol[b] > 0) || !(s.body_kappa[b] >= 0)) fail(pre + "invalid body");
        if (s.body_obj[b] < 0 || s.body_obj[b] >= s.nobj || s.obj_kind[s.body_obj[b]] != 1) fail(pre + "bad body object");
        if (!finite_all(s.body_q + 12 * b, 12) || !finite_all(s.body_qdot + 12 * b, 12)) fail(pre + "non-finite body state");
    }
    for (int i = 0; i < s.nbv; ++i) if (s.bv_body[i] < 0 || s.bv_body[i] >= s.nb) fail(pre + "bad body vertex");
    for (int i = 0; i < 3 * s.nbt; ++i) if (s.btri[i] < 0 || s.btri[i] >= s.nbv) fail(pre + "bad body triangle");
    for (int i = 0; i < 3 * s.nst; ++i) if (s.stri[i] < 0 || s.stri[i] >= s.nsv) fail(pre + "bad static triangle");
    for (int i = 0; i < 2 * s.nex; ++i) if (s.excl[i] < 0 || s.excl[i] >= s.nobj) fail(pre + "bad exclusion");
    for (int k = 0; k < s.ns; ++k) {
        for (int side = 0; side < 2; ++side) {
            int kind = side ? s.sp_kb[k] : s.sp_ka[k], idx = side ? s.sp_ib[k] : s.sp_ia[k];
            int lim = kind == 0 ? s.nv : (kind == 1 ? s.nb : (kind == 2 ? s.nd : -1));
            if (lim < 0 || idx < 0 || idx >= lim) fail(pre + "bad spring " + std::to_string(k));
        }
        if (!(s.sp_k[k] >= 0)) fail(pre + "negative spring stiffness");
    }
    for (int d = 0; d < s.nd; ++d) if (s.driven_body[d] < 0 || s.driven_body[d] >= s.nb) fail(pre + "bad driven body");
    if (s.nj < 0 || (s.nj > 0 && !s.joint_spring)) fail(pre + "bad joint-spring count");
    for (int j = 0; j < s.nj; ++j)
        if (s.joint_spring[j] < 0 || s.joint_spring[j] >= s.ns || s.sp_kb[s.joint_spring[j]] != 1)
            fail(pre + "joint spring " + std::to_string(j) + " is not a spring with a body point on its b side");
}

int pad64(int n) { return (n + TILE - 1) / TILE * TILE; }

struct HostTopo {
    std::vector<std::array<int, 3>> tri;   // scene-local external vertex ids, canonical
    std::vector<std::array<int, 2>> edge;
    std::vector<int> surf;                 // sorted external ids referenced by triangles
};

HostTopo topology(const ipc_scene_desc &s)
{
    HostTopo t;
    static const int fl[4][3] = {{0, 2, 1}, {0, 1, 3}, {0, 3, 2}, {1, 2, 3}};
    std::vector<std::pair<std::array<int, 3>, int>> faces;
    faces.reserve(4 * (size_t)s.nt);
    for (int e = 0; e < s.nt; ++e)
        for (int f = 0; f < 4; ++f) {
            std::array<int, 3> k = {s.tets[4 * e + fl[f][0]], s.tets[4 * e + fl[f][1]], s.tets[4 * e + fl[f][2]]};
            std::sort(k.begin(), k.end());
            faces.push_back({k, 4 * e + f});
        }
    std::sort(faces.begin(), faces.end());
    for (size_t i = 0; i < faces.size();) {
        size_t j = i + 1;
        while (j < faces.size() && faces[j].first == faces[i].first) ++j;
        if (j - i == 1) {
            int e = faces[i].second / 4, f = faces[i].second % 4;
            t.tri.push_back({s.tets[4 * e + fl[f][0]], s.tets[4 * e + fl[f][1]], s.tets[4 * e + fl[f][2]]});
        }
        i = j;
    }
    for (int k = 0; k < s.nbt; ++k)
        t.tri.push_back({s.nv + s.btri[3 * k], s.nv + s.btri[3 * k + 1], s.nv + s.btri[3 * k + 2]});
    for (int k = 0; k < s.nst; ++k)
        t.tri.push_back({s.nv + s.nbv + s.stri[3 * k], s.nv + s.nbv + s.stri[3 * k + 1], s.nv + s.nbv + s.stri[3 * k + 2]});
    for (auto &v : t.tri)
        while (v[0] > v[1] || v[0] > v[2]) std::rotate(v.begin(), v.begin() + 1, v.end());
    std::sort(t.tri.begin(), t.tri.end());
    for (auto &v : t.tri)
        for (int k = 0; k < 3; ++k) {
            int a = v[k], b = v[(k + 1) % 3];
            t.edge.push_back({std::min(a, b), std::max(a, b)});
        }
    std::sort(t.edge.begin(), t.edge.end());
    t.edge.erase(std::unique(t.edge.begin(), t.edge.end()), t.edge.end());
    for (auto &v : t.tri) for (int k = 0; k < 3; ++k) t.surf.push_back(v[k]);
    std::sort(t.surf.begin(), t.surf.end());
    t.surf.erase(std::unique(t.surf.begin(), t.surf.end()), t.surf.end());
    return t;
}

unsigned int spread10(unsigned int v)
{
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

// The order of a scene's first nv + nb nodes: its FEM vertices and its
// bodies' translation nodes together, by the Morton code of their positions
// at creation (10 bits per axis over their bounding box; equal codes keep
// FEM vertices before bodies, each in input order).  Entry m >= 0 is FEM
// vertex m's slot; -1 - b marks body b, whose slot is left as padding (the
// body's 4 nodes follow the region).  The coarse preconditioner's groups are
// runs of this order, so each of its domains is one contiguous node range.
std::vector<int> morton_entries(const ipc_scene_desc &d)
{
    std::vector<int> part(d.nv + d.nb);
    std::iota(part.begin(), part.end(), 0);
    auto pos = [&](int m, int k) { return m < d.nv ? d.X[3 * (size_t)m + k] : d.body_q[12 * (size_t)(m - d.nv) + k]; };
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int m : part)
        for (int k = 0; k < 3; ++k) { lo[k] = std::min(lo[k], pos(m, k)); hi[k] = std::max(hi[k], pos(m, k)); }
    const double ext = std::max(hi[0] - lo[0], std::max(hi[1] - lo[1], hi[2] - lo[2]));
    const double sc = ext > 0.0 ? 1023.0 / ext : 0.0;
    std::vector<unsigned int> key(part.size());
    for (int m : part) {
        unsigned int q[3];
        for (int k = 0; k < 3; ++k) q[k] = (unsigned int)std::min(1023.0, std::max(0.0, (pos(m, k) - lo[k]) * sc));
        key[m] = (spread10(q[0]) << 2) | (spread10(q[1]) << 1) | spread10(q[2]);
    }
    std::stable_sort(part.begin(), part.end(), [&](int a, int b) { return key[a] < key[b]; });
    for (int &m : part) m = m < d.nv ? m : -1 - (m - d.nv);
    return part;
}

} // namespace

void validate_scenes(const ipc_scene_desc *scenes, int n)
{
    if (!scenes || n < 1) fail("need at least one scene");
    for (int s = 0; s < n; ++s) validate(scenes[s], s);
}

void build_const_part(ipc_ctx *c, const double *h2s)
{
    Dev &D = c->d;
    hipStream_t st = c->stream;
    int64_t nv = 9 * (int64_t)std::max(c->nnzb, 1);
    hipLaunchKernelGGL(k_zero_vals, dim3(blocks_for(nv)), dim3(BLOCK), 0, st, nv, D.val_const.p);
    hipLaunchKernelGGL(k_const_mass, dim3(blocks_for(c->N)), dim3(BLOCK), 0, st, c->N, D.node_kind.p, D.diag_slot.p, D.mass.p,
                       D.val_const.p);
    runsum<1>(c, D.n_spc, c->nnzb, D.spc_key.p, D.spc_code.p,
              ValConstSpring{D.sp_ka.p, D.sp_kb.p, D.sp_scene.p, D.sp_xa.p, D.sp_xb.p, D.sp_k.p, h2s}, EmitDiag{D.val_const.p});
}


void create_context(ipc_ctx *c, const ipc_scene_desc *scenes, int n, const int64_t *caps, size_t *plan)
{
    hipStream_t st = c->stream;
    c->n_scenes = n;
    c->sc.resize(n);
    for (int s = 0; s < n; ++s) validate(scenes[s], s);

    // ---- offsets
    int node = 0, tet = 0, body = 0, drv = 0, sp = 0, jt = 0, cv = 0, tri = 0, edge = 0, obj = 0, ex = 0;
    int64_t dof = 0;
    std::vector<HostTopo> topo(n);
    for (int s = 0; s < n; ++s) {
        const ipc_scene_desc &d = scenes[s];
        SceneInfo &S = c->sc[s];
        S.nv = d.nv; S.nt = d.nt; S.nb = d.nb; S.nbv = d.nbv; S.nbt = d.nbt; S.nsv = d.nsv; S.nst = d.nst;
        S.nobj = d.nobj; S.nex = d.nex; S.ns = d.ns; S.nd = d.nd; S.nj = d.nj;
        S.h = d.h; S.g[0] = d.g[0]; S.g[1] = d.g[1]; S.g[2] = d.g[2]; S.dhat = d.dhat; S.kappa = d.kappa; S.mu = d.mu;
        S.eps_v = d.eps_v; S.newton_tol = d.newton_tol; S.pcg_tol = d.pcg_tol; S.ccd_s = d.ccd_s;
        S.max_newton = d.max_newton; S.max_pcg = d.max_pcg;
        for (int k = 0; k < 4; ++k) S.hs[k] = d.half_space[k];
        S.hs_on = d.half_space[0] != 0.0 || d.half_space[1] != 0.0 || d.half_space[2] != 0.0;
        topo[s] = topology(d);
        S.node0 = node; S.nnode = d.nv + 4 * d.nb;
        S.entry = morton_entries(d);
        S.bnode0 = node + (d.nv + d.nb + 3) / 4 * 4;
        S.nnode_pad = pad64(S.bnode0 - node + 4 * d.nb);
        S.tet0 = tet; S.nt_pad = pad64(d.nt);
        S.body0 = body; S.drv0 = drv; S.sp0 = sp; S.jt0 = jt;
        S.cv0 = cv; S.ncv = (int)topo[s].surf.size(); S.nsurf = S.ncv;
        S.tri0 = tri; S.ntri = (int)topo[s].tri.size();
        S.edge0 = edge; S.nedge = (int)topo[s].edge.size();
        S.obj0 = obj;
        S.dof0 = dof;
        node += S.nnode_pad; tet += S.nt_pad; body += d.nb; drv += d.nd; sp += d.ns; jt += d.nj; cv += S.ncv;
        tri += S.ntri; edge += S.nedge; obj += d.nobj; ex += d.nex;
        dof += 3 * (int64_t)S.nnode;
        S.surf_ext = topo[s].surf;
        S.tri_ext.resize(3 * (size_t)S.ntri);
        for (int k = 0; k < S.ntri; ++k) for (int m = 0; m < 3; ++m) S.tri_ext[3 * k + m] = topo[s].tri[k][m];
        S.edge_ext.resize(2 * (size_t)S.nedge);
        for (int k = 0; k < S.nedge; ++k) for (int m = 0; m < 2; ++m) S.edge_ext[2 * k + m] = topo[s].edge[k][m];
    }
    for (int s = 0; s < n; ++s) { c->NFEM += scenes[s].nv; c->TREAL += scenes[s].nt; }
    c->N = node; c->T = tet; c->NB = body; c->ND = drv; c->NJ = jt; c->NS = sp; c->CV = cv; c->NSURF = cv; c->TRI = tri;
    c->EDGE = edge; c->NOBJ = obj; c->NEX = ex; c->ndof = dof; c->ext_nodes = dof / 3;

    // ---- host arrays
    std::vector<double> X(3 * (size_t)node, 0.0), V(3 * (size_t)node, 0.0), mass_dummy;
    std::vector<int> node_scene(node), node_kind(node, 2), ext2node((size_t)c->ext_nodes);
    std::vector<int4> tv(tet);
    std::vector<int> tvalid(tet, 0);
    std::vector<double> tE(tet, 1.0), tnu(tet, 0.25), trho(tet, 0.0);
    std::vector<int> ext2tet;
    std::vector<double> bM(16 * (size_t)std::max(body, 1), 0.0), bvol(body), bkappa(body), bext(3 * (size_t)body);
    std::vector<int> body_node0(body), body_scene(body);
    std::vector<int> ska(sp), sia(sp), skb(sp), sib(sp), sscene(sp);
    std::vector<double> sxa(3 * (size_t)sp), sxb(3 * (size_t)sp), sk(sp);
    std::vector<double> targets(12 * (size_t)std::max(drv, 1), 0.0);
    std::vector<int> driven(drv), joint_sp(jt);
    std::vector<int> cv_node(cv, -1), cv_body(cv, -1), cv_obj(cv), cv_scene(cv);
    std::vector<double> cv_x(3 * (size_t)cv, 0.0);
    std::vector<int4> tri4(tri);
    std::vector<int2> edge2(edge);
    std::vector<double> rest2(edge);
    std::vector<int> okind(obj), excl(2 * (size_t)std::max(ex, 1));
    std::vector<int> tile_node(node / TILE), tile_tet(tet / TILE);
    std::vector<int> adj_ptr(node + 1, 0), adj;
    int exo = 0;
    for (int s = 0; s < n; ++s) {
        const ipc_scene_desc &d = scenes[s];
        SceneInfo &S = c->sc[s];
        for (int i = 0; i < S.nnode_pad; ++i) node_scene[S.node0 + i] = s;
        for (int i = 0; i < S.nnode_pad / TILE; ++i) tile_node[S.node0 / TILE + i] = s;
        for (int i = 0; i < S.nt_pad / TILE; ++i) tile_tet[S.tet0 / TILE + i] = s;
        // FEM vertex i sits at node fem[i] (its slot in the scene's Morton order)
        std::vector<int> fem(d.nv);
        for (int m = 0; m < (int)S.entry.size(); ++m)
            if (S.entry[m] >= 0) fem[S.entry[m]] = S.node0 + m;
        for (int i = 0; i < d.nv; ++i) {
            node_kind[fem[i]] = 0;
            for (int k = 0; k < 3; ++k) { X[3 * (size_t)fem[i] + k] = d.X[3 * i + k]; V[3 * (size_t)fem[i] + k] = d.V[3 * i + k]; }
        }
        for (int b = 0; b < d.nb; ++b)
            for (int cc = 0; cc < 4; ++cc) {
                int nd = S.bnode0 + 4 * b + cc;
                node_kind[nd] = 1;
                for (int k = 0; k < 3; ++k) { X[3 * (size_t)nd + k] = d.body_q[12 * b + 3 * cc + k]; V[3 * (size_t)nd + k] = d.body_qdot[12 * b + 3 * cc + k]; }
            }
        for (int i = 0; i < S.nnode; ++i) ext2node[S.dof0 / 3 + i] = i < d.nv ? fem[i] : S.bnode0 + (i - d.nv);
        for (int e = 0; e < S.nt_pad; ++e) {
            int g = S.tet0 + e;
            if (e < d.nt) {
                tv[g] = make_int4(fem[d.tets[4 * e]], fem[d.tets[4 * e + 1]], fem[d.tets[4 * e + 2]], fem[d.tets[4 * e + 3]]);
                tvalid[g] = 1; tE[g] = d.tet_E[e]; tnu[g] = d.tet_nu[e]; trho[g] = d.tet_rho[e];
                ext2tet.push_back(g);
            } else {
                tv[g] = make_int4(S.node0, S.node0, S.node0, S.node0);
            }
        }
        for (int b = 0; b < d.nb; ++b) {
            int g = S.body0 + b;
            bM[16 * (size_t)g] = d.body_mass[b];
            for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) bM[16 * (size_t)g + (1 + i) * 4 + 1 + j] = d.body_S[9 * b + 3 * i + j];
            bvol[g] = d.body_vol[b]; bkappa[g] = d.body_kappa[b];
            for (int k = 0; k < 3; ++k) bext[3 * (size_t)g + k] = d.body_ext[3 * b + k];
            body_node0[g] = S.bnode0 + 4 * b;
            body_scene[g] = s;
        }
        for (int k = 0; k < d.ns; ++k) {
            int g = S.sp0 + k;
            auto conv = [&](int kind, int idx) { return kind == 0 ? fem[idx] : (kind == 1 ? S.body0 + idx : S.drv0 + idx); };
            ska[g] = d.sp_ka[k]; sia[g] = conv(d.sp_ka[k], d.sp_ia[k]);
            skb[g] = d.sp_kb[k]; sib[g] = conv(d.sp_kb[k], d.sp_ib[k]);
            for (int m = 0; m < 3; ++m) { sxa[3 * (size_t)g + m] = d.sp_xa[3 * k + m]; sxb[3 * (size_t)g + m] = d.sp_xb[3 * k + m]; }
            sk[g] = d.sp_k[k]; sscene[g] = s;
        }
        for (int j = 0; j < d.nj; ++j) joint_sp[S.jt0 + j] = S.sp0 + d.joint_spring[j];
        for (int k = 0; k < d.nd; ++k) {
            driven[S.drv0 + k] = S.body0 + d.driven_body[k];
            for (int m = 0; m < 12; ++m) targets[12 * (size_t)(S.drv0 + k) + m] = d.body_q[12 * d.driven_body[k] + m];
        }
        // contact vertices
        const HostTopo &tp = topo[s];
        std::vector<int> ext2cv(d.nv + d.nbv + d.nsv, -1);
        int static_obj = -1;
        for (int o = 0; o < d.nobj; ++o) if (d.obj_kind[o] == 2) { static_obj = o; break; }
        for (int i = 0; i < S.ncv; ++i) {
            int e = tp.surf[i], g = S.cv0 + i;
            ext2cv[e] = g;
            cv_scene[g] = s;
            if (e < d.nv) { cv_node[g] = fem[e]; cv_obj[g] = S.obj0 + d.vobj[e]; }
            else if (e < d.nv + d.nbv) {
                int j = e - d.nv;
                cv_body[g] = S.body0 + d.bv_body[j];
                cv_obj[g] = S.obj0 + d.body_obj[d.bv_body[j]];
                for (int m = 0; m < 3; ++m) cv_x[3 * (size_t)g + m] = d.bv_xbar[3 * j + m];
            } else {
                int j = e - d.nv - d.nbv;
                cv_obj[g] = static_obj >= 0 ? S.obj0 + static_obj : -1;
                for (int m = 0; m < 3; ++m) cv_x[3 * (size_t)g + m] = d.sv_x[3 * j + m];
            }
        }
        for (int k = 0; k < S.ntri; ++k)
            tri4[S.tri0 + k] = make_int4(ext2cv[tp.tri[k][0]], ext2cv[tp.tri[k][1]], ext2cv[tp.tri[k][2]], s);
        auto rest = [&](int e, double *x) {
            if (e < d.nv) for (int m = 0; m < 3; ++m) x[m] = d.X[3 * e + m];
            else if (e < d.nv + d.nbv) for (int m = 0; m < 3; ++m) x[m] = d.bv_xbar[3 * (e - d.nv) + m];
            else for (int m = 0; m < 3; ++m) x[m] = d.sv_x[3 * (e - d.nv - d.nbv) + m];
        };
        for (int k = 0; k < S.nedge; ++k) {
            edge2[S.edge0 + k] = make_int2(ext2cv[tp.edge[k][0]], ext2cv[tp.edge[k][1]]);
            double a[3], b[3];
            rest(tp.edge[k][0], a); rest(tp.edge[k][1], b);
            double dd = 0.0;
            for (int m = 0; m < 3; ++m) dd += (b[m] - a[m]) * (b[m] - a[m]);
            rest2[S.edge0 + k] = dd;
        }
        for (int o = 0; o < d.nobj; ++o) okind[S.obj0 + o] = d.obj_kind[o];
        for (int k = 0; k < d.nex; ++k) { excl[2 * exo] = S.obj0 + d.excl[2 * k]; excl[2 * exo + 1] = S.obj0 + d.excl[2 * k + 1]; ++exo; }
        // characteristic length L (initial bounding box of FEM vertices and body boxes)
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int i = 0; i < d.nv; ++i)
            for (int k = 0; k < 3; ++k) { lo[k] = std::min(lo[k], d.X[3 * i + k]); hi[k] = std::max(hi[k], d.X[3 * i + k]); }
        for (int b = 0; b < d.nb; ++b)
            for (int k = 0; k < 3; ++k) {
                lo[k] = std::min(lo[k], d.body_q[12 * b + k] - d.body_ext[3 * b + k]);
                hi[k] = std::max(hi[k], d.body_q[12 * b + k] + d.body_ext[3 * b + k]);
            }
        double dd = 0.0;
        for (int k = 0; k < 3; ++k) if (hi[k] > lo[k]) dd += (hi[k] - lo[k]) * (hi[k] - lo[k]);
        S.L = std::sqrt(dd);
        S.thr = S.newton_tol * S.h * S.L;
    }
    // node -> incident tets (fixed order), as codes 4 tet + local vertex, for
    // the lumped mass and the gradient gather
    for (int e = 0; e < tet; ++e)
        if (tvalid[e]) { adj_ptr[tv[e].x + 1]++; adj_ptr[tv[e].y + 1]++; adj_ptr[tv[e].z + 1]++; adj_ptr[tv[e].w + 1]++; }
    for (int i = 0; i < node; ++i) adj_ptr[i + 1] += adj_ptr[i];
    adj.resize(adj_ptr[node]);
    {
        std::vector<int> fill(adj_ptr.begin(), adj_ptr.end() - 1);
        for (int e = 0; e < tet; ++e)
            if (tvalid[e]) {
                adj[fill[tv[e].x]++] = 4 * e; adj[fill[tv[e].y]++] = 4 * e + 1;
                adj[fill[tv[e].z]++] = 4 * e + 2; adj[fill[tv[e].w]++] = 4 * e + 3;
            }
    }
    // Block-CSR pattern over all node rows: tetrahedra, the 4x4 node blocks of
    // every affine body, and the (constant) spring couplings between the nodes
    // of a spring's two sides.  Padding nodes have empty rows.
    auto spring_nodes = [&](int kind, int idx, std::vector<int> &out) {
        if (kind == 0) out.push_back(idx);
        else if (kind == 1) for (int k = 0; k < 4; ++k) out.push_back(body_node0[idx] + k);
    };
    std::vector<int> row_ptr(node + 1, 0), col;
    {
        std::vector<std::vector<int>> cols(node);
        for (int e = 0; e < tet; ++e) {
            if (!tvalid[e]) continue;
            int v[4] = {tv[e].x, tv[e].y, tv[e].z, tv[e].w};
            for (int a = 0; a < 4; ++a) for (int b = 0; b < 4; ++b) cols[v[a]].push_back(v[b]);
        }
        for (int b = 0; b < body; ++b)
            for (int k = 0; k < 4; ++k) for (int m = 0; m < 4; ++m) cols[body_node0[b] + k].push_back(body_node0[b] + m);
        for (int k = 0; k < sp; ++k) {
            std::vector<int> nd;
            spring_nodes(ska[k], sia[k], nd);
            spring_nodes(skb[k], sib[k], nd);
            for (int a : nd) for (int b : nd) cols[a].push_back(b);
        }
        for (int i = 0; i < node; ++i) {
            auto &cl = cols[i];
            if (node_kind[i] == 0) cl.push_back(i);   // every FEM node keeps a diagonal block (mass)
            std::sort(cl.begin(), cl.end());
            cl.erase(std::unique(cl.begin(), cl.end()), cl.end());
            row_ptr[i + 1] = row_ptr[i] + (int)cl.size();
        }
        col.resize(row_ptr[node]);
        for (int i = 0; i < node; ++i) std::copy(cols[i].begin(), cols[i].end(), col.begin() + row_ptr[i]);
    }
    c->nnzb = row_ptr[node];
    c->nnzb_fem = 0;
    std::vector<int> tslot(16 * (size_t)tet, 0), diag_slot(node, -1), bslot(16 * (size_t)std::max(body, 1), 0);
    auto find_slot = [&](int r, int cc) {
        auto b = col.begin() + row_ptr[r], e = col.begin() + row_ptr[r + 1];
        return (int)(std::lower_bound(b, e, cc) - col.begin());
    };
    for (int e = 0; e < tet; ++e) {
        if (!tvalid[e]) continue;
        int v[4] = {tv[e].x, tv[e].y, tv[e].z, tv[e].w};
        for (int a = 0; a < 4; ++a) for (int b = 0; b < 4; ++b) tslot[16 * (size_t)e + 4 * a + b] = find_slot(v[a], v[b]);
    }
    for (int i = 0; i < node; ++i) {
        if (node_kind[i] != 2) diag_slot[i] = find_slot(i, i);
        if (node_kind[i] == 0) c->nnzb_fem += row_ptr[i + 1] - row_ptr[i];
    }
    for (int b = 0; b < body; ++b)
        for (int k = 0; k < 4; ++k) for (int m = 0; m < 4; ++m) bslot[16 * b + 4 * k + m] = find_slot(body_node0[b] + k, body_node0[b] + m);
    // matrix slot -> tet blocks that land in it (tet order)
    std::vector<int> sc_ptr(c->nnzb + 1, 0), sc_list;
    for (int e = 0; e < tet; ++e)
        if (tvalid[e]) for (int q = 0; q < 16; ++q) sc_ptr[tslot[16 * (size_t)e + q] + 1]++;
    for (int i = 0; i < c->nnzb; ++i) sc_ptr[i + 1] += sc_ptr[i];
    sc_list.resize(sc_ptr[c->nnzb]);
    {
        std::vector<int> fill(sc_ptr.begin(), sc_ptr.end() - 1);
        for (int e = 0; e < tet; ++e)
            if (tvalid[e]) for (int q = 0; q < 16; ++q) sc_list[fill[tslot[16 * (size_t)e + q]]++] = 16 * e + q;
    }
    // segment tables (per-scene ranges) used by the segmented reductions
    c->seg_surf.resize(n + 1); c->seg_tri.resize(n + 1); c->seg_edge.resize(n + 1); c->seg_sp.resize(n + 1); c->seg_body.resize(n + 1);
    for (int s = 0; s < n; ++s) {
        c->seg_surf[s] = c->sc[s].cv0; c->seg_tri[s] = c->sc[s].tri0; c->seg_edge[s] = c->sc[s].edge0;
        c->seg_sp[s] = c->sc[s].sp0; c->seg_body[s] = c->sc[s].body0;
    }
    c->seg_surf[n] = cv; c->seg_tri[n] = tri; c->seg_edge[n] = edge; c->seg_sp[n] = sp; c->seg_body[n] = body;
    // half-space entries: the moving surface vertices of each scene that has one
    std::vector<int> hs_cv;
    std::vector<double> hs_plane(4 * (size_t)n, 0.0);
    c->seg_hs.assign(n + 1, 0);
    for (int s = 0; s < n; ++s) {
        const SceneInfo &S = c->sc[s];
        c->seg_hs[s] = (int)hs_cv.size();
        for (int k = 0; k < 4; ++k) hs_plane[4 * (size_t)s + k] = S.hs[k];
        if (!S.hs_on) continue;
        for (int i = 0; i < S.ncv; ++i)
            if (S.surf_ext[i] < scenes[s].nv + scenes[s].nbv) hs_cv.push_back(S.cv0 + i);
    }
    c->seg_hs[n] = (int)hs_cv.size();
    c->M_HS = (int64_t)hs_cv.size();

    // Entry lists of the deterministic run sums (ipc_runsum.h), built once:
    //  spring gradients: code 8 s + 4 side + q -> node, sorted by node;
    //  constant spring blocks: code 64 s + 8 i + j -> matrix slot, sorted by
    //   slot, with i, j the positions of the two nodes in the spring's node
    //   list (side a's nodes, then side b's, as spring_nodes lists them);
    //  contact vertices of every body, in contact-vertex order.
    std::vector<std::pair<int, int>> spg, spc;
    for (int k = 0; k < sp; ++k) {
        std::vector<int> nd;
        for (int side = 0; side < 2; ++side) {
            int kind = side ? skb[k] : ska[k], idx = side ? sib[k] : sia[k];
            if (kind == 0) spg.push_back({idx, 8 * k + 4 * side});
            else if (kind == 1)
                for (int q = 0; q < 4; ++q) spg.push_back({body_node0[idx] + q, 8 * k + 4 * side + q});
            spring_nodes(kind, idx, nd);
        }
        for (int i = 0; i < (int)nd.size(); ++i)
            for (int j = 0; j < (int)nd.size(); ++j) spc.push_back({find_slot(nd[i], nd[j]), 64 * k + 8 * i + j});
    }
    std::sort(spg.begin(), spg.end());
    std::sort(spc.begin(), spc.end());
    std::vector<int> spg_key(spg.size() + 1), spg_code(spg.size() + 1), spc_key(spc.size() + 1), spc_code(spc.size() + 1);
    for (size_t i = 0; i < spg.size(); ++i) { spg_key[i] = spg[i].first; spg_code[i] = spg[i].second; }
    for (size_t i = 0; i < spc.size(); ++i) { spc_key[i] = spc[i].first; spc_code[i] = spc[i].second; }
    std::vector<int> body_cv_ptr(body + 1, 0), body_cv;
    for (int g = 0; g < cv; ++g) if (cv_body[g] >= 0) body_cv_ptr[cv_body[g] + 1]++;
    for (int b = 0; b < body; ++b) body_cv_ptr[b + 1] += body_cv_ptr[b];
    body_cv.resize(body_cv_ptr[body] + 1);
    {
        std::vector<int> fill(body_cv_ptr.begin(), body_cv_ptr.end() - 1);
        for (int g = 0; g < cv; ++g) if (cv_body[g] >= 0) body_cv[fill[cv_body[g]]++] = g;
    }

    // ---- plan only: the device bytes a context over a caller's workspace
    // takes, an upper bound from the sizes above.  Buffers are listed as the
    // creation, set-up, reserve_capacity and the first calls take them; each
    // is rounded up to the arena's 256-byte granule, sums of sorted-entry
    // tables, coarse domains and sort storage are bounded from above.
    if (plan) {
        const int64_t P = std::max<int64_t>(caps[0], 1), C = std::max<int64_t>(caps[1], 1), B = std::max<int64_t>(caps[2], 1);
        const int64_t N = node, T = tet, NB = std::max(body, 1), NS = std::max(sp, 1), CVn = std::max(cv, 1), NZ = std::max(c->nnzb, 1);
        const int64_t Pp = std::max<int64_t>(std::max(tri, edge), 1), Q = std::max<int64_t>(std::max(cv, edge), 1);
        const int64_t NW = std::max<int64_t>(C, N) / TILE + 1, PC = std::max(P, C);
        const int64_t ndom = N / (CG_AGG * CG_DOM) + 2 * (int64_t)n, ngrp = N / CG_AGG + 2 * (int64_t)n;
        const int64_t MH = std::max<int64_t>(c->M_HS, 1);
        const std::vector<int64_t> nbuf = {
            // nodes: state, predictor and solver vectors (14 x 3 doubles, 3 more for one scene), kinds, maps, mass,
            // inverse blocks
            (n == 1 ? 17 : 14) * 24 * N, 4 * N, 4 * N, 4 * (int64_t)(dof / 3) + 4, 8 * N, 72 * N, 8 * (N / TILE + 1), 4 * N, 4 * N,
            // tetrahedra: vertices, inverse rest shape, volume and Lame, modulus and ratio, gradients and blocks,
            // slot and adjacency lists, the temporary density and validity
            16 * T, 72 * T, 8 * T, 8 * T, 8 * T, 8 * T, 8 * T, 4 * T + 4, 96 * std::max<int64_t>(T, 1), 720 * std::max<int64_t>(T, 1),
            4 * (NZ + 1), 4 * (int64_t)sc_list.size() + 4, 4 * (N + 1), 4 * (int64_t)adj.size() + 4, 8 * T, 4 * T, 8 * (T / TILE + 1),
            // matrix: pattern, values, constant part, slots, scene of each block
            4 * (N + 1), 4 * NZ, 4 * N, 72 * NZ, 72 * NZ, 64 * NB, 4 * NZ,
            // bodies
            128 * NB, 8 * NB, 8 * NB, 24 * NB, 4 * NB, 4 * NB, 1152 * NB, 8 * NB, 4 * (NB + 1), 4 * (int64_t)body_cv.size() + 4,
            // springs, drive targets, joint points, their entry lists
            4 * NS, 4 * NS, 4 * NS, 4 * NS, 4 * NS, 24 * NS, 24 * NS, 8 * NS, 8 * NS, 24 * NS,
            8 * (int64_t)spg.size() + 8, 8 * (int64_t)spc.size() + 8, 96 * std::max(drv, 1) + 96, 4 * std::max(drv, 1), 4 * std::max(jt, 1),
            // contact vertices, triangles, edges, objects
            16 * CVn, 24 * CVn, 48 * CVn, 16 * std::max(tri, 1), 8 * std::max(edge, 1), 8 * std::max(edge, 1), 4 * std::max(obj, 1),
            8 * std::max(ex, 1) + 8,
            // per scene: scalars, parameters, segment tables, flags, PCG state, Morton boxes
            8 * NSLOT * (int64_t)n, 64 * (int64_t)n, 24 * (int64_t)n, 4 * (int64_t)n, 16 * (int64_t)(n + 1), 4 * NREGION * (int64_t)(n + 1),
            16 * (int64_t)n, 64 * (int64_t)n, 16 * (int64_t)n, 8 * (int64_t)n, 48 * (int64_t)n, 4 * (int64_t)n, 16, 16,
            // tiles and PCG partials, workgroup records
            4 * (N / TILE + 1), 4 * (T / TILE + 1), 8 * (N / TILE + 1), 32 * (N / TILE + 1), 32 * (N / 256 + 1),
            // coarse correction: groups, domains, inverses
            4 * ngrp, 4 * (ndom + 1), 4 * N, 4 * N, 4 * ndom, 8 * CG_N * CG_N * ndom, 16 * CG_SPLIT * ndom, 4 * CG_AGG * CG_DOM * ndom,
            4 * (ndom + 1), 4 * NB, 4 * NB,
            // reserve_capacity: broad phase
            48 * Pp, 8 * Pp, 8 * Pp, 8 * Pp, 8 * Pp, 4 * Pp, 4 * Pp, 8 * Pp, 4 * Pp, 48 * Pp, 48 * (2 * Pp + 64), 4 * (Pp + 1),
            4 * (Pp + 1), 4 * Pp, 4 * (Q + 1), 4 * (Q + 1), 8 * TRAV_STASH * Q, 8 * Q, 8 * Q, 4 * Q, 4 * Q,
            // candidates, masks, pairs
            8 * std::max(Pp, NW), 4 * (NW + 1), 4 * (NW + 1), 8 * C, 8 * C, 48 * CVn + 8, 8 * P, 8 * P,
            // barrier
            8 * (PC + 1), 8 * (PC / TILE + 1), 96 * P + 24, 4 * 4 * (4 * P + 1), 16 * (P + 1), 360 * (P + 1), 4 * (P + 1),
            4 * 4 * (16 * P + 1),
            // friction lag
            16 * P, 32 * P, 24 * P, 8 * P, 24 * P, 48 * P, 4 * P, 4 * P, 8 * P, 4 * P, 4 * 4 * 16 * P, 96 * P, 4 * 4 * 4 * P,
            8 * (P + 1), 8 * (P / TILE + 1), 24 * CVn + 24,
            // pair-local blocks
            4 * (2 * P + 1), 4 * (2 * P + 1), 16 * B, 7 * 4 * (B + 1), 144 * B, 16,
            // run sums, PCG long rows and partials
            2 * 8 * (9 * (16 * P / TILE + 1) + 1), 8 * (N + 65), 8 * (N / TILE + 1), 32 * (N / TILE + 1), 4 * (N + 1),
            // half-space entries: list, planes, energies and chunk sums, lag, Hessian blocks, slot entries
            4 * MH, 32 * (int64_t)n, 8 * (MH + 1), 8 * (MH + 1), 8 * (MH / TILE + 1), 8 * (MH / TILE + 1), 8 * MH, 24 * MH,
            72 * MH, 4 * 4 * 16 * MH, 4 * (int64_t)n,
            // sort and scan storage (rocprim: a copy of keys and values plus per-block counts), bounded
            16 * std::max<int64_t>(std::max(std::max(16 * P, 16 * MH), B), std::max(Pp, Q)) + (4 << 20)};
        size_t bytes = 0;
        for (int64_t b : nbuf) bytes += Arena::round((size_t)std::max<int64_t>(b, 1));
        *plan = bytes + bytes / 16 + (1 << 20);   // 6 % and 1 MiB against fragmentation of the free list
        return;
    }

    // ---- upload
    Dev &D = c->d;
    D.y.upload(X, st); D.ydot.upload(V, st);
    for (auto *b : {&D.xt, &D.y0, &D.yt, &D.g, &D.p, &D.r, &D.z, &D.q, &D.w, &D.x, &D.v1, &D.v2}) b->alloc(3 * (size_t)node);
    if (n == 1)   // the one-launch PCG step's second r, z and s (a padding node's entries stay 0)
        for (auto *b : {&D.r2, &D.z2, &D.q2}) { b->alloc(3 * (size_t)node); b->zero(st, 3 * (size_t)node); }
    IPC_HIP(hipMemcpyAsync(D.xt.p, D.y.p, 3 * (size_t)node * sizeof(double), hipMemcpyDeviceToDevice, st));
    D.node_scene.upload(node_scene, st); D.node_kind.upload(node_kind, st); D.ext2node.upload(ext2node, st);
    coarse_setup(c);   // groups and domains of the coarse preconditioner: runs of the Morton order
    D.mass.alloc(node); D.dinv.alloc(9 * (size_t)node);
    D.tv.upload(tv, st);
    D.Bm.alloc(9 * (size_t)tet); D.vol.alloc(tet); D.tmu.alloc(tet); D.tlam.alloc(tet);
    D.sc_ptr.upload(sc_ptr, st); D.sc_list.upload(sc_list, st);
    D.tgrad.alloc(12 * (size_t)std::max(tet, 1)); D.telem.alloc(90 * (size_t)std::max(tet, 1));
    D.row_ptr.upload(row_ptr, st); D.col.upload(col, st); D.diag_slot.upload(diag_slot, st);
    {
        std::vector<int> slot_scene(std::max(c->nnzb, 1), 0);
        for (int r = 0; r < node; ++r)
            for (int k = row_ptr[r]; k < row_ptr[r + 1]; ++k) slot_scene[k] = node_scene[r];
        D.slot_scene.upload(slot_scene, st);
    }
    D.val.alloc(9 * (size_t)std::max(c->nnzb, 1));
    D.val_const.alloc(9 * (size_t)std::max(c->nnzb, 1)); D.val_const.zero(st, 9 * (size_t)std::max(c->nnzb, 1));
    D.bslot.upload(bslot, st);
    D.bM.upload(bM, st); D.bvol.upload(bvol, st); D.bkappa.upload(bkappa, st); D.bext.upload(bext, st);
    D.body_node0.upload(body_node0, st); D.body_scene.upload(body_scene, st);
    D.dinvB.alloc(144 * (size_t)std::max(body, 1));
    D.body_part.alloc(std::max(body, 1));
    D.sp_ka.upload(ska, st); D.sp_ia.upload(sia, st); D.sp_kb.upload(skb, st); D.sp_ib.upload(sib, st);
    D.sp_scene.upload(sscene, st); D.sp_xa.upload(sxa, st); D.sp_xb.upload(sxb, st); D.sp_k.upload(sk, st);
    D.sp_part.alloc(std::max(sp, 1));
    D.sp_f.alloc(3 * (size_t)std::max(sp, 1));
    D.spg_key.upload(spg_key, st); D.spg_code.upload(spg_code, st); D.n_spg = (int64_t)spg.size();
    D.spc_key.upload(spc_key, st); D.spc_code.upload(spc_code, st); D.n_spc = (int64_t)spc.size();
    D.body_cv_ptr.upload(body_cv_ptr, st); D.body_cv.upload(body_cv, st);
    D.targets.upload(targets, st); D.driven_body.upload(driven, st); D.joint_sp.upload(joint_sp, st);
    D.cv_node.upload(cv_node, st); D.cv_body.upload(cv_body, st); D.cv_obj.upload(cv_obj, st); D.cv_scene.upload(cv_scene, st);
    D.cv_x.upload(cv_x, st);
    D.xw.alloc(3 * (size_t)std::max(cv, 1)); D.xw1.alloc(3 * (size_t)std::max(cv, 1));
    D.hs_cv.upload(hs_cv, st); D.hs_plane.upload(hs_plane, st);
    hs_setup(c);
    D.tri.upload(tri4, st); D.edge.upload(edge2, st); D.edge_rest2.upload(rest2, st);
    D.obj_kind.upload(okind, st); D.excl.upload(excl, st);
    D.scal.alloc((size_t)n * NSLOT); D.scal.zero(st, (size_t)n * NSLOT);
    D.part_node.alloc(node / TILE + 1); D.part_tet.alloc(tet / TILE + 1);
    D.tile_scene_node.upload(tile_node, st); D.tile_scene_tet.upload(tile_tet, st);
    D.seg.alloc(4 * (size_t)(n + 1));

    // ---- device precompute
    {
        DBuf<double> drho;
        DBuf<int> dvalid;
        D.tE.upload(tE, st); D.tnu.upload(tnu, st); drho.upload(trho, st); dvalid.upload(tvalid, st);
        c->ext_tets = (int64_t)ext2tet.size();
        D.ext2tet.upload(ext2tet, st);
        D.fadj_ptr.upload(adj_ptr, st); D.fadj.upload(adj, st);
        if (tet > 0)
            hipLaunchKernelGGL(k_tet_precompute, dim3(blocks_for(tet)), dim3(BLOCK), 0, st, tet, D.tv.p, D.y.p, D.tE.p, D.tnu.p,
                               D.Bm.p, D.vol.p, D.tmu.p, D.tlam.p, dvalid.p);
        hipLaunchKernelGGL(k_node_mass, dim3(blocks_for(node)), dim3(BLOCK), 0, st, node, D.fadj_ptr.p, D.fadj.p, D.vol.p, drho.p, D.mass.p);
        std::vector<double> h2s(n);
        for (int s = 0; s < n; ++s) h2s[s] = c->sc[s].h * c->sc[s].h;
        DBuf<double> dh2; dh2.upload(h2s, st);
        build_const_part(c, dh2.p);
        // kappa (automatic: 10 * mean FEM vertex mass * |g| * h^2 / dhat)
        DBuf<double> msum; msum.alloc(n);
        for (int s = 0; s < n; ++s)
            if (scenes[s].nv > 0)
                hipLaunchKernelGGL(k_sum_mass, dim3(1), dim3(256), 0, st, (int)c->sc[s].entry.size(), D.mass.p, c->sc[s].node0,
                                   msum.p + s);   // the FEM region: the bodies' slots in it hold no mass
        std::vector<double> hm(n, 0.0);
        IPC_HIP(hipMemcpyAsync(hm.data(), msum.p, n * sizeof(double), hipMemcpyDeviceToHost, st));
        IPC_HIP(hipStreamSynchronize(st));
        for (int s = 0; s < n; ++s) {
            SceneInfo &S = c->sc[s];
            const ipc_scene_desc &d = scenes[s];
            if (d.nv > 0) S.mbar = hm[s] / d.nv;
            else {
                double bm = 0.0;
                for (int b = 0; b < d.nb; ++b) bm += d.body_mass[b];
                S.mbar = d.nbv ? bm / d.nbv : 0.0;
            }
            double gn = std::sqrt(S.g[0] * S.g[0] + S.g[1] * S.g[1] + S.g[2] * S.g[2]);
            if (S.kappa <= 0.0) S.kappa = 10.0 * S.mbar * gn * S.h * S.h / S.dhat;
        }
    }
}

} // namespace ipc
