// Inertia, Stable Neo-Hookean FEM, affine-body orthogonality and point-spring
// terms of the incremental potential (Sec. III-C.1-2, Eq. (1)-(3)).
//
// One thread per tetrahedron / body / spring.  The FEM kernel forms the 9x9
// Hessian of the energy density in F, projects it to PSD in registers (the
// energy's closed-form eigensystem: only negative modes are removed), maps it
// to the 3x3 blocks of the element and writes the 10 upper ones, with its 12
// gradient entries, to per-tet arrays; two gather kernels then sum them per
// matrix slot and per node in a fixed order (no atomics, deterministic).
// Energies are reduced per wavefront (scene-aligned tiles) for a
// deterministic sum.
#include "ipc_device.h"
#include "ipc_internal.h"
#include "ipc_runsum.h"
#include "ipc_kernels.h"
#include "ipc_eigsys.h"

namespace ipc {

// ---------------------------------------------------------------------------
// nodes: inertia of FEM vertices; initialises g (FEM nodes) and zeroes the rest
// ---------------------------------------------------------------------------
__global__ void k_node_inertia(int N, const double *__restrict__ y, const double *__restrict__ xt, const double *__restrict__ mass,
                               const int *__restrict__ kind, double *__restrict__ g, double *__restrict__ part)
{
    int n = blockIdx.x * blockDim.x + threadIdx.x;
    double e = 0.0;
    if (n < N) {
        d3 gv = {0.0, 0.0, 0.0};
        if (kind[n] == 0) {
            double m = mass[n];
            d3 d = {y[3 * (size_t)n] - xt[3 * (size_t)n], y[3 * (size_t)n + 1] - xt[3 * (size_t)n + 1], y[3 * (size_t)n + 2] - xt[3 * (size_t)n + 2]};
            e = 0.5 * m * (d.x * d.x + d.y * d.y + d.z * d.z);
            gv = {m * d.x, m * d.y, m * d.z};
        }
        if (g) st3(g, n, gv);
    }
    e = wave_sum(e);
    if (part && (threadIdx.x & (TILE - 1)) == 0 && n < N) part[n / TILE] = e;
}

// ---------------------------------------------------------------------------
// FEM (rest-stable Stable Neo-Hookean)
// ---------------------------------------------------------------------------
// index of the upper block (A, B), A <= B, of a tet's 4x4 block matrix (0..9)
__host__ __device__ constexpr int tet_ublk(int A, int B) { return A * (7 - A) / 2 + B; }

template <int MODE>   // 0 energy, 1 energy+gradient, 2 gradient+Hessian
__global__ void __launch_bounds__(256) k_fem(int T, const int4 *__restrict__ tv, const double *__restrict__ Bm,
                                             const double *__restrict__ vol, const double *__restrict__ tmu,
                                             const double *__restrict__ tlam, const double *__restrict__ y,
                                             const int *__restrict__ tile_scene, const double *__restrict__ h2s,
                                             double *__restrict__ tgrad, double *__restrict__ telem, int project,
                                             double *__restrict__ part, const int *__restrict__ active)
{
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    double energy = 0.0;
    // active (nullable): only the tets of scenes whose flag is set (a wavefront
    // of tets is one scene's, so the test is uniform over it)
    if (e < T && vol[e] > 0.0 && (!active || active[tile_scene[e / TILE]])) {
        int4 t = tv[e];
        int vi[4] = {t.x, t.y, t.z, t.w};
        d3 x[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) x[a] = ld3(y, vi[a]);
        double c[4][3];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            c[1][j] = Bm[(size_t)(0 * 3 + j) * T + e];
            c[2][j] = Bm[(size_t)(1 * 3 + j) * T + e];
            c[3][j] = Bm[(size_t)(2 * 3 + j) * T + e];
            c[0][j] = -(c[1][j] + c[2][j] + c[3][j]);
        }
        d3 f[3];
#pragma unroll
        for (int j = 0; j < 3; ++j)
            f[j] = {c[0][j] * x[0].x + c[1][j] * x[1].x + c[2][j] * x[2].x + c[3][j] * x[3].x,
                    c[0][j] * x[0].y + c[1][j] * x[1].y + c[2][j] * x[2].y + c[3][j] * x[3].y,
                    c[0][j] * x[0].z + c[1][j] * x[1].z + c[2][j] * x[2].z + c[3][j] * x[3].z};
        double mu = tmu[e], lh = tlam[e] + mu;
        d3 cof[3] = {cr(f[1], f[2]), cr(f[2], f[0]), cr(f[0], f[1])};
        double J = dt(f[0], cof[0]);
        double I2 = dt(f[0], f[0]) + dt(f[1], f[1]) + dt(f[2], f[2]);
        double w = h2s[tile_scene[e / TILE]] * vol[e];
        energy = w * (0.5 * mu * (I2 - 3.0) - mu * (J - 1.0) + 0.5 * lh * (J - 1.0) * (J - 1.0));
        double sc = lh * (J - 1.0) - mu;
        if (MODE >= 1) {
            d3 P[3];
#pragma unroll
            for (int j = 0; j < 3; ++j) P[j] = {mu * f[j].x + sc * cof[j].x, mu * f[j].y + sc * cof[j].y, mu * f[j].z + sc * cof[j].z};
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                d3 ga = {w * (c[a][0] * P[0].x + c[a][1] * P[1].x + c[a][2] * P[2].x),
                         w * (c[a][0] * P[0].y + c[a][1] * P[1].y + c[a][2] * P[2].y),
                         w * (c[a][0] * P[0].z + c[a][1] * P[1].z + c[a][2] * P[2].z)};
                st3(tgrad, a * T + e, ga);
            }
        }
        if (MODE == 2) {
            double H[45];
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int b = 0; b < 3; ++b)
#pragma unroll
                        for (int j = 0; j < 3; ++j) {
                            int R = 3 * a + i, C = 3 * b + j;
                            if (R > C) continue;
                            double v = lh * comp(cof[a], i) * comp(cof[b], j) + (R == C ? mu : 0.0);
                            if (a != b) {
                                int cc = 3 - a - b;
                                double sg = (b == (a + 2) % 3) ? 1.0 : -1.0;
                                v += sc * sg * skew(f[cc], i, j);
                            }
                            H[pk9(R, C)] = v;
                        }
            if (project) {
                double Fm[3][3];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    Fm[0][a] = f[a].x;
                    Fm[1][a] = f[a].y;
                    Fm[2][a] = f[a].z;
                }
                iso::project_snh(H, Fm, mu, lh, sc);
            }
#pragma unroll
            for (int B = 0; B < 4; ++B) {
                double Tm[9][3];   // Tm[(j,r)][q] = sum_l c[B][l] H[(j,r),(l,q)]
#pragma unroll
                for (int R = 0; R < 9; ++R)
#pragma unroll
                    for (int q = 0; q < 3; ++q)
                        Tm[R][q] = c[B][0] * H[pk9(R, q)] + c[B][1] * H[pk9(R, 3 + q)] + c[B][2] * H[pk9(R, 6 + q)];
#pragma unroll
                for (int A = 0; A <= B; ++A) {   // upper blocks only: (B, A) is the transpose
                    double *blk = telem + 9 * ((size_t)tet_ublk(A, B) * T + e);
#pragma unroll
                    for (int r = 0; r < 3; ++r)
#pragma unroll
                        for (int q = 0; q < 3; ++q)
                            blk[3 * r + q] = w * (c[A][0] * Tm[r][q] + c[A][1] * Tm[3 + r][q] + c[A][2] * Tm[6 + r][q]);
                }
            }
        }
    }
    energy = wave_sum(energy);
    if (part && (threadIdx.x & (TILE - 1)) == 0 && e < T) part[e / TILE] = energy;
}

// matrix values: the constant part (lumped mass, springs) plus the tet blocks
// of each slot, summed in tet order; one thread per (slot, entry).  A tet
// stores its 10 upper blocks (A <= B); block (A, B) with A > B is read as
// entry (c, r) of block (B, A).
__global__ void k_bsr_assemble(int64_t n9, int T, const int *__restrict__ sc_ptr, const int *__restrict__ sc_list,
                               const double *__restrict__ telem, const double *__restrict__ vc, double *__restrict__ val,
                               const int *__restrict__ slot_scene, const int *__restrict__ active)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n9) return;
    int k = (int)(i / 9), q = (int)(i % 9), qt = 3 * (q % 3) + q / 3;
    if (active && !active[slot_scene[k]]) return;
    double acc = vc[i];
    // eight contributions at a time: their codes, then their entries, are
    // loaded together; the sum keeps the list order
    const int je = sc_ptr[k + 1];
    for (int j = sc_ptr[k]; j < je; j += 8) {
        int code[8];
        double v[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) code[m] = j + m < je ? sc_list[j + m] : 0;
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            int A = (code[m] >> 2) & 3, B = code[m] & 3;
            bool tr = A > B;
            int u = tr ? tet_ublk(B, A) : tet_ublk(A, B);
            v[m] = j + m < je ? telem[9 * ((size_t)u * T + (code[m] >> 4)) + (tr ? qt : q)] : 0.0;
        }
#pragma unroll
        for (int m = 0; m < 8; ++m)
            if (j + m < je) acc += v[m];
    }
    val[i] = acc;
}

// node gradients of the tets: g[n] += sum over incident (tet, vertex), in order
__global__ void k_fem_grad_gather(int N, int T, const int *__restrict__ adj_ptr, const int *__restrict__ adj,
                                  const double *__restrict__ tgrad, double *__restrict__ g, const int *__restrict__ node_scene,
                                  const int *__restrict__ active)
{
    int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    if (active && !active[node_scene[n]]) return;
    int k0 = adj_ptr[n], k1 = adj_ptr[n + 1];
    if (k0 == k1) return;
    d3 acc = ld3(g, n);
    for (int k = k0; k < k1; ++k) {
        int code = adj[k];
        d3 v = ld3(tgrad, (code & 3) * T + (code >> 2));
        acc.x += v.x; acc.y += v.y; acc.z += v.z;
    }
    st3(g, n, acc);
}

// ---------------------------------------------------------------------------
// affine bodies: inertia (4x4 mass matrix (x) I3) + orthogonality kappa V |AA^T - I|^2
// ---------------------------------------------------------------------------
template <int MODE>   // launched with 64 threads (few bodies: short waves)
__global__ void __launch_bounds__(64) k_body(int NB, const int *__restrict__ node0, const int *__restrict__ bscene, const double *__restrict__ bM,
                       const double *__restrict__ bvol, const double *__restrict__ bkappa, const double *__restrict__ h2s,
                       const double *__restrict__ y, const double *__restrict__ xt, double *__restrict__ g,
                       double *__restrict__ val, const int *__restrict__ bslot, int project, double *__restrict__ part)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= NB) return;
    int n0 = node0[b];
    const double *M = bM + 16 * (size_t)b;
    d3 q[4], dq[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        q[c] = ld3(y, n0 + c);
        d3 t = ld3(xt, n0 + c);
        dq[c] = {q[c].x - t.x, q[c].y - t.y, q[c].z - t.z};
    }
    double E = 0.0;
    d3 gq[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        gq[c] = {0, 0, 0};
#pragma unroll
        for (int c2 = 0; c2 < 4; ++c2) {
            double m = M[4 * c + c2];
            gq[c].x += m * dq[c2].x; gq[c].y += m * dq[c2].y; gq[c].z += m * dq[c2].z;
        }
        E += 0.5 * dt(dq[c], gq[c]);
    }
    // orthogonality: A[r][col] = q[1 + col].r
    double A[3][3];
#pragma unroll
    for (int cl = 0; cl < 3; ++cl) { A[0][cl] = q[1 + cl].x; A[1][cl] = q[1 + cl].y; A[2][cl] = q[1 + cl].z; }
    double C[3][3], AtA[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            C[i][j] = A[i][0] * A[j][0] + A[i][1] * A[j][1] + A[i][2] * A[j][2] - (i == j ? 1.0 : 0.0);
            AtA[i][j] = A[0][i] * A[0][j] + A[1][i] * A[1][j] + A[2][i] * A[2][j];
        }
    double kv = h2s[bscene[b]] * bkappa[b] * bvol[b];
    double eo = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) eo += C[i][j] * C[i][j];
    E += kv * eo;
    if (part) part[b] = E;
    if (MODE == 0) return;
    // gradient: 4 kv (C A)
#pragma unroll
    for (int cl = 0; cl < 3; ++cl) {
        gq[1 + cl].x += 4.0 * kv * (C[0][0] * A[0][cl] + C[0][1] * A[1][cl] + C[0][2] * A[2][cl]);
        gq[1 + cl].y += 4.0 * kv * (C[1][0] * A[0][cl] + C[1][1] * A[1][cl] + C[1][2] * A[2][cl]);
        gq[1 + cl].z += 4.0 * kv * (C[2][0] * A[0][cl] + C[2][1] * A[1][cl] + C[2][2] * A[2][cl]);
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {   // body nodes are owned by this thread: plain read-modify-write
        d3 o = ld3(g, n0 + c);
        st3(g, n0 + c, {o.x + gq[c].x, o.y + gq[c].y, o.z + gq[c].z});
    }
    if (MODE < 2) return;
    double H[45];   // over vec(A) column-major: index 3*col + row
#pragma unroll
    for (int bcol = 0; bcol < 3; ++bcol)
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int dcol = 0; dcol < 3; ++dcol)
#pragma unroll
                for (int cr_ = 0; cr_ < 3; ++cr_) {
                    int R = 3 * bcol + a, Cc = 3 * dcol + cr_;
                    if (R > Cc) continue;
                    H[pk9(R, Cc)] = 4.0 * kv * ((a == cr_ ? AtA[bcol][dcol] : 0.0) + A[a][dcol] * A[cr_][bcol] + (bcol == dcol ? C[a][cr_] : 0.0));
                }
    if (project) iso::project_ortho(H, A, kv);
    // add the 16 node blocks into the block-CSR values (the body's blocks are
    // touched by no other kernel during assembly)
    const int *sl = bslot + 16 * (size_t)b;
#pragma unroll
    for (int ca = 0; ca < 4; ++ca)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            double *blk = val + 9 * (size_t)sl[4 * ca + cb];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    double v = (i == j) ? M[4 * ca + cb] : 0.0;
                    if (ca >= 1 && cb >= 1) v += H[pk9(3 * (ca - 1) + i, 3 * (cb - 1) + j)];
                    blk[3 * i + j] += v;
                }
        }
}

// ---------------------------------------------------------------------------
// point springs: E = h^2 k/2 |a - b|^2, each side a FEM node, a body point or a
// drive target (the link's target affine state applied to the anchor)
// ---------------------------------------------------------------------------
__device__ __forceinline__ d3 spring_side(int kind, int idx, const double *xb, const double *y, const int *body_node0,
                                          const double *targets)
{
    if (kind == 0) return ld3(y, idx);
    d3 w = {xb[0], xb[1], xb[2]};
    if (kind == 1) {
        int n0 = body_node0[idx];
        return xaffine(ld3(y, n0), ld3(y, n0 + 1), ld3(y, n0 + 2), ld3(y, n0 + 3), w);
    }
    const double *q = targets + 12 * (size_t)idx;
    return xaffine(mk(q[0], q[1], q[2]), mk(q[3], q[4], q[5]), mk(q[6], q[7], q[8]), mk(q[9], q[10], q[11]), w);
}

// Gradient entry code 8 s + 4 side + q of spring s: the force on side a
// (+f) or b (-f), times the side's weight q (1 for a FEM vertex; 1, xb0, xb1,
// xb2 for the 4 nodes of a body point).  The entries, sorted by node once at
// creation, are summed per node by the run sums.
struct ValSpring {
    const double *f, *xa, *xb;
    __device__ void operator()(int code, double *a) const
    {
        const int s = code >> 3, side = (code >> 2) & 1, q = code & 3;
        const double sg = side ? -1.0 : 1.0;
        const double w = q == 0 ? sg : sg * (side ? xb : xa)[3 * (size_t)s + q - 1];
        a[0] = w * f[3 * (size_t)s]; a[1] = w * f[3 * (size_t)s + 1]; a[2] = w * f[3 * (size_t)s + 2];
    }
};

template <int MODE>   // 0 energy, 1 energy+gradient
__global__ void k_spring(int NS, const int *__restrict__ ka, const int *__restrict__ ia, const double *__restrict__ xa,
                         const int *__restrict__ kb, const int *__restrict__ ib, const double *__restrict__ xb,
                         const double *__restrict__ k, const int *__restrict__ sscene, const double *__restrict__ h2s,
                         const double *__restrict__ y, const int *__restrict__ body_node0, const double *__restrict__ targets,
                         double *__restrict__ f, double *__restrict__ part)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= NS) return;
    d3 pa = spring_side(ka[s], ia[s], xa + 3 * (size_t)s, y, body_node0, targets);
    d3 pb = spring_side(kb[s], ib[s], xb + 3 * (size_t)s, y, body_node0, targets);
    d3 d = {pa.x - pb.x, pa.y - pb.y, pa.z - pb.z};
    double kk = h2s[sscene[s]] * k[s];
    if (part) part[s] = 0.5 * kk * dt(d, d);
    if (MODE == 0) return;
    st3(f, s, {kk * d.x, kk * d.y, kk * d.z});
}

// ---------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------
void launch_node_inertia(ipc_ctx *c, const double *y, double *g, double *part)
{
    hipLaunchKernelGGL(k_node_inertia, dim3(blocks_for(c->N)), dim3(BLOCK), 0, c->stream, c->N, y, c->d.xt.p, c->d.mass.p,
                       c->d.node_kind.p, g, part);
}

void launch_fem(ipc_ctx *c, int mode, const double *y, double *g, bool project, double *part, const double *h2s)
{
    Dev &D = c->d;
    int64_t n9 = 9 * (int64_t)c->nnzb;
    if (c->T == 0) {
        if (mode == 2) hipLaunchKernelGGL(k_bsr_assemble, dim3(blocks_for(n9, c->asm_block)), dim3(c->asm_block), 0, c->stream, n9, 1, D.sc_ptr.p,
                                          D.sc_list.p, D.telem.p, D.val_const.p, D.val.p, D.slot_scene.p, c->assemble_only);
        return;
    }
    const int *active = mode >= 1 ? c->assemble_only : nullptr;
    auto args = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(blocks_for(c->T, c->fem_block)), dim3(c->fem_block), 0, c->stream, c->T, D.tv.p, D.Bm.p, D.vol.p, D.tmu.p,
                           D.tlam.p, y, D.tile_scene_tet.p, h2s, D.tgrad.p, D.telem.p, (int)project, part, active);
    };
    int k = mode == 2 ? IPC_K_FEM_HESS : (mode == 0 ? IPC_K_FEM_ENERGY : -1);
    if (k >= 0) prof_begin(c, k);
    if (mode == 0) args(k_fem<0>);
    else if (mode == 1) args(k_fem<1>);
    else args(k_fem<2>);
    if (mode >= 1)
        hipLaunchKernelGGL(k_fem_grad_gather, dim3(blocks_for(c->N, c->grad_block)), dim3(c->grad_block), 0, c->stream, c->N, c->T, D.fadj_ptr.p, D.fadj.p,
                           D.tgrad.p, g, D.node_scene.p, active);
    if (mode == 2)
        hipLaunchKernelGGL(k_bsr_assemble, dim3(blocks_for(n9, c->asm_block)), dim3(c->asm_block), 0, c->stream, n9, c->T, D.sc_ptr.p, D.sc_list.p,
                           D.telem.p, D.val_const.p, D.val.p, D.slot_scene.p, active);
    // algorithmic bytes: tet data in (112), per-tet gradient and upper blocks
    // out and back in (96 and 720, twice), node gradient in and out (48),
    // matrix out and its constant part in (2 x 72 per block)
    if (k >= 0)
        prof_end(c, k, mode == 2 ? (112.0 + 2 * 816.0) * c->TREAL + 48.0 * c->NFEM + 144.0 * c->nnzb : 112.0 * c->TREAL + 24.0 * c->NFEM);
}

// The workgroup sizes of the three kernels of the FEM assembly: each is timed
// alone with 64, 128 and 256 threads (reps launches between HIP events on
// the context's stream, on the current state; the gradient goes to a solver
// scratch vector) and the fastest kept, 256 unless another is more than 3 %
// faster.  The sums do not depend on the size (per thread, or per wavefront
// of 64 consecutive tets), so the choice changes no result.  The matrix
// values are left as const + FEM blocks: the next assembly rewrites them.
void autotune_fem(ipc_ctx *c, int reps)
{
    if (c->T == 0) return;
    Dev &D = c->d;
    hipEvent_t e0, e1;
    IPC_HIP(hipEventCreate(&e0));
    IPC_HIP(hipEventCreate(&e1));
    const int64_t n9 = 9 * (int64_t)c->nnzb;
    const int sizes[3] = {64, 128, 256};
    int *choice[3] = {&c->fem_block, &c->asm_block, &c->grad_block};
    for (int which = 0; which < 3; ++which) {
        double t256 = 1e300, best = 1e300;
        int pick = BLOCK;
        for (int bs : sizes) {
            auto launch = [&] {
                if (which == 0)
                    hipLaunchKernelGGL(k_fem<2>, dim3(blocks_for(c->T, bs)), dim3(bs), 0, c->stream, c->T, D.tv.p, D.Bm.p, D.vol.p,
                                       D.tmu.p, D.tlam.p, D.y.p, D.tile_scene_tet.p, D.h2s.p, D.tgrad.p, D.telem.p, 1, D.part_tet.p,
                                       (const int *)nullptr);
                else if (which == 1)
                    hipLaunchKernelGGL(k_bsr_assemble, dim3(blocks_for(n9, bs)), dim3(bs), 0, c->stream, n9, c->T, D.sc_ptr.p,
                                       D.sc_list.p, D.telem.p, D.val_const.p, D.val.p, D.slot_scene.p, (const int *)nullptr);
                else
                    hipLaunchKernelGGL(k_fem_grad_gather, dim3(blocks_for(c->N, bs)), dim3(bs), 0, c->stream, c->N, c->T, D.fadj_ptr.p,
                                       D.fadj.p, D.tgrad.p, D.v2.p, D.node_scene.p, (const int *)nullptr);
            };
            launch();
            IPC_HIP(hipEventRecord(e0, c->stream));
            for (int k = 0; k < reps; ++k) launch();
            IPC_HIP(hipEventRecord(e1, c->stream));
            IPC_HIP(hipEventSynchronize(e1));
            float ms = 0.0f;
            IPC_HIP(hipEventElapsedTime(&ms, e0, e1));
            const double t = (double)ms / reps;
            if (bs == BLOCK) t256 = t;
            if (t < best) { best = t; pick = bs; }
        }
        *choice[which] = best < 0.97 * t256 ? pick : BLOCK;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
}

void launch_body(ipc_ctx *c, int mode, const double *y, double *g, bool project, double *part, const double *h2s)
{
    if (c->NB == 0) return;
    Dev &D = c->d;
    auto args = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(blocks_for(c->NB, 64)), dim3(64), 0, c->stream, c->NB, D.body_node0.p, D.body_scene.p,
                           D.bM.p, D.bvol.p, D.bkappa.p, h2s, y, D.xt.p, g, D.val.p, D.bslot.p, (int)project, part);
    };
    if (mode == 0) args(k_body<0>);
    else if (mode == 1) args(k_body<1>);
    else args(k_body<2>);
}

void launch_spring(ipc_ctx *c, int mode, const double *y, double *g, double *part, const double *h2s)
{
    if (c->NS == 0) return;
    Dev &D = c->d;
    auto args = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(blocks_for(c->NS)), dim3(BLOCK), 0, c->stream, c->NS, D.sp_ka.p, D.sp_ia.p, D.sp_xa.p,
                           D.sp_kb.p, D.sp_ib.p, D.sp_xb.p, D.sp_k.p, D.sp_scene.p, h2s, y, D.body_node0.p, D.targets.p, D.sp_f.p, part);
    };
    if (mode == 0) {
        args(k_spring<0>);
        return;
    }
    args(k_spring<1>);
    runsum<3>(c, D.n_spg, c->N, D.spg_key.p, D.spg_code.p, ValSpring{D.sp_f.p, D.sp_xa.p, D.sp_xb.p}, EmitAdd3{g});
}

} // namespace ipc
