// Dual-mesh mapping (Sec. III-D, Eq. (6)-(7)): W = S^(L) ... S^(1), the L-level
// Loop subdivision of the coarse simulation mesh as one sparse matrix, built
// on the host at creation; X^f = W X^c for many frames per launch.
//
// The application is HBM-bound: W is read once per launch (12 B per
// nonzero) and every frame writes 24 B per fine vertex, while the coarse
// frames (24 B per coarse vertex) stay in L2.  One thread per fine vertex
// keeps its row of W in registers and loops over the frames, so consecutive
// threads write consecutive fine vertices of a frame.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <mutex>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/ipc.h"
#include "../../include/ipc_dualmesh.h"

struct ipc_dualmesh {
    hipStream_t stream = nullptr;
    int n_coarse = 0, n_fine = 0, max_row = 0;
    int64_t nnz = 0;
    std::vector<int> row_ptr, col, tri_fine;
    std::vector<double> val;
    // per block of DM_ROWS rows: its distinct columns (blk_cols from
    // blk_off[b]) and, per nonzero, the column's place in its block's list
    std::vector<int> blk_off, blk_cols, lcol;
    int max_block = 0;
    uint64_t id = 0;   // unique per handle: names the W that the no-alloc path last staged
    int *d_row = nullptr, *d_col = nullptr, *d_lcol = nullptr, *d_boff = nullptr, *d_bcols = nullptr;
    double *d_val = nullptr;
    std::string err;
    ~ipc_dualmesh()
    {
        if (d_row) (void)hipFree(d_row);
        if (d_col) (void)hipFree(d_col);
        if (d_lcol) (void)hipFree(d_lcol);
        if (d_boff) (void)hipFree(d_boff);
        if (d_bcols) (void)hipFree(d_bcols);
        if (d_val) (void)hipFree(d_val);
    }
};

namespace {

std::string g_dm_create_error;

constexpr int DM_ROWS = 256;     // fine rows per workgroup of the staged kernel
constexpr int DM_STAGE = 1024;   // coarse vertices a block may stage in LDS (24 KiB)

struct Invalid : std::runtime_error {
    using std::runtime_error::runtime_error;
};

struct Csr {
    std::vector<int> ptr{0}, col;
    std::vector<double> val;
    int rows() const { return (int)ptr.size() - 1; }
};

double loop_beta(int n)
{
    const double c = 0.375 + 0.25 * std::cos(2.0 * M_PI / n);
    return (0.625 - c * c) / n;
}

// append one row given as (column, weight) pairs: columns ascending, repeats summed
void push_row(Csr &S, std::vector<std::pair<int, double>> &e)
{
    std::sort(e.begin(), e.end(), [](const std::pair<int, double> &a, const std::pair<int, double> &b) { return a.first < b.first; });
    for (size_t k = 0; k < e.size(); ++k) {
        if (k && e[k].first == S.col.back()) S.val.back() += e[k].second;
        else { S.col.push_back(e[k].first); S.val.push_back(e[k].second); }
    }
    S.ptr.push_back((int)S.col.size());
}

// One level: the subdivision matrix S (old vertices, then one row per edge,
// over the old vertices) and the level's triangles.
void loop_level(int n_old, const std::vector<int> &tri, Csr &S, std::vector<int> &tri_out)
{
    const size_t m = tri.size() / 3;
    std::unordered_map<uint64_t, int> eid;
    eid.reserve(3 * m);
    std::vector<int> ea, eb, o0, o1;
    auto key = [](int u, int w) { return ((uint64_t)std::min(u, w) << 32) | (uint64_t)std::max(u, w); };
    std::vector<int> tri_edge(3 * m);
    for (size_t t = 0; t < m; ++t) {
        const int v[3] = {tri[3 * t], tri[3 * t + 1], tri[3 * t + 2]};
        for (int s = 0; s < 3; ++s) {
            const int u = v[s], w = v[(s + 1) % 3], o = v[(s + 2) % 3];
            auto it = eid.find(key(u, w));
            int e;
            if (it == eid.end()) {
                e = (int)ea.size();
                eid.emplace(key(u, w), e);
                ea.push_back(u); eb.push_back(w); o0.push_back(o); o1.push_back(-1);
            } else {
                e = it->second;
                if (o1[e] >= 0) throw Invalid("an edge is shared by more than two triangles");
                o1[e] = o;
            }
            tri_edge[3 * t + s] = e;
        }
    }
    const int ne = (int)ea.size();
    if ((int64_t)n_old + ne > INT32_MAX) throw Invalid("too many fine vertices");
    std::vector<std::vector<int>> nb(n_old), bn(n_old);
    for (int e = 0; e < ne; ++e) {
        nb[ea[e]].push_back(eb[e]);
        nb[eb[e]].push_back(ea[e]);
        if (o1[e] < 0) { bn[ea[e]].push_back(eb[e]); bn[eb[e]].push_back(ea[e]); }
    }
    S = Csr();
    std::vector<std::pair<int, double>> row;
    for (int i = 0; i < n_old; ++i) {
        row.clear();
        if (bn[i].size() > 2) throw Invalid("a vertex lies on more than two boundary edges");
        if (bn[i].size() == 2) {
            row = {{i, 0.75}, {bn[i][0], 0.125}, {bn[i][1], 0.125}};
        } else if (!nb[i].empty()) {
            const int n = (int)nb[i].size();
            const double beta = loop_beta(n);
            row.push_back({i, 1.0 - n * beta});
            for (int j : nb[i]) row.push_back({j, beta});
        } else {
            row.push_back({i, 1.0});
        }
        push_row(S, row);
    }
    for (int e = 0; e < ne; ++e) {
        row.clear();
        if (o1[e] >= 0) row = {{ea[e], 0.375}, {eb[e], 0.375}, {o0[e], 0.125}, {o1[e], 0.125}};
        else row = {{ea[e], 0.5}, {eb[e], 0.5}};
        push_row(S, row);
    }
    tri_out.resize(12 * m);
    for (size_t t = 0; t < m; ++t) {
        const int a = tri[3 * t], b = tri[3 * t + 1], c = tri[3 * t + 2];
        const int ab = n_old + tri_edge[3 * t], bc = n_old + tri_edge[3 * t + 1], ca = n_old + tri_edge[3 * t + 2];
        const int q[12] = {a, ab, ca, b, bc, ab, c, ca, bc, ab, bc, ca};
        for (int k = 0; k < 12; ++k) tri_out[12 * t + k] = q[k];
    }
}

// C = A B (A: rows over B's rows; B: rows over n_cols columns); columns
// ascending per row
Csr multiply(const Csr &A, const Csr &B, int n_cols)
{
    Csr C;
    std::vector<double> acc(n_cols, 0.0);
    std::vector<char> on(n_cols, 0);
    std::vector<int> touched;
    for (int r = 0; r < A.rows(); ++r) {
        touched.clear();
        for (int k = A.ptr[r]; k < A.ptr[r + 1]; ++k) {
            const int i = A.col[k];
            const double a = A.val[k];
            for (int q = B.ptr[i]; q < B.ptr[i + 1]; ++q) {
                const int j = B.col[q];
                if (!on[j]) { on[j] = 1; touched.push_back(j); }
                acc[j] += a * B.val[q];
            }
        }
        std::sort(touched.begin(), touched.end());
        for (int j : touched) { C.col.push_back(j); C.val.push_back(acc[j]); acc[j] = 0.0; on[j] = 0; }
        if (C.col.size() > (size_t)INT32_MAX) throw Invalid("too many nonzeros");
        C.ptr.push_back((int)C.col.size());
    }
    return C;
}

// A fine vertex's 3 doubles, written with non-temporal stores: the output
// (a gigabyte at 100 frames) is written once and never read back by the
// kernel, so it should not displace the coarse frames and W from the caches
// (measured 448 -> 378 us per launch on the cylinder's render mesh).
__device__ __forceinline__ void st_stream(double *o, double x, double y, double z)
{
    __builtin_nontemporal_store(x, o);
    __builtin_nontemporal_store(y, o + 1);
    __builtin_nontemporal_store(z, o + 2);
}

template <int K>
__global__ void __launch_bounds__(256) k_dm_apply(int nf, int nc, int frames, const int *__restrict__ rp, const int *__restrict__ col,
                                                  const double *__restrict__ val, const double *__restrict__ xc,
                                                  double *__restrict__ xf)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nf) return;
    const int k0 = rp[r], n = rp[r + 1] - k0;
    if constexpr (K > 0) {
        int c[K];
        double w[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const bool in = k < n;
            c[k] = in ? col[k0 + k] : 0;
            w[k] = in ? val[k0 + k] : 0.0;
        }
        for (int f = 0; f < frames; ++f) {
            const double *x = xc + (size_t)f * nc * 3;
            double ax = 0.0, ay = 0.0, az = 0.0;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (k < n) {
                    const double *p = x + 3 * (size_t)c[k];
                    ax += w[k] * p[0];
                    ay += w[k] * p[1];
                    az += w[k] * p[2];
                }
            }
            double *o = xf + ((size_t)f * nf + r) * 3;
            st_stream(o, ax, ay, az);
        }
    } else {
        for (int f = 0; f < frames; ++f) {
            const double *x = xc + (size_t)f * nc * 3;
            double ax = 0.0, ay = 0.0, az = 0.0;
            for (int k = 0; k < n; ++k) {
                const double wk = val[k0 + k];
                const double *p = x + 3 * (size_t)col[k0 + k];
                ax += wk * p[0];
                ay += wk * p[1];
                az += wk * p[2];
            }
            double *o = xf + ((size_t)f * nf + r) * 3;
            st_stream(o, ax, ay, az);
        }
    }
}

// Workgroup b takes rows [DM_ROWS b, DM_ROWS b + DM_ROWS): per frame it
// first copies the positions of the block's distinct coarse vertices into
// LDS (each fetched once per block instead of once per use: a block of 256
// consecutive fine rows touches ~100 coarse vertices), then every thread
// sums its row (kept in registers with columns renumbered into the block's
// list) from LDS and writes its fine vertex.
template <int K>
__global__ void __launch_bounds__(DM_ROWS) k_dm_apply_lds(int nf, int nc, int frames, const int *__restrict__ rp,
                                                          const int *__restrict__ lcol, const double *__restrict__ val,
                                                          const int *__restrict__ boff, const int *__restrict__ bcols,
                                                          const double *__restrict__ xc, double *__restrict__ xf)
{
    constexpr int PER = DM_STAGE / DM_ROWS;   // staged vertices per thread, at most
    __shared__ double sx[3 * DM_STAGE];
    const int t = threadIdx.x, r = blockIdx.x * DM_ROWS + t;
    const int u0 = boff[blockIdx.x], U = boff[blockIdx.x + 1] - u0;
    int src[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) src[q] = t + q * DM_ROWS < U ? bcols[u0 + t + q * DM_ROWS] : -1;
    int c[K];
    double w[K];
    int n = 0;
    if (r < nf) {
        const int k0 = rp[r];
        n = rp[r + 1] - k0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const bool in = k < n;
            c[k] = in ? lcol[k0 + k] : 0;
            w[k] = in ? val[k0 + k] : 0.0;
        }
    }
    // the next frame's staged positions are loaded into registers while this
    // frame is summed and stored, so the gather's latency overlaps the work
    double pf[PER][3];
    auto fetch = [&](int f) {
        const double *x = xc + (size_t)f * nc * 3;
#pragma unroll
        for (int q = 0; q < PER; ++q)
            if (src[q] >= 0) {
                pf[q][0] = x[3 * (size_t)src[q]];
                pf[q][1] = x[3 * (size_t)src[q] + 1];
                pf[q][2] = x[3 * (size_t)src[q] + 2];
            }
    };
    if (frames > 0) fetch(0);
    for (int f = 0; f < frames; ++f) {
        __syncthreads();   // the previous frame's reads of sx are done
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            if (src[q] >= 0) {
                const int u = t + q * DM_ROWS;
                sx[3 * u] = pf[q][0];
                sx[3 * u + 1] = pf[q][1];
                sx[3 * u + 2] = pf[q][2];
            }
        }
        if (f + 1 < frames) fetch(f + 1);
        __syncthreads();
        if (r < nf) {
            double ax = 0.0, ay = 0.0, az = 0.0;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (k < n) {
                    ax += w[k] * sx[3 * c[k]];
                    ay += w[k] * sx[3 * c[k] + 1];
                    az += w[k] * sx[3 * c[k] + 2];
                }
            }
            double *o = xf + ((size_t)f * nf + r) * 3;
            st_stream(o, ax, ay, az);
        }
    }
}

// the staged kernel serves every W whose blocks fit in LDS and rows in 16 registers
bool staged(const ipc_dualmesh *m) { return m->max_block <= DM_STAGE && m->max_row <= 16; }

hipError_t upload(ipc_dualmesh *m)
{
    if (m->d_row) return hipSuccess;
    hipError_t e = hipMalloc(&m->d_row, sizeof(int) * m->row_ptr.size());
    if (e == hipSuccess) e = hipMalloc(&m->d_col, sizeof(int) * std::max<size_t>(m->col.size(), 1));
    if (e == hipSuccess) e = hipMalloc(&m->d_val, sizeof(double) * std::max<size_t>(m->val.size(), 1));
    if (e == hipSuccess) e = hipMemcpyAsync(m->d_row, m->row_ptr.data(), sizeof(int) * m->row_ptr.size(), hipMemcpyHostToDevice, m->stream);
    if (e == hipSuccess && !m->col.empty())
        e = hipMemcpyAsync(m->d_col, m->col.data(), sizeof(int) * m->col.size(), hipMemcpyHostToDevice, m->stream);
    if (e == hipSuccess && !m->val.empty())
        e = hipMemcpyAsync(m->d_val, m->val.data(), sizeof(double) * m->val.size(), hipMemcpyHostToDevice, m->stream);
    if (e == hipSuccess && staged(m)) {
        e = hipMalloc(&m->d_lcol, sizeof(int) * std::max<size_t>(m->lcol.size(), 1));
        if (e == hipSuccess) e = hipMalloc(&m->d_boff, sizeof(int) * m->blk_off.size());
        if (e == hipSuccess) e = hipMalloc(&m->d_bcols, sizeof(int) * std::max<size_t>(m->blk_cols.size(), 1));
        if (e == hipSuccess && !m->lcol.empty())
            e = hipMemcpyAsync(m->d_lcol, m->lcol.data(), sizeof(int) * m->lcol.size(), hipMemcpyHostToDevice, m->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(m->d_boff, m->blk_off.data(), sizeof(int) * m->blk_off.size(), hipMemcpyHostToDevice, m->stream);
        if (e == hipSuccess && !m->blk_cols.empty())
            e = hipMemcpyAsync(m->d_bcols, m->blk_cols.data(), sizeof(int) * m->blk_cols.size(), hipMemcpyHostToDevice, m->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
    return e;
}

// W on the device: CSR arrays, and for the staged kernel the renumbered
// columns and the per-block coarse-vertex lists
struct DevW {
    const int *row, *col, *lcol, *boff, *bcols;
    const double *val;
};

hipError_t launch(ipc_dualmesh *m, const DevW &w, const double *xc, double *xf, int frames)
{
    const dim3 grid((m->n_fine + 255) / 256), blk(256);
    const int R = m->max_row;
    if (w.lcol) {
        hipLaunchKernelGGL(k_dm_apply_lds<16>, dim3((m->n_fine + DM_ROWS - 1) / DM_ROWS), dim3(DM_ROWS), 0, m->stream, m->n_fine,
                           m->n_coarse, frames, w.row, w.lcol, w.val, w.boff, w.bcols, xc, xf);
        return hipGetLastError();
    }
#define IPC_DM(KK) hipLaunchKernelGGL(k_dm_apply<KK>, grid, blk, 0, m->stream, m->n_fine, m->n_coarse, frames, w.row, w.col, \
                                      w.val, xc, xf)
    if (R <= 8) IPC_DM(8);
    else if (R <= 16) IPC_DM(16);
    else if (R <= 32) IPC_DM(32);
    else if (R <= 48) IPC_DM(48);
    else if (R <= 64) IPC_DM(64);
    else IPC_DM(0);
#undef IPC_DM
    return hipGetLastError();
}

DevW owned(const ipc_dualmesh *m) { return {m->d_row, m->d_col, m->d_lcol, m->d_boff, m->d_bcols, m->d_val}; }

// ---- the variant that allocates nothing ------------------------------------
// W is staged in a file-scope device array of fixed size instead of memory
// the library allocates.  Every GPU holds its own copy of the array, at its
// own address, taken once per device with hipGetSymbolAddress; the host-side
// name of the array is not a device address and is never passed to a kernel
// or a copy.  The array keeps the W of the last call on that GPU: a call with
// the same handle does not copy it again.
constexpr size_t DM_SCRATCH_BYTES = 16u << 20;
static __device__ __align__(256) unsigned char scratch[DM_SCRATCH_BYTES];
constexpr int DM_MAX_DEVICES = 64;
struct ScratchSlot {
    unsigned char *ptr = nullptr;   // this device's address of the array
    uint64_t holds = 0;             // id of the handle whose W it holds (0: none)
};
std::mutex g_scratch_mu;
ScratchSlot g_scratch[DM_MAX_DEVICES];
uint64_t g_dm_next_id = 1;

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// byte offsets of W's arrays in the array (0 for an unused one); the total
struct ScratchLayout {
    size_t row = 0, col = 0, lcol = 0, val = 0, boff = 0, bcols = 0, total = 0;
};
ScratchLayout scratch_layout(const ipc_dualmesh *m)
{
    ScratchLayout L;
    size_t o = 0;
    L.row = o; o += align256(sizeof(int) * m->row_ptr.size());
    L.val = o; o += align256(sizeof(double) * std::max<size_t>(m->val.size(), 1));
    if (staged(m)) {
        L.lcol = o; o += align256(sizeof(int) * std::max<size_t>(m->lcol.size(), 1));
        L.boff = o; o += align256(sizeof(int) * m->blk_off.size());
        L.bcols = o; o += align256(sizeof(int) * std::max<size_t>(m->blk_cols.size(), 1));
    } else {
        L.col = o; o += align256(sizeof(int) * std::max<size_t>(m->col.size(), 1));
    }
    L.total = o;
    return L;
}

} // namespace

extern "C" int ipc_dualmesh_create(const int32_t *tri_host, int32_t n_tri, int32_t n_vert, int32_t levels, void *hip_stream,
                                   ipc_dualmesh **out)
{
    if (!out) return IPC_E_INVALID;
    *out = nullptr;
    try {
        if (!tri_host || n_tri < 1 || n_vert < 1) throw Invalid("need at least one triangle and one vertex");
        if (levels < 0 || levels > 6) throw Invalid("levels must lie in [0, 6]");
        if ((int64_t)n_tri << (2 * levels) > INT32_MAX / 3) throw Invalid("too many fine triangles");
        std::vector<int> tri(tri_host, tri_host + 3 * (size_t)n_tri);
        for (int t = 0; t < n_tri; ++t) {
            const int a = tri[3 * t], b = tri[3 * t + 1], c = tri[3 * t + 2];
            if (a < 0 || b < 0 || c < 0 || a >= n_vert || b >= n_vert || c >= n_vert) throw Invalid("vertex index out of range");
            if (a == b || b == c || c == a) throw Invalid("a triangle repeats a vertex");
        }
        auto *m = new ipc_dualmesh;
        m->stream = (hipStream_t)hip_stream;
        {
            std::lock_guard<std::mutex> lock(g_scratch_mu);
            m->id = g_dm_next_id++;
        }
        // W = identity, then one level at a time: W <- S W
        Csr W;
        for (int i = 0; i < n_vert; ++i) { W.col.push_back(i); W.val.push_back(1.0); W.ptr.push_back(i + 1); }
        int n = n_vert;
        try {
            for (int l = 0; l < levels; ++l) {
                Csr S;
                std::vector<int> tri_next;
                loop_level(n, tri, S, tri_next);
                W = multiply(S, W, n_vert);
                n = S.rows();
                tri.swap(tri_next);
            }
        } catch (...) {
            delete m;
            throw;
        }
        m->n_coarse = n_vert;
        m->n_fine = n;
        m->row_ptr = std::move(W.ptr);
        m->col = std::move(W.col);
        m->val = std::move(W.val);
        m->nnz = (int64_t)m->col.size();
        for (int r = 0; r < n; ++r) m->max_row = std::max(m->max_row, m->row_ptr[r + 1] - m->row_ptr[r]);
        m->tri_fine = std::move(tri);
        // per block of rows: distinct columns and the nonzeros' places among them
        m->lcol.resize(m->col.size());
        m->blk_off.push_back(0);
        std::vector<int> place(n_vert, -1);
        for (int b0 = 0; b0 < n; b0 += DM_ROWS) {
            const int b1 = std::min(n, b0 + DM_ROWS), first = (int)m->blk_cols.size();
            std::vector<int> cols(m->col.begin() + m->row_ptr[b0], m->col.begin() + m->row_ptr[b1]);
            std::sort(cols.begin(), cols.end());
            cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
            for (size_t u = 0; u < cols.size(); ++u) { place[cols[u]] = (int)u; m->blk_cols.push_back(cols[u]); }
            for (int k = m->row_ptr[b0]; k < m->row_ptr[b1]; ++k) m->lcol[k] = place[m->col[k]];
            for (int j : cols) place[j] = -1;
            m->max_block = std::max(m->max_block, (int)cols.size());
            m->blk_off.push_back((int)m->blk_cols.size());
            (void)first;
        }
        *out = m;
        return IPC_OK;
    } catch (const Invalid &e) {
        g_dm_create_error = e.what();
        return IPC_E_INVALID;
    } catch (const std::exception &e) {
        g_dm_create_error = e.what();
        return IPC_E_DEVICE;
    }
}

extern "C" void ipc_dualmesh_destroy(ipc_dualmesh *m) { delete m; }

extern "C" const char *ipc_dualmesh_last_error(const ipc_dualmesh *m) { return m ? m->err.c_str() : g_dm_create_error.c_str(); }

extern "C" int ipc_dualmesh_query(const ipc_dualmesh *m, int what, int64_t *v)
{
    if (!m || !v) return IPC_E_INVALID;
    switch (what) {
    case IPC_DM_NCOARSE: *v = m->n_coarse; return IPC_OK;
    case IPC_DM_NFINE: *v = m->n_fine; return IPC_OK;
    case IPC_DM_NTRI: *v = (int64_t)(m->tri_fine.size() / 3); return IPC_OK;
    case IPC_DM_NNZ: *v = m->nnz; return IPC_OK;
    case IPC_DM_MAXROW: *v = m->max_row; return IPC_OK;
    }
    return IPC_E_INVALID;
}

extern "C" int ipc_dualmesh_fine_tris(const ipc_dualmesh *m, int32_t *tri_host)
{
    if (!m || !tri_host) return IPC_E_INVALID;
    std::copy(m->tri_fine.begin(), m->tri_fine.end(), tri_host);
    return IPC_OK;
}

extern "C" int ipc_dualmesh_weights(const ipc_dualmesh *m, int32_t *row_ptr, int32_t *col, double *val)
{
    if (!m) return IPC_E_INVALID;
    if (row_ptr) std::copy(m->row_ptr.begin(), m->row_ptr.end(), row_ptr);
    if (col) std::copy(m->col.begin(), m->col.end(), col);
    if (val) std::copy(m->val.begin(), m->val.end(), val);
    return IPC_OK;
}

extern "C" int ipc_dualmesh_apply(ipc_dualmesh *m, const double *xc_dev, double *xf_dev, int32_t n_frames)
{
    if (!m) return IPC_E_INVALID;
    if (!xc_dev || !xf_dev || n_frames < 1) { m->err = "need device arrays and at least one frame"; return IPC_E_INVALID; }
    hipError_t e = upload(m);
    if (e == hipSuccess) e = launch(m, owned(m), xc_dev, xf_dev, n_frames);
    if (e != hipSuccess) { m->err = std::string("HIP: ") + hipGetErrorString(e); return IPC_E_DEVICE; }
    return IPC_OK;
}

extern "C" int ipc_dualmesh_apply_noalloc(ipc_dualmesh *m, const double *xc_dev, double *xf_dev, int32_t n_frames)
{
    if (!m) return IPC_E_INVALID;
    if (!xc_dev || !xf_dev || n_frames < 1) { m->err = "need device arrays and at least one frame"; return IPC_E_INVALID; }
    const ScratchLayout L = scratch_layout(m);
    if (L.total > DM_SCRATCH_BYTES) {
        m->err = "W needs " + std::to_string(L.total) + " bytes of staging; the no-alloc path holds at most " +
                 std::to_string(DM_SCRATCH_BYTES);
        return IPC_E_CAPACITY;
    }
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess && (dev < 0 || dev >= DM_MAX_DEVICES)) { m->err = "device ordinal out of range"; return IPC_E_INVALID; }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    ScratchSlot &S = g_scratch[dev];
    if (e == hipSuccess && !S.ptr) e = hipGetSymbolAddress((void **)&S.ptr, HIP_SYMBOL(scratch));   // once per device
    if (e == hipSuccess && S.holds != m->id) {
        auto put = [&](size_t off, const void *src, size_t bytes) {
            if (e == hipSuccess && bytes) e = hipMemcpyAsync(S.ptr + off, src, bytes, hipMemcpyHostToDevice, m->stream);
        };
        S.holds = 0;
        put(L.row, m->row_ptr.data(), sizeof(int) * m->row_ptr.size());
        put(L.val, m->val.data(), sizeof(double) * m->val.size());
        if (staged(m)) {
            put(L.lcol, m->lcol.data(), sizeof(int) * m->lcol.size());
            put(L.boff, m->blk_off.data(), sizeof(int) * m->blk_off.size());
            put(L.bcols, m->blk_cols.data(), sizeof(int) * m->blk_cols.size());
        } else {
            put(L.col, m->col.data(), sizeof(int) * m->col.size());
        }
        if (e == hipSuccess) S.holds = m->id;
    }
    if (e == hipSuccess) {
        const bool st = staged(m);
        DevW w{(const int *)(S.ptr + L.row), st ? nullptr : (const int *)(S.ptr + L.col), st ? (const int *)(S.ptr + L.lcol) : nullptr,
               st ? (const int *)(S.ptr + L.boff) : nullptr, st ? (const int *)(S.ptr + L.bcols) : nullptr, (const double *)(S.ptr + L.val)};
        e = launch(m, w, xc_dev, xf_dev, n_frames);
    }
    if (e != hipSuccess) { m->err = std::string("HIP: ") + hipGetErrorString(e); return IPC_E_DEVICE; }
    return IPC_OK;
}

extern "C" int ipc_dualmesh_time(ipc_dualmesh *m, const double *xc_dev, double *xf_dev, int32_t n_frames, int32_t reps,
                                 double *avg_us, double *bytes)
{
    if (!m) return IPC_E_INVALID;
    if (!xc_dev || !xf_dev || n_frames < 1 || reps < 1 || !avg_us) { m->err = "invalid timing arguments"; return IPC_E_INVALID; }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = upload(m);
    if (e == hipSuccess) e = launch(m, owned(m), xc_dev, xf_dev, n_frames);   // warm
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipEventRecord(e0, m->stream);
    for (int k = 0; k < reps && e == hipSuccess; ++k) e = launch(m, owned(m), xc_dev, xf_dev, n_frames);
    if (e == hipSuccess) e = hipEventRecord(e1, m->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) { m->err = std::string("HIP: ") + hipGetErrorString(e); return IPC_E_DEVICE; }
    *avg_us = 1e3 * ms / reps;
    if (bytes)
        *bytes = 12.0 * (double)m->nnz + 4.0 * (m->n_fine + 1.0) + 24.0 * (double)n_frames * ((double)m->n_coarse + m->n_fine);
    return IPC_OK;
}
