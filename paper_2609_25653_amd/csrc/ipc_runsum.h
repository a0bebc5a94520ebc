// Deterministic sums over runs of equal keys.
//
// Many contributions (per-pair gradients, per-pair 3x3 blocks, spring forces)
// add into few destinations (a contact vertex, a matrix block, a node).  A
// list of entries (key = destination, code = which contribution) sorted
// stably by key puts every destination's contributions in one contiguous
// run, in an order that depends only on the inputs.  The run sums are then
// formed in a fixed order and written by exactly one thread each, so the
// result is the same bit for bit on every run, unlike floating-point atomics
// whose order of arrival varies.
//
//  k_runsum: one thread per entry.  A segmented inclusive scan over each
//    wavefront's lanes (a run's lanes are contiguous, so "same key as the
//    lane d below" marks the lanes to add) sums every run piece inside the
//    wavefront.  A run that starts and ends inside one wavefront is emitted
//    by its last lane.  A run that crosses a wavefront boundary leaves its
//    piece in that wavefront's first-run or last-run slot.
//  k_runsum_join: one thread per wavefront whose first run started in an
//    earlier wavefront and ends in this one: it adds the pieces from the
//    starting wavefront on, in wavefront order, and emits the sum.
//
// Val(code, a) writes the W doubles of one contribution; Emit(key, a) adds a
// run's W sums into their destination.  Keys < 0 or >= nkeys are skipped.
#pragma once
#include <hip/hip_runtime.h>

#include "ipc_internal.h"

namespace ipc {

// generic values and destinations
struct ValVec3 {   // the 3 doubles at v[3 code]
    const double *v;
    __device__ void operator()(int code, double *a) const
    {
        a[0] = v[3 * (size_t)code]; a[1] = v[3 * (size_t)code + 1]; a[2] = v[3 * (size_t)code + 2];
    }
};
struct EmitAdd3 {  // out[3 key + q] += a[q]
    double *out;
    __device__ void operator()(int key, const double *a) const
    {
        out[3 * (size_t)key] += a[0]; out[3 * (size_t)key + 1] += a[1]; out[3 * (size_t)key + 2] += a[2];
    }
};
struct EmitAdd9 {  // out[9 key + q] += a[q]: a 3x3 block
    double *out;
    __device__ void operator()(int key, const double *a) const
    {
#pragma unroll
        for (int q = 0; q < 9; ++q) out[9 * (size_t)key + q] += a[q];
    }
};

template <int W, class Val, class Emit>
__global__ void __launch_bounds__(256) k_runsum(int m, int nkeys, const int *__restrict__ key, const int *__restrict__ code,
                                                Val val, Emit emit, double *__restrict__ wfirst, double *__restrict__ wlast)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x, lane = threadIdx.x & 63, wave = t >> 6;
    const int k = t < m ? key[t] : -1;
    const bool on = k >= 0 && k < nkeys;
    double a[W];
#pragma unroll
    for (int q = 0; q < W; ++q) a[q] = 0.0;
    if (on) val(code[t], a);
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int kd = __shfl_up(k, d, 64);
        double o[W];
#pragma unroll
        for (int q = 0; q < W; ++q) o[q] = __shfl_up(a[q], d, 64);
        if (lane >= d && kd == k) {
#pragma unroll
            for (int q = 0; q < W; ++q) a[q] += o[q];
        }
    }
    int kp = __shfl_up(k, 1, 64), kn = __shfl_down(k, 1, 64);
    if (lane == 63) kn = t + 1 < m ? key[t + 1] : -1;
    const bool head = lane == 0 || kp != k;
    const unsigned long long hm = __ballot(head);
    const unsigned long long below = lane == 63 ? hm : (hm & ((2ull << lane) - 1ull));
    const int start = 63 - __clzll((long long)below);   // lane of this run piece's first entry
    const bool tail = lane == 63 || kn != k;
    if (!on || !tail) return;
    const int t0 = wave * 64;
    const bool cross_in = start == 0 && t0 > 0 && key[t0 - 1] == k;
    const bool cross_out = lane == 63 && kn == k;
    if (!cross_in && !cross_out) {
        emit(k, a);
        return;
    }
    if (start == 0) {
#pragma unroll
        for (int q = 0; q < W; ++q) wfirst[(size_t)wave * W + q] = a[q];
    }
    if (lane == 63) {
#pragma unroll
        for (int q = 0; q < W; ++q) wlast[(size_t)wave * W + q] = a[q];
    }
}

template <int W, class Emit>
__global__ void __launch_bounds__(256) k_runsum_join(int m, int nkeys, const int *__restrict__ key, Emit emit,
                                                     const double *__restrict__ wfirst, const double *__restrict__ wlast)
{
    const int w = blockIdx.x * blockDim.x + threadIdx.x, nw = (m + 63) / 64;
    if (w <= 0 || w >= nw) return;
    const int t0 = 64 * w, k = key[t0];
    if (k < 0 || k >= nkeys || key[t0 - 1] != k) return;   // this wavefront's first run starts here
    const int tl = min(t0 + 63, m - 1);
    if (key[tl] == k && tl + 1 < m && key[tl + 1] == k) return;   // it goes on: a later wavefront completes it
    int w0 = w - 1;
    while (w0 > 0 && key[64 * w0 - 1] == k) --w0;
    double a[W];
#pragma unroll
    for (int q = 0; q < W; ++q) a[q] = wlast[(size_t)w0 * W + q];
    for (int v = w0 + 1; v < w; ++v)
#pragma unroll
        for (int q = 0; q < W; ++q) a[q] += wlast[(size_t)v * W + q];
#pragma unroll
    for (int q = 0; q < W; ++q) a[q] += wfirst[(size_t)w * W + q];
    emit(k, a);
}

// Run sums of the m sorted entries (key, code): per-wavefront pieces in the
// context's scratch, then the joins.  Stream-ordered on the context's stream.
template <int W, class Val, class Emit>
void runsum(ipc_ctx *c, int64_t m, int nkeys, const int *key, const int *code, Val val, Emit emit)
{
    if (m <= 0) return;
    const int64_t nw = (m + 63) / 64;
    c->d.rs_first.alloc((size_t)W * nw + 1);
    c->d.rs_last.alloc((size_t)W * nw + 1);
    hipLaunchKernelGGL((k_runsum<W, Val, Emit>), dim3(blocks_for(m)), dim3(BLOCK), 0, c->stream, (int)m, nkeys, key, code, val, emit,
                       c->d.rs_first.p, c->d.rs_last.p);
    if (nw > 1)
        hipLaunchKernelGGL((k_runsum_join<W, Emit>), dim3(blocks_for(nw)), dim3(BLOCK), 0, c->stream, (int)m, nkeys, key, emit,
                           c->d.rs_first.p, c->d.rs_last.p);
}

} // namespace ipc
