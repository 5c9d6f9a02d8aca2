// incidence.h -- per-row sums of contact-pair contributions.
//
// The incidence lists (CSR: c_ptr over rows, c_list = pair*4 + slot) are
// sorted by row and, inside a row, by pair index, so every row sum below runs
// in a fixed order and results are deterministic. A light row (at most
// kHeavyRow entries) is summed by one thread; a heavy row (a coarse indenter's
// vertex with hundreds of incident pairs, or a gel vertex under a dense
// contact patch) by a whole block of its own, listed in heavy_rows.
#pragma once

#include "device_util.h"
#include "ipc_internal.h"

namespace ipcg {

// NC components per entry; val(p, a, c) reads component c of pair p, slot a.
// out[c] += the sum over the entries of a light row, in list order, by one
// thread (at most kHeavyRow independent entry loads). U entries are unrolled
// (loads in flight against registers held).
template <int NC, class F, int U = 4>
__device__ __forceinline__ void thread_row_sums(const SceneDev &S, int row, F val, double out[NC])
{
    int e0 = S.c_ptr[row], e1 = S.c_ptr[row + 1];
#pragma unroll U
    for (int t = e0; t < e1; ++t) {
        int src = S.c_list[t];
        int p = src >> 2, a = src & 3;
#pragma unroll
        for (int c = 0; c < NC; ++c) out[c] += val(p, a, c);
    }
}

// Vector sum over the block (blockDim.x a multiple of 64, at most kBlock) in
// a fixed order; every thread gets the result.
template <int NC>
__device__ __forceinline__ void block_sum_vec(double v[NC])
{
    __shared__ double sh[kBlock / kWave][NC];
    int lane = threadIdx.x % kWave, w = threadIdx.x / kWave, nw = blockDim.x / kWave;
#pragma unroll
    for (int c = 0; c < NC; ++c) v[c] = wave_sum(v[c]);
    if (nw == 1) {
#pragma unroll
        for (int c = 0; c < NC; ++c) v[c] = __shfl(v[c], 0, kWave);
        return;
    }
    if (lane == 0)
#pragma unroll
        for (int c = 0; c < NC; ++c) sh[w][c] = v[c];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        double t = 0.0;
        for (int k = 0; k < nw; ++k) t += sh[k][c];
        v[c] = t;
    }
    __syncthreads();
}

// Sum over the entries of one (heavy) row by one wavefront: lane l takes
// entries l, l + 64, ... in order, then a fixed shuffle tree; every lane gets
// the result. No block barrier, so a block's wavefronts sum different rows at
// once.
template <int NC, class F>
__device__ __forceinline__ void wave_row_sums(const SceneDev &S, int row, F val, double out[NC])
{
    int e0 = S.c_ptr[row], e1 = S.c_ptr[row + 1];
    const int lane = (int)(threadIdx.x & (kWave - 1));
#pragma unroll
    for (int c = 0; c < NC; ++c) out[c] = 0.0;
    for (int t = e0 + lane; t < e1; t += kWave) {
        int src = S.c_list[t];
        int p = src >> 2, a = src & 3;
#pragma unroll
        for (int c = 0; c < NC; ++c) out[c] += val(p, a, c);
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        out[c] = wave_sum(out[c]);
        out[c] = __shfl(out[c], 0, kWave);
    }
}

// Sum over the entries of one (heavy) row by a whole block: thread t takes
// entries t, t + blockDim, ... in order, then a fixed-order block sum.
template <int NC, class F>
__device__ __forceinline__ void block_row_sums(const SceneDev &S, int row, F val, double out[NC])
{
    int e0 = S.c_ptr[row], e1 = S.c_ptr[row + 1];
#pragma unroll
    for (int c = 0; c < NC; ++c) out[c] = 0.0;
    for (int t = e0 + (int)threadIdx.x; t < e1; t += (int)blockDim.x) {
        int src = S.c_list[t];
        int p = src >> 2, a = src & 3;
#pragma unroll
        for (int c = 0; c < NC; ++c) out[c] += val(p, a, c);
    }
    block_sum_vec<NC>(out);
}

}  // namespace ipcg
