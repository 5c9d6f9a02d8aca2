// incidence.h -- per-row sums of contact-pair contributions, one wavefront
// per 64 consecutive rows.
//
// The incidence lists (CSR: c_ptr over rows, c_list = pair*4 + slot, c_row =
// row of each entry) are sorted by row and, inside a row, by pair index. A
// wavefront walks the entries of its 64 rows in chunks of 64: every lane
// loads one entry, a segmented inclusive scan keyed by row (fixed shuffle
// order) sums the chunk's entries of each row, and the lane that owns a row
// picks up that row's chunk total from the segment's last lane. A row with
// more than kHeavyRow entries (a coarse indenter's vertices, hundreds of
// incident pairs) is skipped here and summed by a block of its own
// (block_row_sums); the summation order depends only on the lists, so results
// are deterministic.
#pragma once

#include "device_util.h"
#include "ipc_internal.h"

namespace ipcg {

// NC components per entry; val(p, a, c) reads component c of pair p, slot a.
// out[c] += sum over the entries of row r0 + lane (rows >= n contribute 0).
// Every lane of the wavefront must call this with the same r0.
template <int NC, class F>
__device__ __forceinline__ void wave_row_sums(const SceneDev &S, int r0, int lane, F val, double out[NC])
{
    if (r0 >= S.n) return;  // uniform over the wavefront
    int r1 = min(r0 + kWave, S.n);
    int e0 = S.c_ptr[r0], e1 = S.c_ptr[r1];
    int row = r0 + lane;
    int my0 = row < r1 ? S.c_ptr[row] : e1, my1 = row < r1 ? S.c_ptr[row + 1] : e1;
    for (int base = e0; base < e1;) {
        // a heavy row's entries are summed by its own block: jump over them
        int rb = S.c_row[base];
        if (S.hflag[rb]) {
            base = S.c_ptr[rb + 1];
            continue;
        }
        int t = base + lane;
        bool ok = t < e1;
        int key = ok ? S.c_row[t] : INT32_MAX;
        double v[NC];
        if (ok && !S.hflag[key]) {
            int src = S.c_list[t];
            int p = src >> 2, a = src & 3;
#pragma unroll
            for (int c = 0; c < NC; ++c) v[c] = val(p, a, c);
        } else {
#pragma unroll
            for (int c = 0; c < NC; ++c) v[c] = 0.0;
        }
        // segmented inclusive scan (keys are sorted, so segments are contiguous)
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            int ku = __shfl_up(key, o, kWave);
            bool take = lane >= o && ku == key;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                double u = __shfl_up(v[c], o, kWave);
                if (take) v[c] += u;
            }
        }
        // the owner of row r takes the scan value at r's last entry in this chunk
        int last = min(my1, base + kWave) - 1 - base;
        bool mine = my1 > my0 && my0 < base + kWave && my1 > base;
        int srcl = mine ? last : lane;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            double u = __shfl(v[c], srcl, kWave);
            if (mine) out[c] += u;
        }
        base += kWave;
    }
}

// Vector sum over a block of kBlock threads in a fixed order (all threads get it).
template <int NC>
__device__ __forceinline__ void block_sum_vec(double v[NC])
{
    __shared__ double sh[kBlock / kWave][NC];
    int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
#pragma unroll
    for (int c = 0; c < NC; ++c) v[c] = wave_sum(v[c]);
    if (lane == 0)
#pragma unroll
        for (int c = 0; c < NC; ++c) sh[w][c] = v[c];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        double t = 0.0;
        for (int k = 0; k < kBlock / kWave; ++k) t += sh[k][c];
        v[c] = t;
    }
    __syncthreads();
}

// Sum over the entries of one (heavy) row by a whole block: thread t takes
// entries t, t + kBlock, ... in order, then a fixed-order block sum.
template <int NC, class F>
__device__ __forceinline__ void block_row_sums(const SceneDev &S, int row, F val, double out[NC])
{
    int e0 = S.c_ptr[row], e1 = S.c_ptr[row + 1];
#pragma unroll
    for (int c = 0; c < NC; ++c) out[c] = 0.0;
    for (int t = e0 + (int)threadIdx.x; t < e1; t += kBlock) {
        int src = S.c_list[t];
        int p = src >> 2, a = src & 3;
#pragma unroll
        for (int c = 0; c < NC; ++c) out[c] += val(p, a, c);
    }
    block_sum_vec<NC>(out);
}

}  // namespace ipcg
