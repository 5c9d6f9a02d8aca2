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

// Rows of more than kRowInline entries are listed by their owner thread and
// summed by teams of kTeam lanes: team t of the block takes the listed rows
// t, t + teams, ...; lane u of a team adds the row's entries e0 + u,
// e0 + u + kTeam, ... in order (four entries' loads in flight per pass), then
// a fixed xor tree over the team's lanes (every lane of the team ends with the
// same value: the adds commute). A dense contact patch gives rows of 10-50
// entries; one thread would walk them one dependent load pair at a time.
constexpr int kRowInline = 2;
constexpr int kTeam = 8;
static_assert(kTeam == 8 && kBlock % kTeam == 0, "the team sum is an xor tree over eight lanes");

struct RowList {
    int32_t e0[kMasCapM], e1[kMasCapM], dst[kMasCapM];
    int32_t count;
};

// Light row: at most kRowInline entries summed by the calling thread (loads
// issued together), or else listed for the teams. Returns true if listed.
template <class F>
__device__ __forceinline__ bool row_sum_or_list(const SceneDev &S, int row, int dst, F val, double out[3], RowList &rl)
{
    const auto cp = glob(S.c_ptr);
    const auto cl = glob(S.c_list);
    const int e0 = cp[row], e1 = cp[row + 1];
    if (e1 - e0 > kRowInline) {
        int slot = atomicAdd(&rl.count, 1);
        rl.e0[slot] = e0;
        rl.e1[slot] = e1;
        rl.dst[slot] = dst;
        return true;
    }
    int src[kRowInline];
#pragma unroll
    for (int k = 0; k < kRowInline; ++k) src[k] = e0 + k < e1 ? cl[e0 + k] : -1;
#pragma unroll
    for (int k = 0; k < kRowInline; ++k)
        if (src[k] >= 0)
#pragma unroll
            for (int c = 0; c < 3; ++c) out[c] += val(src[k] >> 2, src[k] & 3, c);
    return false;
}

// The teams' pass over a block's list (between two block barriers); put(dst,
// sums) runs on each team's first lane.
template <class F, class P>
__device__ __forceinline__ void team_row_sums(const SceneDev &S, const RowList &rl, F val, P put)
{
    const int tid = (int)threadIdx.x, u = tid % kTeam, teams = (int)blockDim.x / kTeam;
    const int n = rl.count;
    const auto cl = glob(S.c_list);
    for (int h = tid / kTeam; h < n; h += teams) {
        const int e0 = rl.e0[h], e1 = rl.e1[h];
        double acc[3] = {0.0, 0.0, 0.0};
        for (int base = e0 + u; base < e1; base += 4 * kTeam) {
            int src[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) src[k] = base + k * kTeam < e1 ? cl[base + k * kTeam] : -1;
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (src[k] >= 0)
#pragma unroll
                    for (int c = 0; c < 3; ++c) acc[c] += val(src[k] >> 2, src[k] & 3, c);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            acc[c] += __shfl_xor(acc[c], 4, kTeam);
            acc[c] += __shfl_xor(acc[c], 2, kTeam);
            acc[c] += __shfl_xor(acc[c], 1, kTeam);
        }
        if (u == 0) put(rl.dst[h], acc);
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
