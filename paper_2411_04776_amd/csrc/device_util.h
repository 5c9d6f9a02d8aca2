// device_util.h -- wavefront/block reductions and small dense helpers for the
// gfx950 kernels. Reductions run in a fixed tree order (64-lane shuffles,
// then one wave over the per-wave results) so every result is a function of
// the input order only: two runs, or the same scene alone and in a batch,
// produce bit-identical sums.
#pragma once
#include <hip/hip_runtime.h>

#include "ipc_internal.h"

namespace ipcg {

// Global-memory views of device pointers. The arrays of a scene's view are
// reached through generic pointers, so plain accesses compile to flat
// instructions, which also count against the LDS counter: every LDS wait and
// block barrier after them waits for them too. Through these views they are
// global loads and stores, which the latency-bound PCG update kernel keeps in
// flight across its LDS work and barriers.
template <class T>
using gptr = __attribute__((address_space(1))) T *;
template <class T>
__device__ __forceinline__ gptr<T> glob(T *p)
{
    return (gptr<T>)p;
}

__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_down(v, o, kWave);
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
    for (int o = kWave / 2; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, kWave));
    return v;
}
__device__ __forceinline__ double wave_min(double v)
{
    for (int o = kWave / 2; o > 0; o >>= 1) v = fmin(v, __shfl_down(v, o, kWave));
    return v;
}
__device__ __forceinline__ int wave_isum(int v)
{
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_down(v, o, kWave);
    return v;
}

// Block-wide reductions; blockDim.x must be a multiple of 64 and <= 1024.
// The result is valid in thread 0 (and broadcast through shared memory to
// all threads by the *_all variants).
template <int OP>
__device__ __forceinline__ double wave_op(double v)
{
    return OP == 0 ? wave_sum(v) : (OP == 1 ? wave_max(v) : wave_min(v));
}

template <int OP>
__device__ double block_reduce_all(double v, double ident)
{
    __shared__ double sh[16];
    __shared__ double result;
    int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    int nw = (blockDim.x + kWave - 1) / kWave;
    v = wave_op<OP>(v);
    if (lane == 0) sh[w] = v;
    __syncthreads();
    if (w == 0) {
        double t = lane < nw ? sh[lane] : ident;
        t = wave_op<OP>(t);
        if (lane == 0) result = t;
    }
    __syncthreads();
    double r = result;
    __syncthreads();
    return r;
}

__device__ inline double block_sum_all(double v) { return block_reduce_all<0>(v, 0.0); }
__device__ inline double block_max_all(double v) { return block_reduce_all<1>(v, -INFINITY); }
__device__ inline double block_min_all(double v) { return block_reduce_all<2>(v, INFINITY); }

// Sum of partials[0..n) in a fixed order; identical in every block.
__device__ inline double reduce_partials(const double *partials, int n)
{
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) acc += partials[i];
    return block_sum_all(acc);
}

// The same sum computed by one wavefront alone, without block barriers: lane
// l adds partials l, l + 64, ... in order, then a fixed shuffle tree. Every
// wavefront of every block gets the identical value.
__device__ inline double wave_reduce_partials(const double *partials, int n)
{
    int lane = threadIdx.x & (kWave - 1);
    double acc = 0.0;
    for (int i = lane; i < n; i += kWave) acc += partials[i];
    acc = wave_sum(acc);
    return __shfl(acc, 0, kWave);
}

// wave_reduce_partials with eight loads in flight per lane: the same
// additions in the same order (bit-identical), one memory round trip per
// 512 partials instead of one per 64 (a scene of 128k vertices has ~2000).
__device__ inline double wave_reduce_partials_u8(const double *partials, int n)
{
    constexpr int kU = 8;
    int lane = threadIdx.x & (kWave - 1);
    double acc = 0.0;
    for (int base = lane; base < n; base += kU * kWave) {
        double b[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            int i = base + u * kWave;
            b[u] = i < n ? partials[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kU; ++u)
            if (base + u * kWave < n) acc += b[u];
    }
    acc = wave_sum(acc);
    return __shfl(acc, 0, kWave);
}

// The same sum in two parts, for a kernel that can issue the loads before
// other dependent loads: wave_partials_load fetches a lane's first U entries,
// wave_partials_sum adds them and the rest (four loads ahead of the adds) in
// the same order, so the value is bit-identical to wave_reduce_partials. The
// PCG update kernel keeps the plain loop, which measured faster there.
template <int U>
__device__ __forceinline__ void wave_partials_load(const double *partials, int n, double (&a)[U])
{
    int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int u = 0; u < U; ++u) {
        int i = lane + u * kWave;
        a[u] = i < n ? partials[i] : 0.0;
    }
}

template <int U>
__device__ __forceinline__ double wave_partials_sum(const double *partials, int n, const double (&a)[U])
{
    constexpr int kU = 4;
    int lane = threadIdx.x & (kWave - 1);
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u)
        if (lane + u * kWave < n) acc += a[u];
    for (int base = lane + U * kWave; base < n; base += kU * kWave) {
        double b[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            int i = base + u * kWave;
            b[u] = i < n ? partials[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kU; ++u)
            if (base + u * kWave < n) acc += b[u];
    }
    acc = wave_sum(acc);
    return __shfl(acc, 0, kWave);
}

// ---- compensated (double-double style) sums for energies ----------------
struct CSum {
    double s, c;
};
__device__ __forceinline__ CSum csum_add(CSum a, CSum b)
{
    // TwoSum of the leading parts; errors accumulate in c
    double s = a.s + b.s;
    double bp = s - a.s;
    double e = (a.s - (s - bp)) + (b.s - bp);
    CSum r;
    r.s = s;
    r.c = a.c + b.c + e;
    return r;
}
__device__ __forceinline__ CSum wave_csum(CSum v)
{
    for (int o = kWave / 2; o > 0; o >>= 1) {
        CSum w;
        w.s = __shfl_down(v.s, o, kWave);
        w.c = __shfl_down(v.c, o, kWave);
        v = csum_add(v, w);
    }
    return v;
}
__device__ inline CSum block_csum(CSum v)
{
    __shared__ double shs[16], shc[16];
    __shared__ CSum result;
    int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    int nw = (blockDim.x + kWave - 1) / kWave;
    v = wave_csum(v);
    if (lane == 0) {
        shs[w] = v.s;
        shc[w] = v.c;
    }
    __syncthreads();
    if (w == 0) {
        CSum t;
        t.s = lane < nw ? shs[lane] : 0.0;
        t.c = lane < nw ? shc[lane] : 0.0;
        t = wave_csum(t);
        if (lane == 0) result = t;
    }
    __syncthreads();
    CSum r = result;
    __syncthreads();
    return r;
}

// ---- 3x3 helpers (row-major) ----------------------------------------------
__device__ __forceinline__ double det3(const double *M)
{
    return M[0] * (M[4] * M[8] - M[5] * M[7]) - M[1] * (M[3] * M[8] - M[5] * M[6]) +
           M[2] * (M[3] * M[7] - M[4] * M[6]);
}
// inverse by the adjugate; returns the determinant
__device__ __forceinline__ double inverse3(const double *M, double *O)
{
    double c00 = M[4] * M[8] - M[5] * M[7];
    double c01 = M[5] * M[6] - M[3] * M[8];
    double c02 = M[3] * M[7] - M[4] * M[6];
    double d = M[0] * c00 + M[1] * c01 + M[2] * c02;
    double id = 1.0 / d;
    O[0] = c00 * id;
    O[1] = (M[2] * M[7] - M[1] * M[8]) * id;
    O[2] = (M[1] * M[5] - M[2] * M[4]) * id;
    O[3] = c01 * id;
    O[4] = (M[0] * M[8] - M[2] * M[6]) * id;
    O[5] = (M[2] * M[3] - M[0] * M[5]) * id;
    O[6] = c02 * id;
    O[7] = (M[1] * M[6] - M[0] * M[7]) * id;
    O[8] = (M[0] * M[4] - M[1] * M[3]) * id;
    return d;
}

}  // namespace ipcg
