// k_solver.hip -- block-Jacobi PCG, SpMV, vector kernels, scans.
//
// PCG solves H p = -g from p = 0 and stops when the preconditioned residual
// r^T M^-1 r reaches pcg_tol^2 times its initial value. Each iteration is two
// kernels with all scalars kept on the device:
//   A(it): every block reduces the r.z partials of the previous iterations
//          in a fixed order (so all blocks agree bit for bit), decides the
//          stop, forms d = z + beta d_prev for its rows and for the columns it
//          gathers, applies H (BELL blocks + contact incidence lists) and
//          writes q = H d and the d.q partials;
//   B(it): every block reduces the d.q partials, alpha = rz / dq, then
//          p += alpha d, r -= alpha q, z = M^-1 r and the r.z partials.
// The host launches chunks of iterations and reads the done flag once per
// chunk; a finished solve turns the remaining launches into no-ops.
#include <algorithm>

#include "device_util.h"
#include "ipc_internal.h"

namespace ipcg {

struct PcgState {
    int32_t done;
    int32_t iters;
    double stop;
};

// q_row = sum over the row's BELL blocks and contact entries of H_ij * dv_j,
// with dv_j = z_j + beta * dold_j (beta_on = 0: dv = z)
__device__ __forceinline__ void spmv_row(int row, const int32_t *__restrict__ slice_ptr,
                                         const int32_t *__restrict__ bcol, const double *__restrict__ bval,
                                         const int32_t *__restrict__ c_ptr, const int32_t *__restrict__ c_list,
                                         const int32_t *__restrict__ act_v, const double *__restrict__ act_H,
                                         int64_t act_cap, const double *__restrict__ z,
                                         const double *__restrict__ dold, double beta, bool beta_on,
                                         double out[3])
{
    int sl = row / kSlice, lane = row % kSlice;
    int s0 = slice_ptr[sl], s1 = slice_ptr[sl + 1];
    double y0 = 0.0, y1 = 0.0, y2 = 0.0;
    for (int slot = s0; slot < s1; ++slot) {
        int64_t base = (int64_t)slot * kSlice + lane;
        int col = bcol[base];
        if (col < 0) break;
        const double *A = bval + (int64_t)slot * 9 * kSlice + lane;
        double v0 = z[3 * col], v1 = z[3 * col + 1], v2 = z[3 * col + 2];
        if (beta_on) {
            v0 += beta * dold[3 * col];
            v1 += beta * dold[3 * col + 1];
            v2 += beta * dold[3 * col + 2];
        }
        y0 += A[0 * kSlice] * v0 + A[1 * kSlice] * v1 + A[2 * kSlice] * v2;
        y1 += A[3 * kSlice] * v0 + A[4 * kSlice] * v1 + A[5 * kSlice] * v2;
        y2 += A[6 * kSlice] * v0 + A[7 * kSlice] * v1 + A[8 * kSlice] * v2;
    }
    for (int t = c_ptr[row]; t < c_ptr[row + 1]; ++t) {
        int src = c_list[t], p = src >> 2, a = src & 3;
        for (int b = 0; b < 4; ++b) {
            if (b == a) continue;  // the diagonal block lives in the BELL diagonal
            int vb = act_v[(int64_t)b * act_cap + p];
            double v0 = z[3 * vb], v1 = z[3 * vb + 1], v2 = z[3 * vb + 2];
            if (beta_on) {
                v0 += beta * dold[3 * vb];
                v1 += beta * dold[3 * vb + 1];
                v2 += beta * dold[3 * vb + 2];
            }
            const double *H = act_H + p;
            int r0 = 3 * a;
            y0 += H[(int64_t)((r0 + 0) * 12 + 3 * b + 0) * act_cap] * v0 +
                  H[(int64_t)((r0 + 0) * 12 + 3 * b + 1) * act_cap] * v1 +
                  H[(int64_t)((r0 + 0) * 12 + 3 * b + 2) * act_cap] * v2;
            y1 += H[(int64_t)((r0 + 1) * 12 + 3 * b + 0) * act_cap] * v0 +
                  H[(int64_t)((r0 + 1) * 12 + 3 * b + 1) * act_cap] * v1 +
                  H[(int64_t)((r0 + 1) * 12 + 3 * b + 2) * act_cap] * v2;
            y2 += H[(int64_t)((r0 + 2) * 12 + 3 * b + 0) * act_cap] * v0 +
                  H[(int64_t)((r0 + 2) * 12 + 3 * b + 1) * act_cap] * v1 +
                  H[(int64_t)((r0 + 2) * 12 + 3 * b + 2) * act_cap] * v2;
        }
    }
    out[0] = y0;
    out[1] = y1;
    out[2] = y2;
}

__global__ void __launch_bounds__(kBlock) k_pcg_init(int n, const double *__restrict__ grad,
                                                      const double *__restrict__ Minv, double *__restrict__ r,
                                                      double *__restrict__ z, double *__restrict__ sol,
                                                      double *__restrict__ part_rz0, PcgState *st)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    double rz = 0.0;
    if (i < n) {
        double ri[3], zi[3];
        for (int c = 0; c < 3; ++c) ri[c] = -grad[3 * i + c];
        for (int a = 0; a < 3; ++a)
            zi[a] = Minv[9 * i + 3 * a] * ri[0] + Minv[9 * i + 3 * a + 1] * ri[1] + Minv[9 * i + 3 * a + 2] * ri[2];
        for (int c = 0; c < 3; ++c) {
            r[3 * i + c] = ri[c];
            z[3 * i + c] = zi[c];
            sol[3 * i + c] = 0.0;
            rz += ri[c] * zi[c];
        }
    }
    rz = block_sum_all(rz);
    if (threadIdx.x == 0) part_rz0[blockIdx.x] = rz;
    if (i == 0) {
        st->done = 0;
        st->iters = 0;
        st->stop = 0.0;
    }
}

// PCG kernel A: four lanes per matrix row, one 64-row BELL slice per block.
// Lane q of a row sums slots q, q+4, ...; the four partial products are
// combined with lane shuffles in a fixed order. Lane 0 of the row adds the
// contact incidence terms and writes d and q.
constexpr int kLanesPerRow = 4;

__device__ __forceinline__ void spmv_row_part(int row, int part, const int32_t *__restrict__ slice_ptr,
                                              const int32_t *__restrict__ bcol, const double *__restrict__ bval,
                                              const double *__restrict__ z, const double *__restrict__ dold,
                                              double beta, bool beta_on, double y[3])
{
    int sl = row / kSlice, lane = row % kSlice;
    int s0 = slice_ptr[sl], s1 = slice_ptr[sl + 1];
    double y0 = 0.0, y1 = 0.0, y2 = 0.0;
    for (int slot = s0 + part; slot < s1; slot += kLanesPerRow) {
        int64_t base = (int64_t)slot * kSlice + lane;
        int col = bcol[base];
        if (col < 0) break;
        const double *A = bval + (int64_t)slot * 9 * kSlice + lane;
        double v0 = z[3 * col], v1 = z[3 * col + 1], v2 = z[3 * col + 2];
        if (beta_on) {
            v0 += beta * dold[3 * col];
            v1 += beta * dold[3 * col + 1];
            v2 += beta * dold[3 * col + 2];
        }
        y0 += A[0 * kSlice] * v0 + A[1 * kSlice] * v1 + A[2 * kSlice] * v2;
        y1 += A[3 * kSlice] * v0 + A[4 * kSlice] * v1 + A[5 * kSlice] * v2;
        y2 += A[6 * kSlice] * v0 + A[7 * kSlice] * v1 + A[8 * kSlice] * v2;
    }
    y[0] = y0;
    y[1] = y1;
    y[2] = y2;
}

__device__ __forceinline__ void contact_row(int row, const int32_t *__restrict__ c_ptr, const int32_t *__restrict__ c_list,
                                            const int32_t *__restrict__ act_v, const double *__restrict__ act_H,
                                            int64_t act_cap, const double *__restrict__ z,
                                            const double *__restrict__ dold, double beta, bool beta_on, double y[3])
{
    for (int t = c_ptr[row]; t < c_ptr[row + 1]; ++t) {
        int src = c_list[t], p = src >> 2, a = src & 3;
        for (int b = 0; b < 4; ++b) {
            if (b == a) continue;
            int vb = act_v[(int64_t)b * act_cap + p];
            double v[3] = {z[3 * vb], z[3 * vb + 1], z[3 * vb + 2]};
            if (beta_on)
                for (int c = 0; c < 3; ++c) v[c] += beta * dold[3 * vb + c];
            for (int i = 0; i < 3; ++i) {
                const double *H = act_H + (int64_t)((3 * a + i) * 12 + 3 * b) * act_cap + p;
                y[i] += H[0] * v[0] + H[act_cap] * v[1] + H[2 * act_cap] * v[2];
            }
        }
    }
}

__global__ void __launch_bounds__(kBlock) k_pcg_A(
    int it, int n, int nbB, double tol2, const int32_t *__restrict__ slice_ptr, const int32_t *__restrict__ bcol,
    const double *__restrict__ bval, const int32_t *__restrict__ c_ptr, const int32_t *__restrict__ c_list,
    const int32_t *__restrict__ act_v, const double *__restrict__ act_H, int64_t act_cap,
    const double *__restrict__ z, const double *__restrict__ dold, double *__restrict__ dnew,
    double *__restrict__ q, double *__restrict__ part_dq, const double *__restrict__ part_rz, PcgState *st)
{
    if (st->done) return;
    double beta = 0.0;
    if (it == 1) {
        double rz0 = reduce_partials(part_rz, nbB);
        if (!(rz0 > 0.0)) {
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                st->done = 1;
                st->iters = 0;
            }
            return;
        }
        if (blockIdx.x == 0 && threadIdx.x == 0) st->stop = tol2 * rz0;
    } else {
        double rz_cur = reduce_partials(part_rz + (size_t)((it - 1) & 1) * nbB, nbB);
        if (rz_cur <= st->stop) {
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                st->done = 1;
                st->iters = it - 1;
            }
            return;
        }
        double rz_prev = reduce_partials(part_rz + (size_t)(it & 1) * nbB, nbB);
        beta = rz_cur / rz_prev;
    }
    // block = one slice of 64 rows; lanes (4r .. 4r+3) of a wavefront share row r
    int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    int row = blockIdx.x * kSlice + wave * (kWave / kLanesPerRow) + lane / kLanesPerRow;
    int part = lane % kLanesPerRow;
    double y[3] = {0.0, 0.0, 0.0};
    bool live = row < n;
    if (live) spmv_row_part(row, part, slice_ptr, bcol, bval, z, dold, beta, it > 1, y);
    for (int c = 0; c < 3; ++c) {
        y[c] += __shfl_xor(y[c], 1, kWave);
        y[c] += __shfl_xor(y[c], 2, kWave);
    }
    double dq = 0.0;
    if (live && part == 0) {
        contact_row(row, c_ptr, c_list, act_v, act_H, act_cap, z, dold, beta, it > 1, y);
        for (int c = 0; c < 3; ++c) {
            double dv = it > 1 ? z[3 * row + c] + beta * dold[3 * row + c] : z[3 * row + c];
            dnew[3 * row + c] = dv;
            q[3 * row + c] = y[c];
            dq += dv * y[c];
        }
    }
    dq = block_sum_all(dq);
    if (threadIdx.x == 0) part_dq[blockIdx.x] = dq;
}

__global__ void __launch_bounds__(kBlock) k_pcg_B(int it, int n, int nbA, int nb, const double *__restrict__ q,
                                                   const double *__restrict__ dcur, const double *__restrict__ Minv,
                                                   double *__restrict__ sol, double *__restrict__ r,
                                                   double *__restrict__ z, const double *__restrict__ part_dq,
                                                   double *__restrict__ part_rz, PcgState *st)
{
    if (st->done) return;
    double dq = reduce_partials(part_dq, nbA);
    double rz_prev = reduce_partials(part_rz + (size_t)((it - 1) & 1) * nb, nb);
    double alpha = rz_prev / dq;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    double rz = 0.0;
    if (i < n) {
        double ri[3];
        for (int c = 0; c < 3; ++c) {
            sol[3 * i + c] += alpha * dcur[3 * i + c];
            ri[c] = r[3 * i + c] - alpha * q[3 * i + c];
            r[3 * i + c] = ri[c];
        }
        for (int a = 0; a < 3; ++a) {
            double za = Minv[9 * i + 3 * a] * ri[0] + Minv[9 * i + 3 * a + 1] * ri[1] + Minv[9 * i + 3 * a + 2] * ri[2];
            z[3 * i + a] = za;
            rz += ri[a] * za;
        }
    }
    rz = block_sum_all(rz);
    if (threadIdx.x == 0) part_rz[(size_t)(it & 1) * nb + blockIdx.x] = rz;
}

__global__ void k_spmv(int n, const int32_t *__restrict__ slice_ptr, const int32_t *__restrict__ bcol,
                       const double *__restrict__ bval, const int32_t *__restrict__ c_ptr,
                       const int32_t *__restrict__ c_list, const int32_t *__restrict__ act_v,
                       const double *__restrict__ act_H, int64_t act_cap, const double *__restrict__ v,
                       double *__restrict__ y)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double o[3];
    spmv_row(i, slice_ptr, bcol, bval, c_ptr, c_list, act_v, act_H, act_cap, v, nullptr, 0.0, false, o);
    for (int c = 0; c < 3; ++c) y[3 * i + c] = o[c];
}

// max |p| over free DOFs
__global__ void k_pinf(int n, const double *__restrict__ p, const uint8_t *__restrict__ fixed,
                       double *__restrict__ part)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    double v = 0.0;
    if (i < n && !fixed[i]) v = fmax(fabs(p[3 * i]), fmax(fabs(p[3 * i + 1]), fabs(p[3 * i + 2])));
    v = block_max_all(v);
    if (threadIdx.x == 0) part[blockIdx.x] = v;
}

__global__ void k_final_max(int nb, const double *__restrict__ part, double *out)
{
    double v = -INFINITY;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) v = fmax(v, part[i]);
    v = block_max_all(v);
    if (threadIdx.x == 0) *out = v;
}

// x_out = x + alpha p (one rounding per component, as the line search defines)
__global__ void k_trial(int m3, const double *__restrict__ x, const double *__restrict__ p, double alpha,
                        double *__restrict__ out)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m3) out[i] = __dadd_rn(x[i], __dmul_rn(alpha, p[i]));
}

// Step start: keep x^t, inertial predictor for free gel vertices, indenter
// targets from the pose.
__global__ void k_begin_step(int n, int n_gel, const double *__restrict__ x, const double *__restrict__ v,
                             const uint8_t *__restrict__ fixed, const double *__restrict__ Yloc, Pose P, double h,
                             double gx, double gy, double gz, double *__restrict__ xt, double *__restrict__ xtilde,
                             double *__restrict__ yhat)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double g[3] = {gx, gy, gz};
    for (int c = 0; c < 3; ++c) xt[3 * i + c] = x[3 * i + c];
    if (i < n_gel) {
        for (int c = 0; c < 3; ++c) {
            double xv = x[3 * i + c];
            xtilde[3 * i + c] = fixed[i] ? xv : xv + h * v[3 * i + c] + h * h * g[c];
            yhat[3 * i + c] = xv;
        }
    } else {
        const double *y = Yloc + 3 * (i - n_gel);
        for (int c = 0; c < 3; ++c) {
            yhat[3 * i + c] = P.m[c * 4 + 0] * y[0] + P.m[c * 4 + 1] * y[1] + P.m[c * 4 + 2] * y[2] + P.m[c * 4 + 3];
            xtilde[3 * i + c] = x[3 * i + c];
        }
    }
}

__global__ void k_end_step(int m3, const double *__restrict__ x, const double *__restrict__ xt, double inv_h,
                           double *__restrict__ v)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m3) v[i] = (x[i] - xt[i]) * inv_h;
}

__global__ void k_target_lag(int n, int n_gel, const double *__restrict__ x, const double *__restrict__ yhat,
                             double *__restrict__ part)
{
    int i = n_gel + blockIdx.x * blockDim.x + threadIdx.x;
    double v = 0.0;
    if (i < n) {
        double d0 = x[3 * i] - yhat[3 * i], d1 = x[3 * i + 1] - yhat[3 * i + 1], d2 = x[3 * i + 2] - yhat[3 * i + 2];
        v = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    }
    v = block_max_all(v);
    if (threadIdx.x == 0) part[blockIdx.x] = v;
}

__global__ void k_gather_surface(int ns, const int32_t *__restrict__ ids, const double *__restrict__ x,
                                 double *__restrict__ out)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ns) return;
    int v = ids[i];
    out[3 * i] = x[3 * v];
    out[3 * i + 1] = x[3 * v + 1];
    out[3 * i + 2] = x[3 * v + 2];
}

// per-block sums of gel vertex coordinates, then a fixed-order final sum
__global__ void k_mean_part(int n_gel, const double *__restrict__ x, double *__restrict__ part)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    for (int c = 0; c < 3; ++c) {
        double v = i < n_gel ? x[3 * i + c] : 0.0;
        v = block_sum_all(v);
        if (threadIdx.x == 0) part[3 * blockIdx.x + c] = v;
    }
}

__global__ void k_mean_final(int nb, int n_gel, double *__restrict__ part, double *__restrict__ out)
{
    for (int c = 0; c < 3; ++c) {
        double acc = 0.0;
        for (int i = threadIdx.x; i < nb; i += blockDim.x) acc += part[3 * i + c];
        acc = block_sum_all(acc);
        if (threadIdx.x == 0) out[c] = acc / (double)n_gel;
    }
}

// ---- exclusive scan of int32 (three passes) ------------------------------
constexpr int kScanItems = 4;
constexpr int kScanTile = kBlock * kScanItems;

__device__ int block_exclusive_scan(int v, int *total)
{
    __shared__ int sh[kBlock / 64];
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int incl = v;
    for (int o = 1; o < 64; o <<= 1) {
        int t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    if (lane == 63) sh[w] = incl;
    __syncthreads();
    int woff = 0, tot = 0;
    for (int k = 0; k < kBlock / 64; ++k) {
        if (k < w) woff += sh[k];
        tot += sh[k];
    }
    __syncthreads();
    *total = tot;
    return woff + incl - v;
}

__global__ void k_scan_tiles(int n, const int32_t *__restrict__ in, int32_t *__restrict__ tile_sums)
{
    int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    int s = 0;
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) s += in[base + k];
    int tot;
    block_exclusive_scan(s, &tot);
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = tot;
}

__global__ void k_scan_top(int nt, int32_t *__restrict__ tile_sums, int32_t *__restrict__ total)
{
    int carry = 0;
    for (int base = 0; base < nt; base += kBlock) {
        int i = base + threadIdx.x;
        int v = i < nt ? tile_sums[i] : 0;
        int tot;
        int ex = block_exclusive_scan(v, &tot);
        if (i < nt) tile_sums[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ void k_scan_apply(int n, const int32_t *__restrict__ in, const int32_t *__restrict__ tile_off,
                             int32_t *__restrict__ out)
{
    int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    int vals[kScanItems];
    int s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        vals[k] = (base + k < n) ? in[base + k] : 0;
        s += vals[k];
    }
    int tot;
    int ex = block_exclusive_scan(s, &tot) + tile_off[blockIdx.x];
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) out[base + k] = ex;
        ex += vals[k];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == kBlock - 1) out[n] = ex;
}

void ensure_iscratch(Scene &s, size_t n)
{
    if (s.i_scratch_n >= n) return;
    if (s.i_scratch) dfree(s, s.i_scratch);
    size_t want = n < 1024 ? 1024 : n * 2;
    s.i_scratch = dalloc<int32_t>(s, want);
    s.i_scratch_n = want;
}

// out must hold n + 1 entries (out[n] = total); total_dev gets the total too.
void exclusive_scan(Scene &s, const int32_t *in, int32_t *out, int n, int32_t *total_dev)
{
    int nt = (n + kScanTile - 1) / kScanTile;
    if (nt == 0) nt = 1;
    ensure_iscratch(s, (size_t)nt + 1);
    hipLaunchKernelGGL(k_scan_tiles, dim3(nt), dim3(kBlock), 0, s.stream, n, in, s.i_scratch);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kBlock), 0, s.stream, nt, s.i_scratch, total_dev);
    hipLaunchKernelGGL(k_scan_apply, dim3(nt), dim3(kBlock), 0, s.stream, n, in, s.i_scratch, out);
}

// ---- launchers --------------------------------------------------------------

void launch_begin_step(Scene &s, const Pose &pose)
{
    hipLaunchKernelGGL(k_begin_step, dim3(nblocks(s.n)), dim3(kBlock), 0, s.stream, s.n, s.n_gel, s.x, s.v, s.fixed,
                       s.Yloc, pose, s.prm.dt, s.prm.grav[0], s.prm.grav[1], s.prm.grav[2], s.xt, s.xtilde, s.yhat);
}

void launch_end_step(Scene &s)
{
    hipLaunchKernelGGL(k_end_step, dim3(nblocks(3 * s.n)), dim3(kBlock), 0, s.stream, 3 * s.n, s.x, s.xt,
                       1.0 / s.prm.dt, s.v);
}

void launch_trial(Scene &s, const double *x, const double *p, double alpha, double *out)
{
    hipLaunchKernelGGL(k_trial, dim3(nblocks(3 * s.n)), dim3(kBlock), 0, s.stream, 3 * s.n, x, p, alpha, out);
}

void launch_hess_apply(Scene &s, const double *v, double *y)
{
    hipLaunchKernelGGL(k_spmv, dim3(nblocks(s.n)), dim3(kBlock), 0, s.stream, s.n, s.slice_ptr, s.bcol, s.bval,
                       s.c_ptr, s.c_list, s.act_v, s.act_H, s.act_cap, v, y);
}

void launch_gather_surface(Scene &s, double *dst, hipStream_t strm)
{
    int ns = (int)s.h_surf_verts.size();
    hipLaunchKernelGGL(k_gather_surface, dim3(nblocks(ns)), dim3(kBlock), 0, strm, ns, s.surf_verts, s.x, dst);
}

double *run_gel_mean(Scene &s, hipStream_t strm)
{
    int nb = nblocks(s.n_gel);
    hipLaunchKernelGGL(k_mean_part, dim3(nb), dim3(kBlock), 0, strm, s.n_gel, s.x, s.mean_part);
    double *out = s.mean_part + 3 * (size_t)nb;
    hipLaunchKernelGGL(k_mean_final, dim3(1), dim3(kBlock), 0, strm, nb, s.n_gel, s.mean_part, out);
    return out;
}

double run_pinf(Scene &s)
{
    int nb = nblocks(s.n);
    hipLaunchKernelGGL(k_pinf, dim3(nb), dim3(kBlock), 0, s.stream, s.n, s.sol, s.fixed, s.red_scratch);
    hipLaunchKernelGGL(k_final_max, dim3(1), dim3(kBlock), 0, s.stream, nb, s.red_scratch, s.red_scratch + nb);
    IPC_HIP(hipMemcpyAsync(&s.hb->value, s.red_scratch + nb, sizeof(double), hipMemcpyDeviceToHost, s.stream));
    IPC_HIP(hipStreamSynchronize(s.stream));
    return s.hb->value;
}

double run_target_lag(Scene &s)
{
    if (s.n_ind == 0) return 0.0;
    int nb = nblocks(s.n_ind);
    hipLaunchKernelGGL(k_target_lag, dim3(nb), dim3(kBlock), 0, s.stream, s.n, s.n_gel, s.x, s.yhat, s.red_scratch);
    hipLaunchKernelGGL(k_final_max, dim3(1), dim3(kBlock), 0, s.stream, nb, s.red_scratch, s.red_scratch + nb);
    IPC_HIP(hipMemcpyAsync(&s.hb->value, s.red_scratch + nb, sizeof(double), hipMemcpyDeviceToHost, s.stream));
    IPC_HIP(hipStreamSynchronize(s.stream));
    return s.hb->value;
}

int run_pcg(Scene &s, int *hit_cap)
{
    int n = s.n, nbB = nblocks(n), nbA = s.n_slices;
    PcgState *st = reinterpret_cast<PcgState *>(s.pcg_state);
    double *part_dq = s.pcg_part, *part_rz = s.pcg_part + nbA;
    double tol2 = s.prm.pcg_tol * s.prm.pcg_tol;
    int maxit = s.prm.pcg_max_iter > 0 ? s.prm.pcg_max_iter : 30 * n;
    hipLaunchKernelGGL(k_pcg_init, dim3(nbB), dim3(kBlock), 0, s.stream, n, s.grad, s.Minv, s.r, s.z, s.sol, part_rz,
                       st);
    double *dbuf[2] = {s.dA, s.dB};
    int it = 1;
    // first chunk: most of the previous solve's count, then short chunks, so
    // few launches run after convergence
    int chunk = s.last_pcg_iters > 16 ? (s.last_pcg_iters * 7) / 8 : 8;
    *hit_cap = 0;
    hipEvent_t ev[2];
    while (it <= maxit) {
        int c = chunk < maxit - it + 1 ? chunk : maxit - it + 1;
        for (int j = 0; j < c; ++j, ++it) {
            bool timed = (it & 3) == 1;  // time one launch in four when profiling
            if (timed) prof_begin(s, kProfPcgA, ev);
            hipLaunchKernelGGL(k_pcg_A, dim3(nbA), dim3(kBlock), 0, s.stream, it, n, nbB, tol2, s.slice_ptr, s.bcol,
                               s.bval, s.c_ptr, s.c_list, s.act_v, s.act_H, s.act_cap, s.z, dbuf[(it + 1) & 1],
                               dbuf[it & 1], s.q, part_dq, part_rz, st);
            if (timed) prof_end(s, kProfPcgA, ev);
            if (timed) prof_begin(s, kProfPcgB, ev);
            hipLaunchKernelGGL(k_pcg_B, dim3(nbB), dim3(kBlock), 0, s.stream, it, n, nbA, nbB, s.q, dbuf[it & 1],
                               s.Minv, s.sol, s.r, s.z, part_dq, part_rz, st);
            if (timed) prof_end(s, kProfPcgB, ev);
        }
        IPC_HIP(hipMemcpyAsync(&s.hb->flag, &st->done, sizeof(int32_t), hipMemcpyDeviceToHost, s.stream));
        IPC_HIP(hipMemcpyAsync(&s.hb->iters, &st->iters, sizeof(int32_t), hipMemcpyDeviceToHost, s.stream));
        IPC_HIP(hipStreamSynchronize(s.stream));
        prof_collect(s);
        if (s.hb->flag) {
            s.last_pcg_iters = s.hb->iters;
            return s.hb->iters;
        }
        chunk = 8;
    }
    *hit_cap = 1;
    s.last_pcg_iters = maxit;
    return maxit;
}

}  // namespace ipcg
