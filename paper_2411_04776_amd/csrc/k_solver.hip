// k_solver.hip -- block-Jacobi PCG, vector kernels and segmented scans, all
// over a list of scenes (one launch per phase for every scene in the list).
//
// PCG solves H p = -g from p = 0 and stops when the preconditioned residual
// r^T M^-1 r reaches pcg_tol^2 times its initial value. Each iteration is two
// kernels with every scalar kept on the device:
//   A(it): every wavefront of a scene reduces that scene's r.z partials of
//          the previous iteration in a fixed order (all agree bit for bit;
//          no block barrier before the real work) and decides the stop;
//          block 0 keeps r.z for the next launches; a row block then forms d = z + beta
//          d_prev for its rows and for the columns it gathers and applies the
//          elastic BELL matrix (eight lanes per row), a pair block applies
//          each active pair's off-diagonal blocks to its own four vertices;
//          both write their d.q partials;
//   B(it): every wavefront reduces the scene's d.q partials, alpha = rz / dq,
//          each wavefront adds its rows' incident pair products to q
//          (segmented over the incidence lists), then p += alpha d,
//          r -= alpha q, z = M^-1 r and the r.z partials.
// Kernel boundaries cost ~3 us on MI355X against 8-28 us for a cooperative
// grid-wide barrier, so an iteration is two launches rather than one
// persistent kernel. The host launches chunks of iterations and reads the
// per-scene done flags once per chunk; finished scenes turn the remaining
// launches into no-ops.
#include <algorithm>

#include "device_util.h"
#include "incidence.h"
#include "ipc_internal.h"

namespace ipcg {

template <class R>
__device__ __forceinline__ R *as(void *p)
{
    return reinterpret_cast<R *>(p);
}

// partial-sum layout in pcg_part: [d.q of the row blocks: nb_rows][r.z slot 0][r.z slot 1], an
// r.z slot holding nb_vert vertex-block partials then one per heavy row (n + 1 room);
// the pair blocks' d.(H_c d) partials live in pcg_pair
__device__ __forceinline__ double *rz_slot(const SceneDev &S, int it)
{
    return S.pcg_part + S.nb_rows + (size_t)(it & 1) * ((size_t)S.nb_vert + S.n + 1);
}

__device__ __forceinline__ int blocks_for(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }

// coarse-level r.e partials of iteration it (two parity slots)
__device__ __forceinline__ double *mas_slot(const SceneDev &S, int it)
{
    return S.mas_part + (size_t)(it & 1) * S.mas_nblk;
}

// r.z of iteration it: the block-Jacobi part of the vertex blocks (and heavy
// rows), plus the aggregate corrections' part
__device__ __forceinline__ double rz_total(const SceneDev &S, int it, int n_vert_part)
{
    double v = wave_reduce_partials(rz_slot(S, it), n_vert_part);
    if (S.mas_levels > 0) v += wave_reduce_partials(mas_slot(S, it), S.mas_nblk);
    return v;
}

template <class R>
__global__ void __launch_bounds__(kBlock) k_pcg_init(Launch L)
{
    int lb, s = scene_of_block(L, lb);
    const SceneDev &S = *L.sc[s];
    int i = lb * blockDim.x + threadIdx.x;
    R *r = as<R>(S.r), *z = as<R>(S.z), *sol = as<R>(S.sol);
    const R *g = as<R>(S.grad), *Mi = as<R>(S.Minv);
    double rz = 0.0;
    if (i < S.n) {
        R ri[3], zi[3];
        for (int c = 0; c < 3; ++c) ri[c] = -g[3 * i + c];
        for (int a = 0; a < 3; ++a) zi[a] = Mi[9 * i + 3 * a] * ri[0] + Mi[9 * i + 3 * a + 1] * ri[1] + Mi[9 * i + 3 * a + 2] * ri[2];
        for (int c = 0; c < 3; ++c) {
            r[3 * i + c] = ri[c];
            z[3 * i + c] = zi[c];
            sol[3 * i + c] = R(0);
            rz += (double)ri[c] * (double)zi[c];
        }
    }
    rz = block_sum_all(rz);
    if (threadIdx.x == 0) rz_slot(S, 0)[lb] = rz;
    if (i == 0) {
        S.pcg->done = 0;
        S.pcg->iters = 0;
        S.pcg->stop = 0.0;
        L.out[s].pcg_done = 0;
        L.out[s].pcg_iters = 0;
    }
}

// Partial product of one BELL row: lane `part` of the row's kLanesPerRow
// lanes takes slots part, part + kLanesPerRow, ... The vector applied is
// z + beta d_prev (formed at the gathered column) when beta_on, else z.
template <class R>
__device__ __forceinline__ void bell_row_part(const SceneDev &S, int row, int part, const R *__restrict__ z,
                                              const R *__restrict__ dold, R beta, bool beta_on, double y[3])
{
    int sl = row / kSlice, lane = row % kSlice;
    int s0 = S.slice_ptr[sl], s1 = S.slice_ptr[sl + 1];
    const R *__restrict__ bval = as<R>(S.bval);
    const int32_t *__restrict__ bcol = S.bcol;
    R y0 = R(0), y1 = R(0), y2 = R(0);
#pragma unroll 2
    for (int slot = s0 + part; slot < s1; slot += kLanesPerRow) {
        int col = bcol[(int64_t)slot * kSlice + lane];
        if (col >= 0) {
            const R *A = bval + (int64_t)slot * 9 * kSlice + lane;
            R v0 = z[3 * col], v1 = z[3 * col + 1], v2 = z[3 * col + 2];
            if (beta_on) {
                v0 += beta * dold[3 * col];
                v1 += beta * dold[3 * col + 1];
                v2 += beta * dold[3 * col + 2];
            }
            y0 += A[0 * kSlice] * v0 + A[1 * kSlice] * v1 + A[2 * kSlice] * v2;
            y1 += A[3 * kSlice] * v0 + A[4 * kSlice] * v1 + A[5 * kSlice] * v2;
            y2 += A[6 * kSlice] * v0 + A[7 * kSlice] * v1 + A[8 * kSlice] * v2;
        }
    }
    y[0] = y0;
    y[1] = y1;
    y[2] = y2;
}

// The same row with both vectors applied: yz = A z and yd = A d_prev (when
// two), so that nothing here waits for beta.
template <class R>
__device__ __forceinline__ void bell_row_part2(const SceneDev &S, int row, int part, const R *__restrict__ z,
                                               const R *__restrict__ dold, bool two, double yz[3], double yd[3])
{
    int sl = row / kSlice, lane = row % kSlice;
    int s0 = S.slice_ptr[sl], s1 = S.slice_ptr[sl + 1];
    const R *__restrict__ bval = as<R>(S.bval);
    const int32_t *__restrict__ bcol = S.bcol;
    R a0 = R(0), a1 = R(0), a2 = R(0), b0 = R(0), b1 = R(0), b2 = R(0);
#pragma unroll 2
    for (int slot = s0 + part; slot < s1; slot += kLanesPerRow) {
        int col = bcol[(int64_t)slot * kSlice + lane];
        if (col >= 0) {
            const R *A = bval + (int64_t)slot * 9 * kSlice + lane;
            R m[9];
#pragma unroll
            for (int k = 0; k < 9; ++k) m[k] = A[k * kSlice];
            R v0 = z[3 * col], v1 = z[3 * col + 1], v2 = z[3 * col + 2];
            a0 += m[0] * v0 + m[1] * v1 + m[2] * v2;
            a1 += m[3] * v0 + m[4] * v1 + m[5] * v2;
            a2 += m[6] * v0 + m[7] * v1 + m[8] * v2;
            if (two) {
                R w0 = dold[3 * col], w1 = dold[3 * col + 1], w2 = dold[3 * col + 2];
                b0 += m[0] * w0 + m[1] * w1 + m[2] * w2;
                b1 += m[3] * w0 + m[4] * w1 + m[5] * w2;
                b2 += m[6] * w0 + m[7] * w1 + m[8] * w2;
            }
        }
    }
    yz[0] = a0;
    yz[1] = a1;
    yz[2] = a2;
    yd[0] = b0;
    yd[1] = b1;
    yd[2] = b2;
}

// One active pair: y_a = sum over b != a of H_ab d_b for its four slots
// (the diagonal blocks live in the BELL diagonal), stored per pair for the
// row gather; returns sum_a d_a . y_a.
template <class R>
__device__ __forceinline__ double pair_apply(const SceneDev &S, int64_t p, const R *__restrict__ z,
                                             const R *__restrict__ dold, R beta, bool beta_on)
{
    const int64_t cap = S.act_cap;
    const R *__restrict__ H = as<R>(S.act_H);
    R *__restrict__ Y = as<R>(S.act_y);
    R d[4][3];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        int v = S.act_v[(int64_t)a * cap + p];
#pragma unroll
        for (int c = 0; c < 3; ++c) d[a][c] = beta_on ? z[3 * v + c] + beta * dold[3 * v + c] : z[3 * v + c];
    }
    double dy = 0.0;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        double y[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            if (b == a) continue;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const R *h = H + (int64_t)((3 * a + i) * 12 + 3 * b) * cap + p;
                y[i] += (double)(h[0] * d[b][0] + h[cap] * d[b][1] + h[2 * cap] * d[b][2]);
            }
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            R yv = (R)y[i];
            Y[(int64_t)(3 * a + i) * cap + p] = yv;
            dy += (double)d[a][i] * (double)yv;
        }
    }
    return dy;
}

// PCG A(it): a row block first applies the BELL matrix to z and to d_prev
// (no scalar needed), then every wavefront reduces the r.z partials, decides
// the stop and forms beta; the row block finishes d = z + beta d_prev and
// q = K_el d for its rows, a pair block applies each active pair's
// off-diagonal blocks to its own four vertices; both write d.q partials.
template <class R>
__global__ void __launch_bounds__(kBlock) k_pcg_A(Launch L, int it)
{
    int lb, s = scene_of_block(L, lb);
    const SceneDev &S = *L.sc[s];
    const R *z = as<R>(S.z);
    const R *dold = as<R>((it & 1) ? S.dB : S.dA);
    const bool bon = it > 1;
    // kLanesPerRow consecutive lanes share a row
    int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    int row = lb * kRowsPerBlock + wave * (kWave / kLanesPerRow) + lane / kLanesPerRow;
    int part = lane % kLanesPerRow;
    bool rows = lb < S.nb_rows;
    bool live = rows && row < S.n;
    double yz[3] = {0.0, 0.0, 0.0}, yd[3] = {0.0, 0.0, 0.0};
    if (live) bell_row_part2<R>(S, row, part, z, dold, bon, yz, yd);
    if (S.pcg->done) return;
    double beta = 0.0;
    if (it == 1) {
        double rz0 = rz_total(S, 0, S.nb_vert);
        if (!(rz0 > 0.0)) {
            if (lb == 0 && threadIdx.x == 0) {
                S.pcg->done = 1;
                S.pcg->iters = 0;
                L.out[s].pcg_done = 1;
                L.out[s].pcg_iters = 0;
            }
            return;
        }
        if (lb == 0 && threadIdx.x == 0) {
            S.pcg->stop = S.pcg_tol2 * rz0;
            S.pcg->rzv[1] = rz0;
        }
    } else {
        double rz_cur = rz_total(S, it - 1, S.nb_vert + L.out[s].n_heavy);
        bool conv = rz_cur <= S.pcg->stop;
        if (conv || it > S.pcg_maxit) {  // converged, or the scene's iteration cap is spent
            if (lb == 0 && threadIdx.x == 0) {
                S.pcg->done = 1;
                S.pcg->iters = it - 1;
                L.out[s].pcg_done = conv ? 1 : 2;
                L.out[s].pcg_iters = it - 1;
            }
            return;
        }
        // r.z of iteration it - 2, kept by block 0 of the previous launch
        double rz_prev = S.pcg->rzv[(it - 1) & 1];
        beta = rz_cur / rz_prev;
        if (lb == 0 && threadIdx.x == 0) S.pcg->rzv[it & 1] = rz_cur;
    }
    R rb = (R)beta;
    double dq = 0.0;
    if (rows) {
        R *dnew = as<R>((it & 1) ? S.dA : S.dB);
        R *q = as<R>(S.q);
        double y[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            y[c] = yz[c] + beta * yd[c];
#pragma unroll
            for (int o = 1; o < kLanesPerRow; o <<= 1) y[c] += __shfl_xor(y[c], o, kWave);
        }
        if (live && part == 0) {
            for (int c = 0; c < 3; ++c) {
                R dv = bon ? z[3 * row + c] + rb * dold[3 * row + c] : z[3 * row + c];
                R qv = (R)y[c];
                dnew[3 * row + c] = dv;
                q[3 * row + c] = qv;
                dq += (double)dv * (double)qv;
            }
        }
        dq = block_sum_all(dq);
        if (threadIdx.x == 0) S.pcg_part[lb] = dq;
    } else {
        int pb = lb - S.nb_rows;
        int64_t p = (int64_t)pb * blockDim.x + threadIdx.x;
        if (p < L.out[s].n_pair) dq = pair_apply<R>(S, p, z, dold, rb, bon);
        dq = block_sum_all(dq);
        if (threadIdx.x == 0) S.pcg_pair[pb] = dq;
    }
}

// the incident pairs' (H_p d_p)_i of a light row, by one thread
template <class R>
__device__ __forceinline__ void contact_row_light(const SceneDev &S, int row, double qc[3])
{
    const R *Y = as<R>(S.act_y);
    const int64_t cap = S.act_cap;
    thread_row_sums<3>(S, row, [&](int p, int a, int c) { return (double)Y[(int64_t)(3 * a + c) * cap + p]; }, qc);
}

// the same sum for one heavy row, by the whole block
template <class R>
__device__ __forceinline__ void contact_row_heavy(const SceneDev &S, int row, double qc[3])
{
    const R *Y = as<R>(S.act_y);
    const int64_t cap = S.act_cap;
    block_row_sums<3>(S, row, [&](int p, int a, int c) { return (double)Y[(int64_t)(3 * a + c) * cap + p]; }, qc);
}

// one vertex's state for the update, loaded before alpha is known
template <class R>
struct VertexPcg {
    R q[3], d[3], p[3], r[3], M[9];
};

template <class R>
__device__ __forceinline__ void pcg_vertex_load(const SceneDev &S, int i, const R *dcur, VertexPcg<R> &v)
{
    const R *q = as<R>(S.q), *Mi = as<R>(S.Minv), *sol = as<R>(S.sol), *r = as<R>(S.r);
    for (int c = 0; c < 3; ++c) {
        v.q[c] = q[3 * i + c];
        v.d[c] = dcur[3 * i + c];
        v.p[c] = sol[3 * i + c];
        v.r[c] = r[3 * i + c];
    }
    for (int k = 0; k < 9; ++k) v.M[k] = Mi[9 * i + k];
}

// p += alpha d, r -= alpha q (q = K_el d + contact sum), z = M^-1 r; returns r.z
template <class R>
__device__ __forceinline__ double pcg_vertex_update(const SceneDev &S, int i, R alpha, const VertexPcg<R> &v,
                                                    const double qc[3])
{
    R *sol = as<R>(S.sol), *r = as<R>(S.r), *z = as<R>(S.z);
    R ri[3];
    for (int c = 0; c < 3; ++c) {
        R qv = (R)((double)v.q[c] + qc[c]);
        sol[3 * i + c] = v.p[c] + alpha * v.d[c];
        ri[c] = v.r[c] - alpha * qv;
        r[3 * i + c] = ri[c];
    }
    double rz = 0.0;
    for (int a = 0; a < 3; ++a) {
        R za = v.M[3 * a] * ri[0] + v.M[3 * a + 1] * ri[1] + v.M[3 * a + 2] * ri[2];
        z[3 * i + a] = za;
        rz += (double)ri[a] * (double)za;
    }
    return rz;
}

// PCG B(it) over [vertex blocks | one block per heavy incidence row]: the
// vertex data and contact sums are loaded first, then alpha from the d.q
// partials, then the update and the r.z partials.
template <class R>
__global__ void __launch_bounds__(kBlock) k_pcg_B(Launch L, int it)
{
    int lb, s = scene_of_block(L, lb);
    const SceneDev &S = *L.sc[s];
    const R *dcur = as<R>((it & 1) ? S.dA : S.dB);
    if (lb < S.nb_vert) {
        int i = lb * blockDim.x + threadIdx.x;
        bool own = i < S.n && !S.hflag[i];
        VertexPcg<R> v;
        double qc[3] = {0.0, 0.0, 0.0};
        if (own) {
            pcg_vertex_load<R>(S, i, dcur, v);
            contact_row_light<R>(S, i, qc);
        }
        if (S.pcg->done) return;
        double dq = wave_reduce_partials(S.pcg_part, S.nb_rows) + wave_reduce_partials(S.pcg_pair, blocks_for(L.out[s].n_pair));
        R alpha = (R)(S.pcg->rzv[it & 1] / dq);  // r.z of iteration it - 1, stored by A(it)
        double rz = own ? pcg_vertex_update<R>(S, i, alpha, v, qc) : 0.0;
        rz = block_sum_all(rz);
        if (threadIdx.x == 0) rz_slot(S, it)[lb] = rz;
    } else {
        int j = lb - S.nb_vert;
        if (j >= L.out[s].n_heavy) return;
        int row = S.heavy_rows[j];
        double qc[3];
        contact_row_heavy<R>(S, row, qc);
        if (S.pcg->done) return;
        // every lane of the wavefront takes part in the partial reductions
        double dq = wave_reduce_partials(S.pcg_part, S.nb_rows) + wave_reduce_partials(S.pcg_pair, blocks_for(L.out[s].n_pair));
        R alpha = (R)(S.pcg->rzv[it & 1] / dq);
        if (threadIdx.x == 0) {
            VertexPcg<R> v;
            pcg_vertex_load<R>(S, row, dcur, v);
            rz_slot(S, it)[S.nb_vert + j] = pcg_vertex_update<R>(S, row, alpha, v, qc);
        }
    }
}

// ---- multilevel additive preconditioner ----------------------------------
// z = D0^-1 r + sum over levels l of P_l E_l^-1 P_l^T r, with P_l the
// piecewise-constant injection of level-l aggregates of free gel vertices and
// E_l the 3x3 block of the assembled matrix summed over each aggregate
// (translation of the aggregate as a whole). Symmetric positive definite, so
// PCG keeps its guarantees; every sum runs in a fixed order. Level 0 has a
// thread per aggregate, coarser levels a block per aggregate.

// which aggregate a block (and thread) of a kPhMas launch serves; -1: none
__device__ __forceinline__ int mas_agg_of(const SceneDev &S, int lb, bool &per_block)
{
    if (lb < S.mas_nb1) {
        per_block = false;
        int a = lb * kBlock + threadIdx.x;
        return a < S.mas_n[0] ? a : -1;
    }
    per_block = true;
    return S.mas_n[0] + (lb - S.mas_nb1);
}

template <class R>
__global__ void __launch_bounds__(kBlock) k_mas_diag(Launch L)
{
    int lb, s = scene_of_block(L, lb);
    const SceneDev &S = *L.sc[s];
    bool pb;
    int g = mas_agg_of(S, lb, pb);
    const R *bval = as<R>(S.bval);
    double A[9];
    for (int c = 0; c < 9; ++c) A[c] = 0.0;
    int e0 = g >= 0 ? S.mas_dptr[g] : 0, e1 = g >= 0 ? S.mas_dptr[g + 1] : 0;
    int t0 = pb ? e0 + (int)threadIdx.x : e0, dt = pb ? (int)blockDim.x : 1;
    for (int t = t0; t < e1; t += dt) {
        int64_t e = S.mas_dsrc[t];
        int64_t slot = e / kSlice, lane = e % kSlice;
        for (int c = 0; c < 9; ++c) A[c] += (double)bval[(slot * 9 + c) * kSlice + lane];
    }
    if (pb) block_sum_vec<9>(A);
    if (g < 0 || (pb && threadIdx.x != 0)) return;
    double Inv[9];
    inverse3(A, Inv);
    R *Di = as<R>(S.mas_dinv);
    for (int c = 0; c < 9; ++c) Di[9 * (int64_t)g + c] = (R)Inv[c];
}

// restriction of r to every aggregate, e = E^-1 r_agg, and the r.e partials
template <class R>
__global__ void __launch_bounds__(kBlock) k_mas_restrict(Launch L, int it)
{
    int lb, s = scene_of_block(L, lb);
    const SceneDev &S = *L.sc[s];
    if (S.pcg->done) return;
    bool pb;
    int g = mas_agg_of(S, lb, pb);
    const R *r = as<R>(S.r);
    double ra[3] = {0.0, 0.0, 0.0};
    int m0 = g >= 0 ? S.mas_mb[g] : 0, m1 = g >= 0 ? S.mas_me[g] : 0;
    int t0 = pb ? m0 + (int)threadIdx.x : m0, dt = pb ? (int)blockDim.x : 1;
    for (int t = t0; t < m1; t += dt) {
        int i = S.mas_mem[t];
        for (int c = 0; c < 3; ++c) ra[c] += (double)r[3 * i + c];
    }
    if (pb) block_sum_vec<3>(ra);
    double re = 0.0;
    if (g >= 0 && (!pb || threadIdx.x == 0)) {
        const R *Di = as<R>(S.mas_dinv);
        R *E = as<R>(S.mas_e);
        for (int a = 0; a < 3; ++a) {
            R ea = (R)(Di[9 * (int64_t)g + 3 * a] * (R)ra[0] + Di[9 * (int64_t)g + 3 * a + 1] * (R)ra[1] +
                       Di[9 * (int64_t)g + 3 * a + 2] * (R)ra[2]);
            E[3 * (int64_t)g + a] = ea;
            re += ra[a] * (double)ea;
        }
    }
    if (!pb) re = block_sum_all(re);
    if (threadIdx.x == 0) mas_slot(S, it)[lb] = re;
}

// z_i += sum over levels of the corrections of i's aggregates
template <class R>
__global__ void __launch_bounds__(kBlock) k_mas_prolong(Launch L)
{
    int lb, s = scene_of_block(L, lb);
    const SceneDev &S = *L.sc[s];
    if (S.pcg->done) return;
    int i = lb * blockDim.x + threadIdx.x;
    if (i >= S.n || S.mas_levels == 0) return;
    int g0 = S.mas_anc[i];
    if (g0 < 0) return;
    const R *E = as<R>(S.mas_e);
    R *z = as<R>(S.z);
    double zi[3] = {(double)z[3 * i], (double)z[3 * i + 1], (double)z[3 * i + 2]};
    for (int l = 0; l < S.mas_levels; ++l) {
        int g = S.mas_anc[(int64_t)l * S.n + i];
        for (int c = 0; c < 3; ++c) zi[c] += (double)E[3 * (int64_t)g + c];
    }
    for (int c = 0; c < 3; ++c) z[3 * i + c] = (R)zi[c];
}

// y = H v for the test hook (v in S.dB, y in S.q), in the PCG's three parts:
// pair products, BELL rows, then the incident pair products per row
template <class R>
__global__ void __launch_bounds__(kBlock) k_spmv_pairs(Launch L)
{
    int lb, s = scene_of_block(L, lb);
    const SceneDev &S = *L.sc[s];
    int64_t p = (int64_t)lb * blockDim.x + threadIdx.x;
    if (p < L.out[s].n_pair) (void)pair_apply<R>(S, p, as<R>(S.dB), nullptr, R(0), false);
}

template <class R>
__global__ void __launch_bounds__(kBlock) k_spmv_rows(Launch L)
{
    int lb, s = scene_of_block(L, lb);
    const SceneDev &S = *L.sc[s];
    const R *v = as<R>(S.dB);
    R *y = as<R>(S.q);
    int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    int row = lb * kRowsPerBlock + wave * (kWave / kLanesPerRow) + lane / kLanesPerRow;
    int part = lane % kLanesPerRow;
    double o[3] = {0.0, 0.0, 0.0};
    bool live = row < S.n;
    if (live) bell_row_part<R>(S, row, part, v, nullptr, R(0), false, o);
    for (int c = 0; c < 3; ++c)
        for (int k = 1; k < kLanesPerRow; k <<= 1) o[c] += __shfl_xor(o[c], k, kWave);
    if (live && part == 0)
        for (int c = 0; c < 3; ++c) y[3 * row + c] = (R)o[c];
}

template <class R>
__global__ void __launch_bounds__(kBlock) k_spmv_contact(Launch L)
{
    int lb, s = scene_of_block(L, lb);
    const SceneDev &S = *L.sc[s];
    R *y = as<R>(S.q);
    if (lb < S.nb_vert) {
        int i = lb * blockDim.x + threadIdx.x;
        if (i < S.n && !S.hflag[i]) {
            double qc[3] = {0.0, 0.0, 0.0};
            contact_row_light<R>(S, i, qc);
            for (int c = 0; c < 3; ++c) y[3 * i + c] = (R)((double)y[3 * i + c] + qc[c]);
        }
    } else {
        int j = lb - S.nb_vert;
        if (j >= L.out[s].n_heavy) return;
        int row = S.heavy_rows[j];
        double qc[3];
        contact_row_heavy<R>(S, row, qc);
        if (threadIdx.x == 0)
            for (int c = 0; c < 3; ++c) y[3 * row + c] = (R)((double)y[3 * row + c] + qc[c]);
    }
}

// ---- per-vertex kernels ------------------------------------------------------

template <class R>
__global__ void k_pinf(Launch L)
{
    int lb, s = scene_of_block(L, lb);
    const SceneDev &S = *L.sc[s];
    const R *p = as<R>(S.sol);
    int i = lb * blockDim.x + threadIdx.x;
    double v = 0.0;
    if (i < S.n && !S.fixed[i])
        v = fmax(fabs((double)p[3 * i]), fmax(fabs((double)p[3 * i + 1]), fabs((double)p[3 * i + 2])));
    v = block_max_all(v);
    if (threadIdx.x == 0) S.red[lb] = v;
}

// one block per scene: max over the producer's per-block partials
__global__ void k_final_pinf(Launch one, Launch prod)
{
    int lb, s = scene_of_block(one, lb);
    const SceneDev &S = *one.sc[s];
    int nb = blocks_of(prod, s);
    double v = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) v = fmax(v, S.red[i]);
    v = block_max_all(v);
    if (threadIdx.x == 0) one.out[s].pinf = v;
}

// x_trial = x + alpha p (one rounding per component, as the line search
// defines it); alpha per scene
template <class R>
__global__ void k_trial(Launch L, const double *__restrict__ alpha)
{
    int lb, s = scene_of_block(L, lb);
    const SceneDev &S = *L.sc[s];
    const R *p = as<R>(S.sol);
    int i = lb * blockDim.x + threadIdx.x;
    if (i >= S.n) return;
    double a = alpha[s];
    for (int c = 0; c < 3; ++c) S.xtrial[3 * i + c] = __dadd_rn(S.x[3 * i + c], __dmul_rn(a, (double)p[3 * i + c]));
}

__global__ void k_accept(Launch L)
{
    int lb, s = scene_of_block(L, lb);
    const SceneDev &S = *L.sc[s];
    int i = lb * blockDim.x + threadIdx.x;
    if (i >= S.n) return;
    for (int c = 0; c < 3; ++c) S.x[3 * i + c] = S.xtrial[3 * i + c];
}

// step start: keep x^t, inertial predictor for free gel vertices, indenter
// targets from the scene's pose
__global__ void k_begin_step(Launch L)
{
    int lb, s = scene_of_block(L, lb);
    const SceneDev &S = *L.sc[s];
    int i = lb * blockDim.x + threadIdx.x;
    if (i >= S.n) return;
    double h = S.h;
    for (int c = 0; c < 3; ++c) S.xt[3 * i + c] = S.x[3 * i + c];
    if (i < S.n_gel) {
        for (int c = 0; c < 3; ++c) {
            double xv = S.x[3 * i + c];
            S.xtilde[3 * i + c] = S.fixed[i] ? xv : xv + h * S.v[3 * i + c] + h * h * S.grav[c];
            S.yhat[3 * i + c] = xv;
        }
    } else {
        const double *y = S.Yloc + 3 * (i - S.n_gel);
        const double *P = S.pose;
        for (int c = 0; c < 3; ++c) {
            S.yhat[3 * i + c] = P[c * 4 + 0] * y[0] + P[c * 4 + 1] * y[1] + P[c * 4 + 2] * y[2] + P[c * 4 + 3];
            S.xtilde[3 * i + c] = S.x[3 * i + c];
        }
    }
}

__global__ void k_end_step(Launch L)
{
    int lb, s = scene_of_block(L, lb);
    const SceneDev &S = *L.sc[s];
    int i = lb * blockDim.x + threadIdx.x;
    if (i >= S.n) return;
    double inv_h = 1.0 / S.h;
    for (int c = 0; c < 3; ++c) S.v[3 * i + c] = (S.x[3 * i + c] - S.xt[3 * i + c]) * inv_h;
}

// max target lag over indenter vertices and per-block sums of gel positions
__global__ void k_lag_mean(Launch L)
{
    int lb, s = scene_of_block(L, lb);
    const SceneDev &S = *L.sc[s];
    int i = lb * blockDim.x + threadIdx.x;
    double lag = 0.0, m[3] = {0.0, 0.0, 0.0};
    if (i < S.n) {
        if (i >= S.n_gel) {
            double d0 = S.x[3 * i] - S.yhat[3 * i], d1 = S.x[3 * i + 1] - S.yhat[3 * i + 1],
                   d2 = S.x[3 * i + 2] - S.yhat[3 * i + 2];
            lag = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        } else {
            for (int c = 0; c < 3; ++c) m[c] = S.x[3 * i + c];
        }
    }
    lag = block_max_all(lag);
    for (int c = 0; c < 3; ++c) m[c] = block_sum_all(m[c]);
    if (threadIdx.x == 0) {
        S.red[4 * lb] = lag;
        for (int c = 0; c < 3; ++c) S.red[4 * lb + 1 + c] = m[c];
    }
}

__global__ void k_final_lag_mean(Launch one, Launch prod)
{
    int lb, s = scene_of_block(one, lb);
    const SceneDev &S = *one.sc[s];
    int nb = blocks_of(prod, s);
    double lag = 0.0, m[3] = {0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < nb; i += blockDim.x) {
        lag = fmax(lag, S.red[4 * i]);
        for (int c = 0; c < 3; ++c) m[c] += S.red[4 * i + 1 + c];
    }
    lag = block_max_all(lag);
    for (int c = 0; c < 3; ++c) m[c] = block_sum_all(m[c]);
    if (threadIdx.x == 0) {
        one.out[s].lag = lag;
        for (int c = 0; c < 3; ++c) one.out[s].obj[c] = m[c] / (double)S.n_gel;
    }
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

// ---- segmented exclusive scan of per-scene int32 arrays ------------------------
// Each scene's array is cut into tiles of kScanTile values (its own block
// range); per-tile sums are scanned by one block per scene; then each tile
// writes its exclusive prefix. out[len] and the scene's read-back slot get
// the total.

struct ScanSel {
    const int32_t *in;
    int32_t *out;
    int64_t len;
};

__device__ __forceinline__ ScanSel scan_sel(const SceneDev &S, const SceneOut &O, int which)
{
    switch (which) {
    case kScanTri: return {S.ht_count[0], S.ht_start[0], (int64_t)1 << S.ht_bits[0]};
    case kScanEdge: return {S.ht_count[1], S.ht_start[1], (int64_t)1 << S.ht_bits[1]};
    case kScanQuery: return {S.q_count, S.q_off, (int64_t)S.n_pts + S.n_edges};
    case kScanContact: return {S.c_cnt, S.c_ptr, (int64_t)S.n};
    case kScanHeavy: return {S.hflag, S.heavy_idx, (int64_t)S.n};
    case kScanSwFilter: return {S.sw_flag, S.sw_off, S.n_sw_prev};
    default: return {S.act_flag, S.act_off, (int64_t)O.n_cand};
    }
}

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

constexpr int kScanItems = kScanTile / kBlock;

__global__ void __launch_bounds__(kBlock) k_scan_tiles(Launch L, int which)
{
    int lb, s = scene_of_block(L, lb);
    const SceneDev &S = *L.sc[s];
    ScanSel sel = scan_sel(S, L.out[s], which);
    int64_t base = (int64_t)lb * kScanTile + threadIdx.x * kScanItems;
    int sum = 0;
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < sel.len) sum += sel.in[base + k];
    int tot;
    block_exclusive_scan(sum, &tot);
    if (threadIdx.x == 0) S.scan_tmp[lb] = tot;
}

__global__ void __launch_bounds__(kBlock) k_scan_top(Launch one, Launch tiles, int which, int query_sw)
{
    int lb, s = scene_of_block(one, lb);
    const SceneDev &S = *one.sc[s];
    int nt = blocks_of(tiles, s);
    int carry = 0;
    for (int base = 0; base < nt; base += kBlock) {
        int i = base + threadIdx.x;
        int v = i < nt ? S.scan_tmp[i] : 0;
        int tot;
        int ex = block_exclusive_scan(v, &tot);
        if (i < nt) S.scan_tmp[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        SceneOut &O = one.out[s];
        ScanSel sel = scan_sel(S, O, which);
        sel.out[sel.len] = carry;
        if (which == kScanTri) O.ent_tri = carry;
        if (which == kScanEdge) O.ent_edge = carry;
        if (which == kScanQuery) {
            if (query_sw)
                O.n_sw = carry;
            else
                O.n_cand = carry;
        }
        if (which == kScanActive) O.n_act = carry;
        if (which == kScanHeavy) O.n_heavy = carry;
        if (which == kScanSwFilter) O.n_cand = carry;
    }
}

__global__ void __launch_bounds__(kBlock) k_scan_apply(Launch L, int which)
{
    int lb, s = scene_of_block(L, lb);
    const SceneDev &S = *L.sc[s];
    ScanSel sel = scan_sel(S, L.out[s], which);
    int64_t base = (int64_t)lb * kScanTile + threadIdx.x * kScanItems;
    int vals[kScanItems];
    int sum = 0;
    for (int k = 0; k < kScanItems; ++k) {
        vals[k] = (base + k < sel.len) ? sel.in[base + k] : 0;
        sum += vals[k];
    }
    int tot;
    int ex = block_exclusive_scan(sum, &tot) + S.scan_tmp[lb];
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < sel.len) sel.out[base + k] = ex;
        ex += vals[k];
    }
}

// ---- launchers ----------------------------------------------------------------

static bool mixed(const Batch &b) { return b.sc[0]->prm.precision == IPC_MIXED; }

void segmented_scan(Batch &b, ScanWhich which, PhaseKind tiles, const std::vector<int64_t> &len, int query_sw)
{
    size_t ns = b.sc.size();
    std::vector<int32_t> nt(ns), one(ns);
    for (size_t i = 0; i < ns; ++i) {
        nt[i] = len[i] < 0 ? 0 : std::max<int32_t>(1, (int32_t)((len[i] + kScanTile - 1) / kScanTile));
        one[i] = len[i] < 0 ? 0 : 1;
    }
    b.set_phase(tiles, nt);
    b.set_phase(kPhOne, one);
    IPC_LAUNCH(b, k_scan_tiles, tiles, kBlock, (int)which);
    IPC_LAUNCH(b, k_scan_top, kPhOne, kBlock, b.launch(tiles), (int)which, query_sw);
    IPC_LAUNCH(b, k_scan_apply, tiles, kBlock, (int)which);
}

void launch_begin_step(Batch &b) { IPC_LAUNCH(b, k_begin_step, kPhVert, kBlock); }
void launch_end_step(Batch &b) { IPC_LAUNCH(b, k_end_step, kPhVert, kBlock); }

void launch_trial(Batch &b)
{
    if (mixed(b))
        IPC_LAUNCH(b, k_trial<float>, kPhVert, kBlock, (const double *)b.d_alpha);
    else
        IPC_LAUNCH(b, k_trial<double>, kPhVert, kBlock, (const double *)b.d_alpha);
}

void launch_accept(Batch &b) { IPC_LAUNCH(b, k_accept, kPhVert, kBlock); }

static void one_per_active(Batch &b, PhaseKind prod)
{
    std::vector<int32_t> one(b.sc.size());
    for (size_t i = 0; i < b.sc.size(); ++i) one[i] = b.h_off[prod][i + 1] > b.h_off[prod][i] ? 1 : 0;
    b.set_phase(kPhOne, one);
}

void run_lag_and_mean(Batch &b)
{
    IPC_LAUNCH(b, k_lag_mean, kPhVert, kBlock);
    one_per_active(b, kPhVert);
    IPC_LAUNCH(b, k_final_lag_mean, kPhOne, kBlock, b.launch(kPhVert));
}

void launch_gather_surface(Scene &s, double *dst, hipStream_t strm)
{
    int ns = (int)s.h_surf_verts.size();
    hipLaunchKernelGGL(k_gather_surface, dim3(nblocks(ns)), dim3(kBlock), 0, strm, ns, s.h.surf_verts, s.h.x, dst);
}

void run_pinf(Batch &b)
{
    if (mixed(b))
        IPC_LAUNCH(b, k_pinf<float>, kPhVert, kBlock);
    else
        IPC_LAUNCH(b, k_pinf<double>, kPhVert, kBlock);
    one_per_active(b, kPhVert);
    IPC_LAUNCH(b, k_final_pinf, kPhOne, kBlock, b.launch(kPhVert));
}

void launch_mas_diag(Batch &b)
{
    if (mixed(b))
        IPC_LAUNCH(b, k_mas_diag<float>, kPhMas, kBlock);
    else
        IPC_LAUNCH(b, k_mas_diag<double>, kPhMas, kBlock);
}

void launch_hess_apply(Batch &b)
{
    // pair phase as set by the incidence build of the same assembly
    if (mixed(b)) {
        IPC_LAUNCH(b, k_spmv_pairs<float>, kPhActT, kBlock);
        IPC_LAUNCH(b, k_spmv_rows<float>, kPhSlice, kBlock);
        IPC_LAUNCH(b, k_spmv_contact<float>, kPhVertH, kBlock);
    } else {
        IPC_LAUNCH(b, k_spmv_pairs<double>, kPhActT, kBlock);
        IPC_LAUNCH(b, k_spmv_rows<double>, kPhSlice, kBlock);
        IPC_LAUNCH(b, k_spmv_contact<double>, kPhVertH, kBlock);
    }
}

// PCG for every scene with blocks in the kPhVert map (the active-pair counts
// come from the last read-back of the narrow phase).
void run_pcg(Batch &b, std::vector<int> &iters, std::vector<int> &hit_cap)
{
    size_t ns = b.sc.size();
    bool mx = mixed(b);
    std::vector<int32_t> nab(ns, 0);
    for (size_t i = 0; i < ns; ++i)
        if (b.h_off[kPhVert][i + 1] > b.h_off[kPhVert][i]) nab[i] = b.sc[i]->h.nb_rows + nblocks(pair_count(*b.sc[i], b.h_out[i]));
    b.set_phase(kPhPcgA, nab);
    set_heavy_phase(b);
    std::vector<int32_t> mv(ns, 0);
    for (size_t i = 0; i < ns; ++i)
        if (b.h_off[kPhVert][i + 1] > b.h_off[kPhVert][i] && b.sc[i]->h.mas_levels > 0) mv[i] = b.sc[i]->h.nb_vert;
    b.set_phase(kPhMasV, mv);
    if (mx)
        IPC_LAUNCH(b, k_pcg_init<float>, kPhVert, kBlock);
    else
        IPC_LAUNCH(b, k_pcg_init<double>, kPhVert, kBlock);
    auto precondition = [&](int it) {  // aggregate corrections of z for the scenes that use them
        if (mx) {
            IPC_LAUNCH(b, k_mas_restrict<float>, kPhMas, kBlock, it);
            IPC_LAUNCH(b, k_mas_prolong<float>, kPhMasV, kBlock);
        } else {
            IPC_LAUNCH(b, k_mas_restrict<double>, kPhMas, kBlock, it);
            IPC_LAUNCH(b, k_mas_prolong<double>, kPhMasV, kBlock);
        }
    };
    precondition(0);
    int maxit = 0, last = 0;
    for (size_t i = 0; i < ns; ++i) {
        if (b.h_off[kPhVert][i + 1] == b.h_off[kPhVert][i]) continue;
        const Scene &s = *b.sc[i];
        maxit = std::max(maxit, s.h.pcg_maxit);
        last = std::max(last, s.last_pcg_iters);
    }
    iters.assign(ns, 0);
    hit_cap.assign(ns, 0);
    int it = 1;
    int chunk = last > 16 ? (last * 7) / 8 : 8;
    hipEvent_t ev[2];
    // launch it = maxit + 1 too: its A kernel records the cap of the scenes
    // that did not converge
    while (it <= maxit + 1) {
        int c = std::min(chunk, maxit + 2 - it);
        for (int j = 0; j < c; ++j, ++it) {
            bool timed = b.prof() && (it & 3) == 1;  // time one launch in four when profiling
            if (timed) b.prof_begin(kProfPcgA, ev);
            if (mx)
                IPC_LAUNCH(b, k_pcg_A<float>, kPhPcgA, kBlock, it);
            else
                IPC_LAUNCH(b, k_pcg_A<double>, kPhPcgA, kBlock, it);
            if (timed) b.prof_end(kProfPcgA, ev);
            if (timed) b.prof_begin(kProfPcgB, ev);
            if (mx)
                IPC_LAUNCH(b, k_pcg_B<float>, kPhVertH, kBlock, it);
            else
                IPC_LAUNCH(b, k_pcg_B<double>, kPhVertH, kBlock, it);
            precondition(it);
            if (timed) b.prof_end(kProfPcgB, ev);
        }
        b.read_out();
        b.prof_collect();
        bool all = true;
        for (size_t i = 0; i < ns; ++i)
            if (b.h_off[kPhVert][i + 1] > b.h_off[kPhVert][i] && !b.h_out[i].pcg_done) all = false;
        if (all) break;
        chunk = 8;
    }
    for (size_t i = 0; i < ns; ++i) {
        if (b.h_off[kPhVert][i + 1] == b.h_off[kPhVert][i]) continue;
        iters[i] = b.h_out[i].pcg_done ? b.h_out[i].pcg_iters : b.sc[i]->h.pcg_maxit;
        hit_cap[i] = b.h_out[i].pcg_done != 1;
        b.sc[i]->last_pcg_iters = iters[i];
    }
}

}  // namespace ipcg
