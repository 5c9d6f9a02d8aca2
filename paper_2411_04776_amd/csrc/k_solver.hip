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
// r.z slot holding the pcg_nvp update-block partials then one per heavy row (n + 1 room);
// the pair blocks' d.(H_c d) partials live in pcg_pair
__device__ __forceinline__ double *rz_slot(const SceneDev &S, int it)
{
    return S.pcg_part + S.nb_rows + (size_t)(it & 1) * ((size_t)S.pcg_nvp + S.n + 1);
}

// pair blocks of PCG A for n pairs
__device__ __forceinline__ int pair_blocks(int64_t n) { return (int)((n + kPairsPerBlock - 1) / kPairsPerBlock); }

// Partial product of one BELL row: stream `part` of the row's kSpmvStreams
// takes slots part, part + kSpmvStreams, ... The vector applied is
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
    for (int slot = s0 + part; slot < s1; slot += kSpmvStreams) {
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
    for (int slot = s0 + part; slot < s1; slot += kSpmvStreams) {
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

// Both slot streams of one row by one thread, interleaved (two independent
// chains of loads in flight); each stream accumulates its slots in the same
// order and with the same expressions as bell_row_part2, so the partial sums
// are bit-identical to the two-lane form. Used for large lists, whose matrix
// exceeds the caches: its values are streamed with non-temporal loads so the
// gathered vectors keep the cache.
template <class R>
__device__ __forceinline__ void bell_row_both(const SceneDev &S, int row, const R *__restrict__ z,
                                              const R *__restrict__ dold, bool two, double yz[2][3], double yd[2][3])
{
    int sl = row / kSlice, lane = row % kSlice;
    int s0 = S.slice_ptr[sl], s1 = S.slice_ptr[sl + 1];
    const R *__restrict__ bval = as<R>(S.bval);
    const int32_t *__restrict__ bcol = S.bcol;
    R a[2][3] = {{R(0), R(0), R(0)}, {R(0), R(0), R(0)}}, c[2][3] = {{R(0), R(0), R(0)}, {R(0), R(0), R(0)}};
#pragma unroll 2
    for (int slot = s0; slot < s1; slot += 2) {
        int col[2];
        col[0] = bcol[(int64_t)slot * kSlice + lane];
        col[1] = slot + 1 < s1 ? bcol[(int64_t)(slot + 1) * kSlice + lane] : -1;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            if (col[k] < 0) continue;
            const R *A = bval + (int64_t)(slot + k) * 9 * kSlice + lane;
            R m[9];
#pragma unroll
            for (int e = 0; e < 9; ++e) m[e] = __builtin_nontemporal_load(A + e * kSlice);  // read once per launch
            R v0 = z[3 * col[k]], v1 = z[3 * col[k] + 1], v2 = z[3 * col[k] + 2];
            a[k][0] += m[0] * v0 + m[1] * v1 + m[2] * v2;
            a[k][1] += m[3] * v0 + m[4] * v1 + m[5] * v2;
            a[k][2] += m[6] * v0 + m[7] * v1 + m[8] * v2;
            if (two) {
                R w0 = dold[3 * col[k]], w1 = dold[3 * col[k] + 1], w2 = dold[3 * col[k] + 2];
                c[k][0] += m[0] * w0 + m[1] * w1 + m[2] * w2;
                c[k][1] += m[3] * w0 + m[4] * w1 + m[5] * w2;
                c[k][2] += m[6] * w0 + m[7] * w1 + m[8] * w2;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            yz[k][e] = a[k][e];
            yd[k][e] = c[k][e];
        }
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
            Y[12 * p + 3 * a + i] = yv;  // a pair's 12 products together: a row gathers 3 adjacent values
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
// LPR lanes per row (1: a thread runs both slot streams, for coalesced rows in
// large lists; 2: a lane per stream, for latency): the arithmetic is the same
// (streams added in order, the block's d.q summed by one wavefront over its 64
// rows or pairs), so a scene gets the same bits in either form.
template <class R, int LPR>
__global__ void __launch_bounds__(kRowsPerBlock * LPR) k_pcg_A(Launch L, int it, int early)
{
    constexpr int NP = kSpmvStreams / LPR;  // streams per thread
    __shared__ double sdq[kRowsPerBlock];
    int lb, s = scene_of_block(L, lb);
    const SceneDev &S = *L.sc[s];
    // launches past the expected count of this scene's solve: a finished solve costs nothing
    if ((early || it > L.out[s].pcg_early) && S.pcg->done) return;
    // the previous launch's r.z partials load before the matrix rows
    const int nrz = S.pcg_nvp + L.out[s].n_heavy;
    double rzp[2];
    wave_partials_load<2>(rz_slot(S, it - 1), nrz, rzp);
    const R *z = as<R>(S.z);
    const R *dold = as<R>((it & 1) ? S.dB : S.dA);
    const bool bon = it > 1;
    const int t = (int)threadIdx.x, rloc = t / LPR, part0 = t % LPR;
    int row = lb * kRowsPerBlock + rloc;
    bool rows = lb < S.nb_rows;
    bool live = rows && row < S.n;
    double yz[NP][3], yd[NP][3];
#pragma unroll
    for (int q = 0; q < NP; ++q)
#pragma unroll
        for (int c = 0; c < 3; ++c) yz[q][c] = yd[q][c] = 0.0;
    if (live) {
        if constexpr (NP == 2)
            bell_row_both<R>(S, row, z, dold, bon, yz, yd);
        else
            bell_row_part2<R>(S, row, part0, z, dold, bon, yz[0], yd[0]);
    }
    if (S.pcg->done) return;
    double beta = 0.0;
    if (it == 1) {
        double rz0 = wave_partials_sum<2>(rz_slot(S, 0), nrz, rzp);
        if (!(rz0 > 0.0)) {
            if (lb == 0 && t == 0) {
                S.pcg->done = 1;
                S.pcg->iters = 0;
                L.out[s].pcg_done = 1;
                L.out[s].pcg_iters = 0;
            }
            return;
        }
        if (lb == 0 && t == 0) {
            S.pcg->stop = S.pcg_tol2 * rz0;
            S.pcg->rzv[1] = rz0;
        }
    } else {
        double rz_cur = wave_partials_sum<2>(rz_slot(S, it - 1), nrz, rzp);
        bool conv = rz_cur <= S.pcg->stop;
        if (conv || it > S.pcg_maxit) {  // converged, or the scene's iteration cap is spent
            if (lb == 0 && t == 0) {
                S.pcg->done = 1;
                S.pcg->iters = it - 1;
                L.out[s].pcg_done = conv ? 1 : 2;
                L.out[s].pcg_iters = it - 1;
                L.out[s].pcg_early = max(8, ((it - 1) * 7) / 8);  // for the next solve
            }
            return;
        }
        // r.z of iteration it - 2, kept by block 0 of the previous launch
        double rz_prev = S.pcg->rzv[(it - 1) & 1];
        beta = rz_cur / rz_prev;
        if (lb == 0 && t == 0) S.pcg->rzv[it & 1] = rz_cur;
    }
    R rb = (R)beta;
    double dq = 0.0;
    if (rows) {
        R *dnew = as<R>((it & 1) ? S.dA : S.dB);
        R *q = as<R>(S.q);
        double y[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            y[c] = yz[0][c] + beta * yd[0][c];
#pragma unroll
            for (int k = 1; k < NP; ++k) y[c] += yz[k][c] + beta * yd[k][c];
            if (LPR == 2) y[c] += __shfl_xor(y[c], 1, kWave);
        }
        if (live && part0 == 0) {
            for (int c = 0; c < 3; ++c) {
                R dv = bon ? z[3 * row + c] + rb * dold[3 * row + c] : z[3 * row + c];
                R qv = (R)y[c];
                dnew[3 * row + c] = dv;
                q[3 * row + c] = qv;
                dq += (double)dv * (double)qv;
            }
        }
        if (LPR == 2) {
            if (part0 == 0) sdq[rloc] = dq;
            __syncthreads();
            if (t < kWave) dq = sdq[t];
        }
        if (t < kWave) {
            dq = wave_sum(dq);
            if (t == 0) S.pcg_part[lb] = dq;
        }
    } else {
        int pb = lb - S.nb_rows;
        int64_t p = (int64_t)pb * kPairsPerBlock + t;
        if (t < kPairsPerBlock && p < L.out[s].n_pair) dq = pair_apply<R>(S, p, z, dold, rb, bon);
        if (t < kWave) {
            dq = wave_sum(dq);
            if (t == 0) S.pcg_pair[pb] = dq;
        }
    }
}

// the incident pairs' (H_p d_p)_i of a light row, by one thread (two entries
// in flight: the update kernel holds a vertex's PCG state meanwhile, and its
// register count sets how many blocks a CU keeps resident)
template <class R>
__device__ __forceinline__ void contact_row_light(const SceneDev &S, int row, double qc[3])
{
    const R *Y = as<R>(S.act_y);
    auto val = [&](int p, int a, int c) { return (double)Y[12 * (int64_t)p + 3 * a + c]; };
    thread_row_sums<3, decltype(val), 2>(S, row, val, qc);
}

// the same sum for one heavy row, by the whole block
template <class R>
__device__ __forceinline__ void contact_row_heavy(const SceneDev &S, int row, double qc[3])
{
    const R *Y = as<R>(S.act_y);
    block_row_sums<3>(S, row, [&](int p, int a, int c) { return (double)Y[12 * (int64_t)p + 3 * a + c]; }, qc);
}

// one vertex's state for the update, loaded before alpha is known
template <class R>
struct VertexPcg {
    R q[3], d[3], p[3], r[3], M[9];
};

template <class R>
__device__ __forceinline__ void pcg_vertex_load(const SceneDev &S, int i, const R *dcur, VertexPcg<R> &v)
{
    const auto q = glob(as<R>(S.q)), Mi = glob(as<R>(S.Minv)), sol = glob(as<R>(S.sol)), r = glob(as<R>(S.r));
    const auto dc = glob(dcur);
    for (int c = 0; c < 3; ++c) {
        v.q[c] = q[3 * i + c];
        v.d[c] = dc[3 * i + c];
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
    const auto sol = glob(as<R>(S.sol)), r = glob(as<R>(S.r)), z = glob(as<R>(S.z));
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

// ---- multilevel additive preconditioner ----------------------------------
// z = D^-1 r + sum over levels l of P_l E_l^-1 P_l^T r: D the 3x3 diagonal
// blocks, P_l the piecewise-constant injection of the level-l aggregates of
// free gel vertices, E_l = P_l^T A P_l (the assembled block matrix summed over
// each aggregate: the aggregate translating as a whole). Symmetric positive
// definite, so PCG keeps its guarantees. Aggregates nest and a group of
// top-level aggregates is one block, so restriction, the coarse solves and
// prolongation of a group happen in LDS with no grid-wide dependency; every
// sum runs in a fixed order.

// k_mas_diag: each aggregate's own entries (those first shared at its level):
// a wavefront per level-0 aggregate, a block per coarser aggregate
template <class R>
__global__ void __launch_bounds__(kBlock) k_mas_diag(Launch L)
{
    int lb, s = scene_of_block(L, lb);
    const SceneDev &S = *L.sc[s];
    int g, t0, dt;
    bool per_block = lb >= S.mas_nd0;
    if (!per_block) {
        g = lb * (kBlock / kWave) + (int)threadIdx.x / kWave;
        t0 = (int)threadIdx.x % kWave;
        dt = kWave;
        if (g >= S.mas_n[0]) return;  // whole wavefronts leave
    } else {
        g = S.mas_n[0] + (lb - S.mas_nd0);
        t0 = (int)threadIdx.x;
        dt = (int)blockDim.x;
    }
    const R *bval = as<R>(S.bval);
    double A[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) A[c] = 0.0;
    for (int t = S.mas_dptr[g] + t0; t < S.mas_dptr[g + 1]; t += dt) {
        int64_t e = S.mas_dsrc[t];
        int64_t slot = e / kSlice, lane = e % kSlice;
#pragma unroll
        for (int c = 0; c < 9; ++c) A[c] += (double)bval[(slot * 9 + c) * kSlice + lane];
    }
    if (per_block)
        block_sum_vec<9>(A);
    else
#pragma unroll
        for (int c = 0; c < 9; ++c) A[c] = wave_sum(A[c]);
    if (t0 == 0)
#pragma unroll
        for (int c = 0; c < 9; ++c) S.mas_ex[9 * (int64_t)g + c] = A[c];
}

// group's level-l aggregate range [a0, a1) (level-local ids); l = -1: members
__device__ __forceinline__ void mas_group_range(const SceneDev &S, int grp, int l, int &a0, int &a1)
{
    const auto row = glob(S.mas_gofs) + (size_t)(l + 1) * (S.mas_ng + 1);
    a0 = row[grp];
    a1 = row[grp + 1];
}

// k_mas_invert: per group, level by level, E(g) = own entries + the children's
// blocks (in child order), then its inverse
template <class R>
__global__ void __launch_bounds__(kBlock) k_mas_invert(Launch L)
{
    int grp, s = scene_of_block(L, grp);
    const SceneDev &S = *L.sc[s];
    R *Di = as<R>(S.mas_dinv);
    for (int l = 0; l < S.mas_levels; ++l) {
        int a0, a1;
        mas_group_range(S, grp, l, a0, a1);
        for (int a = a0 + (int)threadIdx.x; a < a1; a += blockDim.x) {
            int64_t g = S.mas_off[l] + a;
            double E[9];
#pragma unroll
            for (int c = 0; c < 9; ++c) E[c] = S.mas_ex[9 * g + c];
            if (l > 0)
                for (int ch = S.mas_mb[g]; ch < S.mas_me[g]; ++ch) {
                    int64_t gc = S.mas_off[l - 1] + ch;
#pragma unroll
                    for (int c = 0; c < 9; ++c) E[c] += S.mas_ex[9 * gc + c];
                }
            if (l + 1 < S.mas_levels)  // the parent level reads the whole block
#pragma unroll
                for (int c = 0; c < 9; ++c) S.mas_ex[9 * g + c] = E[c];
            double Inv[9];
            inverse3(E, Inv);
#pragma unroll
            for (int c = 0; c < 9; ++c) Di[9 * g + c] = (R)Inv[c];
        }
        __syncthreads();  // the next level reads these blocks
    }
}

// ---- PCG B(it) --------------------------------------------------------------
// Blocks of a scene: [preconditioner groups | vertex blocks | a block per heavy
// incidence row]. With the multilevel preconditioner the vertex blocks cover
// the vertices outside the aggregates; without it, every vertex. Every block
// loads its vertices' data and contact sums first, then alpha from the d.q
// partials, then p += alpha d, r -= alpha q, z = D^-1 r (plus, in a group,
// the aggregate corrections) and its r.z partial. B(0) starts the solve
// from p = 0, r = -g instead.

// alpha = r.z / d.q for iteration it, d.q from the A launch's partials (its
// SpMV blocks, then its pair blocks) summed by the whole block: thread t adds
// partials t, t + 256, ... in order, a wavefront tree, then the wavefronts in
// order, so every block of the scene forms the same value. dq_issue loads a
// thread's first partials, the scene's done flag and r.z of iteration it - 1
// before the block's vertex loads; dq_stage adds them (and any rest) after
// those and leaves the wavefront sums in LDS; dq_alpha, after a block
// barrier, forms alpha.
constexpr int kDqU = 4;   // SpMV-block partials per thread in flight (1024: a scene of 65k vertices; the rest after)
constexpr int kDqUP = 1;  // pair-block partials per thread in flight
struct DqIssue {
    double part[kDqU], pair[kDqUP];
    double rz;
    int done;
};

__device__ __forceinline__ void dq_issue(const Launch &L, const SceneDev &S, int s, int it, DqIssue &q)
{
    const int t = (int)threadIdx.x, npart = S.nb_rows, npair = pair_blocks(L.out[s].n_pair);
#pragma unroll
    for (int u = 0; u < kDqU; ++u) q.part[u] = t + u * kBlock < npart ? glob(S.pcg_part)[t + u * kBlock] : 0.0;
#pragma unroll
    for (int u = 0; u < kDqUP; ++u) q.pair[u] = t + u * kBlock < npair ? glob(S.pcg_pair)[t + u * kBlock] : 0.0;
    q.rz = glob(S.pcg)->rzv[it & 1];  // stored by A(it)
    q.done = glob(S.pcg)->done;
}

__device__ __forceinline__ void dq_stage(const Launch &L, const SceneDev &S, int s, const DqIssue &q,
                                         double (&sh)[kBlock / kWave][2])
{
    const int t = (int)threadIdx.x, npart = S.nb_rows, npair = pair_blocks(L.out[s].n_pair);
    double a = 0.0, b = 0.0;
#pragma unroll
    for (int u = 0; u < kDqU; ++u)
        if (t + u * kBlock < npart) a += q.part[u];
    for (int i = t + kDqU * kBlock; i < npart; i += kBlock) a += glob(S.pcg_part)[i];
#pragma unroll
    for (int u = 0; u < kDqUP; ++u)
        if (t + u * kBlock < npair) b += q.pair[u];
    for (int i = t + kDqUP * kBlock; i < npair; i += kBlock) b += glob(S.pcg_pair)[i];
    a = wave_sum(a);
    b = wave_sum(b);
    if ((t & (kWave - 1)) == 0) {
        sh[t / kWave][0] = a;
        sh[t / kWave][1] = b;
    }
}

template <class R>
__device__ __forceinline__ R dq_alpha(const DqIssue &q, const double (&sh)[kBlock / kWave][2])
{
    double a = 0.0, b = 0.0;
#pragma unroll
    for (int w = 0; w < kBlock / kWave; ++w) {
        a += sh[w][0];
        b += sh[w][1];
    }
    return (R)(q.rz / (a + b));
}

// start of the solve for vertex i: r = -g, p = 0, z = D^-1 r; returns r.z
template <class R>
__device__ __forceinline__ double pcg_vertex_start(const SceneDev &S, int i, R zo[3], R ri[3])
{
    R *r = as<R>(S.r), *sol = as<R>(S.sol);
    const R *g = as<R>(S.grad), *Mi = as<R>(S.Minv);
    for (int c = 0; c < 3; ++c) ri[c] = -g[3 * i + c];
    double rz = 0.0;
    for (int a = 0; a < 3; ++a) {
        zo[a] = Mi[9 * i + 3 * a] * ri[0] + Mi[9 * i + 3 * a + 1] * ri[1] + Mi[9 * i + 3 * a + 2] * ri[2];
        rz += (double)ri[a] * (double)zo[a];
    }
    for (int c = 0; c < 3; ++c) {
        r[3 * i + c] = ri[c];
        sol[3 * i + c] = R(0);
    }
    return rz;
}

// LDS of an update block: the group's members' r, contact sums and
// corrections, the aggregate sums, the list of rows for the teams, and the
// group's level ranges (block-uniform; read in the level loop)
struct BShared {
    double rm[kMasCapM][3];
    double ra[kMasCapA][3];
    RowList rl;
    int32_t lv[kMasLevels][4];  // first aggregate, end, LDS base, offset of the level's aggregates
    double dq[kBlock / kWave][2];
};

template <class R>
__device__ void pcg_B_vertices(const Launch &L, const SceneDev &S, int s, int vb, int it, int lb, BShared &sh)
{
    int k = vb * blockDim.x + threadIdx.x;
    int i = S.mas_levels > 0 ? (k < S.mas_nother ? S.mas_other[k] : -1) : (k < S.n ? k : -1);
    double rz = 0.0;
    if (it == 0) {
        if (i >= 0) {
            R zo[3], ri[3];
            rz = pcg_vertex_start<R>(S, i, zo, ri);
            R *z = as<R>(S.z);
            for (int c = 0; c < 3; ++c) z[3 * i + c] = zo[c];
        }
    } else {
        const R *dcur = as<R>((it & 1) ? S.dA : S.dB);
        const auto Y = glob(as<R>(S.act_y));
        auto yv = [&](int p, int a, int c) { return (double)Y[12 * (int64_t)p + 3 * a + c]; };
        const bool contact = L.out[s].n_pair > 0;  // the same for the whole scene
        if (contact) {
            if (threadIdx.x == 0) sh.rl.count = 0;
            __syncthreads();
        }
        DqIssue dqi;
        dq_issue(L, S, s, it, dqi);
        bool own = i >= 0 && !glob(S.hflag)[i];  // a heavy row has a block of its own
        VertexPcg<R> v;
        double qc[3] = {0.0, 0.0, 0.0};
        bool listed = false;
        if (own) {
            pcg_vertex_load<R>(S, i, dcur, v);
            if (contact) listed = row_sum_or_list(S, i, (int)threadIdx.x, yv, qc, sh.rl);
        }
        if (dqi.done) return;
        dq_stage(L, S, s, dqi, sh.dq);
        __syncthreads();
        if (contact) {
            team_row_sums(S, sh.rl, yv, [&](int d, const double (&q)[3]) {
                for (int c = 0; c < 3; ++c) sh.rm[d][c] = q[c];
            });
            __syncthreads();
            if (listed)
                for (int c = 0; c < 3; ++c) qc[c] = sh.rm[threadIdx.x][c];
        }
        R alpha = dq_alpha<R>(dqi, sh.dq);
        if (own) rz = pcg_vertex_update<R>(S, i, alpha, v, qc);
    }
    rz = block_sum_all(rz);
    if (threadIdx.x == 0) glob(rz_slot(S, it))[lb] = rz;
}

template <class R>
__device__ void pcg_B_heavy(const Launch &L, const SceneDev &S, int s, int j, int it, BShared &sh)
{
    if (j >= L.out[s].n_heavy) return;
    int row = S.heavy_rows[j];
    // B(0) and the aggregate members (updated by their group) leave a zero partial
    if (it == 0 || (S.mas_levels > 0 && S.mas_vpos[row] >= 0)) {
        if (threadIdx.x == 0) rz_slot(S, it)[S.pcg_nvp + j] = 0.0;
        return;
    }
    const R *dcur = as<R>((it & 1) ? S.dA : S.dB);
    DqIssue dqi;
    dq_issue(L, S, s, it, dqi);
    double qc[3];
    contact_row_heavy<R>(S, row, qc);
    if (dqi.done) return;
    dq_stage(L, S, s, dqi, sh.dq);
    __syncthreads();
    R alpha = dq_alpha<R>(dqi, sh.dq);
    if (threadIdx.x == 0) {
        VertexPcg<R> v;
        pcg_vertex_load<R>(S, row, dcur, v);
        rz_slot(S, it)[S.pcg_nvp + j] = pcg_vertex_update<R>(S, row, alpha, v, qc);
    }
}

// a[l] of a per-level register array at a run-time level: selects, so the
// array stays in registers (dynamic indexing would move it to scratch)
__device__ __forceinline__ int lvl(const int (&a)[kMasLevels], int l)
{
    static_assert(kMasLevels == 3, "lvl selects among three levels");
    return l == 0 ? a[0] : (l == 1 ? a[1] : a[2]);
}

static_assert(kMasCapA <= kMasCapM, "corrections reuse the members' LDS rows");
static_assert(kMasCapM % kBlock == 0, "members per thread");
constexpr int kMasSlots = kMasCapM / kBlock;  // members per thread of a group block

// One group: the members' update, then restriction of the new r to every
// aggregate (members, then children, in order), e = E^-1 r_agg per aggregate,
// and z = D^-1 r + the corrections of the member's aggregates. The r.z
// partial is r.D^-1 r + sum over the group's aggregates of r_agg.e. The
// members' index data is loaded at the start, beside their vertex data; the
// aggregates' member ranges and inverses where they are used.
template <class R>
__device__ void pcg_B_group(const Launch &L, const SceneDev &S, int s, int grp, int it, BShared &sh)
{
    const int nl = S.mas_levels;
    const int tid = (int)threadIdx.x;
    int k0, k1;
    mas_group_range(S, grp, -1, k0, k1);
    // level ranges and LDS bases (each aggregate's member range is read in
    // the level loop: loaded up front, the ranges held enough registers to
    // cost a wavefront per SIMD)
    int ga0[kMasLevels], ga1[kMasLevels], gbase[kMasLevels];
    const R *Di = as<R>(S.mas_dinv);
    {
        int bsum = 0;
#pragma unroll
        for (int l = 0; l < kMasLevels; ++l) {
            int a0 = 0, a1 = 0;
            if (l < nl) mas_group_range(S, grp, l, a0, a1);
            ga0[l] = a0;
            ga1[l] = a1;
            gbase[l] = bsum;
            bsum += a1 - a0;
        }
    }
    if (tid < kMasLevels) {  // the level loop reads these from LDS (block-uniform)
        sh.lv[tid][0] = lvl(ga0, tid);
        sh.lv[tid][1] = lvl(ga1, tid);
        sh.lv[tid][2] = lvl(gbase, tid);
        sh.lv[tid][3] = S.mas_off[tid];
    }
    int vid[kMasSlots], loc[kMasSlots][kMasLevels];
    R zo[kMasSlots][3];
    double rz = 0.0;
#pragma unroll
    for (int j = 0; j < kMasSlots; ++j) {
        int k = k0 + tid + j * kBlock;
        vid[j] = k < k1 ? glob(S.mas_mem)[k] : -1;
#pragma unroll
        for (int l = 0; l < kMasLevels; ++l)
            loc[j][l] = (vid[j] >= 0 && l < nl) ? gbase[l] + glob(S.mas_manc)[(int64_t)l * S.mas_nf + k] - ga0[l] : 0;
    }
    if (it == 0) {
#pragma unroll
        for (int j = 0; j < kMasSlots; ++j)
            if (vid[j] >= 0) {
                R ri[3];
                rz += pcg_vertex_start<R>(S, vid[j], zo[j], ri);
                for (int c = 0; c < 3; ++c) sh.rm[tid + j * kBlock][c] = (double)ri[c];
            }
    } else {
        const bool contact = L.out[s].n_pair > 0;  // the same for the whole scene
        const auto Y = glob(as<R>(S.act_y));
        auto yv = [&](int p, int a, int c) { return (double)Y[12 * (int64_t)p + 3 * a + c]; };
        if (contact) {
            if (tid == 0) sh.rl.count = 0;
            __syncthreads();
        }
        DqIssue dqi;
        dq_issue(L, S, s, it, dqi);
        const R *dcur = as<R>((it & 1) ? S.dA : S.dB);
        VertexPcg<R> v[kMasSlots];
        double qc[kMasSlots][3];
        bool listed[kMasSlots];
#pragma unroll
        for (int j = 0; j < kMasSlots; ++j) {
            listed[j] = false;
            qc[j][0] = qc[j][1] = qc[j][2] = 0.0;
            if (vid[j] >= 0) {
                pcg_vertex_load<R>(S, vid[j], dcur, v[j]);
                if (contact) listed[j] = row_sum_or_list(S, vid[j], tid + j * kBlock, yv, qc[j], sh.rl);
            }
        }
        if (dqi.done) return;
        dq_stage(L, S, s, dqi, sh.dq);
        __syncthreads();
        if (contact) {
            team_row_sums(S, sh.rl, yv, [&](int d, const double (&q)[3]) {
                for (int c = 0; c < 3; ++c) sh.rm[d][c] = q[c];
            });
            __syncthreads();
        }
        R alpha = dq_alpha<R>(dqi, sh.dq);
        const auto sol = glob(as<R>(S.sol)), r = glob(as<R>(S.r));
#pragma unroll
        for (int j = 0; j < kMasSlots; ++j) {
            if (vid[j] < 0) continue;
            int i = vid[j], pos = tid + j * kBlock;
            if (listed[j])
                for (int c = 0; c < 3; ++c) qc[j][c] = sh.rm[pos][c];
            R ri[3];
            for (int c = 0; c < 3; ++c) {
                R qv = (R)((double)v[j].q[c] + qc[j][c]);
                sol[3 * i + c] = v[j].p[c] + alpha * v[j].d[c];
                ri[c] = v[j].r[c] - alpha * qv;
                r[3 * i + c] = ri[c];
            }
            for (int a = 0; a < 3; ++a) {
                zo[j][a] = v[j].M[3 * a] * ri[0] + v[j].M[3 * a + 1] * ri[1] + v[j].M[3 * a + 2] * ri[2];
                rz += (double)ri[a] * (double)zo[j][a];
            }
            for (int c = 0; c < 3; ++c) sh.rm[pos][c] = (double)ri[c];
        }
    }
    __syncthreads();
    // restriction and coarse solves, a barrier per level: the sums of level l
    // are formed while the corrections of level l - 1 are (not unrolled: the
    // unrolled form held every level's state in registers at once)
#pragma unroll 1
    for (int l = 0; l <= kMasLevels; ++l) {
        if (l > nl) break;
        if (l > 0) {
            const int pl = l - 1;
            const int g0 = sh.lv[pl][0], g1 = sh.lv[pl][1], gb = sh.lv[pl][2];
            for (int a = g0 + tid; a < g1; a += kBlock) {
                int lc = gb + a - g0;
                R D[9];
                const int64_t g = (int64_t)sh.lv[pl][3] + a;
#pragma unroll
                for (int c = 0; c < 9; ++c) D[c] = glob(Di)[9 * g + c];
                R sa[3] = {(R)sh.ra[lc][0], (R)sh.ra[lc][1], (R)sh.ra[lc][2]};
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    R e = D[3 * q] * sa[0] + D[3 * q + 1] * sa[1] + D[3 * q + 2] * sa[2];
                    sh.rm[lc][q] = (double)e;
                    rz += sh.ra[lc][q] * (double)e;
                }
            }
        }
        if (l < nl) {
            const int g0 = sh.lv[l][0], g1 = sh.lv[l][1], gb = sh.lv[l][2];
            const int c0 = l > 0 ? sh.lv[l - 1][0] : 0, cb = l > 0 ? sh.lv[l - 1][2] : 0;
            for (int a = g0 + tid; a < g1; a += kBlock) {
                const int64_t g = (int64_t)sh.lv[l][3] + a;
                const int j0 = glob(S.mas_mb)[g], j1 = glob(S.mas_me)[g];
                double acc[3] = {0.0, 0.0, 0.0};
                for (int j = j0; j < j1; ++j) {
                    const double *src = l == 0 ? sh.rm[j - k0] : sh.ra[cb + j - c0];
#pragma unroll
                    for (int c = 0; c < 3; ++c) acc[c] += src[c];
                }
#pragma unroll
                for (int c = 0; c < 3; ++c) sh.ra[gb + a - g0][c] = acc[c];
            }
        }
        __syncthreads();
    }
    // prolongation: z = D^-1 r + the corrections of the member's aggregates
    const auto z = glob(as<R>(S.z));
#pragma unroll
    for (int j = 0; j < kMasSlots; ++j) {
        if (vid[j] < 0) continue;
        double zi[3] = {(double)zo[j][0], (double)zo[j][1], (double)zo[j][2]};
#pragma unroll
        for (int l = 0; l < kMasLevels; ++l) {
            if (l >= nl) break;
#pragma unroll
            for (int c = 0; c < 3; ++c) zi[c] += sh.rm[loc[j][l]][c];
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) z[3 * vid[j] + c] = (R)zi[c];
    }
    rz = block_sum_all(rz);
    if (tid == 0) glob(rz_slot(S, it))[grp] = rz;
}

template <class R>
__global__ void __launch_bounds__(kBlock) k_pcg_B(Launch L, int it, int early)
{
    int lb, s = scene_of_block(L, lb);
    const SceneDev &S = *L.sc[s];
    if ((early || it > L.out[s].pcg_early) && it > 0 && S.pcg->done) return;
    if (it == 0 && lb == 0 && threadIdx.x == 0) {  // a new solve
        S.pcg->done = 0;
        S.pcg->iters = 0;
        S.pcg->stop = 0.0;
        L.out[s].pcg_done = 0;
        L.out[s].pcg_iters = 0;
    }
    __shared__ BShared sh;
    const int ngrp = S.mas_levels > 0 ? S.mas_ng : 0;
    if (lb < ngrp)
        pcg_B_group<R>(L, S, s, lb, it, sh);
    else if (lb < S.pcg_nvp)
        pcg_B_vertices<R>(L, S, s, lb - ngrp, it, lb, sh);
    else
        pcg_B_heavy<R>(L, S, s, lb - S.pcg_nvp, it, sh);
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
    int row = lb * kRowsPerBlock + (int)threadIdx.x;  // a thread per row, both slot streams
    if (row >= S.n) return;
    double o[3] = {0.0, 0.0, 0.0}, o1[3];
    bell_row_part<R>(S, row, 0, v, nullptr, R(0), false, o);
    bell_row_part<R>(S, row, 1, v, nullptr, R(0), false, o1);
    for (int c = 0; c < 3; ++c) y[3 * row + c] = (R)(o[c] + o1[c]);
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

// scene views put in place: block j copies view j of the staged block into
// the slot its pointer names, in 8-byte words
static_assert(sizeof(SceneDev) % 8 == 0, "views are copied in 8-byte words");
constexpr int kViewWords = (int)(sizeof(SceneDev) / 8);
__global__ void __launch_bounds__(kBlock) k_put_views(int n, const uint64_t *__restrict__ src)
{
    const int j = (int)blockIdx.x;
    uint64_t *dst = reinterpret_cast<uint64_t *>(src[j]);
    const uint64_t *from = src + view_head_bytes(n) / 8 + (int64_t)j * kViewWords;
    for (int w = (int)threadIdx.x; w < kViewWords; w += (int)blockDim.x) dst[w] = from[w];
}

// step start: keep x^t, inertial predictor for free gel vertices, indenter
// targets from the scene's pose, attached gel vertices' targets from the case
// pose
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
        if (S.attached && S.attached[i]) {  // the case pose applied to the rest position
            const double *X = S.X0 + 3 * i, *P = S.case_pose;
            for (int c = 0; c < 3; ++c)
                S.yhat[3 * i + c] = P[c * 4 + 0] * X[0] + P[c * 4 + 1] * X[1] + P[c * 4 + 2] * X[2] + P[c * 4 + 3];
        }
    } else {
        const double *y = S.Yloc + 3 * (i - S.n_gel);
        const double *P = S.pose;
        for (int c = 0; c < 3; ++c) {
            S.yhat[3 * i + c] = P[c * 4 + 0] * y[0] + P[c * 4 + 1] * y[1] + P[c * 4 + 2] * y[2] + P[c * 4 + 3];
            S.xtilde[3 * i + c] = S.x[3 * i + c];
            if (S.target_al) S.al_lam[3 * i + c] = 0.0;
        }
    }
}

// augmented-Lagrangian targets: lambda_j -= k_t (y_j - yhat_j) for the
// indenter vertices of the scenes in the launch
__global__ void k_al_update(Launch L)
{
    int lb, s = scene_of_block(L, lb);
    const SceneDev &S = *L.sc[s];
    int i = S.n_gel + lb * blockDim.x + threadIdx.x;
    if (i >= S.n) return;
    for (int c = 0; c < 3; ++c) S.al_lam[3 * i + c] -= S.k_target * (S.x[3 * i + c] - S.yhat[3 * i + c]);
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

void launch_al_update(Batch &b, const std::vector<uint8_t> &on)
{
    std::vector<int32_t> nb(b.sc.size(), 0);
    for (size_t i = 0; i < b.sc.size(); ++i)
        if (on[i]) nb[i] = nblocks(std::max(b.sc[i]->h.n_ind, 1));
    b.set_phase(kPhOne, nb);
    IPC_LAUNCH(b, k_al_update, kPhOne, kBlock);
}

void launch_trial(Batch &b)
{
    if (mixed(b))
        IPC_LAUNCH(b, k_trial<float>, kPhVert, kBlock, (const double *)b.d_alpha);
    else
        IPC_LAUNCH(b, k_trial<double>, kPhVert, kBlock, (const double *)b.d_alpha);
}

void launch_accept(Batch &b) { IPC_LAUNCH(b, k_accept, kPhVert, kBlock); }

void launch_put_views(hipStream_t strm, int n, const void *d_src)
{
    if (n > 0)
        hipLaunchKernelGGL(k_put_views, dim3(n), dim3(kBlock), 0, strm, n, static_cast<const uint64_t *>(d_src));
}

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
    if (mixed(b)) {
        IPC_LAUNCH(b, k_mas_diag<float>, kPhMas, kBlock);
        IPC_LAUNCH(b, k_mas_invert<float>, kPhMasG, kBlock);
    } else {
        IPC_LAUNCH(b, k_mas_diag<double>, kPhMas, kBlock);
        IPC_LAUNCH(b, k_mas_invert<double>, kPhMasG, kBlock);
    }
}

void launch_hess_apply(Batch &b)
{
    // pair phase as set by the incidence build of the same assembly
    if (mixed(b)) {
        IPC_LAUNCH(b, k_spmv_pairs<float>, kPhActT, kBlock);
        IPC_LAUNCH(b, k_spmv_rows<float>, kPhSlice, kRowsPerBlock);
        IPC_LAUNCH(b, k_spmv_contact<float>, kPhVertH, kBlock);
    } else {
        IPC_LAUNCH(b, k_spmv_pairs<double>, kPhActT, kBlock);
        IPC_LAUNCH(b, k_spmv_rows<double>, kPhSlice, kRowsPerBlock);
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
        if (b.h_off[kPhVert][i + 1] > b.h_off[kPhVert][i]) nab[i] = b.sc[i]->h.nb_rows + nblocks(pair_count(*b.sc[i], b.h_out[i]), kPairsPerBlock);
    b.set_phase(kPhPcgA, nab);
    set_heavy_phase(b);
    std::vector<int32_t> nbb(ns, 0);
    for (size_t i = 0; i < ns; ++i)
        if (nab[i] > 0) nbb[i] = b.sc[i]->h.pcg_nvp + heavy_bound(pair_count(*b.sc[i], b.h_out[i]), b.sc[i]->h.n);
    b.set_phase(kPhPcgB, nbb);
    if (mx)
        IPC_LAUNCH(b, k_pcg_B<float>, kPhPcgB, kBlock, 0, 0);
    else
        IPC_LAUNCH(b, k_pcg_B<double>, kPhPcgB, kBlock, 0, 0);
    int maxit = 0, last = 0;
    for (size_t i = 0; i < ns; ++i) {
        if (b.h_off[kPhVert][i + 1] == b.h_off[kPhVert][i]) continue;
        const Scene &s = *b.sc[i];
        maxit = std::max(maxit, s.h.pcg_maxit);
        last = std::max(last, s.last_pcg_iters);
    }
    iters.assign(ns, 0);
    hit_cap.assign(ns, 0);
    // algorithmic bytes of one scene in one A launch: every stored 3x3 block
    // (values and column) once; per vertex the z and d gathers, the d and q
    // writes and its row pointer; per pair its off-diagonal blocks and ids
    // and of one B launch: per vertex q, d, p, r and the 3x3 inverse read and
    // p, r, z written (30 reals); per incidence entry (4 per pair) its index
    // and 3 pair-product values; per preconditioner member its vertex id and
    // three level ids; the SpMV blocks' d.q partials
    std::vector<double> scene_bytes(ns, 0.0), scene_bytes_b(ns, 0.0);
    {
        const double rs = mx ? 4.0 : 8.0;
        for (size_t i = 0; i < ns; ++i) {
            if (nab[i] == 0) continue;
            const Scene &s = *b.sc[i];
            const double np_ = (double)pair_count(s, b.h_out[i]);
            scene_bytes[i] = (9 * rs + 4) * (double)s.nnzb + (12 * rs + 4) * (double)s.h.n + (108 * rs + 16) * np_;
            scene_bytes_b[i] = 30 * rs * (double)s.h.n + 4 * (4 + 3 * rs) * np_ +
                               16.0 * (s.h.mas_levels > 0 ? (double)s.h.mas_nf : 0.0) + 8.0 * (double)s.h.nb_rows;
        }
    }
    // Timed A launches of a chunk get their bytes once the chunk's flags are
    // back: a scene counts in the launch of iteration it when its solve was
    // still running there (not finished, or finished with more than it - 1
    // iterations); finished solves exit before their first load.
    std::vector<std::pair<size_t, int>> timed_a, timed_b;  // (pending event index, it)
    auto launch_bytes = [&](const std::vector<double> &sb, int it_) {
        double v = 0.0;
        for (size_t i = 0; i < ns; ++i) {
            if (sb[i] == 0.0) continue;
            if (!b.h_out[i].pcg_done || it_ <= b.h_out[i].pcg_iters) v += sb[i];
        }
        return v;
    };
    auto settle = [&](std::vector<std::pair<size_t, int>> &timed, const std::vector<double> &sb) {
        for (auto &ta : timed) {
            b.ev_pending[ta.first].bytes = launch_bytes(sb, ta.second);
            // an iteration above the Infinity Cache: its SpMV launch's bytes decide
            b.ev_pending[ta.first].big = launch_bytes(scene_bytes, ta.second) >= kProfBigBytes;
        }
        timed.clear();
    };
    auto settle_bytes = [&]() {
        settle(timed_a, scene_bytes);
        settle(timed_b, scene_bytes_b);
    };
    // large lists are bandwidth-bound: a thread per row reads the slices fully coalesced
    // (lanes per row and chunk lengths from the tuning of the list's largest scene)
    int64_t rows_total = 0;
    const Scene *big = nullptr;
    for (size_t i = 0; i < ns; ++i)
        if (nab[i] > 0) {
            rows_total += b.sc[i]->h.n;
            if (!big || b.sc[i]->h.n > big->h.n) big = b.sc[i];
        }
    const Tuning tn = big ? big->tune : Tuning{};
    const bool one_lane = rows_total >= tn.spmv_one_lane_rows;
    int it = 1;
    // Chunk lengths: a quantile (tuned) of the running scenes' expected
    // remaining iterations (their previous solve's count minus the launches
    // done) times a fraction, at least 8. A short chunk costs a read-back; a
    // long one keeps finished scenes' blocks in the launches (they exit at
    // once, but still take dispatch slots). One scene: the fraction of its own
    // previous count.
    auto next_chunk = [&](double frac) {
        std::vector<int> rem;
        for (size_t i = 0; i < ns; ++i)
            if (nab[i] > 0 && !(it > 1 && b.h_out[i].pcg_done)) rem.push_back(std::max(0, b.sc[i]->last_pcg_iters - (it - 1)));
        if (rem.empty()) return 8;
        std::sort(rem.begin(), rem.end());
        size_t k = (size_t)(tn.pcg_list_quantile * (double)(rem.size() - 1) + 0.5);
        return std::max(8, (int)(frac * rem[std::min(k, rem.size() - 1)]));
    };
    int chunk = last > 16 ? next_chunk(tn.pcg_first_chunk) : 8;
    int early = 0;
    // every launch of a chunk, with the algorithmic bytes of the scenes whose
    // solve was running there (when profiling)
    auto account_chunk = [&](int it0, int it1) {
        if (!b.prof()) return;
        double ba = 0.0, bb = 0.0;
        for (int j = it0; j < it1; ++j)
            for (size_t i = 0; i < ns; ++i) {
                if (nab[i] == 0) continue;
                if (!b.h_out[i].pcg_done || j <= b.h_out[i].pcg_iters) {
                    ba += scene_bytes[i];
                    bb += scene_bytes_b[i];
                }
            }
        b.prof_totals(kProfPcgA, it1 - it0, ba);
        b.prof_totals(kProfPcgB, it1 - it0, bb);
    };
    hipEvent_t ev[2];
    // launch it = maxit + 1 too: its A kernel records the cap of the scenes
    // that did not converge
    while (it <= maxit + 1) {
        int c = std::min(chunk, maxit + 2 - it);
        const int it_chunk = it;
        for (int j = 0; j < c; ++j, ++it) {
            // time one launch in sixteen when profiling: iterations 2, 18, 34, ...
            // of the first chunk (the first iteration applies the matrix to one
            // vector only; later chunks may skip finished scenes early)
            bool timed = b.prof() && (it & 15) == 2 && !early;
            if (timed) b.prof_begin(kProfPcgA, ev);
            if (timed) timed_a.push_back({b.ev_pending.size(), it});
            if (one_lane) {
                if (mx)
                    IPC_LAUNCH(b, (k_pcg_A<float, 1>), kPhPcgA, kRowsPerBlock, it, early);
                else
                    IPC_LAUNCH(b, (k_pcg_A<double, 1>), kPhPcgA, kRowsPerBlock, it, early);
            } else {
                if (mx)
                    IPC_LAUNCH(b, (k_pcg_A<float, 2>), kPhPcgA, 2 * kRowsPerBlock, it, early);
                else
                    IPC_LAUNCH(b, (k_pcg_A<double, 2>), kPhPcgA, 2 * kRowsPerBlock, it, early);
            }
            if (timed) b.prof_end(kProfPcgA, ev, 0.0);
            if (timed) b.prof_begin(kProfPcgB, ev);
            if (timed) timed_b.push_back({b.ev_pending.size(), it});
            if (mx)
                IPC_LAUNCH(b, k_pcg_B<float>, kPhPcgB, kBlock, it, early);
            else
                IPC_LAUNCH(b, k_pcg_B<double>, kPhPcgB, kBlock, it, early);
            if (timed) b.prof_end(kProfPcgB, ev);
        }
        run_pinf(b);  // |p|_inf of the scenes done so far comes back with their flags
        b.read_out();
        settle_bytes();
        account_chunk(it_chunk, it);
        b.prof_collect();
        bool all = true;
        for (size_t i = 0; i < ns; ++i)
            if (b.h_off[kPhVert][i + 1] > b.h_off[kPhVert][i] && !b.h_out[i].pcg_done) all = false;
        if (all) break;
        chunk = next_chunk(tn.pcg_later_chunk);
        early = 1;
        // scenes that finished leave the remaining launches of the list
        bool shrink = false;
        for (size_t i = 0; i < ns; ++i)
            if (nab[i] > 0 && b.h_out[i].pcg_done) {
                nab[i] = nbb[i] = 0;
                shrink = true;
            }
        if (shrink) {
            b.set_phase(kPhPcgA, nab);
            b.set_phase(kPhPcgB, nbb);
        }
    }
    for (size_t i = 0; i < ns; ++i) {
        if (b.h_off[kPhVert][i + 1] == b.h_off[kPhVert][i]) continue;
        iters[i] = b.h_out[i].pcg_done ? b.h_out[i].pcg_iters : b.sc[i]->h.pcg_maxit;
        hit_cap[i] = b.h_out[i].pcg_done != 1;
        b.sc[i]->last_pcg_iters = iters[i];
    }
}

}  // namespace ipcg
