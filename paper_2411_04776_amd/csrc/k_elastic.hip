// k_elastic.hip -- Neo-Hookean element kernel and deterministic assembly.
//
// Energy density (compressible Neo-Hookean, the IPC model's inversion-free
// elasticity cited in the paper's "Choice of the Simulation Methods"):
//   Psi(F) = mu/2 (|F|^2 - 3) - mu ln J + lam/2 (ln J)^2.
// Its Hessian d2Psi/dF2 is projected onto the PSD cone before the chain rule
// to the 12 vertex DOFs (H_e = V D^T Pi+(d2Psi/dF2) D).
//
// gfx950 design: one thread per tet, no 9x9 numeric eigensolver. With
// F = U diag(s) V^T, the 9x9 Hessian splits in the (U,V) frame into a 3x3
// "scaling" block D_ii = mu + (mu - lam lnJ + lam)/s_i^2, D_ij = lam/(s_i s_j)
// and three 2x2 blocks on (Y_ij, Y_ji) with eigenvalues
// mu +- (mu - lam lnJ)/(s_i s_j) and eigenmatrices U (E_ij +- E_ji) V^T / sqrt2.
// The projection clamps these nine eigenvalues; because the PSD projection is
// unique it equals a numeric eigen-decomposition of the 9x9 matrix. The SVD
// comes from a Jacobi eigen-decomposition of F^T F and a Gram-Schmidt QR of FV.
// The element kernel runs in the scene's real type R (FP32 in the mixed form,
// with deformation gradients formed from FP64 position differences).
//
// Element outputs are written SoA (component-major) and summed per matrix
// block / per vertex by gather kernels in a fixed order: no float atomics.
#include "device_util.h"
#include "incidence.h"
#include "ipc_internal.h"

namespace ipcg {

template <class R>
__device__ __forceinline__ R *as(void *p)
{
    return reinterpret_cast<R *>(p);
}

template <class R>
__device__ __forceinline__ R jacobi_rel_tol2();
template <>
__device__ __forceinline__ double jacobi_rel_tol2<double>() { return 1e-36; }
template <>
__device__ __forceinline__ float jacobi_rel_tol2<float>() { return 1e-15f; }

template <class R>
__device__ __forceinline__ void jacobi_rot3(R A[3][3], R V[3][3], int p, int q)
{
    R apq = A[p][q];
    if (apq == R(0)) return;
    R theta = (A[q][q] - A[p][p]) / (R(2) * apq);
    R t = (theta >= R(0) ? R(1) : R(-1)) / (fabs(theta) + sqrt(theta * theta + R(1)));
    R c = R(1) / sqrt(t * t + R(1)), s = t * c;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        R akp = A[k][p], akq = A[k][q];
        A[k][p] = c * akp - s * akq;
        A[k][q] = s * akp + c * akq;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        R apk = A[p][k], aqk = A[q][k];
        A[p][k] = c * apk - s * aqk;
        A[q][k] = s * apk + c * aqk;
    }
    A[p][q] = A[q][p] = R(0);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        R vkp = V[k][p], vkq = V[k][q];
        V[k][p] = c * vkp - s * vkq;
        V[k][q] = s * vkp + c * vkq;
    }
}

// symmetric 3x3 eigen-decomposition by cyclic Jacobi; V columns = vectors
template <class R>
__device__ void sym3_eig(R A[3][3], R V[3][3], R w[3])
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) V[i][j] = (i == j) ? R(1) : R(0);
    for (int sweep = 0; sweep < 20; ++sweep) {
        R off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
        R dg = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
        if (off <= jacobi_rel_tol2<R>() * dg) break;
        jacobi_rot3(A, V, 0, 1);
        jacobi_rot3(A, V, 0, 2);
        jacobi_rot3(A, V, 1, 2);
    }
    w[0] = A[0][0];
    w[1] = A[1][1];
    w[2] = A[2][2];
}

// F = U diag(s) V^T with det U = det V = +1 (requires det F > 0)
template <class R>
__device__ void svd3(const R F[3][3], R U[3][3], R s[3], R V[3][3])
{
    R S[3][3], w[3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) S[i][j] = F[0][i] * F[0][j] + F[1][i] * F[1][j] + F[2][i] * F[2][j];
    sym3_eig(S, V, w);
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2 - a; ++b)
            if (w[b] < w[b + 1]) {
                R t = w[b];
                w[b] = w[b + 1];
                w[b + 1] = t;
                for (int k = 0; k < 3; ++k) {
                    R u = V[k][b];
                    V[k][b] = V[k][b + 1];
                    V[k][b + 1] = u;
                }
            }
    R dv = V[0][0] * (V[1][1] * V[2][2] - V[1][2] * V[2][1]) - V[0][1] * (V[1][0] * V[2][2] - V[1][2] * V[2][0]) +
           V[0][2] * (V[1][0] * V[2][1] - V[1][1] * V[2][0]);
    if (dv < R(0))
        for (int k = 0; k < 3; ++k) V[k][2] = -V[k][2];
    R B[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) B[i][j] = F[i][0] * V[0][j] + F[i][1] * V[1][j] + F[i][2] * V[2][j];
    R n0 = sqrt(B[0][0] * B[0][0] + B[1][0] * B[1][0] + B[2][0] * B[2][0]);
    R u0[3] = {B[0][0] / n0, B[1][0] / n0, B[2][0] / n0};
    R pr = u0[0] * B[0][1] + u0[1] * B[1][1] + u0[2] * B[2][1];
    R t1[3] = {B[0][1] - pr * u0[0], B[1][1] - pr * u0[1], B[2][1] - pr * u0[2]};
    R n1 = sqrt(t1[0] * t1[0] + t1[1] * t1[1] + t1[2] * t1[2]);
    R u1[3] = {t1[0] / n1, t1[1] / n1, t1[2] / n1};
    R u2[3] = {u0[1] * u1[2] - u0[2] * u1[1], u0[2] * u1[0] - u0[0] * u1[2], u0[0] * u1[1] - u0[1] * u1[0]};
    s[0] = n0;
    s[1] = u1[0] * B[0][1] + u1[1] * B[1][1] + u1[2] * B[2][1];
    s[2] = u2[0] * B[0][2] + u2[1] * B[1][2] + u2[2] * B[2][2];
    for (int k = 0; k < 3; ++k) {
        U[k][0] = u0[k];
        U[k][1] = u1[k];
        U[k][2] = u2[k];
    }
}

// block index of the (a,b) 3x3 block, a <= b, in the 10-block element layout:
// diagonal a = 0..3, then (0,1)4 (0,2)5 (0,3)6 (1,2)7 (1,3)8 (2,3)9
__host__ __device__ __forceinline__ int elem_block(int a, int b)
{
    if (a == b) return a;
    return a == 0 ? 3 + b : (a == 1 ? 5 + b : 9);
}

// F = Ds Bm with Ds = [x1-x0, x2-x0, x3-x0] (differences in FP64), and the
// rows q_a of dF/dx (q_0 = -sum of the rows of Bm)
template <class R>
__device__ __forceinline__ void tet_F(const SceneDev &S, const double *x, int e, R F[3][3], R q[4][3], double Fd[9])
{
    int m = S.m;
    int v0 = S.tv[e], v1 = S.tv[m + e], v2 = S.tv[2 * m + e], v3 = S.tv[3 * m + e];
    double B[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) B[k] = S.Bm[(int64_t)k * m + e];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        double x0 = x[3 * v0 + i];
        double d1 = x[3 * v1 + i] - x0, d2 = x[3 * v2 + i] - x0, d3 = x[3 * v3 + i] - x0;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            Fd[i * 3 + j] = d1 * B[0 * 3 + j] + d2 * B[1 * 3 + j] + d3 * B[2 * 3 + j];
            F[i][j] = (R)Fd[i * 3 + j];
        }
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        q[1][j] = (R)B[0 * 3 + j];
        q[2][j] = (R)B[1 * 3 + j];
        q[3][j] = (R)B[2 * 3 + j];
        q[0][j] = (R)(-(B[0 * 3 + j] + B[1 * 3 + j] + B[2 * 3 + j]));
    }
}

template <class R>
__global__ void __launch_bounds__(kBlock) k_elastic_elements(Launch L)
{
    int lb, s = scene_of_block(L, lb);
    const SceneDev &S = *L.sc[s];
    int e = lb * blockDim.x + threadIdx.x;
    int m = S.m;
    if (e >= m) return;
    R *eg = as<R>(S.eg), *eH = as<R>(S.eH);
    R F[3][3], q[4][3];
    double Fd[9];
    tet_F<R>(S, S.x, e, F, q, Fd);
    R V = (R)S.vol[e];
    R mu = (R)S.mu, lam = (R)S.lam;
    R Fm[9] = {F[0][0], F[0][1], F[0][2], F[1][0], F[1][1], F[1][2], F[2][0], F[2][1], F[2][2]};
    double Jd = det3(Fd);
    if (!(Jd > 0.0)) {
        // infeasible state: the line search never accepts one; write zeros
        for (int k = 0; k < 12; ++k) eg[(int64_t)k * m + e] = R(0);
        for (int k = 0; k < 90; ++k) eH[(int64_t)k * m + e] = R(0);
        return;
    }
    R J = (R)Jd;
    R lnJ = (R)log(Jd);
    // F^-T by the adjugate
    R Fi[9];
    {
        R c00 = Fm[4] * Fm[8] - Fm[5] * Fm[7], c01 = Fm[5] * Fm[6] - Fm[3] * Fm[8], c02 = Fm[3] * Fm[7] - Fm[4] * Fm[6];
        R id = R(1) / J;
        Fi[0] = c00 * id;
        Fi[1] = (Fm[2] * Fm[7] - Fm[1] * Fm[8]) * id;
        Fi[2] = (Fm[1] * Fm[5] - Fm[2] * Fm[4]) * id;
        Fi[3] = c01 * id;
        Fi[4] = (Fm[0] * Fm[8] - Fm[2] * Fm[6]) * id;
        Fi[5] = (Fm[2] * Fm[3] - Fm[0] * Fm[5]) * id;
        Fi[6] = c02 * id;
        Fi[7] = (Fm[1] * Fm[6] - Fm[0] * Fm[7]) * id;
        Fi[8] = (Fm[0] * Fm[4] - Fm[1] * Fm[3]) * id;
    }
    // P = mu (F - F^-T) + lam lnJ F^-T; element gradient V P q_a
    R P[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            R fit = Fi[j * 3 + i];
            P[i][j] = mu * (F[i][j] - fit) + lam * lnJ * fit;
        }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            eg[(int64_t)(a * 3 + c) * m + e] = V * (P[c][0] * q[a][0] + P[c][1] * q[a][1] + P[c][2] * q[a][2]);

    // analytic eigensystem of d2Psi/dF2 in the SVD frame
    R U[3][3], sg[3], Vv[3][3];
    svd3<R>(F, U, sg, Vv);
    R cc = mu - lam * lnJ;
    R Dm[3][3], W[3][3], ev[3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) Dm[i][j] = (i == j) ? mu + (cc + lam) / (sg[i] * sg[i]) : lam / (sg[i] * sg[j]);
    sym3_eig<R>(Dm, W, ev);
    R sa[4][3];  // V^T q_a
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int k = 0; k < 3; ++k) sa[a][k] = Vv[0][k] * q[a][0] + Vv[1][k] * q[a][1] + Vv[2][k] * q[a][2];

    R H[10][9];
#pragma unroll
    for (int b = 0; b < 10; ++b)
#pragma unroll
        for (int k = 0; k < 9; ++k) H[b][k] = R(0);

    const R inv_sqrt2 = (R)0.70710678118654752440;
    for (int mode = 0; mode < 9; ++mode) {
        R lamk;
        R t[4][3];
        if (mode < 3) {
            lamk = ev[mode];
            if (!(lamk > R(0))) continue;
            for (int a = 0; a < 4; ++a)
                for (int k = 0; k < 3; ++k) t[a][k] = W[k][mode] * sa[a][k];
        } else {
            int pair = (mode - 3) >> 1, sgn = ((mode - 3) & 1) ? -1 : 1;
            int i = pair == 2 ? 1 : 0, j = pair == 0 ? 1 : 2;
            lamk = mu + (R)sgn * cc / (sg[i] * sg[j]);
            if (!(lamk > R(0))) continue;
            for (int a = 0; a < 4; ++a) {
                t[a][0] = t[a][1] = t[a][2] = R(0);
                t[a][i] = sa[a][j] * inv_sqrt2;
                t[a][j] = (R)sgn * sa[a][i] * inv_sqrt2;
            }
        }
        R gk[4][3];
        for (int a = 0; a < 4; ++a)
            for (int k = 0; k < 3; ++k) gk[a][k] = U[k][0] * t[a][0] + U[k][1] * t[a][1] + U[k][2] * t[a][2];
        R sc = V * lamk;
        for (int a = 0; a < 4; ++a)
            for (int b = a; b < 4; ++b) {
                int blk = elem_block(a, b);
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) H[blk][i * 3 + j] += sc * gk[a][i] * gk[b][j];
            }
    }
#pragma unroll
    for (int b = 0; b < 10; ++b)
#pragma unroll
        for (int k = 0; k < 9; ++k) eH[(int64_t)(b * 9 + k) * m + e] = H[b][k];
}

// Gradient gather: one thread per vertex; elastic element gradients in
// vertex-incidence (tet) order, then inertia / kinematic target, then the sum
// of the vertex's active contact pairs in pair order. Sums in FP64,
// stored in R. A heavy incidence row gets a block of its own after the vertex
// blocks, which also sums the contact diagonal blocks of that row (hdiag).
template <class R>
__device__ __forceinline__ void vertex_gradient(const SceneDev &S, int i, double g[3])
{
    const R *eg = as<R>(S.eg);
    for (int k = S.vt_ptr[i]; k < S.vt_ptr[i + 1]; ++k) {
        int src = S.vt_src[k], e = src >> 2, a = src & 3;
        for (int c = 0; c < 3; ++c) g[c] += (double)eg[(int64_t)(a * 3 + c) * S.m + e];
    }
    if (i < S.n_gel) {
        double kk = S.mass[i] * S.inv_h2;
        for (int c = 0; c < 3; ++c) g[c] += kk * (S.x[3 * i + c] - S.xtilde[3 * i + c]);
        if (S.attached && S.attached[i])
            for (int c = 0; c < 3; ++c) g[c] += S.k_target * (S.x[3 * i + c] - S.yhat[3 * i + c]);
    } else {
        for (int c = 0; c < 3; ++c) g[c] += S.k_target * (S.x[3 * i + c] - S.yhat[3 * i + c]);
        if (S.target_al)
            for (int c = 0; c < 3; ++c) g[c] -= S.al_lam[3 * i + c];
    }
}

template <class R>
__global__ void __launch_bounds__(kBlock) k_assemble_gradient(Launch L)
{
    int lb, s = scene_of_block(L, lb);
    const SceneDev &S = *L.sc[s];
    const R *ag = as<R>(S.act_g), *aH = as<R>(S.act_H);
    const int64_t cap = S.act_cap;
    R *grad = as<R>(S.grad);
    if (lb < S.nb_vert) {
        int i = lb * blockDim.x + threadIdx.x;
        if (i >= S.n || S.hflag[i]) return;
        double g[3] = {0.0, 0.0, 0.0};
        if (!S.fixed[i]) {
            double gc[3] = {0.0, 0.0, 0.0};
            thread_row_sums<3>(S, i, [&](int p, int a, int c) { return (double)ag[(int64_t)(a * 3 + c) * cap + p]; }, gc);
            vertex_gradient<R>(S, i, g);
            for (int c = 0; c < 3; ++c) g[c] += gc[c];
        }
        for (int c = 0; c < 3; ++c) grad[3 * i + c] = (R)g[c];
    } else {
        int j = lb - S.nb_vert;
        if (j >= L.out[s].n_heavy) return;
        int row = S.heavy_rows[j];  // never a fixed vertex: those have no incidence entries
        double gc[12];
        block_row_sums<12>(S, row,
                           [&](int p, int a, int c) {
                               if (c < 3) return (double)ag[(int64_t)(a * 3 + c) * cap + p];
                               int ii = (c - 3) / 3, jj = (c - 3) % 3;
                               return (double)aH[(int64_t)((3 * a + ii) * 12 + 3 * a + jj) * cap + p];
                           },
                           gc);
        if (threadIdx.x == 0) {
            double g[3] = {0.0, 0.0, 0.0};
            vertex_gradient<R>(S, row, g);
            for (int c = 0; c < 3; ++c) grad[3 * row + c] = (R)(g[c] + gc[c]);
            for (int c = 0; c < 9; ++c) S.hdiag[9 * (int64_t)j + c] = gc[3 + c];
        }
    }
}

// Matrix gather: one thread per stored BELL block. Sums the element blocks
// listed for this (row, col) in tet order; the diagonal block also takes the
// inertia / target term and the contact diagonal blocks, and writes the
// inverse used by the block-Jacobi preconditioner. Fixed rows/cols become
// identity / zero.
template <class R>
__global__ void __launch_bounds__(kBlock) k_assemble_bell(Launch L)
{
    int lb, s = scene_of_block(L, lb);
    const SceneDev &S = *L.sc[s];
    int64_t slot_lane = (int64_t)lb * blockDim.x + threadIdx.x;
    int64_t total = (int64_t)S.n_slots * kSlice;
    if (slot_lane >= total) return;
    int64_t slot = slot_lane / kSlice;
    int lane = (int)(slot_lane % kSlice);
    int lo = 0, hi = S.n_slices;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (S.slice_ptr[mid] <= slot) lo = mid; else hi = mid;
    }
    int row = lo * kSlice + lane;
    int k = (int)(slot - S.slice_ptr[lo]);
    int col = S.bcol[slot_lane];
    const R *eH = as<R>(S.eH), *aH = as<R>(S.act_H);
    // contact diagonal blocks (slot 0 is the diagonal)
    double cd[9];
    for (int c = 0; c < 9; ++c) cd[c] = 0.0;
    if (k == 0 && row < S.n) {
        const int64_t cap = S.act_cap;
        if (S.hflag[row]) {  // summed by the row's own block in the gradient kernel
            for (int c = 0; c < 9; ++c) cd[c] = S.hdiag[9 * (int64_t)S.heavy_idx[row] + c];
        } else {
            // one entry's nine loads at a time: four entries in flight held
            // registers for half of the kernel's resident wavefronts, and
            // only the diagonal lanes of contact rows take this path
            auto dblk = [&](int p, int a, int c) {
                int i = c / 3, j = c % 3;
                return (double)aH[(int64_t)((3 * a + i) * 12 + 3 * a + j) * cap + p];
            };
            thread_row_sums<9, decltype(dblk), 1>(S, row, dblk, cd);
        }
    }
    double A[9];
    for (int c = 0; c < 9; ++c) A[c] = 0.0;
    if (col >= 0) {
        for (int t = S.g_ptr[slot_lane]; t < S.g_ptr[slot_lane + 1]; ++t) {
            int src = S.g_src[t];
            int e = src >> 4, a = (src >> 2) & 3, b = src & 3;
            if (a <= b) {
                int blk = elem_block(a, b);
                for (int c = 0; c < 9; ++c) A[c] += (double)eH[(int64_t)(blk * 9 + c) * S.m + e];
            } else {
                int blk = elem_block(b, a);
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) A[i * 3 + j] += (double)eH[(int64_t)(blk * 9 + j * 3 + i) * S.m + e];
            }
        }
        if (k == 0) {
            double dk = row < S.n_gel ? S.mass[row] * S.inv_h2 : S.k_target;
            if (row < S.n_gel && S.attached && S.attached[row]) dk += S.k_target;
            A[0] += dk;
            A[4] += dk;
            A[8] += dk;
            for (int c = 0; c < 9; ++c) A[c] += cd[c];
        }
        if (S.fixed[row] || S.fixed[col]) {
            for (int c = 0; c < 9; ++c) A[c] = 0.0;
            if (k == 0) A[0] = A[4] = A[8] = 1.0;
        }
    }
    R *bval = as<R>(S.bval);
    for (int c = 0; c < 9; ++c) bval[(slot * 9 + c) * kSlice + lane] = (R)A[c];
    if (k == 0 && row < S.n) {
        double Inv[9];
        inverse3(A, Inv);
        R *Mi = as<R>(S.Minv);
        for (int c = 0; c < 9; ++c) Mi[9 * row + c] = (R)Inv[c];
    }
}

// Rest shape: Bm = Dm^-1 (row-major, FP64), V = det(Dm)/6.
__global__ void k_rest_tets(Launch L)
{
    int lb, s = scene_of_block(L, lb);
    const SceneDev &S = *L.sc[s];
    int e = lb * blockDim.x + threadIdx.x;
    int m = S.m;
    if (e >= m) return;
    int v[4];
    for (int a = 0; a < 4; ++a) v[a] = S.tv[(int64_t)a * m + e];
    double D[9];
    for (int i = 0; i < 3; ++i)
        for (int c = 0; c < 3; ++c) D[i * 3 + c] = S.X0[3 * v[c + 1] + i] - S.X0[3 * v[0] + i];
    double Inv[9];
    double det = inverse3(D, Inv);
    for (int k = 0; k < 9; ++k) S.Bm[(int64_t)k * m + e] = Inv[k];
    S.vol[e] = det / 6.0;
}

// lumped mass: rho V / 4 per incident tet, gathered per vertex
__global__ void k_rest_mass(Launch L)
{
    int lb, s = scene_of_block(L, lb);
    const SceneDev &S = *L.sc[s];
    int i = lb * blockDim.x + threadIdx.x;
    if (i >= S.n) return;
    double acc = 0.0;
    for (int k = S.vt_ptr[i]; k < S.vt_ptr[i + 1]; ++k) acc += S.rho * S.vol[S.vt_src[k] >> 2] / 4.0;
    S.mass[i] = acc;
}

// Elastic + inertia + target terms of the incremental potential (FP64), per
// item, into compensated block partials S.red[2 lb], S.red[2 lb + 1]. Items:
// tets, then vertices. out.infeasible is set if a tet has J <= 0.
__global__ void __launch_bounds__(kBlock) k_energy_body(Launch L, int trial)
{
    int lb, s = scene_of_block(L, lb);
    const SceneDev &S = *L.sc[s];
    const double *x = trial ? S.xtrial : S.x;
    int64_t t = (int64_t)lb * blockDim.x + threadIdx.x;
    double val = 0.0;
    if (t < S.m) {
        int e = (int)t;
        double F[3][3], q[4][3], Fd[9];
        tet_F<double>(S, x, e, F, q, Fd);
        double J = det3(Fd);
        if (!(J > 0.0)) {
            atomicOr(&L.out[s].infeasible, 1);
        } else {
            double tr = 0.0;
            for (int k = 0; k < 9; ++k) tr += Fd[k] * Fd[k];
            double lnJ = log(J);
            val = S.vol[e] * (0.5 * S.mu * (tr - 3.0) - S.mu * lnJ + 0.5 * S.lam * lnJ * lnJ);
        }
    } else if (t < (int64_t)S.m + S.n) {
        int i = (int)(t - S.m);
        if (i < S.n_gel) {
            if (!S.fixed[i]) {
                double d0 = x[3 * i] - S.xtilde[3 * i], d1 = x[3 * i + 1] - S.xtilde[3 * i + 1],
                       d2 = x[3 * i + 2] - S.xtilde[3 * i + 2];
                val = S.mass[i] * (0.5 * S.inv_h2) * (d0 * d0 + d1 * d1 + d2 * d2);
                if (S.attached && S.attached[i]) {
                    double e0 = x[3 * i] - S.yhat[3 * i], e1 = x[3 * i + 1] - S.yhat[3 * i + 1],
                           e2 = x[3 * i + 2] - S.yhat[3 * i + 2];
                    val += 0.5 * S.k_target * (e0 * e0 + e1 * e1 + e2 * e2);
                }
            }
        } else {
            double d0 = x[3 * i] - S.yhat[3 * i], d1 = x[3 * i + 1] - S.yhat[3 * i + 1], d2 = x[3 * i + 2] - S.yhat[3 * i + 2];
            val = 0.5 * S.k_target * (d0 * d0 + d1 * d1 + d2 * d2);
            if (S.target_al)
                val -= S.al_lam[3 * i] * d0 + S.al_lam[3 * i + 1] * d1 + S.al_lam[3 * i + 2] * d2;
        }
    }
    CSum c = {val, 0.0};
    c = block_csum(c);
    if (threadIdx.x == 0) {
        S.red[2 * lb] = c.s;
        S.red[2 * lb + 1] = c.c;
    }
}

// ---- launchers --------------------------------------------------------------

static bool mixed(const Batch &b) { return b.sc[0]->prm.precision == IPC_MIXED; }

void launch_elastic_elements(Batch &b)
{
    hipEvent_t ev[2];
    b.prof_begin(kProfElastic, ev);
    if (mixed(b))
        IPC_LAUNCH(b, k_elastic_elements<float>, kPhTet, kBlock);
    else
        IPC_LAUNCH(b, k_elastic_elements<double>, kPhTet, kBlock);
    b.prof_end(kProfElastic, ev);
}

void launch_assemble(Batch &b)
{
    hipEvent_t ev[2];
    b.prof_begin(kProfAssemble, ev);
    if (mixed(b)) {
        IPC_LAUNCH(b, k_assemble_gradient<float>, kPhVertH, kBlock);
        IPC_LAUNCH(b, k_assemble_bell<float>, kPhEntry, kBlock);
    } else {
        IPC_LAUNCH(b, k_assemble_gradient<double>, kPhVertH, kBlock);
        IPC_LAUNCH(b, k_assemble_bell<double>, kPhEntry, kBlock);
    }
    launch_mas_diag(b);
    b.prof_end(kProfAssemble, ev);
}

void launch_rest_precompute(Batch &b)
{
    IPC_LAUNCH(b, k_rest_tets, kPhTet, kBlock);
    IPC_LAUNCH(b, k_rest_mass, kPhVert, kBlock);
}

void launch_energy_body(Batch &b, bool trial) { IPC_LAUNCH(b, k_energy_body, kPhBody, kBlock, (int)trial); }

}  // namespace ipcg
