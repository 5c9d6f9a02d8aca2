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
//
// Element outputs are written SoA (component-major) and summed per matrix
// block / per vertex by gather kernels in a fixed order: no float atomics.
#include "device_util.h"
#include "ipc_internal.h"

namespace ipcg {

__device__ __forceinline__ void jacobi_rot3(double A[3][3], double V[3][3], int p, int q)
{
    double apq = A[p][q];
    if (apq == 0.0) return;
    double theta = (A[q][q] - A[p][p]) / (2.0 * apq);
    double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
    double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double akp = A[k][p], akq = A[k][q];
        A[k][p] = c * akp - s * akq;
        A[k][q] = s * akp + c * akq;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double apk = A[p][k], aqk = A[q][k];
        A[p][k] = c * apk - s * aqk;
        A[q][k] = s * apk + c * aqk;
    }
    A[p][q] = A[q][p] = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double vkp = V[k][p], vkq = V[k][q];
        V[k][p] = c * vkp - s * vkq;
        V[k][q] = s * vkp + c * vkq;
    }
}

// symmetric 3x3 eigen-decomposition by cyclic Jacobi; V columns = vectors
__device__ void sym3_eig(double A[3][3], double V[3][3], double w[3])
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) V[i][j] = (i == j) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 20; ++sweep) {
        double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
        double dg = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
        if (off <= 1e-36 * dg) break;
        jacobi_rot3(A, V, 0, 1);
        jacobi_rot3(A, V, 0, 2);
        jacobi_rot3(A, V, 1, 2);
    }
    w[0] = A[0][0];
    w[1] = A[1][1];
    w[2] = A[2][2];
}

// F = U diag(s) V^T with det U = det V = +1 (requires det F > 0)
__device__ void svd3(const double F[3][3], double U[3][3], double s[3], double V[3][3])
{
    double S[3][3], w[3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) S[i][j] = F[0][i] * F[0][j] + F[1][i] * F[1][j] + F[2][i] * F[2][j];
    sym3_eig(S, V, w);
    // order descending
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2 - a; ++b)
            if (w[b] < w[b + 1]) {
                double t = w[b];
                w[b] = w[b + 1];
                w[b + 1] = t;
                for (int k = 0; k < 3; ++k) {
                    double u = V[k][b];
                    V[k][b] = V[k][b + 1];
                    V[k][b + 1] = u;
                }
            }
    double dv = V[0][0] * (V[1][1] * V[2][2] - V[1][2] * V[2][1]) -
                V[0][1] * (V[1][0] * V[2][2] - V[1][2] * V[2][0]) +
                V[0][2] * (V[1][0] * V[2][1] - V[1][1] * V[2][0]);
    if (dv < 0.0)
        for (int k = 0; k < 3; ++k) V[k][2] = -V[k][2];
    double B[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) B[i][j] = F[i][0] * V[0][j] + F[i][1] * V[1][j] + F[i][2] * V[2][j];
    // Gram-Schmidt QR of B
    double n0 = sqrt(B[0][0] * B[0][0] + B[1][0] * B[1][0] + B[2][0] * B[2][0]);
    double u0[3] = {B[0][0] / n0, B[1][0] / n0, B[2][0] / n0};
    double pr = u0[0] * B[0][1] + u0[1] * B[1][1] + u0[2] * B[2][1];
    double t1[3] = {B[0][1] - pr * u0[0], B[1][1] - pr * u0[1], B[2][1] - pr * u0[2]};
    double n1 = sqrt(t1[0] * t1[0] + t1[1] * t1[1] + t1[2] * t1[2]);
    double u1[3] = {t1[0] / n1, t1[1] / n1, t1[2] / n1};
    double u2[3] = {u0[1] * u1[2] - u0[2] * u1[1], u0[2] * u1[0] - u0[0] * u1[2], u0[0] * u1[1] - u0[1] * u1[0]};
    s[0] = n0;
    s[1] = u1[0] * B[0][1] + u1[1] * B[1][1] + u1[2] * B[2][1];
    s[2] = u2[0] * B[0][2] + u2[1] * B[1][2] + u2[2] * B[2][2];
    for (int k = 0; k < 3; ++k) {
        U[k][0] = u0[k];
        U[k][1] = u1[k];
        U[k][2] = u2[k];
    }
}

// block index of the (a,b) 3x3 block, a <= b, in the 10-block element layout
__host__ __device__ __forceinline__ int elem_block(int a, int b)
{
    if (a == b) return a;
    // (0,1)4 (0,2)5 (0,3)6 (1,2)7 (1,3)8 (2,3)9
    return a == 0 ? 3 + b : (a == 1 ? 5 + b : 9);
}

__device__ __forceinline__ void load_tet(const int32_t *tv, int m, int e, const double *x, int vid[4],
                                         double X[4][3])
{
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        vid[a] = tv[a * m + e];
#pragma unroll
        for (int c = 0; c < 3; ++c) X[a][c] = x[3 * vid[a] + c];
    }
}

// F = Ds Bm with Ds = [x1-x0, x2-x0, x3-x0]
__device__ __forceinline__ void deformation_gradient(const double X[4][3], const double *Bm, int m, int e,
                                                     double F[3][3], double q[4][3])
{
    double B[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) B[k] = Bm[k * m + e];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        double d1 = X[1][i] - X[0][i], d2 = X[2][i] - X[0][i], d3 = X[3][i] - X[0][i];
#pragma unroll
        for (int j = 0; j < 3; ++j) F[i][j] = d1 * B[0 * 3 + j] + d2 * B[1 * 3 + j] + d3 * B[2 * 3 + j];
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        q[1][j] = B[0 * 3 + j];
        q[2][j] = B[1 * 3 + j];
        q[3][j] = B[2 * 3 + j];
        q[0][j] = -(q[1][j] + q[2][j] + q[3][j]);
    }
}

__global__ void __launch_bounds__(kBlock) k_elastic_elements(int m, const int32_t *__restrict__ tv,
                                                              const double *__restrict__ Bm,
                                                              const double *__restrict__ vol,
                                                              const double *__restrict__ x, double mu,
                                                              double lam, double *__restrict__ eg,
                                                              double *__restrict__ eH)
{
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    int vid[4];
    double X[4][3], F[3][3], q[4][3];
    load_tet(tv, m, e, x, vid, X);
    deformation_gradient(X, Bm, m, e, F, q);
    double V = vol[e];
    double Fm[9] = {F[0][0], F[0][1], F[0][2], F[1][0], F[1][1], F[1][2], F[2][0], F[2][1], F[2][2]};
    double J = det3(Fm);
    if (!(J > 0.0)) {
        // infeasible state: the line search never accepts one; write zeros
        for (int k = 0; k < 12; ++k) eg[k * m + e] = 0.0;
        for (int k = 0; k < 90; ++k) eH[k * m + e] = 0.0;
        return;
    }
    double Fi[9];
    inverse3(Fm, Fi);
    double lnJ = log(J);
    // P = mu (F - F^-T) + lam lnJ F^-T
    double P[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double fit = Fi[j * 3 + i];
            P[i][j] = mu * (F[i][j] - fit) + lam * lnJ * fit;
        }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            eg[(a * 3 + c) * m + e] = V * (P[c][0] * q[a][0] + P[c][1] * q[a][1] + P[c][2] * q[a][2]);

    // analytic eigensystem of d2Psi/dF2 in the SVD frame
    double U[3][3], s[3], Vv[3][3];
    svd3(F, U, s, Vv);
    double cc = mu - lam * lnJ;
    double Dm[3][3], W[3][3], ev[3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            Dm[i][j] = (i == j) ? mu + (cc + lam) / (s[i] * s[i]) : lam / (s[i] * s[j]);
    sym3_eig(Dm, W, ev);
    // s_a = V^T q_a
    double sa[4][3];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int k = 0; k < 3; ++k) sa[a][k] = Vv[0][k] * q[a][0] + Vv[1][k] * q[a][1] + Vv[2][k] * q[a][2];

    double H[10][9];
#pragma unroll
    for (int b = 0; b < 10; ++b)
#pragma unroll
        for (int k = 0; k < 9; ++k) H[b][k] = 0.0;

    const double inv_sqrt2 = 0.70710678118654752440;
    for (int mode = 0; mode < 9; ++mode) {
        double lamk;
        double t[4][3];
        if (mode < 3) {
            lamk = ev[mode];
            if (!(lamk > 0.0)) continue;
            for (int a = 0; a < 4; ++a)
                for (int k = 0; k < 3; ++k) t[a][k] = W[k][mode] * sa[a][k];
        } else {
            int pair = (mode - 3) >> 1, sgn = ((mode - 3) & 1) ? -1 : 1;
            int i = pair == 2 ? 1 : 0, j = pair == 0 ? 1 : 2;
            lamk = mu + sgn * cc / (s[i] * s[j]);
            if (!(lamk > 0.0)) continue;
            for (int a = 0; a < 4; ++a) {
                t[a][0] = t[a][1] = t[a][2] = 0.0;
                t[a][i] = sa[a][j] * inv_sqrt2;
                t[a][j] = sgn * sa[a][i] * inv_sqrt2;
            }
        }
        double gk[4][3];
        for (int a = 0; a < 4; ++a)
            for (int k = 0; k < 3; ++k) gk[a][k] = U[k][0] * t[a][0] + U[k][1] * t[a][1] + U[k][2] * t[a][2];
        double sc = V * lamk;
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
        for (int k = 0; k < 9; ++k) eH[(b * 9 + k) * m + e] = H[b][k];
}

// Gradient gather: one thread per vertex; elastic element gradients in
// vertex-incidence order, then inertia / kinematic target, then contact.
__global__ void __launch_bounds__(kBlock) k_assemble_gradient(
    int n, int n_gel, int m, const int32_t *__restrict__ vt_ptr, const int32_t *__restrict__ vt_src,
    const double *__restrict__ eg, const double *__restrict__ x, const double *__restrict__ xtilde,
    const double *__restrict__ yhat, const double *__restrict__ mass, const uint8_t *__restrict__ fixed,
    double inv_h2, double k_target, const int32_t *__restrict__ c_ptr, const int32_t *__restrict__ c_list,
    const double *__restrict__ act_g, int64_t act_cap, double *__restrict__ grad)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double g[3] = {0.0, 0.0, 0.0};
    if (!fixed[i]) {
        for (int k = vt_ptr[i]; k < vt_ptr[i + 1]; ++k) {
            int src = vt_src[k], e = src >> 2, a = src & 3;
            for (int c = 0; c < 3; ++c) g[c] += eg[(a * 3 + c) * m + e];
        }
        if (i < n_gel) {
            double kk = mass[i] * inv_h2;
            for (int c = 0; c < 3; ++c) g[c] += kk * (x[3 * i + c] - xtilde[3 * i + c]);
        } else {
            for (int c = 0; c < 3; ++c) g[c] += k_target * (x[3 * i + c] - yhat[3 * i + c]);
        }
        for (int k = c_ptr[i]; k < c_ptr[i + 1]; ++k) {
            int src = c_list[k], p = src >> 2, a = src & 3;
            for (int c = 0; c < 3; ++c) g[c] += act_g[(int64_t)(a * 3 + c) * act_cap + p];
        }
    }
    for (int c = 0; c < 3; ++c) grad[3 * i + c] = g[c];
}

// Matrix gather: one thread per stored BELL block. Sums the element blocks
// listed for this (row, col) in tet order; the diagonal block also takes the
// inertia / target term and the contact diagonal blocks, and writes the
// inverse used by the block-Jacobi preconditioner. Fixed rows/cols become
// identity / zero.
__global__ void __launch_bounds__(kBlock) k_assemble_bell(
    int n, int n_gel, int m, int n_slices, const int32_t *__restrict__ slice_ptr,
    const int32_t *__restrict__ bcol, const int32_t *__restrict__ g_ptr, const int32_t *__restrict__ g_src,
    const double *__restrict__ eH, const double *__restrict__ mass, const uint8_t *__restrict__ fixed,
    double inv_h2, double k_target, const int32_t *__restrict__ c_ptr, const int32_t *__restrict__ c_list,
    const double *__restrict__ act_H, int64_t act_cap, double *__restrict__ bval, double *__restrict__ Minv)
{
    int64_t slot_lane = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t total = (int64_t)slice_ptr[n_slices] * kSlice;
    if (slot_lane >= total) return;
    int64_t slot = slot_lane / kSlice;
    int lane = (int)(slot_lane % kSlice);
    // slice of this slot: slots are laid out slice by slice; find by search
    int lo = 0, hi = n_slices;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (slice_ptr[mid] <= slot) lo = mid; else hi = mid;
    }
    int row = lo * kSlice + lane;
    int k = (int)(slot - slice_ptr[lo]);
    int col = bcol[slot_lane];
    double A[9];
    for (int c = 0; c < 9; ++c) A[c] = 0.0;
    if (col >= 0) {
        for (int t = g_ptr[slot_lane]; t < g_ptr[slot_lane + 1]; ++t) {
            int src = g_src[t];
            int e = src >> 4, a = (src >> 2) & 3, b = src & 3;
            if (a <= b) {
                int blk = elem_block(a, b);
                for (int c = 0; c < 9; ++c) A[c] += eH[(int64_t)(blk * 9 + c) * m + e];
            } else {
                int blk = elem_block(b, a);
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) A[i * 3 + j] += eH[(int64_t)(blk * 9 + j * 3 + i) * m + e];
            }
        }
        if (k == 0) {
            double dk = row < n_gel ? mass[row] * inv_h2 : k_target;
            A[0] += dk;
            A[4] += dk;
            A[8] += dk;
            for (int t = c_ptr[row]; t < c_ptr[row + 1]; ++t) {
                int src = c_list[t], p = src >> 2, a = src & 3;
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j)
                        A[i * 3 + j] += act_H[(int64_t)((3 * a + i) * 12 + 3 * a + j) * act_cap + p];
            }
        }
        if (fixed[row] || fixed[col]) {
            for (int c = 0; c < 9; ++c) A[c] = 0.0;
            if (k == 0) A[0] = A[4] = A[8] = 1.0;
        }
    }
    for (int c = 0; c < 9; ++c) bval[(slot * 9 + c) * kSlice + lane] = A[c];
    if (k == 0 && row < n) {
        double Inv[9];
        inverse3(A, Inv);
        for (int c = 0; c < 9; ++c) Minv[9 * row + c] = Inv[c];
    }
}

// Rest shape: Bm = Dm^-1 (row-major), V = det(Dm)/6. Mass is gathered per
// vertex from the incidence list (rho V / 4 per incident tet).
__global__ void k_rest_tets(int m, const int32_t *__restrict__ tv, const double *__restrict__ X,
                            double *__restrict__ Bm, double *__restrict__ vol)
{
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    int vid[4];
    double P[4][3];
    load_tet(tv, m, e, X, vid, P);
    double D[9];
    for (int i = 0; i < 3; ++i)
        for (int c = 0; c < 3; ++c) D[i * 3 + c] = P[c + 1][i] - P[0][i];
    double Inv[9];
    double det = inverse3(D, Inv);
    for (int k = 0; k < 9; ++k) Bm[k * m + e] = Inv[k];
    vol[e] = det / 6.0;
}

__global__ void k_rest_mass(int n, const int32_t *__restrict__ vt_ptr, const int32_t *__restrict__ vt_src,
                            const double *__restrict__ vol, double rho, double *__restrict__ mass)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    for (int k = vt_ptr[i]; k < vt_ptr[i + 1]; ++k) acc += rho * vol[vt_src[k] >> 2] / 4.0;
    mass[i] = acc;
}

// Elastic + inertia + target terms of the incremental potential, per item,
// into compensated block partials. Items: tets, then gel vertices, then
// indenter vertices. flag gets 1 if any tet has J <= 0.
__global__ void __launch_bounds__(kBlock) k_energy_body(
    int m, int n, int n_gel, const int32_t *__restrict__ tv, const double *__restrict__ Bm,
    const double *__restrict__ vol, const double *__restrict__ x, const double *__restrict__ xtilde,
    const double *__restrict__ yhat, const double *__restrict__ mass, const uint8_t *__restrict__ fixed,
    double mu, double lam, double inv_2h2, double half_kt, double *__restrict__ part, int32_t *flag)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double val = 0.0;
    if (t < m) {
        int e = (int)t;
        int vid[4];
        double X[4][3], F[3][3], q[4][3];
        load_tet(tv, m, e, x, vid, X);
        deformation_gradient(X, Bm, m, e, F, q);
        double Fm[9] = {F[0][0], F[0][1], F[0][2], F[1][0], F[1][1], F[1][2], F[2][0], F[2][1], F[2][2]};
        double J = det3(Fm);
        if (!(J > 0.0)) {
            atomicOr(flag, 1);
        } else {
            double tr = 0.0;
            for (int k = 0; k < 9; ++k) tr += Fm[k] * Fm[k];
            double lnJ = log(J);
            val = vol[e] * (0.5 * mu * (tr - 3.0) - mu * lnJ + 0.5 * lam * lnJ * lnJ);
        }
    } else if (t < (int64_t)m + n) {
        int i = (int)(t - m);
        if (i < n_gel) {
            if (!fixed[i]) {
                double d0 = x[3 * i] - xtilde[3 * i], d1 = x[3 * i + 1] - xtilde[3 * i + 1],
                       d2 = x[3 * i + 2] - xtilde[3 * i + 2];
                val = mass[i] * inv_2h2 * (d0 * d0 + d1 * d1 + d2 * d2);
            }
        } else {
            double d0 = x[3 * i] - yhat[3 * i], d1 = x[3 * i + 1] - yhat[3 * i + 1],
                   d2 = x[3 * i + 2] - yhat[3 * i + 2];
            val = half_kt * (d0 * d0 + d1 * d1 + d2 * d2);
        }
    }
    CSum c = {val, 0.0};
    c = block_csum(c);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = c.s;
        part[2 * blockIdx.x + 1] = c.c;
    }
}

// ---- launchers --------------------------------------------------------------

void launch_elastic_elements(Scene &s, const double *x)
{
    hipLaunchKernelGGL(k_elastic_elements, dim3(nblocks(s.m)), dim3(kBlock), 0, s.stream, s.m, s.tv, s.Bm,
                       s.vol, x, s.prm.mu, s.prm.lam, s.eg, s.eH);
}

void launch_assemble(Scene &s, const double *x)
{
    double inv_h2 = 1.0 / (s.prm.dt * s.prm.dt);
    hipLaunchKernelGGL(k_assemble_gradient, dim3(nblocks(s.n)), dim3(kBlock), 0, s.stream, s.n, s.n_gel, s.m,
                       s.vt_ptr, s.vt_src, s.eg, x, s.xtilde, s.yhat, s.mass, s.fixed, inv_h2, s.prm.k_target,
                       s.c_ptr, s.c_list, s.act_g, s.act_cap, s.grad);
    int64_t total = (int64_t)s.n_slots * kSlice;
    hipLaunchKernelGGL(k_assemble_bell, dim3(nblocks(total)), dim3(kBlock), 0, s.stream, s.n, s.n_gel, s.m,
                       s.n_slices, s.slice_ptr, s.bcol, s.g_ptr, s.g_src, s.eH, s.mass, s.fixed, inv_h2,
                       s.prm.k_target, s.c_ptr, s.c_list, s.act_H, s.act_cap, s.bval, s.Minv);
}

void launch_rest_precompute(Scene &s)
{
    hipLaunchKernelGGL(k_rest_tets, dim3(nblocks(s.m)), dim3(kBlock), 0, s.stream, s.m, s.tv, s.X0, s.Bm, s.vol);
    hipLaunchKernelGGL(k_rest_mass, dim3(nblocks(s.n)), dim3(kBlock), 0, s.stream, s.n, s.vt_ptr, s.vt_src, s.vol,
                       s.prm.rho, s.mass);
}

// Body part of the incremental potential (tets + vertices), returned as a
// compensated pair (sum, compensation) through the partial buffer.
int launch_energy_body(Scene &s, const double *x, double *part, int32_t *flag)
{
    int64_t items = (int64_t)s.m + s.n;
    int nb = nblocks(items);
    hipLaunchKernelGGL(k_energy_body, dim3(nb), dim3(kBlock), 0, s.stream, s.m, s.n, s.n_gel, s.tv, s.Bm, s.vol, x,
                       s.xtilde, s.yhat, s.mass, s.fixed, s.prm.mu, s.prm.lam,
                       0.5 / (s.prm.dt * s.prm.dt), 0.5 * s.prm.k_target, part, flag);
    return nb;
}

}  // namespace ipcg
