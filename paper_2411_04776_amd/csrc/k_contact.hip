// k_contact.hip -- contact culling, distances, barrier, CCD, contact energy.
//
// Contact model (the IPC model the paper adopts through GIPC, section "Choice
// of the Simulation Methods"): every non-incident point-triangle (PT) and
// edge-edge (EE) pair contributes kappa * w * b(d) with the log barrier
// b(d) = -(d - dhat)^2 ln(d / dhat) on the unsigned distance d < dhat; w = 1
// for PT and the parallel-edge mollifier for EE.
//
// Candidates are defined by a predicate, not by the accelerator: a pair is a
// candidate iff the closed boxes [min - dhat/2, max + dhat/2] of its two
// primitives overlap on all axes (boxes over x, or over x and x + p for the
// swept set). The spatial hash only enumerates; every reported pair passes
// the exact FP64 box test and is reported once, from the cell that holds the
// low corner of the two boxes' intersection. Each query's output segment is
// sorted, so the list comes out in canonical (type, a, b) order.
#include "device_util.h"
#include "ipc_internal.h"

namespace ipcg {

// ---------------------------------------------------------------------------
// distance types and their coefficient tables
// ---------------------------------------------------------------------------
// A type fixes the closest features; within it the squared distance is
// min over beta of |sum_k c_k(beta) x_k|^2 with c = c0 + sum_m beta_m D_m.
// PT vertices: 0 point, 1..3 triangle. EE vertices: 0,1 edge A, 2,3 edge B.
struct DistSpec {
    int np;
    double c0[4];
    double D[2][4];
};

__constant__ DistSpec c_pt_spec[7] = {
    {0, {1, -1, 0, 0}, {{0, 0, 0, 0}, {0, 0, 0, 0}}},   // vertex t0
    {0, {1, 0, -1, 0}, {{0, 0, 0, 0}, {0, 0, 0, 0}}},   // vertex t1
    {0, {1, 0, 0, -1}, {{0, 0, 0, 0}, {0, 0, 0, 0}}},   // vertex t2
    {1, {1, -1, 0, 0}, {{0, 1, -1, 0}, {0, 0, 0, 0}}},  // edge t0 t1
    {1, {1, 0, -1, 0}, {{0, 0, 1, -1}, {0, 0, 0, 0}}},  // edge t1 t2
    {1, {1, 0, 0, -1}, {{0, -1, 0, 1}, {0, 0, 0, 0}}},  // edge t2 t0
    {2, {1, -1, 0, 0}, {{0, 1, -1, 0}, {0, 1, 0, -1}}}, // face
};
__constant__ DistSpec c_ee_spec[9] = {
    {0, {1, 0, -1, 0}, {{0, 0, 0, 0}, {0, 0, 0, 0}}},   // A0-B0
    {0, {1, 0, 0, -1}, {{0, 0, 0, 0}, {0, 0, 0, 0}}},   // A0-B1
    {0, {0, 1, -1, 0}, {{0, 0, 0, 0}, {0, 0, 0, 0}}},   // A1-B0
    {0, {0, 1, 0, -1}, {{0, 0, 0, 0}, {0, 0, 0, 0}}},   // A1-B1
    {1, {1, 0, -1, 0}, {{0, 0, 1, -1}, {0, 0, 0, 0}}},  // A0-edge B
    {1, {0, 1, -1, 0}, {{0, 0, 1, -1}, {0, 0, 0, 0}}},  // A1-edge B
    {1, {1, 0, -1, 0}, {{-1, 1, 0, 0}, {0, 0, 0, 0}}},  // B0-edge A
    {1, {1, 0, 0, -1}, {{-1, 1, 0, 0}, {0, 0, 0, 0}}},  // B1-edge A
    {2, {1, 0, -1, 0}, {{-1, 1, 0, 0}, {0, 0, 1, -1}}}, // line-line
};

constexpr double kEEParallel = 1e-10;  // segment-segment determinant / (|u|^2 |v|^2)
constexpr double kMollifier = 1e-3;    // eps_x = 1e-3 |e0_rest|^2 |e1_rest|^2

__device__ __forceinline__ double d3(const double *a, const double *b)
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// Voronoi-region classification of point p against triangle (a, b, c)
// (Ericson, Real-Time Collision Detection, 5.1.5); ties go to the
// lower-dimensional feature.
__device__ int classify_pt(const double *x)
{
    const double *p = x, *a = x + 3, *b = x + 6, *c = x + 9;
    double ab[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    double ac[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
    double ap[3] = {p[0] - a[0], p[1] - a[1], p[2] - a[2]};
    double d1 = d3(ab, ap), d2 = d3(ac, ap);
    if (d1 <= 0.0 && d2 <= 0.0) return 0;
    double bp[3] = {p[0] - b[0], p[1] - b[1], p[2] - b[2]};
    double d3v = d3(ab, bp), d4 = d3(ac, bp);
    if (d3v >= 0.0 && d4 <= d3v) return 1;
    double vc = d1 * d4 - d3v * d2;
    if (vc <= 0.0 && d1 >= 0.0 && d3v <= 0.0) return 3;
    double cp[3] = {p[0] - c[0], p[1] - c[1], p[2] - c[2]};
    double d5 = d3(ab, cp), d6 = d3(ac, cp);
    if (d6 >= 0.0 && d5 <= d6) return 2;
    double vb = d5 * d2 - d1 * d6;
    if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) return 5;
    double va = d3v * d6 - d5 * d4;
    if (va <= 0.0 && (d4 - d3v) >= 0.0 && (d5 - d6) >= 0.0) return 4;
    return 6;
}

__device__ __forceinline__ double clamp01d(double v) { return v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v); }

// closest segment parameters, clamped (Ericson 5.1.9); nearly parallel
// segments start from A0
__device__ int classify_ee(const double *x)
{
    double u[3] = {x[3] - x[0], x[4] - x[1], x[5] - x[2]};
    double v[3] = {x[9] - x[6], x[10] - x[7], x[11] - x[8]};
    double w[3] = {x[0] - x[6], x[1] - x[7], x[2] - x[8]};
    double a = d3(u, u), e = d3(v, v), f = d3(v, w), c = d3(u, w), b = d3(u, v);
    double den = a * e - b * b;
    double s = den > kEEParallel * a * e ? clamp01d((b * f - c * e) / den) : 0.0;
    double t = (b * s + f) / e;
    if (t < 0.0) {
        t = 0.0;
        s = clamp01d(-c / a);
    } else if (t > 1.0) {
        t = 1.0;
        s = clamp01d((b - c) / a);
    }
    int se = s == 0.0 ? 0 : (s == 1.0 ? 1 : -1);
    int te = t == 0.0 ? 0 : (t == 1.0 ? 1 : -1);
    if (se >= 0 && te >= 0) return 2 * se + te;
    if (se >= 0) return 4 + se;
    if (te >= 0) return 6 + te;
    return 8;
}

// closest-point residual r(beta*) for a type; returns |r|^2. Optionally the
// coefficients at beta*, the parameter directions and their Gram matrix.
__device__ double dist_residual(const DistSpec &sp, const double *x, double r[3], double c[4], double u[2][3],
                                double G[3])
{
    double r0[3];
    for (int i = 0; i < 3; ++i)
        r0[i] = sp.c0[0] * x[i] + sp.c0[1] * x[3 + i] + sp.c0[2] * x[6 + i] + sp.c0[3] * x[9 + i];
    for (int m = 0; m < sp.np; ++m)
        for (int i = 0; i < 3; ++i)
            u[m][i] = sp.D[m][0] * x[i] + sp.D[m][1] * x[3 + i] + sp.D[m][2] * x[6 + i] + sp.D[m][3] * x[9 + i];
    double beta[2] = {0.0, 0.0};
    if (sp.np == 1) {
        G[0] = d3(u[0], u[0]);
        beta[0] = -d3(u[0], r0) / G[0];
    } else if (sp.np == 2) {
        G[0] = d3(u[0], u[0]);
        G[1] = d3(u[0], u[1]);
        G[2] = d3(u[1], u[1]);
        double b0 = -d3(u[0], r0), b1 = -d3(u[1], r0);
        double det = G[0] * G[2] - G[1] * G[1];
        beta[0] = (b0 * G[2] - G[1] * b1) / det;
        beta[1] = (G[0] * b1 - G[1] * b0) / det;
    }
    for (int i = 0; i < 3; ++i) r[i] = r0[i] + beta[0] * (sp.np > 0 ? u[0][i] : 0.0) + beta[1] * (sp.np > 1 ? u[1][i] : 0.0);
    for (int k = 0; k < 4; ++k) c[k] = sp.c0[k] + beta[0] * sp.D[0][k] + beta[1] * sp.D[1][k];
    return d3(r, r);
}

__device__ __forceinline__ double pair_distance(int kind, const double *x)
{
    DistSpec sp = kind == 0 ? c_pt_spec[classify_pt(x)] : c_ee_spec[classify_ee(x)];
    double r[3], c[4], u[2][3], G[3];
    return sqrt(dist_residual(sp, x, r, c, u, G));
}

__device__ __forceinline__ void barrier3(double d, double dhat, double b[3])
{
    double t = d - dhat, L = log(d / dhat);
    b[0] = -t * t * L;
    b[1] = -2.0 * t * L - t * t / d;
    b[2] = -2.0 * L - 4.0 * t / d + t * t / (d * d);
}

// vertex ids of a candidate: PT (p, t0, t1, t2), EE (a0, a1, b0, b1)
struct Topo {
    const int32_t *ev;  // 2 * ne SoA
    const int32_t *trv; // 3 * nt SoA
    int ne, nt;
};
__device__ __forceinline__ void cand_vertices(const Topo &tp, int type, int a, int b, int v[4])
{
    if (type == 0) {
        v[0] = a;
        v[1] = tp.trv[b];
        v[2] = tp.trv[tp.nt + b];
        v[3] = tp.trv[2 * tp.nt + b];
    } else {
        v[0] = tp.ev[a];
        v[1] = tp.ev[tp.ne + a];
        v[2] = tp.ev[b];
        v[3] = tp.ev[tp.ne + b];
    }
}
__device__ __forceinline__ void gather12(const double *x, const int v[4], double x12[12])
{
    for (int k = 0; k < 4; ++k)
        for (int i = 0; i < 3; ++i) x12[3 * k + i] = x[3 * v[k] + i];
}

// ---------------------------------------------------------------------------
// boxes and the spatial hash
// ---------------------------------------------------------------------------

// box over vertex positions at x (and x + p if p != null), inflated by r
__global__ void k_boxes(int N, int nv, const int32_t *__restrict__ vids, int stride, const double *__restrict__ x,
                        const double *__restrict__ p, double r, double *__restrict__ box)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int k = 0; k < nv; ++k) {
        int v = vids[k * stride + i];
        for (int c = 0; c < 3; ++c) {
            double a = x[3 * v + c];
            lo[c] = fmin(lo[c], a);
            hi[c] = fmax(hi[c], a);
            if (p) {
                double b = __dadd_rn(a, p[3 * v + c]);
                lo[c] = fmin(lo[c], b);
                hi[c] = fmax(hi[c], b);
            }
        }
    }
    for (int c = 0; c < 3; ++c) {
        box[c * N + i] = lo[c] - r;
        box[(3 + c) * N + i] = hi[c] + r;
    }
}

// per-block sums of the largest axis extent of each box
__global__ void k_box_extent(int N, const double *__restrict__ box, double *__restrict__ part)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    double e = 0.0;
    if (i < N)
        for (int c = 0; c < 3; ++c) e = fmax(e, box[(3 + c) * N + i] - box[c * N + i]);
    e = block_sum_all(e);
    if (threadIdx.x == 0) part[blockIdx.x] = e;
}

// cell size = mean extent of the edge and triangle boxes (never below the
// inflation dhat): most primitives span 1-3 cells per axis, large ones more
__global__ void k_cell_size(int nb, const double *__restrict__ part, double count, double floor_h,
                            double *cell_h)
{
    double v = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) v += part[i];
    v = block_sum_all(v);
    if (threadIdx.x == 0) *cell_h = fmax(v / count, floor_h);
}

__device__ __forceinline__ int cell_of(double v, double h) { return (int)floor(v / h); }
__device__ __forceinline__ uint32_t cell_hash(int ix, int iy, int iz, uint32_t mask)
{
    return (((uint32_t)ix * 73856093u) ^ ((uint32_t)iy * 19349663u) ^ ((uint32_t)iz * 83492791u)) & mask;
}

// Cells spanned per axis by one box are bounded by this; a larger span means
// a non-finite or absurd position, which is flagged and skipped.
constexpr int kMaxSpan = 4096;

template <bool FILL>
__global__ void k_hash_insert(int N, const double *__restrict__ box, const double *__restrict__ cell_h, uint32_t mask,
                              int32_t *__restrict__ counter, const int32_t *__restrict__ start,
                              int4 *__restrict__ entries, int entry_cap, int32_t *__restrict__ bad)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double h = *cell_h;
    int lo[3], hi[3];
    for (int c = 0; c < 3; ++c) {
        double a = box[c * N + i], b = box[(3 + c) * N + i];
        if (!(a <= b) || !((b - a) / h < (double)kMaxSpan)) {
            if (!FILL) atomicOr(bad, 1);
            return;
        }
        lo[c] = cell_of(a, h);
        hi[c] = cell_of(b, h);
    }
    for (int iz = lo[2]; iz <= hi[2]; ++iz)
        for (int iy = lo[1]; iy <= hi[1]; ++iy)
            for (int ix = lo[0]; ix <= hi[0]; ++ix) {
                uint32_t bkt = cell_hash(ix, iy, iz, mask);
                int pos = atomicAdd(&counter[bkt], 1);
                if (FILL && start[bkt] + pos < entry_cap) entries[start[bkt] + pos] = make_int4(ix, iy, iz, i);
            }
}

struct PairRules {
    const int32_t *pts;
    const uint8_t *fixed;
    int n_gel;
    int self_contact;
};

__device__ __forceinline__ bool pt_admissible(const PairRules &R, int a, int t0, int t1, int t2)
{
    if (a == t0 || a == t1 || a == t2) return false;
    bool ai = a >= R.n_gel, ti = t0 >= R.n_gel;
    if (ai && ti) return false;
    if (!ai && !ti && !R.self_contact) return false;
    if (R.fixed[a] && R.fixed[t0] && R.fixed[t1] && R.fixed[t2]) return false;
    return true;
}
__device__ __forceinline__ bool ee_admissible(const PairRules &R, int a0, int a1, int b0, int b1)
{
    if (a0 == b0 || a0 == b1 || a1 == b0 || a1 == b1) return false;
    bool ai = a0 >= R.n_gel, bi = b0 >= R.n_gel;
    if (ai && bi) return false;
    if (!ai && !bi && !R.self_contact) return false;
    if (R.fixed[a0] && R.fixed[a1] && R.fixed[b0] && R.fixed[b1]) return false;
    return true;
}

// One thread per query primitive (PT: surface point index, EE: edge index).
// COUNT: per-query number of accepted pairs. Else write them at off[q] and
// sort the segment by b.
template <int KIND, bool COUNT>
__global__ void __launch_bounds__(kBlock) k_query(int NA, const double *__restrict__ abox, int NB,
                                                   const double *__restrict__ bbox, Topo tp, PairRules R,
                                                   const double *__restrict__ cell_h, uint32_t mask,
                                                   const int32_t *__restrict__ start, const int4 *__restrict__ entries,
                                                   int entry_cap, int32_t *__restrict__ qcount,
                                                   const int32_t *__restrict__ qoff,
                                                   int32_t *__restrict__ out_type, int32_t *__restrict__ out_a,
                                                   int32_t *__restrict__ out_b, int64_t out_base)
{
    int qa = blockIdx.x * blockDim.x + threadIdx.x;
    if (qa >= NA) return;
    double h = *cell_h;
    double alo[3], ahi[3];
    int clo[3], chi[3];
    for (int c = 0; c < 3; ++c) {
        alo[c] = abox[c * NA + qa];
        ahi[c] = abox[(3 + c) * NA + qa];
        if (!(alo[c] <= ahi[c]) || !((ahi[c] - alo[c]) / h < (double)kMaxSpan)) {
            if (COUNT) qcount[qa] = 0;
            return;
        }
        clo[c] = cell_of(alo[c], h);
        chi[c] = cell_of(ahi[c], h);
    }
    int va[2];
    int a_id;
    if (KIND == 0) {
        va[0] = R.pts[qa];
        a_id = va[0];
    } else {
        va[0] = tp.ev[qa];
        va[1] = tp.ev[tp.ne + qa];
        a_id = qa;
    }
    int count = 0;
    int64_t o = 0;
    if (!COUNT) o = out_base + qoff[qa];
    for (int iz = clo[2]; iz <= chi[2]; ++iz)
        for (int iy = clo[1]; iy <= chi[1]; ++iy)
            for (int ix = clo[0]; ix <= chi[0]; ++ix) {
                uint32_t bkt = cell_hash(ix, iy, iz, mask);
                int kend = min(start[bkt + 1], entry_cap);
                for (int k = start[bkt]; k < kend; ++k) {
                    int4 en = entries[k];
                    if (en.x != ix || en.y != iy || en.z != iz) continue;
                    int b = en.w;
                    if (KIND == 0) {
                        if (!pt_admissible(R, va[0], tp.trv[b], tp.trv[tp.nt + b], tp.trv[2 * tp.nt + b])) continue;
                    } else {
                        if (b <= qa) continue;
                        if (!ee_admissible(R, va[0], va[1], tp.ev[b], tp.ev[tp.ne + b])) continue;
                    }
                    bool ov = true;
                    double corner[3];
                    for (int c = 0; c < 3; ++c) {
                        double blo = bbox[c * NB + b], bhi = bbox[(3 + c) * NB + b];
                        ov = ov && (alo[c] <= bhi) && (blo <= ahi[c]);
                        corner[c] = fmax(alo[c], blo);
                    }
                    if (!ov) continue;
                    if (cell_of(corner[0], h) != ix || cell_of(corner[1], h) != iy || cell_of(corner[2], h) != iz)
                        continue;
                    if (COUNT) {
                        ++count;
                    } else {
                        out_type[o + count] = KIND;
                        out_a[o + count] = a_id;
                        out_b[o + count] = b;
                        ++count;
                    }
                }
            }
    if (COUNT) {
        qcount[qa] = count;
    } else {
        // insertion sort of this query's segment by b
        for (int i = 1; i < count; ++i) {
            int key = out_b[o + i];
            int j = i - 1;
            while (j >= 0 && out_b[o + j] > key) {
                out_b[o + j + 1] = out_b[o + j];
                --j;
            }
            out_b[o + j + 1] = key;
        }
    }
}

// ---------------------------------------------------------------------------
// narrow phase, barrier, incidence
// ---------------------------------------------------------------------------

__global__ void k_narrow(int64_t nc, int64_t cap, const int32_t *__restrict__ cand, Topo tp,
                         const double *__restrict__ x, double dhat, double *__restrict__ dout,
                         int32_t *__restrict__ active)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nc) return;
    int type = cand[i], a = cand[cap + i], b = cand[2 * cap + i];
    int v[4];
    double x12[12];
    cand_vertices(tp, type, a, b, v);
    gather12(x, v, x12);
    double d = pair_distance(type, x12);
    dout[i] = d;
    active[i] = d < dhat ? 1 : 0;
}

__global__ void k_compact(int64_t nc, const int32_t *__restrict__ flag, const int32_t *__restrict__ pos,
                          int32_t *__restrict__ out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nc && flag[i]) out[pos[i]] = (int32_t)i;
}

// Shared per-pair data of the distance derivatives at fixed type: residual r,
// coefficients c at beta*, parameter directions u, and the 12 x np block W of
// s_xb with S = s_bb^-1 (np <= 2).
struct DistDeriv {
    int np;
    double r[3], c[4], W[12][2], S00, S01, S11, s;
};

__device__ void dist_deriv_setup(const DistSpec &sp, const double *x, DistDeriv &dd)
{
    double u[2][3], G[3];
    dd.np = sp.np;
    dd.s = dist_residual(sp, x, dd.r, dd.c, u, G);
    for (int k = 0; k < 4; ++k)
        for (int i = 0; i < 3; ++i)
            for (int m = 0; m < 2; ++m)
                dd.W[3 * k + i][m] = m < sp.np ? 2.0 * (sp.D[m][k] * dd.r[i] + dd.c[k] * u[m][i]) : 0.0;
    dd.S00 = dd.S01 = dd.S11 = 0.0;
    if (sp.np == 1) {
        dd.S00 = 1.0 / (2.0 * G[0]);
    } else if (sp.np == 2) {
        double a = 2.0 * G[0], b = 2.0 * G[1], d = 2.0 * G[2];
        double det = a * d - b * b;
        dd.S00 = d / det;
        dd.S01 = -b / det;
        dd.S11 = a / det;
    }
}

// d2s/dx_p dx_q at fixed type
__device__ __forceinline__ double dist_hess_entry(const DistDeriv &dd, int p, int q)
{
    int k = p / 3, i = p % 3, l = q / 3, j = q % 3;
    double v = (i == j) ? 2.0 * dd.c[k] * dd.c[l] : 0.0;
    if (dd.np > 0) {
        double acc = dd.W[p][0] * dd.S00 * dd.W[q][0];
        if (dd.np == 2)
            acc += dd.W[p][0] * dd.S01 * dd.W[q][1] + dd.W[p][1] * dd.S01 * dd.W[q][0] + dd.W[p][1] * dd.S11 * dd.W[q][1];
        v -= acc;
    }
    return v;
}

// Round-robin (circle method) pairing of 12 indices: in round r the six
// disjoint pairs meet; over 11 rounds every pair meets once.
__device__ __forceinline__ void rr_pair(int round, int i, int &p, int &q)
{
    int pa = i, pb = 11 - i;
    int a = pa == 0 ? 0 : ((pa - 1 + round) % 11) + 1;
    int b = ((pb - 1 + round) % 11) + 1;
    p = a < b ? a : b;
    q = a < b ? b : a;
}

// kappa * w * b(d) for each active pair: gradient and PSD-projected Hessian.
// One wavefront per pair: lanes evaluate Hessian entries, then a parallel
// cyclic Jacobi (six disjoint rotations per round) diagonalises the 12x12 in
// LDS and negative eigenvalues are clamped to zero. Matrices that are already
// PSD are kept as assembled.
__global__ void __launch_bounds__(64) k_barrier(int64_t nact, int64_t act_cap, const int32_t *__restrict__ act_idx,
                                                int64_t cap, const int32_t *__restrict__ cand, Topo tp,
                                                const double *__restrict__ edge_rest_sq,
                                                const double *__restrict__ x, const uint8_t *__restrict__ fixed,
                                                double dhat, double kappa,
                                                int32_t *__restrict__ act_v, double *__restrict__ act_g,
                                                double *__restrict__ act_H)
{
    __shared__ double A[144], V[144], A0[144];
    __shared__ double rc[6], rs[6];
    __shared__ int rp[6], rq[6];
    int64_t k = blockIdx.x;
    if (k >= nact) return;
    const int lane = threadIdx.x;
    int ci = act_idx[k];
    int type = cand[ci], a = cand[cap + ci], b = cand[2 * cap + ci];
    int v[4];
    double x12[12];
    cand_vertices(tp, type, a, b, v);
    gather12(x, v, x12);
    DistSpec sp = type == 0 ? c_pt_spec[classify_pt(x12)] : c_ee_spec[classify_ee(x12)];
    DistDeriv dd;
    dist_deriv_setup(sp, x12, dd);
    double d = sqrt(dd.s);
    double bb[3];
    barrier3(d, dhat, bb);
    // gs = 2 c_k r_i, gd = gs / (2d)
    double inv2d = 1.0 / (2.0 * d), inv4d3 = 1.0 / (4.0 * d * d * d);
    // EE mollifier
    double w = 1.0, m1 = 0.0, m2 = 0.0;
    bool moll = false;
    double ea[3], eb[3], aa = 0.0, bq = 0.0, ab = 0.0;
    if (type == 1) {
        double eps_x = kMollifier * edge_rest_sq[a] * edge_rest_sq[b];
        for (int i = 0; i < 3; ++i) {
            ea[i] = x12[3 + i] - x12[i];
            eb[i] = x12[9 + i] - x12[6 + i];
        }
        double cr[3] = {ea[1] * eb[2] - ea[2] * eb[1], ea[2] * eb[0] - ea[0] * eb[2], ea[0] * eb[1] - ea[1] * eb[0]};
        double cval = d3(cr, cr);
        if (cval < eps_x) {
            moll = true;
            w = -cval * cval / (eps_x * eps_x) + 2.0 * cval / eps_x;
            m1 = -2.0 * cval / (eps_x * eps_x) + 2.0 / eps_x;
            m2 = -2.0 / (eps_x * eps_x);
            aa = d3(ea, ea);
            bq = d3(eb, eb);
            ab = d3(ea, eb);
        }
    }
    const double sa[4] = {-1, 1, 0, 0}, sb[4] = {0, 0, -1, 1};
    auto gs_of = [&](int p) { return 2.0 * dd.c[p / 3] * dd.r[p % 3]; };
    auto gc_of = [&](int p) {
        int kk = p / 3, i = p % 3;
        double ga = 2.0 * bq * ea[i] - 2.0 * ab * eb[i];
        double gb = 2.0 * aa * eb[i] - 2.0 * ab * ea[i];
        return sa[kk] * ga + sb[kk] * gb;
    };
    // entries of the unprojected pair Hessian
    for (int e = lane; e < 144; e += 64) {
        int p = e / 12, q = e % 12;
        double gsp = gs_of(p), gsq = gs_of(q);
        double gdp = gsp * inv2d, gdq = gsq * inv2d;
        double hd = dist_hess_entry(dd, p, q) * inv2d - gsp * gsq * inv4d3;
        double hv = w * (bb[2] * gdp * gdq + bb[1] * hd);
        if (moll) {
            int kp = p / 3, i = p % 3, kq = q / 3, j = q % 3;
            double dij = i == j ? 1.0 : 0.0;
            double haa = 2.0 * bq * dij - 2.0 * eb[i] * eb[j];
            double hbb = 2.0 * aa * dij - 2.0 * ea[i] * ea[j];
            double hab = 4.0 * ea[i] * eb[j] - 2.0 * ab * dij - 2.0 * eb[i] * ea[j];
            double hba = 4.0 * ea[j] * eb[i] - 2.0 * ab * dij - 2.0 * eb[j] * ea[i];
            double hc = sa[kp] * sa[kq] * haa + sb[kp] * sb[kq] * hbb + sa[kp] * sb[kq] * hab + sb[kp] * sa[kq] * hba;
            double gcp = gc_of(p), gcq = gc_of(q);
            hv += bb[0] * (m2 * gcp * gcq + m1 * hc);
            hv += bb[1] * m1 * (gcp * gdq + gdp * gcq);
        }
        A[e] = kappa * hv;
        A0[e] = A[e];
        V[e] = (p == q) ? 1.0 : 0.0;
    }
    if (lane < 12) {
        double gv = w * bb[1] * gs_of(lane) * inv2d;
        if (moll) gv += bb[0] * m1 * gc_of(lane);
        act_g[(int64_t)lane * act_cap + k] = kappa * gv;
    }
    if (lane < 4) act_v[(int64_t)lane * act_cap + k] = v[lane];
    __syncthreads();

    // parallel cyclic Jacobi
    double fro = 0.0;
    for (int e = lane; e < 144; e += 64) fro += A[e] * A[e];
    fro = wave_sum(fro);
    fro = __shfl(fro, 0, 64);
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int e = lane; e < 144; e += 64) {
            int p = e / 12, q = e % 12;
            if (p < q) off += A[e] * A[e];
        }
        off = wave_sum(off);
        off = __shfl(off, 0, 64);
        if (off <= 1e-36 * fro || off == 0.0) break;
        for (int round = 0; round < 11; ++round) {
            if (lane < 6) {
                int p, q;
                rr_pair(round, lane, p, q);
                double apq = A[p * 12 + q];
                double c = 1.0, sn = 0.0;
                if (apq != 0.0) {
                    double theta = (A[q * 12 + q] - A[p * 12 + p]) / (2.0 * apq);
                    double t = fabs(theta) > 1e150 ? 0.5 / theta
                                                   : (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                    c = 1.0 / sqrt(t * t + 1.0);
                    sn = t * c;
                }
                rc[lane] = c;
                rs[lane] = sn;
                rp[lane] = p;
                rq[lane] = q;
            }
            __syncthreads();
            // rows p, q of A and columns p, q of V
            for (int task = lane; task < 72; task += 64) {
                int rr = task / 12, col = task % 12;
                int p = rp[rr], q = rq[rr];
                double c = rc[rr], sn = rs[rr];
                double apk = A[p * 12 + col], aqk = A[q * 12 + col];
                A[p * 12 + col] = c * apk - sn * aqk;
                A[q * 12 + col] = sn * apk + c * aqk;
                double vkp = V[col * 12 + p], vkq = V[col * 12 + q];
                V[col * 12 + p] = c * vkp - sn * vkq;
                V[col * 12 + q] = sn * vkp + c * vkq;
            }
            __syncthreads();
            // columns p, q of A
            for (int task = lane; task < 72; task += 64) {
                int rr = task / 12, row = task % 12;
                int p = rp[rr], q = rq[rr];
                double c = rc[rr], sn = rs[rr];
                double akp = A[row * 12 + p], akq = A[row * 12 + q];
                A[row * 12 + p] = c * akp - sn * akq;
                A[row * 12 + q] = sn * akp + c * akq;
            }
            __syncthreads();
            if (lane < 6 && rs[lane] != 0.0) {
                A[rp[lane] * 12 + rq[lane]] = 0.0;
                A[rq[lane] * 12 + rp[lane]] = 0.0;
            }
            __syncthreads();
        }
    }
    bool neg = false;
    for (int i = 0; i < 12; ++i) neg |= A[i * 12 + i] < 0.0;
    for (int e = lane; e < 144; e += 64) {
        int i = e / 12, j = e % 12;
        double val = A0[e];
        if (neg) {
            val = 0.0;
            for (int kk = 0; kk < 12; ++kk) {
                double wk = A[kk * 12 + kk];
                if (wk > 0.0) val += V[i * 12 + kk] * wk * V[j * 12 + kk];
            }
        }
        // Dirichlet vertices drop out (their identity rows live in the elastic matrix)
        if (fixed[v[i / 3]] || fixed[v[j / 3]]) val = 0.0;
        act_H[(int64_t)e * act_cap + k] = val;
    }
    if (lane < 12 && fixed[v[lane / 3]]) act_g[(int64_t)lane * act_cap + k] = 0.0;
}

template <bool FILL>
__global__ void k_incidence(int64_t nact, int64_t act_cap, const int32_t *__restrict__ act_v,
                            const uint8_t *__restrict__ fixed, int32_t *__restrict__ cnt,
                            const int32_t *__restrict__ ptr, int32_t *__restrict__ list)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nact) return;
    for (int a = 0; a < 4; ++a) {
        int v = act_v[(int64_t)a * act_cap + k];
        if (fixed[v]) continue;
        int pos = atomicAdd(&cnt[v], 1);
        if (FILL) list[ptr[v] + pos] = (int32_t)(k * 4 + a);
    }
}

__global__ void k_incidence_sort(int n, const int32_t *__restrict__ ptr, int32_t *__restrict__ list)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int s0 = ptr[i], s1 = ptr[i + 1];
    for (int k = s0 + 1; k < s1; ++k) {
        int key = list[k];
        int j = k - 1;
        while (j >= s0 && list[j] > key) {
            list[j + 1] = list[j];
            --j;
        }
        list[j + 1] = key;
    }
}

// ---------------------------------------------------------------------------
// additive CCD and contact energy
// ---------------------------------------------------------------------------

// Additive CCD (conservative advancement of Li, Kaufman and Jiang 2021):
// relative motion bound l_p after removing the mean displacement; safe
// sub-steps 0.9 d / l_p until the gap drops below s * d0 (return the last
// safe time) or time passes tmax.
__device__ double accd_pair(int kind, const double *x0, const double *p0, double s, double tmax, int max_iter)
{
    double x[12], p[12], pm[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < 4; ++k)
        for (int i = 0; i < 3; ++i) pm[i] += p0[3 * k + i];
    for (int i = 0; i < 3; ++i) pm[i] /= 4.0;
    double len[4];
    for (int k = 0; k < 4; ++k) {
        for (int i = 0; i < 3; ++i) {
            p[3 * k + i] = p0[3 * k + i] - pm[i];
            x[3 * k + i] = x0[3 * k + i];
        }
        len[k] = sqrt(d3(p + 3 * k, p + 3 * k));
    }
    double lp = kind == 0 ? len[0] + fmax(len[1], fmax(len[2], len[3])) : fmax(len[0], len[1]) + fmax(len[2], len[3]);
    if (lp == 0.0) return tmax;
    double d = pair_distance(kind, x);
    double g = s * d, t = 0.0, tl = (1.0 - s) * d / lp;
    for (int it = 0; it < max_iter; ++it) {
        for (int i = 0; i < 12; ++i) x[i] += tl * p[i];
        d = pair_distance(kind, x);
        if (t > 0.0 && d < g) break;
        t += tl;
        if (t > tmax) return tmax;
        tl = 0.9 * d / lp;
    }
    return t;
}

__global__ void __launch_bounds__(kBlock) k_accd(int64_t nc, int64_t cap, const int32_t *__restrict__ cand, Topo tp,
                                                 const double *__restrict__ x, const double *__restrict__ p, double s,
                                                 int max_iter, double *__restrict__ part)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double t = 1.0;
    if (i < nc) {
        int type = cand[i], a = cand[cap + i], b = cand[2 * cap + i];
        int v[4];
        double x12[12], p12[12];
        cand_vertices(tp, type, a, b, v);
        gather12(x, v, x12);
        gather12(p, v, p12);
        t = accd_pair(type, x12, p12, s, 1.0, max_iter);
    }
    t = block_min_all(t);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ void k_final_min(int nb, const double *__restrict__ part, double *out)
{
    double v = INFINITY;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) v = fmin(v, part[i]);
    v = block_min_all(v);
    if (threadIdx.x == 0) *out = v;
}

__global__ void __launch_bounds__(kBlock) k_energy_contact(int64_t nc, int64_t cap, const int32_t *__restrict__ cand,
                                                           Topo tp, const double *__restrict__ edge_rest_sq,
                                                           const double *__restrict__ x, double dhat, double kappa,
                                                           double *__restrict__ part, int32_t *flag)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double val = 0.0;
    if (i < nc) {
        int type = cand[i], a = cand[cap + i], b = cand[2 * cap + i];
        int v[4];
        double x12[12];
        cand_vertices(tp, type, a, b, v);
        gather12(x, v, x12);
        double d = pair_distance(type, x12);
        if (!(d > 0.0)) {
            atomicOr(flag, 1);
        } else if (d < dhat) {
            double bb[3];
            barrier3(d, dhat, bb);
            double w = 1.0;
            if (type == 1) {
                double eps_x = kMollifier * edge_rest_sq[a] * edge_rest_sq[b];
                double ea[3] = {x12[3] - x12[0], x12[4] - x12[1], x12[5] - x12[2]};
                double eb[3] = {x12[9] - x12[6], x12[10] - x12[7], x12[11] - x12[8]};
                double cr[3] = {ea[1] * eb[2] - ea[2] * eb[1], ea[2] * eb[0] - ea[0] * eb[2],
                                ea[0] * eb[1] - ea[1] * eb[0]};
                double c = d3(cr, cr);
                if (c < eps_x) w = -c * c / (eps_x * eps_x) + 2.0 * c / eps_x;
            }
            val = kappa * w * bb[0];
        }
    }
    CSum cs = {val, 0.0};
    cs = block_csum(cs);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = cs.s;
        part[2 * blockIdx.x + 1] = cs.c;
    }
}

// final compensated sum over body + contact partials
__global__ void k_energy_final(int nb, const double *__restrict__ part, double *out)
{
    CSum acc = {0.0, 0.0};
    for (int i = threadIdx.x; i < nb; i += blockDim.x) {
        CSum t = {part[2 * i], part[2 * i + 1]};
        acc = csum_add(acc, t);
    }
    acc = block_csum(acc);
    if (threadIdx.x == 0) *out = acc.s + acc.c;
}

// ---------------------------------------------------------------------------
// host drivers
// ---------------------------------------------------------------------------

static Topo topo(Scene &s) { return Topo{s.ev, s.trv, s.n_edges, s.n_tris}; }
static PairRules rules(Scene &s) { return PairRules{s.pts, s.fixed, s.n_gel, s.prm.self_contact}; }

void ensure_query(Scene &s, size_t n)
{
    if (s.q_n >= n) return;
    if (s.q_count) dfree(s, s.q_count);
    if (s.q_off) dfree(s, s.q_off);
    s.q_count = dalloc<int32_t>(s, n + 1);
    s.q_off = dalloc<int32_t>(s, n + 1);
    s.q_n = n;
}

void launch_boxes(Scene &s, const double *x, const double *p)
{
    double r = 0.5 * s.prm.dhat;
    hipLaunchKernelGGL(k_boxes, dim3(nblocks(s.n_pts)), dim3(kBlock), 0, s.stream, s.n_pts, 1, s.pts, s.n_pts, x, p, r,
                       s.pbox);
    hipLaunchKernelGGL(k_boxes, dim3(nblocks(s.n_edges)), dim3(kBlock), 0, s.stream, s.n_edges, 2, s.ev, s.n_edges, x,
                       p, r, s.ebox);
    hipLaunchKernelGGL(k_boxes, dim3(nblocks(s.n_tris)), dim3(kBlock), 0, s.stream, s.n_tris, 3, s.trv, s.n_tris, x, p,
                       r, s.tbox);
    int nbe = nblocks(s.n_edges), nbt = nblocks(s.n_tris);
    hipLaunchKernelGGL(k_box_extent, dim3(nbe), dim3(kBlock), 0, s.stream, s.n_edges, s.ebox, s.red_scratch);
    hipLaunchKernelGGL(k_box_extent, dim3(nbt), dim3(kBlock), 0, s.stream, s.n_tris, s.tbox, s.red_scratch + nbe);
    hipLaunchKernelGGL(k_cell_size, dim3(1), dim3(kBlock), 0, s.stream, nbe + nbt, s.red_scratch,
                       (double)(s.n_edges + s.n_tris), 2.0 * r, s.cell_h);
}

// table for N boxes with room for `cap` entries (power-of-two buckets)
static void alloc_table(Scene &s, HashTable &ht, int64_t cap)
{
    if (ht.entries.p) {
        dfree(s, ht.entries.p);
        dfree(s, ht.bucket_count.p);
        dfree(s, ht.bucket_start.p);
    }
    int bits = 10;
    while ((int64_t(1) << bits) < 2 * cap && bits < 28) ++bits;
    ht.table_bits = bits;
    size_t tsize = size_t(1) << bits;
    ht.bucket_count.p = dalloc<int32_t>(s, tsize + 1);
    ht.bucket_start.p = dalloc<int32_t>(s, tsize + 1);
    ht.entries.p = dalloc<int4>(s, (size_t)cap);
    ht.entries.n = (size_t)cap;
}

static void build_hash(Scene &s, HashTable &ht, int N, const double *box, int32_t *bad)
{
    uint32_t tsize = 1u << ht.table_bits, mask = tsize - 1;
    int cap = (int)ht.entries.n;
    IPC_HIP(hipMemsetAsync(ht.bucket_count.p, 0, sizeof(int32_t) * (tsize + 1), s.stream));
    hipLaunchKernelGGL((k_hash_insert<false>), dim3(nblocks(N)), dim3(kBlock), 0, s.stream, N, box, s.cell_h, mask,
                       ht.bucket_count.p, nullptr, nullptr, cap, bad);
    exclusive_scan(s, ht.bucket_count.p, ht.bucket_start.p, (int)tsize, ht.bucket_start.p + tsize);
    IPC_HIP(hipMemsetAsync(ht.bucket_count.p, 0, sizeof(int32_t) * (tsize + 1), s.stream));
    hipLaunchKernelGGL((k_hash_insert<true>), dim3(nblocks(N)), dim3(kBlock), 0, s.stream, N, box, s.cell_h, mask,
                       ht.bucket_count.p, ht.bucket_start.p, ht.entries.p, cap, bad);
}

static void grow_candidates(Scene &s, int32_t **buf, int64_t *cap, int64_t need)
{
    if (*buf && need <= *cap) return;
    int64_t nc = need + need / 2 + 1024;
    if (*buf) dfree(s, *buf);
    *buf = dalloc<int32_t>(s, 3 * nc);
    *cap = nc;
}

// Candidate pairs at x (p null) or over [x, x+p] into *out (SoA triples with
// stride *cap, grown as needed). Returns the count. Hash tables that overflow
// their entry capacity are grown and the phase is redone.
int64_t run_broad_phase(Scene &s, const double *x, const double *p, int32_t **out, int64_t *cap)
{
    if (!s.ht_tri.entries.p) alloc_table(s, s.ht_tri, 16 * (int64_t)std::max(s.n_tris, 1));
    if (!s.ht_edge.entries.p) alloc_table(s, s.ht_edge, 16 * (int64_t)std::max(s.n_edges, 1));
    int32_t *bad = s.pcg_state + 9;
    launch_boxes(s, x, p);
    Topo tp = topo(s);
    PairRules R = rules(s);
    int nq = s.n_pts + s.n_edges;
    ensure_query(s, (size_t)nq);
    for (int attempt = 0; attempt < 4; ++attempt) {
        IPC_HIP(hipMemsetAsync(bad, 0, sizeof(int32_t), s.stream));
        build_hash(s, s.ht_tri, s.n_tris, s.tbox, bad);
        build_hash(s, s.ht_edge, s.n_edges, s.ebox, bad);
        uint32_t mt = (1u << s.ht_tri.table_bits) - 1, me = (1u << s.ht_edge.table_bits) - 1;
        int capt = (int)s.ht_tri.entries.n, cape = (int)s.ht_edge.entries.n;
        hipLaunchKernelGGL((k_query<0, true>), dim3(nblocks(s.n_pts)), dim3(kBlock), 0, s.stream, s.n_pts, s.pbox,
                           s.n_tris, s.tbox, tp, R, s.cell_h, mt, s.ht_tri.bucket_start.p, s.ht_tri.entries.p, capt,
                           s.q_count, nullptr, nullptr, nullptr, nullptr, (int64_t)0);
        hipLaunchKernelGGL((k_query<1, true>), dim3(nblocks(s.n_edges)), dim3(kBlock), 0, s.stream, s.n_edges, s.ebox,
                           s.n_edges, s.ebox, tp, R, s.cell_h, me, s.ht_edge.bucket_start.p, s.ht_edge.entries.p, cape,
                           s.q_count + s.n_pts, nullptr, nullptr, nullptr, nullptr, (int64_t)0);
        exclusive_scan(s, s.q_count, s.q_off, nq, s.q_off + nq);
        int32_t *tt = s.ht_tri.bucket_start.p + ((size_t)1 << s.ht_tri.table_bits);
        int32_t *te = s.ht_edge.bucket_start.p + ((size_t)1 << s.ht_edge.table_bits);
        IPC_HIP(hipMemcpyAsync(&s.hb->flag, s.q_off + nq, sizeof(int32_t), hipMemcpyDeviceToHost, s.stream));
        IPC_HIP(hipMemcpyAsync(&s.hb->iters, bad, sizeof(int32_t), hipMemcpyDeviceToHost, s.stream));
        IPC_HIP(hipMemcpyAsync(&s.hb->count, tt, sizeof(int32_t), hipMemcpyDeviceToHost, s.stream));
        IPC_HIP(hipMemcpyAsync(reinterpret_cast<int32_t *>(&s.hb->count) + 1, te, sizeof(int32_t),
                               hipMemcpyDeviceToHost, s.stream));
        IPC_HIP(hipStreamSynchronize(s.stream));
        if (s.hb->iters) throw InfeasibleError{};
        int32_t ent_t = reinterpret_cast<int32_t *>(&s.hb->count)[0];
        int32_t ent_e = reinterpret_cast<int32_t *>(&s.hb->count)[1];
        bool redo = false;
        if (ent_t > capt) {
            alloc_table(s, s.ht_tri, (int64_t)ent_t * 3 / 2 + 1024);
            redo = true;
        }
        if (ent_e > cape) {
            alloc_table(s, s.ht_edge, (int64_t)ent_e * 3 / 2 + 1024);
            redo = true;
        }
        if (redo) continue;
        int32_t total = s.hb->flag;
        grow_candidates(s, out, cap, total);
        int64_t C = *cap;
        int32_t *ob = *out;
        hipLaunchKernelGGL((k_query<0, false>), dim3(nblocks(s.n_pts)), dim3(kBlock), 0, s.stream, s.n_pts, s.pbox,
                           s.n_tris, s.tbox, tp, R, s.cell_h, mt, s.ht_tri.bucket_start.p, s.ht_tri.entries.p, capt,
                           nullptr, s.q_off, ob, ob + C, ob + 2 * C, (int64_t)0);
        hipLaunchKernelGGL((k_query<1, false>), dim3(nblocks(s.n_edges)), dim3(kBlock), 0, s.stream, s.n_edges,
                           s.ebox, s.n_edges, s.ebox, tp, R, s.cell_h, me, s.ht_edge.bucket_start.p,
                           s.ht_edge.entries.p, cape, nullptr, s.q_off + s.n_pts, ob, ob + C, ob + 2 * C, (int64_t)0);
        return total;
    }
    throw CapacityError{};
}

static void grow_active(Scene &s, int64_t need)
{
    if (s.act_idx && need <= s.act_cap) return;
    int64_t nc = need + need / 2 + 256;
    if (s.act_idx) {
        dfree(s, s.act_idx);
        dfree(s, s.act_v);
        dfree(s, s.act_g);
        dfree(s, s.act_H);
        dfree(s, s.c_list);
    }
    s.act_idx = dalloc<int32_t>(s, nc);
    s.act_v = dalloc<int32_t>(s, 4 * nc);
    s.act_g = dalloc<double>(s, 12 * nc);
    s.act_H = dalloc<double>(s, 144 * nc);
    s.c_list = dalloc<int32_t>(s, 4 * nc);
    s.act_cap = nc;
}

// distances of the static candidates; active = d < dhat, compacted
int64_t run_narrow_phase(Scene &s, const double *x)
{
    int64_t nc = s.n_cand;
    if (nc == 0) {
        s.n_act = 0;
        return 0;
    }
    Topo tp = topo(s);
    hipLaunchKernelGGL(k_narrow, dim3(nblocks(nc)), dim3(kBlock), 0, s.stream, nc, s.cand_cap, s.cand, tp, x,
                       s.prm.dhat, s.cand_d, s.act_flag);
    ensure_query(s, (size_t)nc);
    exclusive_scan(s, s.act_flag, s.q_off, (int)nc, s.q_off + nc);
    IPC_HIP(hipMemcpyAsync(&s.hb->flag, s.q_off + nc, sizeof(int32_t), hipMemcpyDeviceToHost, s.stream));
    IPC_HIP(hipStreamSynchronize(s.stream));
    int64_t na = s.hb->flag;
    grow_active(s, na);
    if (na > 0)
        hipLaunchKernelGGL(k_compact, dim3(nblocks(nc)), dim3(kBlock), 0, s.stream, nc, s.act_flag, s.q_off, s.act_idx);
    s.n_act = na;
    return na;
}

void launch_barrier(Scene &s, const double *x)
{
    if (s.n_act == 0) return;
    Topo tp = topo(s);
    hipLaunchKernelGGL(k_barrier, dim3((unsigned)s.n_act), dim3(64), 0, s.stream, s.n_act, s.act_cap, s.act_idx,
                       s.cand_cap, s.cand, tp, s.edge_rest_sq, x, s.fixed, s.prm.dhat, s.prm.kappa, s.act_v,
                       s.act_g, s.act_H);
}

void launch_contact_incidence(Scene &s)
{
    IPC_HIP(hipMemsetAsync(s.c_cnt, 0, sizeof(int32_t) * (s.n + 1), s.stream));
    if (s.n_act > 0)
        hipLaunchKernelGGL((k_incidence<false>), dim3(nblocks(s.n_act)), dim3(kBlock), 0, s.stream, s.n_act, s.act_cap,
                           s.act_v, s.fixed, s.c_cnt, nullptr, nullptr);
    exclusive_scan(s, s.c_cnt, s.c_ptr, s.n, s.c_ptr + s.n);
    if (s.n_act > 0) {
        IPC_HIP(hipMemsetAsync(s.c_cnt, 0, sizeof(int32_t) * (s.n + 1), s.stream));
        hipLaunchKernelGGL((k_incidence<true>), dim3(nblocks(s.n_act)), dim3(kBlock), 0, s.stream, s.n_act, s.act_cap,
                           s.act_v, s.fixed, s.c_cnt, s.c_ptr, s.c_list);
        hipLaunchKernelGGL(k_incidence_sort, dim3(nblocks(s.n)), dim3(kBlock), 0, s.stream, s.n, s.c_ptr, s.c_list);
    }
}

double run_ccd(Scene &s, const double *x, const double *p)
{
    int64_t nc = s.n_cand_sw;
    if (nc == 0) return 1.0;
    int nb = nblocks(nc);
    Topo tp = topo(s);
    double *part = s.accd_t;
    hipLaunchKernelGGL(k_accd, dim3(nb), dim3(kBlock), 0, s.stream, nc, s.sw_cap, s.cand_sw, tp, x, p, s.prm.ccd_s,
                       s.prm.ccd_max_iter, part);
    hipLaunchKernelGGL(k_final_min, dim3(1), dim3(kBlock), 0, s.stream, nb, part, s.red_scratch);
    IPC_HIP(hipMemcpyAsync(&s.hb->value, s.red_scratch, sizeof(double), hipMemcpyDeviceToHost, s.stream));
    IPC_HIP(hipStreamSynchronize(s.stream));
    return s.hb->value;
}

int launch_energy_body(Scene &s, const double *x, double *part, int32_t *flag);

// Incremental potential at x over the given candidate list. Sets
// *infeasible if a tet has J <= 0 or a pair d <= 0.
double run_energy(Scene &s, const double *x, const int32_t *cand, int64_t nc, int *infeasible)
{
    int32_t *flag = s.pcg_state + 8;
    IPC_HIP(hipMemsetAsync(flag, 0, sizeof(int32_t), s.stream));
    double *part = s.accd_t;  // 2 doubles per block
    int nb_body = launch_energy_body(s, x, part, flag);
    int nb_c = 0;
    int64_t capc = cand == s.cand_sw ? s.sw_cap : s.cand_cap;
    if (nc > 0) {
        nb_c = nblocks(nc);
        Topo tp = topo(s);
        hipLaunchKernelGGL(k_energy_contact, dim3(nb_c), dim3(kBlock), 0, s.stream, nc, capc, cand, tp, s.edge_rest_sq,
                           x, s.prm.dhat, s.prm.kappa, part + 2 * nb_body, flag);
    }
    hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(kBlock), 0, s.stream, nb_body + nb_c, part, s.red_scratch);
    IPC_HIP(hipMemcpyAsync(&s.hb->value, s.red_scratch, sizeof(double), hipMemcpyDeviceToHost, s.stream));
    IPC_HIP(hipMemcpyAsync(&s.hb->flag, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s.stream));
    IPC_HIP(hipStreamSynchronize(s.stream));
    *infeasible = s.hb->flag != 0;
    return *infeasible ? INFINITY : s.hb->value;
}

}  // namespace ipcg
