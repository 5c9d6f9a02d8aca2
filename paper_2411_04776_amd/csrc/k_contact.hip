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
//
// Every kernel runs over a list of scenes (see ipc_internal.h); per-scene
// counts live on the device and are read back once per phase for all scenes.
#include <functional>

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


template <class R>
__device__ __forceinline__ R *as(void *p)
{
    return reinterpret_cast<R *>(p);
}

// ---------------------------------------------------------------------------
// boxes and the spatial hash
// ---------------------------------------------------------------------------

// box over the primitive's vertex positions at x (and x + p for the swept
// set), inflated by dhat/2. kind 0 points, 1 edges, 2 triangles.
template <class R>
__device__ void boxes_body(const SceneDev &S, int lb, int kind, int swept)
{
    int N = kind == 0 ? S.n_pts : (kind == 1 ? S.n_edges : S.n_tris);
    int i = lb * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int32_t *vids = kind == 0 ? S.pts : (kind == 1 ? S.ev : S.trv);
    double *box = kind == 0 ? S.pbox : (kind == 1 ? S.ebox : S.tbox);
    int nv = kind + 1;
    const double *x = S.x;
    const R *p = swept ? as<R>(S.sol) : nullptr;
    double r = 0.5 * S.dhat;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int k = 0; k < nv; ++k) {
        int v = vids[(int64_t)k * N + i];
        for (int c = 0; c < 3; ++c) {
            double a = x[3 * v + c];
            lo[c] = fmin(lo[c], a);
            hi[c] = fmax(hi[c], a);
            if (p) {
                double b = __dadd_rn(a, (double)p[3 * v + c]);
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

__device__ __forceinline__ int blocks_for(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }

// Boxes of points, edges and triangles in one launch (blocks in that order);
// with `extent`, the edge and triangle blocks also write the per-block sums
// of their boxes' largest axis extent (edges at red[0..nbe), triangles after).
template <class R>
__global__ void k_boxes_all(Launch L, int swept, int extent)
{
    int lb, s = scene_of_block(L, lb);
    const SceneDev &S = *L.sc[s];
    const int np = blocks_for(S.n_pts), ne = blocks_for(S.n_edges);
    int kind = lb < np ? 0 : (lb < np + ne ? 1 : 2);
    int kb = kind == 0 ? lb : (kind == 1 ? lb - np : lb - np - ne);
    boxes_body<R>(S, kb, kind, swept);
    if (!extent || kind == 0) return;  // uniform over the block
    int N = kind == 1 ? S.n_edges : S.n_tris;
    const double *box = kind == 1 ? S.ebox : S.tbox;
    int i = kb * blockDim.x + threadIdx.x;
    double e = 0.0;
    if (i < N)
        for (int c = 0; c < 3; ++c) e = fmax(e, box[(3 + c) * N + i] - box[c * N + i]);
    e = block_sum_all(e);
    if (threadIdx.x == 0) S.red[(kind == 1 ? 0 : ne) + kb] = e;
}

// cell size = mean extent of the edge and triangle boxes (never below the
// inflation dhat): most primitives span 1-3 cells per axis, large ones more
__global__ void k_cell_size(Launch one)
{
    int lb, s = scene_of_block(one, lb);
    const SceneDev &S = *one.sc[s];
    int nb = blocks_for(S.n_edges) + blocks_for(S.n_tris);
    double v = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) v += S.red[i];
    v = block_sum_all(v);
    if (threadIdx.x == 0) {
        *S.cell_h = fmax(v / (double)(S.n_edges + S.n_tris), S.dhat);
        one.out[s].bad = 0;  // this broad phase's own verdict (set by its count pass)
    }
}

__device__ __forceinline__ int cell_of(double v, double h) { return (int)floor(v / h); }
// Bucket of a cell's entries of one body (0: the gel, 1: the indenter): a
// primitive looks only in the buckets of the bodies it can pair with (the
// indenter never with itself, the gel with itself only under self-contact),
// so a gel primitive away from the indenter scans empty buckets instead of
// its own mesh neighbours.
__device__ __forceinline__ uint32_t cell_hash(int ix, int iy, int iz, int body, uint32_t mask)
{
    return (((uint32_t)ix * 73856093u) ^ ((uint32_t)iy * 19349663u) ^ ((uint32_t)iz * 83492791u) ^
            (body ? 0x5bd1e995u : 0u)) & mask;
}

// Cells spanned per axis by one box are bounded by this; a larger span means
// a non-finite or absurd position, which is flagged and skipped.
constexpr int kMaxSpan = 4096;

// zero a per-scene int array: 0/1 hash bucket counts, 2 contact counts
__global__ void k_zero(Launch L, int which)
{
    int lb, s = scene_of_block(L, lb);
    const SceneDev &S = *L.sc[s];
    int32_t *a = which == 0 ? S.ht_count[0] : (which == 1 ? S.ht_count[1] : S.c_cnt);
    int64_t len = which == 2 ? (int64_t)S.n + 1 : ((int64_t)1 << S.ht_bits[which]) + 1;
    for (int64_t i = (int64_t)lb * blockDim.x + threadIdx.x; i < len; i += (int64_t)blocks_of(L, s) * blockDim.x)
        a[i] = 0;
}

// zero both hash tables' bucket counts in one launch (table 0's blocks first)
__global__ void k_zero_tables(Launch L)
{
    int lb, s = scene_of_block(L, lb);
    const SceneDev &S = *L.sc[s];
    const int64_t len0 = ((int64_t)1 << S.ht_bits[0]) + 1;
    const int n0 = blocks_for(len0);
    int t = lb < n0 ? 0 : 1;
    int64_t len = t == 0 ? len0 : ((int64_t)1 << S.ht_bits[1]) + 1;
    int64_t i = (int64_t)(t == 0 ? lb : lb - n0) * blockDim.x + threadIdx.x;
    if (i < len) S.ht_count[t][i] = 0;
}

template <bool FILL>
__device__ void hash_insert_body(const Launch &L, int s, const SceneDev &S, int lb, int table)
{
    int N = table == 0 ? S.n_tris : S.n_edges;
    const double *box = table == 0 ? S.tbox : S.ebox;
    int i = lb * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int body = i >= (table == 0 ? S.n_gel_tris : S.n_gel_edges) ? 1 : 0;
    // without self-contact no query looks for a gel edge: a gel edge pairs
    // with indenter edges only, found from the gel side (a < b)
    if (table == 1 && body == 0 && !S.self_contact) return;
    uint32_t mask = (1u << S.ht_bits[table]) - 1;
    int32_t *counter = S.ht_count[table];
    const int32_t *start = S.ht_start[table];
    int4 *entries = S.ht_entries[table];
    int cap = S.ht_cap[table];
    double h = *S.cell_h;
    int lo[3], hi[3];
    for (int c = 0; c < 3; ++c) {
        double a = box[c * N + i], b = box[(3 + c) * N + i];
        if (!(a <= b) || !((b - a) / h < (double)kMaxSpan)) {
            if (!FILL) atomicOr(&L.out[s].bad, 1);
            return;
        }
        lo[c] = cell_of(a, h);
        hi[c] = cell_of(b, h);
    }
    for (int iz = lo[2]; iz <= hi[2]; ++iz)
        for (int iy = lo[1]; iy <= hi[1]; ++iy)
            for (int ix = lo[0]; ix <= hi[0]; ++ix) {
                uint32_t bkt = cell_hash(ix, iy, iz, body, mask);
                int pos = atomicAdd(&counter[bkt], 1);
                if (FILL && start[bkt] + pos < cap) entries[start[bkt] + pos] = make_int4(ix, iy, iz, i);
            }
}

// triangles into table 0, then edges into table 1, in one launch
template <bool FILL>
__global__ void k_hash_insert_all(Launch L)
{
    int lb, s = scene_of_block(L, lb);
    const SceneDev &S = *L.sc[s];
    const int nt = blocks_for(S.n_tris);
    if (lb < nt)
        hash_insert_body<FILL>(L, s, S, lb, 0);
    else
        hash_insert_body<FILL>(L, s, S, lb - nt, 1);
}

__device__ __forceinline__ bool pt_admissible(const SceneDev &S, int a, int t0, int t1, int t2)
{
    if (a == t0 || a == t1 || a == t2) return false;
    bool ai = a >= S.n_gel, ti = t0 >= S.n_gel;
    if (ai && ti) return false;
    if (!ai && !ti && !S.self_contact) return false;
    if (S.fixed[a] && S.fixed[t0] && S.fixed[t1] && S.fixed[t2]) return false;
    return true;
}
__device__ __forceinline__ bool ee_admissible(const SceneDev &S, int a0, int a1, int b0, int b1)
{
    if (a0 == b0 || a0 == b1 || a1 == b0 || a1 == b1) return false;
    bool ai = a0 >= S.n_gel, bi = b0 >= S.n_gel;
    if (ai && bi) return false;
    if (!ai && !bi && !S.self_contact) return false;
    if (S.fixed[a0] && S.fixed[a1] && S.fixed[b0] && S.fixed[b1]) return false;
    return true;
}

// kLanesQ lanes per query primitive (PT: surface point index, EE: edge
// index) split the hash entries of the cells its box spans. COUNT: each lane's number of
// accepted pairs, and the query's total. Else each lane writes its pairs at
// q_off plus the counts of the lanes before it, and lane 0 sorts the query's
// segment by b (each pair is found in exactly one cell, so the sorted segment
// does not depend on the split). swept selects the output list.
template <int KIND, bool COUNT>
__device__ void query_body(const Launch &L, int s, const SceneDev &S, int lb, int swept)
{
    int NA = KIND == 0 ? S.n_pts : S.n_edges;
    int NB = KIND == 0 ? S.n_tris : S.n_edges;
    int64_t gt = (int64_t)lb * blockDim.x + threadIdx.x;
    int qa = (int)(gt / kLanesQ), lane = (int)(gt % kLanesQ);
    const bool live = qa < NA;  // whole lane groups
    const double *abox = KIND == 0 ? S.pbox : S.ebox;
    const double *bbox = KIND == 0 ? S.tbox : S.ebox;
    const int table = KIND == 0 ? 0 : 1;
    uint32_t mask = (1u << S.ht_bits[table]) - 1;
    const int32_t *start = S.ht_start[table];
    const int4 *entries = S.ht_entries[table];
    int cap = S.ht_cap[table];
    int qidx = (KIND == 0 ? 0 : S.n_pts) + qa;
    double h = *S.cell_h;
    double alo[3], ahi[3];
    int clo[3], chi[3];
    bool ok = live;
    for (int c = 0; c < 3 && ok; ++c) {
        alo[c] = abox[c * NA + qa];
        ahi[c] = abox[(3 + c) * NA + qa];
        if (!(alo[c] <= ahi[c]) || !((ahi[c] - alo[c]) / h < (double)kMaxSpan)) {
            ok = false;
            break;
        }
        clo[c] = cell_of(alo[c], h);
        chi[c] = cell_of(ahi[c], h);
    }
    int va0 = -1, va1 = -1, a_id = -1;
    if (ok) {
        if (KIND == 0) {
            va0 = S.pts[qa];
            a_id = va0;
        } else {
            va0 = S.ev[qa];
            va1 = S.ev[S.n_edges + qa];
            a_id = qa;
        }
    }
    int32_t *out = swept ? S.cand_sw : S.cand;
    int64_t ocap = swept ? S.sw_cap : S.cand_cap;
    int64_t o0 = 0, o = 0;
    // the count pass keeps a lane's first kQueryKeep pairs; the fill pass
    // copies them when that was all of them and walks the buckets again only
    // for lanes that found more
    int32_t *keep = S.q_keep + ((int64_t)kLanesQ * qidx + lane) * kQueryKeep;
    bool walk = ok;
    int count = 0;
    if (!COUNT && ok) {
        o0 = S.q_off[qidx];
        o = o0;
        for (int j = 0; j < lane; ++j) o += S.q_lane[(int64_t)kLanesQ * qidx + j];
        const int mine = S.q_lane[(int64_t)kLanesQ * qidx + lane];
        if (mine <= kQueryKeep) {
            walk = false;
            for (int j = 0; j < mine; ++j)
                if (o + j < ocap) {
                    out[o + j] = KIND;
                    out[ocap + o + j] = a_id;
                    out[2 * ocap + o + j] = keep[j];
                }
            count = mine;
        }
    }
    // bodies whose entries this query scans: a gel point or edge looks at
    // the indenter's, and at the gel's under self-contact; an indenter point
    // at the gel's; an indenter edge at none (its pairs with gel edges have
    // the gel edge first). Lanes split the (body, cell) pairs; the sort below
    // puts the query's pairs in b order whatever the split.
    const int b_gel = KIND == 0 ? S.n_gel_tris : S.n_gel_edges;
    bool scan0 = false, scan1 = false;
    if (ok) {
        const bool a_gel = KIND == 0 ? va0 < S.n_gel : qa < S.n_gel_edges;
        scan0 = a_gel ? S.self_contact != 0 : KIND == 0;
        scan1 = a_gel;
    }
    // the (body, cell) pairs in a fixed order, taken by all the query's
    // lanes together; a bucket's entries are split over them (entry k to
    // lane k mod kLanesQ): a query spans one to a few cells, and a bucket
    // beside the indenter holds tens of entries
    for (int body = 0; body < 2 && walk; ++body) {
        if (!(body == 0 ? scan0 : scan1)) continue;
        for (int iz = clo[2]; iz <= chi[2]; ++iz)
            for (int iy = clo[1]; iy <= chi[1]; ++iy)
                for (int ix = clo[0]; ix <= chi[0]; ++ix) {
                    uint32_t bkt = cell_hash(ix, iy, iz, body, mask);
                    int kend = min(start[bkt + 1], cap);
                    for (int k = start[bkt] + lane; k < kend; k += kLanesQ) {
                        int4 en = entries[k];
                        if (en.x != ix || en.y != iy || en.z != iz) continue;
                        int b = en.w;
                        if ((b >= b_gel) != (body == 1)) continue;  // another body's entry in this bucket
                        if (KIND == 1 && b <= qa) continue;
                        // box test first: most bucket entries fail it, and it
                        // needs no index loads
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
                        if (KIND == 0) {
                            if (!pt_admissible(S, va0, S.trv[b], S.trv[S.n_tris + b], S.trv[2 * S.n_tris + b])) continue;
                        } else {
                            if (!ee_admissible(S, va0, va1, S.ev[b], S.ev[S.n_edges + b])) continue;
                        }
                        if (COUNT && count < kQueryKeep) keep[count] = b;
                        if (!COUNT && o + count < ocap) {
                            out[o + count] = KIND;
                            out[ocap + o + count] = a_id;
                            out[2 * ocap + o + count] = b;
                        }
                        ++count;
                    }
                }
    }
    // the query's total over its lanes (every lane of the wavefront takes part)
    int tot = count;
    for (int m = 1; m < kLanesQ; m <<= 1) tot += __shfl_xor(tot, m, kWave);
    if (COUNT) {
        if (live) {
            S.q_lane[(int64_t)kLanesQ * qidx + lane] = count;
            if (lane == 0) S.q_count[qidx] = tot;
        }
    } else {
        __syncthreads();  // the lanes' writes are visible to lane 0
        if (ok && lane == 0) {
            int32_t *ob = out + 2 * ocap + o0;
            int len = (int)min((int64_t)tot, ocap - o0);  // equal to tot once the list has grown
            for (int i = 1; i < len; ++i) {
                int key = ob[i];
                int j = i - 1;
                while (j >= 0 && ob[j] > key) {
                    ob[j + 1] = ob[j];
                    --j;
                }
                ob[j + 1] = key;
            }
        }
    }
}

// point queries, then edge queries, in one launch
template <bool COUNT>
__global__ void __launch_bounds__(kBlock) k_query_all(Launch L, int swept)
{
    int lb, s = scene_of_block(L, lb);
    const SceneDev &S = *L.sc[s];
    const int np = blocks_for((int64_t)S.n_pts * kLanesQ);
    if (lb < np)
        query_body<0, COUNT>(L, s, S, lb, swept);
    else
        query_body<1, COUNT>(L, s, S, lb - np, swept);
}

// Static pairs from the swept list: a swept pair is static at x iff the two
// primitives' boxes at x (the static boxes, from k_boxes) overlap.
template <bool COMPACT>
__global__ void k_sw_filter(Launch L)
{
    int lb, s = scene_of_block(L, lb);
    const SceneDev &S = *L.sc[s];
    int64_t i = (int64_t)lb * blockDim.x + threadIdx.x;
    if (i >= S.n_sw_prev) return;
    const int64_t cap = S.sw_cap;
    int type = S.cand_sw[i], a = S.cand_sw[cap + i], b = S.cand_sw[2 * cap + i];
    if (COMPACT) {
        if (S.sw_flag[i]) {
            int64_t o = S.sw_off[i], oc = S.cand_cap;
            S.cand[o] = type;
            S.cand[oc + o] = a;
            S.cand[2 * oc + o] = b;
        }
        return;
    }
    const double *abox, *bbox;
    int ia, NA, NB;
    if (type == 0) {
        abox = S.pbox;
        NA = S.n_pts;
        ia = S.pt_idx[a];
        bbox = S.tbox;
        NB = S.n_tris;
    } else {
        abox = S.ebox;
        NA = S.n_edges;
        ia = a;
        bbox = S.ebox;
        NB = S.n_edges;
    }
    bool ov = true;
    for (int c = 0; c < 3; ++c) {
        double alo = abox[c * NA + ia], ahi = abox[(3 + c) * NA + ia];
        double blo = bbox[c * NB + b], bhi = bbox[(3 + c) * NB + b];
        ov = ov && (alo <= bhi) && (blo <= ahi);
    }
    S.sw_flag[i] = ov ? 1 : 0;
}

// ---------------------------------------------------------------------------
// narrow phase, barrier, incidence
// ---------------------------------------------------------------------------

__device__ __forceinline__ Topo topo_of(const SceneDev &S) { return Topo{S.ev, S.trv, S.n_edges, S.n_tris}; }

__global__ void k_narrow(Launch L)
{
    int lb, s = scene_of_block(L, lb);
    const SceneDev &S = *L.sc[s];
    int64_t i = (int64_t)lb * blockDim.x + threadIdx.x;
    if (i >= L.out[s].n_cand) return;
    int64_t cap = S.cand_cap;
    int type = S.cand[i], a = S.cand[cap + i], b = S.cand[2 * cap + i];
    int v[4];
    double x12[12];
    cand_vertices(topo_of(S), type, a, b, v);
    gather12(S.x, v, x12);
    double d = pair_distance(type, x12);
    S.cand_d[i] = d;
    S.act_flag[i] = d < S.dhat ? 1 : 0;
}

__global__ void k_compact(Launch L)
{
    int lb, s = scene_of_block(L, lb);
    const SceneDev &S = *L.sc[s];
    int64_t i = (int64_t)lb * blockDim.x + threadIdx.x;
    if (i < L.out[s].n_cand && S.act_flag[i]) S.act_idx[S.act_off[i]] = (int32_t)i;
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

// Cyclic Jacobi on a symmetric 5 x 5 matrix held in registers as its upper
// triangle (rows and columns past the restriction's dimension are zero and
// stay zero): eigenvalues left on the diagonal, eigenvectors in V's columns.
// Every lane of the wavefront runs it on the same matrix (no LDS round
// trips). The rotation zeroing (p, q) is the one of the 12 x 12 Jacobi below:
// a_pp -= t a_pq, a_qq += t a_pq, and for r != p, q
// (a_rp, a_rq) <- (c a_rp - s a_rq, s a_rp + c a_rq).
__device__ __forceinline__ constexpr int ut5(int a, int b)
{
    return a <= b ? a * 5 - a * (a - 1) / 2 + (b - a) : b * 5 - b * (b - 1) / 2 + (a - b);
}

__device__ __forceinline__ void jacobi5(double (&U)[15], double (&V)[5][5])
{
    double fro = 0.0;
#pragma unroll
    for (int a = 0; a < 5; ++a) {
#pragma unroll
        for (int b = 0; b < 5; ++b) V[a][b] = a == b ? 1.0 : 0.0;
#pragma unroll
        for (int b = a; b < 5; ++b) fro += (a == b ? 1.0 : 2.0) * U[ut5(a, b)] * U[ut5(a, b)];
    }
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0;
#pragma unroll
        for (int a = 0; a < 5; ++a)
#pragma unroll
            for (int b = a + 1; b < 5; ++b) off += U[ut5(a, b)] * U[ut5(a, b)];
        if (off <= 0.5e-36 * fro || off == 0.0) break;
#pragma unroll
        for (int p = 0; p < 5; ++p)
#pragma unroll
            for (int q = p + 1; q < 5; ++q) {
                const double apq = U[ut5(p, q)];
                if (apq == 0.0) continue;
                double theta = (U[ut5(q, q)] - U[ut5(p, p)]) / (2.0 * apq);
                double t = fabs(theta) > 1e150 ? 0.5 / theta
                                                : (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
                U[ut5(p, p)] -= t * apq;
                U[ut5(q, q)] += t * apq;
                U[ut5(p, q)] = 0.0;
#pragma unroll
                for (int r = 0; r < 5; ++r) {
                    if (r == p || r == q) continue;
                    double arp = U[ut5(r, p)], arq = U[ut5(r, q)];
                    U[ut5(r, p)] = c * arp - sn * arq;
                    U[ut5(r, q)] = sn * arp + c * arq;
                }
#pragma unroll
                for (int r = 0; r < 5; ++r) {
                    double vrp = V[r][p], vrq = V[r][q];
                    V[r][p] = c * vrp - sn * vrq;
                    V[r][q] = sn * vrp + c * vrq;
                }
            }
    }
}

// kappa * w * b(d) for each active pair: gradient and PSD Hessian.
// One wavefront per pair. Projected form: lanes evaluate Hessian entries, then
// a parallel cyclic Jacobi (six disjoint rotations per round) diagonalises the
// 12x12 in LDS and negative eigenvalues are clamped to zero; matrices that are
// already PSD are kept as assembled. Gauss-Newton form (S.barrier_gn): the
// entries kappa w b''(d) gd_p gd_q, PSD and rank one as they are.
template <class R>
__global__ void __launch_bounds__(64) k_barrier(Launch L)
{
    __shared__ double A[144], V[144], A0[144];
    __shared__ double rc[6], rs[6];
    __shared__ int rp[6], rq[6];
    int lbk, s = scene_of_block(L, lbk);
    const SceneDev &S = *L.sc[s];
    int64_t k = lbk;
    if (k >= L.out[s].n_act) return;
    const int lane = threadIdx.x;
    const int64_t cap = S.cand_cap, act_cap = S.act_cap;
    const double dhat = S.dhat, kappa = S.kappa;
    const double *edge_rest_sq = S.edge_rest_sq;
    const uint8_t *fixed = S.fixed;
    R *act_g = as<R>(S.act_g), *act_H = as<R>(S.act_H);
    int32_t *act_v = S.act_v;
    int ci = S.act_idx[k];
    int type = S.cand[ci], a = S.cand[cap + ci], b = S.cand[2 * cap + ci];
    int v[4];
    double x12[12];
    cand_vertices(topo_of(S), type, a, b, v);
    gather12(S.x, v, x12);
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
    if (S.barrier_gn) {
        double wb2 = kappa * w * bb[2];
        if (lane < 12) {
            double gv = w * bb[1] * gs_of(lane) * inv2d;
            if (moll) gv += bb[0] * m1 * gc_of(lane);
            act_g[(int64_t)lane * act_cap + k] = fixed[v[lane / 3]] ? R(0) : (R)(kappa * gv);
        }
        if (lane < 4) act_v[(int64_t)lane * act_cap + k] = v[lane];
        for (int e = lane; e < 144; e += 64) {
            int p = e / 12, q = e % 12;
            double val = wb2 * (gs_of(p) * inv2d) * (gs_of(q) * inv2d);
            if (fixed[v[p / 3]] || fixed[v[q / 3]]) val = 0.0;
            act_H[(int64_t)e * act_cap + k] = (R)val;
        }
        return;
    }
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
        act_g[(int64_t)lane * act_cap + k] = (R)(kappa * gv);
    }
    if (lane < 4) act_v[(int64_t)lane * act_cap + k] = v[lane];
    __syncthreads();

    if (!moll) {
        // Without the mollifier the pair Hessian's range lies in the span of
        // c (x) e_i (i = 0..2) and the columns of W: s_xx = 2 c c^T (x) I3,
        // grad s = 2 c (x) r and the envelope term W S W^T, so grad d and
        // the Hessian of d do too. Its PSD projection is that of its
        // restriction to an orthonormal basis Q of the span (k <= 5): a k x k
        // Jacobi instead of the 12 x 12 one.
        __shared__ double Q[5][12], AQ[12][5], M[5][5], MV[5][5];
        __shared__ int kq;
        if (lane == 0) {
            double cn = sqrt(dd.c[0] * dd.c[0] + dd.c[1] * dd.c[1] + dd.c[2] * dd.c[2] + dd.c[3] * dd.c[3]);
            for (int i = 0; i < 3; ++i)
                for (int pp = 0; pp < 12; ++pp) Q[i][pp] = pp % 3 == i ? dd.c[pp / 3] / cn : 0.0;
            int kk = 3;
            for (int m = 0; m < dd.np; ++m) {
                double w[12], n0 = 0.0;
                for (int pp = 0; pp < 12; ++pp) {
                    w[pp] = dd.W[pp][m];
                    n0 += w[pp] * w[pp];
                }
                for (int pass = 0; pass < 2; ++pass)  // Gram-Schmidt, repeated once
                    for (int aa2 = 0; aa2 < kk; ++aa2) {
                        double dt = 0.0;
                        for (int pp = 0; pp < 12; ++pp) dt += Q[aa2][pp] * w[pp];
                        for (int pp = 0; pp < 12; ++pp) w[pp] -= dt * Q[aa2][pp];
                    }
                double n = 0.0;
                for (int pp = 0; pp < 12; ++pp) n += w[pp] * w[pp];
                if (n > 1e-24 * n0) {  // a direction already in the span adds none
                    n = sqrt(n);
                    for (int pp = 0; pp < 12; ++pp) Q[kk][pp] = w[pp] / n;
                    ++kk;
                }
            }
            kq = kk;
        }
        __syncthreads();
        const int kd = kq;
        for (int t = lane; t < 12 * kd; t += 64) {  // A Q^T
            int i = t / kd, bq2 = t % kd;
            double acc = 0.0;
            for (int j = 0; j < 12; ++j) acc += A[i * 12 + j] * Q[bq2][j];
            AQ[i][bq2] = acc;
        }
        __syncthreads();
        for (int t = lane; t < kd * kd; t += 64) {  // M = Q A Q^T
            int aa2 = t / kd, bq2 = t % kd;
            double acc = 0.0;
            for (int i = 0; i < 12; ++i) acc += Q[aa2][i] * AQ[i][bq2];
            M[aa2][bq2] = acc;
        }
        __syncthreads();
        {
            double Ur[15], Vr[5][5];
#pragma unroll
            for (int aa2 = 0; aa2 < 5; ++aa2)
#pragma unroll
                for (int bq2 = aa2; bq2 < 5; ++bq2)
                    Ur[ut5(aa2, bq2)] = aa2 < kd && bq2 < kd ? 0.5 * (M[aa2][bq2] + M[bq2][aa2]) : 0.0;
            jacobi5(Ur, Vr);
            __syncthreads();  // every lane has read M
            if (lane == 0)
#pragma unroll
                for (int aa2 = 0; aa2 < 5; ++aa2)
#pragma unroll
                    for (int bq2 = 0; bq2 < 5; ++bq2) {
                        M[aa2][bq2] = aa2 == bq2 ? Ur[ut5(aa2, aa2)] : 0.0;
                        MV[aa2][bq2] = Vr[aa2][bq2];
                    }
        }
        __syncthreads();
        bool negr = false;
        for (int m = 0; m < kd; ++m) negr |= M[m][m] < 0.0;
        if (negr) {
            for (int t = lane; t < 12 * kd; t += 64) {  // P = Q^T MV
                int i = t / kd, m = t % kd;
                double acc = 0.0;
                for (int aa2 = 0; aa2 < kd; ++aa2) acc += Q[aa2][i] * MV[aa2][m];
                AQ[i][m] = acc;
            }
            __syncthreads();
            for (int e = lane; e < 144; e += 64) {
                int i = e / 12, j = e % 12;
                double val = 0.0;
                for (int m = 0; m < kd; ++m)
                    if (M[m][m] > 0.0) val += AQ[i][m] * M[m][m] * AQ[j][m];
                A[e] = val;
            }
            __syncthreads();
        }
        for (int e = lane; e < 144; e += 64) {
            int i = e / 12, j = e % 12;
            double val = negr ? A[e] : A0[e];
            if (fixed[v[i / 3]] || fixed[v[j / 3]]) val = 0.0;
            act_H[(int64_t)e * act_cap + k] = (R)val;
        }
        if (lane < 12 && fixed[v[lane / 3]]) act_g[(int64_t)lane * act_cap + k] = R(0);
        return;
    }

    // mollified edge pairs: parallel cyclic Jacobi
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
        act_H[(int64_t)e * act_cap + k] = (R)val;
    }
    if (lane < 12 && fixed[v[lane / 3]]) act_g[(int64_t)lane * act_cap + k] = R(0);
}


// Incidence lists of the active pairs' free vertices: a counting pass, a scan
// into c_ptr, then a fill in arbitrary order (c_tmp) and a rank pass that
// puts every row's entries in pair order. Rows with more than kHeavyRow
// entries are flagged and listed (their sums get a block each).
template <bool FILL>
__global__ void k_incidence(Launch L)
{
    int lb, s = scene_of_block(L, lb);
    const SceneDev &S = *L.sc[s];
    int64_t k = (int64_t)lb * blockDim.x + threadIdx.x;
    if (k >= L.out[s].n_pair) return;
    for (int a = 0; a < 4; ++a) {
        int v = S.act_v[(int64_t)a * S.act_cap + k];
        if (S.fixed[v]) continue;
        int pos = atomicAdd(&S.c_cnt[v], 1);
        if (FILL) {
            S.c_tmp[S.c_ptr[v] + pos] = (int32_t)(k * 4 + a);
            S.c_row[S.c_ptr[v] + pos] = v;
        }
    }
}

__global__ void k_heavy_flags(Launch L)
{
    int lb, s = scene_of_block(L, lb);
    const SceneDev &S = *L.sc[s];
    int i = lb * blockDim.x + threadIdx.x;
    if (i < S.n) S.hflag[i] = S.c_ptr[i + 1] - S.c_ptr[i] > kHeavyRow ? 1 : 0;
}

__global__ void k_heavy_rows(Launch L)
{
    int lb, s = scene_of_block(L, lb);
    const SceneDev &S = *L.sc[s];
    int i = lb * blockDim.x + threadIdx.x;
    if (i < S.n && S.hflag[i]) S.heavy_rows[S.heavy_idx[i]] = i;
}

// entry t goes to its row's segment at the rank of its key (pair*4 + slot)
__global__ void k_incidence_rank(Launch L)
{
    int lb, s = scene_of_block(L, lb);
    const SceneDev &S = *L.sc[s];
    int t = lb * blockDim.x + threadIdx.x;
    if (t >= S.c_ptr[S.n]) return;
    int v = S.c_row[t];
    int e0 = S.c_ptr[v], e1 = S.c_ptr[v + 1];
    int key = S.c_tmp[t], rank = 0;
    for (int u = e0; u < e1; ++u) rank += S.c_tmp[u] < key ? 1 : 0;
    S.c_list[e0 + rank] = key;
}

// ---------------------------------------------------------------------------
// lagged friction
// ---------------------------------------------------------------------------
// Frictional contact as in IPC, one lag per step: each pair active at x^t
// keeps its normal-force magnitude lambda = kappa w |b'(d)|, the coefficients
// c_k of its closest points and the unit normal n = r / d. During the step
// u = (I - n n^T) sum_k c_k (x_k - x^t_k) and D = mu lambda f0(|u|), f0 being
// IPC's C1 smoothing of |u| over e = eps_v h. Its Hessian (c c^T) (x) M,
// M = (f1/y)(P - uu^T/y^2) + f0'' uu^T/y^2, is PSD without projection.

// friction set from the active pairs at x (called with x = x^t)
__global__ void k_friction_lag(Launch L)
{
    int lb, s = scene_of_block(L, lb);
    const SceneDev &S = *L.sc[s];
    int64_t k = (int64_t)lb * blockDim.x + threadIdx.x;
    if (k >= L.out[s].n_act) return;
    const int64_t cap = S.cand_cap, fc = S.fric_cap;
    int ci = S.act_idx[k];
    int type = S.cand[ci], a = S.cand[cap + ci], b = S.cand[2 * cap + ci];
    int v[4];
    double x12[12];
    cand_vertices(topo_of(S), type, a, b, v);
    gather12(S.x, v, x12);
    DistSpec sp = type == 0 ? c_pt_spec[classify_pt(x12)] : c_ee_spec[classify_ee(x12)];
    double r[3], c[4], u[2][3], G[3];
    double d = sqrt(dist_residual(sp, x12, r, c, u, G));
    double bb[3];
    barrier3(d, S.dhat, bb);
    double w = 1.0;
    if (type == 1) {
        double eps_x = kMollifier * S.edge_rest_sq[a] * S.edge_rest_sq[b];
        double ea[3] = {x12[3] - x12[0], x12[4] - x12[1], x12[5] - x12[2]};
        double eb[3] = {x12[9] - x12[6], x12[10] - x12[7], x12[11] - x12[8]};
        double cr[3] = {ea[1] * eb[2] - ea[2] * eb[1], ea[2] * eb[0] - ea[0] * eb[2], ea[0] * eb[1] - ea[1] * eb[0]};
        double cv = d3(cr, cr);
        if (cv < eps_x) w = -cv * cv / (eps_x * eps_x) + 2.0 * cv / eps_x;
    }
    for (int q = 0; q < 4; ++q) {
        S.fric_v[q * fc + k] = v[q];
        S.fric_c[q * fc + k] = c[q];
    }
    for (int i = 0; i < 3; ++i) S.fric_nrm[i * fc + k] = r[i] / d;
    S.fric_lam[k] = S.kappa * w * fabs(bb[1]);
}

// tangential displacement u of friction pair j at x and its length
__device__ __forceinline__ double fric_u(const SceneDev &S, const double *x, int64_t j, int v[4], double c[4],
                                         double n[3], double u[3])
{
    const int64_t fc = S.fric_cap;
    double r[3] = {0.0, 0.0, 0.0};
    for (int q = 0; q < 4; ++q) {
        v[q] = S.fric_v[q * fc + j];
        c[q] = S.fric_c[q * fc + j];
    }
    for (int i = 0; i < 3; ++i) n[i] = S.fric_nrm[i * fc + j];
    for (int q = 0; q < 4; ++q)
        for (int i = 0; i < 3; ++i) r[i] += c[q] * (x[3 * v[q] + i] - S.xt[3 * v[q] + i]);
    double rn = d3(r, n);
    for (int i = 0; i < 3; ++i) u[i] = r[i] - rn * n[i];
    return sqrt(d3(u, u));
}

// friction pair j as active pair n_act + j: gradient and PSD Hessian at x
template <class R>
__global__ void __launch_bounds__(kBlock) k_friction(Launch L)
{
    int lb, s = scene_of_block(L, lb);
    const SceneDev &S = *L.sc[s];
    int64_t j = (int64_t)lb * blockDim.x + threadIdx.x;
    if (j >= S.n_fric) return;
    int v[4];
    double c[4], n[3], u[3];
    double y = fric_u(S, S.x, j, v, c, n, u);
    double e = S.eps_fric, ml = S.mu_fric * S.fric_lam[j];
    double f1y = y < e ? 2.0 / e - y / (e * e) : 1.0 / y;
    double f2 = y < e ? -2.0 * y / (e * e) + 2.0 / e : 0.0;
    double M[9];
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) {
            double P = (i == k ? 1.0 : 0.0) - n[i] * n[k];
            if (y > 0.0) {
                double uu = u[i] * u[k] / (y * y);
                M[3 * i + k] = f1y * (P - uu) + fmax(f2, 0.0) * uu;
            } else {
                M[3 * i + k] = (2.0 / e) * P;
            }
        }
    const int64_t cap = S.act_cap, q = L.out[s].n_act + j;
    R *act_g = as<R>(S.act_g), *act_H = as<R>(S.act_H);
    bool fx[4];
    for (int a = 0; a < 4; ++a) {
        S.act_v[a * cap + q] = v[a];
        fx[a] = S.fixed[v[a]] != 0;
        for (int i = 0; i < 3; ++i) act_g[(int64_t)(3 * a + i) * cap + q] = fx[a] ? R(0) : (R)(ml * c[a] * f1y * u[i]);
    }
    for (int a = 0; a < 4; ++a)
        for (int i = 0; i < 3; ++i)
            for (int b = 0; b < 4; ++b)
                for (int k = 0; k < 3; ++k) {
                    double h = (fx[a] || fx[b]) ? 0.0 : ml * c[a] * c[b] * M[3 * i + k];
                    act_H[(int64_t)((3 * a + i) * 12 + 3 * b + k) * cap + q] = (R)h;
                }
}

__global__ void k_set_npair(Launch one)
{
    int lb, s = scene_of_block(one, lb);
    const SceneDev &S = *one.sc[s];
    if (threadIdx.x == 0) one.out[s].n_pair = one.out[s].n_act + S.n_fric;
}

// friction energy partials, after the body and barrier partials
__global__ void __launch_bounds__(kBlock) k_energy_fric(Launch L, Launch body, Launch cont, int trial)
{
    int lb, s = scene_of_block(L, lb);
    const SceneDev &S = *L.sc[s];
    const double *x = trial ? S.xtrial : S.x;
    int64_t j = (int64_t)lb * blockDim.x + threadIdx.x;
    double val = 0.0;
    if (j < S.n_fric) {
        int v[4];
        double c[4], n[3], u[3];
        double y = fric_u(S, x, j, v, c, n, u);
        double e = S.eps_fric;
        double f0 = y < e ? -y * y * y / (3.0 * e * e) + y * y / e + e / 3.0 : y;
        val = S.mu_fric * S.fric_lam[j] * f0;
    }
    CSum cs = {val, 0.0};
    cs = block_csum(cs);
    if (threadIdx.x == 0) {
        int off = blocks_of(body, s) + blocks_of(cont, s) + lb;
        S.red[2 * off] = cs.s;
        S.red[2 * off + 1] = cs.c;
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

template <class R>
__global__ void __launch_bounds__(kBlock) k_accd(Launch L)
{
    int lb, s = scene_of_block(L, lb);
    const SceneDev &S = *L.sc[s];
    int64_t i = (int64_t)lb * blockDim.x + threadIdx.x;
    double t = 1.0;
    if (i < L.out[s].n_sw) {
        int64_t cap = S.sw_cap;
        int type = S.cand_sw[i], a = S.cand_sw[cap + i], b = S.cand_sw[2 * cap + i];
        int v[4];
        double x12[12], p12[12];
        cand_vertices(topo_of(S), type, a, b, v);
        gather12(S.x, v, x12);
        const R *p = as<R>(S.sol);
        for (int k = 0; k < 4; ++k)
            for (int c = 0; c < 3; ++c) p12[3 * k + c] = (double)p[3 * v[k] + c];
        t = accd_pair(type, x12, p12, S.ccd_s, 1.0, S.ccd_max_iter);
    }
    t = block_min_all(t);
    if (threadIdx.x == 0) S.red[lb] = t;
}

__global__ void k_final_ccd(Launch one, Launch prod)
{
    int lb, s = scene_of_block(one, lb);
    const SceneDev &S = *one.sc[s];
    int nb = blocks_of(prod, s);
    double v = 1.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) v = fmin(v, S.red[i]);
    v = block_min_all(v);
    if (threadIdx.x == 0) one.out[s].alpha_ccd = v;
}

// barrier energy over the swept candidates, partials after the body partials
__global__ void __launch_bounds__(kBlock) k_energy_contact(Launch L, Launch body, int trial)
{
    int lb, s = scene_of_block(L, lb);
    const SceneDev &S = *L.sc[s];
    const double *x = trial ? S.xtrial : S.x;
    int64_t i = (int64_t)lb * blockDim.x + threadIdx.x;
    double val = 0.0;
    if (i < L.out[s].n_sw) {
        int64_t cap = S.sw_cap;
        int type = S.cand_sw[i], a = S.cand_sw[cap + i], b = S.cand_sw[2 * cap + i];
        int v[4];
        double x12[12];
        cand_vertices(topo_of(S), type, a, b, v);
        gather12(x, v, x12);
        double d = pair_distance(type, x12);
        if (!(d > 0.0)) {
            atomicOr(&L.out[s].infeasible, 1);
        } else if (d < S.dhat) {
            double bb[3];
            barrier3(d, S.dhat, bb);
            double w = 1.0;
            if (type == 1) {
                double eps_x = kMollifier * S.edge_rest_sq[a] * S.edge_rest_sq[b];
                double ea[3] = {x12[3] - x12[0], x12[4] - x12[1], x12[5] - x12[2]};
                double eb[3] = {x12[9] - x12[6], x12[10] - x12[7], x12[11] - x12[8]};
                double cr[3] = {ea[1] * eb[2] - ea[2] * eb[1], ea[2] * eb[0] - ea[0] * eb[2], ea[0] * eb[1] - ea[1] * eb[0]};
                double c = d3(cr, cr);
                if (c < eps_x) w = -c * c / (eps_x * eps_x) + 2.0 * c / eps_x;
            }
            val = S.kappa * w * bb[0];
        }
    }
    CSum cs = {val, 0.0};
    cs = block_csum(cs);
    if (threadIdx.x == 0) {
        int off = blocks_of(body, s) + lb;
        S.red[2 * off] = cs.s;
        S.red[2 * off + 1] = cs.c;
    }
}

__global__ void k_clear_infeasible(Launch one)
{
    int lb, s = scene_of_block(one, lb);
    if (threadIdx.x == 0) one.out[s].infeasible = 0;
}

// final compensated sum over the body and contact partials of one scene
__global__ void k_energy_final(Launch one, Launch body, Launch cont, Launch fric)
{
    int lb, s = scene_of_block(one, lb);
    const SceneDev &S = *one.sc[s];
    int nb = blocks_of(body, s) + blocks_of(cont, s) + blocks_of(fric, s);
    CSum acc = {0.0, 0.0};
    for (int i = threadIdx.x; i < nb; i += blockDim.x) {
        CSum t = {S.red[2 * i], S.red[2 * i + 1]};
        acc = csum_add(acc, t);
    }
    acc = block_csum(acc);
    if (threadIdx.x == 0) one.out[s].energy = acc.s + acc.c;
}

// ---------------------------------------------------------------------------
// host drivers
// ---------------------------------------------------------------------------

static bool mixed(const Batch &b) { return b.sc[0]->prm.precision == IPC_MIXED; }

static std::vector<int32_t> per_scene(const Batch &b, PhaseKind gate, const std::function<int32_t(const Scene &)> &f)
{
    std::vector<int32_t> v(b.sc.size());
    for (size_t i = 0; i < b.sc.size(); ++i)
        v[i] = b.h_off[gate][i + 1] > b.h_off[gate][i] ? f(*b.sc[i]) : 0;
    return v;
}

static void one_per_active(Batch &b, PhaseKind gate)
{
    b.set_phase(kPhOne, per_scene(b, gate, [](const Scene &) { return 1; }));
}

// Candidate pairs at x (which 0) or over [x, x+p] (which 1) for every scene
// active in the vertex phase. Hash tables that overflow their entry capacity
// are grown and the phase is redone.
void run_broad_phase(Batch &b, int which)
{
    hipEvent_t ev[2];
    b.prof_begin(kProfBroad, ev);
    bool mx = mixed(b);
    if (mx)
        IPC_LAUNCH(b, k_boxes_all<float>, kPhPrims, kBlock, which, 1);
    else
        IPC_LAUNCH(b, k_boxes_all<double>, kPhPrims, kBlock, which, 1);
    one_per_active(b, kPhVert);
    IPC_LAUNCH(b, k_cell_size, kPhOne, kBlock);
    size_t ns = b.sc.size();
    std::vector<uint8_t> redo(ns, 0), live(ns, 0);
    for (size_t i = 0; i < ns; ++i) live[i] = b.h_off[kPhVert][i + 1] > b.h_off[kPhVert][i];
    auto tiles_of = [&](int t) {
        std::vector<int32_t> v(ns, 0);
        for (size_t i = 0; i < ns; ++i)
            if (live[i]) v[i] = nblocks((int64_t(1) << b.sc[i]->h.ht_bits[t]) + 1);
        return v;
    };
    for (int attempt = 0; attempt < 4; ++attempt) {
        std::vector<int64_t> lt(ns, -1), le(ns, -1), lq(ns, -1);
        for (size_t i = 0; i < ns; ++i) {
            if (!live[i]) continue;
            const SceneDev &S = b.sc[i]->h;
            lt[i] = int64_t(1) << S.ht_bits[0];
            le[i] = int64_t(1) << S.ht_bits[1];
            lq[i] = (int64_t)S.n_pts + S.n_edges;
        }
        // zero the buckets, count, scan, zero again, fill; then count queries
        std::vector<int32_t> zt = tiles_of(0), ze = tiles_of(1);
        for (size_t i = 0; i < ns; ++i) zt[i] += ze[i];
        b.set_phase(kPhTilesTE, zt);
        IPC_LAUNCH(b, k_zero_tables, kPhTilesTE, kBlock);
        IPC_LAUNCH(b, k_hash_insert_all<false>, kPhTE, kBlock);
        segmented_scan(b, kScanTri, kPhTilesT, lt);
        segmented_scan(b, kScanEdge, kPhTilesE, le);
        IPC_LAUNCH(b, k_zero_tables, kPhTilesTE, kBlock);
        IPC_LAUNCH(b, k_hash_insert_all<true>, kPhTE, kBlock);
        IPC_LAUNCH(b, k_query_all<true>, kPhQAll, kBlock, which);
        segmented_scan(b, kScanQuery, kPhTilesQ, lq, which);
        b.read_out();
        bool any_redo = false;
        for (size_t i = 0; i < ns; ++i) {
            redo[i] = 0;
            if (!live[i]) continue;
            Scene &s = *b.sc[i];
            if (b.h_out[i].bad) {
                b.fail[i] = IPC_E_INFEASIBLE;
                continue;
            }
            try {
                if (b.h_out[i].ent_tri > s.h.ht_cap[0]) {
                    grow_table(s, 0, (int64_t)b.h_out[i].ent_tri * 3 / 2 + 1024);
                    redo[i] = 1;
                }
                if (b.h_out[i].ent_edge > s.h.ht_cap[1]) {
                    grow_table(s, 1, (int64_t)b.h_out[i].ent_edge * 3 / 2 + 1024);
                    redo[i] = 1;
                }
            } catch (const OomError &) {
                b.fail[i] = IPC_E_OOM;
                redo[i] = 0;
            }
            any_redo |= redo[i] != 0;
        }
        if (any_redo && attempt < 3) {
            b.upload_views();
            continue;
        }
        for (size_t i = 0; i < ns; ++i) {
            if (!live[i] || b.fail[i]) continue;
            if (redo[i]) {
                b.fail[i] = IPC_E_CAPACITY;
                continue;
            }
            try {
                grow_candidates(*b.sc[i], which, which ? b.h_out[i].n_sw : b.h_out[i].n_cand);
            } catch (const OomError &) {
                b.fail[i] = IPC_E_OOM;
            }
        }
        b.upload_views();
        // failed scenes still run the fill pass: every write is bounded by
        // their list capacity, and the caller drops them afterwards
        IPC_LAUNCH(b, k_query_all<false>, kPhQAll, kBlock, which);
        b.prof_end(kProfBroad, ev);
        return;
    }
}

void run_static_from_swept(Batch &b)
{
    hipEvent_t ev[2];
    b.prof_begin(kProfBroad, ev);
    size_t ns = b.sc.size();
    if (mixed(b))
        IPC_LAUNCH(b, k_boxes_all<float>, kPhPrims, kBlock, 0, 0);
    else
        IPC_LAUNCH(b, k_boxes_all<double>, kPhPrims, kBlock, 0, 0);
    std::vector<int32_t> nb(ns, 0);
    std::vector<int64_t> len(ns, -1);
    for (size_t i = 0; i < ns; ++i) {
        if (b.h_off[kPhVert][i + 1] == b.h_off[kPhVert][i]) continue;
        Scene &sc = *b.sc[i];
        nb[i] = nblocks(sc.sw_n);
        len[i] = sc.sw_n;
        if (sc.h.n_sw_prev != sc.sw_n) {
            sc.h.n_sw_prev = sc.sw_n;
            sc.dev_dirty = true;
        }
    }
    b.upload_views();
    b.set_phase(kPhCandSw, nb);
    IPC_LAUNCH(b, k_sw_filter<false>, kPhCandSw, kBlock);
    segmented_scan(b, kScanSwFilter, kPhTilesQ, len);
    b.read_out();
    for (size_t i = 0; i < ns; ++i) {
        if (len[i] < 0) continue;
        try {
            grow_candidates(*b.sc[i], 0, b.h_out[i].n_cand);
        } catch (const OomError &) {
            b.fail[i] = IPC_E_OOM;
            nb[i] = 0;
        }
    }
    b.upload_views();
    b.set_phase(kPhCandSw, nb);
    IPC_LAUNCH(b, k_sw_filter<true>, kPhCandSw, kBlock);
    b.prof_end(kProfBroad, ev);
}

// distances of the static candidates; active = d < dhat, compacted
void run_narrow_phase(Batch &b)
{
    hipEvent_t ev[2];
    b.prof_begin(kProfBarrier, ev);
    size_t ns = b.sc.size();
    std::vector<int64_t> len(ns, -1);
    std::vector<int32_t> nbk(ns, 0);
    for (size_t i = 0; i < ns; ++i) {
        if (b.h_off[kPhVert][i + 1] == b.h_off[kPhVert][i]) continue;
        len[i] = b.h_out[i].n_cand;
        nbk[i] = nblocks(b.h_out[i].n_cand);
    }
    b.set_phase(kPhCand, nbk);
    IPC_LAUNCH(b, k_narrow, kPhCand, kBlock);
    segmented_scan(b, kScanActive, kPhTilesA, len);
    b.read_out();
    bool dropped = false;
    for (size_t i = 0; i < ns; ++i) {
        if (len[i] < 0) continue;
        try {
            grow_active(*b.sc[i], pair_count(*b.sc[i], b.h_out[i]));
        } catch (const OomError &) {
            b.fail[i] = IPC_E_OOM;
            nbk[i] = 0;
            dropped = true;
        }
    }
    b.upload_views();
    if (dropped) b.set_phase(kPhCand, nbk);
    IPC_LAUNCH(b, k_compact, kPhCand, kBlock);
    b.prof_end(kProfBarrier, ev);
}

void launch_barrier(Batch &b)
{
    hipEvent_t ev[2];
    b.prof_begin(kProfBarrier, ev);
    size_t ns = b.sc.size();
    std::vector<int32_t> na(ns);
    for (size_t i = 0; i < ns; ++i) na[i] = b.h_off[kPhVert][i + 1] > b.h_off[kPhVert][i] ? b.h_out[i].n_act : 0;
    b.set_phase(kPhAct, na);
    if (mixed(b))
        IPC_LAUNCH(b, k_barrier<float>, kPhAct, 64);
    else
        IPC_LAUNCH(b, k_barrier<double>, kPhAct, 64);
    b.prof_end(kProfBarrier, ev);
}

void launch_contact_incidence(Batch &b)
{
    size_t ns = b.sc.size();
    std::vector<int32_t> na(ns), ne(ns), nz(ns);
    std::vector<int64_t> len(ns, -1);
    for (size_t i = 0; i < ns; ++i) {
        bool on = b.h_off[kPhVert][i + 1] > b.h_off[kPhVert][i];
        na[i] = on ? nblocks(pair_count(*b.sc[i], b.h_out[i])) : 0;
        ne[i] = on ? nblocks(4 * pair_count(*b.sc[i], b.h_out[i])) : 0;
        nz[i] = on ? nblocks((int64_t)b.sc[i]->h.n + 1) : 0;
        len[i] = on ? b.sc[i]->h.n : -1;
    }
    b.set_phase(kPhActT, na);
    b.set_phase(kPhEnt, ne);
    b.set_phase(kPhTilesC, nz);
    IPC_LAUNCH(b, k_zero, kPhTilesC, kBlock, 2);
    IPC_LAUNCH(b, k_incidence<false>, kPhActT, kBlock);
    segmented_scan(b, kScanContact, kPhTilesC, len);
    IPC_LAUNCH(b, k_heavy_flags, kPhVert, kBlock);
    segmented_scan(b, kScanHeavy, kPhTilesC, len);
    IPC_LAUNCH(b, k_heavy_rows, kPhVert, kBlock);
    b.set_phase(kPhTilesC, nz);
    IPC_LAUNCH(b, k_zero, kPhTilesC, kBlock, 2);
    IPC_LAUNCH(b, k_incidence<true>, kPhActT, kBlock);
    IPC_LAUNCH(b, k_incidence_rank, kPhEnt, kBlock);
    set_heavy_phase(b);
}

void set_heavy_phase(Batch &b)
{
    size_t ns = b.sc.size();
    std::vector<int32_t> nh(ns);
    for (size_t i = 0; i < ns; ++i) {
        bool on = b.h_off[kPhVert][i + 1] > b.h_off[kPhVert][i];
        const SceneDev &H = b.sc[i]->h;
        nh[i] = on ? H.nb_vert + heavy_bound(pair_count(*b.sc[i], b.h_out[i]), H.n) : 0;
    }
    b.set_phase(kPhVertH, nh);
}

void launch_friction_lag(Batch &b)
{
    size_t ns = b.sc.size();
    std::vector<int32_t> na(ns, 0);
    for (size_t i = 0; i < ns; ++i)
        if (b.h_off[kPhVert][i + 1] > b.h_off[kPhVert][i]) na[i] = nblocks(b.h_out[i].n_act);
    b.set_phase(kPhActT, na);
    IPC_LAUNCH(b, k_friction_lag, kPhActT, kBlock);
}

void launch_friction(Batch &b)
{
    b.set_phase(kPhFric, per_scene(b, kPhVert, [](const Scene &s) { return nblocks(s.h.n_fric); }));
    if (mixed(b))
        IPC_LAUNCH(b, k_friction<float>, kPhFric, kBlock);
    else
        IPC_LAUNCH(b, k_friction<double>, kPhFric, kBlock);
    one_per_active(b, kPhVert);
    IPC_LAUNCH(b, k_set_npair, kPhOne, 64);
}

void run_ccd(Batch &b)
{
    hipEvent_t ev[2];
    b.prof_begin(kProfCcd, ev);
    size_t ns = b.sc.size();
    std::vector<int32_t> nb(ns);
    for (size_t i = 0; i < ns; ++i)
        nb[i] = b.h_off[kPhVert][i + 1] > b.h_off[kPhVert][i] ? nblocks(b.h_out[i].n_sw) : 0;
    b.set_phase(kPhCandSw, nb);
    if (mixed(b))
        IPC_LAUNCH(b, k_accd<float>, kPhCandSw, kBlock);
    else
        IPC_LAUNCH(b, k_accd<double>, kPhCandSw, kBlock);
    one_per_active(b, kPhVert);
    IPC_LAUNCH(b, k_final_ccd, kPhOne, kBlock, b.launch(kPhCandSw));
    b.prof_end(kProfCcd, ev);
}

void launch_energy_body(Batch &b, bool trial);

// Incremental potential (FP64, compensated) at x or x_trial over the swept
// candidate list, for every scene active in the vertex phase.
void run_energy(Batch &b, bool trial)
{
    hipEvent_t ev[2];
    b.prof_begin(kProfEnergy, ev);
    size_t ns = b.sc.size();
    std::vector<int32_t> nb(ns);
    for (size_t i = 0; i < ns; ++i) {
        nb[i] = b.h_off[kPhVert][i + 1] > b.h_off[kPhVert][i] ? nblocks(b.h_out[i].n_sw) : 0;
        b.h_out[i].infeasible = 0;
    }
    b.set_phase(kPhCandSw, nb);
    b.set_phase(kPhBody, per_scene(b, kPhVert, [](const Scene &s) { return nblocks((int64_t)s.h.m + s.h.n); }));
    b.set_phase(kPhFric, per_scene(b, kPhVert, [](const Scene &s) { return nblocks(s.h.n_fric); }));
    one_per_active(b, kPhVert);
    IPC_LAUNCH(b, k_clear_infeasible, kPhOne, 64);
    launch_energy_body(b, trial);
    IPC_LAUNCH(b, k_energy_contact, kPhCandSw, kBlock, b.launch(kPhBody), (int)trial);
    IPC_LAUNCH(b, k_energy_fric, kPhFric, kBlock, b.launch(kPhBody), b.launch(kPhCandSw), (int)trial);
    one_per_active(b, kPhVert);
    IPC_LAUNCH(b, k_energy_final, kPhOne, kBlock, b.launch(kPhBody), b.launch(kPhCandSw), b.launch(kPhFric));
    b.prof_end(kProfEnergy, ev);
}

}  // namespace ipcg
