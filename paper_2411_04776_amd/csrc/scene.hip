// scene.hip -- scene construction, the Newton step driver and the C ABI.
//
// One step (the GIPC step of the paper's "General GIPC Simulation Pipeline":
// targets of the kinematic vertices are set, then the solver computes new
// positions) is backward Euler on the IPC incremental potential:
//   begin: x^t kept, predictor xtilde = x^t + h v^t + h^2 g, indenter targets
//          yhat = R Y + c from the requested pose;
//   Newton iteration: static candidates at x and their distances (active if
//          d < dhat), barrier and elastic derivatives, deterministic assembly,
//          block-Jacobi PCG for p, stop if |p|_inf <= newton_tol; otherwise
//          swept candidates over [x, x + p], additive CCD bound alpha_ccd,
//          halve alpha from min(1, alpha_ccd) until Phi(x + alpha p) <= Phi(x);
//   commit: v = (x - x^t) / h.
#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <unordered_map>

#include "ipc_internal.h"

namespace ipcg {

static thread_local std::string g_last_error;
void set_error(const std::string &m) { g_last_error = m; }

void *DeviceArena::alloc(size_t bytes)
{
    if (rt.mem_budget > 0 && used + (int64_t)bytes > rt.mem_budget) return nullptr;
    void *p = nullptr;
    if (rt.alloc) {
        p = rt.alloc(bytes, rt.stream, rt.user);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        p = nullptr;
    }
    if (p) used += (int64_t)bytes;
    return p;
}

void DeviceArena::release(void *p, size_t bytes)
{
    if (!p) return;
    if (rt.free)
        rt.free(p, bytes, rt.stream, rt.user);
    else
        (void)hipFree(p);
    used -= (int64_t)bytes;
}

void dfree(Scene &s, void *p)
{
    for (auto it = s.owned.begin(); it != s.owned.end(); ++it)
        if (it->first == p) {
            s.arena.release(p, it->second);
            s.owned.erase(it);
            return;
        }
}

void prof_begin(Scene &s, int kernel, hipEvent_t *pair)
{
    if (!s.prof) return;
    for (int k = 0; k < 2; ++k) {
        if (s.ev_pool.empty()) {
            hipEvent_t e;
            IPC_HIP(hipEventCreate(&e));
            s.ev_pool.push_back(e);
        }
        pair[k] = s.ev_pool.back();
        s.ev_pool.pop_back();
    }
    IPC_HIP(hipEventRecord(pair[0], s.stream));
}

void prof_end(Scene &s, int kernel, hipEvent_t *pair)
{
    if (!s.prof) return;
    IPC_HIP(hipEventRecord(pair[1], s.stream));
    s.ev_pending.push_back({kernel, {pair[0], pair[1]}});
}

void prof_collect(Scene &s)
{
    if (s.ev_pending.empty()) return;
    for (auto &p : s.ev_pending) {
        float ms = 0.f;
        IPC_HIP(hipEventSynchronize(p.second.second));
        IPC_HIP(hipEventElapsedTime(&ms, p.second.first, p.second.second));
        s.prof_acc[p.first].launches++;
        s.prof_acc[p.first].ms += ms;
        s.ev_pool.push_back(p.second.first);
        s.ev_pool.push_back(p.second.second);
    }
    s.ev_pending.clear();
}

Scene::~Scene()
{
    if (stream) (void)hipStreamSynchronize(stream);
    for (auto &p : ev_pending) {
        ev_pool.push_back(p.second.first);
        ev_pool.push_back(p.second.second);
    }
    for (auto e : ev_pool) (void)hipEventDestroy(e);
    for (auto &o : owned) arena.release(o.first, o.second);
    owned.clear();
    if (hb) (void)hipHostFree(hb);
}

// ---------------------------------------------------------------------------
// host-side topology
// ---------------------------------------------------------------------------

static void rotate_min_first(int32_t *t)
{
    int32_t a = t[0], b = t[1], c = t[2];
    if (b < a && b < c) {
        t[0] = b; t[1] = c; t[2] = a;
    } else if (c < a && c < b) {
        t[0] = c; t[1] = a; t[2] = b;
    }
}

static void canonical_tris(std::vector<std::array<int32_t, 3>> &tris)
{
    for (auto &t : tris) rotate_min_first(t.data());
    std::sort(tris.begin(), tris.end());
}

static std::vector<std::array<int32_t, 2>> unique_edges(const std::vector<std::array<int32_t, 3>> &tris)
{
    std::vector<std::array<int32_t, 2>> e;
    e.reserve(tris.size() * 3);
    for (auto &t : tris)
        for (int k = 0; k < 3; ++k) {
            int32_t a = t[k], b = t[(k + 1) % 3];
            e.push_back({std::min(a, b), std::max(a, b)});
        }
    std::sort(e.begin(), e.end());
    e.erase(std::unique(e.begin(), e.end()), e.end());
    return e;
}

static void pose_apply(const double *P, const double *y, double *o)
{
    for (int i = 0; i < 3; ++i) o[i] = P[i * 4 + 0] * y[0] + P[i * 4 + 1] * y[1] + P[i * 4 + 2] * y[2] + P[i * 4 + 3];
}

template <class T>
static T *upload(Scene &s, const std::vector<T> &h)
{
    T *d = dalloc<T>(s, h.size());
    if (!h.empty()) IPC_HIP(hipMemcpyAsync(d, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice, s.stream));
    return d;
}

static int ceil_log2(int64_t v)
{
    int b = 0;
    while ((int64_t(1) << b) < v) ++b;
    return b;
}

static int64_t partial_need(const Scene &s, int64_t nc)
{
    return 2 * ((int64_t)nblocks((int64_t)s.m + s.n) + nblocks(nc) + 16);
}

static int32_t build_scene(Scene &s, const ipc_scene_desc &d)
{
    const int ng = d.n_verts, m = d.n_tets, ni = d.n_ind_verts;
    s.n_gel = ng;
    s.n_ind = ni;
    s.n = ng + ni;
    s.m = m;
    const int n = s.n;
    // ---- validation
    for (int64_t k = 0; k < 4 * (int64_t)m; ++k)
        if (d.T[k] < 0 || d.T[k] >= ng) {
            set_error("tet index out of range");
            return IPC_E_BAD_MESH;
        }
    for (int64_t k = 0; k < 3 * (int64_t)d.n_ind_tris; ++k)
        if (d.ind_tris[k] < 0 || d.ind_tris[k] >= ni) {
            set_error("indenter triangle index out of range");
            return IPC_E_BAD_MESH;
        }
    std::vector<double> X0(3 * (size_t)n);
    std::memcpy(X0.data(), d.X, sizeof(double) * 3 * ng);
    for (int j = 0; j < ni; ++j) pose_apply(d.ind_pose0, d.ind_Y + 3 * j, &X0[3 * (size_t)(ng + j)]);
    for (int e = 0; e < m; ++e) {
        const int32_t *t = d.T + 4 * e;
        double D[9];
        for (int i = 0; i < 3; ++i)
            for (int c = 0; c < 3; ++c) D[i * 3 + c] = d.X[3 * t[c + 1] + i] - d.X[3 * t[0] + i];
        double det = D[0] * (D[4] * D[8] - D[5] * D[7]) - D[1] * (D[3] * D[8] - D[5] * D[6]) +
                     D[2] * (D[3] * D[7] - D[4] * D[6]);
        if (!(det > 0.0)) {
            set_error("tet with non-positive rest volume");
            return IPC_E_BAD_MESH;
        }
    }
    // ---- boundary faces (used once), oriented outward
    static const int FACE[4][3] = {{1, 2, 3}, {0, 3, 2}, {0, 1, 3}, {0, 2, 1}};
    struct FaceRec {
        std::array<int32_t, 3> key;
        int32_t src;
        bool operator<(const FaceRec &o) const { return key < o.key; }
    };
    std::vector<FaceRec> faces(4 * (size_t)m);
    for (int e = 0; e < m; ++e)
        for (int f = 0; f < 4; ++f) {
            std::array<int32_t, 3> k = {d.T[4 * e + FACE[f][0]], d.T[4 * e + FACE[f][1]], d.T[4 * e + FACE[f][2]]};
            std::sort(k.begin(), k.end());
            faces[4 * e + f] = {k, 4 * e + f};
        }
    std::sort(faces.begin(), faces.end());
    std::vector<std::array<int32_t, 3>> gtris, itris;
    for (size_t i = 0; i < faces.size();) {
        size_t j = i + 1;
        while (j < faces.size() && faces[j].key == faces[i].key) ++j;
        if (j - i == 1) {
            int e = faces[i].src / 4, f = faces[i].src % 4;
            gtris.push_back({d.T[4 * e + FACE[f][0]], d.T[4 * e + FACE[f][1]], d.T[4 * e + FACE[f][2]]});
        } else if (j - i > 2) {
            set_error("non-manifold tet mesh (a face shared by more than two tets)");
            return IPC_E_BAD_MESH;
        }
        i = j;
    }
    canonical_tris(gtris);
    for (int k = 0; k < d.n_ind_tris; ++k)
        itris.push_back({d.ind_tris[3 * k] + ng, d.ind_tris[3 * k + 1] + ng, d.ind_tris[3 * k + 2] + ng});
    canonical_tris(itris);
    auto gedges = unique_edges(gtris), iedges = unique_edges(itris);
    s.n_gel_tris = (int)gtris.size();
    s.n_tris = (int)(gtris.size() + itris.size());
    s.n_gel_edges = (int)gedges.size();
    s.n_edges = (int)(gedges.size() + iedges.size());
    s.h_tris.resize(3 * (size_t)s.n_tris);
    s.h_edges.resize(2 * (size_t)s.n_edges);
    {
        size_t k = 0;
        for (auto &t : gtris) { s.h_tris[3 * k] = t[0]; s.h_tris[3 * k + 1] = t[1]; s.h_tris[3 * k + 2] = t[2]; ++k; }
        for (auto &t : itris) { s.h_tris[3 * k] = t[0]; s.h_tris[3 * k + 1] = t[1]; s.h_tris[3 * k + 2] = t[2]; ++k; }
        k = 0;
        for (auto &e : gedges) { s.h_edges[2 * k] = e[0]; s.h_edges[2 * k + 1] = e[1]; ++k; }
        for (auto &e : iedges) { s.h_edges[2 * k] = e[0]; s.h_edges[2 * k + 1] = e[1]; ++k; }
    }
    std::vector<uint8_t> on(n, 0);
    for (int32_t v : s.h_tris) on[v] = 1;
    s.h_pts.clear();
    s.h_surf_verts.clear();
    for (int i = 0; i < n; ++i)
        if (on[i]) {
            s.h_pts.push_back(i);
            if (i < ng) s.h_surf_verts.push_back(i);
        }
    s.n_pts = (int)s.h_pts.size();

    // ---- vertex -> tet incidence (tet order)
    std::vector<int32_t> vt_ptr(n + 1, 0), vt_src(4 * (size_t)m);
    for (int64_t k = 0; k < 4 * (int64_t)m; ++k) vt_ptr[d.T[k] + 1]++;
    for (int i = 0; i < n; ++i) vt_ptr[i + 1] += vt_ptr[i];
    {
        std::vector<int32_t> cur(vt_ptr.begin(), vt_ptr.end() - 1);
        for (int e = 0; e < m; ++e)
            for (int a = 0; a < 4; ++a) vt_src[cur[d.T[4 * e + a]]++] = e * 4 + a;
    }
    // ---- BELL pattern: row = diagonal first, then sorted neighbours
    std::vector<std::vector<int32_t>> nbr(n);
    for (int e = 0; e < m; ++e)
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b)
                if (a != b) nbr[d.T[4 * e + a]].push_back(d.T[4 * e + b]);
    for (auto &l : nbr) {
        std::sort(l.begin(), l.end());
        l.erase(std::unique(l.begin(), l.end()), l.end());
    }
    s.n_slices = (n + kSlice - 1) / kSlice;
    std::vector<int32_t> slice_ptr(s.n_slices + 1, 0);
    for (int sl = 0; sl < s.n_slices; ++sl) {
        int w = 1;
        for (int l = 0; l < kSlice; ++l) {
            int row = sl * kSlice + l;
            if (row < n) w = std::max(w, 1 + (int)nbr[row].size());
        }
        slice_ptr[sl + 1] = slice_ptr[sl] + w;
    }
    s.n_slots = slice_ptr[s.n_slices];
    s.nnzb = 0;
    for (int row = 0; row < n; ++row) s.nnzb += 1 + (int64_t)nbr[row].size();
    size_t nent = (size_t)s.n_slots * kSlice;
    std::vector<int32_t> bcol(nent, -1);
    for (int row = 0; row < n; ++row) {
        int sl = row / kSlice, l = row % kSlice;
        bcol[(size_t)slice_ptr[sl] * kSlice + l] = row;
        for (size_t k = 0; k < nbr[row].size(); ++k) bcol[(size_t)(slice_ptr[sl] + 1 + k) * kSlice + l] = nbr[row][k];
    }
    auto entry_of = [&](int row, int col) -> size_t {
        int sl = row / kSlice, l = row % kSlice;
        int k = 0;
        if (col != row) {
            auto &lst = nbr[row];
            k = 1 + (int)(std::lower_bound(lst.begin(), lst.end(), col) - lst.begin());
        }
        return (size_t)(slice_ptr[sl] + k) * kSlice + l;
    };
    std::vector<int32_t> g_ptr(nent + 1, 0), g_src(16 * (size_t)m);
    for (int e = 0; e < m; ++e)
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) g_ptr[entry_of(d.T[4 * e + a], d.T[4 * e + b]) + 1]++;
    for (size_t i = 0; i < nent; ++i) g_ptr[i + 1] += g_ptr[i];
    {
        std::vector<int32_t> cur(g_ptr.begin(), g_ptr.end() - 1);
        for (int e = 0; e < m; ++e)
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b)
                    g_src[cur[entry_of(d.T[4 * e + a], d.T[4 * e + b])]++] = e * 16 + a * 4 + b;
    }
    s.n_gather = (int64_t)g_src.size();

    // ---- SoA tets, surface arrays
    std::vector<int32_t> tv(4 * (size_t)m);
    for (int e = 0; e < m; ++e)
        for (int a = 0; a < 4; ++a) tv[(size_t)a * m + e] = d.T[4 * e + a];
    std::vector<int32_t> ev(2 * (size_t)s.n_edges), trv(3 * (size_t)s.n_tris);
    for (int k = 0; k < s.n_edges; ++k) {
        ev[k] = s.h_edges[2 * k];
        ev[(size_t)s.n_edges + k] = s.h_edges[2 * k + 1];
    }
    for (int k = 0; k < s.n_tris; ++k)
        for (int c = 0; c < 3; ++c) trv[(size_t)c * s.n_tris + k] = s.h_tris[3 * k + c];
    std::vector<double> ers(s.n_edges);
    for (int k = 0; k < s.n_edges; ++k) {
        const double *a = &X0[3 * (size_t)s.h_edges[2 * k]], *b = &X0[3 * (size_t)s.h_edges[2 * k + 1]];
        double dd[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
        ers[k] = dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2];
    }
    std::vector<uint8_t> fixed(n, 0);
    if (d.fixed)
        for (int i = 0; i < ng; ++i) fixed[i] = d.fixed[i] ? 1 : 0;
    s.h_Yloc.assign(d.ind_Y, d.ind_Y + 3 * (size_t)ni);
    std::memcpy(s.pose0.m, d.ind_pose0, sizeof(double) * 12);

    // ---- device buffers
    size_t n3 = 3 * (size_t)n;
    s.X0 = upload(s, X0);
    s.x = dalloc<double>(s, n3);
    IPC_HIP(hipMemcpyAsync(s.x, s.X0, sizeof(double) * n3, hipMemcpyDeviceToDevice, s.stream));
    s.v = dalloc<double>(s, n3);
    IPC_HIP(hipMemsetAsync(s.v, 0, sizeof(double) * n3, s.stream));
    s.xt = dalloc<double>(s, n3);
    s.xtilde = dalloc<double>(s, n3);
    s.yhat = dalloc<double>(s, n3);
    s.xtrial = dalloc<double>(s, n3);
    IPC_HIP(hipMemcpyAsync(s.xt, s.X0, sizeof(double) * n3, hipMemcpyDeviceToDevice, s.stream));
    IPC_HIP(hipMemcpyAsync(s.xtilde, s.X0, sizeof(double) * n3, hipMemcpyDeviceToDevice, s.stream));
    IPC_HIP(hipMemcpyAsync(s.yhat, s.X0, sizeof(double) * n3, hipMemcpyDeviceToDevice, s.stream));
    s.Yloc = upload(s, s.h_Yloc);
    s.fixed = upload(s, fixed);
    s.mass = dalloc<double>(s, n);
    s.tv = upload(s, tv);
    s.Bm = dalloc<double>(s, 9 * (size_t)m);
    s.vol = dalloc<double>(s, m);
    s.eg = dalloc<double>(s, 12 * (size_t)m);
    s.eH = dalloc<double>(s, 90 * (size_t)m);
    s.vt_ptr = upload(s, vt_ptr);
    s.vt_src = upload(s, vt_src);
    s.slice_ptr = upload(s, slice_ptr);
    s.bcol = upload(s, bcol);
    s.bval = dalloc<double>(s, nent * 9);
    s.g_ptr = upload(s, g_ptr);
    s.g_src = upload(s, g_src);
    s.grad = dalloc<double>(s, n3);
    s.Minv = dalloc<double>(s, 9 * (size_t)n);
    s.pts = upload(s, s.h_pts);
    s.ev = upload(s, ev);
    s.trv = upload(s, trv);
    s.edge_rest_sq = upload(s, ers);
    s.pbox = dalloc<double>(s, 6 * (size_t)std::max(s.n_pts, 1));
    s.ebox = dalloc<double>(s, 6 * (size_t)std::max(s.n_edges, 1));
    s.tbox = dalloc<double>(s, 6 * (size_t)std::max(s.n_tris, 1));
    s.cell_h = dalloc<double>(s, 1);
    int64_t red = 4 * (int64_t)nblocks(std::max({(int64_t)n, (int64_t)s.n_pts, (int64_t)s.n_edges, (int64_t)s.n_tris})) + 64;
    s.red_scratch = dalloc<double>(s, red);
    s.c_ptr = dalloc<int32_t>(s, n + 1);
    s.c_cnt = dalloc<int32_t>(s, n + 1);
    IPC_HIP(hipMemsetAsync(s.c_ptr, 0, sizeof(int32_t) * (n + 1), s.stream));
    s.r = dalloc<double>(s, n3);
    s.z = dalloc<double>(s, n3);
    s.dA = dalloc<double>(s, n3);
    s.dB = dalloc<double>(s, n3);
    s.q = dalloc<double>(s, n3);
    s.sol = dalloc<double>(s, n3);
    s.pcg_part = dalloc<double>(s, (size_t)s.n_slices + 2 * (size_t)nblocks(n) + 8);
    s.pcg_state = dalloc<int32_t>(s, 16);
    IPC_HIP(hipMemsetAsync(s.pcg_state, 0, sizeof(int32_t) * 16, s.stream));
    s.surf_verts = upload(s, s.h_surf_verts);
    s.xw = dalloc<double>(s, n3);
    s.pw = dalloc<double>(s, n3);
    s.yw = dalloc<double>(s, n3);
    s.mean_part = dalloc<double>(s, 3 * (size_t)nblocks(n) + 8);
    // candidates and active pairs start small and grow
    s.cand_cap = 0;
    s.sw_cap = 0;
    s.act_cap = 0;
    IPC_HIP(hipHostMalloc((void **)&s.hb, sizeof(Readback), 0));
    std::memset(s.hb, 0, sizeof(Readback));
    launch_rest_precompute(s);
    IPC_HIP(hipStreamSynchronize(s.stream));
    IPC_HIP(hipGetLastError());
    return IPC_OK;
}

void ensure_cand_aux(Scene &s)
{
    if (s.aux_cap < s.cand_cap) {
        if (s.cand_d) dfree(s, s.cand_d);
        if (s.act_flag) dfree(s, s.act_flag);
        s.cand_d = dalloc<double>(s, s.cand_cap);
        s.act_flag = dalloc<int32_t>(s, s.cand_cap + 1);
        s.aux_cap = s.cand_cap;
    }
    int64_t need = partial_need(s, std::max(s.sw_cap, s.cand_cap));
    if (s.part_cap < need) {
        if (s.accd_t) dfree(s, s.accd_t);
        s.accd_t = dalloc<double>(s, need);
        s.part_cap = need;
    }
}

// ---------------------------------------------------------------------------
// Newton
// ---------------------------------------------------------------------------

using Clock = std::chrono::steady_clock;
static double ms_since(Clock::time_point t0)
{
    return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
}

struct IterOut {
    int result = 0;  // 0 stepped, 1 converged, 2 stall
    int pcg_iters = 0;
    int pcg_cap = 0;
    int halvings = 0;
    double alpha_ccd = 1.0, alpha = 0.0, energy = NAN, pinf = 0.0;
};

// Assemble g and H at x (device pointer): static candidates, active pairs,
// barrier, incidence, elastic elements, gather.
static void assemble_at(Scene &s, const double *x, double *ms)
{
    auto t0 = Clock::now();
    hipEvent_t ev[2];
    prof_begin(s, kProfBroad, ev);
    s.n_cand = run_broad_phase(s, x, nullptr, &s.cand, &s.cand_cap);
    prof_end(s, kProfBroad, ev);
    ensure_cand_aux(s);
    prof_begin(s, kProfBarrier, ev);
    run_narrow_phase(s, x);
    launch_barrier(s, x);
    launch_contact_incidence(s);
    prof_end(s, kProfBarrier, ev);
    if (ms) ms[1] += ms_since(t0);
    t0 = Clock::now();
    prof_begin(s, kProfElastic, ev);
    launch_elastic_elements(s, x);
    prof_end(s, kProfElastic, ev);
    prof_begin(s, kProfAssemble, ev);
    launch_assemble(s, x);
    prof_end(s, kProfAssemble, ev);
    if (ms) {
        IPC_HIP(hipStreamSynchronize(s.stream));
        ms[0] += ms_since(t0);
    }
}

static IterOut newton_iterate(Scene &s, double *x, double *ms)
{
    IterOut o;
    assemble_at(s, x, ms);
    auto t0 = Clock::now();
    o.pcg_iters = run_pcg(s, &o.pcg_cap);
    o.pinf = run_pinf(s);
    if (ms) ms[2] += ms_since(t0);
    if (o.pinf <= s.prm.newton_tol) {
        o.result = 1;
        return o;
    }
    t0 = Clock::now();
    hipEvent_t ev[2];
    prof_begin(s, kProfBroad, ev);
    s.n_cand_sw = run_broad_phase(s, x, s.sol, &s.cand_sw, &s.sw_cap);
    prof_end(s, kProfBroad, ev);
    ensure_cand_aux(s);
    prof_begin(s, kProfCcd, ev);
    o.alpha_ccd = run_ccd(s, x, s.sol);
    prof_end(s, kProfCcd, ev);
    if (ms) ms[3] += ms_since(t0);
    t0 = Clock::now();
    double alpha = std::min(1.0, o.alpha_ccd), alpha0 = alpha;
    int inf = 0;
    prof_begin(s, kProfEnergy, ev);
    double E0 = run_energy(s, x, s.cand_sw, s.n_cand_sw, &inf);
    prof_end(s, kProfEnergy, ev);
    for (;;) {
        launch_trial(s, x, s.sol, alpha, s.xtrial);
        prof_begin(s, kProfEnergy, ev);
        double E = run_energy(s, s.xtrial, s.cand_sw, s.n_cand_sw, &inf);
        prof_end(s, kProfEnergy, ev);
        if (E <= E0) {
            IPC_HIP(hipMemcpyAsync(x, s.xtrial, sizeof(double) * 3 * s.n, hipMemcpyDeviceToDevice, s.stream));
            o.energy = E;
            o.alpha = alpha;
            break;
        }
        alpha *= 0.5;
        o.halvings++;
        if (alpha < s.prm.ls_min_ratio * alpha0) {
            o.result = 2;
            o.energy = E0;
            o.alpha = 0.0;
            break;
        }
    }
    if (ms) ms[4] += ms_since(t0);
    return o;
}

static int32_t step_scene(Scene &s, const ipc_step_req &req, ipc_step_stats *st)
{
    auto t_start = Clock::now();
    ipc_step_stats local;
    if (!st) st = &local;
    std::memset(st, 0, sizeof(*st));
    st->energy = NAN;
    Pose P;
    std::memcpy(P.m, req.pose, sizeof(P.m));
    launch_begin_step(s, P);
    int status = IPC_OK;
    int k;
    bool pcg_warn = false;
    for (k = 0; k < s.prm.max_newton; ++k) {
        IterOut o = newton_iterate(s, s.x, st->ms_phase);
        st->newton_iters++;
        st->pcg_iters += o.pcg_iters;
        st->ls_halvings += o.halvings;
        st->pinf = o.pinf;
        pcg_warn |= o.pcg_cap != 0;
        if (o.result == 1) break;
        st->alpha_ccd = o.alpha_ccd;
        st->alpha = o.alpha;
        st->energy = o.energy;
        if (o.result == 2) {
            status = IPC_W_LS_STALL;
            break;
        }
    }
    if (k == s.prm.max_newton) status = IPC_W_NEWTON_MAXITER;
    if (status == IPC_OK && pcg_warn) status = IPC_W_PCG_MAXITER;
    st->n_candidates = (int32_t)s.n_cand;
    st->n_active = (int32_t)s.n_act;
    launch_end_step(s);
    st->max_target_lag = run_target_lag(s);
    if (status == IPC_OK && st->max_target_lag > 1e-3 * s.prm.dhat) status = IPC_W_TARGET_LAG;
    IPC_HIP(hipStreamSynchronize(s.stream));
    prof_collect(s);
    st->status = status;
    st->ms_total = ms_since(t_start);
    s.step_index++;
    return status;
}

// ---------------------------------------------------------------------------
// C ABI helpers
// ---------------------------------------------------------------------------

template <class F>
static int32_t guarded(F &&f)
{
    try {
        return f();
    } catch (const HipError &e) {
        set_error(std::string("HIP error in ") + e.what + ": " + hipGetErrorString(e.e));
        return IPC_E_DEVICE;
    } catch (const OomError &) {
        set_error("device allocation refused (allocator or memory budget)");
        return IPC_E_OOM;
    } catch (const CapacityError &) {
        set_error("contact list capacity exceeded");
        return IPC_E_CAPACITY;
    } catch (const InfeasibleError &) {
        set_error("non-finite or absurd positions in the contact broad phase");
        return IPC_E_INFEASIBLE;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return IPC_E_OOM;
    } catch (...) {
        set_error("unexpected error");
        return IPC_E_INVALID_ARG;
    }
}

static bool check_desc(const ipc_scene_desc *d)
{
    if (!d || d->n_verts <= 0 || d->n_tets <= 0 || !d->X || !d->T) return false;
    if (d->n_ind_verts < 0 || d->n_ind_tris < 0) return false;
    if (d->n_ind_verts > 0 && (!d->ind_Y || (d->n_ind_tris > 0 && !d->ind_tris))) return false;
    if (!(d->dt > 0) || !(d->dhat > 0) || !(d->kappa > 0) || !(d->E > 0) || !(d->rho > 0)) return false;
    if (!(d->nu > -1.0 && d->nu < 0.5)) return false;
    if (d->precision != IPC_FP64 && d->precision != IPC_MIXED) return false;
    return true;
}

static Params make_params(const ipc_scene_desc &d)
{
    Params p{};
    p.E = d.E;
    p.nu = d.nu;
    p.rho = d.rho;
    p.mu = d.E / (2.0 * (1.0 + d.nu));
    p.lam = d.E * d.nu / ((1.0 + d.nu) * (1.0 - 2.0 * d.nu));
    p.dt = d.dt;
    p.dhat = d.dhat;
    p.kappa = d.kappa;
    p.k_target = d.k_target;
    p.newton_tol = d.newton_tol;
    p.pcg_tol = d.pcg_tol;
    for (int i = 0; i < 3; ++i) p.grav[i] = d.gravity[i];
    p.mu_fric = d.mu_friction;
    p.eps_v = d.eps_v;
    p.ccd_s = d.ccd_s > 0 ? d.ccd_s : 0.1;
    p.ls_min_ratio = d.ls_min_ratio > 0 ? d.ls_min_ratio : std::ldexp(1.0, -30);
    p.self_contact = d.self_contact;
    p.precision = d.precision;
    p.max_newton = d.max_newton > 0 ? d.max_newton : 100;
    p.pcg_max_iter = d.pcg_max_iter;
    p.ccd_max_iter = d.ccd_max_iter > 0 ? d.ccd_max_iter : 10000;
    return p;
}

}  // namespace ipcg

using namespace ipcg;

struct ipc_scene : public ipcg::Scene {
};

struct BatchItem {
    ipc_step_stats st;
    int32_t status;
};
struct ipc_batch {
    ipc_runtime rt{};
    std::mutex mu;
    std::unordered_map<ipc_ticket, BatchItem> done;
    ipc_ticket next = 1;
};

extern "C" {

int32_t ipc_create_scene(const ipc_scene_desc *d, const ipc_runtime *rt, ipc_scene **out)
{
    if (!out) return IPC_E_INVALID_ARG;
    *out = nullptr;
    if (!check_desc(d)) {
        set_error("invalid scene description");
        return IPC_E_INVALID_ARG;
    }
    ipc_scene *s = nullptr;
    int32_t st = guarded([&]() -> int32_t {
        s = new ipc_scene();
        if (rt) s->arena.rt = *rt;
        s->stream = rt ? (hipStream_t)rt->stream : nullptr;
        s->prm = make_params(*d);
        int32_t r = build_scene(*s, *d);
        return r;
    });
    if (st != IPC_OK) {
        delete s;
        return st;
    }
    *out = s;
    return IPC_OK;
}

void ipc_destroy_scene(ipc_scene *s) { delete s; }

int64_t ipc_scene_footprint_bytes(const ipc_scene_desc *d)
{
    if (!check_desc(d)) return -1;
    int64_t n = (int64_t)d->n_verts + d->n_ind_verts, m = d->n_tets;
    int64_t per_vertex = 8 * (3 * 14 + 9 + 1) + 4 * 4 + 1;
    int64_t per_tet = 4 * 4 + 8 * (9 + 1 + 12 + 90) + 4 * 16 + 4 * 4;
    int64_t bell = n * 16 * (72 + 4 + 4);
    int64_t surf = 4 * (int64_t)std::pow((double)d->n_verts, 2.0 / 3.0) + d->n_ind_verts + 2 * d->n_ind_tris;
    int64_t contact = surf * (6 * 8 * 3 + 64 * 4 * 3 + 8 * 16);
    return n * per_vertex + m * per_tet + bell + contact + (8 << 20);
}

int32_t ipc_step(ipc_scene *s, const ipc_step_req *r, ipc_step_stats *st)
{
    if (!s || !r) return IPC_E_INVALID_ARG;
    if (s->busy) return IPC_E_BUSY;
    s->busy = true;
    int32_t rc = guarded([&]() -> int32_t { return step_scene(*s, *r, st); });
    s->busy = false;
    return rc;
}

int32_t ipc_read_surface(const ipc_scene *cs, double *xyz, int64_t cap, int32_t where, void *stream,
                         double obj_pos[3])
{
    if (!cs) return IPC_E_INVALID_ARG;
    ipc_scene *s = const_cast<ipc_scene *>(cs);
    int64_t need = 3 * (int64_t)s->h_surf_verts.size();
    if (xyz && cap < need) {
        set_error("surface buffer too small");
        return IPC_E_INVALID_ARG;
    }
    if (where != IPC_HOST && where != IPC_DEVICE) return IPC_E_INVALID_ARG;
    return guarded([&]() -> int32_t {
        hipStream_t strm = stream ? (hipStream_t)stream : s->stream;
        IPC_HIP(hipStreamSynchronize(s->stream));
        if (xyz) {
            double *dst = where == IPC_DEVICE ? xyz : s->yw;
            launch_gather_surface(*s, dst, strm);
            if (where == IPC_HOST)
                IPC_HIP(hipMemcpyAsync(xyz, s->yw, sizeof(double) * need, hipMemcpyDeviceToHost, strm));
        }
        if (obj_pos) {
            double *dm = run_gel_mean(*s, strm);
            IPC_HIP(hipMemcpyAsync(obj_pos, dm, sizeof(double) * 3, hipMemcpyDeviceToHost, strm));
        }
        IPC_HIP(hipStreamSynchronize(strm));
        return IPC_OK;
    });
}

int32_t ipc_surface_topology(const ipc_scene *s, int32_t *tris, int64_t tri_cap, int32_t *n_tris, int32_t *verts,
                             int64_t vert_cap, int32_t *n_surf_verts)
{
    if (!s) return IPC_E_INVALID_ARG;
    if (n_tris) *n_tris = s->n_gel_tris;
    if (n_surf_verts) *n_surf_verts = (int32_t)s->h_surf_verts.size();
    if (tris) {
        if (tri_cap < 3 * (int64_t)s->n_gel_tris) return IPC_E_INVALID_ARG;
        std::memcpy(tris, s->h_tris.data(), sizeof(int32_t) * 3 * s->n_gel_tris);
    }
    if (verts) {
        if (vert_cap < (int64_t)s->h_surf_verts.size()) return IPC_E_INVALID_ARG;
        std::memcpy(verts, s->h_surf_verts.data(), sizeof(int32_t) * s->h_surf_verts.size());
    }
    return IPC_OK;
}

int32_t ipc_reset(ipc_scene *s)
{
    if (!s) return IPC_E_INVALID_ARG;
    if (s->busy) return IPC_E_BUSY;
    return guarded([&]() -> int32_t {
        size_t b = sizeof(double) * 3 * s->n;
        IPC_HIP(hipMemcpyAsync(s->x, s->X0, b, hipMemcpyDeviceToDevice, s->stream));
        IPC_HIP(hipMemsetAsync(s->v, 0, b, s->stream));
        IPC_HIP(hipMemcpyAsync(s->xt, s->X0, b, hipMemcpyDeviceToDevice, s->stream));
        IPC_HIP(hipMemcpyAsync(s->xtilde, s->X0, b, hipMemcpyDeviceToDevice, s->stream));
        IPC_HIP(hipMemcpyAsync(s->yhat, s->X0, b, hipMemcpyDeviceToDevice, s->stream));
        IPC_HIP(hipStreamSynchronize(s->stream));
        s->step_index = 0;
        return IPC_OK;
    });
}

static const uint64_t kStateMagic = 0x31657461744370ULL;

int64_t ipc_state_bytes(const ipc_scene *s)
{
    if (!s) return -1;
    return 32 + 2 * 3 * (int64_t)s->n * 8;
}

int32_t ipc_save_state(const ipc_scene *cs, void *blob, int64_t cap)
{
    if (!cs || !blob || cap < ipc_state_bytes(cs)) return IPC_E_INVALID_ARG;
    ipc_scene *s = const_cast<ipc_scene *>(cs);
    return guarded([&]() -> int32_t {
        uint64_t hdr[4] = {kStateMagic, (uint64_t)s->n, (uint64_t)s->step_index, 0};
        std::memcpy(blob, hdr, sizeof hdr);
        char *p = (char *)blob + 32;
        size_t b = sizeof(double) * 3 * s->n;
        IPC_HIP(hipMemcpyAsync(p, s->x, b, hipMemcpyDeviceToHost, s->stream));
        IPC_HIP(hipMemcpyAsync(p + b, s->v, b, hipMemcpyDeviceToHost, s->stream));
        IPC_HIP(hipStreamSynchronize(s->stream));
        return IPC_OK;
    });
}

int32_t ipc_load_state(ipc_scene *s, const void *blob, int64_t bytes)
{
    if (!s || !blob || bytes < ipc_state_bytes(s)) return IPC_E_INVALID_ARG;
    uint64_t hdr[4];
    std::memcpy(hdr, blob, sizeof hdr);
    if (hdr[0] != kStateMagic || hdr[1] != (uint64_t)s->n) {
        set_error("state blob does not match this scene");
        return IPC_E_INVALID_ARG;
    }
    return guarded([&]() -> int32_t {
        const char *p = (const char *)blob + 32;
        size_t b = sizeof(double) * 3 * s->n;
        IPC_HIP(hipMemcpyAsync(s->x, p, b, hipMemcpyHostToDevice, s->stream));
        IPC_HIP(hipMemcpyAsync(s->v, p + b, b, hipMemcpyHostToDevice, s->stream));
        IPC_HIP(hipStreamSynchronize(s->stream));
        s->step_index = (int)hdr[2];
        return IPC_OK;
    });
}

int32_t ipc_scene_sizes(const ipc_scene *s, int32_t *o)
{
    if (!s || !o) return IPC_E_INVALID_ARG;
    o[0] = s->n; o[1] = s->n_gel; o[2] = s->m; o[3] = s->n_pts;
    o[4] = s->n_edges; o[5] = s->n_tris; o[6] = s->n_ind; o[7] = s->n_gel_tris;
    return IPC_OK;
}

int32_t ipc_batch_create(const ipc_runtime *rt, ipc_batch **out)
{
    if (!out) return IPC_E_INVALID_ARG;
    *out = new (std::nothrow) ipc_batch();
    if (!*out) return IPC_E_OOM;
    if (rt) (*out)->rt = *rt;
    return IPC_OK;
}

void ipc_batch_destroy(ipc_batch *b) { delete b; }

int32_t ipc_batch_submit(ipc_batch *b, int32_t n, ipc_scene *const *s, const ipc_step_req *r, ipc_ticket *t)
{
    if (!b || n < 0 || (n > 0 && (!s || !r || !t))) return IPC_E_INVALID_ARG;
    for (int i = 0; i < n; ++i) {
        if (!s[i]) return IPC_E_INVALID_ARG;
        if (s[i]->busy) return IPC_E_BUSY;
        for (int j = 0; j < i; ++j)
            if (s[j] == s[i]) return IPC_E_BUSY;
    }
    for (int i = 0; i < n; ++i) {
        BatchItem it;
        std::memset(&it, 0, sizeof it);
        it.status = ipc_step(s[i], &r[i], &it.st);
        std::lock_guard<std::mutex> g(b->mu);
        t[i] = b->next++;
        b->done[t[i]] = it;
    }
    return IPC_OK;
}

int32_t ipc_batch_poll(ipc_batch *b, ipc_ticket t, ipc_step_stats *st)
{
    if (!b) return IPC_E_INVALID_ARG;
    std::lock_guard<std::mutex> g(b->mu);
    auto it = b->done.find(t);
    if (it == b->done.end()) return IPC_E_INVALID_ARG;
    if (st) *st = it->second.st;
    return 1;
}

int32_t ipc_batch_wait(ipc_batch *b, ipc_ticket t, ipc_step_stats *st)
{
    if (!b) return IPC_E_INVALID_ARG;
    std::lock_guard<std::mutex> g(b->mu);
    auto it = b->done.find(t);
    if (it == b->done.end()) return IPC_E_INVALID_ARG;
    if (st) *st = it->second.st;
    int32_t rc = it->second.status;
    b->done.erase(it);
    return rc;
}

const char *ipc_status_str(int32_t s)
{
    switch (s) {
    case IPC_OK: return "ok";
    case IPC_W_NEWTON_MAXITER: return "warning: Newton iteration cap reached";
    case IPC_W_PCG_MAXITER: return "warning: PCG iteration cap reached";
    case IPC_W_LS_STALL: return "warning: line search stalled";
    case IPC_W_TARGET_LAG: return "warning: indenter lags its target";
    case IPC_E_INVALID_ARG: return "error: invalid argument";
    case IPC_E_BAD_MESH: return "error: bad mesh";
    case IPC_E_INFEASIBLE: return "error: infeasible state";
    case IPC_E_OOM: return "error: out of memory";
    case IPC_E_DEVICE: return "error: HIP device error";
    case IPC_E_BUSY: return "error: scene busy";
    case IPC_E_CAPACITY: return "error: contact capacity";
    default: return "unknown status";
    }
}

int32_t ipc_last_error(char *buf, size_t cap)
{
    const std::string &e = ipcg::g_last_error;
    if (buf && cap > 0) {
        size_t k = std::min(cap - 1, e.size());
        std::memcpy(buf, e.data(), k);
        buf[k] = 0;
    }
    return (int32_t)e.size();
}

// ---- test-only ---------------------------------------------------------------

static void upload_vec(ipc_scene *s, double *dst, const double *src)
{
    IPC_HIP(hipMemcpyAsync(dst, src, sizeof(double) * 3 * s->n, hipMemcpyHostToDevice, s->stream));
}
static void download_vec(ipc_scene *s, double *dst, const double *src)
{
    IPC_HIP(hipMemcpyAsync(dst, src, sizeof(double) * 3 * s->n, hipMemcpyDeviceToHost, s->stream));
    IPC_HIP(hipStreamSynchronize(s->stream));
}

int32_t ipcx_begin_step(ipc_scene *s, const ipc_step_req *r)
{
    if (!s || !r) return IPC_E_INVALID_ARG;
    return guarded([&]() -> int32_t {
        Pose P;
        std::memcpy(P.m, r->pose, sizeof(P.m));
        launch_begin_step(*s, P);
        IPC_HIP(hipStreamSynchronize(s->stream));
        return IPC_OK;
    });
}

int32_t ipcx_newton_iterate(ipc_scene *s, const double *x_in, double *x_out, ipc_step_stats *st)
{
    if (!s || !x_in || !x_out) return IPC_E_INVALID_ARG;
    return guarded([&]() -> int32_t {
        upload_vec(s, s->xw, x_in);
        IterOut o = newton_iterate(*s, s->xw, nullptr);
        download_vec(s, x_out, s->xw);
        if (st) {
            std::memset(st, 0, sizeof(*st));
            st->newton_iters = 1;
            st->pcg_iters = o.pcg_iters;
            st->ls_halvings = o.halvings;
            st->n_candidates = (int32_t)s->n_cand;
            st->n_active = (int32_t)s->n_act;
            st->alpha_ccd = o.alpha_ccd;
            st->alpha = o.alpha;
            st->energy = o.energy;
            st->pinf = o.pinf;
            st->status = o.result;
        }
        return o.result;
    });
}

int32_t ipcx_candidates(ipc_scene *s, const double *x, const double *p, int32_t *out, int64_t cap, int64_t *count)
{
    if (!s || !x) return IPC_E_INVALID_ARG;
    return guarded([&]() -> int32_t {
        upload_vec(s, s->xw, x);
        if (p) upload_vec(s, s->pw, p);
        int32_t **buf = p ? &s->cand_sw : &s->cand;
        int64_t *bcap = p ? &s->sw_cap : &s->cand_cap;
        int64_t nc = run_broad_phase(*s, s->xw, p ? s->pw : nullptr, buf, bcap);
        if (p)
            s->n_cand_sw = nc;
        else
            s->n_cand = nc;
        ensure_cand_aux(*s);
        if (count) *count = nc;
        if (out && cap > 0) {
            int64_t w = std::min(cap, nc);
            std::vector<int32_t> h(3 * (size_t)std::max<int64_t>(w, 1));
            for (int c = 0; c < 3; ++c)
                IPC_HIP(hipMemcpyAsync(h.data() + (size_t)c * w, *buf + (size_t)c * *bcap, sizeof(int32_t) * w,
                                       hipMemcpyDeviceToHost, s->stream));
            IPC_HIP(hipStreamSynchronize(s->stream));
            for (int64_t i = 0; i < w; ++i)
                for (int c = 0; c < 3; ++c) out[3 * i + c] = h[(size_t)c * w + i];
        }
        IPC_HIP(hipStreamSynchronize(s->stream));
        return IPC_OK;
    });
}

int32_t ipcx_primitives(const ipc_scene *s, int32_t *points, int32_t *edges, int32_t *tris)
{
    if (!s) return IPC_E_INVALID_ARG;
    if (points) std::memcpy(points, s->h_pts.data(), sizeof(int32_t) * s->h_pts.size());
    if (edges) std::memcpy(edges, s->h_edges.data(), sizeof(int32_t) * s->h_edges.size());
    if (tris) std::memcpy(tris, s->h_tris.data(), sizeof(int32_t) * s->h_tris.size());
    return IPC_OK;
}

int32_t ipcx_gradient(ipc_scene *s, const double *x, double *g)
{
    if (!s || !x || !g) return IPC_E_INVALID_ARG;
    return guarded([&]() -> int32_t {
        upload_vec(s, s->xw, x);
        assemble_at(*s, s->xw, nullptr);
        download_vec(s, g, s->grad);
        return IPC_OK;
    });
}

int32_t ipcx_hess_apply(ipc_scene *s, const double *x, const double *v, double *y)
{
    if (!s || !x || !v || !y) return IPC_E_INVALID_ARG;
    return guarded([&]() -> int32_t {
        upload_vec(s, s->xw, x);
        assemble_at(*s, s->xw, nullptr);
        upload_vec(s, s->pw, v);
        launch_hess_apply(*s, s->pw, s->yw);
        download_vec(s, y, s->yw);
        return IPC_OK;
    });
}

int32_t ipcx_pcg(ipc_scene *s, const double *x, double *p, int32_t *iters)
{
    if (!s || !x || !p) return IPC_E_INVALID_ARG;
    return guarded([&]() -> int32_t {
        upload_vec(s, s->xw, x);
        assemble_at(*s, s->xw, nullptr);
        int cap = 0;
        int it = run_pcg(*s, &cap);
        if (iters) *iters = cap ? -it : it;
        download_vec(s, p, s->sol);
        return IPC_OK;
    });
}

int32_t ipcx_energy(ipc_scene *s, const double *x, double *E)
{
    if (!s || !x || !E) return IPC_E_INVALID_ARG;
    return guarded([&]() -> int32_t {
        upload_vec(s, s->xw, x);
        s->n_cand = run_broad_phase(*s, s->xw, nullptr, &s->cand, &s->cand_cap);
        ensure_cand_aux(*s);
        int inf = 0;
        *E = run_energy(*s, s->xw, s->cand, s->n_cand, &inf);
        return IPC_OK;
    });
}

int32_t ipcx_ccd(ipc_scene *s, const double *x, const double *p, double *alpha)
{
    if (!s || !x || !p || !alpha) return IPC_E_INVALID_ARG;
    return guarded([&]() -> int32_t {
        upload_vec(s, s->xw, x);
        upload_vec(s, s->pw, p);
        s->n_cand_sw = run_broad_phase(*s, s->xw, s->pw, &s->cand_sw, &s->sw_cap);
        ensure_cand_aux(*s);
        *alpha = std::min(1.0, run_ccd(*s, s->xw, s->pw));
        return IPC_OK;
    });
}

int32_t ipcx_profile(ipc_scene *s, int32_t enable)
{
    if (!s) return IPC_E_INVALID_ARG;
    return guarded([&]() -> int32_t {
        IPC_HIP(hipStreamSynchronize(s->stream));
        prof_collect(*s);
        s->prof = enable != 0;
        for (auto &a : s->prof_acc) a = Scene::ProfAcc{};
        return IPC_OK;
    });
}

int32_t ipcx_profile_read(const ipc_scene *s, int32_t kernel, int64_t *launches, double *ms_total)
{
    if (!s || kernel < 0 || kernel >= kProfKernels) return IPC_E_INVALID_ARG;
    if (launches) *launches = s->prof_acc[kernel].launches;
    if (ms_total) *ms_total = s->prof_acc[kernel].ms;
    return IPC_OK;
}

int32_t ipcx_matrix_info(const ipc_scene *s, int64_t *out)
{
    if (!s || !out) return IPC_E_INVALID_ARG;
    out[0] = s->nnzb;
    out[1] = (int64_t)s->n_slots * kSlice;
    out[2] = s->n;
    out[3] = s->n_act;
    out[4] = s->m;
    out[5] = s->n_cand;
    out[6] = s->n_cand_sw;
    out[7] = s->n_gather;
    return IPC_OK;
}

int32_t ipcx_set_state(ipc_scene *s, const double *x, const double *v)
{
    if (!s) return IPC_E_INVALID_ARG;
    return guarded([&]() -> int32_t {
        if (x) upload_vec(s, s->x, x);
        if (v) upload_vec(s, s->v, v);
        IPC_HIP(hipStreamSynchronize(s->stream));
        return IPC_OK;
    });
}

int32_t ipcx_get_state(const ipc_scene *cs, double *x, double *v)
{
    if (!cs) return IPC_E_INVALID_ARG;
    ipc_scene *s = const_cast<ipc_scene *>(cs);
    return guarded([&]() -> int32_t {
        if (x) download_vec(s, x, s->x);
        if (v) download_vec(s, v, s->v);
        return IPC_OK;
    });
}

}  // extern "C"
