// scene.hip -- scene construction, the Newton driver over a list of scenes,
// the continuous-batching engine and the C ABI.
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
// A Newton *round* runs one iteration for every scene of a list that is still
// iterating, one launch per phase for all of them; each scene keeps its own
// iteration count, step length and stop decisions. ipc_step is a round loop
// over a list of one scene. The batch engine keeps a list of scenes in flight
// and admits newly submitted requests at every round boundary (continuous
// batching): work of new scenes overlaps with scenes in mid-step.
#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>

#include <dlfcn.h>
#include <sys/stat.h>

#include <cstdio>
#include <cstdlib>
#include <map>

#include "ipc_internal.h"

namespace ipcg {

// ---------------------------------------------------------------------------
// Tuning file: {"classes": [{"min_verts": 0, "spmv_one_lane_rows": ..., "mas_target": ...,
// "pcg_first_chunk": ..., "pcg_later_chunk": ...}, ...], ...}, written by the
// autotuner; $IPC_TUNING_FILE names it (empty: none), else tuning.json beside
// the library. A scene takes the class with the largest min_verts <= its
// vertex count. Unknown keys are ignored; a missing or unreadable file means
// the built-in defaults.
// ---------------------------------------------------------------------------

namespace {
struct TuneClass {
    int64_t min_verts = 0;
    Tuning t;
};

std::string tuning_path()
{
    const char *e = std::getenv("IPC_TUNING_FILE");
    if (e) return e;
    Dl_info info;
    if (dladdr(reinterpret_cast<void *>(&tuning_for), &info) && info.dli_fname) {
        std::string p = info.dli_fname;
        size_t k = p.rfind('/');
        return (k == std::string::npos ? std::string(".") : p.substr(0, k)) + "/tuning.json";
    }
    return "";
}

// the objects of the "classes" array, each a flat list of "key": number
std::vector<TuneClass> parse_tuning(const std::string &text)
{
    std::vector<TuneClass> out;
    size_t k = text.find("\"classes\"");
    if (k == std::string::npos) return out;
    k = text.find('[', k);
    if (k == std::string::npos) return out;
    size_t i = k + 1;
    while (i < text.size()) {
        while (i < text.size() && (isspace((unsigned char)text[i]) || text[i] == ',')) ++i;
        if (i >= text.size() || text[i] == ']') break;
        if (text[i] != '{') return {};
        size_t e = text.find('}', i);
        if (e == std::string::npos) return {};
        TuneClass c;
        std::string body = text.substr(i + 1, e - i - 1);
        size_t q = 0;
        while ((q = body.find('"', q)) != std::string::npos) {
            size_t q2 = body.find('"', q + 1);
            if (q2 == std::string::npos) break;
            std::string key = body.substr(q + 1, q2 - q - 1);
            size_t colon = body.find(':', q2);
            if (colon == std::string::npos) break;
            char *end = nullptr;
            double v = std::strtod(body.c_str() + colon + 1, &end);
            if (end == body.c_str() + colon + 1) {  // not a number: skip the value (a string or a literal)
                size_t v0 = body.find_first_not_of(" \t\r\n", colon + 1);
                if (v0 != std::string::npos && body[v0] == '"') {
                    size_t v1 = body.find('"', v0 + 1);
                    q = v1 == std::string::npos ? body.size() : v1 + 1;
                } else {
                    size_t v1 = body.find(',', colon + 1);
                    q = v1 == std::string::npos ? body.size() : v1 + 1;
                }
                continue;
            }
            if (key == "min_verts") c.min_verts = (int64_t)v;
            else if (key == "spmv_one_lane_rows") c.t.spmv_one_lane_rows = (int64_t)v;
            else if (key == "mas_target") c.t.mas_target = std::max(1, std::min(kMasCapM, (int)v));
            else if (key == "pcg_first_chunk") c.t.pcg_first_chunk = std::max(0.0, std::min(4.0, v));
            else if (key == "pcg_later_chunk") c.t.pcg_later_chunk = std::max(0.0, std::min(4.0, v));
            else if (key == "pcg_list_quantile") c.t.pcg_list_quantile = std::max(0.0, std::min(1.0, v));
            q = (size_t)(end - body.c_str());
        }
        c.t.from_file = 1;
        out.push_back(c);
        i = e + 1;
    }
    std::sort(out.begin(), out.end(), [](const TuneClass &a, const TuneClass &b) { return a.min_verts < b.min_verts; });
    return out;
}

std::mutex g_tune_mu;
std::map<std::string, std::pair<int64_t, std::vector<TuneClass>>> g_tune_cache;  // path -> (mtime, classes)
}  // namespace

Tuning tuning_for(int n_verts)
{
    std::string path = tuning_path();
    if (path.empty()) return Tuning{};
    struct stat st;
    if (stat(path.c_str(), &st) != 0) return Tuning{};
    int64_t mt = (int64_t)st.st_mtime * 1000000000LL + (int64_t)st.st_mtim.tv_nsec;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(path);
    if (it == g_tune_cache.end() || it->second.first != mt) {
        std::string text;
        if (FILE *f = std::fopen(path.c_str(), "rb")) {
            char buf[4096];
            size_t r;
            while ((r = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, r);
            std::fclose(f);
        }
        g_tune_cache[path] = {mt, parse_tuning(text)};
        it = g_tune_cache.find(path);
    }
    Tuning t{};
    for (const TuneClass &c : it->second.second)
        if (c.min_verts <= n_verts) t = c.t;
    return t;
}

static const double kIdentityPose[12] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0};

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

void *dalloc_bytes(Scene &s, size_t bytes)
{
    if (bytes == 0) bytes = 16;
    bytes = (bytes + 255) & ~size_t(255);
    void *p = s.arena.alloc(bytes);
    if (!p) throw OomError{};
    s.owned.push_back({p, bytes});
    return p;
}

void dfree(Scene &s, void *p)
{
    if (!p) return;
    for (auto it = s.owned.begin(); it != s.owned.end(); ++it)
        if (it->first == p) {
            s.arena.release(p, it->second);
            s.owned.erase(it);
            return;
        }
}

void mark_dirty(Scene &s) { s.dev_dirty = true; }

Scene::~Scene()
{
    if (stream) (void)hipStreamSynchronize(stream);
    (void)hipDeviceSynchronize();
    for (auto &o : owned) arena.release(o.first, o.second);
    owned.clear();
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

static size_t real_size(const Scene &s) { return s.prm.precision == IPC_MIXED ? sizeof(float) : sizeof(double); }

// Allocations that replace existing buffers: all new buffers are obtained
// first, the old ones are released only once every allocation succeeded, so
// a refused allocation leaves the scene as it was.
struct Staged {
    Scene &s;
    std::vector<void *> got;
    explicit Staged(Scene &sc) : s(sc) {}
    ~Staged()
    {
        for (void *p : got) dfree(s, p);
    }
    template <class T>
    T *get(size_t count)
    {
        T *p = dalloc<T>(s, count);
        got.push_back(p);
        return p;
    }
    void *get_bytes(size_t bytes)
    {
        void *p = dalloc_bytes(s, bytes);
        got.push_back(p);
        return p;
    }
    void commit() { got.clear(); }
};

// reduction / scan scratch sized for hash tables of 2^b0 and 2^b1 buckets and
// candidate lists of cc entries (only ever grows)
static void ensure_scratch(Scene &s, int b0, int b1, int64_t cc, int64_t fc)
{
    SceneDev &H = s.h;
    int64_t red = std::max({2 * ((int64_t)nblocks((int64_t)H.m + H.n) + nblocks(cc) + nblocks(fc)) + 16,
                            (int64_t)nblocks(H.n_edges) + nblocks(H.n_tris) + 16, 4 * (int64_t)nblocks(H.n) + 16,
                            (int64_t)nblocks(cc) + 16});
    auto tiles = [](int64_t len) { return (len + kScanTile) / kScanTile + 1; };
    int64_t sc = std::max({tiles((int64_t(1) << b0) + 1), tiles((int64_t(1) << b1) + 1),
                           tiles((int64_t)H.n_pts + H.n_edges), tiles(H.n + 1), tiles(cc + 1)}) + 16;
    bool gr = !H.red || H.red_len < red, gs = !H.scan_tmp || H.scan_len < sc;
    Staged st(s);
    double *nr = gr ? st.get<double>(red) : nullptr;
    int32_t *nsc = gs ? st.get<int32_t>(sc) : nullptr;
    st.commit();
    if (gr) {
        dfree(s, H.red);
        H.red = nr;
        H.red_len = red;
    }
    if (gs) {
        dfree(s, H.scan_tmp);
        H.scan_tmp = nsc;
        H.scan_len = sc;
    }
    if (gr || gs) s.dev_dirty = true;
}

void grow_table(Scene &s, int t, int64_t entries)
{
    SceneDev &H = s.h;
    int bits = 10;  // at least as many buckets as entries: every scan and clear of the buckets
                    // runs once per broad phase, so a sparser table costs more than it saves
    while ((int64_t(1) << bits) < entries && bits < 28) ++bits;
    size_t tsize = size_t(1) << bits;
    Staged st(s);
    int32_t *cnt = st.get<int32_t>(tsize + 1), *start = st.get<int32_t>(tsize + 1);
    int4 *ent = st.get<int4>((size_t)entries);
    ensure_scratch(s, t == 0 ? bits : H.ht_bits[0], t == 1 ? bits : H.ht_bits[1], std::max(H.cand_cap, H.sw_cap),
                   H.fric_cap);
    st.commit();
    dfree(s, H.ht_count[t]);
    dfree(s, H.ht_start[t]);
    dfree(s, H.ht_entries[t]);
    H.ht_bits[t] = bits;
    H.ht_count[t] = cnt;
    H.ht_start[t] = start;
    H.ht_entries[t] = ent;
    H.ht_cap[t] = (int32_t)std::min<int64_t>(entries, INT32_MAX);
    s.dev_dirty = true;
}

void grow_candidates(Scene &s, int which, int64_t need)
{
    SceneDev &H = s.h;
    int32_t *&buf = which ? H.cand_sw : H.cand;
    int64_t &cap = which ? H.sw_cap : H.cand_cap;
    if (buf && need <= cap) return;
    int64_t nc = need + need / 2 + 1024;
    Staged st(s);
    int32_t *nb = st.get<int32_t>(3 * (size_t)nc);
    double *nd = which ? nullptr : st.get<double>(nc);
    int32_t *nf = st.get<int32_t>(nc + 1);
    int32_t *no = st.get<int32_t>(nc + 1);
    ensure_scratch(s, H.ht_bits[0], H.ht_bits[1], std::max({H.cand_cap, H.sw_cap, nc}), H.fric_cap);
    st.commit();
    dfree(s, buf);
    buf = nb;
    cap = nc;
    if (!which) {
        dfree(s, H.cand_d);
        dfree(s, H.act_flag);
        dfree(s, H.act_off);
        H.cand_d = nd;
        H.act_flag = nf;
        H.act_off = no;
    } else {
        dfree(s, H.sw_flag);
        dfree(s, H.sw_off);
        H.sw_flag = nf;
        H.sw_off = no;
    }
    s.dev_dirty = true;
}

void grow_friction(Scene &s, int64_t need)
{
    SceneDev &H = s.h;
    if (H.fric_v && need <= H.fric_cap) return;
    int64_t nc = need + need / 2 + 256;
    Staged st(s);
    int32_t *nv = st.get<int32_t>(4 * (size_t)nc);
    double *ncf = st.get<double>(4 * (size_t)nc), *nn = st.get<double>(3 * (size_t)nc), *nl = st.get<double>(nc);
    ensure_scratch(s, H.ht_bits[0], H.ht_bits[1], std::max(H.cand_cap, H.sw_cap), nc);
    st.commit();
    for (void *old : {(void *)H.fric_v, (void *)H.fric_c, (void *)H.fric_nrm, (void *)H.fric_lam}) dfree(s, old);
    H.fric_v = nv;
    H.fric_c = ncf;
    H.fric_nrm = nn;
    H.fric_lam = nl;
    H.fric_cap = nc;
    s.dev_dirty = true;
}

void grow_active(Scene &s, int64_t need)
{
    SceneDev &H = s.h;
    if (H.act_idx && need <= H.act_cap) return;
    int64_t nc = need + need / 2 + 256;
    size_t rs = real_size(s);
    Staged st(s);
    int32_t *ni = st.get<int32_t>(nc), *nv = st.get<int32_t>(4 * (size_t)nc);
    void *ng = st.get_bytes(12 * (size_t)nc * rs), *nh = st.get_bytes(144 * (size_t)nc * rs);
    void *ny = st.get_bytes(12 * (size_t)nc * rs);
    double *npp = st.get<double>((size_t)nblocks(nc, kPairsPerBlock) + 1);
    int32_t *nl = st.get<int32_t>(4 * (size_t)nc), *nr = st.get<int32_t>(4 * (size_t)nc);
    int32_t *nt = st.get<int32_t>(4 * (size_t)nc);
    st.commit();
    for (void *old : {(void *)H.act_idx, (void *)H.act_v, H.act_g, H.act_H, H.act_y, (void *)H.pcg_pair,
                      (void *)H.c_list, (void *)H.c_row, (void *)H.c_tmp})
        dfree(s, old);
    H.c_tmp = nt;
    H.act_idx = ni;
    H.act_v = nv;
    H.act_g = ng;
    H.act_H = nh;
    H.act_y = ny;
    H.pcg_pair = npp;
    H.c_list = nl;
    H.c_row = nr;
    H.act_cap = nc;
    s.dev_dirty = true;
}

static void activate(Batch &b, const std::vector<uint8_t> &on);

// Host image of the multilevel preconditioner's index arrays (layouts as in SceneDev).
struct MasHost {
    std::vector<int32_t> mem, manc, mb, me, gofs, dptr, dsrc, other, vpos;
};

// Nested aggregates of the free gel vertices. Level 0 bins the rest positions
// into cubic cells of edge twice the mean tet edge, separately for every
// connected body of the mesh; level l + 1 merges the 2x2x2 cells of level l
// (integer halving of the cell key, so levels nest exactly). Members are sorted by (top cell, ..., level-0 cell, vertex), so
// every aggregate is a contiguous run of member positions. A run is split at
// child boundaries wherever it would exceed kMasCapM members or kMasCapA
// aggregates in its subtree (any partition keeps the preconditioner SPD),
// which lets a group of top-level aggregates live in one block's LDS. A level
// that does not coarsen ends the hierarchy. The diagonal lists hold, for each
// aggregate, the BELL entries whose row and column first share an aggregate
// at its level, so the block of the aggregate is its list plus its children's
// blocks.
static void build_multilevel(SceneDev &H, int mas_target, const ipc_scene_desc &d, const std::vector<int32_t> &slice_ptr,
                             const std::vector<int32_t> &bcol, MasHost &M)
{
    const int ng = d.n_verts, m = d.n_tets, n = H.n;
    H.mas_levels = 0;
    H.mas_ng = 0;
    H.mas_nf = 0;
    H.mas_nd0 = 0;
    H.mas_nother = 0;
    std::vector<int32_t> freev;
    for (int i = 0; i < ng; ++i)
        if (!(d.fixed && d.fixed[i])) freev.push_back(i);
    const size_t nf = freev.size();
    if (nf < 2 || m == 0) return;
    double h0 = 0.0, org[3] = {INFINITY, INFINITY, INFINITY};
    for (int e = 0; e < m; ++e) {
        const double *a = d.X + 3 * d.T[4 * e], *b = d.X + 3 * d.T[4 * e + 1];
        h0 += std::sqrt((b[0] - a[0]) * (b[0] - a[0]) + (b[1] - a[1]) * (b[1] - a[1]) + (b[2] - a[2]) * (b[2] - a[2]));
    }
    h0 /= m;
    for (int i = 0; i < ng; ++i)
        for (int c = 0; c < 3; ++c) org[c] = std::min(org[c], d.X[3 * i + c]);
    // connected bodies of the tet mesh: an aggregate never spans two of them
    std::vector<int32_t> comp(ng);
    for (int i = 0; i < ng; ++i) comp[i] = i;
    auto root = [&](int32_t i) {
        while (comp[i] != i) i = comp[i] = comp[comp[i]];
        return i;
    };
    for (int e = 0; e < m; ++e)
        for (int a = 1; a < 4; ++a) {
            int32_t r0 = root(d.T[4 * e]), r1 = root(d.T[4 * e + a]);
            if (r0 != r1) comp[std::max(r0, r1)] = std::min(r0, r1);
        }
    // key = (body, cell): level-0 cells of edge 2 h0, integer halving per level
    std::vector<std::array<int64_t, 4>> key0(nf);
    for (size_t k = 0; k < nf; ++k) {
        key0[k][0] = root(freev[k]);
        for (int c = 0; c < 3; ++c) key0[k][1 + c] = (int64_t)std::floor((d.X[3 * freev[k] + c] - org[c]) / (2.0 * h0));
    }
    auto key_at = [&](size_t k, int l) {
        std::array<int64_t, 4> q = key0[k];
        for (int t = 0; t < l; ++t)
            for (int c = 1; c < 4; ++c) q[c] = q[c] >= 0 ? q[c] / 2 : -((-q[c] + 1) / 2);
        return q;
    };
    std::vector<size_t> ord(nf);
    for (size_t k = 0; k < nf; ++k) ord[k] = k;
    std::sort(ord.begin(), ord.end(), [&](size_t a, size_t b) {
        for (int l = kMasLevels - 1; l >= 0; --l) {
            auto ka = key_at(a, l), kb = key_at(b, l);
            if (ka != kb) return ka < kb;
        }
        return freev[a] < freev[b];
    });
    // aggregates of one level: [b, e) member positions (level 0) or child ids,
    // first member position, members and aggregates in the subtree
    struct Agg {
        int32_t b, e, fm, subm, suba;
    };
    std::vector<std::vector<Agg>> lv;
    {
        std::vector<Agg> a0;
        for (size_t k = 0; k < nf; ++k) {
            bool brk = a0.empty() || key_at(ord[k], 0) != key_at(ord[k - 1], 0) || a0.back().subm >= kMasCapM;
            if (brk)
                a0.push_back({(int32_t)k, (int32_t)k + 1, (int32_t)k, 1, 1});
            else {
                a0.back().e = (int32_t)k + 1;
                a0.back().subm++;
            }
        }
        if (a0.size() >= nf) return;  // cells hold single vertices: nothing to aggregate
        lv.push_back(std::move(a0));
    }
    for (int l = 1; l < kMasLevels; ++l) {
        const std::vector<Agg> &pr = lv.back();
        const int capA = kMasCapA - (kMasLevels - 1 - l);
        std::vector<Agg> nx;
        for (size_t c = 0; c < pr.size(); ++c) {
            const Agg &ch = pr[c];
            bool brk = nx.empty() || key_at(ord[ch.fm], l) != key_at(ord[pr[nx.back().b].fm], l) ||
                       nx.back().subm + ch.subm > kMasCapM || nx.back().suba + ch.suba > capA;
            if (brk)
                nx.push_back({(int32_t)c, (int32_t)c + 1, ch.fm, ch.subm, 1 + ch.suba});
            else {
                nx.back().e = (int32_t)c + 1;
                nx.back().subm += ch.subm;
                nx.back().suba += ch.suba;
            }
        }
        if (nx.size() >= pr.size()) break;
        lv.push_back(std::move(nx));
    }
    const int L = (int)lv.size();
    H.mas_levels = L;
    H.mas_nf = (int)nf;
    int total = 0;
    for (int l = 0; l < L; ++l) {
        H.mas_off[l] = total;
        H.mas_n[l] = (int)lv[l].size();
        total += H.mas_n[l];
    }
    H.mas_off[L] = total;
    H.mas_nd0 = (H.mas_n[0] + kBlock / kWave - 1) / (kBlock / kWave);
    M.mem.resize(nf);
    for (size_t k = 0; k < nf; ++k) M.mem[k] = freev[ord[k]];
    M.mb.clear();
    M.me.clear();
    for (int l = 0; l < L; ++l)
        for (auto &a : lv[l]) {
            M.mb.push_back(a.b);
            M.me.push_back(a.e);
        }
    // level-local aggregate of every member position, and of every vertex
    M.manc.assign((size_t)L * nf, -1);
    for (int a = 0; a < H.mas_n[0]; ++a)
        for (int32_t k = lv[0][a].b; k < lv[0][a].e; ++k) M.manc[k] = a;
    for (int l = 1; l < L; ++l) {
        std::vector<int32_t> par(lv[l - 1].size());
        for (int a = 0; a < H.mas_n[l]; ++a)
            for (int32_t c = lv[l][a].b; c < lv[l][a].e; ++c) par[c] = a;
        for (size_t k = 0; k < nf; ++k) M.manc[(size_t)l * nf + k] = par[M.manc[(size_t)(l - 1) * nf + k]];
    }
    M.vpos.assign(n, -1);
    for (size_t k = 0; k < nf; ++k) M.vpos[M.mem[k]] = (int32_t)k;
    M.other.clear();
    for (int i = 0; i < n; ++i)
        if (M.vpos[i] < 0) M.other.push_back(i);
    H.mas_nother = (int)M.other.size();
    std::vector<int32_t> vanc((size_t)L * n, -1);
    for (int l = 0; l < L; ++l)
        for (size_t k = 0; k < nf; ++k) vanc[(size_t)l * n + M.mem[k]] = M.manc[(size_t)l * nf + k];
    // groups: runs of top-level aggregates
    const std::vector<Agg> &top = lv[L - 1];
    std::vector<int32_t> gstart;  // first top aggregate of each group
    {
        int cm = 0, ca = 0;
        for (size_t t = 0; t < top.size(); ++t) {
            if (gstart.empty() || cm + top[t].subm > mas_target || ca + top[t].suba > kMasCapA) {
                gstart.push_back((int32_t)t);
                cm = ca = 0;
            }
            cm += top[t].subm;
            ca += top[t].suba;
        }
    }
    const int G = (int)gstart.size();
    H.mas_ng = G;
    M.gofs.assign((size_t)(L + 1) * (G + 1), 0);
    for (int g = 0; g <= G; ++g) {
        int32_t pos = g < G ? top[gstart[g]].fm : (int32_t)nf;
        M.gofs[g] = pos;
        for (int l = 0; l < L; ++l) {
            // level-l aggregates that start before member position pos
            auto it = std::lower_bound(lv[l].begin(), lv[l].end(), pos,
                                       [](const Agg &a, int32_t p) { return a.fm < p; });
            M.gofs[(size_t)(l + 1) * (G + 1) + g] = (int32_t)(it - lv[l].begin());
        }
    }
    // diagonal lists
    M.dptr.assign(1, 0);
    M.dsrc.clear();
    for (int l = 0; l < L; ++l)
        for (int a = 0; a < H.mas_n[l]; ++a) {
            const Agg &A = lv[l][a];
            for (int32_t k = A.fm; k < A.fm + A.subm; ++k) {
                int row = M.mem[k];
                int sl = row / kSlice, ln = row % kSlice;
                for (int slot = slice_ptr[sl]; slot < slice_ptr[sl + 1]; ++slot) {
                    size_t e = (size_t)slot * kSlice + ln;
                    int col = bcol[e];
                    if (col < 0 || vanc[(size_t)l * n + col] != a) continue;
                    if (l > 0 && vanc[(size_t)(l - 1) * n + col] == vanc[(size_t)(l - 1) * n + row]) continue;
                    M.dsrc.push_back((int32_t)e);
                }
            }
            M.dptr.push_back((int32_t)M.dsrc.size());
        }
}

static int32_t build_scene(Scene &s, const ipc_scene_desc &d)
{
    int n_gel_tris = 0, n_gel_edges = 0;
    const int ng = d.n_verts, m = d.n_tets, ni = d.n_ind_verts;
    s.h.n_gel = ng;
    s.h.n_ind = ni;
    s.h.n = ng + ni;
    s.h.m = m;
    const int n = s.h.n;
    s.tune = tuning_for(n);
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
    n_gel_tris = (int)gtris.size();
    s.h.n_tris = (int)(gtris.size() + itris.size());
    n_gel_edges = (int)gedges.size();
    s.h.n_edges = (int)(gedges.size() + iedges.size());
    s.h.n_gel_tris = n_gel_tris;
    s.h.n_gel_edges = n_gel_edges;
    s.h_tris.resize(3 * (size_t)s.h.n_tris);
    s.h_edges.resize(2 * (size_t)s.h.n_edges);
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
    s.h.n_pts = (int)s.h_pts.size();

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
    s.h.n_slices = (n + kSlice - 1) / kSlice;
    std::vector<int32_t> slice_ptr(s.h.n_slices + 1, 0);
    for (int sl = 0; sl < s.h.n_slices; ++sl) {
        int w = 1;
        for (int l = 0; l < kSlice; ++l) {
            int row = sl * kSlice + l;
            if (row < n) w = std::max(w, 1 + (int)nbr[row].size());
        }
        slice_ptr[sl + 1] = slice_ptr[sl] + w;
    }
    s.h.n_slots = slice_ptr[s.h.n_slices];
    s.nnzb = 0;
    for (int row = 0; row < n; ++row) s.nnzb += 1 + (int64_t)nbr[row].size();
    size_t nent = (size_t)s.h.n_slots * kSlice;
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

    // ---- multilevel aggregates of the free gel vertices (preconditioner)
    MasHost mas;
    s.h.mas_levels = 0;
    if (s.prm.precond == IPC_PRECOND_MULTILEVEL) build_multilevel(s.h, s.tune.mas_target, d, slice_ptr, bcol, mas);
    s.mas_max_members = s.mas_max_aggs = 0;
    for (int g = 0; g < s.h.mas_ng; ++g) {
        const int G1 = s.h.mas_ng + 1;
        int aggs = 0;
        for (int l = 0; l < s.h.mas_levels; ++l) aggs += mas.gofs[(size_t)(l + 1) * G1 + g + 1] - mas.gofs[(size_t)(l + 1) * G1 + g];
        s.mas_max_members = std::max(s.mas_max_members, mas.gofs[g + 1] - mas.gofs[g]);
        s.mas_max_aggs = std::max(s.mas_max_aggs, aggs);
    }

    // ---- SoA tets, surface arrays
    std::vector<int32_t> tv(4 * (size_t)m);
    for (int e = 0; e < m; ++e)
        for (int a = 0; a < 4; ++a) tv[(size_t)a * m + e] = d.T[4 * e + a];
    std::vector<int32_t> ev(2 * (size_t)s.h.n_edges), trv(3 * (size_t)s.h.n_tris);
    for (int k = 0; k < s.h.n_edges; ++k) {
        ev[k] = s.h_edges[2 * k];
        ev[(size_t)s.h.n_edges + k] = s.h_edges[2 * k + 1];
    }
    for (int k = 0; k < s.h.n_tris; ++k)
        for (int c = 0; c < 3; ++c) trv[(size_t)c * s.h.n_tris + k] = s.h_tris[3 * k + c];
    std::vector<double> ers(s.h.n_edges);
    for (int k = 0; k < s.h.n_edges; ++k) {
        const double *a = &X0[3 * (size_t)s.h_edges[2 * k]], *b = &X0[3 * (size_t)s.h_edges[2 * k + 1]];
        double dd[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
        ers[k] = dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2];
    }
    std::vector<uint8_t> fixed(n, 0);
    if (d.fixed)
        for (int i = 0; i < ng; ++i) fixed[i] = d.fixed[i] ? 1 : 0;
    s.h_Yloc.assign(d.ind_Y, d.ind_Y + 3 * (size_t)ni);
    std::memcpy(s.pose0, d.ind_pose0, sizeof(double) * 12);

    // ---- device buffers and the device view
    SceneDev &H = s.h;
    size_t rs = real_size(s);
    size_t n3 = 3 * (size_t)n;
    H.n_surf = (int)s.h_surf_verts.size();
    H.nb_vert = nblocks(n);
    H.nb_rows = nblocks(n, kRowsPerBlock);
    H.mu = s.prm.mu;
    H.lam = s.prm.lam;
    H.h = s.prm.dt;
    H.inv_h2 = 1.0 / (s.prm.dt * s.prm.dt);
    H.dhat = s.prm.dhat;
    H.kappa = s.prm.kappa;
    H.k_target = s.prm.k_target;
    H.rho = s.prm.rho;
    for (int c = 0; c < 3; ++c) H.grav[c] = s.prm.grav[c];
    H.ccd_s = s.prm.ccd_s;
    H.pcg_tol2 = s.prm.pcg_tol * s.prm.pcg_tol;
    H.mu_fric = s.prm.mu_fric;
    H.barrier_gn = s.prm.barrier_hessian == IPC_BARRIER_GAUSS_NEWTON;
    std::memcpy(H.case_pose, kIdentityPose, sizeof(kIdentityPose));
    H.attached = nullptr;
    if (d.attached) {
        std::vector<uint8_t> at(ng, 0);
        bool any = false;
        for (int i = 0; i < ng; ++i) {
            at[i] = (d.attached[i] && !(d.fixed && d.fixed[i])) ? 1 : 0;
            any |= at[i] != 0;
        }
        if (any) H.attached = upload(s, at);
    }
    H.eps_fric = s.prm.eps_v * s.prm.dt;
    H.n_fric = 0;
    H.self_contact = s.prm.self_contact;
    H.ccd_max_iter = s.prm.ccd_max_iter;
    H.precision = s.prm.precision;
    std::memcpy(H.pose, d.ind_pose0, sizeof(double) * 12);
    H.X0 = upload(s, X0);
    H.x = dalloc<double>(s, n3);
    H.v = dalloc<double>(s, n3);
    H.xt = dalloc<double>(s, n3);
    H.xtilde = dalloc<double>(s, n3);
    H.yhat = dalloc<double>(s, n3);
    H.target_al = s.prm.target_al;
    H.al_lam = dalloc<double>(s, n3);
    IPC_HIP(hipMemsetAsync(H.al_lam, 0, sizeof(double) * n3, s.stream));
    H.xtrial = dalloc<double>(s, n3);
    for (double *p : {H.x, H.xt, H.xtilde, H.yhat, H.xtrial})
        IPC_HIP(hipMemcpyAsync(p, H.X0, sizeof(double) * n3, hipMemcpyDeviceToDevice, s.stream));
    IPC_HIP(hipMemsetAsync(H.v, 0, sizeof(double) * n3, s.stream));
    H.Yloc = upload(s, s.h_Yloc);
    H.fixed = upload(s, fixed);
    H.mass = dalloc<double>(s, n);
    H.tv = upload(s, tv);
    H.Bm = dalloc<double>(s, 9 * (size_t)m);
    H.vol = dalloc<double>(s, m);
    H.eg = dalloc_bytes(s, 12 * (size_t)m * rs);
    H.eH = dalloc_bytes(s, 90 * (size_t)m * rs);
    H.vt_ptr = upload(s, vt_ptr);
    H.vt_src = upload(s, vt_src);
    H.slice_ptr = upload(s, slice_ptr);
    H.bcol = upload(s, bcol);
    H.bval = dalloc_bytes(s, nent * 9 * rs);
    H.g_ptr = upload(s, g_ptr);
    H.g_src = upload(s, g_src);
    H.grad = dalloc_bytes(s, n3 * rs);
    H.Minv = dalloc_bytes(s, 9 * (size_t)n * rs);
    H.pts = upload(s, s.h_pts);
    H.ev = upload(s, ev);
    H.trv = upload(s, trv);
    H.surf_verts = upload(s, s.h_surf_verts);
    {
        std::vector<int32_t> pidx(n, -1);
        for (size_t k = 0; k < s.h_pts.size(); ++k) pidx[s.h_pts[k]] = (int32_t)k;
        H.pt_idx = upload(s, pidx);
        IPC_HIP(hipStreamSynchronize(s.stream));
    }
    H.edge_rest_sq = upload(s, ers);
    H.pbox = dalloc<double>(s, 6 * (size_t)std::max(H.n_pts, 1));
    H.ebox = dalloc<double>(s, 6 * (size_t)std::max(H.n_edges, 1));
    H.tbox = dalloc<double>(s, 6 * (size_t)std::max(H.n_tris, 1));
    H.cell_h = dalloc<double>(s, 1);
    H.c_ptr = dalloc<int32_t>(s, n + 1);
    H.c_cnt = dalloc<int32_t>(s, n + 1);
    IPC_HIP(hipMemsetAsync(H.c_ptr, 0, sizeof(int32_t) * (n + 1), s.stream));
    for (void **p : {&H.r, &H.z, &H.dA, &H.dB, &H.q, &H.sol}) *p = dalloc_bytes(s, n3 * rs);
    IPC_HIP(hipMemsetAsync(H.sol, 0, n3 * rs, s.stream));
    H.pcg_nvp = H.mas_levels > 0 ? H.mas_ng + nblocks(H.mas_nother) : H.nb_vert;
    H.pcg_part = dalloc<double>(s, (size_t)H.nb_rows + 2 * ((size_t)H.pcg_nvp + n + 1) + 8);
    H.hflag = dalloc<int32_t>(s, n + 1);
    H.heavy_idx = dalloc<int32_t>(s, n + 1);
    H.heavy_rows = dalloc<int32_t>(s, n + 1);
    H.hdiag = dalloc<double>(s, 9 * ((size_t)n + 1));
    IPC_HIP(hipMemsetAsync(H.hflag, 0, sizeof(int32_t) * (n + 1), s.stream));
    if (H.mas_levels > 0) {
        int total = H.mas_off[H.mas_levels];
        H.mas_mem = upload(s, mas.mem);
        H.mas_manc = upload(s, mas.manc);
        H.mas_mb = upload(s, mas.mb);
        H.mas_me = upload(s, mas.me);
        H.mas_gofs = upload(s, mas.gofs);
        H.mas_dptr = upload(s, mas.dptr);
        H.mas_dsrc = upload(s, mas.dsrc);
        H.mas_ex = dalloc<double>(s, 9 * (size_t)total);
        H.mas_dinv = dalloc_bytes(s, 9 * (size_t)total * rs);
        H.mas_other = upload(s, mas.other);
        H.mas_vpos = upload(s, mas.vpos);
        IPC_HIP(hipStreamSynchronize(s.stream));  // host vectors above are locals
    }
    H.pcg = dalloc<PcgState>(s, 1);
    IPC_HIP(hipMemsetAsync(H.pcg, 0, sizeof(PcgState), s.stream));
    // entry capacity: a primitive's box spans about five cells (grown when a
    // count pass finds more); without self-contact only the indenter's edges
    // enter the edge table
    grow_table(s, 0, 8 * (int64_t)std::max(H.n_tris, 1));
    grow_table(s, 1, 8 * (int64_t)std::max(H.self_contact ? H.n_edges : H.n_edges - H.n_gel_edges, 1));
    H.q_count = dalloc<int32_t>(s, (size_t)H.n_pts + H.n_edges + 1);
    H.q_off = dalloc<int32_t>(s, (size_t)H.n_pts + H.n_edges + 1);
    H.q_lane = dalloc<int32_t>(s, (size_t)kLanesQ * ((size_t)H.n_pts + H.n_edges) + 1);
    H.q_keep = dalloc<int32_t>(s, (size_t)kQueryKeep * kLanesQ * ((size_t)H.n_pts + H.n_edges) + 1);
    grow_candidates(s, 0, 1024);
    grow_candidates(s, 1, 1024);
    grow_active(s, 256);
    grow_friction(s, s.prm.mu_fric > 0.0 ? 256 : 1);
    H.pcg_maxit = s.prm.pcg_max_iter > 0 ? s.prm.pcg_max_iter : 30 * n;
    s.n_gel_tris = n_gel_tris;
    s.xsave = dalloc<double>(s, n3);
    s.ysurf = dalloc<double>(s, 3 * (size_t)std::max(H.n_surf, 1));
    s.dev = dalloc<SceneDev>(s, 1);
    s.dev_dirty = true;
    // rest shape and lumped mass on the device, through the scene's list of one
    s.solo.reset(new Batch());
    Batch &b = *s.solo;
    b.bind({&s}, s.stream);
    activate(b, {1});
    launch_rest_precompute(b);
    IPC_HIP(hipStreamSynchronize(s.stream));
    return IPC_OK;
}

// ---------------------------------------------------------------------------
// a list of scenes stepping together
// ---------------------------------------------------------------------------

Batch::~Batch()
{
    if (stream) (void)hipStreamSynchronize(stream);
    for (auto &p : ev_pending) {
        ev_pool.push_back(p.a);
        ev_pool.push_back(p.b);
    }
    for (auto e : ev_pool) (void)hipEventDestroy(e);
    (void)hipFree(d_list);
    (void)hipFree(d_offs);
    (void)hipFree(d_vstage);
    (void)hipFree(d_out);
    (void)hipFree(d_alpha);
    if (h_out) (void)hipHostFree(h_out);
    if (h_stage) (void)hipHostFree(h_stage);
}

// The staging buffer starts small (a list of one stages a few hundred bytes
// between read-backs) and doubles, up to kStageMax, whenever it fills up
// between two read-backs: a full buffer costs a stream synchronisation.
constexpr size_t kStageMin = size_t(64) << 10, kStageMax = size_t(64) << 20;

void *Batch::stage_alloc(size_t bytes)
{
    size_t need = (bytes + 63) & ~size_t(63);
    if (!h_stage) {
        stage_cap = std::max(kStageMin, need);
        IPC_HIP(hipHostMalloc((void **)&h_stage, stage_cap, 0));
        stage_used = 0;
    }
    if (stage_used + need > stage_cap) {
        IPC_HIP(hipStreamSynchronize(stream));
        stage_used = 0;
        const size_t grown = std::max(need, std::min(2 * stage_cap, kStageMax));
        if (grown > stage_cap) {
            IPC_HIP(hipHostFree(h_stage));
            h_stage = nullptr;
            stage_cap = grown;
            IPC_HIP(hipHostMalloc((void **)&h_stage, stage_cap, 0));
        }
    }
    void *p = h_stage + stage_used;
    stage_used += need;
    return p;
}

void *Batch::stage(const void *src, size_t bytes)
{
    void *p = stage_alloc(bytes);
    std::memcpy(p, src, bytes);
    return p;
}

void Batch::bind(const std::vector<Scene *> &scenes, hipStream_t strm)
{
    bool same = scenes == sc && strm == stream && d_list;
    int ns = (int)scenes.size();
    fail.assign(ns, 0);
    h_alpha.assign(ns, 0.0);
    if (same) {
        upload_views();
        return;
    }
    stream = strm;
    sc = scenes;
    if (ns > cap) {
        int nc = std::max(ns, std::max(4, 2 * cap));
        IPC_HIP(hipStreamSynchronize(stream));
        (void)hipFree(d_list);
        (void)hipFree(d_offs);
        (void)hipFree(d_vstage);
        (void)hipFree(d_out);
        (void)hipFree(d_alpha);
        if (h_out) (void)hipHostFree(h_out);
        d_list = nullptr;
        d_offs = nullptr;
        d_vstage = nullptr;
        d_out = nullptr;
        d_alpha = nullptr;
        h_out = nullptr;
        for (auto &d : d_off) d = nullptr;
        cap = 0;
        IPC_HIP(hipMalloc(&d_list, sizeof(SceneDev *) * nc));
        IPC_HIP(hipMalloc(&d_offs, sizeof(int32_t) * kPhKinds * (nc + 1)));
        for (int k = 0; k < kPhKinds; ++k) d_off[k] = d_offs + (size_t)k * (nc + 1);
        h_offs.assign((size_t)kPhKinds * (nc + 1), 0);
        IPC_HIP(hipMalloc(&d_vstage, view_stage_bytes(nc)));
        IPC_HIP(hipMalloc(&d_out, sizeof(SceneOut) * nc));
        IPC_HIP(hipMalloc(&d_alpha, sizeof(double) * nc));
        IPC_HIP(hipHostMalloc((void **)&h_out, sizeof(SceneOut) * nc, 0));
        std::memset(h_out, 0, sizeof(SceneOut) * nc);
        IPC_HIP(hipMemsetAsync(d_out, 0, sizeof(SceneOut) * nc, stream));
        cap = nc;
    }
    std::vector<SceneDev *> ptrs(ns);
    for (int i = 0; i < ns; ++i) ptrs[i] = sc[i]->dev;
    if (ns)
        IPC_HIP(hipMemcpyAsync(d_list, stage(ptrs.data(), sizeof(SceneDev *) * ns), sizeof(SceneDev *) * ns,
                               hipMemcpyHostToDevice, stream));
    for (auto &h : h_off) h.clear();
    pend_lo = kPhKinds;
    pend_hi = -1;
    upload_views();
}

void Batch::set_phase(PhaseKind k, const std::vector<int32_t> &per_scene_blocks)
{
    std::vector<int32_t> off(per_scene_blocks.size() + 1, 0);
    for (size_t i = 0; i < per_scene_blocks.size(); ++i) off[i + 1] = off[i] + per_scene_blocks[i];
    if (off == h_off[k]) return;
    h_off[k].swap(off);
    std::copy(h_off[k].begin(), h_off[k].end(), h_offs.begin() + (size_t)k * (cap + 1));
    pend_lo = std::min(pend_lo, (int)k);
    pend_hi = std::max(pend_hi, (int)k);
}

void Batch::flush_phases()
{
    if (pend_hi < 0) return;
    const size_t stride = (size_t)cap + 1, first = (size_t)pend_lo * stride;
    const size_t bytes = sizeof(int32_t) * (size_t)(pend_hi - pend_lo + 1) * stride;
    IPC_HIP(hipMemcpyAsync(d_offs + first, stage(h_offs.data() + first, bytes), bytes, hipMemcpyHostToDevice, stream));
    pend_lo = kPhKinds;
    pend_hi = -1;
}

// One changed view: a copy. Several: one copy of all of them (with their
// slots' addresses) into d_vstage, then a kernel puts each in its slot.
void Batch::upload_views()
{
    std::vector<Scene *> dirty;  // each changed scene once (its flag cleared as it is taken)
    for (Scene *s : sc)
        if (s->dev_dirty) {
            dirty.push_back(s);
            s->dev_dirty = false;
        }
    const int nd = (int)dirty.size();
    if (nd == 0) return;
    if (nd == 1) {
        IPC_HIP(hipMemcpyAsync(dirty[0]->dev, stage(&dirty[0]->h, sizeof(SceneDev)), sizeof(SceneDev),
                               hipMemcpyHostToDevice, stream));
        return;
    }
    const size_t bytes = view_stage_bytes(nd), head = (size_t)view_head_bytes(nd);
    char *p = static_cast<char *>(stage_alloc(bytes));
    for (int j = 0; j < nd; ++j) {
        std::memcpy(p + sizeof(SceneDev *) * j, &dirty[j]->dev, sizeof(SceneDev *));
        std::memcpy(p + head + sizeof(SceneDev) * j, &dirty[j]->h, sizeof(SceneDev));
    }
    IPC_HIP(hipMemcpyAsync(d_vstage, p, bytes, hipMemcpyHostToDevice, stream));
    launch_put_views(stream, nd, d_vstage);
}

void Batch::read_out()
{
    if (sc.empty()) return;
    IPC_HIP(hipMemcpyAsync(h_out, d_out, sizeof(SceneOut) * sc.size(), hipMemcpyDeviceToHost, stream));
    IPC_HIP(hipStreamSynchronize(stream));
    stage_used = 0;
    for (size_t i = 0; i < sc.size(); ++i) sc[i]->last = h_out[i];
}

bool Batch::prof() const { return sink || (sc.size() == 1 && sc[0]->prof); }

void Batch::prof_begin(int kernel, hipEvent_t *pair)
{
    (void)kernel;
    if (!prof()) return;
    for (int k = 0; k < 2; ++k) {
        if (ev_pool.empty()) {
            hipEvent_t e;
            IPC_HIP(hipEventCreate(&e));
            ev_pool.push_back(e);
        }
        pair[k] = ev_pool.back();
        ev_pool.pop_back();
    }
    IPC_HIP(hipEventRecord(pair[0], stream));
}

void Batch::prof_end(int kernel, hipEvent_t *pair, double bytes)
{
    if (!prof()) return;
    IPC_HIP(hipEventRecord(pair[1], stream));
    ev_pending.push_back({kernel, pair[0], pair[1], bytes});
}

void Batch::prof_totals(int kernel, int64_t launches, double bytes)
{
    if (!prof()) return;
    ProfAcc *acc = nullptr;
    std::unique_lock<std::mutex> lk;
    if (sink) {
        lk = std::unique_lock<std::mutex>(sink->mu);
        acc = &sink->acc[kernel];
    } else if (!sc.empty()) {
        acc = &sc[0]->prof_acc[kernel];
    }
    if (acc) {
        acc->launches_all += launches;
        acc->bytes_all += bytes;
    }
}

void Batch::prof_collect()
{
    if (ev_pending.empty()) return;
    for (auto &p : ev_pending) {
        float ms = 0.f;
        IPC_HIP(hipEventSynchronize(p.b));
        IPC_HIP(hipEventElapsedTime(&ms, p.a, p.b));
        ProfAcc *acc = nullptr;
        std::unique_lock<std::mutex> lk;
        if (sink) {
            lk = std::unique_lock<std::mutex>(sink->mu);
            acc = &sink->acc[p.kernel];
        } else if (!sc.empty()) {
            acc = &sc[0]->prof_acc[p.kernel];
        }
        if (acc) {
            acc->launches++;
            acc->ms += ms;
            acc->bytes += p.bytes;
            if (p.big) {
                acc->launches_big++;
                acc->ms_big += ms;
                acc->bytes_big += p.bytes;
            }
        }
        ev_pool.push_back(p.a);
        ev_pool.push_back(p.b);
    }
    ev_pending.clear();
}

// phase maps of the per-item kernels for the scenes with on[i] set; the
// others get no blocks and sit the phases out
static void activate(Batch &b, const std::vector<uint8_t> &on)
{
    size_t ns = b.sc.size();
    std::vector<int32_t> v(ns), t(ns), e(ns), sl(ns), p(ns), ed(ns), tr(ns), bd(ns);
    for (size_t i = 0; i < ns; ++i) {
        const SceneDev &H = b.sc[i]->h;
        bool a = on[i] != 0;
        v[i] = a ? nblocks(H.n) : 0;
        t[i] = a ? nblocks(H.m) : 0;
        e[i] = a ? nblocks((int64_t)H.n_slots * kSlice) : 0;
        sl[i] = a ? H.nb_rows : 0;
        p[i] = a ? nblocks(H.n_pts) : 0;
        ed[i] = a ? nblocks(H.n_edges) : 0;
        tr[i] = a ? nblocks(H.n_tris) : 0;
        bd[i] = a ? nblocks((int64_t)H.m + H.n) : 0;
    }
    b.set_phase(kPhVert, v);
    b.set_phase(kPhTet, t);
    b.set_phase(kPhEntry, e);
    b.set_phase(kPhSlice, sl);
    b.set_phase(kPhPts, p);
    b.set_phase(kPhEdges, ed);
    b.set_phase(kPhTris, tr);
    b.set_phase(kPhBody, bd);
    for (size_t i = 0; i < ns; ++i) {
        const SceneDev &H = b.sc[i]->h;
        p[i] = on[i] ? nblocks((int64_t)H.n_pts * kLanesQ) : 0;
        ed[i] = on[i] ? nblocks((int64_t)H.n_edges * kLanesQ) : 0;
    }
    b.set_phase(kPhQPts, p);
    b.set_phase(kPhQEdges, ed);
    std::vector<int32_t> pr(ns), te(ns), qa(ns);
    for (size_t i = 0; i < ns; ++i) {
        const SceneDev &H = b.sc[i]->h;
        pr[i] = on[i] ? nblocks(H.n_pts) + nblocks(H.n_edges) + nblocks(H.n_tris) : 0;
        te[i] = on[i] ? nblocks(H.n_tris) + nblocks(H.n_edges) : 0;
        qa[i] = on[i] ? nblocks((int64_t)H.n_pts * kLanesQ) + nblocks((int64_t)H.n_edges * kLanesQ) : 0;
    }
    b.set_phase(kPhPrims, pr);
    b.set_phase(kPhTE, te);
    b.set_phase(kPhQAll, qa);
    std::vector<int32_t> ms(ns), mg(ns);
    for (size_t i = 0; i < ns; ++i) {
        const SceneDev &h = b.sc[i]->h;
        bool ml = on[i] && h.mas_levels > 0;
        ms[i] = ml ? h.mas_nd0 + (h.mas_off[h.mas_levels] - h.mas_n[0]) : 0;
        mg[i] = ml ? h.mas_ng : 0;
    }
    b.set_phase(kPhMas, ms);
    b.set_phase(kPhMasG, mg);
}

// ---------------------------------------------------------------------------
// Newton
// ---------------------------------------------------------------------------

using Clock = std::chrono::steady_clock;
static double ms_since(Clock::time_point t0)
{
    return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
}

// Per-scene control of one step inside a list.
struct StepCtl {
    bool active = false;   // still iterating
    bool failed = false;   // an error ended the step (status < 0)
    bool stepped = false;  // the last iteration moved x (else it only measured p)
    int k = 0;             // Newton iterations done
    int status = IPC_OK;
    bool pcg_warn = false;
    ipc_step_stats st{};
    double alpha = 0.0, alpha0 = 0.0, E0 = 0.0;
    int al = 0;            // multiplier updates so far (augmented-Lagrangian targets)
    bool al_step = false;  // the multipliers just changed: the next iteration takes its step
};

// scenes that a host phase marked failed leave the list's phases
static void drop_failed(Batch &b, std::vector<StepCtl> &ctl, std::vector<uint8_t> &on)
{
    bool any = false;
    for (size_t i = 0; i < b.sc.size(); ++i) {
        if (!b.fail[i] || ctl[i].failed) continue;
        ctl[i].failed = true;
        ctl[i].active = false;
        ctl[i].status = b.fail[i];
        if (on[i]) {
            on[i] = 0;
            any = true;
        }
    }
    if (any) activate(b, on);
}

static void static_candidates(Batch &b, std::vector<StepCtl> &ctl, std::vector<uint8_t> &on);

// g and H at x for the scenes with on[i]: static candidates, active pairs,
// barrier, incidence, elastic elements, deterministic gather
static void assemble_round(Batch &b, std::vector<StepCtl> &ctl, std::vector<uint8_t> &on, double *ms)
{
    auto t0 = Clock::now();
    static_candidates(b, ctl, on);
    run_narrow_phase(b);
    drop_failed(b, ctl, on);
    launch_barrier(b);
    launch_friction(b);
    launch_contact_incidence(b);
    ms[1] += ms_since(t0);
    t0 = Clock::now();
    launch_elastic_elements(b);
    launch_assemble(b);
    ms[0] += ms_since(t0);
}

// static candidates at x for the scenes with on[i]: filtered from the kept
// swept list where that list is valid at x, else a hash query
static void static_candidates(Batch &b, std::vector<StepCtl> &ctl, std::vector<uint8_t> &on)
{
    size_t ns = b.sc.size();
    std::vector<uint8_t> on_q(ns, 0), on_f(ns, 0);
    bool any_q = false, any_f = false;
    for (size_t i = 0; i < ns; ++i) {
        if (!on[i]) continue;
        if (b.sc[i]->sw_ok) {
            on_f[i] = 1;
            any_f = true;
        } else {
            on_q[i] = 1;
            any_q = true;
        }
    }
    if (any_q) {
        activate(b, on_q);
        run_broad_phase(b, 0);
    }
    if (any_f) {
        activate(b, on_f);
        run_static_from_swept(b);
    }
    activate(b, on);
    drop_failed(b, ctl, on);
}

// One Newton iteration for every scene with ctl[i].active.
static void newton_round(Batch &b, std::vector<StepCtl> &ctl)
{
    size_t ns = b.sc.size();
    std::vector<uint8_t> on(ns);
    for (size_t i = 0; i < ns; ++i) on[i] = ctl[i].active;
    double ms[8] = {0};
    assemble_round(b, ctl, on, ms);
    auto t0 = Clock::now();
    std::vector<int> iters, caps;
    run_pcg(b, iters, caps);  // also |p|_inf, read back with the PCG's last flags
    ms[2] += ms_since(t0);
    std::vector<uint8_t> ls(ns, 0);
    bool any = false;
    for (size_t i = 0; i < ns; ++i) {
        if (!on[i]) continue;
        StepCtl &c = ctl[i];
        c.st.newton_iters++;
        c.k++;
        c.st.pcg_iters += iters[i];
        c.pcg_warn |= caps[i] != 0;
        c.st.pinf = b.h_out[i].pinf;
        c.st.n_candidates = b.h_out[i].n_cand;
        c.st.n_active = b.h_out[i].n_act;
        c.stepped = false;
        if (b.h_out[i].pinf <= b.sc[i]->prm.newton_tol && !c.al_step) {
            c.active = false;  // converged: this iteration only measured p
        } else {
            ls[i] = 1;
            any = true;
        }
        c.al_step = false;
    }
    // augmented-Lagrangian targets: a scene that converged with its indenter
    // further than the tolerance from its targets updates its multipliers
    // and goes on
    {
        std::vector<uint8_t> al(ns, 0);
        bool any_al = false;
        for (size_t i = 0; i < ns; ++i) {
            const Params &pm = b.sc[i]->prm;
            if (on[i] && !ctl[i].active && !ctl[i].failed && pm.target_al && ctl[i].al < pm.target_al_max) {
                al[i] = 1;
                any_al = true;
            }
        }
        if (any_al) {
            activate(b, al);
            run_lag_and_mean(b);
            b.read_out();
            std::vector<uint8_t> upd(ns, 0);
            bool any_upd = false;
            for (size_t i = 0; i < ns; ++i)
                if (al[i] && b.h_out[i].lag > b.sc[i]->prm.target_al_tol) {
                    upd[i] = 1;
                    any_upd = true;
                }
            if (any_upd) {
                activate(b, upd);
                launch_al_update(b, upd);
                for (size_t i = 0; i < ns; ++i)
                    if (upd[i]) {
                        StepCtl &c = ctl[i];
                        c.active = true;
                        c.al_step = true;
                        c.st.al_updates = ++c.al;
                    }
            }
        }
    }
    if (any) {
        t0 = Clock::now();
        activate(b, ls);
        run_broad_phase(b, 1);
        drop_failed(b, ctl, ls);
        run_ccd(b);
        run_energy(b, false);
        b.read_out();
        for (size_t i = 0; i < ns; ++i)
            if (ls[i]) {
                // x only moves along [x, x + p] from here on, so this list
                // keeps every static pair of the next iterate
                b.sc[i]->sw_ok = true;
                b.sc[i]->sw_n = b.h_out[i].n_sw;
            }
        ms[3] += ms_since(t0);
        t0 = Clock::now();
        for (size_t i = 0; i < ns; ++i)
            if (ls[i]) {
                StepCtl &c = ctl[i];
                c.st.alpha_ccd = b.h_out[i].alpha_ccd;
                c.alpha = std::min(1.0, b.h_out[i].alpha_ccd);
                c.alpha0 = c.alpha;
                c.E0 = b.h_out[i].infeasible ? INFINITY : b.h_out[i].energy;
            }
        // Backtracking: every scene halves its own step until its energy does
        // not increase. The trial count is bounded (a step of 2^-1100 is 0).
        std::vector<uint8_t> pend = ls;
        for (int trial = 0; trial < 1100; ++trial) {
            bool left = false;
            for (size_t i = 0; i < ns; ++i) {
                b.h_alpha[i] = pend[i] ? ctl[i].alpha : 0.0;
                left |= pend[i] != 0;
            }
            if (!left) break;
            IPC_HIP(hipMemcpyAsync(b.d_alpha, b.stage(b.h_alpha.data(), sizeof(double) * ns), sizeof(double) * ns,
                                   hipMemcpyHostToDevice, b.stream));
            activate(b, pend);
            launch_trial(b);
            run_energy(b, true);
            b.read_out();
            std::vector<uint8_t> acc(ns, 0);
            for (size_t i = 0; i < ns; ++i) {
                if (!pend[i]) continue;
                StepCtl &c = ctl[i];
                double E = b.h_out[i].infeasible ? INFINITY : b.h_out[i].energy;
                if (E <= c.E0) {
                    acc[i] = 1;
                    pend[i] = 0;
                    c.stepped = true;
                    c.st.alpha = c.alpha;
                    c.st.energy = E;
                } else {
                    c.alpha *= 0.5;
                    c.st.ls_halvings++;
                    if (c.alpha < b.sc[i]->prm.ls_min_ratio * c.alpha0 || !(c.alpha > 0.0)) {
                        pend[i] = 0;
                        c.status = IPC_W_LS_STALL;
                        c.active = false;
                        c.st.alpha = 0.0;
                        c.st.energy = c.E0;
                    }
                }
            }
            activate(b, acc);
            launch_accept(b);
        }
        for (size_t i = 0; i < ns; ++i)
            if (pend[i]) {  // the bound above was reached
                ctl[i].status = IPC_W_LS_STALL;
                ctl[i].active = false;
                ctl[i].st.alpha = 0.0;
                ctl[i].st.energy = ctl[i].E0;
            }
        ms[4] += ms_since(t0);
    }
    for (size_t i = 0; i < ns; ++i) {
        if (!on[i]) continue;
        for (int k = 0; k < 8; ++k) ctl[i].st.ms_phase[k] += ms[k];
        if (ctl[i].active && ctl[i].k >= b.sc[i]->prm.max_newton) {
            ctl[i].active = false;
            ctl[i].status = IPC_W_NEWTON_MAXITER;
        }
    }
}

static void set_pose(Scene &s, const double *pose)
{
    std::memcpy(s.h.pose, pose, sizeof(double) * 12);
    s.dev_dirty = true;
}

static void set_case_pose(Scene &s, const double *pose)
{
    std::memcpy(s.h.case_pose, pose, sizeof(double) * 12);
    s.dev_dirty = true;
}

// the poses of one step request
static void set_request(Scene &s, const ipc_step_req &r)
{
    set_pose(s, r.pose);
    if (r.case_pose_set) set_case_pose(s, r.case_pose);
}


// predictor and targets of the scenes with on[i] (poses already set), and the
// lagged friction set at x^t of the scenes with friction
static void begin_steps(Batch &b, const std::vector<uint8_t> &on, std::vector<StepCtl> &ctl)
{
    b.upload_views();
    activate(b, on);
    launch_begin_step(b);
    size_t ns = b.sc.size();
    std::vector<uint8_t> onf(ns, 0);
    bool any = false;
    for (size_t i = 0; i < ns; ++i) {
        if (!on[i]) continue;  // scenes in mid-step keep their lagged friction set
        Scene &s = *b.sc[i];
        if (s.h.n_fric) {
            s.h.n_fric = 0;
            s.dev_dirty = true;
        }
        if (s.prm.mu_fric > 0.0) {
            onf[i] = 1;
            any = true;
        }
    }
    b.upload_views();
    if (!any) return;
    static_candidates(b, ctl, onf);
    run_narrow_phase(b);
    drop_failed(b, ctl, onf);
    for (size_t i = 0; i < ns; ++i) {
        if (!onf[i]) continue;
        Scene &s = *b.sc[i];
        try {
            grow_friction(s, b.h_out[i].n_act);
            s.h.n_fric = b.h_out[i].n_act;
            s.dev_dirty = true;
        } catch (const OomError &) {
            b.fail[i] = IPC_E_OOM;
        }
    }
    drop_failed(b, ctl, onf);
    b.upload_views();
    launch_friction_lag(b);
}

// Commit of the scenes with on[i]: v = (x - x^t)/h, target lag, object
// position, final status. A failed step restores x = x^t (its state is then
// as before the step).
static void end_steps(Batch &b, const std::vector<uint8_t> &on, std::vector<StepCtl> &ctl)
{
    size_t ns = b.sc.size();
    std::vector<uint8_t> ok(ns, 0);
    for (size_t i = 0; i < ns; ++i) {
        if (!on[i]) continue;
        if (ctl[i].failed) {
            Scene &s = *b.sc[i];
            s.sw_ok = false;
            IPC_HIP(hipMemcpyAsync(s.h.x, s.h.xt, sizeof(double) * 3 * s.h.n, hipMemcpyDeviceToDevice, b.stream));
        } else {
            ok[i] = 1;
        }
    }
    activate(b, ok);
    launch_end_step(b);
    run_lag_and_mean(b);
    b.read_out();
    b.prof_collect();
    for (size_t i = 0; i < ns; ++i) {
        if (!on[i]) continue;
        StepCtl &c = ctl[i];
        if (!ok[i]) {
            c.st.status = c.status;
            continue;
        }
        Scene &s = *b.sc[i];
        c.st.max_target_lag = b.h_out[i].lag;
        int status = c.status;
        if (status == IPC_OK && c.pcg_warn) status = IPC_W_PCG_MAXITER;
        if (status == IPC_OK && c.st.max_target_lag > 1e-3 * s.prm.dhat) status = IPC_W_TARGET_LAG;
        c.st.status = status;
        s.step_index++;
    }
}

static void start_ctl(StepCtl &c)
{
    c = StepCtl{};
    c.active = true;
    c.st.energy = NAN;
}

// Steps every scene of the list to completion in shared launches.
static void step_list(Batch &b, const std::vector<const ipc_step_req *> &reqs, std::vector<StepCtl> &ctl)
{
    size_t ns = b.sc.size();
    auto t0 = Clock::now();
    for (size_t i = 0; i < ns; ++i) set_request(*b.sc[i], *reqs[i]);
    ctl.assign(ns, StepCtl{});
    for (auto &c : ctl) start_ctl(c);
    std::vector<uint8_t> all(ns, 1);
    begin_steps(b, all, ctl);
    for (;;) {
        bool any = false;
        for (auto &c : ctl) any |= c.active;
        if (!any) break;
        newton_round(b, ctl);
    }
    end_steps(b, all, ctl);
    double ms = ms_since(t0);
    for (auto &c : ctl) c.st.ms_total = ms;
}

// ---------------------------------------------------------------------------
// continuous batching
// ---------------------------------------------------------------------------

struct Request {
    Scene *s;
    ipc_step_req r;
    ipc_ticket t;
};

struct Finished {
    ipc_step_stats st;
    int32_t status;
};

// The engine keeps one list of in-flight steps per class (precision x size:
// scenes of at least IPC_BATCH_LARGE_VERTS vertices form the large class),
// each with a worker thread and a stream of its own, so the Newton rounds of
// small scenes do not wait for the much longer rounds of large ones and the
// classes' launches overlap on the GPU. A worker runs Newton rounds over its
// list; requests submitted meanwhile join the list at the next round
// boundary, finished steps leave it. Admission: the summed device bytes of
// the scenes in flight (all classes) stay within mem_budget (if set); a
// class's list is never left empty while its requests wait.
class Engine {
  public:
    static constexpr int kClasses = 4;
    ipc_runtime rt{};
    int device = 0;
    hipStream_t stream[kClasses] = {};
    bool own_stream[kClasses] = {};

    std::mutex mu;
    std::condition_variable cv_work[kClasses], cv_done;
    std::deque<Request> queue[kClasses];
    std::unordered_map<ipc_ticket, Finished> done;
    std::deque<ipc_ticket> done_order;            // finished tickets, oldest first (consumed ones skipped)
    std::unordered_map<ipc_ticket, int> pending;  // submitted, not yet finished
    ipc_ticket next = 1;
    bool stop = false;
    std::string fatal;  // a device error ends the engine
    std::thread worker[kClasses];

    struct Slot {
        Scene *s;
        ipc_ticket t;
        ipc_step_req req;
        bool fresh;  // admitted this round: begin_step still to run
        Clock::time_point t0;
    };
    struct List {
        Batch b;
        std::vector<Slot> slots;
        std::vector<StepCtl> ctl;
        bool changed = true;
    } lists[kClasses];
    ProfSink prof;
    std::atomic<bool> prof_on{false};

    static int class_of(const Scene &s)
    {
        return (s.prm.precision == IPC_MIXED ? 2 : 0) + (s.h.n >= IPC_BATCH_LARGE_VERTS ? 1 : 0);
    }

    ~Engine()
    {
        {
            std::lock_guard<std::mutex> g(mu);
            stop = true;
        }
        for (auto &c : cv_work) c.notify_all();
        for (auto &w : worker)
            if (w.joinable()) w.join();
        for (int c = 0; c < kClasses; ++c) {
            if (stream[c]) (void)hipStreamSynchronize(stream[c]);
            lists[c].b.stream = nullptr;
        }
        for (int c = 0; c < kClasses; ++c)
            if (own_stream[c] && stream[c]) (void)hipStreamDestroy(stream[c]);
    }

    // caller holds mu
    int64_t in_flight_bytes() const
    {
        int64_t v = 0;
        for (auto &l : lists)
            for (auto &sl : l.slots) v += sl.s->arena.used;
        return v;
    }

    // move waiting requests of class c into its list (caller holds mu)
    void admit(int c)
    {
        int64_t bytes = in_flight_bytes();
        List &l = lists[c];
        while (!queue[c].empty()) {
            Request &q = queue[c].front();
            if (rt.mem_budget > 0 && !l.slots.empty() && bytes + q.s->arena.used > rt.mem_budget) break;
            Slot sl{q.s, q.t, {}, true, Clock::now()};
            sl.req = q.r;
            l.slots.push_back(sl);
            l.ctl.emplace_back();
            l.changed = true;
            bytes += q.s->arena.used;
            queue[c].pop_front();
        }
    }

    // caller holds mu
    void record(ipc_ticket t, const Finished &f)
    {
        done[t] = f;
        done_order.push_back(t);
        pending.erase(t);
    }

    void finish(List &l, const std::vector<uint8_t> &fin)
    {
        std::vector<Slot> keep;
        std::vector<StepCtl> keepc;
        std::lock_guard<std::mutex> g(mu);
        for (size_t i = 0; i < l.slots.size(); ++i) {
            if (!fin[i]) {
                keep.push_back(l.slots[i]);
                keepc.push_back(l.ctl[i]);
                continue;
            }
            Finished f{l.ctl[i].st, l.ctl[i].st.status};
            f.st.ms_total = ms_since(l.slots[i].t0);
            record(l.slots[i].t, f);
            l.slots[i].s->busy = false;
            l.changed = true;
        }
        l.slots.swap(keep);
        l.ctl.swap(keepc);
        cv_done.notify_all();
    }

    void round(List &l, hipStream_t strm)
    {
        size_t ns = l.slots.size();
        if (!ns) return;
        l.b.sink = prof_on.load() ? &prof : nullptr;
        if (l.changed) {
            std::vector<Scene *> sc(ns);
            for (size_t i = 0; i < ns; ++i) sc[i] = l.slots[i].s;
            l.b.bind(sc, strm);
            l.changed = false;
        } else {
            l.b.fail.assign(ns, 0);
        }
        std::vector<uint8_t> fresh(ns, 0);
        bool any_fresh = false;
        for (size_t i = 0; i < ns; ++i)
            if (l.slots[i].fresh) {
                Scene &s = *l.slots[i].s;
                IPC_HIP(hipStreamSynchronize(s.stream));  // earlier work of the scene's own stream
                set_request(s, l.slots[i].req);
                start_ctl(l.ctl[i]);
                l.slots[i].fresh = false;
                fresh[i] = 1;
                any_fresh = true;
            }
        if (any_fresh) begin_steps(l.b, fresh, l.ctl);
        newton_round(l.b, l.ctl);
        std::vector<uint8_t> fin(ns, 0);
        bool any = false;
        for (size_t i = 0; i < ns; ++i)
            if (!l.ctl[i].active) {
                fin[i] = 1;
                any = true;
            }
        if (any) {
            end_steps(l.b, fin, l.ctl);
            finish(l, fin);
        }
    }

    // End every step of class c with IPC_E_DEVICE (its own worker calls this,
    // at a round boundary): after a device error the engine takes no more
    // work; each worker fails its own list and queue, then exits.
    void fail_class(int c, const std::string &msg)
    {
        {
            std::lock_guard<std::mutex> g(mu);
            if (fatal.empty()) fatal = msg;
            Finished f{};
            f.status = IPC_E_DEVICE;
            f.st.status = IPC_E_DEVICE;
            List &l = lists[c];
            for (auto &sl : l.slots) {
                record(sl.t, f);
                sl.s->busy = false;
            }
            l.slots.clear();
            l.ctl.clear();
            l.changed = true;
            for (auto &q : queue[c]) {
                record(q.t, f);
                q.s->busy = false;
            }
            queue[c].clear();
        }
        cv_done.notify_all();
        for (auto &cv : cv_work) cv.notify_all();
    }

    void run(int c)
    {
        if (hipSetDevice(device) != hipSuccess) {
            fail_class(c, "engine could not select its device");
            return;
        }
        List &l = lists[c];
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_work[c].wait(lk, [&] { return stop || !fatal.empty() || !queue[c].empty() || !l.slots.empty(); });
                if (!fatal.empty()) {
                    std::string msg = fatal;
                    lk.unlock();
                    fail_class(c, msg);
                    return;
                }
                if (stop && queue[c].empty() && l.slots.empty()) return;
                admit(c);
            }
            try {
                round(l, stream[c]);
            } catch (const HipError &e) {
                fail_class(c, std::string("HIP error in ") + e.what + ": " + hipGetErrorString(e.e));
                return;
            } catch (...) {
                fail_class(c, "unexpected error in the batch engine");
                return;
            }
        }
    }
};

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

static void set_status_error(int32_t st)
{
    switch (st) {
    case IPC_E_INFEASIBLE: set_error("non-finite or absurd positions in the contact broad phase"); break;
    case IPC_E_OOM: set_error("device allocation refused (allocator or memory budget)"); break;
    case IPC_E_CAPACITY: set_error("contact hash table capacity could not be reached"); break;
    default: break;
    }
}

static bool check_desc(const ipc_scene_desc *d)
{
    if (!d || d->n_verts <= 0 || d->n_tets <= 0 || !d->X || !d->T) return false;
    if (d->n_ind_verts < 0 || d->n_ind_tris < 0) return false;
    if (d->n_ind_verts > 0 && (!d->ind_Y || (d->n_ind_tris > 0 && !d->ind_tris))) return false;
    if (d->n_ind_verts == 0 && d->n_ind_tris > 0) return false;
    if (!(d->dt > 0) || !(d->dhat > 0) || !(d->kappa > 0) || !(d->E > 0) || !(d->rho > 0)) return false;
    if (!(d->nu > -1.0 && d->nu < 0.5)) return false;
    if (!(d->newton_tol >= 0) || !(d->pcg_tol >= 0) || !(d->k_target >= 0)) return false;
    if (d->target_al && !(d->target_al_tol >= 0)) return false;
    if (d->precision != IPC_FP64 && d->precision != IPC_MIXED) return false;
    if (d->pcg_max_iter < 0 || d->max_newton < 0 || d->ccd_max_iter < 0) return false;
    if (!(d->mu_friction >= 0.0) || (d->mu_friction > 0.0 && !(d->eps_v > 0.0))) return false;
    if (d->precond != IPC_PRECOND_MULTILEVEL && d->precond != IPC_PRECOND_JACOBI) return false;
    if (d->barrier_hessian != IPC_BARRIER_PROJECTED && d->barrier_hessian != IPC_BARRIER_GAUSS_NEWTON) return false;
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
    p.precond = d.precond;
    p.barrier_hessian = d.barrier_hessian;
    p.target_al = d.target_al ? 1 : 0;
    p.target_al_tol = d.target_al_tol;
    p.target_al_max = d.target_al_max > 0 ? d.target_al_max : 8;
    return p;
}

// the scene's list of one, bound to its stream
static Batch &solo(Scene &s)
{
    s.solo->bind({&s}, s.stream);
    return *s.solo;
}

static size_t rsize(const Scene &s) { return s.prm.precision == IPC_MIXED ? sizeof(float) : sizeof(double); }

// host FP64 vector -> device array of the scene's real type
static void upload_real(Scene &s, void *dst, const double *src, size_t count)
{
    if (s.prm.precision == IPC_MIXED) {
        std::vector<float> f(src, src + count);
        IPC_HIP(hipMemcpyAsync(dst, f.data(), sizeof(float) * count, hipMemcpyHostToDevice, s.stream));
        IPC_HIP(hipStreamSynchronize(s.stream));
    } else {
        IPC_HIP(hipMemcpyAsync(dst, src, sizeof(double) * count, hipMemcpyHostToDevice, s.stream));
    }
}

static void download_real(Scene &s, double *dst, const void *src, size_t count)
{
    if (s.prm.precision == IPC_MIXED) {
        std::vector<float> f(count);
        IPC_HIP(hipMemcpyAsync(f.data(), src, sizeof(float) * count, hipMemcpyDeviceToHost, s.stream));
        IPC_HIP(hipStreamSynchronize(s.stream));
        for (size_t i = 0; i < count; ++i) dst[i] = f[i];
    } else {
        IPC_HIP(hipMemcpyAsync(dst, src, sizeof(double) * count, hipMemcpyDeviceToHost, s.stream));
        IPC_HIP(hipStreamSynchronize(s.stream));
    }
}

// Test hooks evaluate at a given x without changing the scene's state: x is
// kept in xsave and restored afterwards.
struct HookState {
    Scene &s;
    explicit HookState(Scene &sc, const double *x) : s(sc)
    {
        s.sw_ok = false;  // hooks move x and rebuild the swept list
        size_t b = sizeof(double) * 3 * s.h.n;
        IPC_HIP(hipMemcpyAsync(s.xsave, s.h.x, b, hipMemcpyDeviceToDevice, s.stream));
        if (x) IPC_HIP(hipMemcpyAsync(s.h.x, x, b, hipMemcpyHostToDevice, s.stream));
    }
    ~HookState()
    {
        s.sw_ok = false;
        (void)hipMemcpyAsync(s.h.x, s.xsave, sizeof(double) * 3 * s.h.n, hipMemcpyDeviceToDevice, s.stream);
        (void)hipStreamSynchronize(s.stream);
    }
};

}  // namespace ipcg

using namespace ipcg;

struct ipc_scene : public ipcg::Scene {
};

struct ipc_batch : public ipcg::Engine {
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
        return build_scene(*s, *d);
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
    int64_t rs = d->precision == IPC_MIXED ? 4 : 8;
    int64_t per_vertex = 8 * (3 * 9 + 1) + rs * (3 * 8 + 9) + 4 * 4 + 1;  // nine FP64 3-vectors (the last the target multipliers) and one scalar; the PCG vectors in R
    int64_t per_tet = 4 * 4 + 8 * 10 + rs * (12 + 90) + 4 * 16 + 4 * 4;
    int64_t bell = n * 16 * (9 * rs + 4 + 4);
    int64_t surf = 4 * (int64_t)std::pow((double)d->n_verts, 2.0 / 3.0) + d->n_ind_verts + 2 * d->n_ind_tris;
    int64_t contact = surf * (6 * 8 * 3 + 64 * 4 * 3 + 8 * 16 + 4 * kQueryKeep * kLanesQ) + surf / 4 * (rs * 156 + 4 * 9);
    return n * per_vertex + m * per_tet + bell + contact + (8 << 20);
}

int32_t ipc_step(ipc_scene *s, const ipc_step_req *r, ipc_step_stats *st)
{
    if (!s || !r) return IPC_E_INVALID_ARG;
    bool expect = false;
    if (!s->busy.compare_exchange_strong(expect, true)) return IPC_E_BUSY;
    int32_t rc = guarded([&]() -> int32_t {
        Batch &b = solo(*s);
        std::vector<StepCtl> ctl;
        step_list(b, {r}, ctl);
        if (st) *st = ctl[0].st;
        if (ctl[0].st.status < 0) set_status_error(ctl[0].st.status);
        return ctl[0].st.status;
    });
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
    bool expect = false;
    if (!s->busy.compare_exchange_strong(expect, true)) return IPC_E_BUSY;
    int32_t rc = guarded([&]() -> int32_t {
        hipStream_t strm = stream ? (hipStream_t)stream : s->stream;
        IPC_HIP(hipStreamSynchronize(s->stream));
        if (xyz) {
            double *dst = where == IPC_DEVICE ? xyz : s->ysurf;
            launch_gather_surface(*s, dst, strm);
            if (where == IPC_HOST)
                IPC_HIP(hipMemcpyAsync(xyz, s->ysurf, sizeof(double) * need, hipMemcpyDeviceToHost, strm));
            IPC_HIP(hipStreamSynchronize(strm));
        }
        if (obj_pos) {
            Batch &b = solo(*s);
            activate(b, {1});
            run_lag_and_mean(b);
            b.read_out();
            for (int c = 0; c < 3; ++c) obj_pos[c] = b.h_out[0].obj[c];
        }
        return IPC_OK;
    });
    s->busy = false;
    return rc;
}

int32_t ipc_height_map(const ipc_scene *cs, const ipc_height_map_spec *spec, double *out, int64_t cap,
                       int32_t where, void *stream)
{
    if (!cs || !spec || !out) return IPC_E_INVALID_ARG;
    if (spec->nx <= 0 || spec->ny <= 0 || !(spec->dx > 0.0) || !(spec->dy > 0.0) || !std::isfinite(spec->x0) ||
        !std::isfinite(spec->y0) || !std::isfinite(spec->z_ref)) {
        set_error("invalid height map grid");
        return IPC_E_INVALID_ARG;
    }
    int64_t np = (int64_t)spec->nx * spec->ny;
    if (cap < np) {
        set_error("height map buffer too small");
        return IPC_E_INVALID_ARG;
    }
    if (where != IPC_HOST && where != IPC_DEVICE) return IPC_E_INVALID_ARG;
    ipc_scene *s = const_cast<ipc_scene *>(cs);
    bool expect = false;
    if (!s->busy.compare_exchange_strong(expect, true)) return IPC_E_BUSY;
    int32_t rc = guarded([&]() -> int32_t {
        hipStream_t strm = stream ? (hipStream_t)stream : s->stream;
        IPC_HIP(hipStreamSynchronize(s->stream));
        if (s->hm_cap < np) {
            Staged st(*s);
            auto *nk = st.get<unsigned long long>((size_t)np);
            double *no = st.get<double>((size_t)np);
            st.commit();
            dfree(*s, s->hm_key);
            dfree(*s, s->hm_out);
            s->hm_key = nk;
            s->hm_out = no;
            s->hm_cap = np;
        }
        HeightSpec hs{spec->x0, spec->y0, spec->dx, spec->dy, spec->z_ref, spec->nx, spec->ny};
        double *dst = where == IPC_DEVICE ? out : s->hm_out;
        launch_height_map(*s, hs, s->hm_key, dst, strm);
        if (where == IPC_HOST) IPC_HIP(hipMemcpyAsync(out, s->hm_out, sizeof(double) * np, hipMemcpyDeviceToHost, strm));
        IPC_HIP(hipStreamSynchronize(strm));
        return IPC_OK;
    });
    s->busy = false;
    return rc;
}

// ---------------------------------------------------------------------------
// Height map without device allocation
// ---------------------------------------------------------------------------
// The pixel keys live in one library-owned device array per GPU instead of
// the scene's allocator: callers that may not allocate (HIP graph capture,
// serving loops that forbid hipMalloc) still get the map. Host code never
// passes the array's name to a kernel or a copy: it takes the array's device
// address from hipGetSymbolAddress once per device (with that device
// current) and uses that address only. With IPC_HOST output the keys are
// turned into heights in place and copied out from the same array.
static __device__ __align__(256) unsigned long long scratch[IPC_HEIGHT_MAP_NOALLOC_MAX_PIXELS];

static std::mutex g_scratch_mu;
static std::vector<unsigned long long *> g_scratch_dev;  // per device ordinal, null until looked up

// device address of `scratch` on the current device (looked up on the first
// call made with that device current)
static unsigned long long *scratch_address()
{
    int dev = 0;
    IPC_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((int)g_scratch_dev.size() <= dev) g_scratch_dev.resize(dev + 1, nullptr);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        IPC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) throw HipError(hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
        g_scratch_dev[dev] = static_cast<unsigned long long *>(p);
    }
    return g_scratch_dev[dev];
}

int32_t ipc_height_map_noalloc(const ipc_scene *cs, const ipc_height_map_spec *spec, double *out, int64_t cap,
                               int32_t where, void *stream)
{
    if (!cs || !spec || !out) return IPC_E_INVALID_ARG;
    if (spec->nx <= 0 || spec->ny <= 0 || !(spec->dx > 0.0) || !(spec->dy > 0.0) || !std::isfinite(spec->x0) ||
        !std::isfinite(spec->y0) || !std::isfinite(spec->z_ref)) {
        set_error("invalid height map grid");
        return IPC_E_INVALID_ARG;
    }
    int64_t np = (int64_t)spec->nx * spec->ny;
    if (np > IPC_HEIGHT_MAP_NOALLOC_MAX_PIXELS) {
        set_error("height map grid exceeds IPC_HEIGHT_MAP_NOALLOC_MAX_PIXELS pixels (use ipc_height_map)");
        return IPC_E_INVALID_ARG;
    }
    if (cap < np) {
        set_error("height map buffer too small");
        return IPC_E_INVALID_ARG;
    }
    if (where != IPC_HOST && where != IPC_DEVICE) return IPC_E_INVALID_ARG;
    ipc_scene *s = const_cast<ipc_scene *>(cs);
    bool expect = false;
    if (!s->busy.compare_exchange_strong(expect, true)) return IPC_E_BUSY;
    int32_t rc = guarded([&]() -> int32_t {
        hipStream_t strm = stream ? (hipStream_t)stream : s->stream;
        unsigned long long *key = scratch_address();
        IPC_HIP(hipStreamSynchronize(s->stream));
        HeightSpec hs{spec->x0, spec->y0, spec->dx, spec->dy, spec->z_ref, spec->nx, spec->ny};
        // host output: heights overwrite their own keys (one thread per pixel
        // reads its key, then writes its height to the same 8 bytes)
        double *dst = where == IPC_DEVICE ? out : reinterpret_cast<double *>(key);
        launch_height_map(*s, hs, key, dst, strm);
        if (where == IPC_HOST) IPC_HIP(hipMemcpyAsync(out, key, sizeof(double) * np, hipMemcpyDeviceToHost, strm));
        IPC_HIP(hipStreamSynchronize(strm));
        return IPC_OK;
    });
    s->busy = false;
    return rc;
}

int32_t ipc_surface_topology(const ipc_scene *s, int32_t *tris, int64_t tri_cap, int32_t *n_tris, int32_t *verts,
                             int64_t vert_cap, int32_t *n_surf_verts)
{
    if (!s) return IPC_E_INVALID_ARG;
    if (tris && tri_cap < 3 * (int64_t)s->n_gel_tris) return IPC_E_INVALID_ARG;
    if (verts && vert_cap < (int64_t)s->h_surf_verts.size()) return IPC_E_INVALID_ARG;
    if (n_tris) *n_tris = s->n_gel_tris;
    if (n_surf_verts) *n_surf_verts = (int32_t)s->h_surf_verts.size();
    if (tris) std::memcpy(tris, s->h_tris.data(), sizeof(int32_t) * 3 * s->n_gel_tris);
    if (verts) std::memcpy(verts, s->h_surf_verts.data(), sizeof(int32_t) * s->h_surf_verts.size());
    return IPC_OK;
}

int32_t ipc_reset(ipc_scene *s)
{
    if (!s) return IPC_E_INVALID_ARG;
    bool expect = false;
    if (!s->busy.compare_exchange_strong(expect, true)) return IPC_E_BUSY;
    int32_t rc = guarded([&]() -> int32_t {
        const SceneDev &H = s->h;
        size_t b = sizeof(double) * 3 * H.n;
        for (double *p : {H.x, H.xt, H.xtilde, H.yhat})
            IPC_HIP(hipMemcpyAsync(p, H.X0, b, hipMemcpyDeviceToDevice, s->stream));
        IPC_HIP(hipMemsetAsync(H.v, 0, b, s->stream));
        IPC_HIP(hipStreamSynchronize(s->stream));
        set_pose(*s, s->pose0);
        set_case_pose(*s, kIdentityPose);
        s->step_index = 0;
        s->sw_ok = false;
        s->h.n_fric = 0;
        return IPC_OK;
    });
    s->busy = false;
    return rc;
}

// blob: 4 header words (magic, n, step index, 0), the indenter pose and the
// case pose (12 doubles each), then x and v (3 n doubles each)
static const uint64_t kStateMagic = 0x32657461744370ULL;

int64_t ipc_state_bytes(const ipc_scene *s)
{
    if (!s) return -1;
    return 32 + 24 * 8 + 2 * 3 * (int64_t)s->h.n * 8;
}

int32_t ipc_save_state(const ipc_scene *cs, void *blob, int64_t cap)
{
    if (!cs || !blob || cap < ipc_state_bytes(cs)) return IPC_E_INVALID_ARG;
    ipc_scene *s = const_cast<ipc_scene *>(cs);
    bool expect = false;
    if (!s->busy.compare_exchange_strong(expect, true)) return IPC_E_BUSY;
    int32_t rc = guarded([&]() -> int32_t {
        uint64_t hdr[4] = {kStateMagic, (uint64_t)s->h.n, (uint64_t)s->step_index, 0};
        std::memcpy(blob, hdr, sizeof hdr);
        std::memcpy((char *)blob + 32, s->h.pose, sizeof(double) * 12);
        std::memcpy((char *)blob + 32 + 96, s->h.case_pose, sizeof(double) * 12);
        char *p = (char *)blob + 32 + 192;
        size_t b = sizeof(double) * 3 * s->h.n;
        IPC_HIP(hipMemcpyAsync(p, s->h.x, b, hipMemcpyDeviceToHost, s->stream));
        IPC_HIP(hipMemcpyAsync(p + b, s->h.v, b, hipMemcpyDeviceToHost, s->stream));
        IPC_HIP(hipStreamSynchronize(s->stream));
        return IPC_OK;
    });
    s->busy = false;
    return rc;
}

int32_t ipc_load_state(ipc_scene *s, const void *blob, int64_t bytes)
{
    if (!s || !blob || bytes < ipc_state_bytes(s)) return IPC_E_INVALID_ARG;
    uint64_t hdr[4];
    std::memcpy(hdr, blob, sizeof hdr);
    if (hdr[0] != kStateMagic || hdr[1] != (uint64_t)s->h.n) {
        set_error("state blob does not match this scene");
        return IPC_E_INVALID_ARG;
    }
    bool expect = false;
    if (!s->busy.compare_exchange_strong(expect, true)) return IPC_E_BUSY;
    int32_t rc = guarded([&]() -> int32_t {
        const char *p = (const char *)blob + 32 + 192;
        size_t b = sizeof(double) * 3 * s->h.n;
        IPC_HIP(hipMemcpyAsync(s->h.x, p, b, hipMemcpyHostToDevice, s->stream));
        IPC_HIP(hipMemcpyAsync(s->h.v, p + b, b, hipMemcpyHostToDevice, s->stream));
        IPC_HIP(hipStreamSynchronize(s->stream));
        set_pose(*s, (const double *)((const char *)blob + 32));
        set_case_pose(*s, (const double *)((const char *)blob + 32 + 96));
        s->step_index = (int)hdr[2];
        s->sw_ok = false;
        s->h.n_fric = 0;
        s->dev_dirty = true;
        return IPC_OK;
    });
    s->busy = false;
    return rc;
}

int32_t ipc_scene_sizes(const ipc_scene *s, int32_t *o)
{
    if (!s || !o) return IPC_E_INVALID_ARG;
    const SceneDev &H = s->h;
    o[0] = H.n; o[1] = H.n_gel; o[2] = H.m; o[3] = H.n_pts;
    o[4] = H.n_edges; o[5] = H.n_tris; o[6] = H.n_ind; o[7] = s->n_gel_tris;
    return IPC_OK;
}

int32_t ipc_batch_create(const ipc_runtime *rt, ipc_batch **out)
{
    if (!out) return IPC_E_INVALID_ARG;
    *out = nullptr;
    ipc_batch *b = new (std::nothrow) ipc_batch();
    if (!b) return IPC_E_OOM;
    int32_t rc = guarded([&]() -> int32_t {
        if (rt) b->rt = *rt;
        IPC_HIP(hipGetDevice(&b->device));
        for (int c = 0; c < Engine::kClasses; ++c) {
            if (rt && rt->stream) {
                b->stream[c] = (hipStream_t)rt->stream;
            } else {
                IPC_HIP(hipStreamCreate(&b->stream[c]));
                b->own_stream[c] = true;
            }
        }
        for (int c = 0; c < Engine::kClasses; ++c) b->worker[c] = std::thread([b, c] { b->run(c); });
        return IPC_OK;
    });
    if (rc != IPC_OK) {
        delete b;
        return rc;
    }
    *out = b;
    return IPC_OK;
}

void ipc_batch_destroy(ipc_batch *b) { delete b; }

int32_t ipc_batch_submit(ipc_batch *b, int32_t n, ipc_scene *const *s, const ipc_step_req *r, ipc_ticket *t)
{
    if (!b || n < 0 || (n > 0 && (!s || !r || !t))) return IPC_E_INVALID_ARG;
    for (int i = 0; i < n; ++i) {
        if (!s[i]) return IPC_E_INVALID_ARG;
        for (int j = 0; j < i; ++j)
            if (s[j] == s[i]) return IPC_E_BUSY;
    }
    // claim every scene or none
    for (int i = 0; i < n; ++i) {
        bool expect = false;
        if (!s[i]->busy.compare_exchange_strong(expect, true)) {
            for (int j = 0; j < i; ++j) s[j]->busy = false;
            return IPC_E_BUSY;
        }
    }
    {
        std::lock_guard<std::mutex> g(b->mu);
        if (!b->fatal.empty()) {
            for (int i = 0; i < n; ++i) s[i]->busy = false;
            set_error(b->fatal);
            return IPC_E_DEVICE;
        }
        for (int i = 0; i < n; ++i) {
            t[i] = b->next++;
            b->queue[Engine::class_of(*s[i])].push_back(Request{s[i], r[i], t[i]});
            b->pending[t[i]] = 1;
        }
    }
    for (auto &c : b->cv_work) c.notify_all();
    return IPC_OK;
}

int32_t ipc_batch_poll(ipc_batch *b, ipc_ticket t, ipc_step_stats *st)
{
    if (!b) return IPC_E_INVALID_ARG;
    std::lock_guard<std::mutex> g(b->mu);
    auto it = b->done.find(t);
    if (it == b->done.end()) return b->pending.count(t) ? 0 : IPC_E_INVALID_ARG;
    if (st) *st = it->second.st;
    return 1;
}

int32_t ipc_batch_wait(ipc_batch *b, ipc_ticket t, ipc_step_stats *st)
{
    if (!b) return IPC_E_INVALID_ARG;
    std::unique_lock<std::mutex> lk(b->mu);
    b->cv_done.wait(lk, [&] { return b->done.count(t) || !b->pending.count(t); });
    auto it = b->done.find(t);
    if (it == b->done.end()) return IPC_E_INVALID_ARG;
    if (st) *st = it->second.st;
    int32_t rc = it->second.status;
    b->done.erase(it);
    return rc;
}

int32_t ipc_batch_next(ipc_batch *b, double timeout_ms, ipc_ticket *t, int32_t *status, ipc_step_stats *st)
{
    if (!b || !t) return IPC_E_INVALID_ARG;
    std::unique_lock<std::mutex> lk(b->mu);
    auto ready = [&] {
        while (!b->done_order.empty() && !b->done.count(b->done_order.front())) b->done_order.pop_front();
        return !b->done_order.empty();
    };
    if (!ready()) {
        if (b->pending.empty()) return IPC_E_INVALID_ARG;
        auto pred = [&] { return ready() || b->pending.empty(); };
        if (timeout_ms < 0)
            b->cv_done.wait(lk, pred);
        else
            b->cv_done.wait_for(lk, std::chrono::duration<double, std::milli>(timeout_ms), pred);
        if (!ready()) return b->pending.empty() ? IPC_E_INVALID_ARG : 0;
    }
    ipc_ticket k = b->done_order.front();
    b->done_order.pop_front();
    auto it = b->done.find(k);
    *t = k;
    if (status) *status = it->second.status;
    if (st) *st = it->second.st;
    b->done.erase(it);
    return 1;
}

int32_t ipc_batch_profile(ipc_batch *b, int32_t enable)
{
    if (!b) return IPC_E_INVALID_ARG;
    std::lock_guard<std::mutex> g(b->prof.mu);
    for (auto &a : b->prof.acc) a = ProfAcc{};
    b->prof_on = enable != 0;
    return IPC_OK;
}

int32_t ipc_batch_profile_totals(ipc_batch *b, int32_t kernel, int64_t *launches, double *bytes_total)
{
    if (!b || kernel < 0 || kernel >= kProfKernels) return IPC_E_INVALID_ARG;
    std::lock_guard<std::mutex> g(b->prof.mu);
    if (launches) *launches = b->prof.acc[kernel].launches_all;
    if (bytes_total) *bytes_total = b->prof.acc[kernel].bytes_all;
    return IPC_OK;
}

int32_t ipc_batch_profile_large(ipc_batch *b, int32_t kernel, int64_t *launches, double *ms_total, double *bytes_total)
{
    if (!b || kernel < 0 || kernel >= kProfKernels) return IPC_E_INVALID_ARG;
    std::lock_guard<std::mutex> g(b->prof.mu);
    if (launches) *launches = b->prof.acc[kernel].launches_big;
    if (ms_total) *ms_total = b->prof.acc[kernel].ms_big;
    if (bytes_total) *bytes_total = b->prof.acc[kernel].bytes_big;
    return IPC_OK;
}

int32_t ipc_batch_profile_read(ipc_batch *b, int32_t kernel, int64_t *launches, double *ms_total, double *bytes_total)
{
    if (!b || kernel < 0 || kernel >= kProfKernels) return IPC_E_INVALID_ARG;
    std::lock_guard<std::mutex> g(b->prof.mu);
    if (launches) *launches = b->prof.acc[kernel].launches;
    if (ms_total) *ms_total = b->prof.acc[kernel].ms;
    if (bytes_total) *bytes_total = b->prof.acc[kernel].bytes;
    return IPC_OK;
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

#define IPC_HOOK_BEGIN(s)                                            \
    bool _expect = false;                                            \
    if (!(s)->busy.compare_exchange_strong(_expect, true)) return IPC_E_BUSY; \
    int32_t _rc = guarded([&]() -> int32_t {
#define IPC_HOOK_END(s) \
    });                 \
    (s)->busy = false;  \
    return _rc;

int32_t ipcx_begin_step(ipc_scene *s, const ipc_step_req *r)
{
    if (!s || !r) return IPC_E_INVALID_ARG;
    IPC_HOOK_BEGIN(s)
        Batch &b = solo(*s);
        set_request(*s, *r);
        std::vector<StepCtl> ctl(1);
        start_ctl(ctl[0]);
        std::vector<uint8_t> on(1, 1);
        begin_steps(b, on, ctl);
        IPC_HIP(hipStreamSynchronize(s->stream));
        if (ctl[0].failed) {
            set_status_error(ctl[0].status);
            return ctl[0].status;
        }
        return IPC_OK;
    IPC_HOOK_END(s)
}

// one Newton iteration from x_in; returns 0 stepped, 1 converged, 2 stalled
// (or an error status)
int32_t ipcx_newton_iterate(ipc_scene *s, const double *x_in, double *x_out, ipc_step_stats *st)
{
    if (!s || !x_in || !x_out) return IPC_E_INVALID_ARG;
    IPC_HOOK_BEGIN(s)
        HookState hs(*s, x_in);
        Batch &b = solo(*s);
        std::vector<StepCtl> ctl(1);
        start_ctl(ctl[0]);
        newton_round(b, ctl);
        StepCtl &c = ctl[0];
        IPC_HIP(hipMemcpyAsync(x_out, s->h.x, sizeof(double) * 3 * s->h.n, hipMemcpyDeviceToHost, s->stream));
        IPC_HIP(hipStreamSynchronize(s->stream));
        int32_t res = c.failed ? c.status : (c.stepped ? 0 : (c.status == IPC_W_LS_STALL ? 2 : 1));
        if (c.failed) set_status_error(c.status);
        if (st) {
            *st = c.st;
            st->status = res;
            if (!c.stepped) {
                st->alpha = 0.0;
                if (res == 1) st->energy = NAN;
            }
        }
        return res;
    IPC_HOOK_END(s)
}

int32_t ipcx_candidates(ipc_scene *s, const double *x, const double *p, int32_t *out, int64_t cap, int64_t *count)
{
    if (!s || !x) return IPC_E_INVALID_ARG;
    IPC_HOOK_BEGIN(s)
        HookState hs(*s, x);
        if (p) upload_real(*s, s->h.sol, p, 3 * (size_t)s->h.n);
        Batch &b = solo(*s);
        activate(b, {1});
        int which = p ? 1 : 0;
        run_broad_phase(b, which);
        if (b.fail[0]) {
            set_status_error(b.fail[0]);
            return b.fail[0];
        }
        IPC_HIP(hipStreamSynchronize(s->stream));
        int64_t nc = which ? b.h_out[0].n_sw : b.h_out[0].n_cand;
        const int32_t *buf = which ? s->h.cand_sw : s->h.cand;
        int64_t bcap = which ? s->h.sw_cap : s->h.cand_cap;
        if (count) *count = nc;
        if (out && cap > 0) {
            int64_t w = std::min(cap, nc);
            std::vector<int32_t> h(3 * (size_t)std::max<int64_t>(w, 1));
            for (int c = 0; c < 3; ++c)
                IPC_HIP(hipMemcpyAsync(h.data() + (size_t)c * w, buf + (size_t)c * bcap, sizeof(int32_t) * w,
                                       hipMemcpyDeviceToHost, s->stream));
            IPC_HIP(hipStreamSynchronize(s->stream));
            for (int64_t i = 0; i < w; ++i)
                for (int c = 0; c < 3; ++c) out[3 * i + c] = h[(size_t)c * w + i];
        }
        return IPC_OK;
    IPC_HOOK_END(s)
}

int32_t ipcx_primitives(const ipc_scene *s, int32_t *points, int32_t *edges, int32_t *tris)
{
    if (!s) return IPC_E_INVALID_ARG;
    if (points) std::memcpy(points, s->h_pts.data(), sizeof(int32_t) * s->h_pts.size());
    if (edges) std::memcpy(edges, s->h_edges.data(), sizeof(int32_t) * s->h_edges.size());
    if (tris) std::memcpy(tris, s->h_tris.data(), sizeof(int32_t) * s->h_tris.size());
    return IPC_OK;
}

// assemble at the hook's x; returns a failure status or IPC_OK
static int32_t hook_assemble(Scene &s)
{
    Batch &b = solo(s);
    std::vector<StepCtl> ctl(1);
    start_ctl(ctl[0]);
    std::vector<uint8_t> on(1, 1);
    double ms[8] = {0};
    assemble_round(b, ctl, on, ms);
    if (ctl[0].failed) {
        set_status_error(ctl[0].status);
        return ctl[0].status;
    }
    return IPC_OK;
}

int32_t ipcx_gradient(ipc_scene *s, const double *x, double *g)
{
    if (!s || !x || !g) return IPC_E_INVALID_ARG;
    IPC_HOOK_BEGIN(s)
        HookState hs(*s, x);
        int32_t r = hook_assemble(*s);
        if (r != IPC_OK) return r;
        download_real(*s, g, s->h.grad, 3 * (size_t)s->h.n);
        return IPC_OK;
    IPC_HOOK_END(s)
}

int32_t ipcx_hess_apply(ipc_scene *s, const double *x, const double *v, double *y)
{
    if (!s || !x || !v || !y) return IPC_E_INVALID_ARG;
    IPC_HOOK_BEGIN(s)
        HookState hs(*s, x);
        int32_t r = hook_assemble(*s);
        if (r != IPC_OK) return r;
        upload_real(*s, s->h.dB, v, 3 * (size_t)s->h.n);
        Batch &b = solo(*s);
        launch_hess_apply(b);
        download_real(*s, y, s->h.q, 3 * (size_t)s->h.n);
        return IPC_OK;
    IPC_HOOK_END(s)
}

int32_t ipcx_assemble_elastic(ipc_scene *s, const double *x, double *g, const double *v, double *y)
{
    if (!s || !x || !g || (v != nullptr) != (y != nullptr)) return IPC_E_INVALID_ARG;
    IPC_HOOK_BEGIN(s)
        HookState hs(*s, x);
        Batch &b = solo(*s);
        activate(b, {1});
        // no pair enters the lists: the scene's barrier and friction pair
        // counts read zero for this call
        const int32_t nf = s->h.n_fric;
        s->h.n_fric = 0;
        s->dev_dirty = true;
        b.upload_views();
        SceneOut &o = b.h_out[0];
        o.n_cand = o.n_act = o.n_pair = o.n_heavy = 0;
        IPC_HIP(hipMemcpyAsync(b.d_out, &o, sizeof(SceneOut), hipMemcpyHostToDevice, b.stream));
        launch_contact_incidence(b);
        launch_elastic_elements(b);
        launch_assemble(b);
        if (v) {
            upload_real(*s, s->h.dB, v, 3 * (size_t)s->h.n);
            launch_hess_apply(b);
        }
        s->h.n_fric = nf;
        s->dev_dirty = true;
        b.upload_views();
        download_real(*s, g, s->h.grad, 3 * (size_t)s->h.n);
        if (v) download_real(*s, y, s->h.q, 3 * (size_t)s->h.n);
        return IPC_OK;
    IPC_HOOK_END(s)
}

int32_t ipcx_barrier(ipc_scene *s, const double *x, int64_t cap, int32_t *kind, int32_t *v4, double *g12,
                     double *H144, int64_t *count)
{
    if (!s || !x || cap < 0) return IPC_E_INVALID_ARG;
    IPC_HOOK_BEGIN(s)
        HookState hs(*s, x);
        int32_t r = hook_assemble(*s);
        if (r != IPC_OK) return r;
        Batch &b = solo(*s);
        const int64_t n = b.h_out[0].n_act, w = std::min(cap, n), pc = s->h.act_cap;
        if (count) *count = n;
        if (w > 0) {
            std::vector<int32_t> idx(w), type(std::max<int64_t>(b.h_out[0].n_cand, 1)), vv(4 * (size_t)pc);
            std::vector<double> gg(12 * (size_t)pc), hh(144 * (size_t)pc);
            IPC_HIP(hipMemcpyAsync(idx.data(), s->h.act_idx, sizeof(int32_t) * w, hipMemcpyDeviceToHost, s->stream));
            IPC_HIP(hipMemcpyAsync(type.data(), s->h.cand, sizeof(int32_t) * type.size(), hipMemcpyDeviceToHost,
                                   s->stream));
            IPC_HIP(hipMemcpyAsync(vv.data(), s->h.act_v, sizeof(int32_t) * vv.size(), hipMemcpyDeviceToHost,
                                   s->stream));
            download_real(*s, gg.data(), s->h.act_g, gg.size());
            download_real(*s, hh.data(), s->h.act_H, hh.size());
            // component-major (component * act_cap + pair) to pair-major
            for (int64_t k = 0; k < w; ++k) {
                if (kind) kind[k] = type[idx[k]];
                if (v4)
                    for (int a = 0; a < 4; ++a) v4[4 * k + a] = vv[(size_t)a * pc + k];
                if (g12)
                    for (int e = 0; e < 12; ++e) g12[12 * k + e] = gg[(size_t)e * pc + k];
                if (H144)
                    for (int e = 0; e < 144; ++e) H144[144 * k + e] = hh[(size_t)e * pc + k];
            }
        }
        return IPC_OK;
    IPC_HOOK_END(s)
}

int32_t ipcx_pcg(ipc_scene *s, const double *x, double *p, int32_t *iters)
{
    if (!s || !x || !p) return IPC_E_INVALID_ARG;
    IPC_HOOK_BEGIN(s)
        HookState hs(*s, x);
        int32_t r = hook_assemble(*s);
        if (r != IPC_OK) return r;
        Batch &b = solo(*s);
        std::vector<int> it, capped;
        run_pcg(b, it, capped);
        if (iters) *iters = capped[0] ? -it[0] : it[0];
        download_real(*s, p, s->h.sol, 3 * (size_t)s->h.n);
        return IPC_OK;
    IPC_HOOK_END(s)
}

int32_t ipcx_energy(ipc_scene *s, const double *x, double *E)
{
    if (!s || !x || !E) return IPC_E_INVALID_ARG;
    IPC_HOOK_BEGIN(s)
        HookState hs(*s, x);
        // the energy runs over the swept list; with p = 0 it is the static list at x
        IPC_HIP(hipMemsetAsync(s->h.sol, 0, 3 * (size_t)s->h.n * rsize(*s), s->stream));
        Batch &b = solo(*s);
        activate(b, {1});
        run_broad_phase(b, 1);
        if (b.fail[0]) {
            set_status_error(b.fail[0]);
            return b.fail[0];
        }
        run_energy(b, false);
        b.read_out();
        *E = b.h_out[0].infeasible ? INFINITY : b.h_out[0].energy;
        return IPC_OK;
    IPC_HOOK_END(s)
}

int32_t ipcx_ccd(ipc_scene *s, const double *x, const double *p, double *alpha)
{
    if (!s || !x || !p || !alpha) return IPC_E_INVALID_ARG;
    IPC_HOOK_BEGIN(s)
        HookState hs(*s, x);
        upload_real(*s, s->h.sol, p, 3 * (size_t)s->h.n);
        Batch &b = solo(*s);
        activate(b, {1});
        run_broad_phase(b, 1);
        if (b.fail[0]) {
            set_status_error(b.fail[0]);
            return b.fail[0];
        }
        run_ccd(b);
        b.read_out();
        *alpha = std::min(1.0, b.h_out[0].alpha_ccd);
        return IPC_OK;
    IPC_HOOK_END(s)
}

int32_t ipcx_profile(ipc_scene *s, int32_t enable)
{
    if (!s) return IPC_E_INVALID_ARG;
    IPC_HOOK_BEGIN(s)
        IPC_HIP(hipStreamSynchronize(s->stream));
        s->solo->prof_collect();
        s->prof = enable != 0;
        for (auto &a : s->prof_acc) a = ProfAcc{};
        return IPC_OK;
    IPC_HOOK_END(s)
}

int32_t ipcx_profile_read(const ipc_scene *s, int32_t kernel, int64_t *launches, double *ms_total)
{
    if (!s || kernel < 0 || kernel >= kProfKernels) return IPC_E_INVALID_ARG;
    if (launches) *launches = s->prof_acc[kernel].launches;
    if (ms_total) *ms_total = s->prof_acc[kernel].ms;
    return IPC_OK;
}

int32_t ipcx_profile_totals(const ipc_scene *s, int32_t kernel, int64_t *launches, double *bytes_total)
{
    if (!s || kernel < 0 || kernel >= kProfKernels) return IPC_E_INVALID_ARG;
    if (launches) *launches = s->prof_acc[kernel].launches_all;
    if (bytes_total) *bytes_total = s->prof_acc[kernel].bytes_all;
    return IPC_OK;
}

int32_t ipcx_profile_bytes(const ipc_scene *s, int32_t kernel, double *bytes_total)
{
    if (!s || !bytes_total || kernel < 0 || kernel >= kProfKernels) return IPC_E_INVALID_ARG;
    *bytes_total = s->prof_acc[kernel].bytes;
    return IPC_OK;
}

int32_t ipcx_matrix_info(const ipc_scene *s, int64_t *out)
{
    if (!s || !out) return IPC_E_INVALID_ARG;
    out[0] = s->nnzb;
    out[1] = (int64_t)s->h.n_slots * kSlice;
    out[2] = s->h.n;
    out[3] = s->last.n_act;
    out[4] = s->h.m;
    out[5] = s->last.n_cand;
    out[6] = s->last.n_sw;
    out[7] = s->n_gather;
    return IPC_OK;
}

int32_t ipcx_tuning(const ipc_scene *s, double *out)
{
    if (!s || !out) return IPC_E_INVALID_ARG;
    out[0] = (double)s->tune.spmv_one_lane_rows;
    out[1] = s->tune.mas_target;
    out[2] = s->tune.pcg_first_chunk;
    out[3] = s->tune.pcg_later_chunk;
    out[4] = s->tune.from_file;
    out[5] = s->tune.pcg_list_quantile;
    return IPC_OK;
}

int32_t ipcx_tuning_for(int32_t n_verts, double *out)
{
    if (!out || n_verts < 0) return IPC_E_INVALID_ARG;
    return guarded([&]() -> int32_t {
        Tuning t = tuning_for(n_verts);
        out[0] = (double)t.spmv_one_lane_rows;
        out[1] = t.mas_target;
        out[2] = t.pcg_first_chunk;
        out[3] = t.pcg_later_chunk;
        out[4] = t.from_file;
        out[5] = t.pcg_list_quantile;
        return IPC_OK;
    });
}

int32_t ipcx_struct_sizes(int64_t *out)
{
    if (!out) return IPC_E_INVALID_ARG;
    out[0] = (int64_t)sizeof(ipc_scene_desc);
    out[1] = (int64_t)sizeof(ipc_runtime);
    out[2] = (int64_t)sizeof(ipc_step_req);
    out[3] = (int64_t)sizeof(ipc_step_stats);
    out[4] = (int64_t)sizeof(ipc_height_map_spec);
    return IPC_OK;
}

int32_t ipcx_precond_info(const ipc_scene *s, int64_t *out)
{
    if (!s || !out) return IPC_E_INVALID_ARG;
    for (int k = 0; k < 8; ++k) out[k] = 0;
    const SceneDev &h = s->h;
    out[0] = h.mas_levels;
    out[1] = h.mas_ng;
    for (int l = 0; l < h.mas_levels; ++l) out[2 + l] = h.mas_n[l];
    out[5] = s->mas_max_members;
    out[6] = s->mas_max_aggs;
    out[7] = h.mas_nf;
    return IPC_OK;
}

int32_t ipcx_set_state(ipc_scene *s, const double *x, const double *v)
{
    if (!s) return IPC_E_INVALID_ARG;
    IPC_HOOK_BEGIN(s)
        size_t b = sizeof(double) * 3 * s->h.n;
        if (x) IPC_HIP(hipMemcpyAsync(s->h.x, x, b, hipMemcpyHostToDevice, s->stream));
        if (v) IPC_HIP(hipMemcpyAsync(s->h.v, v, b, hipMemcpyHostToDevice, s->stream));
        IPC_HIP(hipStreamSynchronize(s->stream));
        if (x) s->sw_ok = false;
        return IPC_OK;
    IPC_HOOK_END(s)
}

int32_t ipcx_get_state(const ipc_scene *cs, double *x, double *v)
{
    if (!cs) return IPC_E_INVALID_ARG;
    ipc_scene *s = const_cast<ipc_scene *>(cs);
    IPC_HOOK_BEGIN(s)
        size_t b = sizeof(double) * 3 * s->h.n;
        if (x) IPC_HIP(hipMemcpyAsync(x, s->h.x, b, hipMemcpyDeviceToHost, s->stream));
        if (v) IPC_HIP(hipMemcpyAsync(v, s->h.v, b, hipMemcpyDeviceToHost, s->stream));
        IPC_HIP(hipStreamSynchronize(s->stream));
        return IPC_OK;
    IPC_HOOK_END(s)
}

}  // extern "C"
