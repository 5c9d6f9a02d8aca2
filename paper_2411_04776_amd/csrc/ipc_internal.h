// ipc_internal.h -- internal types of the MI355X IPC gel-pad step library.
//
// Every kernel runs over a *list of scenes*: a launch carries an array of
// per-scene device views (SceneDev) and a block-offset table that gives each
// scene a contiguous range of blocks sized from that scene alone. One scene
// stepping on its own is a list of one; the batched form puts many scenes in
// the same launches. Because a scene's blocks, its per-block partials and its
// reduction order depend only on that scene, its results are bitwise the
// same alone and in any mix.
//
// Layout in HBM (one scene):
//   vertex vectors (x, v, gradient, PCG vectors): interleaved xyz, 3*n values;
//   per-tet data (indices, Dm^-1, volume, element gradient/Hessian blocks):
//     structure of arrays, one array per component (coalesced per wavefront);
//   the elastic matrix: blocked sliced ELL with 3x3 blocks, a slice = 64 rows
//     = one wavefront, padded to its longest row, stored component-major in
//     the slice (value[(slot*9+c)*64 + lane]); slot 0 of a row is its diagonal;
//   contact pairs: structure of arrays over active pairs (4 vertex ids, 12
//     gradient and 144 Hessian components); in SpMV each pair forms its own
//     H_p d_p and the rows gather those through incidence lists sorted by row
//     and pair index (no float atomics anywhere).
// In the mixed form the element Hessians and gradients, matrix values,
// preconditioner, assembled gradient and PCG vectors are FP32 (dot products
// accumulate in FP64); positions, Dm^-1, distances, CCD and energies stay FP64.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <atomic>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "ipc.h"

namespace ipcg {

constexpr int kWave = 64;         // wavefront width on gfx950
constexpr int kXcds = 8;          // accelerator complex dies of an MI355X, each with its own L2
constexpr int kXcdChunk = 64;     // consecutive logical blocks that share an XCD
constexpr int kSlice = 64;        // rows per BELL slice (one wavefront)
constexpr int kBlock = 256;       // threads per block for streaming kernels
constexpr int kSpmvStreams = 2;   // partial sums per SpMV row (slots k, k + 2, ...), added in stream order
constexpr int kRowsPerBlock = 64; // matrix rows per SpMV block (PCG A), a thread or two lanes each
constexpr int kPairsPerBlock = 64;  // contact pairs per pair block of PCG A
constexpr int64_t kSpmvOneLaneRows = 65536;  // lists with at least this many rows: one thread per row
constexpr int kScanTile = 1024;   // elements per scan tile
constexpr int kHeavyRow = 24;     // incidence rows longer than this get a block of their own
constexpr int kQueryKeep = 4;     // pairs a query lane keeps from the count pass for the fill pass
constexpr int kLanesQ = 8;        // broad-phase lanes per query primitive (they split its buckets' entries)
constexpr int kMasLevels = 3;     // aggregate levels of the multilevel preconditioner
constexpr int kMasCapM = 256;     // members of a preconditioner group (one block, held in LDS)
constexpr int kMasCapA = 256;     // aggregates of all levels in a group
constexpr int kMasTarget = 256;   // groups are packed with top-level aggregates up to this many members

// kernels timed by the optional profiler
enum ProfKernel {
    kProfPcgA = 0,        // SpMV + fused direction update (PCG A)
    kProfPcgB = 1,        // PCG vector update + preconditioner (PCG B)
    kProfElastic = 2,     // Neo-Hookean element kernel
    kProfAssemble = 3,    // gradient + matrix gather
    kProfBroad = 4,       // boxes, hash, queries
    kProfBarrier = 5,     // narrow phase + barrier + incidence
    kProfEnergy = 6,      // line-search energy
    kProfCcd = 7,         // additive CCD
    kProfKernels = 8
};

struct PcgState {
    int32_t done;
    int32_t iters;
    double stop;
    double rzv[2];  // r.z of the previous iterations by parity, written once by the SpMV kernel's block 0
};

// Per-scene values produced on the device and read back once per phase for
// the whole list (one copy for all scenes).
struct SceneOut {
    int32_t n_cand;       // static candidates
    int32_t n_sw;         // swept candidates
    int32_t n_act;        // active pairs
    int32_t ent_tri, ent_edge;  // hash entries needed
    int32_t bad;          // non-finite positions seen by the broad phase
    int32_t infeasible;   // energy: a tet with J <= 0 or a pair with d <= 0
    int32_t pcg_done, pcg_iters;
    int32_t n_heavy;      // incidence rows with more than kHeavyRow entries
    int32_t n_pair;       // pairs in the active arrays: n_act barrier pairs, then the friction pairs
    int32_t pcg_early;    // PCG launches past this iteration check the done flag before any load
                          // (7/8 of the slot's last solve, written by the device; a heuristic only:
                          // a finished solve's launches write nothing either way)
    double pinf;          // max |p| over free DOFs
    double alpha_ccd;
    double energy;
    double lag;           // max indenter target lag
    double obj[3];        // mean of gel vertices
};

// Device view of one scene: sizes, parameters and pointers. Pointers to
// precision-dependent arrays are void*; kernels templated on the real type R
// cast them.
struct SceneDev {
    int n, n_gel, n_ind, m, n_pts, n_edges, n_tris, n_slices, n_slots, n_surf;
    int n_gel_tris, n_gel_edges;  // surface primitives of the gel come first (then the indenter's)
    int self_contact, ccd_max_iter, precision, nb_vert, nb_rows, pcg_maxit;
    double mu, lam, h, inv_h2, dhat, kappa, k_target, rho, grav[3], ccd_s, pcg_tol2;
    double mu_fric, eps_fric;  // friction coefficient, smoothing length eps_v h
    int barrier_gn;            // 1: Gauss-Newton pair Hessians kappa w b'' grad d grad d^T
    int target_al;             // 1: indenter target terms carry the multipliers al_lam
    double *al_lam;            // augmented-Lagrangian multipliers, 3 per vertex (indenter vertices)
    uint8_t *attached;         // per gel vertex: pulled to case_pose X0 by k_target (NULL: none)
    double case_pose[12];
    double pose[12];
    double alpha;      // line-search trial step
    // state (FP64)
    double *x, *v, *xt, *xtilde, *yhat, *X0, *Yloc, *xtrial, *mass;
    uint8_t *fixed;
    // tets
    int32_t *tv;
    double *Bm, *vol;
    void *eg, *eH;
    int32_t *vt_ptr, *vt_src;
    // elastic matrix
    int32_t *slice_ptr, *bcol, *g_ptr, *g_src;
    void *bval, *Minv, *grad;
    // surface primitives and broad phase
    int32_t *pts, *ev, *trv, *surf_verts;
    double *edge_rest_sq;
    double *pbox, *ebox, *tbox, *cell_h;
    int32_t *ht_count[2], *ht_start[2];
    int4 *ht_entries[2];
    int32_t ht_bits[2], ht_cap[2];
    int32_t *q_count, *q_off;      // per query primitive (points, then edges): pair counts, offsets
    int32_t *q_lane;               // kLanesQ per query primitive: each lane's pair count
    int32_t *q_keep;               // kLanesQ * kQueryKeep per query primitive: each lane's first pairs (b)
    // candidates: static list and swept list (SoA type, a, b with stride cap)
    int32_t *cand, *cand_sw;
    int64_t cand_cap, sw_cap;
    int64_t n_sw_prev;             // length of the swept list kept from the previous iteration
    double *cand_d;
    int32_t *act_flag, *act_off;   // active flags of the static list and their exclusive scan
    int32_t *sw_flag, *sw_off;     // swept pairs whose boxes at x overlap, and their scan
    int32_t *pt_idx;               // surface point index of a vertex (-1: not on the surface)
    // active pairs
    int32_t *act_idx, *act_v;
    void *act_g, *act_H, *act_y;   // act_y: per-pair products H_p d_p (PCG), 12 per pair, pair-major
    int64_t act_cap;
    double *pcg_pair;              // per-block d.(H_c d) partials of the pair blocks
    // lagged friction set of the step (pairs active at x^t): 4 vertex ids,
    // closest-point coefficients, unit normal, normal-force magnitude
    int32_t *fric_v;
    double *fric_c, *fric_nrm, *fric_lam;
    int64_t fric_cap;
    int32_t n_fric;
    int32_t *c_ptr, *c_cnt, *c_list, *c_row, *c_tmp;
    int32_t *hflag, *heavy_idx, *heavy_rows;  // heavy incidence rows: flag, index (scan), list
    double *hdiag;                            // 9 contact diagonal sums per heavy row
    // multilevel additive preconditioner: nested aggregates of the free gel
    // vertices (level 0 = cells of twice the mean edge, doubling per level);
    // aggregates are numbered level-major (global id = mas_off[l] + local id).
    // The members (free gel vertices) are ordered so that every aggregate of
    // every level is a contiguous range of positions; a group is a run of
    // top-level aggregates handled by one block.
    int mas_levels;                  // 0: block Jacobi only
    int mas_n[kMasLevels];           // aggregates per level
    int mas_off[kMasLevels + 1];
    int mas_nf;                      // members
    int mas_ng;                      // groups
    int mas_nd0;                     // diagonal blocks of level 0 (a wavefront per aggregate)
    int32_t *mas_mem;                // vertex of member position k
    int32_t *mas_manc;               // level-local aggregate of member position k: mas_manc[l * nf + k]
    int32_t *mas_mb, *mas_me;        // per global aggregate: member positions (level 0) or child ids (level l-1)
    int32_t *mas_gofs;               // (levels + 1) rows of ng + 1: member offsets, then per-level aggregate offsets
    int32_t *mas_dptr, *mas_dsrc;    // BELL entries first shared at aggregate g's level, per global aggregate
    double *mas_ex;                  // 9 per aggregate: those entries' sum, then the aggregate's whole block
    void *mas_dinv;                  // 9 per aggregate (R)
    int mas_nother;                  // vertices outside the aggregates (fixed gel, indenter)
    int32_t *mas_other;              // their ids, ascending
    int32_t *mas_vpos;               // member position of each vertex, -1 outside
    int pcg_nvp;                     // PCG update blocks before the heavy rows (and their r.z partials)
    // PCG
    void *r, *z, *dA, *dB, *q, *sol;
    double *pcg_part;
    PcgState *pcg;
    // reduction scratch (doubles) and scan scratch (ints)
    double *red;
    int32_t *scan_tmp;
    int64_t red_len, scan_len;
};

// A launch over a list of scenes: block b belongs to scene s when
// blk_off[s] <= b < blk_off[s+1].
struct Launch {
    SceneDev *const *sc;
    const int32_t *blk_off;
    SceneOut *out;
    int ns;
};

// The logical block of this workgroup. The hardware dispatches workgroup w
// to XCD w % kXcds (each XCD has its own L2); within every run of
// kXcds * kXcdChunk workgroups the logical order is remapped so each XCD gets
// kXcdChunk consecutive blocks: neighbouring blocks of a scene, whose rows
// gather each other's vector entries, share an L2, while the runs keep heavy
// and light blocks (group blocks first, plain vertex blocks after them)
// spread over all XCDs. The last partial run keeps the identity. A bijection
// for any grid size; results do not depend on it (every logical block does
// the same work wherever it runs).
__device__ __forceinline__ int xcd_block()
{
    constexpr int run = kXcds * kXcdChunk;
    const int w = (int)blockIdx.x;
    const int full = ((int)gridDim.x / run) * run;
    if (w >= full) return w;
    const int base = w - w % run, r = w % run;
    return base + (r % kXcds) * kXcdChunk + r / kXcds;
}

__device__ __forceinline__ int scene_of_block(const Launch &L, int &local)
{
    int lo = 0, hi = L.ns;
    int b = xcd_block();
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (L.blk_off[mid] <= b) lo = mid; else hi = mid;
    }
    local = b - L.blk_off[lo];
    return lo;
}
__device__ __forceinline__ int blocks_of(const Launch &L, int s) { return L.blk_off[s + 1] - L.blk_off[s]; }

// Launch and grouping choices picked per size class by the library's
// autotuner (paper_2411_04776_amd/autotune.py) and read from its JSON file
// when a scene is created; the defaults below apply without a file.
struct Tuning {
    int64_t spmv_one_lane_rows = kSpmvOneLaneRows;  // lists with this many rows or more: one thread per SpMV row
    int mas_target = kMasTarget;                    // preconditioner group packing target (members, <= kMasCapM)
    double pcg_first_chunk = 0.875;                 // first PCG chunk: this fraction of the previous solve's count
    double pcg_later_chunk = 0.25;                  // later chunks: this fraction of the remaining count (at least 8)
    double pcg_list_quantile = 0.25;                // in a list: the quantile of the scenes' remaining counts used
    int from_file = 0;                              // 1 if read from a tuning file
};
Tuning tuning_for(int n_verts);  // the tuning file's entry for a scene of n_verts vertices

struct Params {
    double E, nu, rho, mu, lam;
    double dt, dhat, kappa, k_target;
    double newton_tol, pcg_tol;
    double grav[3];
    double mu_fric, eps_v;
    double ccd_s, ls_min_ratio;
    int self_contact, precision, max_newton, pcg_max_iter, ccd_max_iter, precond, barrier_hessian;
    int target_al, target_al_max;  // augmented-Lagrangian indenter targets: on, updates per step
    double target_al_tol;          // lag (m) above which a converged iterate updates the multipliers
};

// Device allocation through the runtime's callbacks (PyTorch's caching
// allocator from Python) or hipMalloc.
struct DeviceArena {
    ipc_runtime rt{};
    int64_t used = 0;
    void *alloc(size_t bytes);
    void release(void *p, size_t bytes);
};

class Batch;

// timed launches of one kernel class: count, summed event milliseconds and
// summed algorithmic bytes (counted for the PCG SpMV)
struct ProfAcc {
    int64_t launches = 0;
    double ms = 0.0;
    double bytes = 0.0;
    int64_t launches_all = 0;  // every launch of the class while profiling (PCG classes)
    double bytes_all = 0.0;    // and their algorithmic bytes
    int64_t launches_big = 0;  // timed PCG launches of iterations whose SpMV moves >= kProfBigBytes
    double ms_big = 0.0, bytes_big = 0.0;
};

// PCG iterations whose SpMV launch's algorithmic bytes exceed the 256 MiB
// Infinity Cache: their traffic cannot be served from it
constexpr double kProfBigBytes = 256.0 * 1024.0 * 1024.0;

// accumulators shared by the lists of a batch engine
struct ProfSink {
    std::mutex mu;
    ProfAcc acc[kProfKernels];
};

class Scene {
  public:
    Params prm{};
    hipStream_t stream = nullptr;
    DeviceArena arena;
    std::vector<std::pair<void *, size_t>> owned;

    SceneDev h{};          // host mirror of the device view
    SceneDev *dev = nullptr;
    bool dev_dirty = true; // h changed since the last upload

    int64_t nnzb = 0, n_gather = 0;
    int n_gel_tris = 0;
    int mas_max_members = 0, mas_max_aggs = 0;  // largest preconditioner group
    unsigned long long *hm_key = nullptr;       // height-map scratch (hm_cap keys)
    int64_t hm_cap = 0;
    double *hm_out = nullptr;                   // staging of a host-bound height map (hm_cap doubles)
    double *xsave = nullptr;   // test hooks: the state x kept across a hook call
    double *ysurf = nullptr;   // staging for surface read-back to the host
    std::unique_ptr<Batch> solo;  // the list of one used by ipc_step and the hooks
    std::vector<int32_t> h_pts, h_edges, h_tris, h_surf_verts;
    std::vector<double> h_Yloc;
    double pose0[12] = {};
    int step_index = 0;
    std::atomic<bool> busy{false};  // a step, read or hook holds the scene
    int last_pcg_iters = 0;
    Tuning tune{};         // launch and grouping choices of the scene's size class
    bool sw_ok = false;    // the swept list holds every static pair at the current x
    int64_t sw_n = 0;      // its length
    SceneOut last{};       // last values read back

    // optional per-kernel timing with HIP events
    bool prof = false;
    ProfAcc prof_acc[kProfKernels];

    ~Scene();
};

// errors
struct HipError {
    hipError_t e;
    const char *what;
    HipError(hipError_t e_, const char *w) : e(e_), what(w) {}
};
struct OomError {};
struct CapacityError {};
struct InfeasibleError {};

#define IPC_HIP(call)                                                   \
    do {                                                                \
        hipError_t _e = (call);                                         \
        if (_e != hipSuccess) throw ipcg::HipError(_e, #call);          \
    } while (0)

void set_error(const std::string &msg);

void *dalloc_bytes(Scene &s, size_t bytes);
template <class T>
T *dalloc(Scene &s, size_t count)
{
    return reinterpret_cast<T *>(dalloc_bytes(s, count * sizeof(T)));
}
void dfree(Scene &s, void *p);

inline int nblocks(int64_t n, int b = kBlock) { return (int)((n + b - 1) / b); }

// ---- a list of scenes stepping together --------------------------------------

// Phases with a block count per scene; a scene with 0 blocks sits the phase out.
enum PhaseKind {
    kPhVert = 0,  // vertices, kBlock threads
    kPhTet,       // tets (+ vertices for the body energy: kPhBody)
    kPhBody,      // tets + vertices
    kPhEntry,     // stored BELL entries
    kPhSlice,     // SpMV row blocks (kRowsPerBlock rows each)
    kPhPcgA,      // SpMV row blocks, then pair blocks (PCG A)
    kPhPts, kPhEdges, kPhTris, kPhSurf, kPhInd,
    kPhQPts, kPhQEdges,  // broad-phase queries: kLanesQ threads per point / edge
    kPhPrims,     // point, then edge, then triangle blocks
    kPhTE,        // triangle, then edge blocks
    kPhQAll,      // point-query, then edge-query blocks
    kPhTilesTE,   // both hash tables' bucket blocks
    kPhCand,      // static candidates
    kPhCandSw,    // swept candidates
    kPhAct,       // active pairs, one 64-thread block each
    kPhActT,      // active pairs, kBlock threads
    kPhEnt,       // incidence entries (4 per active pair), kBlock threads
    kPhFric,      // friction pairs, kBlock threads
    kPhVertH,     // vertex blocks, then one block per heavy incidence row
    kPhMas,       // preconditioner diagonal: a wavefront per level-0 aggregate, a block per coarser one
    kPhMasG,      // preconditioner groups (a block each)
    kPhPcgB,      // PCG update: groups, vertex blocks, then a block per heavy incidence row
    kPhOne,       // one block per scene
    kPhTilesT, kPhTilesE, kPhTilesQ, kPhTilesC, kPhTilesA,  // scan tiles
    kPhKinds
};

class Batch {
  public:
    std::vector<Scene *> sc;
    hipStream_t stream = nullptr;
    SceneDev **d_list = nullptr;     // device array of scene view pointers
    int32_t *d_offs = nullptr;       // the block-offset tables, one allocation: table k at k * (cap + 1)
    int32_t *d_off[kPhKinds] = {};   // device block-offset table of each phase (into d_offs)
    std::vector<int32_t> h_off[kPhKinds];
    std::vector<int32_t> h_offs;     // host image of d_offs
    int pend_lo = kPhKinds, pend_hi = -1;  // tables changed since the last upload
    char *d_vstage = nullptr;        // device staging of several scene views (cap of them)
    SceneOut *d_out = nullptr;       // per-scene read-back slots (device)
    SceneOut *h_out = nullptr;       // pinned
    double *d_alpha = nullptr;       // per-scene line-search step (device)
    std::vector<double> h_alpha;
    std::vector<int32_t> fail;       // per-scene error status set by host phases (0 = fine)
    int cap = 0;
    // pinned staging for host-to-device copies of phase maps, views and steps:
    // slots are reused only after the stream has been synchronized
    char *h_stage = nullptr;
    size_t stage_cap = 0, stage_used = 0;
    void *stage_alloc(size_t bytes);
    void *stage(const void *src, size_t bytes);
    std::vector<hipEvent_t> ev_pool;
    struct PendingEv {
        int kernel;
        hipEvent_t a, b;
        double bytes;
        bool big = false;  // a PCG iteration whose SpMV launch moves >= kProfBigBytes
    };
    std::vector<PendingEv> ev_pending;
    ProfSink *sink = nullptr;  // engine lists: timings go here (any list size)

    ~Batch();
    void bind(const std::vector<Scene *> &scenes, hipStream_t strm);
    Launch launch(PhaseKind k) const { return Launch{d_list, d_off[k], d_out, (int)sc.size()}; }
    int blocks(PhaseKind k) const { return h_off[k].empty() ? 0 : h_off[k].back(); }
    // a changed table is uploaded by the next launch (flush_phases), together
    // with the other tables changed since: one copy of their range of d_offs
    void set_phase(PhaseKind k, const std::vector<int32_t> &per_scene_blocks);
    void flush_phases();
    void upload_views();
    void read_out();
    bool prof() const;
    void prof_begin(int kernel, hipEvent_t *pair);
    void prof_end(int kernel, hipEvent_t *pair, double bytes = 0.0);
    void prof_collect();
    void prof_totals(int kernel, int64_t launches, double bytes);  // every launch, not only the timed ones
};

// launch `kernel` over phase `kind` of batch b with `bs` threads per block;
// the first kernel argument is the phase's Launch descriptor
#define IPC_LAUNCH(b, kernel, kind, bs, ...)                                                              \
    do {                                                                                                  \
        int _nb = (b).blocks(kind);                                                                       \
        if (_nb > 0) {                                                                                    \
            (b).flush_phases();                                                                           \
            hipLaunchKernelGGL(kernel, dim3(_nb), dim3(bs), 0, (b).stream, (b).launch(kind), ##__VA_ARGS__); \
        }                                                                                                 \
    } while (0)

// ---- kernel launchers (defined in the .hip files) -------------------------

void launch_begin_step(Batch &b);
void launch_end_step(Batch &b);
void launch_al_update(Batch &b, const std::vector<uint8_t> &on);
void launch_trial(Batch &b);       // uses b.h_alpha (uploaded by the caller to b.d_alpha)
void launch_accept(Batch &b);
// n scene views staged at d_src (n destination pointers, padded to 64 bytes,
// then the n views) put in place by one kernel
__host__ __device__ inline int64_t view_head_bytes(int64_t n) { return (n * 8 + 63) / 64 * 64; }
inline size_t view_stage_bytes(int64_t n) { return (size_t)(view_head_bytes(n) + n * (int64_t)sizeof(SceneDev)); }
void launch_put_views(hipStream_t strm, int n, const void *d_src);
void launch_rest_precompute(Batch &b);
void run_lag_and_mean(Batch &b);
void launch_gather_surface(Scene &s, double *dst, hipStream_t strm);
// pixel grid of a height map (mirrors ipc_height_map_spec)
struct HeightSpec {
    double x0, y0, dx, dy, z_ref;
    int nx, ny;
};
void launch_height_map(Scene &s, const HeightSpec &hs, unsigned long long *key, double *out, hipStream_t strm);

void launch_elastic_elements(Batch &b);
void launch_assemble(Batch &b);
void launch_mas_diag(Batch &b);  // 3x3 aggregate blocks of the assembled matrix, inverted

// 0: static at x, 1: swept over [x, x + p]. A scene whose positions are not
// finite, or whose tables or lists cannot grow, gets b.fail set and must be
// dropped from the phase maps by the caller before the next phase.
void run_broad_phase(Batch &b, int which);
// Static candidates at x taken from the swept list of the previous iteration
// (valid when x moved only along that iteration's segment: every pair whose
// boxes overlap at x is in it); same predicate, same canonical order.
void run_static_from_swept(Batch &b);
void run_narrow_phase(Batch &b);
void launch_barrier(Batch &b);
// friction set from the active pairs at x^t (after the narrow phase at x^t)
void launch_friction_lag(Batch &b);
// friction pairs appended after the barrier pairs, then n_pair for every scene
void launch_friction(Batch &b);
void launch_contact_incidence(Batch &b);
void run_ccd(Batch &b);
void run_energy(Batch &b, bool trial);
void launch_energy_body(Batch &b, bool trial);

void run_pcg(Batch &b, std::vector<int> &iters, std::vector<int> &hit_cap);
// per-scene upper bound on heavy incidence rows, from the active-pair count
inline int heavy_bound(int64_t n_act, int n) { return n_act > 0 ? (int)std::min<int64_t>(n, 4 * n_act / (kHeavyRow + 1) + 1) : 0; }
void set_heavy_phase(Batch &b);  // kPhVertH from the last read-back active-pair counts
void run_pinf(Batch &b);
void launch_hess_apply(Batch &b);  // y (S.q) = H v (S.dB)

enum ScanWhich { kScanTri = 0, kScanEdge = 1, kScanQuery = 2, kScanContact = 3, kScanActive = 4, kScanHeavy = 5,
                 kScanSwFilter = 6 };
// len[s] < 0: scene s sits out; query_sw selects the swept-candidate total
void segmented_scan(Batch &b, ScanWhich which, PhaseKind tiles, const std::vector<int64_t> &len, int query_sw = 0);

void mark_dirty(Scene &s);
// per-scene growth of the dynamic buffers (host; sets s.dev_dirty)
void grow_table(Scene &s, int table, int64_t entries);
void grow_candidates(Scene &s, int which, int64_t need);
void grow_active(Scene &s, int64_t need);
void grow_friction(Scene &s, int64_t need);
// barrier + friction pairs of a scene from its last read-back active-pair count
inline int64_t pair_count(const Scene &s, const SceneOut &o) { return (int64_t)o.n_act + s.h.n_fric; }

}  // namespace ipcg
