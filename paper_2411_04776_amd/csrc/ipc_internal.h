// ipc_internal.h -- internal types of the MI355X IPC gel-pad step library.
//
// Layout in HBM (one scene):
//   vertex vectors (x, v, gradient, PCG vectors): interleaved xyz, 3*n values,
//     streamed contiguously by the vector kernels;
//   per-tet data (indices, Dm^-1, volume, element gradient/Hessian blocks):
//     structure of arrays, one array per component, so a wavefront of 64
//     tets reads 64 consecutive values per component;
//   the elastic matrix: blocked sliced ELL with 3x3 blocks, a slice = 64
//     rows = one wavefront, each slice padded to its longest row, stored
//     component-major inside the slice (value[(slot*9+c)*64 + lane]) so that
//     every load of a slot is one coalesced 512-byte access; slot 0 of every
//     row is its diagonal block;
//   contact pairs: structure of arrays over active pairs (4 vertex ids,
//     12 gradient and 144 Hessian components), applied in SpMV through a
//     per-vertex incidence list sorted by pair index (no float atomics).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "ipc.h"

namespace ipcg {

constexpr int kSlice = 64;        // rows per BELL slice (one wavefront)
constexpr int kBlock = 256;       // threads per block for streaming kernels
constexpr int kElemBlocks = 10;   // upper-triangle 3x3 blocks of a 12x12 element matrix

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

// Rigid pose [R|c], row-major 3x4, passed to kernels by value.
struct Pose {
    double m[12];
};

struct Params {
    double E, nu, rho, mu, lam;
    double dt, dhat, kappa, k_target;
    double newton_tol, pcg_tol;
    double grav[3];
    double mu_fric, eps_v;
    double ccd_s, ls_min_ratio;
    int self_contact, precision, max_newton, pcg_max_iter, ccd_max_iter;
};

// Small values read back to the host after a phase (pinned host memory).
struct Readback {
    int64_t count;       // candidate / active counts
    int32_t flag;        // overflow / infeasible / done flags
    int32_t iters;
    double value;        // reduced scalar (energy, alpha, |p|_inf)
    double value2;
};

class Scene;

// Device allocation through the runtime's callbacks (PyTorch's caching
// allocator from Python) or hipMalloc.
struct DeviceArena {
    ipc_runtime rt{};
    int64_t used = 0;
    void *alloc(size_t bytes);
    void release(void *p, size_t bytes);
};

template <class T>
struct DArr {
    T *p = nullptr;
    size_t n = 0;
};

// Broad-phase working set for one primitive family used as a hash target.
struct HashTable {
    int32_t table_bits = 0;
    DArr<int32_t> bucket_count;   // table_size + 1
    DArr<int32_t> bucket_start;   // table_size + 1
    DArr<int4> entries;           // (ix, iy, iz, id)
};

class Scene {
  public:
    Params prm{};
    hipStream_t stream = nullptr;
    DeviceArena arena;
    std::vector<std::pair<void *, size_t>> owned;

    // sizes
    int n = 0, n_gel = 0, n_ind = 0, m = 0;
    int n_pts = 0, n_edges = 0, n_tris = 0, n_gel_tris = 0, n_gel_edges = 0;
    int n_slices = 0, n_slots = 0;     // BELL
    int64_t n_gather = 0;              // BSR gather entries

    // host copies of topology (ABI queries, tests)
    std::vector<int32_t> h_pts, h_edges, h_tris, h_surf_verts;
    std::vector<double> h_Yloc;
    Pose pose0{};

    // state
    double *x = nullptr, *v = nullptr, *xt = nullptr, *xtilde = nullptr, *yhat = nullptr;
    double *X0 = nullptr, *Yloc = nullptr, *xtrial = nullptr;
    uint8_t *fixed = nullptr;
    double *mass = nullptr;
    // tets (SoA)
    int32_t *tv = nullptr;       // 4 * m
    double *Bm = nullptr;        // 9 * m
    double *vol = nullptr;       // m
    double *eg = nullptr;        // 12 * m element gradients
    double *eH = nullptr;        // 90 * m element Hessian blocks
    int32_t *vt_ptr = nullptr, *vt_src = nullptr;   // vertex -> (tet*4 + local)
    // BELL matrix
    int32_t *slice_ptr = nullptr;    // n_slices + 1, in slots
    int32_t *bcol = nullptr;         // n_slots * 64
    double *bval = nullptr;          // n_slots * 9 * 64
    int32_t *g_ptr = nullptr;        // n_slots * 64 + 1
    int32_t *g_src = nullptr;        // tet*16 + a*4 + b
    double *grad = nullptr, *Minv = nullptr;
    // surface primitives
    int32_t *pts = nullptr, *ev = nullptr, *trv = nullptr;   // ev: 2*ne SoA, trv: 3*nt SoA
    double *edge_rest_sq = nullptr;
    // boxes (SoA lo xyz, hi xyz)
    double *pbox = nullptr, *ebox = nullptr, *tbox = nullptr;
    HashTable ht_tri, ht_edge;
    double *cell_h = nullptr;        // device scalar
    double *red_scratch = nullptr;   // reduction partials
    int32_t *i_scratch = nullptr;    // integer scan scratch
    size_t i_scratch_n = 0;
    int32_t *q_count = nullptr, *q_off = nullptr;  // per query counts / offsets
    size_t q_n = 0;
    // candidates
    int64_t cand_cap = 0;
    int32_t *cand = nullptr;         // 3 * cand_cap (type, a, b) SoA
    int64_t n_cand = 0;
    int64_t sw_cap = 0;
    int32_t *cand_sw = nullptr;
    int64_t n_cand_sw = 0;
    double *cand_d = nullptr;        // cand_cap
    int32_t *act_flag = nullptr;     // cand_cap + 1
    // active pairs
    int64_t act_cap = 0, n_act = 0;
    int32_t *act_idx = nullptr;      // act_cap
    int32_t *act_v = nullptr;        // 4 * act_cap
    double *act_g = nullptr;         // 12 * act_cap
    double *act_H = nullptr;         // 144 * act_cap
    int32_t *c_ptr = nullptr;        // n + 1
    int32_t *c_cnt = nullptr;        // n
    int32_t *c_list = nullptr;       // 4 * act_cap
    // PCG
    double *r = nullptr, *z = nullptr, *dA = nullptr, *dB = nullptr, *q = nullptr, *sol = nullptr;
    double *pcg_part = nullptr;      // 3 * nblocks partials
    int32_t *pcg_state = nullptr;    // done flag, iterations
    double *accd_t = nullptr;        // reduction partials of CCD / energy
    int64_t part_cap = 0;
    int64_t aux_cap = 0;             // capacity of cand_d / act_flag
    int32_t *surf_verts = nullptr;   // gel surface vertex ids, ascending
    double *xw = nullptr, *pw = nullptr, *yw = nullptr;  // work vectors (test hooks, readback)
    double *mean_part = nullptr;
    Readback *hb = nullptr;          // pinned
    int step_index = 0;
    bool busy = false;
    int last_pcg_iters = 0;          // iterations of the last PCG solve
    int64_t nnzb = 0;                // stored (non-padding) elastic blocks

    // optional per-kernel timing with HIP events on the scene's stream
    bool prof = false;
    struct ProfAcc {
        int64_t launches = 0;
        double ms = 0.0;
    } prof_acc[kProfKernels];
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_pending;

    ~Scene();
};

// ---- kernel launchers (defined in the .hip files) -------------------------

// predictor / misc
void launch_begin_step(Scene &s, const Pose &pose);
void launch_end_step(Scene &s);
void launch_trial(Scene &s, const double *x, const double *p, double alpha, double *out);
void launch_rest_precompute(Scene &s);

// elasticity and assembly
void launch_elastic_elements(Scene &s, const double *x);
void launch_assemble(Scene &s, const double *x);

// contact
void launch_boxes(Scene &s, const double *x, const double *p);
int64_t run_broad_phase(Scene &s, const double *x, const double *p, int32_t **out, int64_t *cap);
int64_t run_narrow_phase(Scene &s, const double *x);
void launch_barrier(Scene &s, const double *x);
void launch_contact_incidence(Scene &s);
double run_ccd(Scene &s, const double *x, const double *p);
double run_energy(Scene &s, const double *x, const int32_t *cand, int64_t nc, int *infeasible);

void ensure_cand_aux(Scene &s);
void launch_gather_surface(Scene &s, double *dst, hipStream_t strm);
double *run_gel_mean(Scene &s, hipStream_t strm);
double run_target_lag(Scene &s);

// solver
int run_pcg(Scene &s, int *hit_cap);
double run_pinf(Scene &s);
void launch_hess_apply(Scene &s, const double *v, double *y);

// scan helpers
void exclusive_scan(Scene &s, const int32_t *in, int32_t *out, int n, int32_t *total_dev);
void ensure_iscratch(Scene &s, size_t n);
void ensure_query(Scene &s, size_t n);

// profiler: prof_begin/prof_end bracket launches of one kernel class;
// prof_collect (after a stream sync) accumulates the elapsed times
void prof_begin(Scene &s, int kernel, hipEvent_t *pair);
void prof_end(Scene &s, int kernel, hipEvent_t *pair);
void prof_collect(Scene &s);

// errors
void set_error(const std::string &msg);
int32_t hip_fail(hipError_t e, const char *where);

#define IPC_HIP(call)                                                   \
    do {                                                                \
        hipError_t _e = (call);                                         \
        if (_e != hipSuccess) throw ipcg::HipError(_e, #call);          \
    } while (0)

struct HipError {
    hipError_t e;
    const char *what;
    HipError(hipError_t e_, const char *w) : e(e_), what(w) {}
};
struct OomError {};
struct CapacityError {};
struct InfeasibleError {};

template <class T>
T *dalloc(Scene &s, size_t count)
{
    size_t bytes = count * sizeof(T);
    if (bytes == 0) bytes = sizeof(T);
    void *p = s.arena.alloc(bytes);
    if (!p) throw OomError{};
    s.owned.push_back({p, bytes});
    return reinterpret_cast<T *>(p);
}
void dfree(Scene &s, void *p);

inline int nblocks(int64_t n, int b = kBlock) { return (int)((n + b - 1) / b); }

}  // namespace ipcg
