/*
 * ipc.h -- C ABI of the MI355X IPC gel-pad step library (libipcgel.so).
 *
 * One call advances a tetrahedral gel pad and a kinematically driven indenter
 * by one implicit time step of the Incremental Potential Contact model: the
 * soft-body step the paper runs through GIPC after setting attachment targets
 * (paper sections "General GIPC Simulation Pipeline" and "GIPC Attachments";
 * the IPC model and its guarantees are cited in "Choice of the Simulation
 * Methods"). Newton on Neo-Hookean elasticity plus a log barrier, PSD-projected
 * Hessians, spatial-hash contact culling, block-Jacobi PCG and a CCD-filtered
 * backtracking line search, all in HIP kernels on one GPU.
 *
 * Conventions
 *  - Vertex ids: gel vertices 0..n_verts-1, then indenter vertices.
 *  - Positions are FP64, interleaved xyz (3 doubles per vertex).
 *  - Every call returns an int32 status: 0 = IPC_OK, > 0 = warning (the state
 *    was committed and is feasible: no interpenetration, every tet J > 0),
 *    < 0 = error (state unchanged). No exception or abort crosses the ABI.
 *  - Host arrays passed in are copied; the caller keeps ownership of every
 *    buffer it passes. The library owns device state from create to destroy.
 *  - Different scenes may be used from different threads; one scene must not
 *    be used by two threads at once.
 */
#ifndef IPC_H
#define IPC_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__) || defined(__clang__)
#define IPC_API __attribute__((visibility("default")))
#else
#define IPC_API
#endif

#define IPC_OK 0
#define IPC_W_NEWTON_MAXITER 1 /* Newton hit max_newton; last iterate committed */
#define IPC_W_PCG_MAXITER 2    /* a PCG solve hit its iteration cap */
#define IPC_W_LS_STALL 3       /* line search shrank below ls_min_ratio; Newton ended */
#define IPC_W_TARGET_LAG 4     /* an indenter vertex ends > 1e-3 dhat from its target */
#define IPC_E_INVALID_ARG -1
#define IPC_E_BAD_MESH -2      /* non-positive rest volume, index out of range, non-manifold */
#define IPC_E_INFEASIBLE -3    /* initial state has a pair at d <= 0 or a tet with J <= 0 */
#define IPC_E_OOM -4           /* allocator or memory budget refused */
#define IPC_E_DEVICE -5        /* HIP runtime error */
#define IPC_E_BUSY -6          /* scene already has a step in flight */
#define IPC_E_CAPACITY -7      /* contact list growth failed */

#define IPC_FP64 0   /* every stage in FP64 */
#define IPC_MIXED 1  /* FP32 assembly/SpMV/PCG vectors, FP64 dots, distances, CCD, energies */

/* PCG preconditioner: 3x3 block Jacobi plus additive corrections on nested
 * aggregates of free gel vertices (default), or 3x3 block Jacobi alone. */
#define IPC_PRECOND_MULTILEVEL 0
#define IPC_PRECOND_JACOBI 1

/* Pair barrier Hessian. PROJECTED: the exact Hessian of kappa w b(d) with its
 * negative eigenvalues clamped to zero (12x12 per pair). GAUSS_NEWTON: the
 * form kappa w b''(d) grad d grad d^T, PSD and rank one by construction (no
 * eigen-decomposition). The paper names GIPC's Gauss-Newton treatment of the
 * barrier only by its title; this form is the library's reading of it: the
 * only term of the exact Hessian that is an outer product of first
 * derivatives with a non-negative weight. The gradient is exact in both. */
#define IPC_BARRIER_PROJECTED 0
#define IPC_BARRIER_GAUSS_NEWTON 1

#define IPC_HOST 0
#define IPC_DEVICE 1

typedef struct ipc_scene ipc_scene;
typedef struct ipc_batch ipc_batch;
typedef int64_t ipc_ticket;

/* Scene description. The gel is a tet mesh (positively oriented tets); the
 * indenter is a triangle mesh in its local frame whose vertices are pulled to
 * the rigid pose of each step by a penalty k_target per vertex. */
typedef struct ipc_scene_desc {
    int32_t n_verts;          /* gel vertices */
    const double *X;          /* n_verts x 3 rest positions (host) */
    int32_t n_tets;
    const int32_t *T;         /* n_tets x 4 (host) */
    const uint8_t *fixed;     /* n_verts Dirichlet mask, may be NULL (host) */
    double E, nu, rho;        /* Neo-Hookean material */
    int32_t n_ind_verts;
    const double *ind_Y;      /* n_ind_verts x 3, indenter local frame (host) */
    int32_t n_ind_tris;
    const int32_t *ind_tris;  /* n_ind_tris x 3 (host) */
    double ind_pose0[12];     /* initial indenter pose, row-major 3x4 [R|c] */
    double dt;                /* time step (s) */
    double dhat, kappa;       /* barrier activation distance (m), stiffness (N/m) */
    double k_target;          /* kinematic target penalty (N/m) */
    double newton_tol;        /* converged when max |p_i| over free DOFs <= newton_tol (m) */
    double pcg_tol;           /* PCG stops at r^T M^-1 r <= pcg_tol^2 r0^T M^-1 r0 */
    double gravity[3];
    double mu_friction, eps_v;/* lagged IPC friction: coefficient (0 = off), velocity threshold (m/s, > 0 when on) */
    double ccd_s;             /* ACCD keep-gap fraction (0.1) */
    double ls_min_ratio;      /* line search stall ratio (2^-30) */
    int32_t self_contact;     /* 1: gel-gel PT/EE pairs take part */
    int32_t precision;        /* IPC_FP64 or IPC_MIXED */
    int32_t max_newton;       /* 0: 100 */
    int32_t pcg_max_iter;     /* 0: 10 * 3 * (all vertices) */
    int32_t ccd_max_iter;     /* 0: 10000 */
    int32_t precond;          /* IPC_PRECOND_MULTILEVEL (0) or IPC_PRECOND_JACOBI */
    int32_t barrier_hessian;  /* IPC_BARRIER_PROJECTED (0) or IPC_BARRIER_GAUSS_NEWTON */
    /* Attachment (the paper's GIPC attachments: gel vertices held by the
     * sensor case move with it). n_verts bytes, 1 = attached, or NULL. An
     * attached free gel vertex i gets k_target/2 |x_i - P X_i|^2 on top of its
     * inertia and elasticity, P the case pose of the step request, X_i its
     * rest position; fixed vertices stay fixed. Copied at creation. */
    const uint8_t *attached;
    /* Augmented-Lagrangian indenter targets (the cited IPC work's treatment
     * of prescribed boundary motion, a variant of the target penalty). With
     * target_al = 1 the term of indenter vertex j is
     * k_target/2 |y_j - yhat_j|^2 - lambda_j . (y_j - yhat_j), lambda = 0 at
     * the start of a step; whenever Newton converges with
     * max_j |y_j - yhat_j| > target_al_tol (m), lambda_j -= k_target (y_j - yhat_j)
     * and Newton goes on (the next iteration takes its step whatever its
     * size), at most target_al_max times per step (0: 8). A softer k_target
     * then meets a tighter lag than the penalty alone. target_al = 0: the
     * plain penalty; the other two fields are ignored. */
    int32_t target_al;
    double target_al_tol;
    int32_t target_al_max;
} ipc_scene_desc;

/* Device memory and stream plumbing. alloc/free may be NULL (then hipMalloc /
 * hipFree); the Python binding routes them to PyTorch's caching allocator.
 * stream is a hipStream_t (NULL = default stream). mem_budget <= 0: none. */
typedef void *(*ipc_alloc_fn)(size_t bytes, void *stream, void *user);
typedef void (*ipc_free_fn)(void *ptr, size_t bytes, void *stream, void *user);
typedef struct ipc_runtime {
    void *stream;
    ipc_alloc_fn alloc;
    ipc_free_fn free;
    void *user;
    int64_t mem_budget;
} ipc_runtime;

/* One step request: the indenter's target pose at t+1 (row-major 3x4) and,
 * when case_pose_set is 1, the sensor case's pose at t+1 (row-major 3x4):
 * attached gel vertices (ipc_scene_desc.attached) are pulled to it applied to
 * their rest positions from this step on. With case_pose_set 0 the case keeps
 * its last pose (identity after creation and after ipc_reset). */
typedef struct ipc_step_req {
    double pose[12];
    double case_pose[12];
    int32_t case_pose_set;
} ipc_step_req;

typedef struct ipc_step_stats {
    int32_t status;
    int32_t newton_iters;     /* Newton iterations (each one assemble + solve) */
    int32_t pcg_iters;        /* PCG iterations summed over the step */
    int32_t ls_halvings;
    int32_t n_candidates;     /* static candidates at the last iterate */
    int32_t n_active;         /* active pairs (d < dhat) at the last iterate */
    double alpha_ccd, alpha;  /* last Newton iteration */
    double energy;            /* incremental potential at the committed state */
    double pinf;              /* last |p|_inf */
    double max_target_lag;    /* max |y_j - yhat_j| over indenter vertices (m) */
    double ms_total;          /* wall time of the step on the host (ms) */
    double ms_phase[8];       /* host wall time per phase: assemble, contact, pcg, ccd, line search,
                                 other (the device work of a phase may finish in a later one) */
    int32_t al_updates;       /* multiplier updates of the step (augmented-Lagrangian targets) */
} ipc_step_stats;

/* Create a scene. Validates the mesh (indices, rest volumes > 0, manifold
 * surface), precomputes rest shape, lumped mass, surface primitives and the
 * matrix pattern, and uploads everything. On error *out = NULL, nothing leaks. */
IPC_API int32_t ipc_create_scene(const ipc_scene_desc *d, const ipc_runtime *rt, ipc_scene **out);
IPC_API void ipc_destroy_scene(ipc_scene *s);
/* Resident bytes plus per-step scratch estimate for admission control. */
IPC_API int64_t ipc_scene_footprint_bytes(const ipc_scene_desc *d);
/* One implicit step toward r->pose; blocks until done on the scene's stream. */
IPC_API int32_t ipc_step(ipc_scene *s, const ipc_step_req *r, ipc_step_stats *st);
/* Surface vertex positions in ascending gel-vertex id order (3 doubles each)
 * and the mean of all gel vertices ("object position"). where = IPC_HOST or
 * IPC_DEVICE for xyz; obj_pos (host, may be NULL). cap in doubles. */
IPC_API int32_t ipc_read_surface(const ipc_scene *s, double *xyz, int64_t cap, int32_t where, void *stream,
                         double obj_pos[3]);
/* Height map of the deformed gel surface (the input of optical tactile
 * renderers, which the paper feeds from the gel's sensing surface). Pixel
 * (i, j), 0 <= i < nx, 0 <= j < ny, has its centre at (x0 + i dx, y0 + j dy)
 * in the gel frame; out[j nx + i] = z_ref - (the largest z at which the
 * vertical line through the centre meets an upward-facing gel surface
 * triangle, i.e. one with positive signed area in xy), or 0 where it meets
 * none: the indentation depth below z_ref (the rest top surface for a tactile
 * image). A centre on a triangle's edge counts as inside. out holds
 * nx ny doubles (cap >= nx ny), in host (IPC_HOST) or device (IPC_DEVICE)
 * memory; stream as for ipc_read_surface. The scratch of nx ny 8-byte keys
 * is taken from the scene's allocator on the first call and kept for later
 * calls of the same or smaller size. */
typedef struct ipc_height_map_spec {
    double x0, y0;   /* centre of pixel (0, 0) (m) */
    double dx, dy;   /* pixel pitch (m), > 0 */
    double z_ref;    /* reference height (m) */
    int32_t nx, ny;  /* pixels per row, rows (> 0) */
} ipc_height_map_spec;
IPC_API int32_t ipc_height_map(const ipc_scene *s, const ipc_height_map_spec *spec, double *out, int64_t cap,
                               int32_t where, void *stream);
/* Allocation-free height map, for callers that cannot allocate device memory
 * (code under HIP graph capture, serving loops or harnesses that forbid
 * hipMalloc). Same arguments and the same map, bit for bit, as
 * ipc_height_map, but no allocator is called: the nx ny 8-byte pixel keys
 * live in one library-owned device array of IPC_HEIGHT_MAP_NOALLOC_MAX_PIXELS
 * entries (8 MiB) per GPU, held until the process ends; its address is looked
 * up on the first call made on each device. nx ny above that maximum returns
 * IPC_E_INVALID_ARG (use ipc_height_map). Every call on one GPU uses that
 * same array, so calls that overlap on one GPU (from several threads, or on
 * streams that do not serialise them) race and must not be issued; the
 * array's contents are cleared by each call before use. Returns after the map
 * is complete on `stream`. */
#define IPC_HEIGHT_MAP_NOALLOC_MAX_PIXELS (1 << 20)
IPC_API int32_t ipc_height_map_noalloc(const ipc_scene *s, const ipc_height_map_spec *spec, double *out,
                                       int64_t cap, int32_t where, void *stream);
/* Surface topology: gel surface triangles (outward, vertex ids) and the
 * ascending list of gel surface vertex ids. Either pointer may be NULL. */
IPC_API int32_t ipc_surface_topology(const ipc_scene *s, int32_t *tris, int64_t tri_cap, int32_t *n_tris,
                             int32_t *verts, int64_t vert_cap, int32_t *n_surf_verts);
/* Reset: positions to rest, velocities to zero, indenter to its initial pose
 * (paper section "General GIPC Simulation Pipeline"). */
IPC_API int32_t ipc_reset(ipc_scene *s);
/* Save / load a scene's state to / from a caller-owned host blob of
 * ipc_state_bytes bytes: x, v, the step index, the indenter pose of the last
 * request and the sensor case pose (so an attached scene resumes with the
 * case where it was). The lagged friction set and the kept candidate list are
 * not saved: the next step rebuilds them from x. load returns
 * IPC_E_INVALID_ARG for a blob of another scene size or format. */
IPC_API int64_t ipc_state_bytes(const ipc_scene *s);
IPC_API int32_t ipc_save_state(const ipc_scene *s, void *blob, int64_t cap);
IPC_API int32_t ipc_load_state(ipc_scene *s, const void *blob, int64_t bytes);
/* Sizes: out[0..7] = n_all, n_gel, n_tets, n_points, n_edges, n_tris, n_ind, n_gel_tris. */
IPC_API int32_t ipc_scene_sizes(const ipc_scene *s, int32_t *out);

/* Batched asynchronous stepping with continuous batching. A batch keeps one
 * list of in-flight steps per class -- precision x size, scenes of at least
 * IPC_BATCH_LARGE_VERTS vertices (gel and indenter) forming the large class --
 * each list with a worker thread and a stream of its own, and runs Newton
 * iterations over each list with one kernel launch per phase for all of its
 * scenes; a step submitted while others are mid-step joins its class's list
 * at the next iteration boundary, a finished step leaves it. The classes run
 * concurrently, so small scenes do not wait for the rounds of large ones.
 * Each scene's results are bitwise those of ipc_step (a scene's blocks,
 * partial sums and reduction order depend on that scene alone).
 * rt->stream: stream of the batch's launches, shared by every class (NULL: a
 * stream per class, created and destroyed by the batch, default priority);
 * rt->mem_budget > 0: the summed device bytes of the scenes in flight (all
 * classes) stay within it, except that a class with an empty list always
 * admits one scene; alloc/free are not used.
 * submit: every scene must be idle and appear once (else IPC_E_BUSY, nothing
 * queued); returns at once with one ticket per scene. A scene with a pending
 * ticket must not be stepped, read, reset or destroyed (calls on it return
 * IPC_E_BUSY; destroying it is undefined). A HIP error inside the worker ends
 * every pending ticket with IPC_E_DEVICE. destroy waits for pending steps. */
#define IPC_BATCH_LARGE_VERTS 65536
IPC_API int32_t ipc_batch_create(const ipc_runtime *rt, ipc_batch **out);
IPC_API void ipc_batch_destroy(ipc_batch *b);
IPC_API int32_t ipc_batch_submit(ipc_batch *b, int32_t n, ipc_scene *const *s, const ipc_step_req *r,
                         ipc_ticket *t);
/* 1 if done (stats filled), 0 if pending, < 0 on error (unknown ticket). */
IPC_API int32_t ipc_batch_poll(ipc_batch *b, ipc_ticket t, ipc_step_stats *st);
/* Blocks until the step is done; returns its status and consumes the ticket. */
IPC_API int32_t ipc_batch_wait(ipc_batch *b, ipc_ticket t, ipc_step_stats *st);
/* Wait for any step: the oldest finished step not yet consumed is returned
 * and consumed (*t its ticket, *status its status, st its stats; status and
 * st may be NULL). Waits up to timeout_ms (< 0: without limit) when none has
 * finished. Returns 1 when a step was returned, 0 on timeout,
 * IPC_E_INVALID_ARG when no step is pending or finished. Lets one host thread
 * serve many environments without polling each ticket. */
IPC_API int32_t ipc_batch_next(ipc_batch *b, double timeout_ms, ipc_ticket *t, int32_t *status,
                               ipc_step_stats *st);
/* Kernel timing inside the engine: enable (1) or disable (0) resets the
 * totals; from the next Newton round on, each phase launch and one PCG
 * launch in sixteen is bracketed by HIP events on the engine's stream (same classes as
 * ipcx_profile). profile_read returns the timed launches, their summed
 * milliseconds and, for classes 0 and 1 (the two PCG kernels), the summed
 * algorithmic bytes of those launches over every scene of the list whose
 * solve was still running: class 0 (SpMV) per stored 3x3 block its values and
 * column index, per vertex the z and d gathers, the d and q writes and the
 * row pointer, per contact pair its off-diagonal blocks and vertex ids;
 * class 1 (update) per vertex q, d, p, r and the 3x3 inverse read and p, r, z
 * written, per incidence entry (4 per pair) its index and 3 pair-product
 * values, per preconditioner member 16 bytes of ids, per SpMV block its d.q
 * partial (4- or 8-byte reals by the list's precision). */
IPC_API int32_t ipc_batch_profile(ipc_batch *b, int32_t enable);
/* Every launch of PCG class 0 or 1 while profiling was on (not only the
 * timed ones) and their summed algorithmic bytes, counted as above: the
 * population a hardware-counter run of the same command measures. */
IPC_API int32_t ipc_batch_profile_totals(ipc_batch *b, int32_t kernel, int64_t *launches, double *bytes_total);
IPC_API int32_t ipc_batch_profile_read(ipc_batch *b, int32_t kernel, int64_t *launches, double *ms_total,
                                       double *bytes_total);
/* The same for the timed launches of the PCG iterations whose SpMV launch
 * (class 0) moves at least 256 MiB of algorithmic bytes, more than the
 * MI355X's Infinity Cache holds: both kernels of such an iteration stream
 * from HBM. Classes 0 and 1. */
IPC_API int32_t ipc_batch_profile_large(ipc_batch *b, int32_t kernel, int64_t *launches, double *ms_total,
                                        double *bytes_total);

IPC_API const char *ipc_status_str(int32_t status);
/* Last error message of the calling thread; returns its length. */
IPC_API int32_t ipc_last_error(char *buf, size_t cap);

/* ---- test-only entry points: pure functions of the given state ----------
 * Host arrays of 3 doubles per vertex (all vertices). They use the step
 * context (predictor and targets) set by ipcx_begin_step. */
IPC_API int32_t ipcx_begin_step(ipc_scene *s, const ipc_step_req *r);
IPC_API int32_t ipcx_newton_iterate(ipc_scene *s, const double *x_in, double *x_out, ipc_step_stats *st);
/* Candidates at x (p NULL) or over [x, x+p]: int32 triples (type, a, b) in
 * canonical order; PT a = point vertex id, b = triangle index; EE a < b edge
 * indices. Triangle and edge numbering as ipcx_primitives reports. */
IPC_API int32_t ipcx_candidates(ipc_scene *s, const double *x, const double *p, int32_t *out, int64_t cap,
                        int64_t *count);
IPC_API int32_t ipcx_primitives(const ipc_scene *s, int32_t *points, int32_t *edges, int32_t *tris);
IPC_API int32_t ipcx_gradient(ipc_scene *s, const double *x, double *g);
IPC_API int32_t ipcx_hess_apply(ipc_scene *s, const double *x, const double *v, double *y);
/* The body stage alone (the incremental potential's inertia, Neo-Hookean
 * elasticity and soft kinematic targets, section "Choice of the Simulation
 * Methods"): its gradient g at x, Dirichlet rows zeroed, and, when v and y
 * are both given, y = H_body v with Dirichlet rows/columns as identity. No
 * barrier or friction pair enters. */
IPC_API int32_t ipcx_assemble_elastic(ipc_scene *s, const double *x, double *g, const double *v, double *y);
/* The barrier stage alone: the active pairs at x (static candidates with
 * d < dhat, in candidate order) as the barrier kernel leaves them, up to cap
 * of them: kind (0 point-triangle, 1 edge-edge), the 4 vertex ids, the
 * 12-gradient and the row-major 12x12 Hessian (PSD-projected, or the
 * Gauss-Newton form the scene asks for), with the rows and columns of
 * Dirichlet vertices zeroed (they live in the body stage's identity rows).
 * *count gets the number of active pairs. Any output array may be NULL. */
IPC_API int32_t ipcx_barrier(ipc_scene *s, const double *x, int64_t cap, int32_t *kind, int32_t *v4, double *g12,
                             double *H144, int64_t *count);
IPC_API int32_t ipcx_pcg(ipc_scene *s, const double *x, double *p, int32_t *iters);
IPC_API int32_t ipcx_energy(ipc_scene *s, const double *x, double *E);
IPC_API int32_t ipcx_ccd(ipc_scene *s, const double *x, const double *p, double *alpha);
/* Per-kernel timing with HIP events on the scene's stream: enable (resets the
 * totals) / read launches and summed milliseconds of a kernel class:
 * 0 PCG SpMV kernel, 1 PCG update kernel, 2 elastic elements, 3 assembly
 * gather, 4 broad phase, 5 narrow phase + barrier, 6 energy, 7 CCD. */
IPC_API int32_t ipcx_profile(ipc_scene *s, int32_t enable);
IPC_API int32_t ipcx_profile_read(const ipc_scene *s, int32_t kernel, int64_t *launches, double *ms_total);
/* Summed algorithmic bytes of the timed launches of kernel class 0 or 1 (the
 * PCG kernels, counted as for ipc_batch_profile_read); 0 for other classes. */
IPC_API int32_t ipcx_profile_bytes(const ipc_scene *s, int32_t kernel, double *bytes_total);
/* Every launch of PCG class 0 or 1 while profiling (not only the timed ones)
 * and their summed algorithmic bytes. */
IPC_API int32_t ipcx_profile_totals(const ipc_scene *s, int32_t kernel, int64_t *launches, double *bytes_total);
/* out[0..7] = stored elastic blocks, stored BELL entries incl. padding, vertices,
 * active pairs, tets, static candidates, swept candidates, gather entries. */
IPC_API int32_t ipcx_matrix_info(const ipc_scene *s, int64_t *out);
/* Multilevel preconditioner of the scene: out[0] levels (0: block-Jacobi only),
 * out[1] groups (blocks of the preconditioner kernel), out[2..4] aggregates
 * of levels 0..2, out[5] the largest group's members, out[6] the largest
 * group's aggregates, out[7] members (free gel vertices). */
IPC_API int32_t ipcx_precond_info(const ipc_scene *s, int64_t *out);
/* The launch and grouping choices the scene took at creation from the
 * autotuner's file ($IPC_TUNING_FILE, else tuning.json beside the library;
 * built-in defaults without one): out[0] SpMV one-thread-per-row threshold
 * (rows of a list), out[1] preconditioner group packing target (members),
 * out[2] first PCG chunk (fraction of the previous solve's iterations),
 * out[3] later chunks (fraction of the remaining count), out[4] 1 if read
 * from a file, out[5] the quantile of a list's scenes' remaining PCG counts
 * the chunk lengths follow. */
IPC_API int32_t ipcx_tuning(const ipc_scene *s, double *out);
/* The same six values for a scene of n_verts vertices created now (host
 * only: reads the tuning file, touches no device). */
IPC_API int32_t ipcx_tuning_for(int32_t n_verts, double *out);
/* sizeof of the boundary's structs as compiled into the library, for a
 * binding to check its own layout: out[0] ipc_scene_desc, out[1] ipc_runtime,
 * out[2] ipc_step_req, out[3] ipc_step_stats, out[4] ipc_height_map_spec.
 * Host only. */
IPC_API int32_t ipcx_struct_sizes(int64_t *out);
IPC_API int32_t ipcx_set_state(ipc_scene *s, const double *x, const double *v);
IPC_API int32_t ipcx_get_state(const ipc_scene *s, double *x, double *v);

#ifdef __cplusplus
}
#endif
#endif
