/*
 * ipc_oracle.h -- plain FP64 CPU oracle of one IPC implicit step of a tet gel
 * pad pressed by a kinematically driven indenter.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library may include, link
 * or call this. It exists so that tests, the smoke check and the CPU baseline
 * leg of the benchmark can check the HIP path against a slow, obviously
 * correct reference written from the method's definition.
 *
 * What it follows: the paper integrates the IPC soft-body model (cited in its
 * "Choice of the Simulation Methods" section: intersection- and inversion-free,
 * any material parameters) through GIPC, whose step updates every soft vertex
 * once the attachment targets are in place (section "General GIPC Simulation
 * Pipeline"). The paper prints no formula for that step, so the energy,
 * barrier, distances, CCD, PCG and line search below are the standard
 * formulation of the cited IPC work; where the paper leaves a choice open, the
 * choice taken is stated at the place it is made.
 *
 * Conventions shared with the product library by *specification only* (no
 * shared code): vertex ids = gel vertices then indenter vertices; primitive
 * numbering and candidate order as documented at ora_candidates().
 */
#ifndef IPC_ORACLE_H
#define IPC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ora_params {
    double E, nu, rho;          /* Young's modulus (Pa), Poisson ratio, density (kg/m^3) */
    double h;                   /* time step (s) */
    double dhat, kappa;         /* barrier activation distance (m), stiffness (N/m) */
    double k_target;            /* kinematic target penalty per indenter vertex (N/m) */
    double newton_tol;          /* stop when max |p_i| over free DOFs <= this (m) */
    double pcg_tol;             /* PCG stops at r^T M^-1 r <= pcg_tol^2 * (its initial value) */
    double gravity[3];
    double ccd_s;               /* ACCD keep-gap fraction */
    double ls_min_ratio;        /* line search stalls below alpha0 * this */
    int32_t self_contact;       /* 1: include gel-gel PT/EE pairs */
    int32_t max_newton;
    int32_t pcg_max_iter;       /* 0: 10 * (3 n) */
    int32_t ccd_max_iter;
    double mu_fric;             /* friction coefficient (0: no friction) */
    double eps_v;               /* friction velocity threshold (m/s); the smoothing length is eps_v h */
    int32_t barrier_hessian;    /* 0: PSD-projected pair Hessians, 1: Gauss-Newton form (ora_pair_barrier) */
    /* Augmented-Lagrangian indenter targets: with target_al = 1 the target
     * term of indenter vertex j is k_t/2 |y_j - yhat_j|^2 - lambda_j . (y_j - yhat_j),
     * lambda = 0 at the start of a step; each time Newton converges with
     * max_j |y_j - yhat_j| > target_al_tol (m), lambda_j -= k_t (y_j - yhat_j)
     * and Newton goes on, at most target_al_max times per step (0: 8). */
    int32_t target_al;
    double target_al_tol;
    int32_t target_al_max;
} ora_params;

typedef struct ora_stats {
    int32_t newton_iters, pcg_iters, n_candidates, n_active, status, ls_halvings;
    double alpha_ccd, alpha, energy, pinf, max_target_lag;
    int32_t al_updates;         /* multiplier updates of the step (augmented-Lagrangian targets) */
} ora_stats;

typedef struct ora_scene ora_scene;

/* status codes (mirrors of the public library's numbering) */
#define ORA_OK 0
#define ORA_W_NEWTON_MAXITER 1
#define ORA_W_PCG_MAXITER 2
#define ORA_W_LS_STALL 3
#define ORA_W_TARGET_LAG 4
#define ORA_E_INVALID_ARG -1
#define ORA_E_BAD_MESH -2
#define ORA_E_INFEASIBLE -3

ora_scene *ora_scene_create(int32_t n_gel, const double *X, int32_t n_tet, const int32_t *T,
                            const uint8_t *fixed, int32_t n_ind, const double *Y_local,
                            int32_t n_ind_tri, const int32_t *ind_tri, const double *pose0,
                            const ora_params *prm, int32_t *status);
void ora_scene_destroy(ora_scene *s);
/* out[0..7] = n_all, n_gel, n_tet, n_points, n_edges, n_tris, n_ind, n_gel_tris */
void ora_scene_sizes(const ora_scene *s, int32_t *out);
void ora_scene_surface(const ora_scene *s, int32_t *points, int32_t *edges, int32_t *tris);
void ora_scene_rest(const ora_scene *s, double *vol, double *mass);
void ora_get_x(const ora_scene *s, double *x);
void ora_set_x(ora_scene *s, const double *x);
void ora_get_v(const ora_scene *s, double *v);
void ora_set_v(ora_scene *s, const double *v);
void ora_reset(ora_scene *s);
/* Attachment: mask (n_gel bytes, NULL: none) of free gel vertices pulled by
 * k_target/2 |x_i - P_case X_i|^2 to the case pose applied to their rest
 * position; the case pose (3x4 row-major, identity at creation) is read by
 * ora_begin_step. */
void ora_set_attachment(ora_scene *s, const uint8_t *mask);
void ora_set_case_pose(ora_scene *s, const double *pose);

/* Start a step toward indenter pose `pose` (row-major 3x4): stores x^t, the
 * inertial predictor and the indenter targets. */
void ora_begin_step(ora_scene *s, const double *pose);
/* One Newton iteration from x_in (teacher forcing). Returns 1 if converged
 * (x_out = x_in), 0 if a step was taken, 2 on line-search stall. */
int32_t ora_newton_iterate(ora_scene *s, const double *x_in, double *x_out, ora_stats *st);
/* Full step: begin_step + Newton loop + velocity update. Returns a status. */
int32_t ora_step(ora_scene *s, const double *pose, ora_stats *st);

/* Candidates (type, a, b) at x (p == NULL: static boxes) or over [x, x+p]
 * (swept boxes). PT: a = point vertex id, b = triangle index; EE: a < b edge
 * indices. Sorted by (type, a, b). Writes at most `cap` triples, returns count. */
int32_t ora_candidates(const ora_scene *s, const double *x, const double *p, int32_t *out,
                       int32_t cap);
/* Incremental potential at x (static candidates at x), +inf if infeasible. */
double ora_energy(ora_scene *s, const double *x);
/* Gradient at x with Dirichlet rows zeroed. */
void ora_gradient(ora_scene *s, const double *x, double *g);
/* y = H(x) v with the PSD-projected Hessian and Dirichlet rows/cols replaced by identity. */
void ora_hess_apply(ora_scene *s, const double *x, const double *v, double *y);
/* Gradient of each term of Phi at x (inertia, elasticity, soft targets,
 * barrier, friction), Dirichlet rows NOT zeroed; 3n doubles each or NULL. */
void ora_gradient_terms(ora_scene *s, const double *x, double *g_inertia, double *g_elastic, double *g_target,
                        double *g_contact, double *g_friction);
/* y = H_body v: inertia, elasticity and soft targets only (no barrier or
 * friction pair), Dirichlet rows/cols replaced by identity. */
void ora_hess_apply_body(ora_scene *s, const double *x, const double *v, double *y);
/* The active barrier pairs at x (static candidates with d < dhat, in candidate
 * order), as the assembly forms them: kind (0 PT, 1 EE), 4 vertex ids, the
 * 12-gradient and the 12x12 Hessian (row-major; PSD-projected or Gauss-Newton
 * as the scene's parameters say), before Dirichlet rows are dropped. Writes at
 * most cap pairs (any array may be NULL); returns the count. */
int32_t ora_contact_pairs(ora_scene *s, const double *x, int32_t cap, int32_t *kind, int32_t *v4, double *g12,
                          double *H144);
/* Dense 3n x 3n form of the matrix ora_hess_apply applies (small scenes only). */
void ora_hess_dense(ora_scene *s, const double *x, double *H);
/* Block-Jacobi PCG solve of H p = -g at x; returns iterations. */
int32_t ora_pcg(ora_scene *s, const double *x, double *p);
/* min(1, min over swept candidates of ACCD time of impact). */
double ora_ccd(ora_scene *s, const double *x, const double *p);
/* Per-candidate unsigned distance and type at x for a candidate list. */
void ora_candidate_distances(const ora_scene *s, const double *x, int32_t nc, const int32_t *cand,
                             double *d, int32_t *type);

/* ---- element-level functions (pins) ---- */
double ora_nh_psi(const double *F, double mu, double lam);
void ora_nh_pk1(const double *F, double mu, double lam, double *P);
void ora_nh_hessian(const double *F, double mu, double lam, double *H81);
void ora_tet_elastic(const double *x12, const double *Bm, double vol, double mu, double lam,
                     double *E, double *g12, double *H144);
void ora_sym_eig(int32_t n, const double *A, double *w, double *V);
void ora_psd_project(int32_t n, double *A);
double ora_pt_distance(const double *x12, int32_t *type);
double ora_ee_distance(const double *x12, int32_t *type);
/* kind 0 = PT, 1 = EE; grad/hess of the unsigned distance, unprojected */
double ora_distance_derivs(int32_t kind, const double *x12, double *g12, double *H144);
void ora_barrier_scalar(double d, double dhat, double *b3);
/* pair barrier energy (kappa * w * b), gradient and Hessian; project: 0 exact,
 * 1 PSD-projected, 2 Gauss-Newton kappa w b'' grad d grad d^T */
double ora_pair_barrier(int32_t kind, const double *x12, double dhat, double kappa, double eps_x,
                        int32_t project, double *g12, double *H144);
double ora_accd(int32_t kind, const double *x12, const double *p12, double s, double tmax,
                int32_t max_iter);
/* Friction smoothing: f3 = {f0(y), f0'(y), f0''(y)} for the smoothing length eps. */
void ora_friction_f(double y, double eps, double *f3);
/* One lagged friction pair: contact coefficients c4 and unit normal nrm from
 * x^t (xt12), normal-force magnitude folded into mu_lam = mu * lambda.
 * Returns D; g12 / H144 (PSD) may be NULL. */
double ora_pair_friction(const double *x12, const double *xt12, const double *c4, const double *nrm,
                         double mu_lam, double eps, double *g12, double *H144);
/* Lagged friction set of the current step: count, and per pair (when the
 * arrays are not NULL) 4 vertex ids, 4 coefficients, the normal, lambda. */
int32_t ora_friction_set(const ora_scene *s, int32_t *v4, double *c4, double *nrm, double *lam);

#ifdef __cplusplus
}
#endif
#endif
