/*
 * ipc_oracle.c -- plain FP64 CPU oracle of one IPC implicit step.
 *
 * TEST INFRASTRUCTURE ONLY: the slow, obviously correct reference that the HIP
 * library is checked against. Only tests, the smoke check and the benchmark's
 * CPU-baseline leg may load it. It shares no code with the product library.
 *
 * Single thread, plain loops, FP64 throughout, built with -O2
 * -ffp-contract=off and no fast-math so that per-primitive formulas round the
 * same way as the GPU path's FP64 contact code.
 *
 * The paper (TacEx) integrates GIPC, a GPU variant of the IPC model it cites in
 * "Choice of the Simulation Methods"; one GIPC step updates every soft vertex
 * once the attachment targets are in place ("General GIPC Simulation
 * Pipeline", "GIPC Attachments"). The paper prints no formulas for that step,
 * so every formula here is the standard IPC formulation of the cited IPC work
 * (Li et al. 2020): incremental potential with a log barrier on unsigned
 * point-triangle / edge-edge distances, PSD-projected Newton, CCD-filtered
 * backtracking line search. Where the paper leaves a choice open, the choice
 * taken is stated at the place it is made.
 */
#include "ipc_oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* EE pairs whose segment-segment normal-equation determinant is below this
 * fraction of |u|^2 |v|^2 are treated as parallel (closest points then come
 * from an endpoint). */
#define ORA_EE_PARALLEL 1e-10
/* EE mollifier threshold factor: eps_x = 1e-3 |e0_rest|^2 |e1_rest|^2. */
#define ORA_MOLLIFIER_FACTOR 1e-3

/* ======================================================================== */
/* small dense helpers                                                       */
/* ======================================================================== */

static void sub3(const double *a, const double *b, double *o)
{
    o[0] = a[0] - b[0];
    o[1] = a[1] - b[1];
    o[2] = a[2] - b[2];
}
static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double *a, const double *b, double *o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
static double det3(const double *M) /* row-major 3x3 */
{
    return M[0] * (M[4] * M[8] - M[5] * M[7]) - M[1] * (M[3] * M[8] - M[5] * M[6]) +
           M[2] * (M[3] * M[7] - M[4] * M[6]);
}
/* inverse of a row-major 3x3 by the adjugate; returns the determinant */
static double inv3(const double *M, double *O)
{
    double d = det3(M);
    O[0] = (M[4] * M[8] - M[5] * M[7]) / d;
    O[1] = (M[2] * M[7] - M[1] * M[8]) / d;
    O[2] = (M[1] * M[5] - M[2] * M[4]) / d;
    O[3] = (M[5] * M[6] - M[3] * M[8]) / d;
    O[4] = (M[0] * M[8] - M[2] * M[6]) / d;
    O[5] = (M[2] * M[3] - M[0] * M[5]) / d;
    O[6] = (M[3] * M[7] - M[4] * M[6]) / d;
    O[7] = (M[1] * M[6] - M[0] * M[7]) / d;
    O[8] = (M[0] * M[4] - M[1] * M[3]) / d;
    return d;
}

/* Neumaier (improved Kahan) compensated summation. */
typedef struct {
    double s, c;
} nsum;
static void nsum_add(nsum *a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v))
        a->c += (a->s - t) + v;
    else
        a->c += (v - t) + a->s;
    a->s = t;
}
static double nsum_get(const nsum *a) { return a->s + a->c; }

/* ======================================================================== */
/* symmetric eigen-decomposition (cyclic Jacobi) and PSD projection          */
/* ======================================================================== */

/* Cyclic-by-row Jacobi (Golub & Van Loan, section 8.5): A = V diag(w) V^T.
 * A is n x n row-major symmetric; V columns are eigenvectors. */
void ora_sym_eig(int32_t n, const double *A_in, double *w, double *V)
{
    double *A = (double *)malloc(sizeof(double) * n * n);
    memcpy(A, A_in, sizeof(double) * n * n);
    for (int i = 0; i < n * n; ++i) V[i] = 0.0;
    for (int i = 0; i < n; ++i) V[i * n + i] = 1.0;
    double fro = 0.0;
    for (int i = 0; i < n * n; ++i) fro += A[i] * A[i];
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) off += A[p * n + q] * A[p * n + q];
        if (off <= 1e-36 * fro || off == 0.0) break;
        for (int p = 0; p < n; ++p) {
            for (int q = p + 1; q < n; ++q) {
                double apq = A[p * n + q];
                if (apq == 0.0) continue;
                double app = A[p * n + p], aqq = A[q * n + q];
                double theta = (aqq - app) / (2.0 * apq);
                double t;
                if (fabs(theta) > 1e150)
                    t = 0.5 / theta;
                else
                    t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                /* A <- J^T A J with J the rotation in the (p,q) plane */
                for (int k = 0; k < n; ++k) {
                    double akp = A[k * n + p], akq = A[k * n + q];
                    A[k * n + p] = c * akp - s * akq;
                    A[k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {
                    double apk = A[p * n + k], aqk = A[q * n + k];
                    A[p * n + k] = c * apk - s * aqk;
                    A[q * n + k] = s * apk + c * aqk;
                }
                A[p * n + q] = 0.0;
                A[q * n + p] = 0.0;
                for (int k = 0; k < n; ++k) {
                    double vkp = V[k * n + p], vkq = V[k * n + q];
                    V[k * n + p] = c * vkp - s * vkq;
                    V[k * n + q] = s * vkp + c * vkq;
                }
            }
        }
    }
    for (int i = 0; i < n; ++i) w[i] = A[i * n + i];
    free(A);
}

/* Nearest PSD matrix in the Frobenius norm: clamp negative eigenvalues to 0. */
void ora_psd_project(int32_t n, double *A)
{
    double w[12], V[144];
    double *wp = w, *Vp = V;
    if (n > 12) {
        wp = (double *)malloc(sizeof(double) * n);
        Vp = (double *)malloc(sizeof(double) * n * n);
    }
    ora_sym_eig(n, A, wp, Vp);
    int any_neg = 0;
    for (int i = 0; i < n; ++i) any_neg |= (wp[i] < 0.0);
    if (any_neg) {
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double acc = 0.0;
                for (int k = 0; k < n; ++k)
                    if (wp[k] > 0.0) acc += Vp[i * n + k] * wp[k] * Vp[j * n + k];
                A[i * n + j] = acc;
            }
    }
    if (n > 12) {
        free(wp);
        free(Vp);
    }
}

/* ======================================================================== */
/* Neo-Hookean elasticity                                                    */
/* ======================================================================== */
/* Compressible Neo-Hookean density
 *   Psi(F) = mu/2 (tr F^T F - 3) - mu ln J + lam/2 (ln J)^2,  +inf for J <= 0,
 * with Lame parameters from E and nu. F is row-major, vec index i*3+j. */

double ora_nh_psi(const double *F, double mu, double lam)
{
    double J = det3(F);
    if (!(J > 0.0)) return INFINITY;
    double tr = 0.0;
    for (int i = 0; i < 9; ++i) tr += F[i] * F[i];
    double lnJ = log(J);
    return 0.5 * mu * (tr - 3.0) - mu * lnJ + 0.5 * lam * lnJ * lnJ;
}

static void inv_transpose3(const double *F, double *FiT)
{
    double Fi[9];
    inv3(F, Fi);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) FiT[i * 3 + j] = Fi[j * 3 + i];
}

/* first Piola-Kirchhoff stress P = mu (F - F^-T) + lam ln J F^-T */
void ora_nh_pk1(const double *F, double mu, double lam, double *P)
{
    double FiT[9];
    inv_transpose3(F, FiT);
    double lnJ = log(det3(F));
    for (int i = 0; i < 9; ++i) P[i] = mu * (F[i] - FiT[i]) + lam * lnJ * FiT[i];
}

/* dP_ij/dF_kl = mu d_ik d_jl + (mu - lam lnJ) FiT_il FiT_kj + lam FiT_ij FiT_kl */
void ora_nh_hessian(const double *F, double mu, double lam, double *H)
{
    double FiT[9];
    inv_transpose3(F, FiT);
    double lnJ = log(det3(F));
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l) {
                    double v = (mu - lam * lnJ) * FiT[i * 3 + l] * FiT[k * 3 + j] +
                               lam * FiT[i * 3 + j] * FiT[k * 3 + l];
                    if (i == k && j == l) v += mu;
                    H[(i * 3 + j) * 9 + (k * 3 + l)] = v;
                }
}

/* Linear map D (9x12) from the tet's stacked vertex positions to vec(F) for
 * F = Ds Bm, Ds = [x1-x0, x2-x0, x3-x0]: dF_ij/dx_{a,c} = delta_ic q_a[j] with
 * q_a = row a-1 of Bm (a = 1..3) and q_0 = -(sum of rows of Bm). */
static void tet_dFdx(const double *Bm, double *D)
{
    double q[4][3];
    for (int j = 0; j < 3; ++j) {
        q[1][j] = Bm[0 * 3 + j];
        q[2][j] = Bm[1 * 3 + j];
        q[3][j] = Bm[2 * 3 + j];
        q[0][j] = -(q[1][j] + q[2][j] + q[3][j]);
    }
    for (int r = 0; r < 9 * 12; ++r) D[r] = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            for (int a = 0; a < 4; ++a) D[(i * 3 + j) * 12 + (a * 3 + i)] = q[a][j];
}

static void tet_F(const double *x12, const double *Bm, double *F)
{
    double Ds[9];
    for (int i = 0; i < 3; ++i)
        for (int c = 0; c < 3; ++c) Ds[i * 3 + c] = x12[(c + 1) * 3 + i] - x12[i];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += Ds[i * 3 + k] * Bm[k * 3 + j];
            F[i * 3 + j] = acc;
        }
}

/* Element energy V Psi(F), gradient V D^T vec(P), and Hessian
 * V D^T Pi+(d2Psi/dF2) D, with Pi+ the PSD projection of the 9x9 stage. */
void ora_tet_elastic(const double *x12, const double *Bm, double vol, double mu, double lam,
                     double *E, double *g12, double *H144)
{
    double F[9], D[108];
    tet_F(x12, Bm, F);
    double psi = ora_nh_psi(F, mu, lam);
    if (E) *E = vol * psi;
    if (!isfinite(psi)) return;
    tet_dFdx(Bm, D);
    if (g12) {
        double P[9];
        ora_nh_pk1(F, mu, lam, P);
        for (int c = 0; c < 12; ++c) {
            double acc = 0.0;
            for (int r = 0; r < 9; ++r) acc += D[r * 12 + c] * P[r];
            g12[c] = vol * acc;
        }
    }
    if (H144) {
        double Hf[81], HD[9 * 12];
        ora_nh_hessian(F, mu, lam, Hf);
        ora_psd_project(9, Hf);
        for (int r = 0; r < 9; ++r)
            for (int c = 0; c < 12; ++c) {
                double acc = 0.0;
                for (int k = 0; k < 9; ++k) acc += Hf[r * 9 + k] * D[k * 12 + c];
                HD[r * 12 + c] = acc;
            }
        for (int a = 0; a < 12; ++a)
            for (int b = 0; b < 12; ++b) {
                double acc = 0.0;
                for (int k = 0; k < 9; ++k) acc += D[k * 12 + a] * HD[k * 12 + b];
                H144[a * 12 + b] = vol * acc;
            }
    }
}

/* ======================================================================== */
/* unsigned distances                                                        */
/* ======================================================================== */
/* A distance "type" names the pair of closest features. Within one type the
 * squared distance is s(x) = min_beta |r(x,beta)|^2 with
 *   r = sum_k c_k(beta) x_k,  c(beta) = c0 + sum_m beta_m Dm,
 * beta unconstrained on the features' affine hulls (0, 1 or 2 parameters).
 *
 * PT (x0 = point, x1..x3 = triangle t0,t1,t2):
 *   0..2 vertex t0/t1/t2, 3 edge t0t1, 4 edge t1t2, 5 edge t2t0, 6 face.
 * EE (x0,x1 = edge A, x2,x3 = edge B):
 *   0 A0-B0, 1 A0-B1, 2 A1-B0, 3 A1-B1, 4 A0-edgeB, 5 A1-edgeB,
 *   6 B0-edgeA, 7 B1-edgeA, 8 line-line. */

typedef struct {
    int np;
    double c0[4];
    double D[2][4];
} dist_spec;

static dist_spec pt_spec(int type)
{
    dist_spec s;
    memset(&s, 0, sizeof s);
    s.c0[0] = 1.0;
    switch (type) {
    case 0: s.c0[1] = -1.0; break;
    case 1: s.c0[2] = -1.0; break;
    case 2: s.c0[3] = -1.0; break;
    case 3: /* p - (t0 + b (t1 - t0)) */
        s.np = 1; s.c0[1] = -1.0; s.D[0][1] = 1.0; s.D[0][2] = -1.0; break;
    case 4: /* p - (t1 + b (t2 - t1)) */
        s.np = 1; s.c0[2] = -1.0; s.D[0][2] = 1.0; s.D[0][3] = -1.0; break;
    case 5: /* p - (t2 + b (t0 - t2)) */
        s.np = 1; s.c0[3] = -1.0; s.D[0][3] = 1.0; s.D[0][1] = -1.0; break;
    default: /* p - (t0 + b1 (t1 - t0) + b2 (t2 - t0)) */
        s.np = 2; s.c0[1] = -1.0;
        s.D[0][1] = 1.0; s.D[0][2] = -1.0;
        s.D[1][1] = 1.0; s.D[1][3] = -1.0;
        break;
    }
    return s;
}

static dist_spec ee_spec(int type)
{
    dist_spec s;
    memset(&s, 0, sizeof s);
    switch (type) {
    case 0: s.c0[0] = 1; s.c0[2] = -1; break;
    case 1: s.c0[0] = 1; s.c0[3] = -1; break;
    case 2: s.c0[1] = 1; s.c0[2] = -1; break;
    case 3: s.c0[1] = 1; s.c0[3] = -1; break;
    case 4: /* A0 - (B0 + t (B1 - B0)) */
        s.np = 1; s.c0[0] = 1; s.c0[2] = -1; s.D[0][2] = 1; s.D[0][3] = -1; break;
    case 5:
        s.np = 1; s.c0[1] = 1; s.c0[2] = -1; s.D[0][2] = 1; s.D[0][3] = -1; break;
    case 6: /* (A0 + u (A1 - A0)) - B0 */
        s.np = 1; s.c0[0] = 1; s.c0[2] = -1; s.D[0][0] = -1; s.D[0][1] = 1; break;
    case 7:
        s.np = 1; s.c0[0] = 1; s.c0[3] = -1; s.D[0][0] = -1; s.D[0][1] = 1; break;
    default: /* (A0 + u (A1 - A0)) - (B0 + t (B1 - B0)) */
        s.np = 2; s.c0[0] = 1; s.c0[2] = -1;
        s.D[0][0] = -1; s.D[0][1] = 1;
        s.D[1][2] = 1; s.D[1][3] = -1;
        break;
    }
    return s;
}

/* Closest features of point p and triangle (a,b,c) by the Voronoi-region tests
 * of Ericson, Real-Time Collision Detection, section 5.1.5. Ties (<=) go to
 * the lower-dimensional feature. */
static int pt_type(const double *x12)
{
    const double *p = x12, *a = x12 + 3, *b = x12 + 6, *c = x12 + 9;
    double ab[3], ac[3], ap[3], bp[3], cp[3];
    sub3(b, a, ab);
    sub3(c, a, ac);
    sub3(p, a, ap);
    double d1 = dot3(ab, ap), d2 = dot3(ac, ap);
    if (d1 <= 0.0 && d2 <= 0.0) return 0;
    sub3(p, b, bp);
    double d3 = dot3(ab, bp), d4 = dot3(ac, bp);
    if (d3 >= 0.0 && d4 <= d3) return 1;
    double vc = d1 * d4 - d3 * d2;
    if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) return 3;
    sub3(p, c, cp);
    double d5 = dot3(ab, cp), d6 = dot3(ac, cp);
    if (d6 >= 0.0 && d5 <= d6) return 2;
    double vb = d5 * d2 - d1 * d6;
    if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) return 5;
    double va = d3 * d6 - d5 * d4;
    if (va <= 0.0 && (d4 - d3) >= 0.0 && (d5 - d6) >= 0.0) return 4;
    return 6;
}

static double clamp01(double v) { return v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v); }

/* Closest points of segments A = [A0,A1], B = [B0,B1] by clamped parameters
 * (Ericson, section 5.1.9), then named by which parameters sit at an end.
 * Near-parallel segments start from A0 (s = 0). */
static int ee_type(const double *x12)
{
    const double *p1 = x12, *q1 = x12 + 3, *p2 = x12 + 6, *q2 = x12 + 9;
    double d1[3], d2[3], r[3];
    sub3(q1, p1, d1);
    sub3(q2, p2, d2);
    sub3(p1, p2, r);
    double a = dot3(d1, d1), e = dot3(d2, d2), f = dot3(d2, r);
    double c = dot3(d1, r), b = dot3(d1, d2);
    double denom = a * e - b * b;
    double s, t;
    if (denom > ORA_EE_PARALLEL * a * e)
        s = clamp01((b * f - c * e) / denom);
    else
        s = 0.0;
    t = (b * s + f) / e;
    if (t < 0.0) {
        t = 0.0;
        s = clamp01(-c / a);
    } else if (t > 1.0) {
        t = 1.0;
        s = clamp01((b - c) / a);
    }
    int s_end = (s == 0.0) ? 0 : (s == 1.0 ? 1 : -1);
    int t_end = (t == 0.0) ? 0 : (t == 1.0 ? 1 : -1);
    if (s_end >= 0 && t_end >= 0) return s_end * 2 + t_end; /* 0..3 */
    if (s_end >= 0) return 4 + s_end;                        /* A end vs edge B */
    if (t_end >= 0) return 6 + t_end;                        /* B end vs edge A */
    return 8;
}

/* Solve the normal equations for beta*, return r at beta*, and the
 * coefficients c(beta*) and the parameter directions u_m = sum_k Dm_k x_k. */
static void dist_solve(const dist_spec *sp, const double *x12, double *r, double *c, double u[2][3],
                       double G[2][2])
{
    double r0[3] = {0, 0, 0};
    for (int k = 0; k < 4; ++k)
        for (int i = 0; i < 3; ++i) r0[i] += sp->c0[k] * x12[k * 3 + i];
    for (int m = 0; m < sp->np; ++m) {
        for (int i = 0; i < 3; ++i) u[m][i] = 0.0;
        for (int k = 0; k < 4; ++k)
            for (int i = 0; i < 3; ++i) u[m][i] += sp->D[m][k] * x12[k * 3 + i];
    }
    double beta[2] = {0, 0};
    if (sp->np == 1) {
        G[0][0] = dot3(u[0], u[0]);
        beta[0] = -dot3(u[0], r0) / G[0][0];
    } else if (sp->np == 2) {
        G[0][0] = dot3(u[0], u[0]);
        G[0][1] = dot3(u[0], u[1]);
        G[1][0] = G[0][1];
        G[1][1] = dot3(u[1], u[1]);
        double b0 = -dot3(u[0], r0), b1 = -dot3(u[1], r0);
        double det = G[0][0] * G[1][1] - G[0][1] * G[1][0];
        beta[0] = (b0 * G[1][1] - G[0][1] * b1) / det;
        beta[1] = (G[0][0] * b1 - G[1][0] * b0) / det;
    }
    for (int i = 0; i < 3; ++i) {
        r[i] = r0[i];
        for (int m = 0; m < sp->np; ++m) r[i] += beta[m] * u[m][i];
    }
    for (int k = 0; k < 4; ++k) {
        c[k] = sp->c0[k];
        for (int m = 0; m < sp->np; ++m) c[k] += beta[m] * sp->D[m][k];
    }
}

static double dist_sq_of_type(const dist_spec *sp, const double *x12)
{
    double r[3], c[4], u[2][3], G[2][2];
    dist_solve(sp, x12, r, c, u, G);
    return dot3(r, r);
}

double ora_pt_distance(const double *x12, int32_t *type)
{
    int t = pt_type(x12);
    if (type) *type = t;
    dist_spec sp = pt_spec(t);
    return sqrt(dist_sq_of_type(&sp, x12));
}

double ora_ee_distance(const double *x12, int32_t *type)
{
    int t = ee_type(x12);
    if (type) *type = t;
    dist_spec sp = ee_spec(t);
    return sqrt(dist_sq_of_type(&sp, x12));
}

/* Gradient and Hessian of s(x) = |r(x, beta*(x))|^2 at fixed type. With
 * s_beta = 0 at beta* (implicit function theorem):
 *   grad s = s_x,  hess s = s_xx - s_xb s_bb^-1 s_bx,
 * s_x[k] = 2 c_k r, s_xx[k,l] = 2 c_k c_l I, s_bb = 2 G,
 * s_xb[k,m] = 2 (Dm_k r + c_k u_m). Returns s. */
static double dist_sq_derivs(const dist_spec *sp, const double *x12, double *gs, double *Hs)
{
    double r[3], c[4], u[2][3], G[2][2];
    dist_solve(sp, x12, r, c, u, G);
    for (int k = 0; k < 4; ++k)
        for (int i = 0; i < 3; ++i) gs[k * 3 + i] = 2.0 * c[k] * r[i];
    for (int a = 0; a < 12; ++a)
        for (int b = 0; b < 12; ++b) Hs[a * 12 + b] = 0.0;
    for (int k = 0; k < 4; ++k)
        for (int l = 0; l < 4; ++l)
            for (int i = 0; i < 3; ++i) Hs[(k * 3 + i) * 12 + (l * 3 + i)] = 2.0 * c[k] * c[l];
    if (sp->np > 0) {
        double W[12][2];
        for (int k = 0; k < 4; ++k)
            for (int i = 0; i < 3; ++i)
                for (int m = 0; m < sp->np; ++m)
                    W[k * 3 + i][m] = 2.0 * (sp->D[m][k] * r[i] + c[k] * u[m][i]);
        double Sinv[2][2];
        if (sp->np == 1) {
            Sinv[0][0] = 1.0 / (2.0 * G[0][0]);
        } else {
            double S00 = 2.0 * G[0][0], S01 = 2.0 * G[0][1], S11 = 2.0 * G[1][1];
            double det = S00 * S11 - S01 * S01;
            Sinv[0][0] = S11 / det;
            Sinv[1][1] = S00 / det;
            Sinv[0][1] = -S01 / det;
            Sinv[1][0] = -S01 / det;
        }
        for (int a = 0; a < 12; ++a)
            for (int b = 0; b < 12; ++b) {
                double acc = 0.0;
                for (int m = 0; m < sp->np; ++m)
                    for (int n = 0; n < sp->np; ++n) acc += W[a][m] * Sinv[m][n] * W[b][n];
                Hs[a * 12 + b] -= acc;
            }
    }
    return dot3(r, r);
}

/* d = sqrt(s): grad d = grad s / (2d), hess d = hess s / (2d) - gs gs^T / (4 d^3) */
double ora_distance_derivs(int32_t kind, const double *x12, double *gd, double *Hd)
{
    dist_spec sp = kind == 0 ? pt_spec(pt_type(x12)) : ee_spec(ee_type(x12));
    double gs[12], Hs[144];
    double s = dist_sq_derivs(&sp, x12, gs, Hs);
    double d = sqrt(s);
    for (int a = 0; a < 12; ++a) gd[a] = gs[a] / (2.0 * d);
    for (int a = 0; a < 12; ++a)
        for (int b = 0; b < 12; ++b)
            Hd[a * 12 + b] = Hs[a * 12 + b] / (2.0 * d) - gs[a] * gs[b] / (4.0 * d * d * d);
    return d;
}

/* ======================================================================== */
/* barrier and mollifier                                                     */
/* ======================================================================== */

/* b(d) = -(d - dhat)^2 ln(d / dhat) for 0 < d < dhat, 0 beyond; b3 = {b, b', b''} */
void ora_barrier_scalar(double d, double dhat, double *b3)
{
    if (d >= dhat) {
        b3[0] = b3[1] = b3[2] = 0.0;
        return;
    }
    if (!(d > 0.0)) {
        b3[0] = INFINITY;
        b3[1] = -INFINITY;
        b3[2] = INFINITY;
        return;
    }
    double t = d - dhat, L = log(d / dhat);
    b3[0] = -t * t * L;
    b3[1] = -2.0 * t * L - t * t / d;
    b3[2] = -2.0 * L - 4.0 * t / d + t * t / (d * d);
}

/* EE mollifier m(c) = -c^2/eps^2 + 2c/eps for c < eps, 1 otherwise, with
 * c = |e0 x e1|^2. m3 = {m, dm/dc, d2m/dc2}. */
static void mollifier(double c, double eps, double *m3)
{
    if (c < eps) {
        m3[0] = -c * c / (eps * eps) + 2.0 * c / eps;
        m3[1] = -2.0 * c / (eps * eps) + 2.0 / eps;
        m3[2] = -2.0 / (eps * eps);
    } else {
        m3[0] = 1.0;
        m3[1] = 0.0;
        m3[2] = 0.0;
    }
}

/* c = |a x b|^2 with a = x1 - x0, b = x3 - x2, and its gradient/Hessian in x */
static double ee_cross_sq(const double *x12, double *gc, double *Hc)
{
    double a[3], b[3], axb[3];
    sub3(x12 + 3, x12, a);
    sub3(x12 + 9, x12 + 6, b);
    cross3(a, b, axb);
    double c = dot3(axb, axb);
    if (!gc) return c;
    double aa = dot3(a, a), bb = dot3(b, b), ab = dot3(a, b);
    double ga[3], gb[3];
    for (int i = 0; i < 3; ++i) {
        ga[i] = 2.0 * bb * a[i] - 2.0 * ab * b[i];
        gb[i] = 2.0 * aa * b[i] - 2.0 * ab * a[i];
    }
    for (int i = 0; i < 3; ++i) {
        gc[0 + i] = -ga[i];
        gc[3 + i] = ga[i];
        gc[6 + i] = -gb[i];
        gc[9 + i] = gb[i];
    }
    /* second derivatives in (a,b) */
    double Haa[9], Hbb[9], Hab[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double dij = (i == j) ? 1.0 : 0.0;
            Haa[i * 3 + j] = 2.0 * bb * dij - 2.0 * b[i] * b[j];
            Hbb[i * 3 + j] = 2.0 * aa * dij - 2.0 * a[i] * a[j];
            Hab[i * 3 + j] = 4.0 * a[i] * b[j] - 2.0 * ab * dij - 2.0 * b[i] * a[j];
        }
    /* chain rule: a = x1 - x0 (signs -1,+1 on vertices 0,1), b = x3 - x2 */
    const double sa[4] = {-1, 1, 0, 0}, sb[4] = {0, 0, -1, 1};
    for (int k = 0; k < 4; ++k)
        for (int l = 0; l < 4; ++l)
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    double v = sa[k] * sa[l] * Haa[i * 3 + j] + sb[k] * sb[l] * Hbb[i * 3 + j] +
                               sa[k] * sb[l] * Hab[i * 3 + j] + sb[k] * sa[l] * Hab[j * 3 + i];
                    Hc[(k * 3 + i) * 12 + (l * 3 + j)] = v;
                }
    return c;
}

/* kappa * w * b(d) for one pair with gradient and Hessian. w = 1 for PT;
 * w = mollifier for EE. project: 0 the exact Hessian, 1 its PSD projection,
 * 2 the Gauss-Newton form kappa w b''(d) grad d grad d^T. The paper names
 * GIPC's Gauss-Newton treatment of the barrier only by its title, so this form
 * is a reading: of the exact Hessian it keeps the one term that is an outer
 * product of first derivatives with a non-negative weight (b'' > 0 on
 * (0, dhat), w >= 0) and drops the distance curvature b' grad^2 d, the
 * mollifier's own curvature and the mollifier-distance cross terms; it is PSD
 * with rank one by construction. The gradient is exact in every mode.
 * Returns the energy. */
double ora_pair_barrier(int32_t kind, const double *x12, double dhat, double kappa, double eps_x,
                        int32_t project, double *g12, double *H144)
{
    double gd[12], Hd[144];
    double d = ora_distance_derivs(kind, x12, gd, Hd);
    double b3[3];
    ora_barrier_scalar(d, dhat, b3);
    if (d >= dhat) {
        if (g12) memset(g12, 0, sizeof(double) * 12);
        if (H144) memset(H144, 0, sizeof(double) * 144);
        return 0.0;
    }
    double w = 1.0;
    double m3[3] = {1.0, 0.0, 0.0}, gc[12], Hc[144];
    if (kind == 1) {
        double c = ee_cross_sq(x12, gc, Hc);
        mollifier(c, eps_x, m3);
        w = m3[0];
    }
    double E = kappa * w * b3[0];
    if (g12)
        for (int a = 0; a < 12; ++a) {
            double v = w * b3[1] * gd[a];
            if (kind == 1) v += b3[0] * m3[1] * gc[a];
            g12[a] = kappa * v;
        }
    if (H144 && project == 2) {
        for (int a = 0; a < 12; ++a)
            for (int b = 0; b < 12; ++b) H144[a * 12 + b] = kappa * (w * b3[2] * gd[a] * gd[b]);
    } else if (H144) {
        for (int a = 0; a < 12; ++a)
            for (int b = 0; b < 12; ++b) {
                double v = w * (b3[2] * gd[a] * gd[b] + b3[1] * Hd[a * 12 + b]);
                if (kind == 1) {
                    v += b3[0] * (m3[2] * gc[a] * gc[b] + m3[1] * Hc[a * 12 + b]);
                    v += b3[1] * m3[1] * (gc[a] * gd[b] + gd[a] * gc[b]);
                }
                H144[a * 12 + b] = kappa * v;
            }
        if (project) ora_psd_project(12, H144);
    }
    return E;
}

/* ======================================================================== */
/* additive CCD (conservative advancement)                                   */
/* ======================================================================== */
/* Additive CCD of Li, Kaufman and Jiang ("Codimensional IPC", 2021): remove
 * the mean displacement, bound the relative motion by l_p, then advance in
 * safe sub-steps of 0.9 d / l_p until the distance falls below the keep gap
 * s * d0 (return the last safe time) or the time passes tmax (no impact). */
double ora_accd(int32_t kind, const double *x12, const double *p12, double s, double tmax,
                int32_t max_iter)
{
    double x[12], p[12], pbar[3] = {0, 0, 0};
    memcpy(x, x12, sizeof x);
    for (int k = 0; k < 4; ++k)
        for (int i = 0; i < 3; ++i) pbar[i] += p12[k * 3 + i];
    for (int i = 0; i < 3; ++i) pbar[i] /= 4.0;
    double len[4];
    for (int k = 0; k < 4; ++k) {
        for (int i = 0; i < 3; ++i) p[k * 3 + i] = p12[k * 3 + i] - pbar[i];
        len[k] = sqrt(dot3(p + k * 3, p + k * 3));
    }
    double lp;
    if (kind == 0) {
        double m = len[1];
        if (len[2] > m) m = len[2];
        if (len[3] > m) m = len[3];
        lp = len[0] + m;
    } else {
        lp = (len[0] > len[1] ? len[0] : len[1]) + (len[2] > len[3] ? len[2] : len[3]);
    }
    if (lp == 0.0) return tmax;
    double d = kind == 0 ? ora_pt_distance(x, NULL) : ora_ee_distance(x, NULL);
    double g = s * d;
    double t = 0.0;
    double tl = (1.0 - s) * d / lp;
    for (int it = 0; it < max_iter; ++it) {
        for (int i = 0; i < 12; ++i) x[i] += tl * p[i];
        d = kind == 0 ? ora_pt_distance(x, NULL) : ora_ee_distance(x, NULL);
        if (t > 0.0 && d < g) break;
        t += tl;
        if (t > tmax) return tmax;
        tl = 0.9 * d / lp;
    }
    return t;
}

/* ======================================================================== */
/* scene                                                                     */
/* ======================================================================== */

struct ora_scene {
    ora_params prm;
    int n, n_gel, n_tet, n_ind;
    double mu, lam;
    double *X;      /* rest positions of all vertices (indenter at pose0) */
    double *Yloc;   /* indenter local vertices */
    double *pose0;  /* 12 */
    int32_t *T;
    uint8_t *fixed; /* per vertex; indenter vertices are never fixed */
    double *Bm;     /* Dm^-1 per tet (9) */
    double *vol, *mass;
    /* surface primitives */
    int n_pts, n_edges, n_tris, n_gel_tris, n_gel_edges;
    int32_t *pts;   /* vertex ids */
    int32_t *edges; /* 2 per edge */
    int32_t *tris;  /* 3 per tri */
    double *edge_rest_sq;
    /* state */
    double *x, *v;
    /* step context */
    double *xt, *xtilde, *yhat; /* yhat: 3 per vertex, meaningful for indenter vertices */
    double *lam_al;             /* augmented-Lagrangian multipliers, 3 per vertex (indenter vertices) */
    int al_step;                /* 1: the multipliers just changed; the next iteration takes its step */
    /* lagged friction set of the step (pairs active at x^t) */
    int n_fric;
    int32_t *fric_v;  /* 4 per pair */
    double *fric_c;   /* 4 per pair: closest-point coefficients at x^t */
    double *fric_nrm; /* 3 per pair: unit contact normal at x^t */
    double *fric_lam; /* normal-force magnitude at x^t */
    /* attachment: free gel vertices pulled to case pose o rest position */
    uint8_t *attached; /* per gel vertex, NULL: none */
    double case_pose[12];
};

static int is_attached(const ora_scene *s, int i);

typedef struct {
    int32_t a, b, c, src;
} rec4;

static int cmp_rec3(const void *p, const void *q)
{
    const rec4 *A = (const rec4 *)p, *B = (const rec4 *)q;
    if (A->a != B->a) return A->a < B->a ? -1 : 1;
    if (A->b != B->b) return A->b < B->b ? -1 : 1;
    if (A->c != B->c) return A->c < B->c ? -1 : 1;
    return 0;
}

/* rotate (a,b,c) so the smallest id comes first, keeping orientation */
static void rotate_min_first(int32_t *t)
{
    int32_t a = t[0], b = t[1], c = t[2];
    if (b < a && b < c) {
        t[0] = b; t[1] = c; t[2] = a;
    } else if (c < a && c < b) {
        t[0] = c; t[1] = a; t[2] = b;
    }
}

static void sort_tris(int32_t *tris, int nt)
{
    rec4 *r = (rec4 *)malloc(sizeof(rec4) * (nt > 0 ? nt : 1));
    for (int i = 0; i < nt; ++i) {
        rotate_min_first(tris + 3 * i);
        r[i].a = tris[3 * i];
        r[i].b = tris[3 * i + 1];
        r[i].c = tris[3 * i + 2];
        r[i].src = i;
    }
    qsort(r, nt, sizeof(rec4), cmp_rec3);
    for (int i = 0; i < nt; ++i) {
        tris[3 * i] = r[i].a;
        tris[3 * i + 1] = r[i].b;
        tris[3 * i + 2] = r[i].c;
    }
    free(r);
}

/* unique sorted (min,max) edges of a triangle list; returns count */
static int tri_edges(const int32_t *tris, int nt, int32_t **out)
{
    rec4 *r = (rec4 *)malloc(sizeof(rec4) * (3 * nt > 0 ? 3 * nt : 1));
    for (int i = 0; i < nt; ++i)
        for (int k = 0; k < 3; ++k) {
            int32_t a = tris[3 * i + k], b = tris[3 * i + (k + 1) % 3];
            r[3 * i + k].a = a < b ? a : b;
            r[3 * i + k].b = a < b ? b : a;
            r[3 * i + k].c = 0;
            r[3 * i + k].src = 0;
        }
    qsort(r, 3 * nt, sizeof(rec4), cmp_rec3);
    int32_t *e = (int32_t *)malloc(sizeof(int32_t) * 2 * (3 * nt > 0 ? 3 * nt : 1));
    int ne = 0;
    for (int i = 0; i < 3 * nt; ++i) {
        if (i > 0 && r[i].a == r[i - 1].a && r[i].b == r[i - 1].b) continue;
        e[2 * ne] = r[i].a;
        e[2 * ne + 1] = r[i].b;
        ++ne;
    }
    free(r);
    *out = e;
    return ne;
}

static void apply_pose(const double *P, const double *y, double *o)
{
    for (int i = 0; i < 3; ++i)
        o[i] = P[i * 4 + 0] * y[0] + P[i * 4 + 1] * y[1] + P[i * 4 + 2] * y[2] + P[i * 4 + 3];
}

ora_scene *ora_scene_create(int32_t n_gel, const double *X, int32_t n_tet, const int32_t *T,
                            const uint8_t *fixed, int32_t n_ind, const double *Y_local,
                            int32_t n_ind_tri, const int32_t *ind_tri, const double *pose0,
                            const ora_params *prm, int32_t *status)
{
    *status = ORA_OK;
    if (n_gel <= 0 || n_tet <= 0 || n_ind < 0 || !X || !T || !prm) {
        *status = ORA_E_INVALID_ARG;
        return NULL;
    }
    for (int e = 0; e < 4 * n_tet; ++e)
        if (T[e] < 0 || T[e] >= n_gel) {
            *status = ORA_E_BAD_MESH;
            return NULL;
        }
    for (int e = 0; e < 3 * n_ind_tri; ++e)
        if (ind_tri[e] < 0 || ind_tri[e] >= n_ind) {
            *status = ORA_E_BAD_MESH;
            return NULL;
        }
    ora_scene *s = (ora_scene *)calloc(1, sizeof(ora_scene));
    s->prm = *prm;
    s->n_gel = n_gel;
    s->n_ind = n_ind;
    s->n = n_gel + n_ind;
    s->n_tet = n_tet;
    s->mu = prm->E / (2.0 * (1.0 + prm->nu));
    s->lam = prm->E * prm->nu / ((1.0 + prm->nu) * (1.0 - 2.0 * prm->nu));
    int n = s->n;
    s->X = (double *)malloc(sizeof(double) * 3 * n);
    s->Yloc = (double *)malloc(sizeof(double) * 3 * (n_ind > 0 ? n_ind : 1));
    s->pose0 = (double *)malloc(sizeof(double) * 12);
    memcpy(s->pose0, pose0, sizeof(double) * 12);
    for (int k = 0; k < 12; ++k) s->case_pose[k] = (k % 5 == 0) ? 1.0 : 0.0; /* identity */
    memcpy(s->X, X, sizeof(double) * 3 * n_gel);
    if (n_ind) memcpy(s->Yloc, Y_local, sizeof(double) * 3 * n_ind);
    for (int j = 0; j < n_ind; ++j) apply_pose(pose0, Y_local + 3 * j, s->X + 3 * (n_gel + j));
    s->T = (int32_t *)malloc(sizeof(int32_t) * 4 * n_tet);
    memcpy(s->T, T, sizeof(int32_t) * 4 * n_tet);
    s->fixed = (uint8_t *)calloc(n, 1);
    if (fixed) memcpy(s->fixed, fixed, n_gel);

    /* rest shape: Dm = [X1-X0, X2-X0, X3-X0] (columns), V = det(Dm)/6, Bm = Dm^-1 */
    s->Bm = (double *)malloc(sizeof(double) * 9 * n_tet);
    s->vol = (double *)malloc(sizeof(double) * n_tet);
    s->mass = (double *)calloc(n, sizeof(double));
    for (int e = 0; e < n_tet; ++e) {
        const int32_t *t = T + 4 * e;
        double Dm[9];
        for (int i = 0; i < 3; ++i)
            for (int c = 0; c < 3; ++c) Dm[i * 3 + c] = X[3 * t[c + 1] + i] - X[3 * t[0] + i];
        double V = det3(Dm) / 6.0;
        if (!(V > 0.0)) {
            *status = ORA_E_BAD_MESH;
            ora_scene_destroy(s);
            return NULL;
        }
        inv3(Dm, s->Bm + 9 * e);
        s->vol[e] = V;
        for (int k = 0; k < 4; ++k) s->mass[t[k]] += prm->rho * V / 4.0;
    }

    /* boundary faces: tet faces used exactly once, oriented outward */
    static const int FACE[4][3] = {{1, 2, 3}, {0, 3, 2}, {0, 1, 3}, {0, 2, 1}};
    rec4 *fr = (rec4 *)malloc(sizeof(rec4) * 4 * n_tet);
    int32_t *fo = (int32_t *)malloc(sizeof(int32_t) * 12 * n_tet);
    for (int e = 0; e < n_tet; ++e)
        for (int f = 0; f < 4; ++f) {
            int32_t v[3] = {T[4 * e + FACE[f][0]], T[4 * e + FACE[f][1]], T[4 * e + FACE[f][2]]};
            memcpy(fo + 3 * (4 * e + f), v, sizeof v);
            /* sorted key */
            int32_t a = v[0], b = v[1], c = v[2], tmp;
            if (a > b) { tmp = a; a = b; b = tmp; }
            if (b > c) { tmp = b; b = c; c = tmp; }
            if (a > b) { tmp = a; a = b; b = tmp; }
            fr[4 * e + f].a = a;
            fr[4 * e + f].b = b;
            fr[4 * e + f].c = c;
            fr[4 * e + f].src = 4 * e + f;
        }
    qsort(fr, 4 * n_tet, sizeof(rec4), cmp_rec3);
    int nb = 0;
    int32_t *btris = (int32_t *)malloc(sizeof(int32_t) * 3 * (4 * n_tet + n_ind_tri + 1));
    for (int i = 0; i < 4 * n_tet;) {
        int j = i + 1;
        while (j < 4 * n_tet && cmp_rec3(&fr[i], &fr[j]) == 0) ++j;
        if (j - i == 1) {
            memcpy(btris + 3 * nb, fo + 3 * fr[i].src, sizeof(int32_t) * 3);
            ++nb;
        } else if (j - i > 2) {
            *status = ORA_E_BAD_MESH; /* non-manifold */
        }
        i = j;
    }
    free(fr);
    free(fo);
    if (*status != ORA_OK) {
        free(btris);
        ora_scene_destroy(s);
        return NULL;
    }
    sort_tris(btris, nb);
    s->n_gel_tris = nb;
    int32_t *itris = btris + 3 * nb;
    for (int i = 0; i < n_ind_tri; ++i)
        for (int k = 0; k < 3; ++k) itris[3 * i + k] = ind_tri[3 * i + k] + n_gel;
    sort_tris(itris, n_ind_tri);
    s->n_tris = nb + n_ind_tri;
    s->tris = btris;

    int32_t *ge, *ie;
    int nge = tri_edges(btris, nb, &ge);
    int nie = tri_edges(itris, n_ind_tri, &ie);
    s->n_gel_edges = nge;
    s->n_edges = nge + nie;
    s->edges = (int32_t *)malloc(sizeof(int32_t) * 2 * (s->n_edges > 0 ? s->n_edges : 1));
    memcpy(s->edges, ge, sizeof(int32_t) * 2 * nge);
    memcpy(s->edges + 2 * nge, ie, sizeof(int32_t) * 2 * nie);
    free(ge);
    free(ie);
    s->edge_rest_sq = (double *)malloc(sizeof(double) * (s->n_edges > 0 ? s->n_edges : 1));
    for (int i = 0; i < s->n_edges; ++i) {
        double d[3];
        sub3(s->X + 3 * s->edges[2 * i + 1], s->X + 3 * s->edges[2 * i], d);
        s->edge_rest_sq[i] = dot3(d, d);
    }

    /* points: vertices of any surface triangle, ascending */
    uint8_t *on = (uint8_t *)calloc(n, 1);
    for (int i = 0; i < 3 * s->n_tris; ++i) on[s->tris[i]] = 1;
    s->n_pts = 0;
    for (int i = 0; i < n; ++i) s->n_pts += on[i];
    s->pts = (int32_t *)malloc(sizeof(int32_t) * (s->n_pts > 0 ? s->n_pts : 1));
    for (int i = 0, k = 0; i < n; ++i)
        if (on[i]) s->pts[k++] = i;
    free(on);

    s->x = (double *)malloc(sizeof(double) * 3 * n);
    s->v = (double *)calloc(3 * n, sizeof(double));
    s->xt = (double *)malloc(sizeof(double) * 3 * n);
    s->xtilde = (double *)malloc(sizeof(double) * 3 * n);
    s->yhat = (double *)malloc(sizeof(double) * 3 * n);
    s->lam_al = (double *)calloc(3 * (size_t)n, sizeof(double));
    memcpy(s->x, s->X, sizeof(double) * 3 * n);
    memcpy(s->xt, s->X, sizeof(double) * 3 * n);
    memcpy(s->xtilde, s->X, sizeof(double) * 3 * n);
    memcpy(s->yhat, s->X, sizeof(double) * 3 * n);
    return s;
}

void ora_scene_destroy(ora_scene *s)
{
    if (!s) return;
    free(s->X); free(s->Yloc); free(s->pose0); free(s->T); free(s->fixed);
    free(s->Bm); free(s->vol); free(s->mass);
    free(s->pts); free(s->edges); free(s->tris); free(s->edge_rest_sq);
    free(s->x); free(s->v); free(s->xt); free(s->xtilde); free(s->yhat); free(s->lam_al);
    free(s->attached);
    free(s->fric_v); free(s->fric_c); free(s->fric_nrm); free(s->fric_lam);
    free(s);
}

void ora_scene_sizes(const ora_scene *s, int32_t *o)
{
    o[0] = s->n; o[1] = s->n_gel; o[2] = s->n_tet; o[3] = s->n_pts;
    o[4] = s->n_edges; o[5] = s->n_tris; o[6] = s->n_ind; o[7] = s->n_gel_tris;
}

void ora_scene_surface(const ora_scene *s, int32_t *points, int32_t *edges, int32_t *tris)
{
    if (points) memcpy(points, s->pts, sizeof(int32_t) * s->n_pts);
    if (edges) memcpy(edges, s->edges, sizeof(int32_t) * 2 * s->n_edges);
    if (tris) memcpy(tris, s->tris, sizeof(int32_t) * 3 * s->n_tris);
}

void ora_scene_rest(const ora_scene *s, double *vol, double *mass)
{
    if (vol) memcpy(vol, s->vol, sizeof(double) * s->n_tet);
    if (mass) memcpy(mass, s->mass, sizeof(double) * s->n);
}

void ora_get_x(const ora_scene *s, double *x) { memcpy(x, s->x, sizeof(double) * 3 * s->n); }
void ora_set_x(ora_scene *s, const double *x) { memcpy(s->x, x, sizeof(double) * 3 * s->n); }
void ora_get_v(const ora_scene *s, double *v) { memcpy(v, s->v, sizeof(double) * 3 * s->n); }
void ora_set_v(ora_scene *s, const double *v) { memcpy(s->v, v, sizeof(double) * 3 * s->n); }

/* reset: positions to rest, velocities to zero (paper section "General GIPC
 * Simulation Pipeline": saved initial positions restored, velocities 0) */
void ora_reset(ora_scene *s)
{
    memcpy(s->x, s->X, sizeof(double) * 3 * s->n);
    memset(s->v, 0, sizeof(double) * 3 * s->n);
    memcpy(s->xt, s->X, sizeof(double) * 3 * s->n);
    memcpy(s->xtilde, s->X, sizeof(double) * 3 * s->n);
    memcpy(s->yhat, s->X, sizeof(double) * 3 * s->n);
    s->n_fric = 0;
    for (int k = 0; k < 12; ++k) s->case_pose[k] = (k % 5 == 0) ? 1.0 : 0.0;
}

/* ======================================================================== */
/* candidates: the closed box-overlap predicate over all pairs              */
/* ======================================================================== */

/* box of a primitive with vertices vs[0..nv): [min - r, max + r] over x (and
 * x + p when p != NULL), r = dhat / 2 */
static void prim_box(const double *x, const double *p, const int32_t *vs, int nv, double r,
                     double *lo, double *hi)
{
    for (int i = 0; i < 3; ++i) {
        double mn = x[3 * vs[0] + i], mx = mn;
        for (int k = 0; k < nv; ++k) {
            double a = x[3 * vs[k] + i];
            if (a < mn) mn = a;
            if (a > mx) mx = a;
            if (p) {
                double b = x[3 * vs[k] + i] + p[3 * vs[k] + i];
                if (b < mn) mn = b;
                if (b > mx) mx = b;
            }
        }
        lo[i] = mn - r;
        hi[i] = mx + r;
    }
}

static int boxes_overlap(const double *alo, const double *ahi, const double *blo, const double *bhi)
{
    for (int i = 0; i < 3; ++i)
        if (!(alo[i] <= bhi[i] && blo[i] <= ahi[i])) return 0;
    return 1;
}

typedef struct {
    int32_t *v;
    int n, cap;
} ivec;
static void ivec_push3(ivec *a, int32_t t, int32_t x, int32_t y)
{
    if (a->n + 3 > a->cap) {
        a->cap = a->cap ? 2 * a->cap : 3 * 1024;
        a->v = (int32_t *)realloc(a->v, sizeof(int32_t) * a->cap);
    }
    a->v[a->n++] = t;
    a->v[a->n++] = x;
    a->v[a->n++] = y;
}

/* Pair rules: PT pairs take every surface point against every surface
 * triangle, EE pairs every edge against every later edge. Skipped: pairs
 * sharing a vertex, indenter-indenter pairs, gel-gel pairs without
 * self-contact, and pairs whose four vertices are all fixed. */
static void candidates_list(const ora_scene *s, const double *x, const double *p, ivec *out)
{
    double r = 0.5 * s->prm.dhat;
    int ng = s->n_gel;
    double *tlo = (double *)malloc(sizeof(double) * 3 * (s->n_tris + 1));
    double *thi = (double *)malloc(sizeof(double) * 3 * (s->n_tris + 1));
    for (int t = 0; t < s->n_tris; ++t) prim_box(x, p, s->tris + 3 * t, 3, r, tlo + 3 * t, thi + 3 * t);
    for (int ip = 0; ip < s->n_pts; ++ip) {
        int32_t a = s->pts[ip];
        double lo[3], hi[3];
        prim_box(x, p, &a, 1, r, lo, hi);
        for (int t = 0; t < s->n_tris; ++t) {
            const int32_t *tv = s->tris + 3 * t;
            if (tv[0] == a || tv[1] == a || tv[2] == a) continue;
            int a_ind = a >= ng, t_ind = tv[0] >= ng;
            if (a_ind && t_ind) continue;
            if (!a_ind && !t_ind && !s->prm.self_contact) continue;
            if (s->fixed[a] && s->fixed[tv[0]] && s->fixed[tv[1]] && s->fixed[tv[2]]) continue;
            if (boxes_overlap(lo, hi, tlo + 3 * t, thi + 3 * t)) ivec_push3(out, 0, a, t);
        }
    }
    free(tlo);
    free(thi);
    double *elo = (double *)malloc(sizeof(double) * 3 * (s->n_edges + 1));
    double *ehi = (double *)malloc(sizeof(double) * 3 * (s->n_edges + 1));
    for (int e = 0; e < s->n_edges; ++e) prim_box(x, p, s->edges + 2 * e, 2, r, elo + 3 * e, ehi + 3 * e);
    for (int ea = 0; ea < s->n_edges; ++ea) {
        const int32_t *va = s->edges + 2 * ea;
        for (int eb = ea + 1; eb < s->n_edges; ++eb) {
            const int32_t *vb = s->edges + 2 * eb;
            if (va[0] == vb[0] || va[0] == vb[1] || va[1] == vb[0] || va[1] == vb[1]) continue;
            int a_ind = va[0] >= ng, b_ind = vb[0] >= ng;
            if (a_ind && b_ind) continue;
            if (!a_ind && !b_ind && !s->prm.self_contact) continue;
            if (s->fixed[va[0]] && s->fixed[va[1]] && s->fixed[vb[0]] && s->fixed[vb[1]]) continue;
            if (boxes_overlap(elo + 3 * ea, ehi + 3 * ea, elo + 3 * eb, ehi + 3 * eb))
                ivec_push3(out, 1, ea, eb);
        }
    }
    free(elo);
    free(ehi);
}

int32_t ora_candidates(const ora_scene *s, const double *x, const double *p, int32_t *out, int32_t cap)
{
    ivec c = {0, 0, 0};
    candidates_list(s, x, p, &c);
    int nc = c.n / 3;
    int w = nc < cap ? nc : cap;
    if (out && w > 0) memcpy(out, c.v, sizeof(int32_t) * 3 * w);
    free(c.v);
    return nc;
}

/* the 4 vertex ids of a candidate: PT (p, t0, t1, t2), EE (a0, a1, b0, b1) */
static void cand_verts(const ora_scene *s, const int32_t *c, int32_t *v)
{
    if (c[0] == 0) {
        v[0] = c[1];
        v[1] = s->tris[3 * c[2]];
        v[2] = s->tris[3 * c[2] + 1];
        v[3] = s->tris[3 * c[2] + 2];
    } else {
        v[0] = s->edges[2 * c[1]];
        v[1] = s->edges[2 * c[1] + 1];
        v[2] = s->edges[2 * c[2]];
        v[3] = s->edges[2 * c[2] + 1];
    }
}

static void gather12(const double *x, const int32_t *v, double *x12)
{
    for (int k = 0; k < 4; ++k)
        for (int i = 0; i < 3; ++i) x12[k * 3 + i] = x[3 * v[k] + i];
}

static double cand_eps_x(const ora_scene *s, const int32_t *c)
{
    return ORA_MOLLIFIER_FACTOR * s->edge_rest_sq[c[1]] * s->edge_rest_sq[c[2]];
}

void ora_candidate_distances(const ora_scene *s, const double *x, int32_t nc, const int32_t *cand,
                             double *d, int32_t *type)
{
    for (int i = 0; i < nc; ++i) {
        int32_t v[4];
        double x12[12];
        cand_verts(s, cand + 3 * i, v);
        gather12(x, v, x12);
        int32_t t;
        d[i] = cand[3 * i] == 0 ? ora_pt_distance(x12, &t) : ora_ee_distance(x12, &t);
        if (type) type[i] = t;
    }
}

/* ======================================================================== */
/* incremental potential                                                     */
/* ======================================================================== */
/* Phi(x) = sum_i m_i/(2h^2) |x_i - xtilde_i|^2 + sum_e V_e Psi(F_e)
 *        + sum_j k_t/2 |y_j - yhat_j|^2 + kappa sum_c w_c b(d_c)
 * (backward Euler incremental potential divided by h^2; barrier unsquared).
 * Summed with Neumaier compensation in the order: vertices, tets, indenter
 * vertices, candidates. */
static double friction_energy(const ora_scene *s, const double *x);

static double energy_with(const ora_scene *s, const double *x, const ivec *cand)
{
    nsum acc = {0.0, 0.0};
    double h2 = s->prm.h * s->prm.h;
    for (int i = 0; i < s->n_gel; ++i) {
        if (s->fixed[i]) continue;
        double d[3];
        sub3(x + 3 * i, s->xtilde + 3 * i, d);
        nsum_add(&acc, s->mass[i] / (2.0 * h2) * dot3(d, d));
    }
    for (int e = 0; e < s->n_tet; ++e) {
        double x12[12], E;
        gather12(x, s->T + 4 * e, x12);
        ora_tet_elastic(x12, s->Bm + 9 * e, s->vol[e], s->mu, s->lam, &E, NULL, NULL);
        if (!isfinite(E)) return INFINITY;
        nsum_add(&acc, E);
    }
    for (int j = s->n_gel; j < s->n; ++j) {
        double d[3];
        sub3(x + 3 * j, s->yhat + 3 * j, d);
        nsum_add(&acc, 0.5 * s->prm.k_target * dot3(d, d));
        if (s->prm.target_al) nsum_add(&acc, -dot3(s->lam_al + 3 * j, d));
    }
    for (int i = 0; i < s->n_gel; ++i) {
        if (!is_attached(s, i)) continue;
        double d[3];
        sub3(x + 3 * i, s->yhat + 3 * i, d);
        nsum_add(&acc, 0.5 * s->prm.k_target * dot3(d, d));
    }
    for (int i = 0; i < cand->n / 3; ++i) {
        const int32_t *c = cand->v + 3 * i;
        int32_t v[4];
        double x12[12];
        cand_verts(s, c, v);
        gather12(x, v, x12);
        double d = c[0] == 0 ? ora_pt_distance(x12, NULL) : ora_ee_distance(x12, NULL);
        if (!(d > 0.0)) return INFINITY;
        if (d >= s->prm.dhat) continue;
        double b3[3];
        ora_barrier_scalar(d, s->prm.dhat, b3);
        double w = 1.0;
        if (c[0] == 1) {
            double m3[3];
            mollifier(ee_cross_sq(x12, NULL, NULL), cand_eps_x(s, c), m3);
            w = m3[0];
        }
        nsum_add(&acc, s->prm.kappa * w * b3[0]);
    }
    if (s->n_fric) nsum_add(&acc, friction_energy(s, x));
    return nsum_get(&acc);
}

double ora_energy(ora_scene *s, const double *x)
{
    ivec c = {0, 0, 0};
    candidates_list(s, x, NULL, &c);
    double E = energy_with(s, x, &c);
    free(c.v);
    return E;
}

/* ======================================================================== */
/* lagged friction                                                           */
/* ======================================================================== */
/* Frictional contact as in IPC (Li et al. 2020): the dissipative potential
 * D(x) = sum_c mu lambda_c f0(|u_c|) with one lag per step. For every pair
 * active at x^t, lambda_c = kappa w |b'(d)| (the barrier's normal force there,
 * EE mollifier w held fixed), the coefficients c_k of the closest points (the
 * residual r = sum_k c_k x_k whose length is d) and the unit normal n = r / d
 * are frozen; the tangential relative displacement is
 *   u_c = (I - n n^T) sum_k c_k (x_k - x^t_k),
 * and f0 is IPC's C1 smoothing of |u| over the length e = eps_v h:
 *   f0(y) = -y^3 / (3 e^2) + y^2 / e + e / 3 for y < e, y otherwise.
 * Its Hessian is (c c^T) (x) M with M = (f1 / y)(P - uu^T/y^2) + f1' uu^T/y^2
 * (P = I - nn^T), positive semi-definite (both scalars >= 0); at y = 0 the
 * limit M = (2 / e) P. */

void ora_friction_f(double y, double eps, double *f3)
{
    if (y < eps) {
        f3[0] = -y * y * y / (3.0 * eps * eps) + y * y / eps + eps / 3.0;
        f3[1] = -y * y / (eps * eps) + 2.0 * y / eps;
        f3[2] = -2.0 * y / (eps * eps) + 2.0 / eps;
    } else {
        f3[0] = y;
        f3[1] = 1.0;
        f3[2] = 0.0;
    }
}

double ora_pair_friction(const double *x12, const double *xt12, const double *c4, const double *nrm,
                         double mu_lam, double eps, double *g12, double *H144)
{
    double r[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < 4; ++k)
        for (int i = 0; i < 3; ++i) r[i] += c4[k] * (x12[3 * k + i] - xt12[3 * k + i]);
    double rn = dot3(r, nrm);
    double u[3];
    for (int i = 0; i < 3; ++i) u[i] = r[i] - rn * nrm[i];
    double y = sqrt(dot3(u, u));
    double f[3];
    ora_friction_f(y, eps, f);
    /* f1(y) / y, finite at y = 0 */
    double f1y = y < eps ? 2.0 / eps - y / (eps * eps) : 1.0 / y;
    if (g12)
        for (int k = 0; k < 4; ++k)
            for (int i = 0; i < 3; ++i) g12[3 * k + i] = mu_lam * c4[k] * f1y * u[i];
    if (H144) {
        double M[9];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double P = (i == j ? 1.0 : 0.0) - nrm[i] * nrm[j];
                if (y > 0.0) {
                    double uu = u[i] * u[j] / (y * y);
                    double f2 = f[2] > 0.0 ? f[2] : 0.0;
                    M[3 * i + j] = f1y * (P - uu) + f2 * uu;
                } else {
                    M[3 * i + j] = (2.0 / eps) * P;
                }
            }
        for (int k = 0; k < 4; ++k)
            for (int l = 0; l < 4; ++l)
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j)
                        H144[(3 * k + i) * 12 + 3 * l + j] = mu_lam * c4[k] * c4[l] * M[3 * i + j];
    }
    return mu_lam * f[0];
}

/* the friction set of a step: every static candidate active at x^t */
static void friction_lag(ora_scene *s)
{
    free(s->fric_v); free(s->fric_c); free(s->fric_nrm); free(s->fric_lam);
    s->fric_v = NULL; s->fric_c = NULL; s->fric_nrm = NULL; s->fric_lam = NULL;
    s->n_fric = 0;
    if (!(s->prm.mu_fric > 0.0)) return;
    ivec cand = {0, 0, 0};
    candidates_list(s, s->xt, NULL, &cand);
    int nc = cand.n / 3;
    s->fric_v = (int32_t *)malloc(sizeof(int32_t) * 4 * (nc + 1));
    s->fric_c = (double *)malloc(sizeof(double) * 4 * (nc + 1));
    s->fric_nrm = (double *)malloc(sizeof(double) * 3 * (nc + 1));
    s->fric_lam = (double *)malloc(sizeof(double) * (nc + 1));
    for (int i = 0; i < nc; ++i) {
        const int32_t *c = cand.v + 3 * i;
        int32_t v[4];
        double x12[12];
        cand_verts(s, c, v);
        gather12(s->xt, v, x12);
        dist_spec sp = c[0] == 0 ? pt_spec(pt_type(x12)) : ee_spec(ee_type(x12));
        double r[3], cc[4], uu[2][3], G[2][2];
        dist_solve(&sp, x12, r, cc, uu, G);
        double d = sqrt(dot3(r, r));
        if (!(d < s->prm.dhat) || !(d > 0.0)) continue;
        double b3[3];
        ora_barrier_scalar(d, s->prm.dhat, b3);
        double w = 1.0;
        if (c[0] == 1) {
            double m3[3];
            mollifier(ee_cross_sq(x12, NULL, NULL), cand_eps_x(s, c), m3);
            w = m3[0];
        }
        int k = s->n_fric++;
        memcpy(s->fric_v + 4 * k, v, sizeof v);
        memcpy(s->fric_c + 4 * k, cc, sizeof cc);
        for (int j = 0; j < 3; ++j) s->fric_nrm[3 * k + j] = r[j] / d;
        s->fric_lam[k] = s->prm.kappa * w * fabs(b3[1]);
    }
    free(cand.v);
}

int32_t ora_friction_set(const ora_scene *s, int32_t *v4, double *c4, double *nrm, double *lam)
{
    if (v4) memcpy(v4, s->fric_v, sizeof(int32_t) * 4 * s->n_fric);
    if (c4) memcpy(c4, s->fric_c, sizeof(double) * 4 * s->n_fric);
    if (nrm) memcpy(nrm, s->fric_nrm, sizeof(double) * 3 * s->n_fric);
    if (lam) memcpy(lam, s->fric_lam, sizeof(double) * s->n_fric);
    return s->n_fric;
}

static double friction_energy(const ora_scene *s, const double *x)
{
    nsum acc = {0.0, 0.0};
    double eps = s->prm.eps_v * s->prm.h;
    for (int k = 0; k < s->n_fric; ++k) {
        double x12[12], xt12[12];
        gather12(x, s->fric_v + 4 * k, x12);
        gather12(s->xt, s->fric_v + 4 * k, xt12);
        nsum_add(&acc, ora_pair_friction(x12, xt12, s->fric_c + 4 * k, s->fric_nrm + 3 * k,
                                         s->prm.mu_fric * s->fric_lam[k], eps, NULL, NULL));
    }
    return nsum_get(&acc);
}

/* ======================================================================== */
/* assembly: gradient, element Hessians, contact Hessians                   */
/* ======================================================================== */

typedef struct {
    int n;
    double *g;     /* 3n */
    double *Hel;   /* 144 per tet */
    int n_c;
    int32_t *cv;   /* 4 vertex ids per active contact, then per friction pair */
    double *Hc;    /* 144 per active contact, then per friction pair */
    int n_f;       /* friction pairs (after the n_c contacts) */
    double *diag;  /* 9 per vertex: block diagonal of H */
    int n_cand;
    int32_t *ckind; /* per active contact: 0 PT, 1 EE */
    double *gc;     /* 12 per active contact: its barrier gradient */
} assembly;

static void assembly_free(assembly *A)
{
    free(A->g); free(A->Hel); free(A->cv); free(A->Hc); free(A->diag); free(A->ckind); free(A->gc);
}

static void assemble(const ora_scene *s, const double *x, assembly *A)
{
    int n = s->n;
    double h2 = s->prm.h * s->prm.h;
    A->n = n;
    A->g = (double *)calloc(3 * n, sizeof(double));
    A->diag = (double *)calloc(9 * n, sizeof(double));
    A->Hel = (double *)malloc(sizeof(double) * 144 * s->n_tet);
    /* inertia and kinematic targets */
    for (int i = 0; i < s->n_gel; ++i) {
        double k = s->mass[i] / h2;
        for (int c = 0; c < 3; ++c) {
            A->g[3 * i + c] += k * (x[3 * i + c] - s->xtilde[3 * i + c]);
            A->diag[9 * i + 4 * c] += k;
        }
    }
    for (int j = s->n_gel; j < n; ++j)
        for (int c = 0; c < 3; ++c) {
            A->g[3 * j + c] += s->prm.k_target * (x[3 * j + c] - s->yhat[3 * j + c]) - s->lam_al[3 * j + c];
            A->diag[9 * j + 4 * c] += s->prm.k_target;
        }
    for (int i = 0; i < s->n_gel; ++i)
        if (is_attached(s, i))
            for (int c = 0; c < 3; ++c) {
                A->g[3 * i + c] += s->prm.k_target * (x[3 * i + c] - s->yhat[3 * i + c]);
                A->diag[9 * i + 4 * c] += s->prm.k_target;
            }
    /* elasticity */
    for (int e = 0; e < s->n_tet; ++e) {
        const int32_t *t = s->T + 4 * e;
        double x12[12], g12[12], E;
        double *H = A->Hel + 144 * e;
        gather12(x, t, x12);
        ora_tet_elastic(x12, s->Bm + 9 * e, s->vol[e], s->mu, s->lam, &E, g12, H);
        for (int a = 0; a < 4; ++a)
            for (int c = 0; c < 3; ++c) A->g[3 * t[a] + c] += g12[3 * a + c];
        for (int a = 0; a < 4; ++a)
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) A->diag[9 * t[a] + 3 * i + j] += H[(3 * a + i) * 12 + 3 * a + j];
    }
    /* barrier over active static candidates */
    ivec cand = {0, 0, 0};
    candidates_list(s, x, NULL, &cand);
    A->n_cand = cand.n / 3;
    A->n_c = 0;
    A->cv = (int32_t *)malloc(sizeof(int32_t) * 4 * (A->n_cand + s->n_fric + 1));
    A->Hc = (double *)malloc(sizeof(double) * 144 * (A->n_cand + s->n_fric + 1));
    A->ckind = (int32_t *)malloc(sizeof(int32_t) * (A->n_cand + 1));
    A->gc = (double *)malloc(sizeof(double) * 12 * (A->n_cand + 1));
    for (int i = 0; i < A->n_cand; ++i) {
        const int32_t *c = cand.v + 3 * i;
        int32_t v[4];
        double x12[12];
        cand_verts(s, c, v);
        gather12(x, v, x12);
        double d = c[0] == 0 ? ora_pt_distance(x12, NULL) : ora_ee_distance(x12, NULL);
        if (!(d < s->prm.dhat)) continue;
        double g12[12];
        double eps_x = c[0] == 1 ? cand_eps_x(s, c) : 0.0;
        double *H = A->Hc + 144 * A->n_c;
        ora_pair_barrier(c[0], x12, s->prm.dhat, s->prm.kappa, eps_x, s->prm.barrier_hessian == 1 ? 2 : 1, g12, H);
        memcpy(A->cv + 4 * A->n_c, v, sizeof v);
        A->ckind[A->n_c] = c[0];
        memcpy(A->gc + 12 * A->n_c, g12, sizeof g12);
        for (int a = 0; a < 4; ++a)
            for (int k = 0; k < 3; ++k) A->g[3 * v[a] + k] += g12[3 * a + k];
        for (int a = 0; a < 4; ++a)
            for (int ii = 0; ii < 3; ++ii)
                for (int jj = 0; jj < 3; ++jj)
                    A->diag[9 * v[a] + 3 * ii + jj] += H[(3 * a + ii) * 12 + 3 * a + jj];
        A->n_c++;
    }
    free(cand.v);
    /* lagged friction pairs */
    A->n_f = 0;
    double eps = s->prm.eps_v * s->prm.h;
    for (int k = 0; k < s->n_fric; ++k) {
        const int32_t *v = s->fric_v + 4 * k;
        double x12[12], xt12[12], g12[12];
        gather12(x, v, x12);
        gather12(s->xt, v, xt12);
        int slot = A->n_c + A->n_f;
        double *H = A->Hc + 144 * slot;
        ora_pair_friction(x12, xt12, s->fric_c + 4 * k, s->fric_nrm + 3 * k, s->prm.mu_fric * s->fric_lam[k], eps,
                          g12, H);
        memcpy(A->cv + 4 * slot, v, sizeof(int32_t) * 4);
        for (int a = 0; a < 4; ++a)
            for (int c = 0; c < 3; ++c) A->g[3 * v[a] + c] += g12[3 * a + c];
        for (int a = 0; a < 4; ++a)
            for (int ii = 0; ii < 3; ++ii)
                for (int jj = 0; jj < 3; ++jj)
                    A->diag[9 * v[a] + 3 * ii + jj] += H[(3 * a + ii) * 12 + 3 * a + jj];
        A->n_f++;
    }
    /* Dirichlet: zero gradient, identity diagonal block */
    for (int i = 0; i < n; ++i)
        if (s->fixed[i]) {
            for (int c = 0; c < 3; ++c) A->g[3 * i + c] = 0.0;
            for (int k = 0; k < 9; ++k) A->diag[9 * i + k] = (k % 4 == 0) ? 1.0 : 0.0;
        }
}

/* y = H v with fixed rows/columns replaced by the identity */
static void hess_apply(const ora_scene *s, const assembly *A, const double *v, double *y)
{
    int n = s->n;
    double h2 = s->prm.h * s->prm.h;
    for (int i = 0; i < 3 * n; ++i) y[i] = 0.0;
    for (int i = 0; i < s->n_gel; ++i)
        for (int c = 0; c < 3; ++c) y[3 * i + c] += s->mass[i] / h2 * v[3 * i + c];
    for (int j = s->n_gel; j < n; ++j)
        for (int c = 0; c < 3; ++c) y[3 * j + c] += s->prm.k_target * v[3 * j + c];
    for (int i = 0; i < s->n_gel; ++i)
        if (is_attached(s, i))
            for (int c = 0; c < 3; ++c) y[3 * i + c] += s->prm.k_target * v[3 * i + c];
    for (int e = 0; e < s->n_tet; ++e) {
        const int32_t *t = s->T + 4 * e;
        const double *H = A->Hel + 144 * e;
        for (int a = 0; a < 4; ++a) {
            if (s->fixed[t[a]]) continue;
            for (int b = 0; b < 4; ++b) {
                if (s->fixed[t[b]]) continue;
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j)
                        y[3 * t[a] + i] += H[(3 * a + i) * 12 + 3 * b + j] * v[3 * t[b] + j];
            }
        }
    }
    for (int k = 0; k < A->n_c + A->n_f; ++k) {
        const int32_t *cv = A->cv + 4 * k;
        const double *H = A->Hc + 144 * k;
        for (int a = 0; a < 4; ++a) {
            if (s->fixed[cv[a]]) continue;
            for (int b = 0; b < 4; ++b) {
                if (s->fixed[cv[b]]) continue;
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j)
                        y[3 * cv[a] + i] += H[(3 * a + i) * 12 + 3 * b + j] * v[3 * cv[b] + j];
            }
        }
    }
    for (int i = 0; i < n; ++i)
        if (s->fixed[i])
            for (int c = 0; c < 3; ++c) y[3 * i + c] = v[3 * i + c];
}

static double dotn(int m, const double *a, const double *b)
{
    double acc = 0.0;
    for (int i = 0; i < m; ++i) acc += a[i] * b[i];
    return acc;
}

/* Block-Jacobi preconditioned CG for H p = -g from p = 0. Stops when the
 * preconditioned residual norm r^T M^-1 r falls to tol^2 times its initial
 * value (rows weighted by their own diagonal stiffness, so the stiff
 * kinematic-target rows do not mask the gel rows). Returns iterations
 * (negative if the cap was hit). */
static int pcg_solve(const ora_scene *s, const assembly *A, double *p)
{
    int n = s->n, m = 3 * n;
    double *Minv = (double *)malloc(sizeof(double) * 9 * n);
    for (int i = 0; i < n; ++i) inv3(A->diag + 9 * i, Minv + 9 * i);
    double *r = (double *)malloc(sizeof(double) * m);
    double *z = (double *)malloc(sizeof(double) * m);
    double *d = (double *)malloc(sizeof(double) * m);
    double *q = (double *)malloc(sizeof(double) * m);
    for (int i = 0; i < m; ++i) {
        p[i] = 0.0;
        r[i] = -A->g[i];
    }
    int maxit = s->prm.pcg_max_iter > 0 ? s->prm.pcg_max_iter : 10 * m;
    int it = 0;
    for (int i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a)
            z[3 * i + a] = Minv[9 * i + 3 * a] * r[3 * i] + Minv[9 * i + 3 * a + 1] * r[3 * i + 1] +
                           Minv[9 * i + 3 * a + 2] * r[3 * i + 2];
    double rz = dotn(m, r, z);
    double stop = s->prm.pcg_tol * s->prm.pcg_tol * rz;
    if (rz > 0.0) {
        memcpy(d, z, sizeof(double) * m);
        for (it = 1; it <= maxit; ++it) {
            hess_apply(s, A, d, q);
            double alpha = rz / dotn(m, d, q);
            for (int i = 0; i < m; ++i) {
                p[i] += alpha * d[i];
                r[i] -= alpha * q[i];
            }
            for (int i = 0; i < n; ++i)
                for (int a = 0; a < 3; ++a)
                    z[3 * i + a] = Minv[9 * i + 3 * a] * r[3 * i] + Minv[9 * i + 3 * a + 1] * r[3 * i + 1] +
                                   Minv[9 * i + 3 * a + 2] * r[3 * i + 2];
            double rz_new = dotn(m, r, z);
            if (rz_new <= stop) break;
            double beta = rz_new / rz;
            rz = rz_new;
            for (int i = 0; i < m; ++i) d[i] = z[i] + beta * d[i];
        }
        if (it > maxit) it = -maxit;
    }
    free(Minv); free(r); free(z); free(d); free(q);
    return it;
}

void ora_gradient(ora_scene *s, const double *x, double *g)
{
    assembly A;
    memset(&A, 0, sizeof A);
    assemble(s, x, &A);
    memcpy(g, A.g, sizeof(double) * 3 * s->n);
    assembly_free(&A);
}

/* The gradient of each term of Phi separately, at x, with no Dirichlet
 * rows zeroed (so the forces on fixed vertices, i.e. the support reactions,
 * can be read): inertia m_i/h^2 (x_i - xtilde_i) on free gel vertices,
 * elasticity sum_e V_e dPsi/dx, the soft targets k_t (x - yhat) (indenter and
 * attached vertices), the barrier over the active static candidates at x and
 * the lagged friction. Each output is 3n doubles, or NULL to skip it. The
 * force a term exerts on a vertex is minus its gradient. */
void ora_gradient_terms(ora_scene *s, const double *x, double *g_inertia, double *g_elastic, double *g_target,
                        double *g_contact, double *g_friction)
{
    int n = s->n;
    double h2 = s->prm.h * s->prm.h;
    double *outs[5] = {g_inertia, g_elastic, g_target, g_contact, g_friction};
    for (int k = 0; k < 5; ++k)
        if (outs[k]) memset(outs[k], 0, sizeof(double) * 3 * n);
    if (g_inertia)
        for (int i = 0; i < s->n_gel; ++i) {
            if (s->fixed[i]) continue;
            for (int c = 0; c < 3; ++c) g_inertia[3 * i + c] = s->mass[i] / h2 * (x[3 * i + c] - s->xtilde[3 * i + c]);
        }
    if (g_elastic)
        for (int e = 0; e < s->n_tet; ++e) {
            const int32_t *t = s->T + 4 * e;
            double x12[12], g12[12], E;
            gather12(x, t, x12);
            ora_tet_elastic(x12, s->Bm + 9 * e, s->vol[e], s->mu, s->lam, &E, g12, NULL);
            for (int a = 0; a < 4; ++a)
                for (int c = 0; c < 3; ++c) g_elastic[3 * t[a] + c] += g12[3 * a + c];
        }
    if (g_target) {
        for (int j = s->n_gel; j < n; ++j)
            for (int c = 0; c < 3; ++c)
                g_target[3 * j + c] = s->prm.k_target * (x[3 * j + c] - s->yhat[3 * j + c]) - s->lam_al[3 * j + c];
        for (int i = 0; i < s->n_gel; ++i)
            if (is_attached(s, i))
                for (int c = 0; c < 3; ++c)
                    g_target[3 * i + c] = s->prm.k_target * (x[3 * i + c] - s->yhat[3 * i + c]);
    }
    if (g_contact) {
        ivec cand = {0, 0, 0};
        candidates_list(s, x, NULL, &cand);
        for (int i = 0; i < cand.n / 3; ++i) {
            const int32_t *c = cand.v + 3 * i;
            int32_t v[4];
            double x12[12], g12[12];
            cand_verts(s, c, v);
            gather12(x, v, x12);
            double d = c[0] == 0 ? ora_pt_distance(x12, NULL) : ora_ee_distance(x12, NULL);
            if (!(d < s->prm.dhat)) continue;
            double eps_x = c[0] == 1 ? cand_eps_x(s, c) : 0.0;
            ora_pair_barrier(c[0], x12, s->prm.dhat, s->prm.kappa, eps_x, 0, g12, NULL);
            for (int a = 0; a < 4; ++a)
                for (int k = 0; k < 3; ++k) g_contact[3 * v[a] + k] += g12[3 * a + k];
        }
        free(cand.v);
    }
    if (g_friction) {
        double eps = s->prm.eps_v * s->prm.h;
        for (int k = 0; k < s->n_fric; ++k) {
            const int32_t *v = s->fric_v + 4 * k;
            double x12[12], xt12[12], g12[12];
            gather12(x, v, x12);
            gather12(s->xt, v, xt12);
            ora_pair_friction(x12, xt12, s->fric_c + 4 * k, s->fric_nrm + 3 * k, s->prm.mu_fric * s->fric_lam[k], eps,
                              g12, NULL);
            for (int a = 0; a < 4; ++a)
                for (int c = 0; c < 3; ++c) g_friction[3 * v[a] + c] += g12[3 * a + c];
        }
    }
}

void ora_hess_apply(ora_scene *s, const double *x, const double *v, double *y)
{
    assembly A;
    memset(&A, 0, sizeof A);
    assemble(s, x, &A);
    hess_apply(s, &A, v, y);
    assembly_free(&A);
}

void ora_hess_apply_body(ora_scene *s, const double *x, const double *v, double *y)
{
    assembly A;
    memset(&A, 0, sizeof A);
    assemble(s, x, &A);
    A.n_c = A.n_f = 0; /* the body terms only: no barrier or friction pair */
    hess_apply(s, &A, v, y);
    assembly_free(&A);
}

int32_t ora_contact_pairs(ora_scene *s, const double *x, int32_t cap, int32_t *kind, int32_t *v4, double *g12,
                          double *H144)
{
    assembly A;
    memset(&A, 0, sizeof A);
    assemble(s, x, &A);
    int n = A.n_c;
    for (int k = 0; k < n && k < cap; ++k) {
        if (kind) kind[k] = A.ckind[k];
        if (v4) memcpy(v4 + 4 * k, A.cv + 4 * k, sizeof(int32_t) * 4);
        if (g12) memcpy(g12 + 12 * k, A.gc + 12 * k, sizeof(double) * 12);
        if (H144) memcpy(H144 + 144 * k, A.Hc + 144 * k, sizeof(double) * 144);
    }
    assembly_free(&A);
    return n;
}

void ora_hess_dense(ora_scene *s, const double *x, double *H)
{
    assembly A;
    memset(&A, 0, sizeof A);
    assemble(s, x, &A);
    int m = 3 * s->n;
    double *e = (double *)calloc(m, sizeof(double));
    double *y = (double *)malloc(sizeof(double) * m);
    for (int j = 0; j < m; ++j) {
        e[j] = 1.0;
        hess_apply(s, &A, e, y);
        for (int i = 0; i < m; ++i) H[(size_t)i * m + j] = y[i];
        e[j] = 0.0;
    }
    free(e);
    free(y);
    assembly_free(&A);
}

int32_t ora_pcg(ora_scene *s, const double *x, double *p)
{
    assembly A;
    memset(&A, 0, sizeof A);
    assemble(s, x, &A);
    int it = pcg_solve(s, &A, p);
    assembly_free(&A);
    return it;
}

static double ccd_with(const ora_scene *s, const double *x, const double *p, const ivec *cand)
{
    double t = 1.0;
    for (int i = 0; i < cand->n / 3; ++i) {
        const int32_t *c = cand->v + 3 * i;
        int32_t v[4];
        double x12[12], p12[12];
        cand_verts(s, c, v);
        gather12(x, v, x12);
        gather12(p, v, p12);
        double toi = ora_accd(c[0], x12, p12, s->prm.ccd_s, 1.0, s->prm.ccd_max_iter);
        if (toi < t) t = toi;
    }
    return t;
}

double ora_ccd(ora_scene *s, const double *x, const double *p)
{
    ivec c = {0, 0, 0};
    candidates_list(s, x, p, &c);
    double t = ccd_with(s, x, p, &c);
    free(c.v);
    return t;
}

/* ======================================================================== */
/* Newton                                                                    */
/* ======================================================================== */
/* attachment                                                                */
/* ======================================================================== */
/* The paper's GIPC attachments move the gel with the sensor case: gel
 * vertices inside the case keep fixed offsets in the case frame and get the
 * case pose applied to them as target values before each solve ("GIPC
 * Attachments"). Here an attached free gel vertex i is pulled to its target
 * yhat_i = case pose applied to its rest position by the same penalty
 * k_t/2 |x_i - yhat_i|^2 that drives the indenter (on top of its inertia and
 * elasticity). Fixed vertices stay fixed. */
static int is_attached(const ora_scene *s, int i) { return s->attached && s->attached[i] && !s->fixed[i]; }

void ora_set_attachment(ora_scene *s, const uint8_t *mask)
{
    free(s->attached);
    s->attached = NULL;
    if (!mask) return;
    s->attached = (uint8_t *)malloc((size_t)s->n_gel);
    memcpy(s->attached, mask, (size_t)s->n_gel);
}

void ora_set_case_pose(ora_scene *s, const double *pose) { memcpy(s->case_pose, pose, sizeof(double) * 12); }

/* ======================================================================== */

/* max_j |y_j - yhat_j| over indenter vertices */
static double target_lag(const ora_scene *s, const double *x)
{
    double lag = 0.0;
    for (int j = s->n_gel; j < s->n; ++j) {
        double d[3];
        sub3(x + 3 * j, s->yhat + 3 * j, d);
        double l = sqrt(dot3(d, d));
        if (l > lag) lag = l;
    }
    return lag;
}

void ora_begin_step(ora_scene *s, const double *pose)
{
    int n = s->n;
    double h = s->prm.h;
    memcpy(s->xt, s->x, sizeof(double) * 3 * n);
    for (int i = 0; i < s->n_gel; ++i)
        for (int c = 0; c < 3; ++c) {
            if (s->fixed[i])
                s->xtilde[3 * i + c] = s->x[3 * i + c];
            else
                s->xtilde[3 * i + c] = s->x[3 * i + c] + h * s->v[3 * i + c] + h * h * s->prm.gravity[c];
        }
    for (int j = 0; j < s->n_ind; ++j) {
        apply_pose(pose, s->Yloc + 3 * j, s->yhat + 3 * (s->n_gel + j));
        for (int c = 0; c < 3; ++c) s->xtilde[3 * (s->n_gel + j) + c] = s->x[3 * (s->n_gel + j) + c];
    }
    for (int i = 0; i < s->n_gel; ++i)
        if (is_attached(s, i)) apply_pose(s->case_pose, s->X + 3 * i, s->yhat + 3 * i);
    memset(s->lam_al, 0, sizeof(double) * 3 * n);
    s->al_step = 0;
    friction_lag(s);
}

/* One projected-Newton iteration of the incremental potential:
 * candidates and active set at x, assemble g and H, PCG for p, converged if
 * |p|_inf <= tol; otherwise swept candidates over [x, x+p], ACCD step bound,
 * halve alpha from min(1, alpha_ccd) until Phi(x + alpha p) <= Phi(x). */
int32_t ora_newton_iterate(ora_scene *s, const double *x_in, double *x_out, ora_stats *st)
{
    int n = s->n, m = 3 * n;
    assembly A;
    memset(&A, 0, sizeof A);
    assemble(s, x_in, &A);
    double *p = (double *)malloc(sizeof(double) * m);
    int it = pcg_solve(s, &A, p);
    if (st) {
        st->pcg_iters += it < 0 ? -it : it;
        st->n_candidates = A.n_cand;
        st->n_active = A.n_c;
        if (it < 0) st->status = ORA_W_PCG_MAXITER;
    }
    assembly_free(&A);
    double pinf = 0.0;
    for (int i = 0; i < n; ++i) {
        if (s->fixed[i]) continue;
        for (int c = 0; c < 3; ++c)
            if (fabs(p[3 * i + c]) > pinf) pinf = fabs(p[3 * i + c]);
    }
    if (st) st->pinf = pinf;
    memcpy(x_out, x_in, sizeof(double) * m);
    /* after a multiplier update the step moves the indenter by about its
     * remaining lag, below the Newton tolerance: it is taken regardless */
    if (pinf <= s->prm.newton_tol && !s->al_step) {
        free(p);
        return 1;
    }
    s->al_step = 0;
    ivec sw = {0, 0, 0};
    candidates_list(s, x_in, p, &sw);
    double accd = ccd_with(s, x_in, p, &sw);
    double alpha = accd < 1.0 ? accd : 1.0;
    double alpha0 = alpha;
    double E0 = energy_with(s, x_in, &sw);
    double *xt = (double *)malloc(sizeof(double) * m);
    int ret = 0, halvings = 0;
    for (;;) {
        for (int i = 0; i < m; ++i) xt[i] = x_in[i] + alpha * p[i];
        double E = energy_with(s, xt, &sw);
        if (E <= E0) {
            memcpy(x_out, xt, sizeof(double) * m);
            if (st) st->energy = E;
            break;
        }
        alpha *= 0.5;
        ++halvings;
        if (alpha < s->prm.ls_min_ratio * alpha0) {
            ret = 2;
            if (st) st->energy = E0;
            break;
        }
    }
    if (st) {
        st->alpha_ccd = accd;
        st->alpha = ret == 2 ? 0.0 : alpha;
        st->ls_halvings += halvings;
    }
    free(xt);
    free(sw.v);
    free(p);
    return ret;
}

int32_t ora_step(ora_scene *s, const double *pose, ora_stats *st)
{
    ora_stats local;
    if (!st) st = &local;
    memset(st, 0, sizeof *st);
    ora_begin_step(s, pose);
    int n = s->n, m = 3 * n;
    double *xn = (double *)malloc(sizeof(double) * m);
    int status = ORA_OK, k;
    int pcg_warn = 0;
    const int al_max = s->prm.target_al_max > 0 ? s->prm.target_al_max : 8;
    int al = 0;
    for (k = 0; k < s->prm.max_newton; ++k) {
        st->status = 0;
        int r = ora_newton_iterate(s, s->x, xn, st);
        st->newton_iters++;
        if (st->status == ORA_W_PCG_MAXITER) pcg_warn = 1;
        if (r == 1) {
            /* converged for the current multipliers: update them while the
             * indenter is further than the tolerance from its targets */
            if (s->prm.target_al && al < al_max && target_lag(s, s->x) > s->prm.target_al_tol) {
                for (int j = s->n_gel; j < n; ++j)
                    for (int c = 0; c < 3; ++c)
                        s->lam_al[3 * j + c] -= s->prm.k_target * (s->x[3 * j + c] - s->yhat[3 * j + c]);
                ++al;
                s->al_step = 1;
                continue;
            }
            break;
        }
        memcpy(s->x, xn, sizeof(double) * m);
        if (r == 2) {
            status = ORA_W_LS_STALL;
            break;
        }
    }
    if (k == s->prm.max_newton) status = ORA_W_NEWTON_MAXITER;
    if (status == ORA_OK && pcg_warn) status = ORA_W_PCG_MAXITER;
    for (int i = 0; i < m; ++i) s->v[i] = (s->x[i] - s->xt[i]) / s->prm.h;
    double lag = target_lag(s, s->x);
    st->max_target_lag = lag;
    st->al_updates = al;
    if (status == ORA_OK && lag > 1e-3 * s->prm.dhat) status = ORA_W_TARGET_LAG;
    st->status = status;
    free(xn);
    return status;
}
