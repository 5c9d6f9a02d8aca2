"""ctypes wrapper of the plain FP64 CPU oracle (ipc_oracle.c).

TEST INFRASTRUCTURE ONLY: tests, the smoke check and the benchmark's CPU
baseline leg may load this module; the product library never does.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ipc_oracle.c")
_LIB = os.path.join(_HERE, "libipc_oracle.so")

# -O2, no fast-math, no FMA contraction: per-primitive formulas round like the
# GPU path's FP64 contact code.
CFLAGS = ["-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math"]


def build(force: bool = False) -> str:
    newest = max(os.path.getmtime(_SRC), os.path.getmtime(os.path.join(_HERE, "ipc_oracle.h")))
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < newest:
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", _LIB, "-lm"])
    return _LIB


class Params(C.Structure):
    _fields_ = [
        ("E", C.c_double), ("nu", C.c_double), ("rho", C.c_double),
        ("h", C.c_double), ("dhat", C.c_double), ("kappa", C.c_double),
        ("k_target", C.c_double), ("newton_tol", C.c_double), ("pcg_tol", C.c_double),
        ("gravity", C.c_double * 3), ("ccd_s", C.c_double), ("ls_min_ratio", C.c_double),
        ("self_contact", C.c_int32), ("max_newton", C.c_int32),
        ("pcg_max_iter", C.c_int32), ("ccd_max_iter", C.c_int32),
        ("mu_fric", C.c_double), ("eps_v", C.c_double), ("barrier_hessian", C.c_int32),
        ("target_al", C.c_int32), ("target_al_tol", C.c_double), ("target_al_max", C.c_int32),
    ]


class Stats(C.Structure):
    _fields_ = [
        ("newton_iters", C.c_int32), ("pcg_iters", C.c_int32), ("n_candidates", C.c_int32),
        ("n_active", C.c_int32), ("status", C.c_int32), ("ls_halvings", C.c_int32),
        ("alpha_ccd", C.c_double), ("alpha", C.c_double), ("energy", C.c_double),
        ("pinf", C.c_double), ("max_target_lag", C.c_double), ("al_updates", C.c_int32),
    ]

    def asdict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None
_D = C.POINTER(C.c_double)
_I = C.POINTER(C.c_int32)
_U8 = C.POINTER(C.c_uint8)


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        L = _lib
        L.ora_scene_create.restype = C.c_void_p
        L.ora_scene_create.argtypes = [C.c_int32, _D, C.c_int32, _I, _U8, C.c_int32, _D, C.c_int32,
                                       _I, _D, C.POINTER(Params), _I]
        L.ora_scene_destroy.argtypes = [C.c_void_p]
        for f in ("ora_scene_sizes",):
            getattr(L, f).argtypes = [C.c_void_p, _I]
        L.ora_scene_surface.argtypes = [C.c_void_p, _I, _I, _I]
        L.ora_scene_rest.argtypes = [C.c_void_p, _D, _D]
        for f in ("ora_get_x", "ora_set_x", "ora_get_v", "ora_set_v", "ora_begin_step"):
            getattr(L, f).argtypes = [C.c_void_p, _D]
        L.ora_reset.argtypes = [C.c_void_p]
        L.ora_set_attachment.restype = None
        L.ora_set_attachment.argtypes = [C.c_void_p, _U8]
        L.ora_set_case_pose.restype = None
        L.ora_set_case_pose.argtypes = [C.c_void_p, _D]
        L.ora_newton_iterate.restype = C.c_int32
        L.ora_newton_iterate.argtypes = [C.c_void_p, _D, _D, C.POINTER(Stats)]
        L.ora_step.restype = C.c_int32
        L.ora_step.argtypes = [C.c_void_p, _D, C.POINTER(Stats)]
        L.ora_candidates.restype = C.c_int32
        L.ora_candidates.argtypes = [C.c_void_p, _D, _D, _I, C.c_int32]
        L.ora_energy.restype = C.c_double
        L.ora_energy.argtypes = [C.c_void_p, _D]
        L.ora_gradient.argtypes = [C.c_void_p, _D, _D]
        L.ora_gradient_terms.argtypes = [C.c_void_p, _D, _D, _D, _D, _D, _D]
        L.ora_hess_apply.argtypes = [C.c_void_p, _D, _D, _D]
        L.ora_hess_apply_body.argtypes = [C.c_void_p, _D, _D, _D]
        L.ora_contact_pairs.restype = C.c_int32
        L.ora_contact_pairs.argtypes = [C.c_void_p, _D, C.c_int32, _I, _I, _D, _D]
        L.ora_hess_dense.argtypes = [C.c_void_p, _D, _D]
        L.ora_pcg.restype = C.c_int32
        L.ora_pcg.argtypes = [C.c_void_p, _D, _D]
        L.ora_ccd.restype = C.c_double
        L.ora_ccd.argtypes = [C.c_void_p, _D, _D]
        L.ora_candidate_distances.argtypes = [C.c_void_p, _D, C.c_int32, _I, _D, _I]
        L.ora_nh_psi.restype = C.c_double
        L.ora_nh_psi.argtypes = [_D, C.c_double, C.c_double]
        L.ora_nh_pk1.argtypes = [_D, C.c_double, C.c_double, _D]
        L.ora_nh_hessian.argtypes = [_D, C.c_double, C.c_double, _D]
        L.ora_tet_elastic.argtypes = [_D, _D, C.c_double, C.c_double, C.c_double, _D, _D, _D]
        L.ora_sym_eig.argtypes = [C.c_int32, _D, _D, _D]
        L.ora_psd_project.argtypes = [C.c_int32, _D]
        L.ora_pt_distance.restype = C.c_double
        L.ora_pt_distance.argtypes = [_D, _I]
        L.ora_ee_distance.restype = C.c_double
        L.ora_ee_distance.argtypes = [_D, _I]
        L.ora_distance_derivs.restype = C.c_double
        L.ora_distance_derivs.argtypes = [C.c_int32, _D, _D, _D]
        L.ora_barrier_scalar.argtypes = [C.c_double, C.c_double, _D]
        L.ora_pair_barrier.restype = C.c_double
        L.ora_pair_barrier.argtypes = [C.c_int32, _D, C.c_double, C.c_double, C.c_double, C.c_int32,
                                       _D, _D]
        L.ora_accd.restype = C.c_double
        L.ora_accd.argtypes = [C.c_int32, _D, _D, C.c_double, C.c_double, C.c_int32]
        L.ora_friction_f.argtypes = [C.c_double, C.c_double, _D]
        L.ora_pair_friction.restype = C.c_double
        L.ora_pair_friction.argtypes = [_D, _D, _D, _D, C.c_double, C.c_double, _D, _D]
        L.ora_friction_set.restype = C.c_int32
        L.ora_friction_set.argtypes = [C.c_void_p, _I, _D, _D, _D]
    return _lib


def _d(a):
    return a.ctypes.data_as(_D)


def _i(a):
    return a.ctypes.data_as(_I)


def f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


# ---------------------------------------------------------------------------
# element-level functions
# ---------------------------------------------------------------------------

def lame(E, nu):
    return E / (2 * (1 + nu)), E * nu / ((1 + nu) * (1 - 2 * nu))


def nh_psi(F, mu, lam):
    return lib().ora_nh_psi(_d(f64(F)), mu, lam)


def nh_pk1(F, mu, lam):
    P = np.zeros(9)
    lib().ora_nh_pk1(_d(f64(F)), mu, lam, _d(P))
    return P.reshape(3, 3)


def nh_hessian(F, mu, lam):
    H = np.zeros(81)
    lib().ora_nh_hessian(_d(f64(F)), mu, lam, _d(H))
    return H.reshape(9, 9)


def tet_elastic(x12, Bm, vol, mu, lam):
    E = np.zeros(1)
    g = np.zeros(12)
    H = np.zeros(144)
    lib().ora_tet_elastic(_d(f64(x12)), _d(f64(Bm)), vol, mu, lam, _d(E), _d(g), _d(H))
    return E[0], g, H.reshape(12, 12)


def sym_eig(A):
    A = f64(A)
    n = A.shape[0]
    w = np.zeros(n)
    V = np.zeros((n, n))
    lib().ora_sym_eig(n, _d(A), _d(w), _d(V))
    return w, V


def psd_project(A):
    A = f64(A).copy()
    lib().ora_psd_project(A.shape[0], _d(A))
    return A


def pt_distance(x12):
    t = np.zeros(1, dtype=np.int32)
    d = lib().ora_pt_distance(_d(f64(x12)), _i(t))
    return d, int(t[0])


def ee_distance(x12):
    t = np.zeros(1, dtype=np.int32)
    d = lib().ora_ee_distance(_d(f64(x12)), _i(t))
    return d, int(t[0])


def distance_derivs(kind, x12):
    g = np.zeros(12)
    H = np.zeros(144)
    d = lib().ora_distance_derivs(kind, _d(f64(x12)), _d(g), _d(H))
    return d, g, H.reshape(12, 12)


def barrier_scalar(d, dhat):
    b = np.zeros(3)
    lib().ora_barrier_scalar(d, dhat, _d(b))
    return b


def pair_barrier(kind, x12, dhat, kappa, eps_x, project=True):
    """project: False/0 exact Hessian, True/1 PSD-projected, 2 Gauss-Newton form."""
    g = np.zeros(12)
    H = np.zeros(144)
    E = lib().ora_pair_barrier(kind, _d(f64(x12)), dhat, kappa, eps_x, int(project), _d(g), _d(H))
    return E, g, H.reshape(12, 12)


def accd(kind, x12, p12, s=0.1, tmax=1.0, max_iter=10000):
    return lib().ora_accd(kind, _d(f64(x12)), _d(f64(p12)), s, tmax, max_iter)


def friction_f(y, eps):
    """(f0, f0', f0'') of the friction smoothing at y for length eps."""
    f = np.zeros(3)
    lib().ora_friction_f(float(y), float(eps), _d(f))
    return f


def pair_friction(x12, xt12, c4, nrm, mu_lam, eps):
    """Lagged friction energy of one pair, its gradient (12) and PSD Hessian (12x12)."""
    g = np.zeros(12)
    H = np.zeros(144)
    D = lib().ora_pair_friction(_d(f64(x12)), _d(f64(xt12)), _d(f64(c4)), _d(f64(nrm)), float(mu_lam),
                                float(eps), _d(g), _d(H))
    return D, g, H.reshape(12, 12)


# ---------------------------------------------------------------------------
# scene-level
# ---------------------------------------------------------------------------

def default_params(scene, pcg_tol=1e-12, **kw) -> Params:
    p = Params()
    p.E, p.nu, p.rho = scene.E, scene.nu, scene.rho
    p.h = scene.dt
    p.dhat, p.kappa, p.k_target = scene.dhat, scene.kappa, scene.k_target
    p.newton_tol = scene.newton_tol
    p.pcg_tol = pcg_tol
    for i in range(3):
        p.gravity[i] = scene.gravity[i]
    p.ccd_s = 0.1
    p.ls_min_ratio = 2.0 ** -30
    p.self_contact = int(scene.self_contact)
    p.max_newton = 100
    p.pcg_max_iter = 0
    p.ccd_max_iter = 10000
    meta = scene.meta or {}
    p.mu_fric = float(meta.get("mu", 0.0))
    p.eps_v = float(meta.get("eps_v", 1e-3))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


class OracleScene:
    """One oracle scene built from a scenes.Scene."""

    def __init__(self, scene, **params):
        self.scene = scene
        self.params = default_params(scene, **params)
        self._X = f64(scene.X)
        self._T = i32(scene.T)
        self._fixed = np.ascontiguousarray(scene.fixed, dtype=np.uint8)
        self._Y = f64(scene.Y)
        self._F = i32(scene.F)
        self._P0 = f64(scene.poses[0])
        st = np.zeros(1, dtype=np.int32)
        self.ptr = lib().ora_scene_create(
            len(self._X), _d(self._X), len(self._T), _i(self._T),
            self._fixed.ctypes.data_as(_U8), len(self._Y), _d(self._Y), len(self._F), _i(self._F),
            _d(self._P0), C.byref(self.params), _i(st))
        self.status = int(st[0])
        if not self.ptr:
            raise ValueError(f"oracle scene creation failed: status {self.status}")
        sz = np.zeros(8, dtype=np.int32)
        lib().ora_scene_sizes(self.ptr, _i(sz))
        (self.n, self.n_gel, self.n_tet, self.n_pts, self.n_edges, self.n_tris, self.n_ind,
         self.n_gel_tris) = map(int, sz)
        self.step_index = 0
        at = getattr(scene, "attached", None)
        if at is not None:
            self._attached = np.ascontiguousarray(at, dtype=np.uint8)
            lib().ora_set_attachment(self.ptr, self._attached.ctypes.data_as(_U8))

    def set_case_pose(self, pose):
        lib().ora_set_case_pose(self.ptr, _d(f64(pose)))

    def __del__(self):
        if getattr(self, "ptr", None):
            lib().ora_scene_destroy(self.ptr)
            self.ptr = None

    # surface
    def surface(self):
        pts = np.zeros(self.n_pts, dtype=np.int32)
        edges = np.zeros((self.n_edges, 2), dtype=np.int32)
        tris = np.zeros((self.n_tris, 3), dtype=np.int32)
        lib().ora_scene_surface(self.ptr, _i(pts), _i(edges), _i(tris))
        return pts, edges, tris

    def rest(self):
        vol = np.zeros(self.n_tet)
        mass = np.zeros(self.n)
        lib().ora_scene_rest(self.ptr, _d(vol), _d(mass))
        return vol, mass

    def friction_set(self):
        """Lagged friction pairs of the current step: (v4, c4, normal, lambda)."""
        n = lib().ora_friction_set(self.ptr, None, None, None, None)
        v4 = np.zeros((max(n, 1), 4), dtype=np.int32)
        c4 = np.zeros((max(n, 1), 4))
        nrm = np.zeros((max(n, 1), 3))
        lam = np.zeros(max(n, 1))
        lib().ora_friction_set(self.ptr, _i(v4), _d(c4), _d(nrm), _d(lam))
        return v4[:n], c4[:n], nrm[:n], lam[:n]

    @property
    def x(self):
        x = np.zeros((self.n, 3))
        lib().ora_get_x(self.ptr, _d(x))
        return x

    @x.setter
    def x(self, val):
        lib().ora_set_x(self.ptr, _d(f64(val)))

    @property
    def v(self):
        v = np.zeros((self.n, 3))
        lib().ora_get_v(self.ptr, _d(v))
        return v

    @v.setter
    def v(self, val):
        lib().ora_set_v(self.ptr, _d(f64(val)))

    def reset(self):
        lib().ora_reset(self.ptr)
        self.step_index = 0

    def begin_step(self, pose, case_pose=None):
        if case_pose is not None:
            self.set_case_pose(case_pose)
        lib().ora_begin_step(self.ptr, _d(f64(pose)))

    def newton_iterate(self, x_in):
        out = np.zeros((self.n, 3))
        st = Stats()
        r = lib().ora_newton_iterate(self.ptr, _d(f64(x_in)), _d(out), C.byref(st))
        return int(r), out, st

    def step(self, pose=None, case_pose=None):
        if pose is None:
            pose = self.scene.poses[self.step_index + 1]
        cp = getattr(self.scene, "case_poses", None)
        if case_pose is None and cp is not None:
            case_pose = cp[self.step_index + 1]
        if case_pose is not None:
            self.set_case_pose(case_pose)
        st = Stats()
        r = lib().ora_step(self.ptr, _d(f64(pose)), C.byref(st))
        self.step_index += 1
        return int(r), st

    def candidates(self, x, p=None, cap=None):
        xx = f64(x)
        pp = f64(p) if p is not None else None
        n = lib().ora_candidates(self.ptr, _d(xx), _d(pp) if pp is not None else None, None, 0)
        out = np.zeros((max(n, 1), 3), dtype=np.int32)
        lib().ora_candidates(self.ptr, _d(xx), _d(pp) if pp is not None else None, _i(out), n)
        return out[:n]

    def candidate_distances(self, x, cand):
        cand = i32(cand)
        d = np.zeros(len(cand))
        t = np.zeros(len(cand), dtype=np.int32)
        lib().ora_candidate_distances(self.ptr, _d(f64(x)), len(cand), _i(cand), _d(d), _i(t))
        return d, t

    def energy(self, x):
        return lib().ora_energy(self.ptr, _d(f64(x)))

    def gradient(self, x):
        g = np.zeros((self.n, 3))
        lib().ora_gradient(self.ptr, _d(f64(x)), _d(g))
        return g

    def gradient_terms(self, x):
        """Per-term gradients at x (Dirichlet rows kept): dict of (n,3) arrays
        'inertia', 'elastic', 'target', 'contact', 'friction'. The force of a
        term on a vertex is minus its gradient."""
        names = ("inertia", "elastic", "target", "contact", "friction")
        out = {k: np.zeros((self.n, 3)) for k in names}
        lib().ora_gradient_terms(self.ptr, _d(f64(x)), *[_d(out[k]) for k in names])
        return out

    def hess_apply(self, x, v):
        y = np.zeros((self.n, 3))
        lib().ora_hess_apply(self.ptr, _d(f64(x)), _d(f64(v)), _d(y))
        return y

    def hess_apply_body(self, x, v):
        """H v of the inertia, elastic and soft-target terms only."""
        y = np.zeros((self.n, 3))
        lib().ora_hess_apply_body(self.ptr, _d(f64(x)), _d(f64(v)), _d(y))
        return y

    def contact_pairs(self, x):
        """The active barrier pairs at x as the assembly forms them: kind
        (n,), vertex ids (n, 4), gradients (n, 12), Hessians (n, 12, 12),
        Dirichlet rows not yet dropped."""
        xx = f64(x)
        n = lib().ora_contact_pairs(self.ptr, _d(xx), 0, None, None, None, None)
        kind = np.zeros(max(n, 1), dtype=np.int32)
        v4 = np.zeros((max(n, 1), 4), dtype=np.int32)
        g = np.zeros((max(n, 1), 12))
        H = np.zeros((max(n, 1), 12, 12))
        lib().ora_contact_pairs(self.ptr, _d(xx), n, _i(kind), _i(v4), _d(g), _d(H))
        return kind[:n], v4[:n], g[:n], H[:n]

    def hess_dense(self, x):
        m = 3 * self.n
        H = np.zeros((m, m))
        lib().ora_hess_dense(self.ptr, _d(f64(x)), _d(H))
        return H

    def pcg(self, x):
        p = np.zeros((self.n, 3))
        it = lib().ora_pcg(self.ptr, _d(f64(x)), _d(p))
        return p, int(it)

    def ccd(self, x, p):
        return lib().ora_ccd(self.ptr, _d(f64(x)), _d(f64(p)))
