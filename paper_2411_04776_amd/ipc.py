"""Thin ctypes binding of libipcgel.so (C ABI in include/ipc.h).

Argument marshalling only: every stage of the step runs in the library's HIP
kernels. PyTorch supplies device memory (its caching allocator, through the
runtime's alloc/free callbacks) and the stream. If the library is missing the
import fails loudly; there is no CPU fallback.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import sys
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libipcgel.so")

IPC_OK = 0
IPC_W_NEWTON_MAXITER = 1
IPC_W_PCG_MAXITER = 2
IPC_W_LS_STALL = 3
IPC_W_TARGET_LAG = 4
IPC_E_INVALID_ARG = -1
IPC_E_BAD_MESH = -2
IPC_E_INFEASIBLE = -3
IPC_E_OOM = -4
IPC_E_DEVICE = -5
IPC_E_BUSY = -6
IPC_E_CAPACITY = -7
IPC_FP64 = 0
IPC_MIXED = 1
IPC_HOST = 0
IPC_DEVICE = 1
IPC_PRECOND_MULTILEVEL = 0
IPC_PRECOND_JACOBI = 1
IPC_BARRIER_PROJECTED = 0
IPC_BARRIER_GAUSS_NEWTON = 1
IPC_BATCH_LARGE_VERTS = 65536       # engine size classes: scenes with at least this many vertices are large
IPC_HEIGHT_MAP_NOALLOC_MAX_PIXELS = 1 << 20

_D = C.POINTER(C.c_double)
_I = C.POINTER(C.c_int32)
_I64 = C.POINTER(C.c_int64)
_U8 = C.POINTER(C.c_uint8)

ALLOC_FN = C.CFUNCTYPE(C.c_size_t, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)


class ipc_scene_desc(C.Structure):
    _fields_ = [
        ("n_verts", C.c_int32), ("X", _D), ("n_tets", C.c_int32), ("T", _I), ("fixed", _U8),
        ("E", C.c_double), ("nu", C.c_double), ("rho", C.c_double),
        ("n_ind_verts", C.c_int32), ("ind_Y", _D), ("n_ind_tris", C.c_int32), ("ind_tris", _I),
        ("ind_pose0", C.c_double * 12),
        ("dt", C.c_double), ("dhat", C.c_double), ("kappa", C.c_double), ("k_target", C.c_double),
        ("newton_tol", C.c_double), ("pcg_tol", C.c_double), ("gravity", C.c_double * 3),
        ("mu_friction", C.c_double), ("eps_v", C.c_double), ("ccd_s", C.c_double),
        ("ls_min_ratio", C.c_double),
        ("self_contact", C.c_int32), ("precision", C.c_int32), ("max_newton", C.c_int32),
        ("pcg_max_iter", C.c_int32), ("ccd_max_iter", C.c_int32), ("precond", C.c_int32),
        ("barrier_hessian", C.c_int32), ("attached", _U8),
        ("target_al", C.c_int32), ("target_al_tol", C.c_double), ("target_al_max", C.c_int32),
    ]


class ipc_runtime(C.Structure):
    _fields_ = [("stream", C.c_void_p), ("alloc", ALLOC_FN), ("free", FREE_FN), ("user", C.c_void_p),
                ("mem_budget", C.c_int64)]


class ipc_step_req(C.Structure):
    _fields_ = [("pose", C.c_double * 12), ("case_pose", C.c_double * 12), ("case_pose_set", C.c_int32)]


class ipc_height_map_spec(C.Structure):
    _fields_ = [("x0", C.c_double), ("y0", C.c_double), ("dx", C.c_double), ("dy", C.c_double),
                ("z_ref", C.c_double), ("nx", C.c_int32), ("ny", C.c_int32)]


class ipc_step_stats(C.Structure):
    _fields_ = [
        ("status", C.c_int32), ("newton_iters", C.c_int32), ("pcg_iters", C.c_int32),
        ("ls_halvings", C.c_int32), ("n_candidates", C.c_int32), ("n_active", C.c_int32),
        ("alpha_ccd", C.c_double), ("alpha", C.c_double), ("energy", C.c_double), ("pinf", C.c_double),
        ("max_target_lag", C.c_double), ("ms_total", C.c_double), ("ms_phase", C.c_double * 8),
        ("al_updates", C.c_int32),
    ]

    def asdict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "ms_phase"}
        d["ms_phase"] = list(self.ms_phase)
        return d


_SIGS = {
    "ipc_create_scene": (C.c_int32, [C.POINTER(ipc_scene_desc), C.POINTER(ipc_runtime), C.POINTER(C.c_void_p)]),
    "ipc_destroy_scene": (None, [C.c_void_p]),
    "ipc_scene_footprint_bytes": (C.c_int64, [C.POINTER(ipc_scene_desc)]),
    "ipc_step": (C.c_int32, [C.c_void_p, C.POINTER(ipc_step_req), C.POINTER(ipc_step_stats)]),
    "ipc_read_surface": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_void_p, _D]),
    "ipc_surface_topology": (C.c_int32, [C.c_void_p, _I, C.c_int64, _I, _I, C.c_int64, _I]),
    "ipc_height_map": (C.c_int32, [C.c_void_p, C.POINTER(ipc_height_map_spec), C.c_void_p, C.c_int64, C.c_int32,
                                   C.c_void_p]),
    "ipc_height_map_noalloc": (C.c_int32, [C.c_void_p, C.POINTER(ipc_height_map_spec), C.c_void_p, C.c_int64,
                                           C.c_int32, C.c_void_p]),
    "ipc_reset": (C.c_int32, [C.c_void_p]),
    "ipc_state_bytes": (C.c_int64, [C.c_void_p]),
    "ipc_save_state": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int64]),
    "ipc_load_state": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int64]),
    "ipc_scene_sizes": (C.c_int32, [C.c_void_p, _I]),
    "ipc_batch_create": (C.c_int32, [C.POINTER(ipc_runtime), C.POINTER(C.c_void_p)]),
    "ipc_batch_destroy": (None, [C.c_void_p]),
    "ipc_batch_submit": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(C.c_void_p), C.POINTER(ipc_step_req), _I64]),
    "ipc_batch_poll": (C.c_int32, [C.c_void_p, C.c_int64, C.POINTER(ipc_step_stats)]),
    "ipc_batch_wait": (C.c_int32, [C.c_void_p, C.c_int64, C.POINTER(ipc_step_stats)]),
    "ipc_batch_next": (C.c_int32, [C.c_void_p, C.c_double, _I64, _I, C.POINTER(ipc_step_stats)]),
    "ipc_batch_profile": (C.c_int32, [C.c_void_p, C.c_int32]),
    "ipc_batch_profile_totals": (C.c_int32, [C.c_void_p, C.c_int32, _I64, _D]),
    "ipc_batch_profile_read": (C.c_int32, [C.c_void_p, C.c_int32, _I64, _D, _D]),
    "ipc_batch_profile_large": (C.c_int32, [C.c_void_p, C.c_int32, _I64, _D, _D]),
    "ipc_status_str": (C.c_char_p, [C.c_int32]),
    "ipc_last_error": (C.c_int32, [C.c_char_p, C.c_size_t]),
    "ipcx_begin_step": (C.c_int32, [C.c_void_p, C.POINTER(ipc_step_req)]),
    "ipcx_newton_iterate": (C.c_int32, [C.c_void_p, _D, _D, C.POINTER(ipc_step_stats)]),
    "ipcx_candidates": (C.c_int32, [C.c_void_p, _D, _D, _I, C.c_int64, _I64]),
    "ipcx_primitives": (C.c_int32, [C.c_void_p, _I, _I, _I]),
    "ipcx_gradient": (C.c_int32, [C.c_void_p, _D, _D]),
    "ipcx_hess_apply": (C.c_int32, [C.c_void_p, _D, _D, _D]),
    "ipcx_assemble_elastic": (C.c_int32, [C.c_void_p, _D, _D, _D, _D]),
    "ipcx_barrier": (C.c_int32, [C.c_void_p, _D, C.c_int64, _I, _I, _D, _D, _I64]),
    "ipcx_pcg": (C.c_int32, [C.c_void_p, _D, _D, _I]),
    "ipcx_energy": (C.c_int32, [C.c_void_p, _D, _D]),
    "ipcx_ccd": (C.c_int32, [C.c_void_p, _D, _D, _D]),
    "ipcx_profile": (C.c_int32, [C.c_void_p, C.c_int32]),
    "ipcx_profile_read": (C.c_int32, [C.c_void_p, C.c_int32, _I64, _D]),
    "ipcx_profile_bytes": (C.c_int32, [C.c_void_p, C.c_int32, _D]),
    "ipcx_profile_totals": (C.c_int32, [C.c_void_p, C.c_int32, _I64, _D]),
    "ipcx_tuning": (C.c_int32, [C.c_void_p, _D]),
    "ipcx_tuning_for": (C.c_int32, [C.c_int32, _D]),
    "ipcx_struct_sizes": (C.c_int32, [C.POINTER(C.c_int64)]),
    "ipcx_matrix_info": (C.c_int32, [C.c_void_p, _I64]),
    "ipcx_precond_info": (C.c_int32, [C.c_void_p, _I64]),
    "ipcx_set_state": (C.c_int32, [C.c_void_p, _D, _D]),
    "ipcx_get_state": (C.c_int32, [C.c_void_p, _D, _D]),
}

EXPORTED = tuple(_SIGS)

_lib = None


def lib():
    """Load libipcgel.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                               "(run __graft_entry__.build() or paper_2411_04776_amd/build.py)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


# names of the C ABI, callable directly from this module
def __getattr__(name):
    if name in _SIGS:
        return getattr(lib(), name)
    raise AttributeError(name)


def last_error() -> str:
    buf = C.create_string_buffer(1024)
    lib().ipc_last_error(buf, 1024)
    return buf.value.decode()


class IPCError(RuntimeError):
    def __init__(self, code, where):
        msg = lib().ipc_status_str(code).decode()
        super().__init__(f"{where}: {msg} ({code}) {last_error()}")
        self.code = code


def _check(code, where):
    if code < 0:
        raise IPCError(code, where)
    return code


def _d(a):
    return a.ctypes.data_as(_D)


def _i(a):
    return a.ctypes.data_as(_I)


# ---------------------------------------------------------------------------
# PyTorch memory and stream plumbing
# ---------------------------------------------------------------------------

class TorchRuntime:
    """ipc_runtime whose alloc/free go to PyTorch's caching allocator on the
    current device and whose stream is a torch stream."""

    def __init__(self, stream=None, mem_budget: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the IPC step runs only on the HIP device")
        self.torch = torch
        self.device = torch.cuda.current_device()
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._alloc = ALLOC_FN(self._alloc_cb)
        self._free = FREE_FN(self._free_cb)
        self.rt = ipc_runtime()
        self.rt.stream = C.c_void_p(self.stream.cuda_stream)
        self.rt.alloc = self._alloc
        self.rt.free = self._free
        self.rt.user = None
        self.rt.mem_budget = int(mem_budget)

    def _alloc_cb(self, nbytes, stream, user):
        try:
            return int(self.torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream))
        except Exception:  # out of memory: report NULL to the library
            return 0

    def _free_cb(self, ptr, nbytes, stream, user, _finalizing=sys.is_finalizing):
        # At interpreter shutdown torch (and HIP) may already be torn down;
        # the process is ending, so its device memory goes with it. (The
        # check is bound at definition: module globals such as `sys` may be
        # gone by the time a late callback runs.)
        if _finalizing():
            return
        self.torch.cuda.caching_allocator_delete(int(ptr))


# Scenes and engines still open at exit are closed by an atexit hook, which
# runs before module teardown (the hook is registered after torch is
# imported, and atexit runs hooks last-in first-out), so their device frees
# reach a live caching allocator instead of running from __del__ during
# interpreter finalisation.
_live = weakref.WeakSet()


def _close_live():
    objs = list(_live)
    # engines first: destroying one waits for the steps of scenes it holds
    for obj in sorted(objs, key=lambda o: not isinstance(o, Batch)):
        try:
            obj.close()
        except Exception:
            pass


_atexit_registered = False


def _track(obj):
    global _atexit_registered
    if not _atexit_registered:
        import torch  # noqa: F401  (imported first, so its own exit hooks run after ours)
        atexit.register(_close_live)
        _atexit_registered = True
    _live.add(obj)


def make_desc(scene, precision=IPC_FP64, pcg_tol=1e-12, max_newton=100, keep=None,
              precond=IPC_PRECOND_MULTILEVEL, barrier_hessian=IPC_BARRIER_PROJECTED,
              target_al=False, target_al_tol=0.0, target_al_max=0) -> ipc_scene_desc:
    """ipc_scene_desc of a scenes.Scene; `keep` collects the numpy arrays that
    must outlive the create call."""
    X = np.ascontiguousarray(scene.X, dtype=np.float64)
    T = np.ascontiguousarray(scene.T, dtype=np.int32)
    fx = np.ascontiguousarray(scene.fixed, dtype=np.uint8)
    Y = np.ascontiguousarray(scene.Y, dtype=np.float64)
    F = np.ascontiguousarray(scene.F, dtype=np.int32)
    if keep is not None:
        keep.extend([X, T, fx, Y, F])
    d = ipc_scene_desc()
    d.n_verts, d.X = len(X), _d(X)
    d.n_tets, d.T = len(T), _i(T)
    d.fixed = fx.ctypes.data_as(_U8)
    d.E, d.nu, d.rho = scene.E, scene.nu, scene.rho
    d.n_ind_verts, d.ind_Y = len(Y), _d(Y)
    d.n_ind_tris, d.ind_tris = len(F), _i(F)
    for k, v in enumerate(np.asarray(scene.poses[0], dtype=np.float64).ravel()):
        d.ind_pose0[k] = v
    d.dt, d.dhat, d.kappa, d.k_target = scene.dt, scene.dhat, scene.kappa, scene.k_target
    d.newton_tol, d.pcg_tol = scene.newton_tol, pcg_tol
    for k in range(3):
        d.gravity[k] = scene.gravity[k]
    d.mu_friction = scene.meta.get("mu", 0.0) if scene.meta else 0.0
    d.eps_v = scene.meta.get("eps_v", 0.0) if scene.meta else 0.0
    d.ccd_s = 0.1
    d.ls_min_ratio = 2.0 ** -30
    d.self_contact = int(scene.self_contact)
    d.precision = precision
    d.max_newton = max_newton
    d.pcg_max_iter = 0
    d.ccd_max_iter = 10000
    d.precond = precond
    d.barrier_hessian = barrier_hessian
    d.target_al = int(bool(target_al))
    d.target_al_tol = target_al_tol
    d.target_al_max = target_al_max
    at = getattr(scene, "attached", None)
    if at is not None:
        at = np.ascontiguousarray(at, dtype=np.uint8)
        if keep is not None:
            keep.append(at)
        d.attached = at.ctypes.data_as(_U8)
    return d


def req_of(pose, case_pose=None) -> ipc_step_req:
    r = ipc_step_req()
    for k, v in enumerate(np.asarray(pose, dtype=np.float64).ravel()):
        r.pose[k] = v
    if case_pose is not None:
        for k, v in enumerate(np.asarray(case_pose, dtype=np.float64).ravel()):
            r.case_pose[k] = v
        r.case_pose_set = 1
    return r


def scene_case_pose(scene, step):
    """The scene's case pose for `step` (None when the scene has none)."""
    cp = getattr(scene, "case_poses", None)
    return None if cp is None else cp[step]


def tuning_for(n_verts):
    """The autotuner's choices a scene of n_verts vertices would take now."""
    o = np.zeros(6)
    _check(lib().ipcx_tuning_for(int(n_verts), _d(o)), "ipcx_tuning_for")
    return {"spmv_one_lane_rows": int(o[0]), "mas_target": int(o[1]), "pcg_first_chunk": float(o[2]),
            "pcg_later_chunk": float(o[3]), "from_file": bool(o[4]),
            "pcg_list_quantile": float(o[5])}


class GelScene:
    """One library scene built from a scenes.Scene."""

    def __init__(self, scene, runtime: TorchRuntime | None = None, precision=IPC_FP64, pcg_tol=1e-12,
                 max_newton=100, precond=IPC_PRECOND_MULTILEVEL, barrier_hessian=IPC_BARRIER_PROJECTED,
                 target_al=False, target_al_tol=0.0, target_al_max=0):
        self.scene = scene
        self.runtime = runtime or TorchRuntime()
        keep = []
        self.desc = make_desc(scene, precision, pcg_tol, max_newton, keep, precond, barrier_hessian,
                              target_al, target_al_tol, target_al_max)
        self._keep = keep
        h = C.c_void_p()
        _check(lib().ipc_create_scene(C.byref(self.desc), C.byref(self.runtime.rt), C.byref(h)),
               "ipc_create_scene")
        self.ptr = h
        _track(self)
        sz = np.zeros(8, dtype=np.int32)
        lib().ipc_scene_sizes(self.ptr, _i(sz))
        (self.n, self.n_gel, self.n_tet, self.n_pts, self.n_edges, self.n_tris, self.n_ind,
         self.n_gel_tris) = map(int, sz)
        self.step_index = 0

    def close(self):
        if getattr(self, "ptr", None):
            lib().ipc_destroy_scene(self.ptr)
            self.ptr = None

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return  # the atexit hook closed it, or the process is ending anyway
        try:
            self.close()
        except Exception:
            pass

    def step(self, pose=None, case_pose=None):
        if pose is None:
            pose = self.scene.poses[self.step_index + 1]
        if case_pose is None:
            case_pose = scene_case_pose(self.scene, self.step_index + 1)
        st = ipc_step_stats()
        rc = _check(lib().ipc_step(self.ptr, C.byref(req_of(pose, case_pose)), C.byref(st)), "ipc_step")
        self.step_index += 1
        return rc, st

    def height_map(self, x0, y0, dx, dy, nx, ny, z_ref, device_out=None):
        """Indentation depth below z_ref of the deformed gel surface on an
        nx x ny pixel grid (row j, column i at (x0 + i dx, y0 + j dy)); host
        (ny, nx) array, or written into a device tensor of nx ny doubles."""
        sp = ipc_height_map_spec(float(x0), float(y0), float(dx), float(dy), float(z_ref), int(nx), int(ny))
        if device_out is not None:
            _check(lib().ipc_height_map(self.ptr, C.byref(sp), C.c_void_p(device_out.data_ptr()), device_out.numel(),
                                        IPC_DEVICE, None), "ipc_height_map")
            return device_out
        out = np.zeros((int(ny), int(nx)))
        _check(lib().ipc_height_map(self.ptr, C.byref(sp), out.ctypes.data_as(C.c_void_p), out.size, IPC_HOST, None),
               "ipc_height_map")
        return out

    def height_map_noalloc(self, x0, y0, dx, dy, nx, ny, z_ref, device_out=None):
        """height_map through the allocation-free entry point (pixel keys in
        the library's own device array, at most IPC_HEIGHT_MAP_NOALLOC_MAX_PIXELS)."""
        sp = ipc_height_map_spec(float(x0), float(y0), float(dx), float(dy), float(z_ref), int(nx), int(ny))
        if device_out is not None:
            _check(lib().ipc_height_map_noalloc(self.ptr, C.byref(sp), C.c_void_p(device_out.data_ptr()),
                                                device_out.numel(), IPC_DEVICE, None), "ipc_height_map_noalloc")
            return device_out
        out = np.zeros((int(ny), int(nx)))
        _check(lib().ipc_height_map_noalloc(self.ptr, C.byref(sp), out.ctypes.data_as(C.c_void_p), out.size,
                                            IPC_HOST, None), "ipc_height_map_noalloc")
        return out

    def read_surface(self, device_out=None):
        """Surface positions (host numpy, or into a device tensor) and the
        object position (mean of all gel vertices)."""
        ns = C.c_int32()
        lib().ipc_surface_topology(self.ptr, None, 0, None, None, 0, C.byref(ns))
        obj = np.zeros(3)
        if device_out is not None:
            _check(lib().ipc_read_surface(self.ptr, C.c_void_p(device_out.data_ptr()), device_out.numel(),
                                          IPC_DEVICE, C.c_void_p(self.runtime.stream.cuda_stream), _d(obj)),
                   "ipc_read_surface")
            return device_out, obj
        out = np.zeros((ns.value, 3))
        _check(lib().ipc_read_surface(self.ptr, out.ctypes.data_as(C.c_void_p), out.size, IPC_HOST, None, _d(obj)),
               "ipc_read_surface")
        return out, obj

    def surface_topology(self):
        nt, ns = C.c_int32(), C.c_int32()
        lib().ipc_surface_topology(self.ptr, None, 0, C.byref(nt), None, 0, C.byref(ns))
        tris = np.zeros((nt.value, 3), dtype=np.int32)
        verts = np.zeros(ns.value, dtype=np.int32)
        _check(lib().ipc_surface_topology(self.ptr, _i(tris), tris.size, C.byref(nt), _i(verts), verts.size,
                                          C.byref(ns)), "ipc_surface_topology")
        return tris, verts

    def reset(self):
        _check(lib().ipc_reset(self.ptr), "ipc_reset")
        self.step_index = 0

    def save_state(self) -> bytes:
        nb = lib().ipc_state_bytes(self.ptr)
        buf = C.create_string_buffer(nb)
        _check(lib().ipc_save_state(self.ptr, buf, nb), "ipc_save_state")
        return buf.raw

    def load_state(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        _check(lib().ipc_load_state(self.ptr, buf, len(blob)), "ipc_load_state")

    # ---- test-only hooks ----
    def begin_step(self, pose, case_pose=None):
        _check(lib().ipcx_begin_step(self.ptr, C.byref(req_of(pose, case_pose))), "ipcx_begin_step")

    def newton_iterate(self, x_in):
        x_in = np.ascontiguousarray(x_in, dtype=np.float64)
        out = np.zeros_like(x_in)
        st = ipc_step_stats()
        rc = _check(lib().ipcx_newton_iterate(self.ptr, _d(x_in), _d(out), C.byref(st)), "ipcx_newton_iterate")
        return rc, out, st

    def candidates(self, x, p=None):
        x = np.ascontiguousarray(x, dtype=np.float64)
        pp = None if p is None else np.ascontiguousarray(p, dtype=np.float64)
        cnt = C.c_int64()
        _check(lib().ipcx_candidates(self.ptr, _d(x), None if pp is None else _d(pp), None, 0, C.byref(cnt)),
               "ipcx_candidates")
        out = np.zeros((max(cnt.value, 1), 3), dtype=np.int32)
        _check(lib().ipcx_candidates(self.ptr, _d(x), None if pp is None else _d(pp), _i(out), cnt.value,
                                     C.byref(cnt)), "ipcx_candidates")
        return out[:cnt.value]

    def primitives(self):
        pts = np.zeros(self.n_pts, dtype=np.int32)
        edges = np.zeros((self.n_edges, 2), dtype=np.int32)
        tris = np.zeros((self.n_tris, 3), dtype=np.int32)
        lib().ipcx_primitives(self.ptr, _i(pts), _i(edges), _i(tris))
        return pts, edges, tris

    def gradient(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        g = np.zeros_like(x)
        _check(lib().ipcx_gradient(self.ptr, _d(x), _d(g)), "ipcx_gradient")
        return g

    def hess_apply(self, x, v):
        x = np.ascontiguousarray(x, dtype=np.float64)
        v = np.ascontiguousarray(v, dtype=np.float64)
        y = np.zeros_like(x)
        _check(lib().ipcx_hess_apply(self.ptr, _d(x), _d(v), _d(y)), "ipcx_hess_apply")
        return y

    def assemble_elastic(self, x, v=None):
        """The body stage alone: its gradient at x, and H_body v if v is given."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        g = np.zeros_like(x)
        if v is None:
            _check(lib().ipcx_assemble_elastic(self.ptr, _d(x), _d(g), None, None), "ipcx_assemble_elastic")
            return g
        v = np.ascontiguousarray(v, dtype=np.float64)
        y = np.zeros_like(x)
        _check(lib().ipcx_assemble_elastic(self.ptr, _d(x), _d(g), _d(v), _d(y)), "ipcx_assemble_elastic")
        return g, y

    def barrier_pairs(self, x):
        """The barrier stage alone: kind (n,), vertex ids (n, 4), gradients
        (n, 12), Hessians (n, 12, 12) of the active pairs at x."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        cnt = C.c_int64()
        _check(lib().ipcx_barrier(self.ptr, _d(x), 0, None, None, None, None, C.byref(cnt)), "ipcx_barrier")
        n = cnt.value
        kind = np.zeros(max(n, 1), dtype=np.int32)
        v4 = np.zeros((max(n, 1), 4), dtype=np.int32)
        g = np.zeros((max(n, 1), 12))
        H = np.zeros((max(n, 1), 12, 12))
        _check(lib().ipcx_barrier(self.ptr, _d(x), n, _i(kind), _i(v4), _d(g), _d(H), C.byref(cnt)), "ipcx_barrier")
        return kind[:n], v4[:n], g[:n], H[:n]

    def pcg(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        p = np.zeros_like(x)
        it = C.c_int32()
        _check(lib().ipcx_pcg(self.ptr, _d(x), _d(p), C.byref(it)), "ipcx_pcg")
        return p, it.value

    def energy(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        E = C.c_double()
        _check(lib().ipcx_energy(self.ptr, _d(x), C.byref(E)), "ipcx_energy")
        return E.value

    def ccd(self, x, p):
        x = np.ascontiguousarray(x, dtype=np.float64)
        p = np.ascontiguousarray(p, dtype=np.float64)
        a = C.c_double()
        _check(lib().ipcx_ccd(self.ptr, _d(x), _d(p), C.byref(a)), "ipcx_ccd")
        return a.value

    def profile(self, enable=True):
        _check(lib().ipcx_profile(self.ptr, int(enable)), "ipcx_profile")

    PROF_KERNELS = ("pcg_spmv", "pcg_update", "elastic", "assemble", "broad_phase", "barrier", "energy", "ccd")

    def profile_read(self):
        out = {}
        for k, name in enumerate(self.PROF_KERNELS):
            n = C.c_int64()
            ms = C.c_double()
            lib().ipcx_profile_read(self.ptr, k, C.byref(n), C.byref(ms))
            out[name] = (n.value, ms.value)
        return out

    def profile_totals(self, kernel):
        """(launches, summed algorithmic bytes) of every launch of PCG class
        0 or 1 while profiling was on."""
        n = C.c_int64()
        by = C.c_double()
        _check(lib().ipcx_profile_totals(self.ptr, int(kernel), C.byref(n), C.byref(by)), "ipcx_profile_totals")
        return n.value, by.value

    def profile_bytes(self, kernel):
        """Summed algorithmic bytes of the timed launches of PCG kernel class
        0 (SpMV) or 1 (update)."""
        by = C.c_double()
        _check(lib().ipcx_profile_bytes(self.ptr, int(kernel), C.byref(by)), "ipcx_profile_bytes")
        return by.value

    def matrix_info(self):
        o = np.zeros(8, dtype=np.int64)
        lib().ipcx_matrix_info(self.ptr, o.ctypes.data_as(_I64))
        keys = ("nnzb", "bell_entries", "n", "n_active", "n_tets", "n_cand", "n_cand_swept", "n_gather")
        return dict(zip(keys, map(int, o)))

    def tuning(self):
        """The autotuner's choices this scene took at creation."""
        o = np.zeros(6)
        _check(lib().ipcx_tuning(self.ptr, _d(o)), "ipcx_tuning")
        return {"spmv_one_lane_rows": int(o[0]), "mas_target": int(o[1]), "pcg_first_chunk": float(o[2]),
                "pcg_later_chunk": float(o[3]), "from_file": bool(o[4]),
            "pcg_list_quantile": float(o[5])}

    def precond_info(self):
        o = np.zeros(8, dtype=np.int64)
        _check(lib().ipcx_precond_info(self.ptr, o.ctypes.data_as(_I64)), "ipcx_precond_info")
        keys = ("levels", "groups", "aggs0", "aggs1", "aggs2", "max_group_members", "max_group_aggs", "members")
        return dict(zip(keys, map(int, o)))

    @property
    def x(self):
        x = np.zeros((self.n, 3))
        _check(lib().ipcx_get_state(self.ptr, _d(x), None), "ipcx_get_state")
        return x

    @x.setter
    def x(self, val):
        val = np.ascontiguousarray(val, dtype=np.float64)
        _check(lib().ipcx_set_state(self.ptr, _d(val), None), "ipcx_set_state")

    @property
    def v(self):
        v = np.zeros((self.n, 3))
        _check(lib().ipcx_get_state(self.ptr, None, _d(v)), "ipcx_get_state")
        return v

    @v.setter
    def v(self, val):
        val = np.ascontiguousarray(val, dtype=np.float64)
        _check(lib().ipcx_set_state(self.ptr, None, _d(val)), "ipcx_set_state")


class Batch:
    """The library's continuous-batching engine (ipc_batch_*).

    submit() queues one step per scene and returns tickets at once; a native
    worker thread runs every in-flight step in shared launches (one launch per
    phase for the whole list) and admits newly submitted steps at each Newton
    iteration boundary. Results are bitwise those of GelScene.step().
    mem_budget > 0 caps the summed device bytes of the scenes in flight."""

    def __init__(self, stream=None, mem_budget: int = 0):
        self.rt = ipc_runtime()
        self.rt.stream = None if stream is None else C.c_void_p(stream.cuda_stream)
        self.rt.alloc = ALLOC_FN()
        self.rt.free = FREE_FN()
        self.rt.user = None
        self.rt.mem_budget = int(mem_budget)
        h = C.c_void_p()
        _check(lib().ipc_batch_create(C.byref(self.rt), C.byref(h)), "ipc_batch_create")
        self.ptr = h
        _track(self)

    def close(self):
        if getattr(self, "ptr", None):
            lib().ipc_batch_destroy(self.ptr)
            self.ptr = None

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def submit(self, scenes, poses=None):
        """Queue one step for each GelScene (pose: the scene's next trajectory
        pose unless given). Returns the tickets."""
        n = len(scenes)
        if poses is None:
            poses = [g.scene.poses[g.step_index + 1] for g in scenes]
        ptrs = (C.c_void_p * n)(*[g.ptr.value for g in scenes])
        reqs = (ipc_step_req * n)(*[req_of(p, scene_case_pose(g.scene, g.step_index + 1))
                                     for p, g in zip(poses, scenes)])
        tk = np.zeros(n, dtype=np.int64)
        _check(lib().ipc_batch_submit(self.ptr, n, ptrs, reqs, tk.ctypes.data_as(_I64)), "ipc_batch_submit")
        for g in scenes:
            g.step_index += 1
        return [int(t) for t in tk]

    def poll(self, ticket):
        """(done, stats): done is True once the step has finished."""
        st = ipc_step_stats()
        rc = _check(lib().ipc_batch_poll(self.ptr, int(ticket), C.byref(st)), "ipc_batch_poll")
        return rc == 1, st

    def wait(self, ticket):
        """Block until the step is done; returns (status, stats). The ticket
        is consumed."""
        st = ipc_step_stats()
        rc = lib().ipc_batch_wait(self.ptr, int(ticket), C.byref(st))
        if rc < 0:
            raise IPCError(rc, "ipc_batch_wait")
        return rc, st

    def next(self, timeout_ms=-1.0):
        """The oldest finished step not yet consumed: (ticket, status, stats),
        waiting up to timeout_ms (< 0: without limit); None on timeout."""
        t = np.zeros(1, dtype=np.int64)
        stt = C.c_int32()
        st = ipc_step_stats()
        rc = _check(lib().ipc_batch_next(self.ptr, float(timeout_ms), t.ctypes.data_as(_I64), C.byref(stt),
                                         C.byref(st)), "ipc_batch_next")
        return (int(t[0]), int(stt.value), st) if rc == 1 else None

    def profile(self, enable=True):
        _check(lib().ipc_batch_profile(self.ptr, int(bool(enable))), "ipc_batch_profile")

    def profile_totals(self, kernel):
        """(launches, summed algorithmic bytes) of every launch of PCG class
        0 or 1 while profiling was on."""
        n = np.zeros(1, dtype=np.int64)
        by = np.zeros(1)
        _check(lib().ipc_batch_profile_totals(self.ptr, int(kernel), n.ctypes.data_as(_I64), _d(by)),
               "ipc_batch_profile_totals")
        return int(n[0]), float(by[0])

    def profile_read(self, kernel):
        """(timed launches, summed ms, summed algorithmic bytes) of a kernel class."""
        n = np.zeros(1, dtype=np.int64)
        ms = np.zeros(1)
        by = np.zeros(1)
        _check(lib().ipc_batch_profile_read(self.ptr, int(kernel), n.ctypes.data_as(_I64), _d(ms), _d(by)),
               "ipc_batch_profile_read")
        return int(n[0]), float(ms[0]), float(by[0])

    def profile_large(self, kernel):
        """(timed launches, summed ms, summed algorithmic bytes) of a PCG
        kernel class, over the iterations whose SpMV launch moves at least
        256 MiB (more than the Infinity Cache holds)."""
        n = np.zeros(1, dtype=np.int64)
        ms = np.zeros(1)
        by = np.zeros(1)
        _check(lib().ipc_batch_profile_large(self.ptr, int(kernel), n.ctypes.data_as(_I64), _d(ms), _d(by)),
               "ipc_batch_profile_large")
        return int(n[0]), float(ms[0]), float(by[0])
