"""ipc_height_map_noalloc (the allocation-free entry point) through the C ABI
against ipc_height_map on the same scene state: equal bit for bit (same
kernels, same FP64 expressions), host and device output, two calls in a row
with the second on a smaller grid (the shared device array keeps the first
call's keys; each call must clear what it uses), and a grid above the
array's size refused on the host with IPC_E_INVALID_ARG."""
import ctypes as C
import sys

import numpy as np
import pytest

from paper_2411_04776_amd import scenes as S

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ipc():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_2411_04776_amd import ipc as I
    I.lib()
    return I


def dented(sc, depth=4e-4, seed=11):
    """Rest state with a seeded Gaussian dent and jitter on the free vertices."""
    X = sc.X
    rng = np.random.default_rng(seed)
    c = X.mean(0)
    r2 = ((X[:, 0] - c[0]) ** 2 + (X[:, 1] - c[1]) ** 2) / (3e-3) ** 2
    x = X.copy()
    x[:, 2] -= depth * np.exp(-r2) * (X[:, 2] / X[:, 2].max())
    x += rng.normal(0, 2e-6, x.shape) * (1 - sc.fixed[:, None])
    return x


def test_noalloc_height_map_equals_allocating_one(ipc):
    import torch
    sc = S.config2()
    g = ipc.GelScene(sc)
    full = g.x.copy()
    full[:len(sc.X)] = dented(sc)
    g.x = full
    X = sc.X
    ztop = X[:, 2].max()
    lo, hi = X.min(0), X.max(0)
    # first call: 640 x 800 (512,000 pixels); second: a smaller, shifted grid
    for (nx, ny) in ((640, 800), (200, 150)):
        dx, dy = (hi[0] - lo[0]) / (nx - 5), (hi[1] - lo[1]) / (ny - 5)
        x0, y0 = lo[0] - 2 * dx, lo[1] - 2 * dy
        say(f"  grid {nx}x{ny}: host output")
        ref = g.height_map(x0, y0, dx, dy, nx, ny, ztop)
        got = g.height_map_noalloc(x0, y0, dx, dy, nx, ny, ztop)
        say(f"    max depth {ref.max():.3e} m, equal {np.array_equal(ref, got)}")
        assert ref.max() > 1e-4
        assert np.array_equal(ref, got)
        say(f"  grid {nx}x{ny}: device output")
        dev = torch.full((nx * ny,), -1.0, dtype=torch.float64, device="cuda")
        g.height_map_noalloc(x0, y0, dx, dy, nx, ny, ztop, device_out=dev)
        torch.cuda.synchronize()
        assert np.array_equal(dev.cpu().numpy().reshape(ny, nx), ref)
    g.close()


def test_noalloc_height_map_second_scene_and_limits(ipc):
    # a second scene on the same GPU shares the array: a smaller call right
    # after the larger ones above sees none of their pixels
    sc = S.config1()
    g = ipc.GelScene(sc)
    X = sc.X
    nx, ny = 64, 48
    lo, hi = X.min(0), X.max(0)
    dx, dy = (hi[0] - lo[0]) / (nx - 5), (hi[1] - lo[1]) / (ny - 5)
    x0, y0 = lo[0] - 2 * dx, lo[1] - 2 * dy
    ref = g.height_map(x0, y0, dx, dy, nx, ny, X[:, 2].max())
    got = g.height_map_noalloc(x0, y0, dx, dy, nx, ny, X[:, 2].max())
    assert np.array_equal(ref, got)
    far = g.height_map_noalloc(1.0, 1.0, dx, dy, 8, 8, X[:, 2].max())
    assert np.all(far == 0.0)
    # above the array's size: refused before any launch
    L = ipc.lib()
    cap = (1 << 20) + 1
    out = np.zeros(cap)
    sp = ipc.ipc_height_map_spec(x0, y0, dx, dy, 0.0, cap, 1)
    rc = L.ipc_height_map_noalloc(g.ptr, C.byref(sp), out.ctypes.data_as(C.c_void_p), cap, ipc.IPC_HOST, None)
    assert rc == ipc.IPC_E_INVALID_ARG
    with pytest.raises(ipc.IPCError):
        g.height_map_noalloc(x0, y0, -dx, dy, nx, ny, 0.0)
    g.close()
