"""ipc_height_map through the C ABI against the oracle's height map on the
same positions (the oracle's own trajectory states, set into the scene):
every pixel equal (both evaluate the same FP64 expressions, correctly
rounded, in the same order), checked to 1e-15 m."""
import sys
import time

import numpy as np
import pytest

import oracle as O
from oracle.height_map import height_map
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


def grid_of(X, nx, ny, margin=2):
    lo, hi = X.min(0), X.max(0)
    dx, dy = (hi[0] - lo[0]) / (nx - 2 * margin - 1), (hi[1] - lo[1]) / (ny - 2 * margin - 1)
    return lo[0] - margin * dx, lo[1] - margin * dy, dx, dy


@pytest.mark.parametrize("name", ["config1", "config2"])
def test_height_map_matches_oracle(ipc, name):
    sc = S.config1() if name == "config1" else S.config2()
    o = O.OracleScene(sc)
    g = ipc.GelScene(sc)
    _, _, tris = o.surface()
    gt = tris[:o.n_gel_tris]
    X = sc.X
    ztop = X[:, 2].max()
    nx, ny = (160, 200) if name == "config1" else (320, 400)
    x0, y0, dx, dy = grid_of(X, nx, ny)
    # the rest state, a seeded Gaussian dent with jitter, and (config 1) the
    # oracle's own state after three steps
    rng = np.random.default_rng(7)
    x = o.x.copy()
    c = X.mean(0)
    r2 = ((X[:, 0] - c[0]) ** 2 + (X[:, 1] - c[1]) ** 2) / (3e-3) ** 2
    x[:o.n_gel, 2] -= 4e-4 * np.exp(-r2) * (X[:, 2] / X[:, 2].max())
    x[:o.n_gel] += rng.normal(0, 2e-6, (o.n_gel, 3)) * (1 - sc.fixed[:, None])
    states = [o.x, x]
    if name == "config1":
        for k in range(1, 4):
            o.step(sc.poses[k])
        states.append(o.x)
    for x in states:
        g.x = x
        t0 = time.perf_counter()
        mg = g.height_map(x0, y0, dx, dy, nx, ny, ztop)
        tg = time.perf_counter() - t0
        mo = height_map(x, gt, x0, y0, dx, dy, nx, ny, ztop)
        diff = np.abs(mg - mo).max()
        say(f"  {name}: {nx}x{ny} px, max depth {mo.max():.3e} m, max |gpu - oracle| {diff:.1e}, "
            f"exact {np.mean(mg == mo):.4f}, call {1e3 * tg:.2f} ms")
        assert diff <= 1e-15
    # a grid that misses the gel: all zero; a one-pixel grid
    far = g.height_map(1.0, 1.0, dx, dy, 8, 8, ztop)
    assert np.all(far == 0.0)
    one = g.height_map(X[:, 0].mean(), X[:, 1].mean(), dx, dy, 1, 1, ztop)
    assert one.shape == (1, 1)


def test_height_map_device_output_and_errors(ipc):
    import torch
    sc = S.config1()
    g = ipc.GelScene(sc)
    X = sc.X
    x0, y0, dx, dy = grid_of(X, 64, 48)
    host = g.height_map(x0, y0, dx, dy, 64, 48, X[:, 2].max())
    dev = torch.empty(64 * 48, dtype=torch.float64, device="cuda")
    g.height_map(x0, y0, dx, dy, 64, 48, X[:, 2].max(), device_out=dev)
    assert np.array_equal(dev.cpu().numpy().reshape(48, 64), host)
    with pytest.raises(ipc.IPCError):
        g.height_map(x0, y0, -dx, dy, 64, 48, 0.0)
    with pytest.raises(ipc.IPCError):
        g.height_map(x0, y0, dx, dy, 0, 48, 0.0)
