"""Fixed-error check of the benchmarked configuration: config 2 (40x50x8 gel,
cylinder seed 0) stepped through all 50 steps at the benchmark's PCG
tolerance (1e-3; 1e-4 too) ends within 1e-4 L of the FP64 oracle's final positions
(tests/golden/c2_seed0_final.txt, written by make_c2_final.py from the oracle
at PCG tolerance 1e-12), in FP64 and in the mixed form, with either
preconditioner and with the Gauss-Newton barrier Hessian."""
import os
import sys

import numpy as np
import pytest

from paper_2411_04776_amd import scenes as S

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_seed0_final.txt")


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


def golden():
    rows = np.loadtxt(GOLDEN, comments="#")
    return rows[:, 0].astype(np.int64), rows[:, 1:4]


@pytest.mark.parametrize("form", ["fp64", "mixed", "fp64-jacobi", "fp64-gauss-newton", "fp64-tol1e-4"])
def test_c2_final_error_at_benchmark_tolerance(ipc, form):
    idx, ref = golden()
    sc = S.config2(0)
    kw = dict(pcg_tol=1e-4 if form == "fp64-tol1e-4" else 1e-3)
    if form == "mixed":
        kw["precision"] = ipc.IPC_MIXED
    if form == "fp64-jacobi":
        kw["precond"] = ipc.IPC_PRECOND_JACOBI
    if form == "fp64-gauss-newton":
        kw["barrier_hessian"] = ipc.IPC_BARRIER_GAUSS_NEWTON
    g = ipc.GelScene(sc, **kw)
    newton = 0
    for k in range(sc.n_steps):
        rc, st = g.step()
        assert rc in (0, 4), (k, rc)
        newton += st.newton_iters
    L = sc.bbox_diag
    err = np.linalg.norm(g.x[idx] - ref, axis=1).max() / L
    say(f"  {form}: 50 steps, {newton} Newton iterations, final error / L = {err:.3e} ({err * L * 1e6:.3f} um)")
    assert err <= 1e-4
