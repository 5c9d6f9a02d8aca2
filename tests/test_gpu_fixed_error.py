"""Fixed-error check of config 2 (40x50x8 gel): stepped through all 50 steps
at the benchmark's PCG tolerance (3e-5), the final positions of every gel
vertex end within 1e-4 L of the FP64 oracle's
(tests/golden/c2_seed{S}_final.npz, written by make_fullsize.py from the
oracle at PCG tolerance 1e-12): seed 0 (cylinder) in FP64 and in the mixed
form, with either preconditioner and with the Gauss-Newton barrier Hessian;
seeds 1-5 (cube edge, bumpy plate, ...) in FP64 and mixed. Seed 5 (a bumpy
plate) ends its last step at the Newton cap in the oracle's run (100
iterations, |p|_inf still above 1e-6 m) and in both HIP forms (1.99e-6 m):
a warning with a feasible state, accepted here; its final positions still
meet the bound. Seed 3 (a
cylinder) sets the tolerance: its worst vertex, beside the contact edge where
the soft barrier lets looser solves take the trajectory elsewhere, ends
1e-5 L away at 3e-5, 5.6e-5 L at 1e-4 with the 512-member preconditioner
groups and 5.2e-4 L at 1e-4 with the 256-member ones, 6.1e-4 L at 1e-3; at
3e-5 and 1e-5 the two preconditioners agree (8.9e-6 / 1.0e-5 and 5.3e-6 /
5.2e-6). Seed 0 at 1e-3 (3.0e-5 L) is recorded as a form of its own.

The Gauss-Newton form is held to the oracle's trajectory in the same form
(c2_seed0_gn_final.npz): its Newton stop test reads that form's direction,
so it leaves each non-convex step at its own point. Against the projected
oracle it ends 1.1e-4 L away at a vertex on the cylinder's edge, and a
tighter Newton tolerance moves it further (4e-4 L at a quarter): it does
not converge toward the projected form's path."""
import os
import sys

import numpy as np
import pytest

from paper_2411_04776_amd import scenes as S

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
BENCH_PCG_TOL = 3e-5


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


def golden(seed, gn=False):
    name = f"c2_seed{seed}_gn_final.npz" if gn else f"c2_seed{seed}_final.npz"
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.skip(f"{name} not generated")
    z = np.load(path)
    return z["dx"].astype(np.float64), float(z["L"])


def run(ipc, seed, form):
    dx, L = golden(seed, gn=form == "fp64-gauss-newton")
    sc = S.config2(seed)
    ref = sc.X + dx
    kw = dict(pcg_tol=1e-3 if form == "fp64-tol1e-3" else BENCH_PCG_TOL)
    if form == "mixed":
        kw["precision"] = ipc.IPC_MIXED
    if form == "fp64-jacobi":
        kw["precond"] = ipc.IPC_PRECOND_JACOBI
    if form == "fp64-gauss-newton":
        kw["barrier_hessian"] = ipc.IPC_BARRIER_GAUSS_NEWTON
    g = ipc.GelScene(sc, **kw)
    newton = 0
    capped = []
    for k in range(sc.n_steps):
        rc, st = g.step()
        # 1: the Newton cap spent with a feasible state committed (the
        # oracle's own run of seed 5 ends its last step there too)
        assert rc in (0, 1, 4), (k, rc)
        if rc == 1:
            capped.append((k + 1, round(st.pinf * 1e6, 3)))
        newton += st.newton_iters
    d = np.linalg.norm(g.x[:len(ref)] - ref, axis=1)
    err = d.max() / L
    say(f"  seed {seed} ({sc.meta['kind']}) {form}: 50 steps, {newton} Newton iterations, final error / L = "
        f"{err:.3e} ({err * L * 1e6:.3f} um, at vertex {int(d.argmax())}), mean {d.mean() / L:.2e}"
        + (f"; Newton cap at (step, |p|_inf um) {capped}" if capped else ""))
    g.close()
    return err


@pytest.mark.parametrize("form", ["fp64", "mixed", "fp64-jacobi", "fp64-gauss-newton", "fp64-tol1e-3"])
def test_c2_seed0_final_error(ipc, form):
    assert run(ipc, 0, form) <= 1e-4


@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("form", ["fp64", "mixed"])
def test_c2_other_seeds_final_error(ipc, seed, form):
    assert run(ipc, seed, form) <= 1e-4
