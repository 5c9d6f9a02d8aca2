"""Lagged friction on the HIP path against the FP64 oracle.

The friction set of a step (pairs active at x^t with their normal force,
closest-point coefficients and normal) is built on the device at the step
start; during the step every friction pair adds mu*lambda*f0(|u|) and its
gradient and PSD Hessian to the system as an extra pair after the barrier
pairs.

Tolerances (FP64 path, L = rest-gel bbox diagonal):
  gradient, H v                           1e-11 of the largest entry of the row block (gel, indenter)
  energy                                  1e-13 relative
  one teacher-forced Newton iterate       1e-9 L
  free-running sliding trajectory          1e-8 L at every step
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2411_04776_amd import scenes as S
from parity_util import assert_rows_close

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


def test_friction_free_running_matches_oracle(ipc):
    sc = S.tiny_slide_scene(mu=0.5)
    g = ipc.GelScene(sc)
    o = O.OracleScene(sc)
    L = sc.bbox_diag
    for k in range(1, sc.n_steps + 1):
        rc, st = g.step()
        o.step(sc.poses[k])
        err = np.abs(g.x - o.x).max() / L
        say(f"  slide step {k}: rc={rc} newton={st.newton_iters} active={st.n_active} "
            f"friction pairs={len(o.friction_set()[3])} err/L={err:.2e}")
        assert rc in (0, 4)
        assert err <= 1e-8


def test_friction_teacher_forced_and_derivatives(ipc):
    sc = S.tiny_slide_scene(mu=0.5)
    L = sc.bbox_diag
    o = O.OracleScene(sc)
    for k in range(1, sc.n_steps):
        o.step(sc.poses[k])
    g = ipc.GelScene(sc)
    g.x, g.v = o.x, o.v
    pose = sc.poses[sc.n_steps]
    o.begin_step(pose)
    g.begin_step(pose)
    assert len(o.friction_set()[3]) > 0
    x = o.x
    for it in range(3):
        r, xo, _ = o.newton_iterate(x)
        rg, xg, _ = g.newton_iterate(x)
        if r != 0:
            break
        assert rg == 0
        err = np.abs(xg - xo).max() / L
        say(f"  slide iterate {it}: err/L={err:.2e}")
        assert err <= 1e-9
        x = xo
    go, gg = o.gradient(x), g.gradient(x)
    assert_rows_close(gg, go, o.n_gel, 1e-11)
    v = np.random.default_rng(2).normal(size=x.shape)
    yo, yg = o.hess_apply(x, v), g.hess_apply(x, v)
    assert_rows_close(yg, yo, o.n_gel, 1e-11)
    Eo, Eg = o.energy(x), g.energy(x)
    assert abs(Eg - Eo) <= 1e-13 * abs(Eo)


def test_friction_batched_bitwise_and_mixed(ipc):
    """A friction scene stepped in a list with others is bitwise the same as
    alone; the mixed form stays within 1e-4 L of the FP64 oracle."""
    sc = S.tiny_slide_scene(mu=0.5)
    alone = ipc.GelScene(sc, pcg_tol=1e-8)
    ref = []
    for _ in range(sc.n_steps):
        alone.step()
        ref.append(alone.x)
    gs = [ipc.GelScene(sc, pcg_tol=1e-8), ipc.GelScene(S.tiny_scene(steps=sc.n_steps), pcg_tol=1e-8)]
    b = ipc.Batch()
    for k in range(sc.n_steps):
        tks = b.submit(gs)
        for t in tks:
            b.wait(t)
        assert np.array_equal(gs[0].x, ref[k])
    b.close()
    m = ipc.GelScene(sc, precision=ipc.IPC_MIXED, pcg_tol=1e-7)
    o = O.OracleScene(sc)
    for k in range(1, sc.n_steps + 1):
        m.step()
        o.step(sc.poses[k])
    err = np.abs(m.x - o.x).max() / sc.bbox_diag
    say("  mixed sliding final err/L", err)
    assert err <= 1e-4
