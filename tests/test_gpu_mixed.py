"""Mixed precision against the FP64 oracle.

The mixed form computes the element gradients and Hessians, the assembled
matrix and preconditioner, the SpMV and the PCG vectors in FP32 with FP64
dot-product accumulation; positions, distances, CCD, barrier energies, the
line-search sums and the Newton stopping test stay FP64.

Tolerances (mixed path, L = rest-gel bbox diagonal):
  one teacher-forced Newton iterate        1e-4 L
  free-running config-1 trajectory         1e-4 L at the final step
  invariants (every tet J > 0, every candidate pair d > 0) after every step
"""
import sys

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

MIXED_PCG_TOL = 1e-7  # inner solves converged far enough that the iterate error is the mixed form's, not PCG's


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


def test_mixed_teacher_forced_newton_iterates(ipc, c1_oracle_trajectory):
    sc, traj, _ = c1_oracle_trajectory
    L = sc.bbox_diag
    g = ipc.GelScene(sc, precision=ipc.IPC_MIXED, pcg_tol=MIXED_PCG_TOL)
    worst = 0.0
    checked = 0
    for step, (x0, v0, pose, xs) in enumerate(traj):
        if step not in (0, 3, 6, 9):
            continue
        g.x = x0
        g.v = v0
        g.begin_step(pose)
        for k in range(min(len(xs) - 1, 4)):
            rc, xg, st = g.newton_iterate(xs[k])
            assert rc == 0
            err = np.abs(xg - xs[k + 1]).max() / L
            worst = max(worst, err)
            checked += 1
            say(f"  mixed step {step} iterate {k}: err/L = {err:.3e} alpha={st.alpha:.4f} pcg={st.pcg_iters}")
            assert err <= 1e-4
    assert checked >= 8
    say("mixed teacher-forced worst err/L", worst)


def test_mixed_free_running_trajectory(ipc, c1_oracle_trajectory):
    sc, _, x_oracle_final = c1_oracle_trajectory
    L = sc.bbox_diag
    g = ipc.GelScene(sc, precision=ipc.IPC_MIXED, pcg_tol=MIXED_PCG_TOL)
    o = O.OracleScene(sc)
    T = sc.T
    for step in range(1, sc.n_steps + 1):
        rc, st = g.step()
        say(f"  mixed step {step}: rc={rc} newton={st.newton_iters} pcg={st.pcg_iters} active={st.n_active} "
            f"ms={st.ms_total:.1f}")
        assert rc in (0, 4)
        x = g.x
        P = x[T]
        J = np.linalg.det(np.stack([P[:, 1] - P[:, 0], P[:, 2] - P[:, 0], P[:, 3] - P[:, 0]], 2))
        assert J.min() > 0
        c = o.candidates(x)
        assert o.candidate_distances(x, c)[0].min() > 0
    err = np.abs(g.x - x_oracle_final).max() / L
    say("mixed free-running final-step error / L =", err, " (um:", err * L * 1e6, ")")
    assert err <= 1e-4


def test_mixed_gradient_close_to_fp64(ipc):
    """The FP32 element gradients gathered in FP64 stay within FP32 rounding of
    the FP64 oracle's gradient (relative to its largest entry)."""
    from paper_2411_04776_amd import scenes as S
    sc = S.config1()
    g = ipc.GelScene(sc, precision=ipc.IPC_MIXED, pcg_tol=MIXED_PCG_TOL)
    o = O.OracleScene(sc)
    pose = sc.poses[3]
    g.begin_step(pose)
    o.begin_step(pose)
    x = o.x.copy()
    x[o.n_gel:] -= np.array([0, 0, 0.8 * sc.dhat])  # indenter inside the barrier band of the top surface
    rng = np.random.default_rng(3)
    x[:o.n_gel] += rng.normal(0, 0.05 * sc.dhat, (o.n_gel, 3)) * (1 - sc.fixed[:, None])
    go, gg = o.gradient(x), g.gradient(x)
    scale = np.abs(go).max()
    err = np.abs(gg - go).max() / scale
    say("mixed gradient rel err", err)
    assert err <= 1e-5
