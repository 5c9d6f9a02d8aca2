"""Attachment-driven gel (the sensor case moves the gel's bottom layer)
through the C ABI against the oracle: free-running FP64 trajectory to 1e-8 L
and mixed to 1e-4 L, teacher-forced iterates to 1e-9 L, the engine (case
poses carried by the step requests) bit for bit against ipc_step, and the
quasi-static rigid following of the case."""
import math
import sys

import numpy as np
import pytest

import oracle as O
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


def scene():
    return S.attached_scene(grid=(8, 10, 3), steps=6, depth=0.6e-3, tilt_deg=3.0, radius=4e-3)


@pytest.fixture(scope="module")
def attach_run():
    sc = scene()
    o = O.OracleScene(sc)
    traj = []
    for step in range(1, sc.n_steps + 1):
        pose, cpose = sc.poses[step], sc.case_poses[step]
        x0, v0 = o.x, o.v
        o.begin_step(pose, case_pose=cpose)
        xs = [x0]
        x = x0
        for _ in range(100):
            r, xn, st = o.newton_iterate(x)
            if r != 0:
                break
            xs.append(xn)
            x = xn
        traj.append((x0, v0, pose, cpose, xs))
        o.step(pose, case_pose=cpose)
    return sc, traj, o


@pytest.mark.parametrize("precision", [0, 1])
def test_attached_free_running(ipc, attach_run, precision):
    sc, traj, o = attach_run
    L = sc.bbox_diag
    g = ipc.GelScene(sc, precision=precision, pcg_tol=1e-12 if precision == 0 else 1e-7)
    for step in range(1, sc.n_steps + 1):
        rc, st = g.step()
        say(f"  prec {precision} step {step}: rc={rc} newton={st.newton_iters} (oracle {len(traj[step - 1][4]) - 1}) "
            f"active={st.n_active}")
        assert rc in (0, 4)
    err = np.abs(g.x - o.x).max() / L
    say("  final error / L", err)
    assert err <= (1e-8 if precision == 0 else 1e-4)
    assert st.n_active > 0


def test_attached_teacher_forced(ipc, attach_run):
    sc, traj, _ = attach_run
    L = sc.bbox_diag
    g = ipc.GelScene(sc)
    checked = 0
    for x0, v0, pose, cpose, xs in traj:
        g.x = x0
        g.v = v0
        g.begin_step(pose, case_pose=cpose)
        for k in range(min(len(xs) - 1, 3)):
            rc, xg, st = g.newton_iterate(xs[k])
            assert rc == 0
            assert np.abs(xg - xs[k + 1]).max() / L <= 1e-9
            checked += 1
    assert checked >= 10


def test_attached_engine_equals_alone(ipc):
    sc = scene()
    a = ipc.GelScene(sc)
    for _ in range(3):
        a.step()
    b_s = ipc.GelScene(sc)
    eng = ipc.Batch()
    for _ in range(3):
        for t in eng.submit([b_s]):
            rc, _ = eng.wait(t)
            assert rc == 0
    eng.close()
    assert np.array_equal(a.x, b_s.x)


def test_quasi_static_rigid_following(ipc):
    """Negligible inertia, no contact: the gel takes the case's rigid motion."""
    sc = S.attached_scene(grid=(5, 4, 3), steps=1)
    sc.rho = 1e-9
    sc.Y = sc.Y + np.array([0.0, 0.0, 0.05])
    sc.newton_tol = 1e-12
    g = ipc.GelScene(sc)
    Rc = S.rotation((0.3, -0.2, 1.0), math.radians(4.0))
    t = np.array([2e-4, 1e-4, -1e-4])
    rc, st = g.step(case_pose=S.pose_matrix(Rc, t))
    assert rc == 0
    err = np.abs(g.x[:len(sc.X)] - (sc.X @ Rc.T + t)).max()
    say("  rigid following error (m)", err)
    assert err <= 1e-10
