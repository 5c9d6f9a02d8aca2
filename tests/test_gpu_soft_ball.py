"""Two deformable bodies: the gel pad and a soft ball squeezed onto it by a
rigid plate (the soft-ball workload of the paper's GIPC timing table, at a
test size). Candidates bit-exact (gel-ball pairs among them), gradient and
H v to 1e-11, teacher-forced Newton iterates to 1e-9 L against the oracle;
a free-running trajectory keeps every tet positive and every pair apart and
ends within 1e-4 L of the oracle's."""
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


@pytest.fixture(scope="module")
def ball_run():
    """The oracle's tiny soft-ball trajectory: per step (x^t, v^t, pose, iterates)."""
    sc = S.soft_ball_scene("tiny", steps=8)
    o = O.OracleScene(sc)
    traj = []
    for step in range(1, sc.n_steps + 1):
        pose = sc.poses[step]
        x0, v0 = o.x, o.v
        o.begin_step(pose)
        xs = [x0]
        x = x0
        for _ in range(100):
            r, xn, st = o.newton_iterate(x)
            if r != 0:
                break
            xs.append(xn)
            x = xn
        traj.append((x0, v0, pose, xs))
        o.step(pose)
    return sc, traj, o


def gel_ball_pairs(o, sc, cand):
    ng = sc.meta["n_gel"]
    _, edges, tris = o.surface()
    n = 0
    for t, a, b in cand:
        vs = [a, *tris[b]] if t == 0 else [*edges[a], *edges[b]]
        sides = {int(v < ng) for v in vs if v < o.n_gel}
        n += len(sides) == 2
    return n


def test_soft_ball_candidates_and_derivatives(ipc, ball_run):
    sc, traj, o = ball_run
    g = ipc.GelScene(sc)
    # the last step's first Newton iterate: in contact, far from equilibrium
    pose = traj[-1][2]
    x = traj[-1][3][1]
    g.x = traj[-1][0]
    g.v = traj[-1][1]
    g.begin_step(pose)
    oo = O.OracleScene(sc)
    oo.x = traj[-1][0]
    oo.v = traj[-1][1]
    oo.begin_step(pose)
    c_o = oo.candidates(x)
    c_g = g.candidates(x)
    assert c_g.shape == c_o.shape and np.array_equal(c_g, c_o)
    d, _ = oo.candidate_distances(x, c_o)
    act = c_o[d < sc.dhat]
    nb = gel_ball_pairs(oo, sc, act)
    say(f"  active pairs {len(act)}, gel-ball {nb}")
    assert nb > 0
    gg, go = g.gradient(x), oo.gradient(x)
    assert_rows_close(gg, go, oo.n_gel, 1e-11)
    rng = np.random.default_rng(1)
    v = rng.normal(size=x.shape)
    yg, yo = g.hess_apply(x, v), oo.hess_apply(x, v)
    assert_rows_close(yg, yo, oo.n_gel, 1e-11)


def test_soft_ball_teacher_forced_iterates(ipc, ball_run):
    sc, traj, _ = ball_run
    L = sc.bbox_diag
    g = ipc.GelScene(sc)
    checked = 0
    for step, (x0, v0, pose, xs) in enumerate(traj):
        g.x = x0
        g.v = v0
        g.begin_step(pose)
        for k in range(min(len(xs) - 1, 3)):
            rc, xg, st = g.newton_iterate(xs[k])
            assert rc == 0
            err = np.abs(xg - xs[k + 1]).max() / L
            checked += 1
            assert err <= 1e-9, (step, k, err)
    assert checked >= 12


def test_soft_ball_free_running(ipc, ball_run):
    sc, traj, o = ball_run
    L = sc.bbox_diag
    g = ipc.GelScene(sc)
    oc = O.OracleScene(sc)
    T = sc.T
    for step in range(1, sc.n_steps + 1):
        rc, st = g.step()
        say(f"  step {step}: rc={rc} newton={st.newton_iters} (oracle {len(traj[step - 1][3]) - 1}) active={st.n_active}")
        assert rc in (0, 1, 4)
        x = g.x
        P = x[T]
        J = np.linalg.det(np.stack([P[:, 1] - P[:, 0], P[:, 2] - P[:, 0], P[:, 3] - P[:, 0]], 2))
        assert J.min() > 0
        c = oc.candidates(x)
        assert oc.candidate_distances(x, c)[0].min() > 0
    err = np.abs(g.x - o.x).max() / L
    say("  free-running final error / L", err)
    assert err <= 1e-4
