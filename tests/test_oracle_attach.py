"""The oracle's attachment (gel vertices held by the sensor case): with
negligible inertia and no contact the gel follows a rigid case motion
exactly (translation and rotation: the elastic energy vanishes on rigid
motions, so the minimiser puts every attached vertex on its target); the
gradient equals finite differences of the energy with attachments active;
reset restores the identity case pose."""
import math

import numpy as np

import oracle as O
from paper_2411_04776_amd import scenes as S


def far_attached_scene(rho=1e-9):
    sc = S.attached_scene(grid=(5, 4, 3), steps=1)
    sc.rho = rho
    sc.Y = sc.Y + np.array([0.0, 0.0, 0.05])  # the sphere far above: no contact
    sc.newton_tol = 1e-12
    return sc


def test_rigid_case_motion_is_followed():
    for Rc, t in ((np.eye(3), np.array([1e-4, -2e-4, 3e-4])),
                  (S.rotation((0.3, -0.2, 1.0), math.radians(4.0)), np.array([2e-4, 1e-4, -1e-4]))):
        sc = far_attached_scene()
        o = O.OracleScene(sc)
        P = S.pose_matrix(Rc, t)
        r, st = o.step(sc.poses[1], case_pose=P)
        assert r == 0
        ref = sc.X @ Rc.T + t
        err = np.abs(o.x[:o.n_gel] - ref).max()
        assert err <= 1e-10, err


def test_gradient_matches_energy_differences():
    sc = S.attached_scene(grid=(4, 4, 3), steps=2)
    o = O.OracleScene(sc)
    o.begin_step(sc.poses[1], case_pose=S.pose_matrix(S.rotation((1, 0, 0), 0.02), np.array([0, 1e-4, 2e-4])))
    rng = np.random.default_rng(0)
    x = o.x + rng.normal(0, 3e-5, o.x.shape)
    x[o.n_gel:] = o.x[o.n_gel:]
    g = o.gradient(x)
    for _ in range(6):
        i, c = int(rng.integers(0, o.n_gel)), int(rng.integers(0, 3))
        h = 1e-7
        xp, xm = x.copy(), x.copy()
        xp[i, c] += h
        xm[i, c] -= h
        fd = (o.energy(xp) - o.energy(xm)) / (2 * h)
        assert abs(fd - g[i, c]) <= 1e-4 * max(abs(g[i, c]), 1e-3), (i, c, fd, g[i, c])
    # an attached vertex feels the case pull: its gradient changes with the case pose
    at = np.where(sc.attached)[0][0]
    o2 = O.OracleScene(sc)
    o2.begin_step(sc.poses[1])
    assert np.abs(o2.gradient(x)[at] - g[at]).max() > 1.0


def test_reset_restores_identity_case():
    sc = far_attached_scene(rho=1000.0)
    o = O.OracleScene(sc)
    o.step(sc.poses[1], case_pose=S.pose_matrix(np.eye(3), np.array([0, 0, 2e-4])))
    moved = o.x.copy()
    o.reset()
    o2 = O.OracleScene(sc)
    r1, _ = o.step(sc.poses[1])
    r2, _ = o2.step(sc.poses[1])
    assert np.array_equal(o.x, o2.x)
    assert not np.array_equal(o.x, moved)
