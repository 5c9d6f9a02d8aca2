"""Oracle assembly, PCG and Newton against finite differences, a dense direct
solve, scipy's L-BFGS-B, and the invariants the IPC model guarantees
(no inversion, no interpenetration, monotone energy)."""
import numpy as np
import pytest
from scipy.optimize import minimize

import oracle as O
from paper_2411_04776_amd import scenes as S


def pressed_state(o, depth_frac=0.8, seed=0):
    """A feasible state with active contacts: indenter lowered into dhat."""
    sc = o.scene
    x = o.x
    x[o.n_gel:] -= np.array([0, 0, depth_frac * sc.dhat])
    rng = np.random.default_rng(seed)
    x[:o.n_gel] += rng.normal(0, 0.05 * sc.dhat, (o.n_gel, 3)) * (1 - sc.fixed[:, None])
    return x


def test_gradient_is_fd_of_energy_with_contact():
    sc = S.tiny_scene()
    o = O.OracleScene(sc)
    o.begin_step(sc.poses[1])
    x = pressed_state(o)
    c = o.candidates(x)
    d, _ = o.candidate_distances(x, c)
    assert (d < sc.dhat).sum() >= 3
    g = o.gradient(x)
    h = 1e-9
    rng = np.random.default_rng(1)
    free = np.nonzero(np.concatenate([1 - sc.fixed, np.ones(o.n_ind)]))[0]
    # DOFs of vertices in active pairs plus a random sample
    _, e, t = o.surface()
    verts = set()
    for row, dd in zip(c, d):
        if dd < sc.dhat:
            verts |= set(([row[1]] + list(t[row[2]])) if row[0] == 0 else list(e[row[1]]) + list(e[row[2]]))
    verts = sorted(v for v in verts if v in set(free))
    verts += list(rng.choice(free, 6, replace=False))
    gscale = np.abs(g).max()
    for v in verts:
        for k in range(3):
            xp, xm = x.copy(), x.copy()
            xp[v, k] += h
            xm[v, k] -= h
            fd = (o.energy(xp) - o.energy(xm)) / (2 * h)
            assert abs(fd - g[v, k]) <= 1e-6 * gscale + 1e-5 * abs(g[v, k]), (v, k, fd, g[v, k])
    assert np.abs(g[:o.n_gel][sc.fixed.astype(bool)]).max() == 0.0


def test_hessian_symmetric_psd_and_pcg_matches_direct_solve():
    sc = S.tiny_scene()
    o = O.OracleScene(sc, pcg_tol=1e-14)
    o.begin_step(sc.poses[1])
    x = pressed_state(o)
    H = o.hess_dense(x)
    assert H.shape[0] <= 3000
    assert np.abs(H - H.T).max() <= 1e-12 * np.abs(H).max()
    assert np.linalg.eigvalsh(H).min() > 0
    g = o.gradient(x).ravel()
    p_direct = np.linalg.solve(H, -g)
    p, its = o.pcg(x)
    assert its > 0
    assert np.linalg.norm(p.ravel() - p_direct) <= 1e-10 * np.linalg.norm(p_direct)
    # hess_apply agrees with the dense matrix
    v = np.random.default_rng(2).normal(size=H.shape[0])
    assert np.abs(o.hess_apply(x, v.reshape(-1, 3)).ravel() - H @ v).max() <= 1e-12 * np.abs(H @ v).max()


def test_rest_state_is_stationary_bit_exactly():
    sc = S.config1()
    o = O.OracleScene(sc)
    x0 = o.x
    for _ in range(2):
        r, st = o.step(sc.poses[0])  # target = current pose, no load
        assert r == 0 and st.newton_iters == 1
    assert np.array_equal(o.x, x0)
    assert np.array_equal(o.v, np.zeros_like(x0))


def test_newton_matches_lbfgsb_without_contact():
    sc = S.tiny_scene()
    sc.gravity = (0.0, 0.0, -800.0)
    sc.poses = sc.poses.copy()
    sc.poses[:, 2, 3] += 5e-3  # indenter far above the gel: no contact
    sc.poses[1] = sc.poses[0]  # and at rest on its target: only the gel moves
    sc.newton_tol = 1e-13  # converge fully: the comparison is with the minimiser itself
    o = O.OracleScene(sc, pcg_tol=1e-14)
    x0 = o.x
    r, st = o.step()
    assert r == 0
    x_newton = o.x
    L = sc.bbox_diag
    # same problem with L-BFGS-B from the same start
    o2 = O.OracleScene(sc)
    o2.begin_step(sc.poses[1])
    free = np.concatenate([1 - sc.fixed, np.ones(o2.n_ind, dtype=np.uint8)]).astype(bool)
    Phi0 = o2.energy(x0)
    delta = 1e-5  # displacement unit of the search variable (metres)
    scale = np.abs(o2.gradient(x0)).max() * delta

    def f(z):
        x = x0.copy()
        x[free] += z.reshape(-1, 3) * delta
        return (o2.energy(x) - Phi0) / scale, (o2.gradient(x)[free].ravel() * delta / scale)

    res = minimize(f, np.zeros(3 * free.sum()), jac=True, method="L-BFGS-B",
                   options={"maxiter": 20000, "maxcor": 50, "ftol": 1e-30, "gtol": 1e-14})
    x_lb = x0.copy()
    x_lb[free] += res.x.reshape(-1, 3) * delta
    sag = np.abs(x_newton - x0).max()
    assert sag > 1e-4 * L  # gravity produced a visible deformation
    assert np.abs(x_newton - x_lb).max() <= 1e-7 * L


def test_trajectory_invariants():
    """Each accepted Newton iterate lowers the energy, keeps every tet
    positively oriented and every candidate pair at positive distance."""
    sc = S.tiny_scene(depth=0.6e-3, steps=4)
    o = O.OracleScene(sc)
    T = sc.T
    for step in range(1, 5):
        o.begin_step(sc.poses[step])
        x = o.x
        E_prev = o.energy(x)
        for k in range(100):
            r, xn, st = o.newton_iterate(x)
            if r == 1:
                break
            E = o.energy(xn)
            assert E <= E_prev
            E_prev = E
            P = xn[T]
            J = np.linalg.det(np.stack([P[:, 1] - P[:, 0], P[:, 2] - P[:, 0], P[:, 3] - P[:, 0]], 2))
            assert J.min() > 0
            c = o.candidates(xn)
            if len(c):
                assert o.candidate_distances(xn, c)[0].min() > 0
            x = xn
        o.x = x
    # the indenter went below the undeformed top: the gel must be pushed down
    assert o.x[:o.n_gel, 2].min() < sc.X[:, 2].max() - 0.2e-3


def test_step_reports_and_velocity():
    sc = S.tiny_scene()
    o = O.OracleScene(sc)
    x0 = o.x
    r, st = o.step()
    assert r in (0, 4)
    v = o.v
    assert np.allclose(v, (o.x - x0) / sc.dt, rtol=0, atol=1e-15)
    assert st.newton_iters >= 1 and st.pcg_iters >= 1
    o.reset()
    assert np.array_equal(o.x, x0) and not o.v.any()
