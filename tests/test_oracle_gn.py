"""The oracle's Gauss-Newton pair barrier Hessian (ora_pair_barrier with
project = 2): kappa * w * b''(d) * grad d grad d^T.

Pinned without the oracle's own derivative code: b'' and b' by finite
differences of the barrier value, grad d by central differences of the
distance function, w from the pair energy divided by kappa * b(d), and the
exact-minus-Gauss-Newton difference against the closed-form Hessian of a
point-point distance, (I - u u^T) / d. A Newton run with the Gauss-Newton
Hessian reaches the same minimiser as the projected-Newton run (the gradient
is exact in both).
"""
import numpy as np
import pytest

import oracle as O
from paper_2411_04776_amd import scenes as S

DHAT = 1e-4
KAPPA = 1e4


def fd_b(d, k):
    """k-th derivative of b at d by central differences of the barrier value."""
    h = 1e-3 * d
    b = lambda t: O.barrier_scalar(t, DHAT)[0]
    if k == 1:
        return (b(d + h) - b(d - h)) / (2 * h)
    return (b(d + h) - 2 * b(d) + b(d - h)) / (h * h)


def fd_grad_distance(kind, x12):
    f = (lambda x: O.pt_distance(x)[0]) if kind == 0 else (lambda x: O.ee_distance(x)[0])
    g = np.zeros(12)
    for i in range(12):
        h = 1e-10
        xp, xm = x12.copy(), x12.copy()
        xp[i] += h
        xm[i] -= h
        g[i] = (f(xp) - f(xm)) / (2 * h)
    return g


def pt_config(rng, face=True):
    tri = np.array([[0, 0, 0], [1e-3, 0, 0], [0, 1e-3, 0]]) + rng.normal(0, 5e-6, (3, 3))
    if face:
        p = np.array([2.5e-4, 3e-4, 0]) + np.array([0, 0, rng.uniform(0.2, 0.8) * DHAT])
    else:  # beyond vertex t0: point-point
        p = tri[0] + np.array([-3e-5, -2e-5, rng.uniform(0.1, 0.5) * DHAT])
    return np.concatenate([p, tri.ravel()])


def ee_config(rng, parallel=False):
    a0, a1 = np.array([0, 0, 0.0]), np.array([1e-3, 0, 0])
    if parallel:
        b0 = np.array([2e-4, -5e-7, 0.6 * DHAT])
        b1 = np.array([1.2e-3, 5e-7, 0.6 * DHAT])
    else:
        b0 = np.array([5e-4, -5e-4, rng.uniform(0.2, 0.8) * DHAT])
        b1 = np.array([4e-4, 5e-4, b0[2]])
    return np.concatenate([a0, a1, b0, b1])


@pytest.mark.parametrize("case", ["pt_face", "pt_vertex", "ee_cross", "ee_parallel"])
def test_gn_is_kappa_w_bpp_outer_product(case):
    rng = np.random.default_rng(11)
    kind = 0 if case.startswith("pt") else 1
    x12 = pt_config(rng, case == "pt_face") if kind == 0 else ee_config(rng, case == "ee_parallel")
    d = O.pt_distance(x12)[0] if kind == 0 else O.ee_distance(x12)[0]
    assert 0 < d < DHAT
    eps_x = 1e-3 * (1e-3 ** 2) * (1e-3 ** 2)
    E, g, H = O.pair_barrier(kind, x12, DHAT, KAPPA, eps_x, project=2)
    w = E / (KAPPA * O.barrier_scalar(d, DHAT)[0])
    if case == "ee_parallel":
        assert w < 1.0  # the mollifier is active
    else:
        assert abs(w - 1.0) < 1e-12
    gd = fd_grad_distance(kind, x12)
    ref = KAPPA * w * fd_b(d, 2) * np.outer(gd, gd)
    assert np.abs(H - ref).max() <= 1e-5 * np.abs(ref).max()
    # PSD, rank one
    ev = np.linalg.eigvalsh(0.5 * (H + H.T))
    assert ev[0] >= -1e-12 * ev[-1]
    assert ev[-2] <= 1e-10 * ev[-1]
    # the gradient is the exact one in every mode
    _, g_exact, _ = O.pair_barrier(kind, x12, DHAT, KAPPA, eps_x, project=0)
    assert np.array_equal(g, g_exact)


def test_exact_minus_gn_is_point_point_curvature():
    """Point-point closest features: grad^2 d = (I - u u^T)/d on the point and
    the triangle vertex (signs + - / - +), so exact - GN = kappa b'(d) grad^2 d."""
    rng = np.random.default_rng(3)
    for _ in range(5):
        x12 = pt_config(rng, face=False)
        d, t = O.pt_distance(x12)
        assert t == 0  # vertex t0
        _, _, He = O.pair_barrier(0, x12, DHAT, KAPPA, 1.0, project=0)
        _, _, Hg = O.pair_barrier(0, x12, DHAT, KAPPA, 1.0, project=2)
        u = (x12[0:3] - x12[3:6]) / d
        C = (np.eye(3) - np.outer(u, u)) / d
        ref = np.zeros((12, 12))
        ref[0:3, 0:3], ref[0:3, 3:6], ref[3:6, 0:3], ref[3:6, 3:6] = C, -C, -C, C
        ref *= KAPPA * fd_b(d, 1)
        assert np.abs((He - Hg) - ref).max() <= 1e-5 * np.abs(ref).max()


def test_gn_newton_reaches_the_projected_minimiser():
    sc = S.tiny_scene(steps=3)
    sc.newton_tol = 1e-11
    a = O.OracleScene(sc)
    b = O.OracleScene(sc, barrier_hessian=1)
    L = sc.bbox_diag
    for k in range(1, sc.n_steps + 1):
        ra, sa = a.step(sc.poses[k])
        rb, sb = b.step(sc.poses[k])
        assert ra == 0 and rb == 0
        assert sa.n_active == sb.n_active
        err = np.abs(a.x - b.x).max() / L
        assert err <= 1e-9, (k, err)
