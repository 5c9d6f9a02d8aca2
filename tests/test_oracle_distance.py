"""Oracle distances, barrier and mollifier against closed forms, brute-force
minimisation and finite differences."""
import math

import numpy as np
import pytest
from scipy.optimize import minimize

import oracle as O

DHAT = 1e-4
KAPPA = 1e4
MM = 1e-3


def pt_brute(x12):
    """Distance point-triangle by constrained minimisation over barycentrics."""
    p, a, b, c = x12.reshape(4, 3)
    best = (np.inf, None)
    for u in np.linspace(0, 1, 41):
        for v in np.linspace(0, 1 - u, max(2, int(41 * (1 - u)))):
            q = a + u * (b - a) + v * (c - a)
            dd = np.sum((p - q) ** 2)
            if dd < best[0]:
                best = (dd, (u, v))
    f = lambda z: np.sum((p - (a + z[0] * (b - a) + z[1] * (c - a))) ** 2) / MM ** 2
    cons = [{"type": "ineq", "fun": lambda z: 1 - z[0] - z[1]}]
    r = minimize(f, best[1], method="SLSQP", bounds=[(0, 1), (0, 1)], constraints=cons,
                 options={"ftol": 1e-20, "maxiter": 500})
    return math.sqrt(min(r.fun, best[0] / MM ** 2)) * MM


def ee_brute(x12):
    a0, a1, b0, b1 = x12.reshape(4, 3)
    f = lambda z: np.sum((a0 + z[0] * (a1 - a0) - b0 - z[1] * (b1 - b0)) ** 2) / MM ** 2
    best = min(((f((s, t)), (s, t)) for s in np.linspace(0, 1, 41) for t in np.linspace(0, 1, 41)))
    r = minimize(f, best[1], method="L-BFGS-B", bounds=[(0, 1), (0, 1)],
                 options={"ftol": 1e-22, "gtol": 1e-16, "maxiter": 1000})
    return math.sqrt(min(r.fun, best[0])) * MM


def test_pt_closed_forms():
    tri = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], dtype=float) * MM
    # above the interior: distance = height, face type
    d, t = O.pt_distance(np.concatenate([[0.2 * MM, 0.3 * MM, 0.05 * MM], tri.ravel()]))
    assert t == 6 and abs(d - 0.05 * MM) <= 1e-18
    # beyond vertex t0: Euclidean distance to it
    p = np.array([-0.3, -0.4, 0.0]) * MM
    d, t = O.pt_distance(np.concatenate([p, tri.ravel()]))
    assert t == 0 and abs(d - 0.5 * MM) <= 1e-18
    # beside edge t0t1 (y < 0, 0 < x < 1): distance to the edge line
    p = np.array([0.5, -0.3, 0.4]) * MM
    d, t = O.pt_distance(np.concatenate([p, tri.ravel()]))
    assert t == 3 and abs(d - 0.5 * MM) <= 1e-18
    # beside the hypotenuse t1t2
    p = np.array([1.0, 1.0, 0.0]) * MM
    d, t = O.pt_distance(np.concatenate([p, tri.ravel()]))
    assert t == 4 and abs(d - math.sqrt(0.5) * MM) <= 1e-17
    # tie on the boundary of a vertex region goes to the vertex
    p = np.array([0.0, 0.0, 0.3]) * MM
    _, t = O.pt_distance(np.concatenate([p, tri.ravel()]))
    assert t == 0


def test_ee_closed_forms():
    # skew perpendicular segments crossing in projection: separation
    x = np.array([[-1, 0, 0], [1, 0, 0], [0, -1, 0.3], [0, 1, 0.3]], dtype=float) * MM
    d, t = O.ee_distance(x.ravel())
    assert t == 8 and abs(d - 0.3 * MM) <= 1e-18
    # parallel overlapping edges: separation, reduced to a point-edge type
    x = np.array([[0, 0, 0], [2, 0, 0], [1, 0, 0.2], [3, 0, 0.2]], dtype=float) * MM
    d, t = O.ee_distance(x.ravel())
    assert t in (4, 5, 6, 7) and abs(d - 0.2 * MM) <= 1e-18
    # collinear disjoint: endpoint to endpoint
    x = np.array([[0, 0, 0], [1, 0, 0], [1.5, 0, 0], [3, 0, 0]], dtype=float) * MM
    d, t = O.ee_distance(x.ravel())
    assert t == 2 and abs(d - 0.5 * MM) <= 1e-18
    # endpoint of B against the interior of A
    x = np.array([[0, 0, 0], [2, 0, 0], [1, 0.5, 0.3], [1, 2, 0.3]], dtype=float) * MM
    d, t = O.ee_distance(x.ravel())
    assert t == 6 and abs(d - math.hypot(0.5, 0.3) * MM) <= 1e-17


def test_distances_match_brute_force():
    rng = np.random.default_rng(10)
    for _ in range(60):
        x = rng.uniform(-1, 1, 12) * MM
        d, _ = O.pt_distance(x)
        assert abs(d - pt_brute(x)) <= 1e-9 * MM
        d, _ = O.ee_distance(x)
        assert abs(d - ee_brute(x)) <= 1e-9 * MM


def _fd_check(kind, x, tol=1e-6):
    d, g, H = O.distance_derivs(kind, x)
    dist = O.pt_distance if kind == 0 else O.ee_distance
    t0 = dist(x)[1]
    h = 1e-7 * MM
    gfd = np.zeros(12)
    Hfd = np.zeros((12, 12))
    for k in range(12):
        e = np.zeros(12)
        e[k] = h
        assert dist(x + e)[1] == t0 and dist(x - e)[1] == t0
        gfd[k] = (dist(x + e)[0] - dist(x - e)[0]) / (2 * h)
        Hfd[:, k] = (O.distance_derivs(kind, x + e)[1] - O.distance_derivs(kind, x - e)[1]) / (2 * h)
    assert np.abs(g - gfd).max() <= tol * np.abs(g).max()
    assert np.abs(H - Hfd).max() <= tol * np.abs(H).max()
    assert np.abs(H - H.T).max() <= 1e-10 * np.abs(H).max()
    return t0


def test_distance_derivatives_every_type():
    rng = np.random.default_rng(11)
    seen_pt, seen_ee = set(), set()
    tries = 0
    while (len(seen_pt) < 7 or len(seen_ee) < 9) and tries < 20000:
        tries += 1
        x = rng.uniform(-1, 1, 12) * MM
        if rng.random() < 0.3:  # push toward degenerate-feature types
            x[9:12] = x[6:9] + rng.uniform(-0.3, 0.3, 3) * MM
        _, tp = O.pt_distance(x)
        _, te = O.ee_distance(x)
        # stay clear of region boundaries so FD does not cross them
        ok = lambda fn, t: all(fn(x + e)[1] == t for e in rng.uniform(-1e-5, 1e-5, (6, 12)) * MM)
        if tp not in seen_pt and ok(O.pt_distance, tp):
            _fd_check(0, x)
            seen_pt.add(tp)
        if te not in seen_ee and ok(O.ee_distance, te):
            _fd_check(1, x)
            seen_ee.add(te)
    assert seen_pt == set(range(7))
    assert seen_ee == set(range(9))


def test_barrier_closed_forms():
    assert np.array_equal(O.barrier_scalar(DHAT, DHAT), [0, 0, 0])
    assert np.array_equal(O.barrier_scalar(2 * DHAT, DHAT), [0, 0, 0])
    b = O.barrier_scalar(DHAT / 2, DHAT)
    assert abs(b[0] - 0.25 * math.log(2) * DHAT ** 2) <= 1e-15 * DHAT ** 2
    assert abs(b[1] + (math.log(2) + 0.5) * DHAT) <= 1e-15 * DHAT
    assert abs(b[2] - (5 + 2 * math.log(2))) <= 1e-13
    assert abs(b[2] - 6.386294361119891) <= 1e-12
    # derivatives by finite differences on (0, dhat)
    for d in np.linspace(0.05, 0.95, 10) * DHAT:
        h = 1e-6 * DHAT
        bp, bm = O.barrier_scalar(d + h, DHAT), O.barrier_scalar(d - h, DHAT)
        b = O.barrier_scalar(d, DHAT)
        assert abs((bp[0] - bm[0]) / (2 * h) - b[1]) <= 1e-6 * abs(b[1])
        assert abs((bp[1] - bm[1]) / (2 * h) - b[2]) <= 1e-6 * abs(b[2])
    assert np.isinf(O.barrier_scalar(0.0, DHAT)[0])


def _pair_fd(kind, x, eps_x):
    E, g, H = O.pair_barrier(kind, x, DHAT, KAPPA, eps_x, project=False)
    h = 1e-7 * MM
    gfd = np.zeros(12)
    Hfd = np.zeros((12, 12))
    for k in range(12):
        e = np.zeros(12)
        e[k] = h
        Ep, gp, _ = O.pair_barrier(kind, x + e, DHAT, KAPPA, eps_x, project=False)
        Em, gm, _ = O.pair_barrier(kind, x - e, DHAT, KAPPA, eps_x, project=False)
        gfd[k] = (Ep - Em) / (2 * h)
        Hfd[:, k] = (gp - gm) / (2 * h)
    assert np.abs(g - gfd).max() <= 1e-6 * np.abs(g).max()
    assert np.abs(H - Hfd).max() <= 1e-5 * np.abs(H).max()
    _, _, Hp = O.pair_barrier(kind, x, DHAT, KAPPA, eps_x, project=True)
    w, V = np.linalg.eigh(H)
    assert np.abs(Hp - (V * np.maximum(w, 0)) @ V.T).max() <= 1e-10 * np.abs(H).max()
    return E


def test_pair_barrier_fd_pt_and_ee():
    tri = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], dtype=float) * MM
    x = np.concatenate([[0.25 * MM, 0.3 * MM, 0.4 * DHAT], tri.ravel()])
    E = _pair_fd(0, x, 0.0)
    b = O.barrier_scalar(0.4 * DHAT, DHAT)[0]
    assert abs(E - KAPPA * b) <= 1e-12 * KAPPA * b
    # skew edges, mollifier inactive
    x = np.array([[-1, 0, 0], [1, 0, 0], [0, -1, 0], [0.3, 1, 0]], dtype=float) * MM
    x[2:, 2] = 0.5 * DHAT
    a, bb = x[1] - x[0], x[3] - x[2]
    eps_x = 1e-3 * np.dot(a, a) * np.dot(bb, bb)
    assert np.sum(np.cross(a, bb) ** 2) > eps_x
    E = _pair_fd(1, x.ravel(), eps_x)
    assert abs(E - KAPPA * O.barrier_scalar(0.5 * DHAT, DHAT)[0]) <= 1e-9 * E
    # nearly parallel edges, mollifier active (c < eps_x)
    x = np.array([[-1, 0, 0], [1, 0, 0], [-0.5, 0.002, 0.3 * DHAT / MM], [0.5, -0.002, 0.3 * DHAT / MM]]) * MM
    a, bb = x[1] - x[0], x[3] - x[2]
    eps_x = 1e-3 * np.dot(a, a) * np.dot(bb, bb)
    assert np.sum(np.cross(a, bb) ** 2) < eps_x
    _pair_fd(1, x.ravel(), eps_x)


def test_mollifier_continuity():
    """w*b is continuous where c crosses eps_x (m(eps_x) = 1)."""
    x = np.array([[-1, 0, 0], [1, 0, 0], [-0.5, 0, 0.5 * DHAT / MM], [0.5, 0, 0.5 * DHAT / MM]]) * MM
    a = x[1] - x[0]
    # rotate edge B about z to sweep c = |a x b|^2 through eps_x
    eps_x = 1e-3 * 4 * MM ** 2 * 1 * MM ** 2
    Es = []
    for ang in np.linspace(0.0, 0.08, 400):
        y = x.copy()
        y[2] = [-0.5 * math.cos(ang) * MM, -0.5 * math.sin(ang) * MM, x[2, 2]]
        y[3] = [0.5 * math.cos(ang) * MM, 0.5 * math.sin(ang) * MM, x[3, 2]]
        Es.append(O.pair_barrier(1, y.ravel(), DHAT, KAPPA, eps_x)[0])
    Es = np.array(Es)
    assert Es[0] == 0.0  # parallel: mollified to zero
    assert np.abs(np.diff(Es)).max() <= 0.02 * Es.max()
