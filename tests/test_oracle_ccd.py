"""Oracle additive CCD against exact times of impact and dense sampling."""
import math

import numpy as np

import oracle as O

MM = 1e-3
S = 0.1


def test_point_plane_straight_approach():
    tri = np.array([[-1, -1, 0], [2, -1, 0], [-1, 2, 0]], dtype=float) * MM
    for z0, v in ((0.5, 1.0), (0.1, 3.0), (0.01, 0.02), (1.0, 0.5)):
        x = np.concatenate([[0.2 * MM, 0.1 * MM, z0 * MM], tri.ravel()])
        p = np.zeros(12)
        p[2] = -v * MM
        toi = O.accd(0, x, p, S, 1.0)
        exact = z0 / v  # contact time; beyond 1 means no contact in the step
        if exact > 1.0:
            assert toi == 1.0
        else:
            assert toi <= exact
            # the returned time keeps at least the keep-gap s * d0
            gap = z0 * MM - toi * v * MM
            assert gap >= S * z0 * MM * (1 - 1e-12)
            # and is not absurdly conservative: within a few sub-steps of (1-s) d0
            assert toi >= 0.5 * (1 - S) * exact


def test_no_motion_or_separating():
    rng = np.random.default_rng(0)
    x = rng.uniform(-1, 1, 12) * MM
    assert O.accd(0, x, np.zeros(12)) == 1.0
    # pure common translation: zero relative motion
    p = np.tile([0.3 * MM, -0.2 * MM, 5 * MM], 4)
    assert O.accd(1, x, p) == 1.0


def _true_toi(kind, x, p, n=4000):
    """First time the true distance reaches (near) zero by dense sampling and
    bisection; None if it stays positive on [0, 1]."""
    dist = O.pt_distance if kind == 0 else O.ee_distance
    ts = np.linspace(0, 1, n + 1)
    ds = np.array([dist(x + t * p)[0] for t in ts])
    hit = np.nonzero(ds <= 1e-12 * MM)[0]
    # refine a local minimum below a tiny threshold
    k = int(np.argmin(ds))
    return ds, (ts[hit[0]] if len(hit) else None), ts[k]


def test_random_pairs_never_overshoot():
    rng = np.random.default_rng(1)
    checked = 0
    for trial in range(400):
        kind = trial % 2
        x = rng.uniform(-1, 1, 12) * MM
        # aim the first primitive through the second one
        p = rng.normal(0, 0.2, 12) * MM
        target = x[3:6] if kind == 0 else 0.5 * (x[6:9] + x[9:12])
        src = x[0:3] if kind == 0 else 0.5 * (x[0:3] + x[3:6])
        shift = (target - src) * rng.uniform(0.8, 2.0)
        if kind == 0:
            p[0:3] += shift
        else:
            p[0:6] += np.tile(shift, 2)
        toi = O.accd(kind, x, p, S, 1.0)
        dist = O.pt_distance if kind == 0 else O.ee_distance
        d0 = dist(x)[0]
        assert 0.0 <= toi <= 1.0
        # distance stays positive on [0, toi] (dense sampling)
        ts = np.linspace(0.0, toi, 2001)
        dmin = min(dist(x + t * p)[0] for t in ts)
        assert dmin > 0.0
        # keep-gap at the returned time
        if toi < 1.0:
            assert dist(x + toi * p)[0] >= S * d0 * (1 - 1e-9)
            checked += 1
    assert checked > 50


def test_exact_crossing_time_bound():
    """Edge sweeping through another edge: exact crossing time from the
    closed form; ACCD returns an earlier time."""
    a = np.array([[-1, 0, 0.3], [1, 0, 0.3]]) * MM
    b = np.array([[0, -1, 0], [0, 1, 0]]) * MM
    x = np.concatenate([a.ravel(), b.ravel()])
    p = np.zeros(12)
    p[2] = p[5] = -0.6 * MM  # edge A moves down 0.6 mm: crosses at t = 0.5
    toi = O.accd(1, x, p, S, 1.0)
    assert toi <= 0.5
    assert 0.3 * MM - toi * 0.6 * MM >= S * 0.3 * MM * (1 - 1e-12)
