"""Pins of the oracle's lagged IPC friction (closed forms, finite differences,
invariants). The friction potential follows IPC's frictional contact: per pair
active at the step start, D = mu * lambda * f0(|u|) with u the tangential
relative displacement of the frozen closest points and f0 the C1 smoothing of
|u| over the length eps_v * h."""
import numpy as np
import pytest

import oracle as O
from paper_2411_04776_amd import scenes as S


def test_smoothing_closed_form_and_continuity():
    e = 1e-5
    for y in np.linspace(0.0, e, 11)[:-1]:
        f = O.friction_f(y, e)
        # f0(y) - y = (e - y)^3 / (3 e^2) on [0, e): the smoothing sits above |u| and touches it at e
        assert np.isclose(f[0] - y, (e - y) ** 3 / (3 * e * e), rtol=1e-12, atol=1e-22)
        assert 0.0 <= f[1] <= 1.0 and f[2] >= 0.0
    lo, hi = O.friction_f(e * (1 - 1e-12), e), O.friction_f(e, e)
    assert np.isclose(lo[0], hi[0], rtol=1e-9) and np.isclose(lo[1], hi[1], rtol=1e-9)
    f0 = O.friction_f(0.0, e)
    assert np.isclose(f0[0], e / 3) and f0[1] == 0.0 and np.isclose(f0[2], 2 / e)
    assert np.array_equal(O.friction_f(3 * e, e), [3 * e, 1.0, 0.0])


def _pair(rng, scale):
    xt = rng.normal(size=12) * 1e-3
    c4 = np.array([1.0, -0.2, -0.5, -0.3])  # PT interior: c = (1, -(1-b1-b2), -b1, -b2)
    n = rng.normal(size=3)
    n /= np.linalg.norm(n)
    x = xt + rng.normal(size=12) * scale
    return x, xt, c4, n


@pytest.mark.parametrize("scale", [2e-6, 3e-5])
def test_gradient_and_hessian_by_finite_differences(scale):
    rng = np.random.default_rng(11)
    e, ml = 1e-5, 0.7
    for _ in range(4):
        x, xt, c4, n = _pair(rng, scale)
        D, g, H = O.pair_friction(x, xt, c4, n, ml, e)
        h = 1e-9
        gfd = np.array([(O.pair_friction(x + h * np.eye(12)[k], xt, c4, n, ml, e)[0] -
                         O.pair_friction(x - h * np.eye(12)[k], xt, c4, n, ml, e)[0]) / (2 * h) for k in range(12)])
        assert np.allclose(g, gfd, rtol=1e-5, atol=1e-7 * np.abs(g).max())
        Hfd = np.array([(O.pair_friction(x + h * np.eye(12)[k], xt, c4, n, ml, e)[1] -
                         O.pair_friction(x - h * np.eye(12)[k], xt, c4, n, ml, e)[1]) / (2 * h) for k in range(12)])
        # the analytic Hessian is the PSD-clamped one; here f0'' >= 0, so it is exact
        assert np.allclose(H, Hfd, rtol=1e-4, atol=1e-5 * np.abs(H).max())
        assert np.allclose(H, H.T, atol=1e-12 * np.abs(H).max())
        assert np.linalg.eigvalsh(H).min() >= -1e-9 * np.abs(H).max()


def test_normal_motion_gives_no_force_and_sliding_gives_coulomb():
    rng = np.random.default_rng(5)
    e, mu, lam = 1e-5, 0.5, 2.0
    x, xt, c4, n = _pair(rng, 0.0)
    # move every vertex along the normal only: u = 0, no tangential force
    xn = xt + (rng.normal(size=4)[:, None] * 1e-4 * n[None, :]).ravel()
    D, g, _ = O.pair_friction(xn, xt, c4, n, mu * lam, e)
    assert np.abs(g).max() <= 1e-12 * mu * lam and np.isclose(D, mu * lam * e / 3)
    # full sliding (|u| >> e): force on slot k is mu * lambda * |c_k| along -+u (Coulomb)
    t = np.cross(n, [1.0, 0.0, 0.0])
    t /= np.linalg.norm(t)
    xs = xt.copy()
    xs[:3] += 50 * e * t
    D, g, _ = O.pair_friction(xs, xt, c4, n, mu * lam, e)
    for k in range(4):
        gk = g[3 * k:3 * k + 3]
        assert np.isclose(np.linalg.norm(gk), mu * lam * abs(c4[k]), rtol=1e-12)
        assert np.isclose(abs(gk @ t), np.linalg.norm(gk), rtol=1e-12)
    assert np.isclose(D, mu * lam * 50 * e, rtol=1e-12)


def test_scene_lag_set_and_drag():
    """Sliding contact: the lagged set holds the pairs active at x^t with
    positive normal force, and friction drags the gel top along the slide."""
    fr = S.tiny_slide_scene(mu=0.5)
    nf = S.tiny_slide_scene(mu=0.0)
    o1, o0 = O.OracleScene(fr), O.OracleScene(nf)
    for k in range(1, fr.n_steps + 1):
        x_before = o1.x
        o1.begin_step(fr.poses[k])
        v4, c4, nrm, lam = o1.friction_set()
        cand = o1.candidates(x_before)
        d, _ = o1.candidate_distances(x_before, cand)
        assert len(lam) == int((d < fr.dhat).sum())
        assert (lam > 0).all() and np.allclose(np.linalg.norm(nrm, axis=1), 1.0)
        o1.step(fr.poses[k])
        o0.step(nf.poses[k])
    top = np.where(np.isclose(fr.X[:, 2], fr.X[:, 2].max()))[0]
    dx1 = (o1.x[top, 0] - fr.X[top, 0]).mean()
    dx0 = (o0.x[top, 0] - nf.X[top, 0]).mean()
    assert dx1 > dx0 + 1e-7, (dx1, dx0)
