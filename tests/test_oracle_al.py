"""The oracle's augmented-Lagrangian indenter targets (the IPC treatment of
prescribed boundary motion, a variant of the target penalty): with a soft
target stiffness the penalty alone leaves the indenter lagging its targets
by about its contact force over k_t, while the multiplier updates bring the
lag under the tolerance within a few updates; at the converged state the
targets' pull k_t (y - yhat) - lambda balances the contact force on the
indenter, and the gradient equals finite differences of the energy with the
multipliers in place."""
import dataclasses

import numpy as np

import oracle as O
from paper_2411_04776_amd import scenes as S

KT = 1e5      # N/m: soft enough for the penalty alone to lag by micrometres
TOL = 1e-9    # m


def soft_scene():
    return dataclasses.replace(S.tiny_scene(steps=3), k_target=KT)


def test_multipliers_remove_the_lag():
    sc = soft_scene()
    pen = O.OracleScene(sc)
    al = O.OracleScene(sc, target_al=1, target_al_tol=TOL)
    for k in range(1, sc.n_steps + 1):
        rp, sp = pen.step(sc.poses[k])
        ra, sa = al.step(sc.poses[k])
        assert sp.max_target_lag > 1000 * TOL          # the penalty alone lags
        assert sa.max_target_lag <= TOL, sa.max_target_lag
        assert 1 <= sa.al_updates <= 8 and ra == 0
        assert sp.al_updates == 0


def test_converged_state_balances_the_contact_force():
    sc = soft_scene()
    o = O.OracleScene(sc, target_al=1, target_al_tol=TOL, newton_tol=1e-10)
    for k in range(1, sc.n_steps + 1):
        o.step(sc.poses[k])
    t = o.gradient_terms(o.x)
    ng = o.n_gel
    f_target = t["target"][ng:].sum(0)    # k_t (y - yhat) - lambda, summed over the indenter
    f_contact = t["contact"][ng:].sum(0)
    scale = np.abs(f_contact).max()
    assert scale > 1e-3                      # the indenter is pressing
    assert np.abs(f_target + f_contact).max() <= 1e-6 * scale
    # the pull is carried by the multipliers, not by a lag: k_t |y - yhat| is tiny
    lag = np.linalg.norm(o.x[ng:] - S.apply_pose(sc.poses[sc.n_steps], sc.Y), axis=1).max()
    assert KT * lag <= 1e-3 * scale


def test_gradient_matches_energy_differences_with_multipliers():
    sc = soft_scene()
    o = O.OracleScene(sc, target_al=1, target_al_tol=TOL)
    r, st = o.step(sc.poses[1])
    assert st.al_updates >= 1
    rng = np.random.default_rng(3)
    x = o.x + rng.normal(0, 2e-6, o.x.shape)   # multipliers of the step stay in place
    g = o.gradient(x)
    free = np.nonzero(~np.asarray(sc.fixed, bool))[0]
    for i in list(range(o.n_gel, o.n_gel + 6)) + list(rng.choice(free, 4, replace=False)):
        for c in range(3):
            h = 1e-9
            xp, xm = x.copy(), x.copy()
            xp[i, c] += h
            xm[i, c] -= h
            fd = (o.energy(xp) - o.energy(xm)) / (2 * h)
            assert abs(fd - g[i, c]) <= 1e-5 * max(abs(g[i, c]), 1e-2), (i, c, fd, g[i, c])
