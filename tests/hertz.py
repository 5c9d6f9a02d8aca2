"""Hertz contact check: measurement helpers shared by the oracle pin
(test_oracle_hertz.py) and the GPU check (test_gpu_hertz.py).

Closed form (Hertz, rigid sphere of radius R on an elastic half-space):
F = 4/3 E* sqrt(R) delta^(3/2), E* = E / (1 - nu^2), contact radius
a = sqrt(R delta). delta is the approach of the sphere into the body: for a
rigid indenter, the downward displacement of the body's surface point on the
contact axis. Here it is read off the top vertex under the sphere's centre
(the grid has one there), which folds the barrier's contact gap in: the
sphere stops d short of the surface, and the surface moves by the sphere's
descent past first touch plus that gap.

F is the total normal force the contact transmits: the z-sum over gel
vertices of the barrier gradient (the barrier pushes the gel down with minus
that gradient). At equilibrium it equals the support reaction at the fixed
bottom (the z-sum over fixed vertices of the elastic gradient) and the pull
of the soft targets on the indenter; both are reported.
"""
import numpy as np


def e_star(E, nu):
    return E / (1.0 - nu * nu)


def hertz_force(delta, R, E, nu):
    return 4.0 / 3.0 * e_star(E, nu) * np.sqrt(R) * np.asarray(delta) ** 1.5


def center_vertex(sc):
    """Id of the top gel vertex under the sphere's centre."""
    X = sc.X
    top = X[:, 2] >= X[:, 2].max() - 1e-12
    cx, cy = sc.meta["center"]
    d = np.where(top, (X[:, 0] - cx) ** 2 + (X[:, 1] - cy) ** 2, np.inf)
    i = int(np.argmin(d))
    assert d[i] < 1e-16, "grid has no vertex under the centre"
    return i


def measure(sc, oracle_scene, x, pose):
    """Contact force, its two equilibrium counterparts, the surface
    depression on the axis and the descent past first touch, at state x for
    the step toward `pose` (the oracle scene's step context is set to it)."""
    o = oracle_scene
    o.begin_step(pose)
    g = o.gradient_terms(x)
    n_gel = len(sc.X)
    F_contact = float(g["contact"][:n_gel, 2].sum())
    F_support = float(g["elastic"][:n_gel][sc.fixed.astype(bool), 2].sum())
    F_target = float(g["target"][n_gel:, 2].sum())   # k_t (y - yhat): the indenter held up against its target
    ic = center_vertex(sc)
    delta = float(sc.X[ic, 2] - x[ic, 2])
    z_low0 = (sc.Y @ sc.poses[0][:, :3].T + sc.poses[0][:, 3])[:, 2].min()
    z_low = x[n_gel:, 2].min()
    descent = float(z_low0 - z_low - sc.meta["gap0"])
    return {"F": F_contact, "F_support": F_support, "F_target": F_target, "delta": delta,
            "descent": descent}


def fit(deltas, forces, R, E, nu):
    """Least-squares exponent of log F against log delta, and the prefactor
    ratio: the geometric mean of F / F_hertz(delta) (the fitted prefactor
    with the exponent held at 3/2, over Hertz's)."""
    ld, lf = np.log(np.asarray(deltas)), np.log(np.asarray(forces))
    expo = float(np.polyfit(ld, lf, 1)[0])
    ratio = float(np.exp(np.mean(lf - np.log(hertz_force(deltas, R, E, nu)))))
    return expo, ratio


def layer_correction(delta, R, h, nu):
    """Factor on Hertz's force for a sphere pressing an elastic layer of
    thickness h bonded to a rigid base (series in chi = sqrt(R delta) / h,
    Dimitriadis et al., Biophys. J. 82, 2002, bonded case): the fixed bottom
    of a block of finite thickness stiffens the response by up to ~27% at
    chi = 0.21 (R = 20 mm, delta = 0.5 mm, h = 15 mm, nu = 0.45)."""
    chi = np.sqrt(R * np.asarray(delta)) / h
    a0 = -(1.2876 - 1.4678 * nu + 1.3442 * nu * nu) / (1.0 - nu)
    b0 = (0.6387 - 1.0277 * nu + 1.5164 * nu * nu) / (1.0 - nu)
    pi = np.pi
    return (1.0 - 2.0 * a0 / pi * chi + 4.0 * a0 * a0 / pi ** 2 * chi ** 2
            - 8.0 / pi ** 3 * (a0 ** 3 + 4.0 * pi ** 2 / 15.0 * b0) * chi ** 3
            + 16.0 * a0 / pi ** 4 * (a0 ** 3 + 3.0 * pi ** 2 / 5.0 * b0) * chi ** 4)


def fit_layer(deltas, forces, R, h, E, nu):
    """Prefactor ratio against the layer-corrected closed form (geometric
    mean of F / (F_hertz * layer_correction))."""
    d = np.asarray(deltas)
    ref = hertz_force(d, R, E, nu) * layer_correction(d, R, h, nu)
    return float(np.exp(np.mean(np.log(np.asarray(forces)) - np.log(ref))))
