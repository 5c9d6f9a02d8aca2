"""The oracle's height map (oracle/height_map.py) against what the geometry
fixes: zero depth on the undeformed gel, a sheared gel's top plane in closed
form, a single lowered vertex on a pixel centre, and an all-pixels brute force
on a tiny mesh."""
import numpy as np

import oracle as O
from oracle.height_map import height_map
from paper_2411_04776_amd import scenes as S


def gel_surface(nx, ny, nz):
    sc = S.tiny_scene(grid=(nx, ny, nz))
    o = O.OracleScene(sc)
    _, _, tris = o.surface()
    return sc, o, tris[:o.n_gel_tris], o.x[:o.n_gel]


def test_rest_gel_has_zero_depth():
    sc, o, tris, X = gel_surface(6, 5, 3)
    ztop = X[:, 2].max()
    lo, hi = X.min(0), X.max(0)
    dx = (hi[0] - lo[0]) / 37
    m = height_map(X, tris, lo[0] - 3 * dx, lo[1] - 3 * dx, dx, dx, 45, 45, ztop)
    px = lo[0] - 3 * dx + np.arange(45) * dx
    py = lo[1] - 3 * dx + np.arange(45) * dx
    PX, PY = np.meshgrid(px, py)
    inside = (PX > lo[0]) & (PX < hi[0]) & (PY > lo[1]) & (PY < hi[1])
    outside = (PX < lo[0]) | (PX > hi[0]) | (PY < lo[1]) | (PY > hi[1])
    assert np.abs(m[inside]).max() <= 1e-15
    assert np.all(m[outside] == 0.0)


def test_sheared_gel_top_plane():
    sc, o, tris, X = gel_surface(7, 6, 3)
    al, be, ga = 0.03, -0.02, -1e-4
    Xs = X.copy()
    Xs[:, 2] += al * X[:, 0] + be * X[:, 1] + ga
    ztop = X[:, 2].max()
    lo, hi = X.min(0), X.max(0)
    nx = ny = 30
    dx, dy = (hi[0] - lo[0]) / (nx + 1), (hi[1] - lo[1]) / (ny + 1)
    x0, y0 = lo[0] + dx, lo[1] + dy
    m = height_map(Xs, tris, x0, y0, dx, dy, nx, ny, ztop)
    PX, PY = np.meshgrid(x0 + np.arange(nx) * dx, y0 + np.arange(ny) * dy)
    ref = ztop - (ztop + al * PX + be * PY + ga)
    assert np.abs(m - ref).max() <= 1e-15


def test_lowered_vertex_on_a_pixel_centre():
    sc, o, tris, X = gel_surface(6, 6, 3)
    xs = np.unique(X[:, 0])
    ys = np.unique(X[:, 1])
    ztop = X[:, 2].max()
    k = np.where((X[:, 0] == xs[2]) & (X[:, 1] == ys[3]) & (X[:, 2] == ztop))[0][0]
    d = 3e-5
    Xd = X.copy()
    Xd[k, 2] -= d
    dx, dy = xs[1] - xs[0], ys[1] - ys[0]
    m = height_map(Xd, tris, xs[0], ys[0], dx, dy, len(xs), len(ys), ztop)
    assert abs(m[3, 2] - d) <= 1e-18
    m[3, 2] = 0.0
    assert np.abs(m).max() <= 1e-18  # every other vertex stays on the top plane


def test_brute_force_tiny():
    sc, o, tris, X = gel_surface(4, 4, 3)
    rng = np.random.default_rng(0)
    Xp = X + rng.normal(0, 2e-5, X.shape)
    ztop = X[:, 2].max()
    lo, hi = X.min(0), X.max(0)
    nx, ny = 17, 13
    dx, dy = (hi[0] - lo[0]) / 15, (hi[1] - lo[1]) / 11
    x0, y0 = lo[0] - dx, lo[1] - dy
    m = height_map(Xp, tris, x0, y0, dx, dy, nx, ny, ztop)
    for j in range(ny):
        for i in range(nx):
            p = (x0 + i * dx, y0 + j * dy)
            best = None
            for t in tris:
                a, b, c = Xp[t[0]], Xp[t[1]], Xp[t[2]]
                area = (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0])
                if area <= 0.0:
                    continue
                w = [(c[0] - b[0]) * (p[1] - b[1]) - (c[1] - b[1]) * (p[0] - b[0]),
                     (a[0] - c[0]) * (p[1] - c[1]) - (a[1] - c[1]) * (p[0] - c[0]),
                     (b[0] - a[0]) * (p[1] - a[1]) - (b[1] - a[1]) * (p[0] - a[0])]
                if all(v >= 0 for v in w):
                    z = (w[0] * a[2] + w[1] * b[2] + w[2] * c[2]) / area
                    best = z if best is None else max(best, z)
            assert m[j, i] == (0.0 if best is None else ztop - best)
