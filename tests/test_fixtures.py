"""Scene fixtures and the oracle's mesh precompute against closed forms.

Counts follow from the grid: (nx-1)(ny-1)(nz-1) hexes x 6 Kuhn tets; every
boundary quad gives two surface triangles; the surface of a box is a sphere
(Euler characteristic 2). Volumes and masses follow from the box size.
"""
import numpy as np
import pytest

import oracle as O
from paper_2411_04776_amd import scenes as S


def grid_counts(nx, ny, nz):
    n = nx * ny * nz
    m = 6 * (nx - 1) * (ny - 1) * (nz - 1)
    quads = 2 * ((nx - 1) * (ny - 1) + (nx - 1) * (nz - 1) + (ny - 1) * (nz - 1))
    surf_v = n - max(nx - 2, 0) * max(ny - 2, 0) * max(nz - 2, 0)
    return n, m, 2 * quads, surf_v


@pytest.mark.parametrize("grid,tets", [((16, 20, 4), 5130), ((40, 50, 8), 80262), ((80, 100, 16), 703890)])
def test_grid_counts_and_volume(grid, tets):
    X, T, fixed = S.grid_gel(*grid)
    n, m, _, _ = grid_counts(*grid)
    assert X.shape == (n, 3) and T.shape == (m, 4) and m == tets
    assert fixed.sum() == grid[0] * grid[1]
    P = X[T]
    D = np.stack([P[:, 1] - P[:, 0], P[:, 2] - P[:, 0], P[:, 3] - P[:, 0]], axis=2)
    vol = np.linalg.det(D) / 6.0
    assert vol.min() > 0
    assert abs(vol.sum() - np.prod(S.GEL_SIZE)) < 1e-12 * np.prod(S.GEL_SIZE) * 100


def test_icosphere_counts():
    for sub, nf, nv in ((0, 20, 12), (1, 80, 42), (2, 320, 162), (4, 5120, 2562)):
        V, F = S.icosphere(sub, 5e-3)
        assert F.shape == (nf, 3) and V.shape == (nv, 3)
        assert np.allclose(np.linalg.norm(V, axis=1), 5e-3)
        # closed: V - E + F = 2
        e = {tuple(sorted((a, b))) for t in F for a, b in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0]))}
        assert nv - len(e) + nf == 2
        if sub == 2:
            assert len(e) == 480


def _signed_volume(V, F):
    a, b, c = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    return np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6.0


def test_indenter_meshes_closed_and_outward():
    for V, F in (S.cylinder(3e-3, 30e-3), S.box(7e-3), S.icosphere(2, 5e-3)):
        assert _signed_volume(V, F) > 0  # outward orientation
        e = {}
        for t in F:
            for a, b in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0])):
                e[(a, b)] = e.get((a, b), 0) + 1
        # closed and consistently oriented: every directed edge once, its reverse once
        assert all(v == 1 for v in e.values())
        assert all((b, a) in e for (a, b) in e)
    V, F = S.box(7e-3)
    assert abs(_signed_volume(V, F) - 7e-3 ** 3) < 1e-15


@pytest.mark.parametrize("grid", [(16, 20, 4), (5, 7, 3)])
def test_oracle_surface_extraction(grid):
    sc = S.config1() if grid == (16, 20, 4) else S.tiny_scene(grid=grid)
    o = O.OracleScene(sc)
    n, m, nst, nsv = grid_counts(*grid)
    assert o.n_gel == n and o.n_tet == m
    assert o.n_gel_tris == nst
    pts, edges, tris = o.surface()
    gel_pts = pts[pts < o.n_gel]
    assert len(gel_pts) == nsv
    gel_tris = tris[:o.n_gel_tris]
    gel_edges = edges[(edges < o.n_gel).all(axis=1)]
    # Euler characteristic of the box surface
    assert nsv - len(gel_edges) + nst == 2
    # outward: divergence theorem gives the rest volume
    vol = _signed_volume(sc.X, gel_tris)
    assert abs(vol - np.prod(sc.X.max(0) - sc.X.min(0))) < 1e-9 * vol
    # canonical numbering: triangles rotated min-first and sorted; edges sorted
    assert (gel_tris[:, 0] < gel_tris[:, 1]).all() and (gel_tris[:, 0] < gel_tris[:, 2]).all()
    assert (np.diff(gel_tris[:, 0]) >= 0).all()
    assert (edges[:, 0] < edges[:, 1]).all()
    # rest volumes and lumped masses
    vol_e, mass = o.rest()
    assert abs(vol_e.sum() - vol) < 1e-9 * vol
    assert abs(mass[:o.n_gel].sum() - sc.rho * vol) < 1e-9 * sc.rho * vol
    assert (mass[o.n_gel:] == 0).all()


def test_config1_counts():
    o = O.OracleScene(S.config1())
    assert (o.n_gel, o.n_tet, o.n_gel_tris) == (1280, 5130, 1548)
    assert o.n_ind == 162 and o.n_tris == 1548 + 320 and o.n_edges == 2322 + 480
    assert o.n_pts == 776 + 162


def test_bad_mesh_rejected():
    sc = S.tiny_scene()
    T = sc.T.copy()
    T[0, [1, 2]] = T[0, [2, 1]]  # inverted tet
    sc.T = T
    with pytest.raises(ValueError):
        O.OracleScene(sc)


def test_initial_pose_touchdown_gap():
    sc = S.config1()
    y0 = S.apply_pose(sc.poses[0], sc.Y)
    assert abs(y0[:, 2].min() - (S.GEL_SIZE[2] + S.DHAT)) < 1e-15
    y10 = S.apply_pose(sc.poses[10], sc.Y)
    assert abs((y0[:, 2].min() - y10[:, 2].min()) - 1e-3) < 1e-15
