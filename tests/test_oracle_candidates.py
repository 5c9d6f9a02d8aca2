"""Oracle candidate sets against an independent all-pairs numpy evaluation of
the closed box-overlap predicate, and completeness against true distances."""
import numpy as np
import pytest

import oracle as O
from paper_2411_04776_amd import scenes as S


def numpy_candidates(o, x, p=None, use_boxes=True):
    """All-pairs box predicate, vectorised; same pair rules as documented.
    use_boxes=False returns every pair the rules admit."""
    pts, edges, tris = o.surface()
    fixed = np.zeros(o.n, dtype=bool)
    fixed[:o.n_gel] = o.scene.fixed.astype(bool)
    r = 0.5 * o.scene.dhat
    ends = [x] if p is None else [x, x + p]

    def boxes(idx):
        lo = np.min(np.stack([e[idx] for e in ends], 0), axis=(0, 2))
        hi = np.max(np.stack([e[idx] for e in ends], 0), axis=(0, 2))
        return lo - r, hi + r

    plo, phi = boxes(pts[:, None])
    tlo, thi = boxes(tris)
    elo, ehi = boxes(edges)
    def ov(alo, ahi, blo, bhi):
        if not use_boxes:
            return np.ones((len(alo), len(blo)), dtype=bool)
        return np.all((alo[:, None] <= bhi[None]) & (blo[None] <= ahi[:, None]), axis=2)
    ng = o.n_gel
    out = set()
    M = ov(plo, phi, tlo, thi)
    for i, j in zip(*np.nonzero(M)):
        a, tv = pts[i], tris[j]
        if a in tv:
            continue
        ai, ti = a >= ng, tv[0] >= ng
        if ai and ti:
            continue
        if not ai and not ti and not o.scene.self_contact:
            continue
        if fixed[a] and fixed[tv].all():
            continue
        out.add((0, int(a), int(j)))
    M = ov(elo, ehi, elo, ehi)
    for i, j in zip(*np.nonzero(np.triu(M, 1))):
        va, vb = edges[i], edges[j]
        if set(va) & set(vb):
            continue
        ai, bi = va[0] >= ng, vb[0] >= ng
        if ai and bi:
            continue
        if not ai and not bi and not o.scene.self_contact:
            continue
        if fixed[va].all() and fixed[vb].all():
            continue
        out.add((1, int(i), int(j)))
    return out


def _states(o, rng):
    sc = o.scene
    x0 = o.x
    yield x0, None
    # press the indenter into the contact zone and jiggle the gel
    x = x0.copy()
    x[o.n_gel:] -= np.array([0, 0, 0.6 * sc.dhat])
    x[:o.n_gel] += rng.normal(0, 0.15 * sc.dhat, (o.n_gel, 3)) * (1 - sc.fixed[:, None])
    yield x, None
    p = rng.normal(0, 0.5 * sc.dhat, x.shape)
    p[:o.n_gel][sc.fixed.astype(bool)] = 0
    yield x, p


@pytest.mark.parametrize("self_contact", [True, False])
def test_candidates_equal_numpy_all_pairs(self_contact):
    sc = S.tiny_scene(self_contact=self_contact)
    o = O.OracleScene(sc)
    rng = np.random.default_rng(3)
    for x, p in _states(o, rng):
        c = o.candidates(x, p)
        assert len(c) == len({tuple(r) for r in c})
        # canonical order (type, a, b)
        keys = c[:, 0].astype(np.int64) << 40 | c[:, 1].astype(np.int64) << 20 | c[:, 2]
        assert (np.diff(keys) > 0).all()
        assert {tuple(map(int, r)) for r in c} == numpy_candidates(o, x, p)


def test_candidates_complete_against_true_distance():
    """Every non-excluded pair closer than dhat is a static candidate."""
    sc = S.tiny_scene()
    o = O.OracleScene(sc)
    pts, edges, tris = o.surface()
    rng = np.random.default_rng(4)
    x = o.x
    x[o.n_gel:] -= np.array([0, 0, 0.9 * sc.dhat])
    x[:o.n_gel] += rng.normal(0, 0.05 * sc.dhat, (o.n_gel, 3)) * (1 - sc.fixed[:, None])
    cand = {tuple(map(int, r)) for r in o.candidates(x)}
    allc = np.array(sorted(numpy_candidates(o, x, use_boxes=False)), dtype=np.int32)
    d, _ = o.candidate_distances(x, allc)
    close = {tuple(map(int, r)) for r, dd in zip(allc, d) if dd < sc.dhat}
    assert len(close) >= 5, "state must put some pairs inside dhat"
    assert close <= cand


def test_rest_state_has_no_active_pair():
    o = O.OracleScene(S.config1())
    x = o.x
    c = o.candidates(x)
    d, _ = o.candidate_distances(x, c)
    assert len(c) > 1000
    assert d.min() > o.scene.dhat
