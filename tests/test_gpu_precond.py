"""The multilevel additive preconditioner through the C ABI.

The preconditioner changes the PCG path but not the solution: at a tight
tolerance the Newton direction is the same as with block-Jacobi. Against the
oracle this is checked on config 1 (test_gpu_parity) and through every
Newton-iterate and trajectory test, which run the multilevel default. The
8x8x64 gel here has thin layers, so its cells stack more vertices than one
block holds and the aggregate runs are split (the group caps are checked
before any kernel runs); its reference is the block-Jacobi path (which
follows the oracle iteration by iteration), since the oracle needs minutes
for this ill-conditioned system.
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2411_04776_amd import scenes as S

pytestmark = pytest.mark.gpu

CAP_MEMBERS = 256    # members of one preconditioner group (LDS rows)
CAP_AGGS = 256       # aggregates of one group


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ipc():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_2411_04776_amd import ipc as I
    I.lib()
    return I


def pressed(x, n_gel, fixed, dhat, frac=0.85, seed=4, jiggle=0.05):
    x = x.copy()
    x[n_gel:] -= np.array([0, 0, frac * dhat])
    rng = np.random.default_rng(seed)
    x[:n_gel] += rng.normal(0, jiggle * dhat, (n_gel, 3)) * (1 - fixed[:, None])
    return x


def layered_scene():
    return S.tiny_scene(grid=(8, 8, 64), radius=1.5e-3, subdiv=2)


def check_info(info, sc):
    n_free = int(len(sc.fixed) - np.count_nonzero(sc.fixed))
    assert info["members"] == n_free
    assert 1 <= info["levels"] <= 3
    assert info["max_group_members"] <= CAP_MEMBERS
    assert info["max_group_aggs"] <= CAP_AGGS
    counts = [info[f"aggs{l}"] for l in range(info["levels"])]
    assert all(a > b for a, b in zip(counts, counts[1:]))
    assert counts[0] < n_free
    assert info["groups"] >= 1


@pytest.mark.parametrize("name", ["config1", "config2", "layered"])
def test_hierarchy_invariants(ipc, name):
    sc = {"config1": S.config1, "config2": S.config2, "layered": layered_scene}[name]()
    g = ipc.GelScene(sc)
    info = g.precond_info()
    say(name, info)
    check_info(info, sc)
    j = ipc.GelScene(sc, precond=ipc.IPC_PRECOND_JACOBI)
    assert j.precond_info()["levels"] == 0


def test_split_aggregates_pcg_parity(ipc):
    sc = layered_scene()
    g = ipc.GelScene(sc)
    info = g.precond_info()
    say("layered", info)
    check_info(info, sc)
    # runs longer than a group were split: the largest group is near the cap
    assert info["max_group_members"] > CAP_MEMBERS // 2
    j = ipc.GelScene(sc, precond=ipc.IPC_PRECOND_JACOBI)
    g.begin_step(sc.poses[1])
    j.begin_step(sc.poses[1])
    x = pressed(g.x, len(sc.fixed), sc.fixed, sc.dhat)
    pj, itj = j.pcg(x)
    pg, itg = g.pcg(x)
    L = sc.bbox_diag
    say("  pcg iterations multilevel/block-Jacobi", itg, itj, "max diff / L", np.abs(pg - pj).max() / L)
    assert itg < itj
    assert np.abs(pg - pj).max() <= 1e-9 * L


@pytest.mark.parametrize("precision", [0, 1])
def test_mixed_preconditioners_in_one_list(ipc, precision):
    """A list holding scenes with either preconditioner steps each of them
    bit for bit as it steps alone."""
    tol = 1e-8 if precision == 0 else 1e-6
    pcs = [ipc.IPC_PRECOND_MULTILEVEL, ipc.IPC_PRECOND_JACOBI, ipc.IPC_PRECOND_MULTILEVEL]
    scs = [S.uneven_scene(7000 + k, steps=2, grid=(14, 12, 5)) for k in range(3)]
    alone = []
    for sc, pc in zip(scs, pcs):
        g = ipc.GelScene(sc, precision=precision, pcg_tol=tol, precond=pc)
        for k in range(sc.n_steps):
            rc, _ = g.step()
            assert rc == 0
        alone.append(g.x)
    gs = [ipc.GelScene(sc, precision=precision, pcg_tol=tol, precond=pc) for sc, pc in zip(scs, pcs)]
    b = ipc.Batch()
    for k in range(scs[0].n_steps):
        for t in b.submit(gs):
            rc, _ = b.wait(t)
            assert rc == 0
    b.close()
    for g, xa in zip(gs, alone):
        assert np.array_equal(g.x, xa)


def test_heavy_member_rows_trajectory(ipc):
    """A fine icosphere on a coarse gel: a free gel vertex (an aggregate
    member) collects more incident contact entries than one thread sums, so
    its group block sums that row cooperatively. Three steps against the
    oracle."""
    sc = S.tiny_scene(grid=(5, 5, 3), radius=2e-3, subdiv=4, steps=3)
    L = sc.bbox_diag
    g = ipc.GelScene(sc)
    o = O.OracleScene(sc)
    heavy = 0
    for k in range(sc.n_steps):
        rc, st = g.step()
        o.step(sc.poses[k + 1])
        assert rc == 0
        err = np.abs(g.x - o.x).max() / L
        c = o.candidates(o.x)
        d, _ = o.candidate_distances(o.x, c)
        _, edges, tris = o.surface()
        cnt = np.zeros(o.n, int)
        for t, a, b in c[d < sc.dhat]:
            for v in ([a, *tris[b]] if t == 0 else [*edges[a], *edges[b]]):
                cnt[v] += 1
        heavy = max(heavy, int((cnt[:o.n_gel] * (1 - sc.fixed) > 24).sum()))
        say(f"  step {k + 1}: newton {st.newton_iters} pcg {st.pcg_iters} err/L {err:.2e} heavy gel rows {heavy}")
        assert err <= 1e-9
    assert heavy >= 1
