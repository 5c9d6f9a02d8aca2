"""The HIP path's body and barrier stages, each on its own, against the FP64
oracle through the C ABI (ipcx_assemble_elastic, ipcx_barrier), and the two
stages adding up to the whole gradient and H v.

Tolerances (FP64 path): body gradient and H_body v 1e-11 of the largest
entry of the row block (summation order only); the active pairs' kinds and
vertex ids bit-exact (candidate order); each pair's gradient 1e-11 and its
projected Hessian 1e-10 of that pair's largest entry (the HIP path projects
in the pair's rank-5 span with its own 5x5 Jacobi, the oracle with a 12x12
Jacobi: the same matrix up to rounding).
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2411_04776_amd import scenes as S
from parity_util import assert_rows_close

pytestmark = pytest.mark.gpu


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


def pressed(o, sc, frac=0.85, seed=2, jiggle=0.05):
    x = o.x.copy()
    x[o.n_gel:] -= np.array([0.0, 0.0, frac * sc.dhat])
    rng = np.random.default_rng(seed)
    x[:o.n_gel] += rng.normal(0, jiggle * sc.dhat, (o.n_gel, 3)) * (1 - sc.fixed[:, None])
    return x


def fixed_all(o, sc):
    f = np.zeros(o.n, dtype=bool)
    f[:o.n_gel] = sc.fixed.astype(bool)
    return f


def pair_products(kind, v4, H, v):
    y = np.zeros_like(v)
    for k in range(len(kind)):
        y[v4[k]] += (H[k] @ v[v4[k]].reshape(12)).reshape(4, 3)
    return y


CASES = [("tiny", 0), ("config1", 0), ("config1", 1)]


def make(name):
    return S.tiny_scene() if name == "tiny" else S.config1()


@pytest.mark.parametrize("name,gn", CASES)
def test_body_stage(ipc, name, gn):
    sc = make(name)
    say("body stage", sc.name, "gauss-newton" if gn else "projected")
    g = ipc.GelScene(sc, barrier_hessian=ipc.IPC_BARRIER_GAUSS_NEWTON if gn else ipc.IPC_BARRIER_PROJECTED)
    o = O.OracleScene(sc, barrier_hessian=gn)
    g.begin_step(sc.poses[1])
    o.begin_step(sc.poses[1])
    x = pressed(o, sc)
    fixed = fixed_all(o, sc)
    t = o.gradient_terms(x)
    gb_o = t["inertia"] + t["elastic"] + t["target"]
    gb_o[fixed] = 0.0
    v = np.random.default_rng(4).normal(size=x.shape)
    gb, yb = g.assemble_elastic(x, v)
    assert_rows_close(gb, gb_o, o.n_gel, 1e-11)
    assert_rows_close(yb, o.hess_apply_body(x, v), o.n_gel, 1e-11)
    g.close()


@pytest.mark.parametrize("name,gn", CASES)
def test_barrier_stage(ipc, name, gn):
    sc = make(name)
    g = ipc.GelScene(sc, barrier_hessian=ipc.IPC_BARRIER_GAUSS_NEWTON if gn else ipc.IPC_BARRIER_PROJECTED)
    o = O.OracleScene(sc, barrier_hessian=gn)
    g.begin_step(sc.poses[1])
    o.begin_step(sc.poses[1])
    x = pressed(o, sc)
    fixed = fixed_all(o, sc)
    kg, vg, gg, Hg = g.barrier_pairs(x)
    ko, vo, go, Ho = o.contact_pairs(x)
    say(f"barrier stage {sc.name} {'gauss-newton' if gn else 'projected'}: {len(kg)} pairs "
        f"({int((kg == 0).sum())} PT, {int((kg == 1).sum())} EE), oracle {len(ko)}")
    assert len(ko) > 0
    assert np.array_equal(kg, ko) and np.array_equal(vg, vo)
    worst_g = worst_H = 0.0
    for k in range(len(ko)):
        m = np.repeat(~fixed[vo[k]], 3)  # Dirichlet rows and columns drop out of the pair terms
        g_ref, H_ref = go[k] * m, Ho[k] * np.outer(m, m)
        sg, sH = np.abs(g_ref).max(), np.abs(H_ref).max()
        if sg > 0:
            worst_g = max(worst_g, np.abs(gg[k] - g_ref).max() / sg)
        else:
            assert np.abs(gg[k]).max() == 0.0
        if sH > 0:
            worst_H = max(worst_H, np.abs(Hg[k] - H_ref).max() / sH)
        else:
            assert np.abs(Hg[k]).max() == 0.0
    say(f"    worst pair gradient {worst_g:.2e}, Hessian {worst_H:.2e} of the pair's largest entry")
    assert worst_g <= 1e-11 and worst_H <= 1e-10
    g.close()


@pytest.mark.parametrize("name,gn", CASES)
def test_stages_add_up(ipc, name, gn):
    """The library's whole gradient and H v are its two stages' sums."""
    sc = make(name)
    g = ipc.GelScene(sc, barrier_hessian=ipc.IPC_BARRIER_GAUSS_NEWTON if gn else ipc.IPC_BARRIER_PROJECTED)
    o = O.OracleScene(sc, barrier_hessian=gn)
    g.begin_step(sc.poses[1])
    o.begin_step(sc.poses[1])
    x = pressed(o, sc)
    v = np.random.default_rng(6).normal(size=x.shape)
    gb, yb = g.assemble_elastic(x, v)
    kind, v4, g12, H = g.barrier_pairs(x)
    gc = np.zeros_like(x)
    for k in range(len(kind)):
        np.add.at(gc, v4[k], g12[k].reshape(4, 3))
    say("stages add up", sc.name, "gauss-newton" if gn else "projected", len(kind), "pairs")
    assert_rows_close(gb + gc, g.gradient(x), o.n_gel, 1e-11)
    assert_rows_close(yb + pair_products(kind, v4, H, v), g.hess_apply(x, v), o.n_gel, 1e-11)
    g.close()
