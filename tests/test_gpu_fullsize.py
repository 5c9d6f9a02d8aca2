"""HIP path against the FP64 oracle at the sizes that carry the benchmark's
claims, through the C ABI. Every expected value is the oracle's, written by
tests/golden/make_fullsize.py (offsets stored as float32: at most 2^-24 of
one Newton step of rounding, < 1e-10 L).

* config 5 (80x100x16 gel, 703,890 tets, sphere, friction mu = 0.5): a
  constructed pressed-and-sliding state (scenes.pressed_state: the sphere
  0.9 mm past first touch after 20 slide steps), friction lagged there, one
  Newton iterate of the next step: candidates bit-exact, the iterate within
  1e-9 L in FP64 and 1e-4 L in the mixed form.
* config 2 seeds 0-2 (cylinder, cube edge, 128x128 bumpy plate): the
  oracle's own state after step 25 (rounded to float32 offsets: that rounded
  state is the input of both sides), the first two Newton iterates of step 26
  teacher-forced within 1e-9 L, candidates bit-exact, gradient and H v
  within 1e-11 per row block (gel rows and indenter rows each against their
  own largest entry).
* config 3: the 16 sampled scenes of the 256-scene list (0, 16, ..., 240),
  all 20 steps from rest at the benchmark's PCG tolerance, in the batched
  mixed form (the engine, all 16 in one list) and one at a time in plain
  FP64: final positions within 1e-4 L of the oracle's (fixed error).
"""
import os
import sys

import numpy as np
import pytest

import oracle as O
from paper_2411_04776_amd import scenes as S

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
BENCH_PCG_TOL = 3e-5


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


def golden(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.skip(f"{name} not generated")
    return np.load(path)


def rest_all(sc, step):
    return np.concatenate([sc.X, S.apply_pose(sc.poses[step], sc.Y)])


def block_close(a, b, n_gel, rel):
    """|a - b| within rel of the largest |b| entry, gel rows and indenter
    rows each against their own scale."""
    for sl in (slice(0, n_gel), slice(n_gel, None)):
        scale = np.abs(b[sl]).max()
        if scale == 0.0:
            assert np.abs(a[sl]).max() == 0.0
            continue
        d = np.abs(a[sl] - b[sl]).max()
        if d > rel * scale:
            return False, d / scale
    return True, 0.0


@pytest.fixture(scope="module")
def c5_case():
    z = golden("c5_tf.npz")
    sc = S.config5()
    step = int(z["step"])
    x0, v0 = S.pressed_state(sc, step - 1)
    return sc, step, x0, v0, x0 + z["it1"].astype(np.float64)


def test_c5_candidates_bit_exact(ipc, c5_case):
    sc, step, x0, v0, _ = c5_case
    o = O.OracleScene(sc)
    co = o.candidates(x0)
    g = ipc.GelScene(sc, precision=ipc.IPC_MIXED)
    cg = g.candidates(x0)
    d, _ = o.candidate_distances(x0, co)
    say(f"  config 5 pressed state: {len(cg)} candidates (oracle {len(co)}), {(d < sc.dhat).sum()} active, "
        f"min d = {d.min() / sc.dhat:.3f} dhat")
    assert cg.shape == co.shape and np.array_equal(cg, co)
    g.close()


@pytest.mark.parametrize("form", ["fp64", "mixed"])
def test_c5_teacher_forced_iterate(ipc, c5_case, form):
    sc, step, x0, v0, ref = c5_case
    L = sc.bbox_diag
    prec = ipc.IPC_FP64 if form == "fp64" else ipc.IPC_MIXED
    g = ipc.GelScene(sc, precision=prec, pcg_tol=1e-12 if form == "fp64" else 1e-7)
    g.x = x0
    g.v = v0
    g.begin_step(sc.poses[step])
    rc, xg, st = g.newton_iterate(x0)
    assert rc == 0
    err = np.abs(xg - ref).max() / L
    say(f"  config 5 {form}: iterate alpha={st.alpha:.6f} pcg={st.pcg_iters} active={st.n_active} "
        f"err/L={err:.3e} (largest move {np.abs(ref - x0).max():.3e} m)")
    assert err <= (1e-9 if form == "fp64" else 1e-4)
    g.close()


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_c2_teacher_forced_iterates(ipc, seed):
    z = golden(f"c2_seed{seed}_tf.npz")
    sc = S.config2(seed)
    step = int(z["step"])
    x0 = rest_all(sc, step - 1) + z["dx"].astype(np.float64)
    v0 = z["dv"].astype(np.float64)
    x1 = x0 + z["it1"].astype(np.float64)
    x2 = x1 + z["it2"].astype(np.float64)
    L = sc.bbox_diag
    n_gel = len(sc.X)
    o = O.OracleScene(sc)
    o.x, o.v = x0, v0
    o.begin_step(sc.poses[step])
    g = ipc.GelScene(sc)
    g.x, g.v = x0, v0
    g.begin_step(sc.poses[step])
    co, cg = o.candidates(x0), g.candidates(x0)
    say(f"  config 2 seed {seed} ({sc.meta['kind']}): {len(cg)} candidates at the state after step {step - 1}")
    assert cg.shape == co.shape and np.array_equal(cg, co)
    ok, r = block_close(g.gradient(x0), o.gradient(x0), n_gel, 1e-11)
    assert ok, f"gradient off by {r:.2e} of its row block's scale"
    rng = np.random.default_rng(seed)
    v = rng.normal(size=x0.shape)
    ok, r = block_close(g.hess_apply(x0, v), o.hess_apply(x0, v), n_gel, 1e-11)
    assert ok, f"H v off by {r:.2e} of its row block's scale"
    for k, (xin, ref) in enumerate(((x0, x1), (x1, x2))):
        rc, xg, st = g.newton_iterate(xin)
        assert rc == 0
        err = np.abs(xg - ref).max() / L
        say(f"    iterate {k + 1}: alpha={st.alpha:.6f} pcg={st.pcg_iters} active={st.n_active} err/L={err:.3e}")
        assert err <= 1e-9
    g.close()


def c3_goldens():
    out = {}
    for i in range(0, 256, 16):
        path = os.path.join(GOLDEN, f"c3_{i}_final.npz")
        if os.path.exists(path):
            out[i] = np.load(path)
    return out


def test_c3_sampled_final_error(ipc):
    gz = c3_goldens()
    if len(gz) < 16:
        pytest.skip(f"only {len(gz)} of the 16 config-3 goldens generated")
    scs = {i: S.config3_scene(i) for i in gz}
    # batched, mixed: all 16 in one list through the engine
    gs = {i: ipc.GelScene(sc, precision=ipc.IPC_MIXED, pcg_tol=BENCH_PCG_TOL) for i, sc in scs.items()}
    b = ipc.Batch()
    for k in range(20):
        for t in b.submit(list(gs.values())):
            rc, st = b.wait(t)
            assert rc >= 0, rc
    b.close()
    worst = {}
    for name, runs in (("batched mixed", gs),):
        for i, g in runs.items():
            ref = scs[i].X + gz[i]["dx"].astype(np.float64)
            worst[(name, i)] = float(np.linalg.norm(g.x[:len(ref)] - ref, axis=1).max() / float(gz[i]["L"]))
    for g in gs.values():
        g.close()
    # one at a time, plain FP64
    for i, sc in scs.items():
        g = ipc.GelScene(sc, precision=ipc.IPC_FP64, pcg_tol=BENCH_PCG_TOL)
        for k in range(20):
            rc, st = g.step()
            assert rc >= 0, rc
        ref = sc.X + gz[i]["dx"].astype(np.float64)
        worst[("per-scene fp64", i)] = float(np.linalg.norm(g.x[:len(ref)] - ref, axis=1).max() / float(gz[i]["L"]))
        g.close()
    for name in ("batched mixed", "per-scene fp64"):
        e = [v for (n, _), v in worst.items() if n == name]
        say(f"  config 3, 16 sampled scenes, {name}: final error / L max {max(e):.3e}, median {np.median(e):.3e}")
        assert max(e) <= 1e-4
