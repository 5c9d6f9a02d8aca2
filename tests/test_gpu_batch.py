"""Lists of scenes in shared launches and the continuous-batching engine.

Every kernel runs over a list of scenes with one block range per scene, and a
scene's partial sums and reduction order depend on that scene alone, so its
trajectory is bitwise the same stepped alone (ipc_step) or through the batch
engine in any mix: uneven sizes, both precisions, scenes joining while others
are mid-step, and admission limited by a memory budget.
"""
import sys
import time

import numpy as np
import pytest

from paper_2411_04776_amd import scenes as S

pytestmark = pytest.mark.gpu

PCG_TOL = {0: 1e-8, 1: 1e-5}


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


def mix():
    return [S.tiny_scene(), S.config1(), S.config3_scene(3, steps=6),
            S.tiny_scene(grid=(6, 5, 4), radius=1.5e-3, subdiv=2)]


def run_alone(ipc, sc, steps, precision):
    g = ipc.GelScene(sc, precision=precision, pcg_tol=PCG_TOL[precision])
    xs, sts = [], []
    for _ in range(steps):
        rc, st = g.step()
        xs.append(g.x)
        sts.append((rc, st.newton_iters, st.pcg_iters, st.ls_halvings))
    g.close()
    return xs, sts


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_bitwise_equals_alone(ipc, precision):
    scs = mix()
    steps = 3
    ref = [run_alone(ipc, sc, steps, precision) for sc in scs]
    gs = [ipc.GelScene(sc, precision=precision, pcg_tol=PCG_TOL[precision]) for sc in scs]
    b = ipc.Batch()
    for k in range(steps):
        tks = b.submit(gs)
        for i, t in enumerate(tks):
            rc, st = b.wait(t)
            got = (rc, st.newton_iters, st.pcg_iters, st.ls_halvings)
            say(f"  prec {precision} step {k + 1} {scs[i].name}: {got}")
            assert got == ref[i][1][k]
            assert np.array_equal(gs[i].x, ref[i][0][k])
    b.close()


def test_continuous_batching_staggered_mixed_precisions(ipc):
    """Scenes start at different times, each submits its next step as soon as
    the previous one is done; FP64 and mixed scenes share the engine."""
    scs = mix()
    precs = [0, 1, 0, 1]
    steps = 2
    ref = [run_alone(ipc, sc, steps, p) for sc, p in zip(scs, precs)]
    gs = [ipc.GelScene(sc, precision=p, pcg_tol=PCG_TOL[p]) for sc, p in zip(scs, precs)]
    b = ipc.Batch()
    start = [0.0, 0.004, 0.015, 0.030]
    done = [0] * len(gs)
    ticket = [None] * len(gs)
    t0 = time.perf_counter()
    while min(done) < steps:
        now = time.perf_counter() - t0
        for i, g in enumerate(gs):
            if ticket[i] is None and done[i] < steps and now >= start[i]:
                ticket[i] = b.submit([g])[0]
            elif ticket[i] is not None:
                fin, _ = b.poll(ticket[i])
                if fin:
                    rc, st = b.wait(ticket[i])
                    ticket[i] = None
                    got = (rc, st.newton_iters, st.pcg_iters, st.ls_halvings)
                    assert got == ref[i][1][done[i]], (scs[i].name, got, ref[i][1][done[i]])
                    assert np.array_equal(g.x, ref[i][0][done[i]])
                    done[i] += 1
                    say(f"  {scs[i].name} step {done[i]} ok ({st.ms_total:.1f} ms)")
        time.sleep(0.0005)
        assert time.perf_counter() - t0 < 120
    b.close()


def test_memory_budget_admission(ipc):
    """A budget below one scene's footprint admits one scene at a time; the
    results do not change."""
    scs = mix()[:3]
    ref = [run_alone(ipc, sc, 1, 0) for sc in scs]
    gs = [ipc.GelScene(sc, pcg_tol=PCG_TOL[0]) for sc in scs]
    b = ipc.Batch(mem_budget=1)
    tks = b.submit(gs)
    for i, t in enumerate(tks):
        rc, st = b.wait(t)
        assert (rc, st.newton_iters, st.pcg_iters, st.ls_halvings) == ref[i][1][0]
        assert np.array_equal(gs[i].x, ref[i][0][0])
    b.close()


def test_busy_scene_rejected(ipc):
    sc = S.config1()
    g = ipc.GelScene(sc)
    b = ipc.Batch()
    t = b.submit([g])[0]
    with pytest.raises(ipc.IPCError) as e:
        b.submit([g])
    assert e.value.code == ipc.IPC_E_BUSY
    # the same scene twice in one submit is refused as a whole
    g2 = ipc.GelScene(S.tiny_scene())
    with pytest.raises(ipc.IPCError):
        b.submit([g2, g2])
    rc, st = b.wait(t)
    assert rc in (0, 4)
    with pytest.raises(ipc.IPCError):
        b.wait(t)  # a ticket is consumed by wait
    rc, st = g2.step()  # idle again: a plain step works
    assert rc in (0, 4)
    b.close()


def test_engine_profile_counts(ipc):
    """The engine's kernel timing: timed SpMV launches, positive time and the
    algorithmic bytes of the list (at least every stored block once per
    timed launch); disabling resets nothing until enabled again."""
    scs = mix()[:3]
    gs = [ipc.GelScene(sc, precision=1, pcg_tol=PCG_TOL[1]) for sc in scs]
    b = ipc.Batch()
    b.profile(True)
    for t in b.submit(gs):
        rc, _ = b.wait(t)
        assert rc == 0
    n, ms, by = b.profile_read(0)
    say(f"  engine SpMV: {n} timed launches, {ms:.3f} ms, {by / max(n, 1):.0f} B per launch")
    assert n > 0 and ms > 0
    min_bytes = min(40 * g.matrix_info()["nnzb"] for g in gs)
    assert by >= n * min_bytes
    b.profile(False)
    assert b.profile_read(0)[0] == 0
    b.close()


def test_large_list_bitwise_equals_alone(ipc):
    """A list above 65536 matrix rows runs the SpMV with a thread per row,
    a scene alone with two lanes per row; both forms give the same bits."""
    scs = [S.uneven_scene(6000 + k, steps=2) for k in range(16)]
    rows = sum(len(sc.X) + len(sc.Y) for sc in scs)
    say(f"  list rows {rows}")
    assert rows >= 65536
    ref = []
    for sc in scs:
        g = ipc.GelScene(sc, precision=1, pcg_tol=PCG_TOL[1])
        rc, st = g.step()
        ref.append((rc, st.newton_iters, st.pcg_iters, g.x))
        g.close()
    gs = [ipc.GelScene(sc, precision=1, pcg_tol=PCG_TOL[1]) for sc in scs]
    b = ipc.Batch()
    for i, t in enumerate(b.submit(gs)):
        rc, st = b.wait(t)
        assert (rc, st.newton_iters, st.pcg_iters) == ref[i][:3]
        assert np.array_equal(gs[i].x, ref[i][3])
    b.close()


def test_size_classes_and_wait_any(ipc):
    """A scene above IPC_BATCH_LARGE_VERTS steps in the large class (its own
    list, worker and stream) while small scenes of both precisions keep
    stepping; every result is bitwise the one alone, and the wait-any call
    hands back every ticket exactly once."""
    big = S.uneven_scene(7200, steps=3, grid=(64, 64, 17))
    assert len(big.X) + len(big.Y) >= 65536
    scs = [big] + mix()
    precs = [1, 0, 1, 0, 1]
    steps = 2
    ref = [run_alone(ipc, sc, steps, p) for sc, p in zip(scs, precs)]
    gs = [ipc.GelScene(sc, precision=p, pcg_tol=PCG_TOL[p]) for sc, p in zip(scs, precs)]
    b = ipc.Batch()
    with pytest.raises(ipc.IPCError):
        b.next(0.0)  # nothing pending or finished
    for k in range(steps):
        tks = b.submit(gs[:1])
        tks += b.submit(gs[1:])
        seen, order = {}, []
        while len(seen) < len(tks):
            r = b.next(10000.0)
            assert r is not None, "wait-any timed out"
            t, rc, st = r
            assert t in tks and t not in seen
            i = tks.index(t)
            seen[t] = (rc, st.newton_iters, st.pcg_iters, st.ls_halvings)
            order.append(i)
        say(f"  step {k + 1}: completion order {order}")
        for i, t in enumerate(tks):
            assert seen[t] == ref[i][1][k], (i, seen[t], ref[i][1][k])
            assert np.array_equal(gs[i].x, ref[i][0][k])
    b.close()
