"""Engine and scene-state regressions through the C ABI.

* A friction scene in mid-step keeps its lagged friction set when the engine
  admits another request (the admission's step start touches only the
  admitted scenes): its trajectory is bitwise the one it takes alone.
* A broad-phase verdict of non-finite positions belongs to that broad phase
  only: after a failed step, ipc_reset and the next step succeed, bitwise as
  on a fresh scene, and a later scene stepping in the same engine slot is not
  refused.
* ipc_save_state / ipc_load_state carry the sensor case pose: an attached
  scene loaded from a blob steps (case pose not re-sent) exactly as the
  saved run does.
"""
import ctypes as C
import sys
import time

import numpy as np
import pytest

from paper_2411_04776_amd import scenes as S

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


def test_friction_scene_keeps_lag_set_across_admissions(ipc):
    slide = S.tiny_slide_scene(mu=0.5)
    steps = slide.n_steps
    alone = ipc.GelScene(slide)
    ref = []
    for _ in range(steps):
        rc, st = alone.step()
        ref.append((rc, st.newton_iters, st.pcg_iters, alone.x))
    alone.close()

    g = ipc.GelScene(slide)
    other_scs = [S.tiny_scene(steps=40), S.tiny_scene(grid=(5, 4, 3), steps=40)]
    others = [ipc.GelScene(sc) for sc in other_scs]
    eng = ipc.Batch()
    admitted_mid = 0
    for k in range(steps):
        (t,) = eng.submit([g])
        # keep admitting short steps of the other scenes while the slide step runs
        pend = {}
        t0 = time.perf_counter()
        while True:
            done, _ = eng.poll(t)
            if done:
                break
            for j, o in enumerate(others):
                if j in pend:
                    ok, _ = eng.poll(pend[j])
                    if not ok:
                        continue
                    eng.wait(pend[j])
                    del pend[j]
                if o.step_index + 1 < len(o.scene.poses):
                    (pend[j],) = eng.submit([o])
                    admitted_mid += 1
            time.sleep(0.0002)
            assert time.perf_counter() - t0 < 60
        rc, st = eng.wait(t)
        for tk in pend.values():
            eng.wait(tk)
        say(f"  slide step {k + 1}: rc={rc} newton={st.newton_iters} (alone {ref[k][1]}) "
            f"other admissions so far {admitted_mid}")
        assert (rc, st.newton_iters, st.pcg_iters) == ref[k][:3]
        assert np.array_equal(g.x, ref[k][3])
    eng.close()
    assert admitted_mid >= steps


def test_broad_phase_failure_does_not_stick(ipc):
    sc = S.tiny_scene()
    fresh = ipc.GelScene(sc)
    rc0, _ = fresh.step()
    x_ref = fresh.x
    fresh.close()

    g = ipc.GelScene(sc)
    bad = np.full_like(g.x, np.nan)  # every box non-finite: the broad phase flags the scene
    g.x = bad
    with pytest.raises(ipc.IPCError) as e:
        g.step()
    assert e.value.code == ipc.IPC_E_INFEASIBLE
    g.reset()
    rc, _ = g.step()
    assert rc == rc0
    assert np.array_equal(g.x, x_ref)

    # the same through the engine: the failed scene's slot is reused by a healthy one
    h = ipc.GelScene(sc)
    h.x = bad
    eng = ipc.Batch()
    (t,) = eng.submit([h])
    with pytest.raises(ipc.IPCError) as e:
        eng.wait(t)
    assert e.value.code == ipc.IPC_E_INFEASIBLE
    h2 = ipc.GelScene(sc)
    (t,) = eng.submit([h2])
    rc, _ = eng.wait(t)
    assert rc == rc0
    assert np.array_equal(h2.x, x_ref)
    h.reset()
    (t,) = eng.submit([h])
    rc, _ = eng.wait(t)
    assert rc == rc0
    assert np.array_equal(h.x, x_ref)
    eng.close()


def test_state_blob_restores_case_pose(ipc):
    sc = S.attached_scene(grid=(8, 10, 3), steps=6, depth=0.6e-3, tilt_deg=3.0, radius=4e-3)
    a = ipc.GelScene(sc)
    for _ in range(3):
        a.step()
    blob = a.save_state()
    # the next step re-sends the indenter pose only: the case keeps its pose
    st = ipc.ipc_step_stats()
    r = ipc.req_of(sc.poses[4])  # case_pose_set = 0
    rc_a = ipc.lib().ipc_step(a.ptr, C.byref(r), C.byref(st))
    xa = a.x

    b = ipc.GelScene(sc)
    b.step(case_pose=S.pose_matrix(np.eye(3), np.array([0.0, 0.0, 2e-4])))  # a different case pose
    b.load_state(blob)
    rc_b = ipc.lib().ipc_step(b.ptr, C.byref(r), C.byref(st))
    say(f"  after load: rc {rc_b} (saved run {rc_a})")
    assert rc_b == rc_a
    assert np.array_equal(b.x, xa)
