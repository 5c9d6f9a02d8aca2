"""Writes the full-size oracle goldens (tests/golden/*.npz). Calls only the
oracle and the seeded scene generators; every stored value is the FP64
oracle's, at PCG tolerance 1e-12 (the parity setting).

  c2 SEED   config 2 (40x50x8 gel, 1.5 mm over 50 steps, dt 5e-3 s) from
            rest: c2_seed{SEED}_final.npz = gel positions after step 50; for
            seeds 0-2 also c2_seed{SEED}_tf.npz = a pressed state (the
            trajectory's state after step 25, positions and velocities
            rounded to float32 offsets: that rounded state is the input) and
            the oracle's first two Newton iterates of step 26 from it.
            About 2-3 h per seed on one core.
  c2gn SEED the same trajectory with the Gauss-Newton pair barrier Hessian
            (the oracle's barrier_hessian = 1): c2_seed{SEED}_gn_final.npz.
            Newton stops where the direction of that form is small, so its
            path through the non-convex steps is its own: the GPU's
            Gauss-Newton form is held to this trajectory.
  c3 I      scene I of the 256-scene uneven batch (seed 1000 + I), all 20
            steps: c3_{I}_final.npz = gel positions after step 20.
  c5        config 5 (80x100x16 gel, sphere r = 8 mm, friction mu = 0.5):
            the constructed pressed-and-sliding state of step 60
            (scenes.pressed_state: sphere 0.9 mm past first touch after 20
            slide steps, zero velocities, the same bits on every machine),
            the oracle's first Newton iterate of step 61 from it, friction
            lagged at that state: c5_tf.npz.

  hertz_curve  the Hertz check scene (30x30x15 mm block, 41x41x21 grid,
            sphere R = 20 mm, dhat = 10 um, quasi-static) pressed 0.5 mm in
            10 steps at PCG tolerance 1e-8: hertz_41x41x21_oracle.txt = per
            step the contact force, the support reaction, the targets' pull
            on the indenter, the surface depression on the axis and the
            descent past first touch.
  hertz_tf  the same scene's constructed pressed state of step 4
            (scenes.pressed_state, sphere 0.2 mm past first touch, gap
            0.9 dhat: the chords of the gel's top under the 20 mm sphere sag
            by up to 3.5 um) and the oracle's first Newton iterate of step 5 from it:
            hertz_tf.npz.

Offsets are stored as float32 (positions: offsets from the rest positions;
iterates: offsets from the iterate's input), so a stored iterate carries at
most 2^-24 of one Newton step of rounding (< 1e-10 L here). Positions of
the fixed-error goldens are float32 offsets from rest as well (rounding
< 1e-9 L against a 1e-4 L bound)."""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
from paper_2411_04776_amd import scenes as S  # noqa: E402


def rest_all(sc, step):
    return np.concatenate([sc.X, S.apply_pose(sc.poses[step], sc.Y)])


def f32_offset(x, ref):
    return (x - ref).astype(np.float32)


def log(*a):
    print(*a, flush=True)


def iterates(sc, x0, v0, step, count, **kw):
    """The oracle's first `count` Newton iterates of `step` from (x0, v0)."""
    o = O.OracleScene(sc, pcg_tol=1e-12, **kw)
    o.x = x0
    o.v = v0
    o.begin_step(sc.poses[step])
    xs = [x0]
    for k in range(count):
        t = time.time()
        r, xn, st = o.newton_iterate(xs[-1])
        log(f"  iterate {k + 1}: r={r} pcg={st.pcg_iters} active={st.n_active} alpha={st.alpha:.6f} "
            f"alpha_ccd={st.alpha_ccd:.6f} ({time.time() - t:.0f} s)")
        assert r == 0, "expected a Newton step"
        xs.append(xn)
    return xs


def c2(seed, gn=False):
    sc = S.config2(seed)
    o = O.OracleScene(sc, pcg_tol=1e-12, barrier_hessian=1 if gn else 0)
    t0 = time.time()
    n = len(sc.X)
    for k in range(1, sc.n_steps + 1):
        rc, st = o.step(sc.poses[k])
        log(f"c2 seed {seed} step {k}: rc={rc} newton={st.newton_iters} pcg={st.pcg_iters} "
            f"active={st.n_active} ({time.time() - t0:.0f} s)")
        if k == 25 and seed in (0, 1, 2) and not gn:
            ref = rest_all(sc, 25)
            dx = f32_offset(o.x, ref)
            dv = o.v.astype(np.float32)
            x0 = ref + dx.astype(np.float64)
            v0 = dv.astype(np.float64)
            xs = iterates(sc, x0, v0, 26, 2)
            np.savez_compressed(os.path.join(HERE, f"c2_seed{seed}_tf.npz"), step=26, dx=dx, dv=dv,
                                it1=f32_offset(xs[1], xs[0]), it2=f32_offset(xs[2], xs[1]),
                                L=sc.bbox_diag, name=sc.name)
    name = f"c2_seed{seed}_gn_final.npz" if gn else f"c2_seed{seed}_final.npz"
    np.savez_compressed(os.path.join(HERE, name), steps=sc.n_steps,
                        dx=f32_offset(o.x[:n], sc.X), L=sc.bbox_diag, name=sc.name)


def c3(i):
    sc = S.config3_scene(i)
    o = O.OracleScene(sc, pcg_tol=1e-12)
    t0 = time.time()
    n = len(sc.X)
    for k in range(1, sc.n_steps + 1):
        rc, st = o.step(sc.poses[k])
        log(f"c3 scene {i} step {k}: rc={rc} newton={st.newton_iters} pcg={st.pcg_iters} "
            f"active={st.n_active} ({time.time() - t0:.0f} s)")
    np.savez_compressed(os.path.join(HERE, f"c3_{i}_final.npz"), steps=sc.n_steps,
                        dx=f32_offset(o.x[:n], sc.X), L=sc.bbox_diag, name=sc.name)


def c5():
    sc = S.config5()
    x0, v0 = S.pressed_state(sc, 60)
    xs = iterates(sc, x0, v0, 61, 1)
    np.savez_compressed(os.path.join(HERE, "c5_tf.npz"), step=61, it1=f32_offset(xs[1], xs[0]),
                        L=sc.bbox_diag, name=sc.name)


def hertz_curve():
    sys.path.insert(0, os.path.dirname(HERE))
    import hertz as H
    sc = S.hertz_scene()
    o = O.OracleScene(sc, pcg_tol=1e-8)
    m = O.OracleScene(sc)
    t0 = time.time()
    rows = []
    for k in range(1, sc.n_steps + 1):
        rc, st = o.step(sc.poses[k])
        r = H.measure(sc, m, o.x, sc.poses[k])
        log(f"hertz step {k}: rc={rc} newton={st.newton_iters} pcg={st.pcg_iters} active={st.n_active} "
            f"{r} ({time.time() - t0:.0f} s)")
        rows.append((k, rc, st.newton_iters, r["F"], r["F_support"], r["F_target"], r["delta"], r["descent"]))
    with open(os.path.join(HERE, "hertz_41x41x21_oracle.txt"), "w") as f:
        f.write(f"# FP64 oracle, {sc.name}: 30x30x15 mm block, sphere R = 20 mm, dhat = 1e-5 m, kappa = 1e4,\n")
        f.write("# dt = 1 s, Newton tolerance 1e-8 m, PCG tolerance 1e-8; written by tests/golden/make_fullsize.py\n")
        f.write("# step status newton F_contact(N) F_support(N) F_target(N) delta_axis(m) descent_past_touch(m)\n")
        for row in rows:
            f.write(" ".join(repr(float(v)) if isinstance(v, float) else str(v) for v in row) + "\n")


def hertz_tf():
    sc = S.hertz_scene()
    x0, v0 = S.pressed_state(sc, 4, gap_frac=0.9)
    xs = iterates(sc, x0, v0, 5, 1)
    np.savez_compressed(os.path.join(HERE, "hertz_tf.npz"), step=5, it1=f32_offset(xs[1], xs[0]),
                        L=sc.bbox_diag, name=sc.name)


if __name__ == "__main__":
    what = sys.argv[1]
    if what == "c2":
        c2(int(sys.argv[2]))
    elif what == "c2gn":
        c2(int(sys.argv[2]), gn=True)
    elif what == "c3":
        c3(int(sys.argv[2]))
    elif what == "c5":
        c5()
    elif what == "hertz_curve":
        hertz_curve()
    elif what == "hertz_tf":
        hertz_tf()
    else:
        raise SystemExit(__doc__)
