#!/usr/bin/env python3
"""Benchmark of the IPC gel-pad step on one MI355X.

Workload: the larger single-scene configuration -- a 40x50x8 vertex gel
(16,000 vertices, 80,262 tets) over a 20x25x4 mm box, bottom face fixed,
pressed 1.5 mm over 50 steps (dt = 5e-3 s) by the seed's indenter (seed 0:
a capped cylinder), plain FP64. A "step" is one ipc_step: the whole Newton
solve of one time step (candidates, distances, barrier, elasticity, PCG,
CCD, line search). Inputs are resident in HBM before the timed region.

Prints one JSON line: env-steps/s (value), Newton iters/s, p50/p99 step
latency, the roofline of the dominant kernel (PCG SpMV) from HIP events on
the library's stream, and the FP64 CPU oracle timed on a bounded sample.
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


PCG_SOURCES = ("paper_2411_04776_amd/csrc/k_solver.hip", "paper_2411_04776_amd/csrc/incidence.h",
               "paper_2411_04776_amd/csrc/device_util.h", "paper_2411_04776_amd/csrc/ipc_internal.h")
TRAFFIC_PROFILES = {"k_pcg_A": "profiles/k_pcg_A_c2_fp64_pmc.md", "k_pcg_B": "profiles/k_pcg_B_c2_fp64_pmc.md"}


def precond_code(args):
    from paper_2411_04776_amd import ipc
    return ipc.IPC_PRECOND_JACOBI if args.precond == "jacobi" else ipc.IPC_PRECOND_MULTILEVEL


def barrier_code(args):
    from paper_2411_04776_amd import ipc
    return ipc.IPC_BARRIER_GAUSS_NEWTON if args.barrier_hessian == "gauss-newton" else ipc.IPC_BARRIER_PROJECTED


def pcg_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in PCG_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of a PCG kernel from the committed rocprofv3 --pmc
    summary (FETCH_SIZE and WRITE_SIZE scaled by a copy kernel of known size),
    or None when the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, TRAFFIC_PROFILES[kernel])
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and line.strip().startswith(("traffic_bytes_per_launch", "kernel_source_sha256")):
                k, v = line.strip().split(":", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel_source_sha256") != pcg_source_hash():
        return None
    try:
        return int(float(vals["traffic_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def update_bytes_per_launch(info, n_active, members):
    """Algorithmic bytes of one PCG update launch (k_pcg_B, FP64): per vertex
    q, d, p, r and the 3x3 inverse read (21 values) and p, r, z written (9),
    per incidence entry (4 per active pair) its index and 3 pair-product
    values, per preconditioner member its vertex id and three level ids, and
    the SpMV blocks' d.q partials once."""
    n = info["n"]
    return 240 * n + 28 * 4 * n_active + 16 * members + 8 * ((n + 63) // 64)


def spmv_bytes_per_launch(info, n_active):
    """Algorithmic bytes of one PCG SpMV launch (FP64): each stored 3x3 block
    (72 B values + 4 B column) once, per vertex the z and d gathers and the d,
    q writes (4 x 24 B) plus its row pointers, and per active contact pair the
    off-diagonal 3x3 blocks of its 4 rows (108 doubles) and vertex ids."""
    n = info["n"]
    return 76 * info["nnzb"] + 100 * n + 880 * n_active


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--seed", type=int, default=0)
    # PCG tolerance of the timed runs: the loosest that keeps the final error of
    # config 2 far inside 1e-4 L (tests/test_gpu_fixed_error.py: 8e-6 L)
    ap.add_argument("--pcg-tol", type=float, default=1e-3)
    ap.add_argument("--precond", choices=["multilevel", "jacobi"], default="multilevel",
                    help="PCG preconditioner: additive multilevel aggregates or block-Jacobi")
    ap.add_argument("--barrier-hessian", choices=["projected", "gauss-newton"], default="projected",
                    help="pair barrier Hessian: PSD-projected exact Hessian or the Gauss-Newton form")
    ap.add_argument("--cpu-budget", type=float, default=20.0, help="seconds of oracle work for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch", type=int, default=256, help="scenes of the batched uneven-scene leg (0: skip)")
    ap.add_argument("--batch-steps", type=int, default=4)
    ap.add_argument("--serve", type=int, default=64, help="environments of the serving leg (0: skip)")
    ap.add_argument("--no-soft-ball", action="store_true", help="skip the soft-ball leg")
    ap.add_argument("--serve-requests", type=int, default=400)
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="only copy a buffer of this many MiB with torch (HBM counter calibration) and exit")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU: the library has no multi-GPU path (scenes are independent and "
              "would shard across GPUs without communication). Use --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.warmup + args.steps > 50:
        print("warmup + steps must fit the 50-step trajectory", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2411_04776_amd import ipc, scenes

    torch.cuda.set_device(0)
    if args.copy_probe_mb:
        n = args.copy_probe_mb << 20
        a = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": n, "copy_probe_bytes_written": n}), flush=True)
        return
    sc = scenes.config2(args.seed)
    g = ipc.GelScene(sc, precision=ipc.IPC_FP64, pcg_tol=args.pcg_tol, precond=precond_code(args),
                     barrier_hessian=barrier_code(args))
    for _ in range(args.warmup):
        rc, st = g.step()
        print(f"warmup step {g.step_index}: rc={rc} newton={st.newton_iters} pcg={st.pcg_iters} "
              f"ms={st.ms_total:.1f}", file=sys.stderr, flush=True)
    x_start, v_start = g.x, g.v
    g.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat, newton, pcg, active = [], 0, 0, []
    for _ in range(args.steps):
        rc, st = g.step()
        lat.append(st.ms_total)
        newton += st.newton_iters
        pcg += st.pcg_iters
        active.append(st.n_active)
        print(f"step {g.step_index}: rc={rc} newton={st.newton_iters} pcg={st.pcg_iters} "
              f"active={st.n_active} alpha_ccd={st.alpha_ccd:.3g} halvings={st.ls_halvings} "
              f"ms={st.ms_total:.1f}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    prof = g.profile_read()
    info = g.matrix_info()
    g.profile(False)

    # the two PCG kernels (the dominant launches): achieved = algorithmic
    # bytes per launch / mean event-timed launch duration
    n_act_mean = float(np.mean(active)) if active else 0.0
    members = g.precond_info()["members"]
    pcg_k = {}
    for cls, kname, what, nbytes in (
            ("pcg_spmv", "k_pcg_A", "PCG SpMV + direction update", spmv_bytes_per_launch(info, n_act_mean)),
            ("pcg_update", "k_pcg_B", "PCG update + multilevel preconditioner", update_bytes_per_launch(info, n_act_mean, members))):
        n_launch, ms = prof[cls]
        avg_s = ms / 1e3 / max(n_launch, 1)
        achieved = nbytes / avg_s / 1e9 if avg_s > 0 else 0.0
        pcg_k[kname] = {
            "kernel": f"{kname} ({what})", "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(kname),
            "traffic_source": TRAFFIC_PROFILES[kname], "bytes_per_launch": int(nbytes), "timed_launches": int(n_launch),
            "timing": "HIP events around 1 in 16 launches in the timed region", "avg_launch_us": round(avg_s * 1e6, 3),
            "event_ms": round(ms, 3)}
    dom_k = max(pcg_k, key=lambda k: pcg_k[k]["event_ms"])
    other = [k for k in pcg_k if k != dom_k][0]
    roofline = dict(pcg_k[dom_k])
    # PCG classes time one launch in sixteen: scale them to all pcg iterations
    est = {k: v[1] for k, v in prof.items()}
    for cls in ("pcg_spmv", "pcg_update"):
        if prof[cls][0] > 0:
            est[cls] = prof[cls][1] / prof[cls][0] * pcg
    roofline["share_of_event_time"] = {k: round(v / max(sum(est.values()), 1e-12), 4) for k, v in est.items()}
    roofline["dominant_by_event_time"] = max(est, key=est.get)
    roofline["other_pcg_kernel"] = pcg_k[other]
    roofline["note"] = ("one 16k-vertex scene is latency-bound (a chain of dependent loads and block barriers per "
                        "launch, ~250 blocks for 256 CUs); the batch leg's pcg_spmv_roofline is the bandwidth case")

    line = {
        "metric": "env-steps/sec", "value": round(args.steps / elapsed, 4), "unit": "env-steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "newton_iters_per_sec": round(newton / elapsed, 3),
        "pcg_iters_per_newton": round(pcg / max(newton, 1), 1),
        "latency_ms": {"p50": round(statistics.median(lat), 3),
                       "p99": round(float(np.percentile(lat, 99)), 3)},
        "config": {"workload": f"40x50x8 gel (16000 v, 80262 tets), {sc.meta['kind']} indenter seed "
                               f"{args.seed}, 1.5 mm over 50 steps, dt 5e-3 s, FP64, steps "
                               f"{args.warmup + 1}-{args.warmup + args.steps}",
                   "precision": "fp64", "pcg_tol": args.pcg_tol, "precond": args.precond,
                   "barrier_hessian": args.barrier_hessian, "newton_tol_m": sc.newton_tol,
                   "dhat_m": sc.dhat, "kappa": sc.kappa},
        "roofline": roofline,
    }

    g.close()
    if args.batch > 0:
        line["batch"] = batch_leg(args, ipc, scenes, torch)
    if args.serve > 0:
        line["serving"] = serving_leg(args, ipc, torch)
    if not args.no_soft_ball:
        line["soft_ball"] = soft_ball_leg(args, ipc, scenes, torch)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(sc, x_start, v_start, args, newton / args.steps)

    print(json.dumps(line), flush=True)


def batch_leg(args, ipc, scenes, torch):
    """Uneven scenes (grid U{12..40}xU{15..50}xU{3..8}, random indenters)
    stepped together through the continuous-batching engine, mixed precision:
    every Newton phase is one launch for the whole list. Also the same first
    16 scenes stepped one at a time (ipc_step) for the batching gain."""
    rt = ipc.TorchRuntime()
    t0 = time.perf_counter()
    scs = [scenes.config3_scene(i) for i in range(args.batch)]
    gs = [ipc.GelScene(sc, runtime=rt, precision=ipc.IPC_MIXED, pcg_tol=args.pcg_tol,
                         precond=precond_code(args), barrier_hessian=barrier_code(args)) for sc in scs]
    build_s = time.perf_counter() - t0
    nv = sum(len(sc.X) for sc in scs)
    nt = sum(len(sc.T) for sc in scs)
    eng = ipc.Batch()

    def list_step():
        tks = eng.submit(gs)
        newton = 0
        for t in tks:
            rc, st = eng.wait(t)
            if rc < 0:
                raise RuntimeError(f"batched step failed: {rc}")
            newton += st.newton_iters
        return newton

    list_step()  # warm-up: first contact, buffer growth
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    newton = 0
    for _ in range(args.batch_steps):
        newton += list_step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    # one more list step with the engine's HIP-event timing of the SpMV (kernel
    # class 0): achieved = algorithmic bytes of the timed launches / their time
    eng.profile(True)
    list_step()
    n_a, ms_a, by_a = eng.profile_read(0)
    eng.profile(False)
    eng.close()
    spmv = None
    if n_a and ms_a > 0:
        gbs = by_a / (ms_a * 1e-3) / 1e9
        spmv = {"kernel": "k_pcg_A over the list (PCG SpMV + direction update)", "bound": "hbm",
                "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                "timed_launches": n_a, "avg_launch_us": round(1e3 * ms_a / n_a, 2),
                "bytes_per_launch": int(by_a / n_a),
                "timing": "engine HIP events around 1 in 16 launches of one list step"}
    # the same scenes one at a time, from the same states
    k = min(16, len(gs))
    states = [g.save_state() for g in gs[:k]]
    t0 = time.perf_counter()
    alone_steps = 0
    for g in gs[:k]:
        for _ in range(args.batch_steps):
            g.step()
            alone_steps += 1
    torch.cuda.synchronize()
    el_alone = time.perf_counter() - t0
    for g, b in zip(gs[:k], states):
        g.load_state(b)
    for g in gs:
        g.close()
    steps = args.batch_steps * len(gs)
    print(f"batch leg: {len(gs)} scenes, {steps} env-steps in {el:.2f} s", file=sys.stderr, flush=True)
    return {"workload": f"{len(gs)} uneven scenes ({nv} v, {nt} tets in total), seeds 1000-{999 + len(gs)}, "
                        f"steps 2-{1 + args.batch_steps}, mixed precision, continuous-batching engine",
            "env_steps_per_s": round(steps / el, 2), "newton_iters_per_s": round(newton / el, 1),
            "ms_per_list_step": round(1e3 * el / args.batch_steps, 2), "scene_build_s": round(build_s, 2),
            "alone_env_steps_per_s": round(alone_steps / el_alone, 2), "alone_scenes": k,
            "pcg_spmv_roofline": spmv}


# GIPC ms per frame of the paper's timing table (soft ball, RTX 3080 Ti; context only)
PAPER_SOFT_BALL_MS = {"small": 24.95, "medium": 110.47, "large": 221.61}


def soft_ball_leg(args, ipc, scenes, torch):
    """Gel pad + soft ball squeezed by a rigid plate at the three mesh sizes
    of the paper's GIPC timing table (gel + ball vertex/tet counts), FP64,
    20 steps each after one untimed step, with both pair-Hessian forms (the
    projected one and the Gauss-Newton one GIPC uses); ms per step beside the
    paper's per-frame times on its own hardware (a different scene: context)."""
    out = {}
    forms = (("projected", ipc.IPC_BARRIER_PROJECTED), ("gauss_newton", ipc.IPC_BARRIER_GAUSS_NEWTON))
    for size in ("small", "medium", "large"):
        sc = scenes.soft_ball_scene(size, steps=21)
        out[size] = {"verts": len(sc.X), "tets": len(sc.T), "pcg_tol": min(args.pcg_tol, 1e-4),
                     "paper_gipc_ms_per_frame": PAPER_SOFT_BALL_MS[size]}
        for name, code in forms:
            # the floating ball's near-rigid modes make Newton sensitive to inexact
            # steps: this leg solves PCG to 1e-4 (fewer Newton iterations than 1e-3)
            g = ipc.GelScene(sc, precision=ipc.IPC_FP64, pcg_tol=min(args.pcg_tol, 1e-4), precond=precond_code(args),
                             barrier_hessian=code)
            g.step()
            torch.cuda.synchronize()
            newton, pcg, t = 0, 0, []
            for _ in range(sc.n_steps - 1):
                t0 = time.perf_counter()
                rc, st = g.step()
                t.append(time.perf_counter() - t0)
                newton += st.newton_iters
                pcg += st.pcg_iters
            g.close()
            out[size][name] = {"ms_per_step": round(1e3 * sum(t) / len(t), 2),
                               "p99_ms": round(1e3 * sorted(t)[int(0.99 * (len(t) - 1))], 2),
                               "newton_per_step": round(newton / len(t), 2),
                               "pcg_per_newton": round(pcg / max(newton, 1), 1)}
        print(f"soft ball {size}: {out[size]}", file=sys.stderr, flush=True)
    return out


def serving_leg(args, ipc, torch):
    """Request loop: Poisson arrivals over environments whose scenes stay
    resident in HBM, at most one request in flight per environment, each
    handed to the continuous-batching engine; latency = completion - arrival."""
    from paper_2411_04776_amd import serve
    envs = serve.serving_envs(args.serve, large_frac=0.0)
    srv = serve.Server(envs, precision=ipc.IPC_MIXED, pcg_tol=args.pcg_tol, precond=precond_code(args))
    # warm every scene once (contact set-up, buffer growth), then the closed-loop
    # capacity with every environment in flight; the open loop offers 70% of it
    def closed_round():
        tks = srv.engine.submit(srv.envs, [srv.next_pose(g) for g in srv.envs])
        for t in tks:
            srv.engine.wait(t)

    closed_round()
    t0 = time.perf_counter()
    for _ in range(2):
        closed_round()
    capacity = 2 * len(srv.envs) / (time.perf_counter() - t0)
    rate = 0.7 * capacity
    res = srv.run(rate_hz=rate, n_requests=args.serve_requests, seed=7, time_limit_s=60.0)
    srv.close()
    return {"workload": f"{args.serve} environments (uneven scenes, seeds 5000-{4999 + args.serve}), "
                        f"Poisson arrivals at {rate:.0f} req/s, mixed precision",
            "closed_loop_env_steps_per_s": round(capacity, 2),
            "completed": res.completed, "env_steps_per_s": round(res.env_steps_per_s, 2),
            "newton_iters_per_s": round(res.newton_iters_per_s, 1),
            "latency_ms": {"p50": round(res.latency_ms_p50, 2), "p99": round(res.latency_ms_p99, 2)},
            "admitted": res.admitted, "refused": res.refused, "footprint_gib": round(res.footprint_gb, 3),
            "statuses": {str(k): v for k, v in res.statuses.items()}}


def cpu_baseline(sc, x0, v0, args, newton_per_step):
    """FP64 oracle, single thread, teacher-forced from the GPU state at the
    start of the timed region: Newton iterations of the first timed step until
    the budget is spent; env-steps/s = (Newton iters/s) / (Newton iters per
    step measured on the GPU for the same steps)."""
    import oracle
    o = oracle.OracleScene(sc, pcg_tol=args.pcg_tol)
    o.x = x0
    o.v = v0
    o.begin_step(sc.poses[args.warmup + 1])
    x = x0
    t0 = time.perf_counter()
    iters = 0
    while True:
        r, xn, st = o.newton_iterate(x)
        iters += 1
        x = xn
        if r != 0 or time.perf_counter() - t0 > args.cpu_budget:
            break
    dt = time.perf_counter() - t0
    it_per_s = iters / dt
    return {"value": round(it_per_s / max(newton_per_step, 1e-9), 6), "unit": "env-steps/s", "cores": 1,
            "kind": "oracle",
            "newton_iters_per_sec": round(it_per_s, 4),
            "sample": f"{iters} oracle Newton iterations ({dt:.1f} s) of step {args.warmup + 1} from the GPU "
                      f"state, scaled by {newton_per_step:.2f} Newton iterations per step"}


if __name__ == "__main__":
    main()
