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
    ap.add_argument("--pcg-tol", type=float, default=1e-4)
    ap.add_argument("--cpu-budget", type=float, default=20.0, help="seconds of oracle work for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU: this build has no multi-GPU path (scenes shard across GPUs "
              "without communication; see DESIGN.md). Use --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.warmup + args.steps > 50:
        print("warmup + steps must fit the 50-step trajectory", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2411_04776_amd import ipc, scenes

    torch.cuda.set_device(0)
    sc = scenes.config2(args.seed)
    g = ipc.GelScene(sc, precision=ipc.IPC_FP64, pcg_tol=args.pcg_tol)
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
              f"active={st.n_active} ms={st.ms_total:.1f}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    prof = g.profile_read()
    info = g.matrix_info()
    g.profile(False)

    # dominant kernel: the one with the largest summed event time
    dom = max(prof, key=lambda k: prof[k][1])
    n_launch, ms = prof["pcg_spmv"]
    avg_s = ms / 1e3 / max(n_launch, 1)
    n_act_mean = float(np.mean(active)) if active else 0.0
    bytes_launch = spmv_bytes_per_launch(info, n_act_mean)
    achieved = bytes_launch / avg_s / 1e9 if avg_s > 0 else 0.0
    roofline = {
        "kernel": "k_pcg_A (PCG SpMV + direction update)",
        "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
        "bytes_per_launch": int(bytes_launch), "timed_launches": int(n_launch), "timing": "HIP events around 1 in 4 launches in the timed region",
        "avg_launch_us": round(avg_s * 1e6, 3),
        "share_of_event_time": {k: round(v[1] / max(sum(w[1] for w in prof.values()), 1e-12), 4)
                                for k, v in prof.items()},
        "dominant_by_event_time": dom,
    }

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
                   "precision": "fp64", "pcg_tol": args.pcg_tol, "newton_tol_m": sc.newton_tol,
                   "dhat_m": sc.dhat, "kappa": sc.kappa},
        "roofline": roofline,
    }

    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(sc, x_start, v_start, args, newton / args.steps)

    print(json.dumps(line), flush=True)


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
