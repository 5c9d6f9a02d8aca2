"""Autotuner of the library's launch and grouping choices, per size class.

The library reads its choices from tuning.json beside libipcgel.so when a
scene is created (or from $IPC_TUNING_FILE): per size class (scenes of at
least min_verts vertices) the SpMV form (one thread per matrix row for lists
of at least spmv_one_lane_rows rows, else two lanes per row), the packing
target of the multilevel preconditioner's groups (members per block of the
update kernel), and the PCG chunk lengths (launches between two reads of the
per-scene convergence flags: the first chunk a fraction of the previous
solve's iteration count, later ones another fraction of the remaining
count; in a list, of a quantile of its scenes' counts).

This script measures them on the GPU: for each class a representative
workload (small: a list of uneven config-3 scenes through the batching
engine; large: an 80x100x16 scene of the serving mix), mixed precision, a
warm-up step, a reset to rest, a few untimed steps and the timed middle
of the episode; coordinate descent
over the candidate values (two sweeps, each measurement the best of two
runs), env-steps/s as the objective. It writes the chosen values and every
measurement to tuning.json.

  python -m paper_2411_04776_amd.autotune [--out PATH] [--small-scenes N]
"""
from __future__ import annotations

import argparse
import json
import os
import tempfile
import time

import numpy as np

from . import ipc, scenes

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(HERE, "tuning.json")

SPACE = {
    "spmv_one_lane_rows": [0, 1 << 40],          # always one thread per row / always two lanes per row
    "mas_target": [64, 128, 192, 256],
    "pcg_first_chunk": [0.5, 0.75, 0.875, 1.0],
    "pcg_later_chunk": [0.125, 0.25, 0.5],
    "pcg_list_quantile": [0.0, 0.1, 0.25, 0.5, 1.0],
}
DEFAULTS = {"spmv_one_lane_rows": 65536, "mas_target": 256, "pcg_first_chunk": 0.875, "pcg_later_chunk": 0.25,
            "pcg_list_quantile": 0.25}


def _workload(name, small_scenes):
    """Scenes, untimed steps after the reset, timed steps (the middle of the
    20-step episode, where contact builds up)."""
    if name == "small":
        return [scenes.config3_scene(i, steps=20) for i in range(small_scenes)], 6, 8
    return [scenes.serving_scene(9, large=True)], 6, 6


def _write(path, classes):
    with open(path, "w") as f:
        json.dump({"classes": classes}, f)


def measure(name, small_scenes, classes, tmp, pcg_tol=3e-5):
    """env-steps/s of the class's workload with the given class table."""
    import torch
    _write(tmp, classes)
    os.environ["IPC_TUNING_FILE"] = tmp
    scs, warm, timed = _workload(name, small_scenes)
    rt = ipc.TorchRuntime()
    gs = [ipc.GelScene(sc, runtime=rt, precision=ipc.IPC_MIXED, pcg_tol=pcg_tol) for sc in scs]
    eng = ipc.Batch()

    def list_step():
        for t in eng.submit(gs):
            rc, _ = eng.wait(t)
            if rc < 0:
                raise RuntimeError(f"step failed: {rc}")

    list_step()   # contact set-up and buffer growth
    for g in gs:
        g.reset()
    for _ in range(warm):
        list_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(timed):
        list_step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    eng.close()
    for g in gs:
        g.close()
    return timed * len(gs) / el


def tune(out=DEFAULT_OUT, small_scenes=128, sweeps=2, reps=2, log=print):
    import torch
    torch.cuda.set_device(0)
    classes = [dict(min_verts=0, name="small", **DEFAULTS),
               dict(min_verts=ipc.IPC_BATCH_LARGE_VERTS, name="large", **DEFAULTS)]
    records = []
    fd, tmp = tempfile.mkstemp(suffix=".json")
    os.close(fd)
    try:
        for ci, cls in enumerate(classes):
            name = cls["name"]
            best = measure(name, small_scenes, classes, tmp)
            records.append({"class": name, "params": {k: cls[k] for k in SPACE}, "env_steps_per_s": best})
            log(f"{name}: start {best:.1f} env-steps/s with {dict((k, cls[k]) for k in SPACE)}")
            for sweep in range(sweeps):
                for key, values in SPACE.items():
                    for v in values:
                        if v == classes[ci][key]:
                            continue
                        trial = [dict(c) for c in classes]
                        trial[ci][key] = v
                        r = max(measure(name, small_scenes, trial, tmp) for _ in range(reps))
                        records.append({"class": name, "params": {k: trial[ci][k] for k in SPACE},
                                        "env_steps_per_s": r})
                        log(f"{name}: sweep {sweep + 1} {key}={v}: {r:.1f} env-steps/s (best {best:.1f})")
                        if r > best * 1.01:  # a change must beat the noise
                            best = r
                            classes = trial
            log(f"{name}: chosen {dict((k, classes[ci][k]) for k in SPACE)} at {best:.1f} env-steps/s")
    finally:
        os.environ.pop("IPC_TUNING_FILE", None)
        os.unlink(tmp)
    doc = {"classes": classes,
           "device": __import__("torch").cuda.get_device_name(0),
           "objective": "env-steps/s, mixed precision, PCG tolerance 3e-5; small: a list of "
                        f"{small_scenes} config-3 scenes through the batching engine (steps 7-14 of the episode); "
                        "large: one 80x100x16 serving scene (steps 7-12); best of two runs",
           "measurements": records}
    with open(out, "w") as f:
        json.dump(doc, f, indent=1)
    log(f"wrote {out}")
    return doc


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--small-scenes", type=int, default=128)
    ap.add_argument("--sweeps", type=int, default=2)
    args = ap.parse_args()
    tune(args.out, args.small_scenes, args.sweeps, log=lambda *a: print(*a, flush=True))


if __name__ == "__main__":
    main()
