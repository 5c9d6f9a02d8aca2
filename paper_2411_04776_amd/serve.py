"""Serving loop: ipc_step requests from many environments, as they arrive.

Every environment owns one scene whose state stays resident in HBM between
its steps. A scene is admitted (created on the device) only while the summed
footprint of the admitted scenes (ipc_scene_footprint_bytes) fits the
memory budget; environments that do not fit are refused at start-up. Requests
arrive as a Poisson process over the admitted environments, at most one in
flight per environment; each one is handed to the library's
continuous-batching engine, which runs every in-flight step in shared
launches and takes new steps in at each Newton-iteration boundary. Latency of
a request = completion time - arrival time.

The loop itself only generates arrivals and collects completions (the
engine's wait-any, ipc_batch_next, so one thread serves every environment);
all stepping runs in the native engine, whose size classes step the large
scenes in a list and on a stream of their own.
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np

from . import ipc, scenes


LARGE_VERTS = ipc.IPC_BATCH_LARGE_VERTS   # the engine's size classes


@dataclasses.dataclass
class ServeResult:
    completed: int          # requests completed within the arrival window
    wall_s: float           # the arrival window
    env_steps_per_s: float  # completions per second within the window
    newton_iters_per_s: float
    latency_ms_p50: float   # of the requests completed within the window
    latency_ms_p99: float
    admitted: int
    refused: int
    footprint_gb: float
    statuses: dict
    by_class: dict          # "small" / "large": completed, p50, p99 (ms)
    offered_hz: float
    arrived: int            # requests that arrived within the window
    backlog: int            # of them, not completed by its end (in flight or waiting)


def footprint(scene, precision) -> int:
    d = ipc.make_desc(scene, precision=precision, keep=[])
    return int(ipc.lib().ipc_scene_footprint_bytes(d))


def _pct(v, q):
    return float(np.percentile(np.asarray(v) * 1e3, q)) if len(v) else float("nan")


class Server:
    """Admitted environments and the engine that steps them."""

    def __init__(self, env_scenes, precision=ipc.IPC_MIXED, pcg_tol=1e-5, precond=ipc.IPC_PRECOND_MULTILEVEL,
                 mem_budget_bytes=200 << 30, runtime=None):
        self.precision = precision
        self.envs = []
        self.refused = 0
        used = 0
        rt = runtime or ipc.TorchRuntime()
        for sc in env_scenes:
            need = footprint(sc, precision)
            if used + need > mem_budget_bytes:
                self.refused += 1
                continue
            self.envs.append(ipc.GelScene(sc, runtime=rt, precision=precision, pcg_tol=pcg_tol, precond=precond))
            used += need
        self.footprint = used
        self.large = [g.n >= LARGE_VERTS for g in self.envs]
        self.engine = ipc.Batch()

    def next_pose(self, g):
        """Episode motion: the scene's trajectory, then reset and start over."""
        if g.step_index >= g.scene.n_steps:
            g.reset()
        return g.scene.poses[g.step_index + 1]

    def run(self, rate_hz: float, duration_s: float = 8.0, seed: int = 7) -> ServeResult:
        """Poisson arrivals at rate_hz over the environments (uniformly) for
        duration_s, at most one request in flight per environment (a request
        for a busy environment waits for it); every due arrival is submitted
        in one call and completions are taken with the engine's wait-any.
        Throughput and latency are those of the requests completed within
        the window (steady state: above capacity the backlog grows and
        latency with it); afterwards the requests in flight are drained and
        the waiting ones dropped."""
        rng = np.random.default_rng(seed)
        n = len(self.envs)
        busy = [False] * n
        waiting = [[] for _ in range(n)]   # arrival times of requests for a busy environment
        owner = {}                         # ticket -> (env, arrival)
        lat = {False: [], True: []}
        newton, statuses = 0, {}
        t0 = time.perf_counter()
        t_end = t0 + duration_s
        next_arrival = t0 + rng.exponential(1.0 / rate_hz)
        arrived = done = 0

        def submit(items):
            gs = [self.envs[e] for e, _ in items]
            tks = self.engine.submit(gs, [self.next_pose(g) for g in gs])
            for (e, arr), t in zip(items, tks):
                owner[t] = (e, arr)

        while True:
            now = time.perf_counter()
            if now >= t_end:
                break
            due = []
            while next_arrival <= now and next_arrival < t_end:
                e = int(rng.integers(0, n))
                if busy[e]:
                    waiting[e].append(next_arrival)
                else:
                    busy[e] = True
                    due.append((e, next_arrival))
                arrived += 1
                next_arrival += rng.exponential(1.0 / rate_hz)
            if due:
                submit(due)
            timeout = max(0.0, min(next_arrival, t_end) - time.perf_counter()) * 1e3
            if not owner:
                time.sleep(timeout / 1e3)
                continue
            r = self.engine.next(timeout)
            follow = []
            while r is not None:
                t, rc, st = r
                e, arr = owner.pop(t)
                fin = time.perf_counter()
                if fin <= t_end:
                    lat[self.large[e]].append(fin - arr)
                    newton += st.newton_iters
                    statuses[rc] = statuses.get(rc, 0) + 1
                    done += 1
                if waiting[e] and fin < t_end:
                    follow.append((e, waiting[e].pop(0)))
                else:
                    busy[e] = False
                r = self.engine.next(0.0) if owner else None
            if follow:
                submit(follow)
        wall = time.perf_counter() - t0
        backlog = len(owner) + sum(len(w) for w in waiting)
        while owner:  # drain the requests in flight (not counted)
            r = self.engine.next(-1.0)
            owner.pop(r[0], None)
        allv = lat[False] + lat[True]
        by = {name: {"completed": len(lat[k]), "p50_ms": round(_pct(lat[k], 50), 3),
                     "p99_ms": round(_pct(lat[k], 99), 3)}
              for name, k in (("small", False), ("large", True)) if lat[k]}
        return ServeResult(done, wall, done / wall, newton / wall, _pct(allv, 50), _pct(allv, 99), len(self.envs),
                           self.refused, self.footprint / 2 ** 30, statuses, by, rate_hz, arrived, backlog)

    def close(self):
        self.engine.close()
        for g in self.envs:
            g.close()


def serving_envs(n_envs: int, large_frac: float = 0.1):
    """Environment scenes: the uneven batch distribution, every
    round(1/large_frac)-th environment at 80x100x16 (env i uses seed 5000 + i)."""
    every = int(round(1.0 / large_frac)) if large_frac > 0 else 0
    return [scenes.serving_scene(i, large=bool(every) and i % every == every - 1) for i in range(n_envs)]
