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

The loop itself only generates arrivals and collects completions; all
stepping runs in the native engine (ipc_batch_submit / ipc_batch_poll).
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np

from . import ipc, scenes


@dataclasses.dataclass
class ServeResult:
    completed: int
    wall_s: float
    env_steps_per_s: float
    newton_iters_per_s: float
    latency_ms_p50: float
    latency_ms_p99: float
    admitted: int
    refused: int
    footprint_gb: float
    statuses: dict


def footprint(scene, precision) -> int:
    d = ipc.make_desc(scene, precision=precision, keep=[])
    return int(ipc.lib().ipc_scene_footprint_bytes(d))


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
        self.engine = ipc.Batch()

    def next_pose(self, g):
        """Episode motion: the scene's trajectory, then reset and start over."""
        if g.step_index >= g.scene.n_steps:
            g.reset()
        return g.scene.poses[g.step_index + 1]

    def run(self, rate_hz: float, n_requests: int, seed: int = 7, time_limit_s: float = 60.0) -> ServeResult:
        rng = np.random.default_rng(seed)
        n = len(self.envs)
        busy = [None] * n          # (ticket, arrival time) of the env's request in flight
        waiting = []               # arrivals whose env was busy: (arrival, env)
        lat, newton, statuses = [], 0, {}
        t0 = time.perf_counter()
        next_arrival = t0 + rng.exponential(1.0 / rate_hz)
        issued = done = 0
        while done < n_requests:
            now = time.perf_counter()
            if now - t0 > time_limit_s:
                break
            while issued < n_requests and next_arrival <= now:
                waiting.append((next_arrival, int(rng.integers(0, n))))
                issued += 1
                next_arrival += rng.exponential(1.0 / rate_hz)
            # hand arrivals to idle environments, oldest first
            still = []
            for arr, e in waiting:
                if busy[e] is None:
                    g = self.envs[e]
                    pose = self.next_pose(g)
                    busy[e] = (self.engine.submit([g], [pose])[0], arr)
                else:
                    still.append((arr, e))
            waiting = still
            for e in range(n):
                if busy[e] is None:
                    continue
                fin, _ = self.engine.poll(busy[e][0])
                if fin:
                    rc, st = self.engine.wait(busy[e][0])
                    lat.append(time.perf_counter() - busy[e][1])
                    newton += st.newton_iters
                    statuses[rc] = statuses.get(rc, 0) + 1
                    busy[e] = None
                    done += 1
            time.sleep(0.0002)
        for e in range(n):  # drain
            if busy[e] is not None:
                rc, st = self.engine.wait(busy[e][0])
        wall = time.perf_counter() - t0
        lat_ms = np.array(lat) * 1e3 if lat else np.array([np.nan])
        return ServeResult(done, wall, done / wall, newton / wall, float(np.percentile(lat_ms, 50)),
                           float(np.percentile(lat_ms, 99)), len(self.envs), self.refused,
                           self.footprint / 2 ** 30, statuses)

    def close(self):
        self.engine.close()
        for g in self.envs:
            g.close()


def serving_envs(n_envs: int, large_frac: float = 0.1):
    """Environment scenes: the uneven batch distribution, every
    round(1/large_frac)-th environment at 80x100x16 (env i uses seed 5000 + i)."""
    every = int(round(1.0 / large_frac)) if large_frac > 0 else 0
    return [scenes.serving_scene(i, large=bool(every) and i % every == every - 1) for i in range(n_envs)]
