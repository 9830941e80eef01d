"""Serving loop over libsf: scenes arrive as requests, are admitted while their
device footprint fits a budget, advance together, and leave when evacuated
or after a tick limit.

Continuous batching: every iteration runs one batched tick (sf_batch_step)
over all resident scenes; requests that arrived meanwhile are admitted
between iterations as memory and slots free up, and a changed membership
builds a new batch (the scenes' device state stays where it is).  Scene
state never leaves the device between ticks.  All arithmetic runs in the HIP
library; this module only schedules.

Building a scene (validation, static fields) takes milliseconds.  By default
admitted scenes are built one after another on a worker thread, on a stream
of their own, while the resident scenes keep ticking (the library's calls
release the interpreter lock); a scene joins the batch at the first tick
after its build completes, and scenes being built hold their memory and
slot from the moment of admission.  With `background_builds=False` the
builds run between ticks instead, at most `max_admit_per_tick` of them
between two ticks.

The per-tick latency a resident scene sees is the wall time between two of
its ticks (admissions and retirements included).
"""
from __future__ import annotations

import collections
import dataclasses
import queue as _queue
import threading
import time
from typing import Callable, List, Optional

import numpy as np

from . import sf

# Device bytes a resident scene holds (the library's per-scene arrays):
# per su  D (4 B), exit mask (1), the claim record (claim word, registration
# count, padding: 16), occupancy bits (1/8), and S (FP64, 8 B) and P (4 B) per su of rows padded to
# a multiple of 32 columns; per pedestrian  keys (8),
# positions, targets, id map (4 each), flags (1); plus counters, the stamp and
# the scene's share of a batch's layout (views, workgroup maps, work items,
# stamp tables): < 1 MiB.
BYTES_PER_SU = 4 + 1 + 16 + 0.125
BYTES_PER_PADDED_SU = 8 + 4
BYTES_PER_PED = 8 + 4 + 4 + 4 + 1
FIXED_BYTES = 1 << 20
# Temporaries of scene creation, released when the build ends: per su the
# obstacle mask (1 B), five bitmaps (obstacles, two visited sets, two
# frontiers: 5/8 B) and the FP64 obstacle field (8 B).
BUILD_BYTES_PER_SU = 1 + 5 * 0.125 + 8


def footprint_bytes(scene) -> int:
    """Device bytes a resident scene holds."""
    su = int(scene.width) * int(scene.height)
    padded = (int(scene.width) + 31) // 32 * 32 * int(scene.height)
    return int(su * BYTES_PER_SU + padded * BYTES_PER_PADDED_SU
               + int(np.asarray(scene.pos).shape[0]) * BYTES_PER_PED + FIXED_BYTES)


def build_bytes(scene) -> int:
    """Device bytes a scene holds on top of its footprint while it is built."""
    return int(int(scene.width) * int(scene.height) * BUILD_BYTES_PER_SU)


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float  # seconds after the start of the run
    make_scene: Callable[[], object]  # materialised when first considered for admission
    max_steps: int = 2000
    _scene: object = None

    def scene(self):
        if self._scene is None:
            self._scene = self.make_scene()
        return self._scene


@dataclasses.dataclass
class Finished:
    rid: int
    arrival: float
    admitted: float
    finished: float
    steps: int
    stats: dict
    positions: Optional[np.ndarray] = None


@dataclasses.dataclass
class _Resident:
    req: Request
    scene: object
    gpu: object
    admitted: float
    bytes: int
    steps: int = 0
    last: Optional[dict] = None


def poisson_arrivals(rate: float, duration: float, seed: int) -> np.ndarray:
    """Arrival times of a Poisson stream of `rate` per second over [0, duration)."""
    rng = np.random.Generator(np.random.PCG64([seed, int(rate * 1000)]))
    n = int(rate * duration * 2 + 64)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n))
    while t[-1] < duration:
        t = np.concatenate([t, t[-1] + np.cumsum(rng.exponential(1.0 / rate, size=n))])
    return t[t < duration]


class Server:
    """Admits, batches and retires scenes; see the module docstring."""

    def __init__(self, budget_bytes: int, max_scenes: int = 512, stream=None,
                 tiling: Optional[dict] = None, keep_positions: bool = False,
                 clock=time.perf_counter, max_admit_per_tick: int = 1,
                 create_stream=None, background_builds: bool = True,
                 max_building: int = 2):
        self.budget = int(budget_bytes)
        self.max_scenes = int(max_scenes)
        self.stream = stream
        self.tiling = tiling
        self.keep_positions = keep_positions
        self.clock = clock
        self.max_admit_per_tick = int(max_admit_per_tick)
        self.background = bool(background_builds)
        # admitted scenes waiting for or in their build (background mode)
        self.max_building = max(1, int(max_building))
        # stream on which admitted scenes are built: in background mode one
        # that does not wait for the ticks (a torch stream), otherwise the
        # tick stream
        self.create_stream = create_stream
        if self.create_stream is None and not self.background:
            self.create_stream = stream

    def _builder(self, jobs, done, stream):
        device = getattr(stream, "device", None)
        if device is not None:  # the current device is per thread
            import torch

            torch.cuda.set_device(device)
        while True:
            job = jobs.get()
            if job is None:
                return
            req, scene, need, extra = job
            try:
                done.put((req, need, extra, sf.GpuScene(scene, stream=stream), None))
            except BaseException as e:  # reported by the serving loop
                done.put((req, need, extra, None, e))

    def run(self, requests: List[Request], stop_admitting_at: Optional[float] = None,
            drain: bool = True, deadline: Optional[float] = None) -> dict:
        """Serve `requests` (sorted by arrival).  Admission stops at
        `stop_admitting_at` seconds (None: never); with `drain`, resident
        scenes then run to completion; `deadline` ends the run regardless."""
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        queue: collections.deque = collections.deque()
        resident: List[_Resident] = []
        finished: List[Finished] = []
        used = 0
        batch = None
        tick_ms: List[float] = []  # one batched tick (launch to completion)
        step_ms: List[float] = []  # between consecutive ticks (the latency a scene sees)
        last_end = None
        resident_count: List[int] = []
        admitted_n = 0
        max_used = 0
        max_resident = 0
        t0 = self.clock()

        def now():
            return self.clock() - t0

        building = 0
        jobs: "_queue.Queue" = _queue.Queue()
        done_q: "_queue.Queue" = _queue.Queue()
        worker = None
        if self.background:
            cs = self.create_stream
            if cs is None:
                import torch

                cs = torch.cuda.Stream()
            worker = threading.Thread(target=self._builder, args=(jobs, done_q, cs),
                                      name="sf-scene-builder", daemon=True)
            worker.start()

        def join_built(item):
            nonlocal building, used
            req, need, extra, g, err = item
            building -= 1
            used -= extra  # the build's temporaries are released
            if err is not None:
                used -= need
                raise err
            resident.append(_Resident(req, None, g, now(), need))

        try:
            while True:
                t = now()
                if deadline is not None and t >= deadline:
                    break
                admitting = stop_admitting_at is None or t < stop_admitting_at
                while pending and pending[0].arrival <= t:
                    queue.append(pending.popleft())
                changed = False
                # scenes whose build completed join before this tick
                if self.background:
                    while True:
                        try:
                            item = done_q.get_nowait()
                        except _queue.Empty:
                            break
                        join_built(item)
                        changed = True
                # admission in arrival order while the head of the queue fits
                # (synchronous builds: all at once while nothing is resident)
                admitted_now = 0
                while admitting and queue and len(resident) + building < self.max_scenes:
                    if self.background:
                        if building >= self.max_building:
                            break
                    elif admitted_now >= self.max_admit_per_tick and resident:
                        break
                    req = queue[0]
                    scene = req.scene()
                    need = footprint_bytes(scene)
                    extra = build_bytes(scene)
                    if used + need + extra > self.budget:
                        if not resident and not building:
                            raise ValueError(f"request {req.rid} needs {need} B, more than "
                                             f"the whole budget of {self.budget} B")
                        break
                    queue.popleft()
                    req._scene = None  # the device copy is the state from here on
                    used += need + extra
                    admitted_n += 1
                    admitted_now += 1
                    max_used = max(max_used, used)
                    if self.background:
                        building += 1
                        jobs.put((req, scene, need, extra))
                        continue
                    if batch is not None:
                        batch.close()
                        batch = None
                    g = sf.GpuScene(scene, stream=self.create_stream)
                    used -= extra
                    resident.append(_Resident(req, None, g, now(), need))
                    changed = True
                if not resident and building:
                    # nothing to tick: wait for the first build
                    join_built(done_q.get())
                    changed = True
                max_resident = max(max_resident, len(resident))
                if not resident:
                    last_end = None
                    if not admitting or (not pending and not queue and not building):
                        break
                    if pending and not queue:
                        wait = pending[0].arrival - now()
                        if wait > 0:
                            time.sleep(min(wait, 0.05))
                    continue
                if not admitting and not drain:
                    break
                if batch is None or changed:
                    if batch is not None:
                        batch.close()
                    batch = sf.Batch([r.gpu for r in resident], tiling=self.tiling,
                                     stream=self.stream)
                ts = self.clock()
                batch.step(1)
                totals = batch.stats()  # waits for the tick
                te = self.clock()
                tick_ms.append(1000.0 * (te - ts))
                if last_end is not None:
                    step_ms.append(1000.0 * (te - last_end))
                last_end = te
                resident_count.append(len(resident))
                done = []
                for r, s in zip(resident, totals):
                    r.steps += 1
                    r.last = s
                    if s["live"] == 0 or r.steps >= r.req.max_steps:
                        done.append((r, s))
                if done:
                    batch.close()
                    batch = None
                    for r, s in done:
                        pos = r.gpu.positions() if self.keep_positions else None
                        finished.append(Finished(r.req.rid, r.req.arrival, r.admitted, now(),
                                                 r.steps, s, pos))
                        r.gpu.close()
                        used -= r.bytes
                    ids = {id(r) for r, _ in done}
                    resident = [r for r in resident if id(r) not in ids]
        finally:
            if worker is not None:
                jobs.put(None)
                worker.join()
                while True:  # builds that completed after the loop ended
                    try:
                        item = done_q.get_nowait()
                    except _queue.Empty:
                        break
                    if item[3] is not None:
                        item[3].close()
            if batch is not None:
                batch.close()
            for r in resident:
                r.gpu.close()
        wall = now()
        ped_steps = sum(f.stats["ped_steps"] for f in finished) + \
            sum(r.last["ped_steps"] for r in resident if r.last is not None)
        lat = np.array(tick_ms) if tick_ms else np.zeros(1)
        stp = np.array(step_ms) if step_ms else lat
        waits = np.array([f.admitted - f.arrival for f in finished]) if finished else np.zeros(1)
        return {
            "wall_s": wall,
            "requests": len(requests),
            "admitted": admitted_n,
            "finished": len(finished),
            "unfinished_resident": len(resident),
            "still_queued": len(queue) + len(pending),
            "scenes_per_s": len(finished) / wall if wall > 0 else 0.0,
            "ticks": len(tick_ms),
            "step_latency_ms_p50": float(np.percentile(stp, 50)),
            "step_latency_ms_p99": float(np.percentile(stp, 99)),
            "tick_ms_p50": float(np.percentile(lat, 50)),
            "tick_ms_p99": float(np.percentile(lat, 99)),
            "tick_ms_mean": float(lat.mean()),
            "resident_mean": float(np.mean(resident_count)) if resident_count else 0.0,
            "admission_wait_s_p50": float(np.percentile(waits, 50)),
            "admission_wait_s_p99": float(np.percentile(waits, 99)),
            "ped_steps": int(ped_steps),
            "ped_steps_per_s": ped_steps / wall if wall > 0 else 0.0,
            "max_used_bytes": int(max_used),
            "max_resident": int(max_resident),
            "results": finished,
        }
