"""Continuous-batching render server over mgs_render_forward.

* Maps stay resident on the device; requests name a map and a camera.
* A scheduler thread admits queued requests in arrival order while the
  device-memory budget allows (outputs plus an estimate of the workspace, which
  is learned per (map, resolution) from the sizes the library reports), packs
  them into one batch of up to `max_batch` views - any mix of maps and
  resolutions - and hands the batch to an idle worker.
* Each worker is a persistent thread that owns a HIP stream and a workspace;
  one library call renders its whole batch (one persistent blend launch over
  all the batch's tiles).  While one worker's batch runs, the scheduler forms
  the next batch from the requests that arrived meanwhile, so work overlaps on
  the device.  The workers live as long as the server: a batch costs no thread
  start, and the library's per-thread state (its pinned read-back word) is set
  up once per worker.
* Latency is completion minus arrival; `stats()` reports p50 / p99 and
  renders/s.

The execution backend is pluggable (`executor`), so the scheduling logic can
be exercised on the CPU with a fake executor.
"""
from __future__ import annotations

import gc
import threading
import time
from collections import deque
from concurrent.futures import Future
from dataclasses import dataclass, field
from typing import Deque, Dict, List, Optional

import numpy as np


@dataclass
class Request:
    map_id: int
    view: object               # api.View (its .map is set by the batcher)
    arrival: float = 0.0
    future: Future = field(default_factory=Future)
    est_bytes: int = 0
    rid: int = 0


@dataclass
class Result:
    rgb: object                # [3,H,W] device tensor
    depth: object              # [H,W]
    latency_s: float
    batch_size: int


class GpuExecutor:
    """Renders batches with the HIP library; one stream + workspace per worker."""

    def __init__(self, maps: Dict[int, object], n_workers: int = 2, device="cuda"):
        import torch

        from .api import Workspace
        self.torch = torch
        self.maps = maps
        self.device = device
        self.streams = [torch.cuda.Stream(device=device) for _ in range(n_workers)]
        self.ws = [Workspace(device) for _ in range(n_workers)]
        self.ws_per_pixel: Dict[tuple, float] = {}
        self.lock = threading.Lock()

    def map_bytes(self) -> int:
        return sum(m.nbytes() for m in self.maps.values())

    def workspace_bytes(self, req: Request) -> int:
        """Workspace this request adds to a batch: learned bytes per pixel for its
        (map, resolution), else a bound from the map size and the pixel count."""
        v = req.view
        key = (req.map_id, v.W, v.H)
        n = self.maps[req.map_id].n
        with self.lock:
            per_px = self.ws_per_pixel.get(key)
        return int((per_px * v.W * v.H) if per_px is not None else 96 * n + 64 * v.W * v.H)

    def estimate_bytes(self, req: Request) -> int:
        return self.workspace_bytes(req) + 20 * req.view.W * req.view.H

    def run(self, worker: int, batch: List[Request]):
        from .api import View, render_forward
        torch = self.torch
        ids = sorted({r.map_id for r in batch})
        slot = {mid: i for i, mid in enumerate(ids)}
        maps = [self.maps[mid] for mid in ids]
        views = []
        for r in batch:
            v = r.view
            views.append(View(v.W, v.H, v.fx, v.fy, v.cx, v.cy, v.Tcw, v.near, slot[r.map_id]))
        s = self.streams[worker]
        # grow the worker's workspace ahead of the call, with headroom, so that
        # growth (a large device allocation) is rare and no call is repeated
        self.ws[worker].ensure(sum(self.workspace_bytes(r) for r in batch), slack=2.0)
        with torch.cuda.stream(s):
            st = render_forward(maps, views, ws=self.ws[worker], stream=s)
            ev = torch.cuda.Event()
            ev.record(s)
        npix = sum(v.W * v.H for v in views)
        per_px = st.info.ws_required / max(npix, 1)
        with self.lock:
            for r in batch:
                key = (r.map_id, r.view.W, r.view.H)
                old = self.ws_per_pixel.get(key)
                self.ws_per_pixel[key] = per_px if old is None else max(0.8 * old + 0.2 * per_px, per_px)
        ev.synchronize()
        return [st.view_images(i)[:2] for i in range(len(batch))]


def invalid_view(view) -> Optional[str]:
    """Why the library would refuse this view (and with it every view of its
    call), or None: image size, focal lengths, principal point, and a pose that
    is not finite (which the library would render as background)."""
    if not (1 <= int(view.W) <= 16384 and 1 <= int(view.H) <= 16384):
        return f"image size {view.W}x{view.H} outside 1..16384"
    if not (np.isfinite(view.fx) and np.isfinite(view.fy) and view.fx > 0 and view.fy > 0):
        return "focal lengths must be finite and positive"
    if not (np.isfinite(view.cx) and np.isfinite(view.cy)):
        return "principal point must be finite"
    if getattr(view, "Tcw", None) is not None and not np.all(np.isfinite(np.asarray(view.Tcw, np.float64))):
        return "pose must be finite"
    return None


class RenderServer:
    def __init__(self, executor, mem_budget_bytes: int, max_batch: int = 16, n_workers: Optional[int] = None,
                 freeze_gc: bool = True):
        """freeze_gc: move the objects alive at start-up out of Python's cyclic
        collector (gc.freeze), so that a full collection, which otherwise scans
        every object of a torch process and holds the interpreter for tens of
        milliseconds, cannot stall the requests in flight."""
        if freeze_gc:
            gc.freeze()
        self.ex = executor
        self.budget = int(mem_budget_bytes)
        self.max_batch = max_batch
        self.n_workers = n_workers if n_workers is not None else len(getattr(executor, "streams", [None, None]))
        self.queue: Deque[Request] = deque()
        self.lock = threading.Lock()
        self.cv = threading.Condition(self.lock)  # scheduler: requests queued or a worker idle
        # one condition per worker on the same lock: a batch was assigned to it
        self.wcv = [threading.Condition(self.lock) for _ in range(self.n_workers)]
        self.assigned: List[Optional[tuple]] = [None] * self.n_workers
        self.in_use = 0
        self.idle = list(range(self.n_workers))
        self.stopping = False
        self.workers_stop = False
        self.latencies: List[float] = []
        self.lat_by_res: Dict[tuple, List[float]] = {}
        self.completed = 0
        self.batches = 0
        self.t_first: Optional[float] = None
        self.t_last: Optional[float] = None
        self._rid = 0
        self.workers = [threading.Thread(target=self._worker, args=(w,), daemon=True, name=f"render-worker-{w}")
                        for w in range(self.n_workers)]
        for t in self.workers:
            t.start()
        self.sched = threading.Thread(target=self._schedule, daemon=True, name="render-scheduler")
        self.sched.start()

    # ------------------------------------------------------------ client side
    def submit(self, map_id: int, view, arrival: Optional[float] = None) -> Future:
        req = Request(map_id, view, time.perf_counter() if arrival is None else arrival)
        why = invalid_view(view)
        if why is not None:  # refused alone: in a batch it would fail the whole call
            req.future.set_exception(ValueError(why))
            return req.future
        req.est_bytes = self.ex.estimate_bytes(req)
        if req.est_bytes > self.budget:
            req.future.set_exception(MemoryError(f"request needs ~{req.est_bytes} B, budget {self.budget} B"))
            return req.future
        with self.cv:
            req.rid = self._rid
            self._rid += 1
            self.queue.append(req)
            self.cv.notify_all()
        return req.future

    def close(self):
        with self.cv:
            self.stopping = True
            self.cv.notify_all()
        self.sched.join()

    def stats(self) -> dict:
        lat = np.array(self.latencies) * 1e3
        dur = (self.t_last - self.t_first) if self.completed and self.t_last > self.t_first else float("nan")
        return {"completed": self.completed, "batches": self.batches,
                "renders_per_s": self.completed / dur if dur == dur else float("nan"),
                "p50_ms": float(np.percentile(lat, 50)) if len(lat) else float("nan"),
                "p99_ms": float(np.percentile(lat, 99)) if len(lat) else float("nan"),
                "mean_batch": self.completed / max(self.batches, 1),
                "by_resolution": {f"{w}x{h}": {"n": len(v), "p50_ms": float(np.percentile(np.array(v) * 1e3, 50)),
                                               "p99_ms": float(np.percentile(np.array(v) * 1e3, 99))}
                                  for (w, h), v in sorted(self.lat_by_res.items())}}

    # ------------------------------------------------------------ scheduler
    def _take_batch(self) -> List[Request]:
        """Admit queued requests in arrival order while memory allows."""
        batch, need = [], 0
        while self.queue and len(batch) < self.max_batch:
            r = self.queue[0]
            if self.in_use + need + r.est_bytes > self.budget and (batch or self.in_use > 0):
                break
            batch.append(self.queue.popleft())
            need += r.est_bytes
        return batch

    def _schedule(self):
        while True:
            with self.cv:
                while not self.stopping and not (self.queue and self.idle):
                    self.cv.wait()
                if self.stopping and not self.queue:
                    break
                batch = self._take_batch()
                if not batch:
                    self.cv.wait(0.001)
                    continue
                worker = self.idle.pop()
                need = sum(r.est_bytes for r in batch)
                self.in_use += need
                self.assigned[worker] = (batch, need)
                self.wcv[worker].notify()
        # drain: wait for the batches in flight, then stop the workers
        with self.cv:
            while len(self.idle) < self.n_workers:
                self.cv.wait()
            self.workers_stop = True
            for c in self.wcv:
                c.notify()
        for t in self.workers:
            t.join()

    def _worker(self, worker: int):
        while True:
            with self.lock:
                while self.assigned[worker] is None and not self.workers_stop:
                    self.wcv[worker].wait()
                if self.assigned[worker] is None:
                    return
                batch, need = self.assigned[worker]
                self.assigned[worker] = None
            self._run(worker, batch, need)

    def _run(self, worker: int, batch: List[Request], need: int):
        try:
            outs = self.ex.run(worker, batch)
            err = None
        except Exception as e:  # a failing batch fails its own requests only
            outs, err = None, e
        now = time.perf_counter()
        with self.cv:
            self.in_use -= need
            self.idle.append(worker)
            self.batches += 1
            for i, r in enumerate(batch):
                if err is not None:
                    r.future.set_exception(err)
                    continue
                lat = now - r.arrival
                self.latencies.append(lat)
                self.lat_by_res.setdefault((r.view.W, r.view.H), []).append(lat)
                self.completed += 1
                self.t_first = r.arrival if self.t_first is None else min(self.t_first, r.arrival)
                self.t_last = now if self.t_last is None else max(self.t_last, now)
                r.future.set_result(Result(outs[i][0], outs[i][1], lat, len(batch)))
            self.cv.notify_all()


def poisson_load(server: RenderServer, rate_hz: float, n: int, make_request, seed: int = 0):
    """Open-loop Poisson arrivals: submit n requests at exponential gaps."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, size=n)
    futs = []
    t0 = time.perf_counter()
    t = t0
    for i in range(n):
        t += gaps[i]
        delay = t - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        map_id, view = make_request(i)
        futs.append(server.submit(map_id, view, arrival=t))
    for f in futs:
        f.result()
    return futs
