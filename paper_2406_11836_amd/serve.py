"""Continuous-batching render server over a scene resident in HBM.

The paper's central manager parses incoming render requests and hands them
to the sub-models (Sec. 3.4).  Here all sub-models (KD cells) live on one GPU:
a dispatcher replays a request trace in real time, admits arrived requests
into the next batch whenever a worker (one HIP stream each) is free and the
batch's memory estimate fits the budget, and renders the batch with one call
sequence (projection for all views at once, then binning, partial render and
merge).  Two workers are the default, so that the work of a batch that is
admitted while another is on the GPU overlaps it on the device (each worker
has its own stream and buffers); a request that arrives while both are busy
waits for the next free one.  Batches are kept small (two views): a batch of
views at 100M Gaussians holds about 10 GB of per-(view, Gaussian) arrays per
view, and small batches on two workers gave both the lowest tail latency and
the highest frame rate on the city trace (one worker with batches of eight,
and three or four workers, were slower).  Per view, KD cells that cannot
reach the image (rgs_cell_visibility, a conservative test in the library)
are culled before projection.

Latency of a request = host time at which its batch completed - its
scheduled arrival time.  The plain path for comparison is the same trace,
FIFO, one view at a time, unpartitioned (K = 1).
"""
from __future__ import annotations

import collections
import math
import queue
import threading
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import raster


@dataclass
class Request:
    rid: int
    cam: dict
    t_arrival: float
    t_done: float = float("nan")
    batch_size: int = 0
    image: torch.Tensor | None = None


class Server:
    def __init__(self, params, kd: raster.KD, *, max_batch: int = 2, workers: int = 2, eps_T: float = 5e-5,
                 cull: bool = True, mem_budget: float | None = None, keep_images: bool = False,
                 device: str = "cuda"):
        self.params = params
        self.kd = kd
        self.max_batch = int(max_batch)
        self.n_workers = int(workers)
        self.eps_T = eps_T
        self.cull = cull and kd.L > 0 and kd.cell_bounds_host is not None
        self.keep_images = keep_images
        self.device = torch.device(device)
        self.n = int(params["means"].shape[1])
        if mem_budget is None:
            # device memory not in use: free plus what torch's cache holds unused
            free, _ = torch.cuda.mem_get_info(self.device)
            cached = torch.cuda.memory_reserved(self.device) - torch.cuda.memory_allocated(self.device)
            mem_budget = 0.6 * (free + cached)
        self.mem_budget = float(mem_budget)
        self.batch_hist = collections.Counter()
        self.batch_log = []  # (views, pixels, seconds on the worker) per completed batch
        self.peak_mem_est = 0.0
        self.busy_s = 0.0

    # memory estimate of one view: per-(view, Gaussian) projection and pair
    # arrays plus per-pixel instance, partial-map and workspace storage
    def est_bytes(self, cam) -> float:
        px = float(cam["W"]) * float(cam["H"])
        return self.n * 120.0 + px * 320.0

    def _worker(self, wid, jobs: queue.Queue, done: queue.Queue, warm_cams):
        try:
            dev = self.device if self.device.index is not None else torch.device("cuda", torch.cuda.current_device())
            torch.cuda.set_device(dev)
            stream = torch.cuda.Stream(device=dev)  # default priority
            rast = raster.Rasterizer(str(dev), reuse=True)  # no allocation per batch once warm
            if warm_cams:
                # size the buffers for the largest batch before the trace starts
                with torch.cuda.stream(stream):
                    masks = rast.cell_visibility(self.kd, warm_cams) if self.cull else None
                    rast.forward(self.params, self.kd, warm_cams, self.eps_T, cell_visible=masks)
                    stream.synchronize()
            done.put((wid, None, 0.0, None))  # ready
        except BaseException as e:  # report set-up failures too
            done.put((wid, [], 0.0, e))
            return
        while True:
            batch = jobs.get()
            if batch is None:
                return
            try:
                t0 = time.perf_counter()
                with torch.cuda.stream(stream):
                    cams = [r.cam for r in batch]
                    masks = rast.cell_visibility(self.kd, cams) if self.cull else None
                    st = rast.forward(self.params, self.kd, cams, self.eps_T, cell_visible=masks)
                    imgs = [img.clone() for img, _ in st.images()] if self.keep_images else None
                    stream.synchronize()
                t1 = time.perf_counter()
                for k, r in enumerate(batch):
                    r.t_done = t1
                    r.batch_size = len(batch)
                    if imgs is not None:
                        r.image = imgs[k]
                del st
                done.put((wid, batch, t1 - t0, None))
            except BaseException as e:  # report to the dispatcher instead of dying silently
                done.put((wid, batch, 0.0, e))
                return

    def run(self, reqs: list[Request], stall_timeout_s: float = 120.0) -> None:
        """Replay the trace (arrival times relative to now) until every request is
        done.  Raises if a worker fails or nothing completes for stall_timeout_s."""
        jobs = [queue.Queue() for _ in range(self.n_workers)]
        done: queue.Queue = queue.Queue()
        # warm-up batch: the trace's largest views, as many as a batch holds
        warm = sorted((r.cam for r in reqs), key=lambda c: -int(c["W"]) * int(c["H"]))[: self.max_batch]
        threads = [threading.Thread(target=self._worker, args=(w, jobs[w], done, warm), daemon=True)
                   for w in range(self.n_workers)]
        for t in threads:
            t.start()
        for _ in range(self.n_workers):
            w, b, _, err = done.get()
            if err is not None:
                for q in jobs:
                    q.put(None)
                raise RuntimeError("render worker %d failed to start" % w) from err
        idle = list(range(self.n_workers))
        inflight_mem = {w: 0.0 for w in range(self.n_workers)}
        pending: collections.deque = collections.deque()
        nxt, finished = 0, 0
        t0 = time.perf_counter()
        for r in reqs:
            r.t_arrival_abs = t0 + r.t_arrival
        last_progress = time.perf_counter()
        try:
            while finished < len(reqs):
                now = time.perf_counter()
                while nxt < len(reqs) and reqs[nxt].t_arrival_abs <= now:
                    pending.append(reqs[nxt])
                    nxt += 1
                while True:
                    try:
                        w, b, dt, err = done.get_nowait()
                    except queue.Empty:
                        break
                    if err is not None:
                        raise RuntimeError("render worker %d failed" % w) from err
                    finished += len(b)
                    self.busy_s += dt
                    self.batch_log.append((len(b), sum(int(r.cam["W"]) * int(r.cam["H"]) for r in b), dt))
                    inflight_mem[w] = 0.0
                    idle.append(w)
                    last_progress = now
                if now - last_progress > stall_timeout_s:
                    raise RuntimeError("serving made no progress for %.0f s" % stall_timeout_s)
                while idle and pending:
                    inflight = sum(inflight_mem.values())
                    budget = self.mem_budget - inflight
                    batch, est = [], 0.0
                    while pending and len(batch) < self.max_batch:
                        e = self.est_bytes(pending[0].cam)
                        # a request larger than the whole budget still runs, alone
                        if est + e > budget and (batch or inflight > 0.0):
                            break
                        batch.append(pending.popleft())
                        est += e
                    if not batch:
                        break  # wait for memory to free up
                    w = idle.pop(0)
                    inflight_mem[w] = est
                    self.peak_mem_est = max(self.peak_mem_est, sum(inflight_mem.values()))
                    self.batch_hist[len(batch)] += 1
                    jobs[w].put(batch)
                if finished < len(reqs):
                    time.sleep(0.0002)
        finally:
            for q in jobs:
                q.put(None)
            for t in threads:
                t.join()


def serve_trace(rate: float, n_req: int, seed: int, xy_range: float = 900.0, res_mix=None):
    """Poisson arrivals at `rate` per second with aerial poses: (x, y) uniform
    in [-xy_range, xy_range]^2, altitude U(50, 400), yaw U(0, 2 pi), pitch
    U(-90, -30) degrees; resolutions 40% 1280x720, 40% 1920x1080, 20% 3840x2160."""
    from . import scenes
    rng = np.random.default_rng(seed)
    res_mix = res_mix or [((1280, 720), 0.4), ((1920, 1080), 0.4), ((3840, 2160), 0.2)]
    sizes = [r for r, _ in res_mix]
    probs = np.array([p for _, p in res_mix])
    t = 0.0
    reqs = []
    for i in range(n_req):
        t += rng.exponential(1.0 / rate)
        W, H = sizes[int(rng.choice(len(sizes), p=probs))]
        cam = scenes.aerial_camera(rng, W, H, xy_range, rng.uniform(50, 400), rng.uniform(-90, -30))
        reqs.append(Request(i, cam, t))
    return reqs


def latency_stats(reqs, warmup: int, server: Server | None = None) -> dict:
    lat = np.array([(r.t_done - r.t_arrival_abs) * 1e3 for r in reqs[warmup:]])
    t_first = min(r.t_arrival_abs for r in reqs[warmup:])
    t_last = max(r.t_done for r in reqs[warmup:])
    out = {"p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
           "mean_ms": round(float(lat.mean()), 3), "frames_per_s": round(len(lat) / (t_last - t_first), 2),
           "completed": int(len(lat))}
    if server is not None:
        wall = max(r.t_done for r in reqs) - min(r.t_arrival_abs for r in reqs)
        out["gpu_busy_frac"] = round(server.busy_s / max(wall, 1e-9) / server.n_workers, 3)
        out["batch_hist"] = {int(k): int(v) for k, v in sorted(server.batch_hist.items())}
        out["peak_mem_est_gb"] = round(server.peak_mem_est / 1e9, 2)
    return out
