#!/usr/bin/env python3
"""Throughput of the merged K-cell forward + backward pass on one MI355X.

Workload: 1,000,000 Gaussians (64 anisotropic clusters + 30% on a ground
plane, SH degree 3, fp32), one 1600x1060 view, K = 8 KD cells; the loss is
L1 + 0.2 (1 - SSIM) against a seeded uniform-noise target.  One step is the
whole hot path: view upload, projection + SH, binning and sorting, partial
render (with the merge in the same launch), loss, merge backward, partial-render backward with the per-pair
reduction, projection backward.  Inputs are seeded synthetic arrays already
resident in HBM when the timed region starts; the KD partition (once per
scene) is outside it.

Timing: W warm-up steps, then K steps timed as a whole (mean step time; no
event inside the region), then K steps with an event between steps (median
step time) and K steps with an event at every stage boundary (the per-stage
split and the kernel times of the roofline entries).

Prints one JSON line: Mpix/s (= H W / step time), the per-stage split; for
every step of the path its algorithmic bytes and FLOP, the time they need at
HBM or FP32 peak and the achieved fraction (and the HBM bytes the counters
saw, when the committed counter summary matches the sources); the overall
fraction (sum of the floors over the step time); the roofline of the
dominant kernel (partial-render backward, measured with HIP events on its
launch stream); config 1's absolute times; a bounded serving leg (100M
Gaussians resident, Poisson traces at 200 and 800 req/s, batched K = 64
against the plain one-view-at-a-time path: p50/p99 latency, frames/s); and
the CPU oracle timed on bounded pixel samples of the same workload, with all
host threads and with one.

Other modes: --serve (the full serving study), --batched (config 4's fused
16-view pass against 16 sequential passes), --train c3|c4 (training
steps/s), --partition (KD tree against the fixed grid, the paper's subsets).
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP32_VECTOR_PEAK_TFLOPS = 157.3   # MI355X fp32 vector (256 CU x 4 SIMD x 16 lanes x 2.4 GHz x 2 FMA x 2 packed)
HBM_PEAK_GBS = 8000.0
HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "paper_2406_11836_amd", "csrc")
TRAFFIC_FILE = os.path.join(HERE, "profiles", "hbm_traffic_1M_1600x1060_K8.txt")


# Algorithmic work of each step of the path per unit (bytes the method must
# move, FLOP it must compute), from the counts of the seeded workload:
#   N Gaussians, V visible (view, Gaussian) pairs, I instances, Ib of them
#   ahead of their slot's last contributor (the backward's), S slots, P tested
#   (pixel, instance) pairs, Pc contributing, HW pixels.
def row_work(c):
    N, I, S, HW = c["N"], c["I"], c["S"], c["HW"]
    return {
        # SH 3 parameters in (236 B) + the 64 B record out; ~300 FLOP per Gaussian
        "project": (300.0 * N, 300.0 * N),
        # bin: counts / rects read twice (2 x 24 B per Gaussian) + 16 B per instance
        # written; sort floor: one read and one write of key + value (24 B) per instance
        "bin_sort": (48.0 * N + 16.0 * I + 24.0 * I, 0.0),
        # 7 FLOP per rejected pair, 22 per contributing pair (exp counted once);
        # 48 B per instance per slot + 20 B per pixel per slot; the merged image
        # and T_final (16 B per pixel) written by the same launch
        "render_fwd": (48.0 * I + 20.0 * 256 * S + 16.0 * HW, 7.0 * (c["P_f"] - c["Pc_f"]) + 22.0 * c["Pc_f"]),
        # L1 36 B per pixel; SSIM ~220 FLOP per pixel-channel
        "loss": (36.0 * HW, 220.0 * 3 * HW),
        "merge_bwd": (48.0 * 256 * S, 0.0),
        # 7 FLOP per rejected pair, 55 per contributing pair; per instance it visits
        # 72 B read (value + record) and a 36 B gradient record written; 24 B per
        # pixel per slot (T, last, dT, dC)
        "render_bwd": (108.0 * c["Ib"] + 24.0 * 256 * S, 7.0 * (c["P_b"] - c["Pc_b"]) + 55.0 * c["Pc_b"]),
        # the records (36 B per visited instance) and a bit per instance read, 36 B
        # per Gaussian written
        "pair_reduce": (36.0 * c["Ib"] + I / 8.0 + 36.0 * N, 0.0),
        # ~570 B and ~600 FLOP per Gaussian
        "project_bwd": (570.0 * N, 600.0 * N),
    }


def floor_s(b, f):
    return max(b / (HBM_PEAK_GBS * 1e9), f / (FP32_VECTOR_PEAK_TFLOPS * 1e12))


def source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in sorted(os.listdir(CSRC)):
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()


def measured_traffic():
    """Per-kernel HBM bytes per step (all of the kernel's dispatches in one
    step) from the committed counter summary (FETCH_SIZE and WRITE_SIZE, each
    scaled by the same counter's reading on a copy of known size); empty when
    absent or when any kernel source changed since the counters were taken."""
    out = {}
    try:
        with open(TRAFFIC_FILE) as fh:
            lines = fh.read().splitlines()
    except OSError:
        return out
    sha = None
    for line in lines:
        if line.startswith("source_sha256:"):
            sha = line.split(":", 1)[1].strip()
        elif line.startswith("kernel "):
            parts = line.split()
            out[parts[1]] = float(parts[-1])
    return out if sha == source_hash() else {}


def cpu_baseline(p, cam, L, target_s: float):
    """The CPU oracle as it stands (fp64 values, fp32 decisions) on bounded
    random pixel samples of the same view: one run = projection of every
    Gaussian, per-pixel forward and backward of the sample, projection
    backward.  Median of 3 runs with every host thread and with one thread;
    sample sizes chosen from a short probe so that a run takes about
    target_s seconds."""
    import platform
    import statistics

    import numpy as np

    import oracle
    okd = oracle.kd_partition(p["means"], p["log_scales"], L)
    order, _ = oracle.cell_order(L, okd["split"], cam["o"])
    rng = np.random.default_rng(99)
    W, H = cam["W"], cam["H"]

    def run(npix):
        pix = np.stack([rng.integers(0, W, npix), rng.integers(0, H, npix)], 1).astype(np.int32)
        dimg = rng.normal(size=(npix, 3)) * 1e-6
        t0 = time.perf_counter()
        pr = oracle.project(p, cam, okd, 0)
        oracle.render(pr, cam, okd, order, pix, 5e-5)
        g2d = oracle.render_bwd(pr, cam, okd, order, pix, dimg, None, 5e-5)
        oracle.project_bwd(p, cam, pr, g2d)
        return time.perf_counter() - t0

    def measure(threads):
        oracle.set_threads(threads)
        t1 = run(64)
        t2 = run(320)
        per_px = max((t2 - t1) / 256.0, 1e-7)
        fixed = max(t1 - 64 * per_px, 0.0)
        npix = int(max(64, min(200_000, (target_s - fixed) / per_px)))
        times = [run(npix) for _ in range(3)]
        t = statistics.median(times)
        return npix / t / 1e6, npix, t, threads

    all_threads = oracle.num_threads()
    res_all = measure(all_threads)
    res_one = measure(1)
    oracle.set_threads(all_threads)
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": round(res_all[0], 6), "unit": "Mpix/s", "cores": res_all[3], "kind": "oracle",
            "sample": "%d random pixels of the 1600x1060 view per run (median of 3 runs, %.2f s), fwd+bwd incl. "
                      "projection of all 1M Gaussians and its backward, loss excluded" % (res_all[1], res_all[2]),
            "value_1thread": round(res_one[0], 6),
            "sample_1thread": "%d pixels per run, median of 3 runs, %.2f s" % (res_one[1], res_one[2]),
            "cpu_model": model, "host_threads": os.cpu_count()}


def serving(n: int, rates, n_req: int, warmup_req: int, paths=("batched", "batched_K1", "plain")):
    """Continuous-batching server (K = 64 with cell culling, and K = 1) against
    the one-view-at-a-time plain (K = 1) path on the same Poisson traces (the
    first warmup_req requests of each trace are warm-up)."""
    import torch

    from paper_2406_11836_amd import raster, scenes, serve

    t0 = time.perf_counter()
    p = scenes.scene_city_device(n, seed=50, D=3)
    rast = raster.Rasterizer("cuda:0")
    kd64 = rast.kd_partition(p, 6)
    # resident layout: Gaussians grouped by cell, Morton order inside a cell
    p, _ = rast.group_by_cell(p, kd64)
    kd64 = rast.kd_partition(p, 6)
    kd1 = rast.kd_partition(p, 0, own_mask=False)
    torch.cuda.synchronize()
    prep_s = time.perf_counter() - t0
    out = {"workload": "%d Gaussians SH3 resident (grouped by cell), Poisson requests, 40%% 1280x720 / 40%% "
                       "1920x1080 / 20%% 3840x2160; batched: K=64 KD cells with cell culling, two workers (streams) "
                       "overlapping on the device, <= 2 views per batch; "
                       "plain: K=1, FIFO, one view at a time" % n,
           "requests_per_rate": n_req, "warmup_requests": warmup_req, "scene_prep_s": round(prep_s, 2), "rates": {}}
    cfg = {"batched": (kd64, dict(max_batch=2, workers=2, cull=True)),
           "batched_K1": (kd1, dict(max_batch=2, workers=2, cull=False)),
           "plain": (kd1, dict(max_batch=1, workers=1, cull=False))}
    for rate in rates:
        res = {}
        for name in paths:
            kd, kw = cfg[name]
            reqs = serve.serve_trace(rate, n_req, seed=int(30 + rate))
            torch.cuda.empty_cache()  # the previous server's buffers go back to the device
            srv = serve.Server(p, kd, **kw)
            srv.run(reqs)
            res[name] = serve.latency_stats(reqs, warmup_req, srv)
            print("serve rate %g %s %s" % (rate, name, res[name]), file=sys.stderr, flush=True)
        out["rates"][str(int(rate))] = res
    return out


def batched(args):
    """16 views of uneven resolution in one fused pass (per-view L1, summed)
    against 16 sequential single-view plain (K = 1) passes on the same views."""
    import numpy as np
    import torch

    from paper_2406_11836_amd import raster, scenes

    p = scenes.scene_clusters(4_000_000, seed=40, D=3)
    cams = scenes.config4_cameras(16)
    targets = [torch.from_numpy(scenes.target_image(42 + k, c["W"], c["H"])).cuda() for k, c in enumerate(cams)]
    rast = raster.Rasterizer("cuda:0")
    dp = raster.to_device(p)
    kd16 = rast.kd_partition(dp, 4)
    kd1 = rast.kd_partition(dp, 0)

    def fused(kd):
        st = rast.forward(dp, kd, cams, 5e-5)
        d = torch.empty_like(st.image)
        po = 0
        for (img, _), tg, c in zip(st.images(), targets, cams):
            _, dv = rast.loss(img, tg, 0.0)
            n = 3 * c["W"] * c["H"]
            d[po: po + n] = dv.view(-1)
            po += n
        return rast.backward(st, dp, d)

    def sequential(kd):
        acc = None
        for c, tg in zip(cams, targets):
            st = rast.forward(dp, kd, [c], 5e-5)
            _, dv = rast.loss(st.image.view(3, c["H"], c["W"]), tg, 0.0)
            g = rast.backward(st, dp, dv.view(-1))
            acc = g if acc is None else {k: acc[k] + g[k] for k in raster.PARAM_KEYS}
        return acc

    def timeit(fn, steps, warm):
        for _ in range(warm):
            fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / steps

    t_f = timeit(lambda: fused(kd16), args.steps, args.warmup)
    t_s16 = timeit(lambda: sequential(kd16), max(2, args.steps // 2), 1)
    t_f1 = timeit(lambda: fused(kd1), max(2, args.steps // 2), 1)
    t_s1 = timeit(lambda: sequential(kd1), max(2, args.steps // 2), 1)
    pix = sum(c["W"] * c["H"] for c in cams)
    return {"metric": "batched 16-view fwd+bwd Mpix/s @4M splats K=16 (fused pass vs 16 sequential passes)",
            "value": round(pix / (t_f * 1e-3) / 1e6, 3), "unit": "Mpix/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": round(t_f, 3), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "4M Gaussians SH3, 16 views of {960x540,1600x1060,1920x1080,3840x2160}, K=16, L1",
                       "total_pixels": pix, "resolutions": [[c["W"], c["H"]] for c in cams]},
            "ms": {"fused_K16": round(t_f, 3), "sequential_K16": round(t_s16, 3),
                   "fused_K1": round(t_f1, 3), "sequential_K1": round(t_s1, 3)},
            "speedup_fused_vs_sequential_K16": round(t_s16 / t_f, 3),
            "speedup_fused_vs_sequential_K1": round(t_s1 / t_f1, 3)}


def c1_times(rast, reps: int = 20):
    """Config 1 (20k Gaussians, 256x256, L1): forward + backward ms, unpartitioned
    and with K = 4 cells (median of reps after 3 warm-up steps).  Launch-bound
    at this size: absolute times only."""
    import statistics

    import torch

    from paper_2406_11836_amd import raster, scenes
    p, cam, tgt, L = scenes.config1()
    dp = raster.to_device(p)
    target = torch.from_numpy(tgt).cuda()
    out = {}
    for Ld in (0, L):
        kd = rast.kd_partition(dp, Ld)

        def step():
            st = rast.forward(dp, kd, [cam], 5e-5, no_sync=True)
            _, d = rast.loss(st.image.view(3, 256, 256), target, 0.0)
            rast.backward(st, dp, d.view(-1))

        for _ in range(3):
            step()
        ts = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            step()
            b.record()
            b.synchronize()
            ts.append(a.elapsed_time(b))
        out["K%d_ms" % (1 << Ld)] = round(statistics.median(ts), 4)
    return out


def train_bench(args):
    """Training steps/s (forward, loss, backward, fused Adam, position rate
    decay) at config 3 (16M-Gaussian city, one 3840x2160 view per step, K = 32,
    L1 + 0.2 (1 - SSIM)) or config 4 (4M clustered Gaussians, the 16
    uneven views in one fused pass, K = 16, L1)."""
    import numpy as np
    import torch

    from paper_2406_11836_amd import raster, scenes, train
    if args.train == "c3":
        p = scenes.scene_city_device(16_000_000, seed=30, D=3)
        rng = np.random.default_rng(31)
        views = [[scenes.aerial_camera(rng, 3840, 2160, 800.0, 150.0, -45.0)] for _ in range(8)]
        Ld, ssim_w = 5, 0.2
    else:
        p = raster.to_device(scenes.scene_clusters(4_000_000, seed=40, D=3))
        views = [scenes.config4_cameras(16)]
        Ld, ssim_w = 4, 0.0
    targets = [[torch.from_numpy(scenes.target_image(300 + 17 * i + j, c["W"], c["H"])).cuda()
                for j, c in enumerate(v)] for i, v in enumerate(views)]
    tr = train.Trainer(p, Ld, max_steps=30000, repartition_every=0, ssim_weight=ssim_w)
    for i in range(args.warmup):
        tr.step(views[i % len(views)], targets[i % len(views)])
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for i in range(args.steps):
        lv = tr.step(views[i % len(views)], targets[i % len(views)])
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / args.steps
    # one re-partition (KD rebuild + regroup of parameters and both Adam moments), timed alone
    c, d = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c.record()
    tr.repartition()
    d.record()
    torch.cuda.synchronize()
    pix = sum(cc["W"] * cc["H"] for cc in views[0])
    return {"metric": "training steps/s (%s)" % args.train, "value": round(1000.0 / ms, 3), "unit": "steps/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "config 3: 16M-Gaussian aerial city SH3, one 3840x2160 view per step, K=32, "
                                   "L1+0.2(1-SSIM), fused Adam (fp32 states)" if args.train == "c3" else
                                   "config 4: 4M clustered Gaussians SH3, 16 uneven views per step in one fused "
                                   "pass, K=16, per-view L1, fused Adam (fp32 states)",
                       "gaussians": int(p["means"].shape[1]), "pixels_per_step": pix, "cells": 1 << Ld},
            "mpix_per_s": round(pix / (ms * 1e-3) / 1e6, 3), "repartition_ms": round(c.elapsed_time(d), 3),
            "last_loss": round(float(lv.item()), 6)}


def partition_bench(args):
    """KD tree against the fixed-size grid (Table 2's comparison) on config 2
    and config 4: per-cell Gaussian counts, instances, slots and the render
    time of each cell's slots alone (the spread stands in for the workers'
    imbalance); and the paper's subsets N_k as the render set for the margin
    factors 3, 4 and 6 (escaped contributions, image error against the exact
    render), with eps_T = 0."""
    import ctypes as C

    import numpy as np
    import torch

    from paper_2406_11836_amd import _lib as Lb
    from paper_2406_11836_amd import raster, scenes
    rast = raster.Rasterizer("cuda:0")
    out = {"metric": "partition diagnostics (KD vs fixed grid; paper subsets)", "configs": {}}
    cases = []
    p2, cam2, _, L2 = scenes.config2()
    cases.append(("config2", raster.to_device(p2), [cam2], L2))
    if not args.partition_quick:
        p4 = scenes.scene_clusters(4_000_000, seed=40, D=3)
        cases.append(("config4", raster.to_device(p4), scenes.config4_cameras(16), 4))
    for name, dp, cams, Ld in cases:
        res = {}
        for rule_name, rule in (("kd", Lb.RGS_SPLIT_MEDIAN), ("grid", Lb.RGS_SPLIT_MIDPOINT)):
            kd = rast.kd_partition(dp, Ld, rule=rule)
            st = rast.forward(dp, kd, cams, 5e-5)
            torch.cuda.synchronize()
            K = 1 << Ld
            S = int(st.bins["counters"][2].item())
            keys = st.bins["slot_key"][:S].cpu().numpy().astype(np.int64)
            rng_ = st.bins["slot_range"][: 2 * S].view(S, 2).cpu().numpy().astype(np.int64)
            ranks = rast.cell_ranks(kd, cams)
            # cell of each slot: rank in its view's order -> cell id
            tile_off = np.cumsum([0] + [((c["W"] + 15) // 16) * ((c["H"] + 15) // 16) for c in cams])
            gt = keys >> Ld
            view = np.searchsorted(tile_off, gt, side="right") - 1
            cell_of_rank = np.argsort(ranks, 1)
            cell = cell_of_rank[view, keys & (K - 1)]
            inst = np.bincount(cell, weights=rng_[:, 1] - rng_[:, 0], minlength=K).astype(np.int64)
            slots = np.bincount(cell, minlength=K)
            # time each cell's slots alone, as a worker holding one cell renders
            # them (every pixel starting from P = 1): a slot table with only
            # that cell's slots (the forward walks a tile's slots from
            # tile_slot), copied into buffers of the full capacities
            T = int(st.total_tiles)
            cap = int(st.slot_capacity)
            ms = []
            bs = st.bins_struct
            saved = (bs.slot_key, bs.slot_range, bs.tile_slot)
            for k in range(K):
                sel = np.nonzero(cell == k)[0]
                if sel.size == 0:
                    ms.append(0.0)
                    continue
                idx = torch.from_numpy(sel).cuda()
                sk = torch.zeros(cap, dtype=torch.int32, device="cuda")
                sr = torch.zeros(2 * cap, dtype=torch.int32, device="cuda")
                sk[: sel.size] = st.bins["slot_key"][idx]
                sr[: 2 * sel.size] = st.bins["slot_range"][: 2 * S].view(S, 2)[idx].reshape(-1)
                tsl = torch.from_numpy(np.searchsorted(gt[sel], np.arange(T + 1), side="left").astype(np.int32)).cuda()
                bs.slot_key, bs.slot_range, bs.tile_slot = sk.data_ptr(), sr.data_ptr(), tsl.data_ptr()
                ts = []
                for rep in range(4):
                    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    pt = st.parts_struct()
                    ks = kd.struct()
                    ps = st.proj_struct()
                    a.record()
                    Lb.check("rgs_render_partial", rast.lib.rgs_render_partial(
                        C.byref(ps), st.n, C.byref(bs), st.cam_arr, len(cams), raster._p(st.views), C.byref(ks),
                        5e-5, C.byref(pt), None, raster._stream()))
                    b.record()
                    b.synchronize()
                    if rep:
                        ts.append(a.elapsed_time(b))
                ms.append(float(np.median(ts)))
                del sk, sr, tsl
            bs.slot_key, bs.slot_range, bs.tile_slot = saved
            counts = kd.counts.cpu().numpy()
            res[rule_name] = {"gaussians_per_cell": counts.tolist(), "instances_per_cell": inst.tolist(),
                              "slots_per_cell": slots.tolist(), "render_ms_per_cell": [round(x, 4) for x in ms],
                              "count_max_over_min": round(float(counts.max() / max(counts.min(), 1)), 3),
                              "render_ms_max_over_mean": round(float(np.max(ms) / max(np.mean(ms), 1e-9)), 3)}
            print("partition %s %s %s" % (name, rule_name, res[rule_name]), file=sys.stderr, flush=True)
        if name == "config2":
            esc = []
            stats0 = torch.zeros(2, dtype=torch.int64, device="cuda")
            stats1 = torch.zeros(2, dtype=torch.int64, device="cuda")
            for f in (3.0, 4.0, 6.0):
                kd = rast.kd_partition(dp, Ld, d_factor=f)
                stats0.zero_()
                stats1.zero_()
                a = rast.forward(dp, kd, cams, 0.0, stats=stats0).image.clone()
                b = rast.forward(dp, kd, cams, 0.0, stats=stats1, cells=Lb.RGS_CELLS_PAPER_SUBSETS).image
                torch.cuda.synchronize()
                esc.append({"d_factor": f, "escaped_contributions": int(stats0[1] - stats1[1]),
                            "contributions": int(stats0[1]), "max_abs_image_error": float((a - b).abs().max()),
                            "mean_abs_image_error": float((a - b).abs().mean())})
            kd = rast.kd_partition(dp, Ld)
            a = rast.forward(dp, kd, cams, 0.0).image.clone()
            b = rast.forward(dp, kd, cams, 0.0, cells=Lb.RGS_CELLS_EXCLUSIVE).image
            res["paper_subsets"] = esc
            res["exclusive_cells"] = {"max_abs_image_error": float((a - b).abs().max()),
                                      "mean_abs_image_error": float((a - b).abs().mean())}
        out["configs"][name] = res
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cpu-seconds", type=float, default=3.0, help="seconds per CPU-baseline run (3 runs x 2)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true", help="skip the bounded serving leg of the default run")
    ap.add_argument("--no-c1", action="store_true", help="skip config 1's absolute times (e.g. for profiling)")
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--serve", action="store_true",
                    help="full serving study: 100M-Gaussian city resident in HBM, Poisson traces at 50/200/800 req/s")
    ap.add_argument("--serve-n", type=int, default=100_000_000)
    ap.add_argument("--serve-requests", type=int, default=2100)
    ap.add_argument("--serve-rates", type=str, default="50,200,800")
    ap.add_argument("--batched", action="store_true",
                    help="16-view batched step (4M Gaussians): one fused pass against 16 sequential passes, at K=16 and K=1")
    ap.add_argument("--train", choices=["c3", "c4"], help="training steps/s at config 3 or config 4")
    ap.add_argument("--partition", action="store_true", help="KD vs fixed grid, paper subsets (diagnostics)")
    ap.add_argument("--partition-quick", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one 256 MiB device-to-device copy first (reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library's kernels run on one device and there is no multi-GPU "
              "path (the cross-GPU merge would be an all-to-all of partial maps by screen strip). "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2406_11836_amd import raster, scenes

    torch.cuda.set_device(0)
    if args.batched:
        print(json.dumps(batched(args)))
        return
    if args.serve:
        print(json.dumps(serving(args.serve_n, [float(x) for x in args.serve_rates.split(",")], args.serve_requests,
                                 100)))
        return
    if args.train:
        print(json.dumps(train_bench(args)))
        return
    if args.partition:
        print(json.dumps(partition_bench(args)))
        return
    if args.calib_copy:
        a = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    p, cam, tgt, L = scenes.config2(n=args.n)
    W, H = cam["W"], cam["H"]
    rast = raster.Rasterizer("cuda:0")
    dp = raster.to_device(p)
    kd = rast.kd_partition(dp, L)
    target = torch.from_numpy(tgt).cuda()
    eps_T = 5e-5
    ssim_w = 0.2

    def step(marks=None, stats=None, bstats=None, no_sync=True):
        # binning without a host wait: the capacity comes from the statistics pass
        st = rast.forward(dp, kd, [cam], eps_T, stats=stats, marks=marks, no_sync=no_sync)
        lv, d = rast.loss(st.image.view(3, H, W), target, ssim_w)
        raster._mark(marks, "loss")
        g = rast.backward(st, dp, d.view(-1), None, marks=marks, stats=bstats)
        raster._mark(marks, "end")
        return st, g, lv

    # pair statistics of the forward and backward render (one extra untimed pass)
    stats = torch.zeros(2, dtype=torch.int64, device="cuda")
    bstats = torch.zeros(2, dtype=torch.int64, device="cuda")
    st0, _, lv0 = step(stats=stats, bstats=bstats, no_sync=False)
    torch.cuda.synchronize()
    n_eval, n_con = (int(v) for v in stats.cpu().tolist())
    nb_eval, nb_con = (int(v) for v in bstats.cpu().tolist())
    n_inst = int(st0.bins_struct.n_instances)
    n_slots = int(st0.bins["counters"][2].item())
    n_vis = int(st0.bins["counters"][0].item())
    # instances the backward visits: those ahead of their slot's last contributor
    last = st0.parts["last"][: n_slots * 256].view(n_slots, 256).to(torch.int64).amax(dim=1)
    srange = st0.bins["slot_range"][: 2 * n_slots].view(n_slots, 2).to(torch.int64)
    n_inst_bwd = int(torch.minimum(last, srange[:, 1] - srange[:, 0]).sum().item())
    del st0, last, srange

    # no cyclic garbage collection from the warm-up to the end of the three
    # passes: a collection pause on the host can leave the stream idle between
    # two launches (and a pause right before the timed region lets the clocks
    # drop for its first steps)
    gc.collect()
    gc.disable()
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    stage_ms = {}
    step_ms = []
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t_start.record()
    last = None
    for _ in range(args.steps):
        last = step()
    t_end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_step = t_start.elapsed_time(t_end) / args.steps
    if last[0].overflow():
        raise RuntimeError("instance capacity exceeded in a timed step")
    del last
    # Per-step times (an event between steps) and the stage breakdown (an event
    # at every stage boundary, the kernel times of the roofline entries) come
    # from two further passes of the same steps: every recorded event adds a
    # gap of a few microseconds on the stream, which stays out of the
    # headline's timed region.
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    ev[0].record()
    for i in range(args.steps):
        step()
        ev[i + 1].record()
    torch.cuda.synchronize()
    step_ms = [ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)]
    all_marks = []
    for _ in range(args.steps):
        marks = []
        step(marks=marks)
        all_marks.append(marks)
    torch.cuda.synchronize()
    gc.enable()
    marked_ms = []
    for marks in all_marks:
        for (a, ea), (b, eb) in zip(marks[:-1], marks[1:]):
            if b in ("bwd_start", "end"):
                continue
            stage_ms.setdefault(b, []).append(ea.elapsed_time(eb))
        marked_ms.append(marks[0][1].elapsed_time(marks[-1][1]))
    stages = {k: float(np.mean(v)) for k, v in stage_ms.items()}

    mpix = (W * H) / (ms_step * 1e-3) / 1e6
    counts = dict(N=args.n, I=n_inst, Ib=n_inst_bwd, S=n_slots, HW=W * H, P_f=n_eval, Pc_f=n_con, P_b=nb_eval,
                  Pc_b=nb_con)
    work = row_work(counts)
    traffic = measured_traffic()
    rows = {}
    floor_total = 0.0
    for name, (b, f) in work.items():
        fl = floor_s(b, f)
        floor_total += fl
        t = stages[name] * 1e-3
        rows[name] = {"ms": round(stages[name], 4), "algorithmic_bytes": int(b), "algorithmic_flop": int(f),
                      "floor_ms": round(fl * 1e3, 4), "frac": round(fl / t, 4),
                      "bound": "hbm" if b / (HBM_PEAK_GBS * 1e9) >= f / (FP32_VECTOR_PEAK_TFLOPS * 1e12) else "alu"}
    # HBM bytes from the counters (per dispatch, summed over the row's kernels)
    row_kernels = {"project": ["k_project"],
                   "bin_sort": ["k_vis_count", "k_vis_compact", "k_rs_hist", "k_rs_colscan", "k_rs_scatter",
                                "k_pair_counts", "k_scan_reduce", "k_scan_apply", "k_emit", "k_slot_bounds",
                                "k_slot_build", "k_class_place"],
                   "render_fwd": ["k_render_fwd"],
                   "loss": ["k_ssim_fwd_tiled", "k_ssim_bwd_tiled"],
                   "merge_bwd": ["k_merge_bwd"], "render_bwd": ["k_slot_work", "k_slot_place", "k_render_bwd"],
                   "pair_reduce": ["k_pair_seg", "k_pair_gather"],
                   "project_bwd": ["k_project_bwd_geo", "k_project_bwd_sh"]}
    for name, ks in row_kernels.items():
        if traffic and all(k in traffic for k in ks):
            tb = sum(traffic[k] for k in ks)
            rows[name]["traffic_bytes"] = int(tb)
            rows[name]["traffic_frac_of_hbm_peak"] = round(tb / (stages[name] * 1e-3) / (HBM_PEAK_GBS * 1e9), 4)
    # roofline of the dominant kernel: the partial-render backward (one kernel per
    # call of rgs_render_partial_bwd_records, timed by events on its stream)
    fb = work["render_bwd"][1]
    ach_b = fb / (stages["render_bwd"] * 1e-3) / 1e12
    roof = {"kernel": "k_render_bwd", "bound": "alu", "achieved": round(ach_b, 3),
            "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(ach_b / FP32_VECTOR_PEAK_TFLOPS, 4),
            "traffic": traffic.get("k_render_bwd"), "algorithmic_flop": int(fb), "pairs_tested": nb_eval,
            "pairs_contributing": nb_con, "flop_per_rejected_pair": 7, "flop_per_contributing_pair": 55,
            "avg_ms": round(stages["render_bwd"], 4)}
    ff = work["render_fwd"][1]
    ach_f = ff / (stages["render_fwd"] * 1e-3) / 1e12
    roof_f = {"kernel": "k_render_fwd", "bound": "alu", "achieved": round(ach_f, 3),
              "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(ach_f / FP32_VECTOR_PEAK_TFLOPS, 4),
              "traffic": traffic.get("k_render_fwd"), "algorithmic_flop": int(ff), "pairs_tested": n_eval,
              "pairs_contributing": n_con, "flop_per_rejected_pair": 7, "flop_per_contributing_pair": 22,
              "avg_ms": round(stages["render_fwd"], 4)}

    c1 = None if args.no_c1 else c1_times(rast)
    serve_res = None
    if not args.no_serve:
        serve_res = serving(args.serve_n, [200.0, 800.0], 300, 50, paths=("batched", "plain"))
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(p, cam, L, args.cpu_seconds)

    out = {
        "metric": "fwd+bwd ms & Mpix/s @1M splats 1600x1060 K=8; serve p50/p99 ms vs plain path",
        "value": round(mpix, 3), "unit": "Mpix/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4), "ms_per_step_median": round(float(np.median(step_ms)), 4),
        "ms_per_step_marked": round(float(np.mean(marked_ms)), 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic (seeded clusters + ground plane scene, uniform-noise target)",
        "config": {"workload": "1M Gaussians SH3, 1600x1060, K=8 KD cells, L1+0.2(1-SSIM) fwd+bwd",
                   "gaussians": args.n, "width": W, "height": H, "cells": 1 << L, "eps_T": eps_T},
        "breakdown_ms": {k: round(v, 4) for k, v in stages.items()},
        "counts": {"visible_pairs": n_vis, "instances": n_inst, "instances_backward": n_inst_bwd, "slots": n_slots},
        "loss": round(float(lv0.item()), 6),
        "wall_s": round(wall, 3),
        "roofline": roof,
        "roofline_render_fwd": roof_f,
        "rows": rows,
        "overall_roofline_frac": round(floor_total / (ms_step * 1e-3), 4),
        "config1_ms": c1,
        "serve": serve_res,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
