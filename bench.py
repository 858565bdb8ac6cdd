#!/usr/bin/env python3
"""Throughput of the merged K-cell forward + backward pass on one MI355X.

Workload: 1,000,000 Gaussians (64 anisotropic clusters + 30% on a ground
plane, SH degree 3, fp32), one 1600x1060 view, K = 8 KD cells; the loss is
L1 + 0.2 (1 - SSIM) against a seeded uniform-noise target.  One step is the
whole hot path: view upload, projection + SH, binning and sorting, partial
render, merge, loss, merge backward, partial-render backward with the per-pair
reduction, projection backward.  Inputs are seeded synthetic arrays already
resident in HBM when the timed region starts; the KD partition (once per
scene) is outside it.

Prints one JSON line: Mpix/s (= H W / step time), the per-stage split, the
roofline of the dominant kernel (partial-render forward or backward,
measured with HIP events on its launch stream) and the CPU oracle timed on a
bounded pixel sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP32_VECTOR_PEAK_TFLOPS = 157.3   # MI355X fp32 vector (256 CU x 2.4 GHz; counts packed FMA)
HBM_PEAK_GBS = 8000.0
# algorithmic work per (pixel, instance) pair of the partial render (row a5)
FLOP_PER_EVAL_PAIR = 7.0          # dy, two FMA for d^2, compare, plus the per-column dx terms / 4
FLOP_PER_CONTRIB_PAIR = 14.0      # exp argument, exp, alpha G, clamp, weight, 3 FMA colour, 1 - s, T update, stop test
# ... and of its backward (row a9): the same decision per re-tested pair, and per contributing pair
# exp argument, exp, alpha G, clamp, 1 - s, reciprocal, T before (7), <dC, c> - <dC, B> (6),
# d sigma (3), weight and 3 colour terms (4), <dC, B> update (2), q and d alpha (2), 5 raw sums (5)
# = 29, plus 9 for the pair's share of the per-wave sum of 9 values over 64 lanes
FLOP_BWD_EVAL_PAIR = 7.0
FLOP_BWD_CONTRIB_PAIR = 38.0


HERE = os.path.dirname(os.path.abspath(__file__))
TRAFFIC_FILES = {k: os.path.join(HERE, "profiles", "%s_1M_1600x1060_K8_hbm.txt" % k)
                 for k in ("k_render_fwd", "k_render_bwd")}
RENDER_SOURCES = ("paper_2406_11836_amd/csrc/render.hip", "paper_2406_11836_amd/csrc/common.hpp")


def render_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in RENDER_SOURCES:
        with open(os.path.join(HERE, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel: str):
    """HBM bytes per k_render_fwd launch from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, each scaled by the same counter on a copy of
    known size); None when absent or when the kernel sources changed since."""
    try:
        kv = {}
        with open(TRAFFIC_FILES[kernel]) as fh:
            for line in fh:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("source_sha256") != render_source_hash():
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def cpu_baseline(p, cam, L, target_s: float):
    """The CPU oracle (fp64 values, fp32 decisions) on a bounded random pixel
    sample of the same view: projection of all Gaussians, per-pixel forward
    and backward, projection backward.  Returns Mpix/s and the sample size."""
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

    # calibrate: fixed cost (projection of every Gaussian) + per-pixel cost
    t1 = run(256)
    t2 = run(2048)
    per_px = max((t2 - t1) / (2048 - 256), 1e-7)
    fixed = max(t1 - 256 * per_px, 0.0)
    n = int(max(2048, min(2_000_000, (target_s - fixed) / per_px)))
    t = run(n)
    return n / t / 1e6, n, t


def serving(args):
    """Continuous-batching server (K = 64 with cell culling, and K = 1) against
    the one-view-at-a-time plain (K = 1) path on the same Poisson traces (first
    100 requests of each are warm-up)."""
    import torch

    from paper_2406_11836_amd import raster, scenes, serve

    t0 = time.perf_counter()
    p = scenes.scene_city_device(args.serve_n, seed=50, D=3)
    rast = raster.Rasterizer("cuda:0")
    kd64 = rast.kd_partition(p, 6)
    # resident layout: Gaussians grouped by cell, Morton order inside a cell
    p, _ = rast.group_by_cell(p, kd64)
    kd64 = rast.kd_partition(p, 6)
    kd1 = rast.kd_partition(p, 0, own_mask=False)
    torch.cuda.synchronize()
    prep_s = time.perf_counter() - t0
    out = {"metric": "serve p50/p99 ms & frames/s @100M splats K=64 vs plain path", "unit": "ms",
           "n_gpus": 1, "dtype": "f32", "data": "synthetic (device-generated aerial city)",
           "config": {"workload": "%d Gaussians SH3 resident (grouped by cell), K=64, Poisson requests, 40%% 1280x720 / 40%% "
                                  "1920x1080 / 20%% 3840x2160" % args.serve_n, "requests_per_rate": args.serve_requests,
                      "warmup_requests": 100},
           "scene_prep_s": round(prep_s, 2), "rates": {}}
    for rate in [float(x) for x in args.serve_rates.split(",")]:
        res = {}
        for name, kd, kw in (("batched", kd64, dict(max_batch=8, workers=1, cull=True)),
                             ("batched_K1", kd1, dict(max_batch=8, workers=1, cull=False)),
                             ("plain", kd1, dict(max_batch=1, workers=1, cull=False))):
            reqs = serve.serve_trace(rate, args.serve_requests, seed=int(30 + rate))
            torch.cuda.empty_cache()  # the previous server's buffers go back to the device
            srv = serve.Server(p, kd, **kw)
            srv.run(reqs)
            res[name] = serve.latency_stats(reqs, 100, srv)
            print("rate %g %s %s" % (rate, name, res[name]), file=sys.stderr, flush=True)
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--serve", action="store_true",
                    help="serving: 100M-Gaussian city resident in HBM, Poisson traces, continuous batching vs plain path")
    ap.add_argument("--serve-n", type=int, default=100_000_000)
    ap.add_argument("--serve-requests", type=int, default=2100)
    ap.add_argument("--serve-rates", type=str, default="50,200,800")
    ap.add_argument("--batched", action="store_true",
                    help="16-view batched step (4M Gaussians): one fused pass against 16 sequential passes, at K=16 and K=1")
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
        print(json.dumps(serving(args)))
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
    del st0

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    stage_ms = {}
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t_start.record()
    last = None
    for _ in range(args.steps):
        marks = []
        last = step(marks=marks)
        for (a, ea), (b, eb) in zip(marks[:-1], marks[1:]):
            if b in ("bwd_start",):
                continue
            stage_ms.setdefault(b, []).append((ea, eb))
    t_end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_step = t_start.elapsed_time(t_end) / args.steps
    if last[0].overflow():
        raise RuntimeError("instance capacity exceeded in a timed step")
    stages = {k: float(np.mean([ea.elapsed_time(eb) for ea, eb in v])) for k, v in stage_ms.items()}

    mpix = (W * H) / (ms_step * 1e-3) / 1e6
    # roofline of the dominant kernel: the partial-render backward (one kernel per
    # call of rgs_render_partial_bwd_records, timed by events on its stream)
    t_rb = stages["render_bwd"] * 1e-3
    flops_b = FLOP_BWD_EVAL_PAIR * nb_eval + FLOP_BWD_CONTRIB_PAIR * nb_con
    ach_b = flops_b / t_rb / 1e12
    roof = {"kernel": "k_render_bwd", "bound": "alu", "achieved": round(ach_b, 3),
            "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(ach_b / FP32_VECTOR_PEAK_TFLOPS, 4),
            "traffic": measured_traffic("k_render_bwd"), "algorithmic_flop": flops_b, "pairs_tested": nb_eval,
            "pairs_contributing": nb_con, "avg_ms": round(stages["render_bwd"], 4)}
    # the partial-render forward, for comparison
    t_rf = stages["render_fwd"] * 1e-3
    flops = FLOP_PER_EVAL_PAIR * n_eval + FLOP_PER_CONTRIB_PAIR * n_con
    achieved = flops / t_rf / 1e12
    roof_f = {"kernel": "k_render_fwd", "bound": "alu", "achieved": round(achieved, 3),
              "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4),
              "traffic": measured_traffic("k_render_fwd"), "algorithmic_flop": flops, "pairs_in_rect": n_eval,
              "pairs_contributing": n_con, "avg_ms": round(stages["render_fwd"], 4)}

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        v, npx, t = cpu_baseline(p, cam, L, args.cpu_seconds)
        cpu = {"value": round(v, 6), "unit": "Mpix/s", "cores": oracle.num_threads(), "kind": "oracle",
               "sample": "%d random pixels of the 1600x1060 view, fwd+bwd incl. projection of all 1M Gaussians "
                         "and its backward (loss excluded), %.1f s" % (npx, t)}

    out = {
        "metric": "fwd+bwd ms & Mpix/s @1M splats 1600x1060 K=8; serve p50/p99 ms vs plain path",
        "value": round(mpix, 3), "unit": "Mpix/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic (seeded clusters + ground plane scene, uniform-noise target)",
        "config": {"workload": "1M Gaussians SH3, 1600x1060, K=8 KD cells, L1+0.2(1-SSIM) fwd+bwd",
                   "gaussians": args.n, "width": W, "height": H, "cells": 1 << L, "eps_T": eps_T},
        "breakdown_ms": {k: round(v, 4) for k, v in stages.items()},
        "counts": {"visible_pairs": n_vis, "instances": n_inst, "slots": n_slots},
        "loss": round(float(lv0.item()), 6),
        "wall_s": round(wall, 3),
        "roofline": roof,
        "roofline_render_fwd": roof_f,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
