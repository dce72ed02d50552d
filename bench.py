#!/usr/bin/env python3
"""Training-step benchmark of the MI355X differentiable Gaussian rasterizer.

One step is the hot path of a 3DGS training iteration on one view: cluster cull
and compaction, projection, depth sort, binning, tile sort, forward raster, the
weighted-L1 loss gradient, the backward raster with the opacity-gradient
statistic and the projection backward, all in the library's HIP kernels. The
scene is the synthetic 1M-Gaussian SH3 room at 1600x1064 (Morton-ordered once
beforehand, as a trainer does every few epochs; that reorder is timed separately).

    python bench.py [--gpus 1] [--steps K] [--warmup W]

prints one JSON line: ms per step (mean over K steps enqueued back to back), the
p50/p99 of single steps (200 after 20 warm-up, each alone on the device), per-stage
times, the roofline of the dominant kernel measured with HIP events on the
stream it runs on, the FP64 CPU reference timed on the same view, the FP16-blend
variant, the deterministic (fixed-point) backward, a 16-view cycle over the room
(one view per step, so that the scene does not stay resident in the 256 MB
Infinity Cache as it does for one repeated view),
the cluster-granular Adam step that follows the backward (over the kept clusters
and, for comparison, over all), whole training iterations with that step (as a
separate call and fused into the backward), a densification round (variance metric, split and
clone, opacity decay, Morton re-sort) and the render-serving stream (p50/p99
latency, views/s).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fwd+bwd raster ms/iter at 1M Gaussians 1600×1064; p50/p99 render latency"
# MI355X peaks: HBM3E 8 TB/s; FP32 vector 157.3 TFLOP/s (256 CUs x 4 SIMD x 16 lanes x
# 2.4 GHz x 2 flops per FMA x 2 for packed FP32).
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
# Algorithmic FLOPs of the raster per (pixel, Gaussian) evaluation up to the pixel's
# last blend (exponent 2 FMA, exp, alpha = min(0.99, o G)) and per blended fragment
# (forward: 1 - alpha, T', weight, 3 colour FMAs; backward: weight, 3 colour-gradient
# FMAs, 3 behind-colour FMAs, two 3-term dot products, 1 - alpha, reciprocal,
# dL/dalpha, g_o, dL/dE, the three scanline moments, the opacity sum, its square
# sum, the count and the transmittance update).
# HBM traffic per launch of the dominant kernel from rocprofv3 --pmc FETCH_SIZE and
# WRITE_SIZE runs of this bench (profiles/room-1M-1600x1064_raster_bwd_pmc.md), scaled
# by the same counters read on a plain 1 GiB device copy (FETCH_SIZE reads half of the
# bytes copied, WRITE_SIZE all of them). Valid only for the kernel sources the counters
# were taken on: any change to them makes the bench report traffic = null.
TRAFFIC = {"k_raster_bwd": {"workload": "room-1000k-SH3-1600x1064",
                            "sources": ["paper_2503_01199_amd/csrc/raster_bwd.hip",
                                        "paper_2503_01199_amd/csrc/raster_common.h",
                                        "paper_2503_01199_amd/csrc/gsr_internal.h"],
                            "sha1": "d4d70c5a30764955ca5c714cffa9055acc75b3e0",
                            "fetch_kib": 70280.3, "write_kib": 99531.2,
                            "valu_insts": 127987504, "valu_busy": 0.936, "valu_utilization": 0.7288}}
FETCH_SCALE = 1048576.0 / 524300.0
WRITE_SCALE = 1.0
FWD_FLOP_EVAL = 7
FWD_FLOP_FRAG = 9
BWD_FLOP_EVAL = 7
BWD_FLOP_FRAG = 41


def recorded_counters(kernel, workload):
    """The counters recorded for `kernel` on `workload`, or None when they were taken
    on another workload or its sources have changed since."""
    import hashlib
    t = TRAFFIC.get(kernel)
    if t is None or t["workload"] != workload:
        return None
    h = hashlib.sha1()
    for f in t["sources"]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return t if h.hexdigest() == t["sha1"] else None


def measured_traffic(kernel, workload):
    """HBM bytes per launch from the recorded FETCH_SIZE / WRITE_SIZE, or None."""
    t = recorded_counters(kernel, workload)
    if t is None:
        return None
    return int(round((t["fetch_kib"] * FETCH_SCALE + t["write_kib"] * WRITE_SCALE) * 1024))


def recorded_valu(kernel, workload):
    """VALU figures of the kernel from its recorded counters (rocprofv3 --pmc runs of
    this bench, same sources): wave instructions issued (SQ_INSTS_VALU) and VALU
    busy, the share of the SIMDs' cycles spent issuing VALU instructions while the
    GPU was active (rocprofv3's derived VALUBusy = SQ_ACTIVE_INST_VALU x 4 / SIMDs /
    GRBM_GUI_ACTIVE). Empty without a record."""
    t = recorded_counters(kernel, workload)
    if t is None:
        return {}
    return {k: t[k] for k in ("valu_insts", "valu_busy", "valu_utilization") if k in t}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def percentile(xs, p):
    s = sorted(xs)
    k = (len(s) - 1) * p / 100.0
    lo, hi = math.floor(k), math.ceil(k)
    return s[lo] + (s[hi] - s[lo]) * (k - lo)


def stage_bytes(info, st_n, sh_degree, views, pixels, stats=True):
    """Algorithmic HBM bytes of each stage of one step in this library's layouts (the
    bytes the stage must move once; re-reads, cache hits and atomics' read-modify-
    write traffic are not counted). R records = visible slots x views, M instances,
    T tiles, P pixels; parameter rows of pb = 4 (11 + 3K) bytes."""
    K = (sh_degree + 1) ** 2
    pb = 4 * (3 + 3 + 4 + 1 + 3 * K)
    nv = info["n_visible_slots"]
    R = nv * views
    M = info["instances"]
    T = info["tiles"]
    P = pixels
    nc = info["clusters"]
    tile_bits = max(1, int(math.ceil(math.log2(max(T, 2)))))
    passes = (tile_bits + 7) // 8
    return {
        # means and log-scales read; bounds (8 floats) and the flag written; the scan
        "cluster": st_n * 24 + nc * (32 + 4) + nc * 12,
        # visible clusters' parameter rows read (the compaction is fused); record,
        # depth key, tile count, rect, compact index and the zeroed gradient row written
        "preprocess": nv * pb + R * (48 + 4 + 4 + 8 + 48) + nv * 4,
        # 4 passes of 8 bits over (key, value): histogram read, then per pass the pair
        # read (keys only in the first) and written
        "depth_sort": R * 4 + R * (4 + 8) + 3 * R * 16,
        # index, gathered tile count and offset
        "offsets": R * 12,
        # per record its index, count, offset and rect; per instance (tile, record)
        "emit": R * 20 + M * 8,
        "tile_sort": M * 4 + passes * M * 16,
        "ranges": M * 4 + T * 8,
        # per instance its record index, record and band mask; per pixel image, T, last
        "raster_fwd": M * (4 + 48 + 4) + P * 20,
        # per instance index, record and mask; per pixel dL/dI, T, last
        "raster_bwd": M * (4 + 48 + 4) + P * 20,
        # parameter rows and screen gradient rows read, every parameter gradient
        # written, statistic read and written
        "preprocess_bwd": nv * pb + R * 48 + st_n * pb + (st_n * 24 if stats else 0),
    }


def step_roofline(stages, nbytes, work_fwd, work_bwd, l1_bytes, ms_per_step):
    """Roofline of the whole step: each stage's lower bound max(bytes / HBM peak,
    FLOPs / FP32 peak), summed over stages (and the loss-gradient kernel), over the
    measured step time. Also each stage's achieved GB/s and its own bound's fraction."""
    flops = {"raster_fwd": work_fwd, "raster_bwd": work_bwd}
    per = {}
    t_min = l1_bytes / (HBM_PEAK_GBS * 1e9)
    for k, b in nbytes.items():
        ms = stages.get(k)
        if ms is None or ms <= 0:
            continue
        tb = b / (HBM_PEAK_GBS * 1e9)
        tf = flops.get(k, 0) / (FP32_PEAK_TFLOPS * 1e12)
        t = max(tb, tf)
        t_min += t
        per[k] = {"ms": ms, "bytes": int(b), "GBs": round(b / (ms * 1e-3) / 1e9, 1),
                  "bound": "alu" if tf > tb else "hbm", "frac": round(t / (ms * 1e-3), 4)}
    return {"t_min_ms": round(t_min * 1e3, 4), "frac": round(t_min * 1e3 / ms_per_step, 4), "stages": per,
            "loss_grad_bytes": int(l1_bytes)}


def build_workload(name, n_override=None):
    from paper_2503_01199_amd import scenes
    if name == "room":
        sc = scenes.room_scene(n_override or 1_000_000)
        cams = [scenes.room_camera()]
        desc = "room-%dk-SH3-1600x1064" % (sc.n // 1000)
    elif name == "spheres":
        sc = scenes.spheres_planes_scene(n_override or 200_000)
        cams = [scenes.spheres_planes_camera()]
        desc = "spheres-%dk-SH3-800x800" % (sc.n // 1000)
    elif name == "unbounded":
        sc = scenes.unbounded_scene(n_override or 3_000_000)
        cams = scenes.orbit_cameras(8)
        desc = "unbounded-%dk-SH3-8x1920x1080" % (sc.n // 1000)
    elif name == "tiny":
        sc = scenes.tiny_scene(n_override or 1024)
        cams = [scenes.tiny_camera()]
        desc = "tiny-%d-SH0-128x128" % sc.n
    else:
        raise SystemExit("unknown workload %s" % name)
    return sc, cams, desc


ADAM_LR = {"means": 1.6e-4, "log_scales": 5e-3, "quats": 1e-3, "opacity_logits": 2.5e-2, "sh_dc": 2.5e-3,
           "sh_rest": 1.25e-4}


def adam_leg(rz, st, grads, visible, steps):
    """Cluster-granular Adam (Sec. 3.2.3) over the frame's kept clusters, and the
    dense update over every cluster for comparison: per-launch times from HIP events
    on the launch stream and the algorithmic HBM bytes (parameter, gradient and both
    moments read, parameter and moments written: 28 B per float of a row)."""
    import torch
    keys = ("means", "log_scales", "quats", "opacity_logits", "sh")
    params = {k: t.clone() for k, t in zip(keys, st.tensors())}
    m = {k: torch.zeros_like(t) for k, t in params.items()}
    v = {k: torch.zeros_like(t) for k, t in params.items()}
    row_floats = sum(t[0].numel() for t in params.values())
    kept = int(visible.to(torch.int64).sum().item())
    nc = visible.numel()
    full_rows = min(st.n, kept * 128) if kept < nc else st.n  # the last cluster may be partial
    out = {}
    for name, vis, rows in (("sparse", visible, full_rows), ("dense", None, st.n)):
        t = [0]

        def launch():
            t[0] += 1
            rz.sparse_adam(params, grads, m, v, vis, ADAM_LR, t[0])
        for _ in range(3):
            launch()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        for _ in range(steps):
            launch()
        b.record()
        b.synchronize()
        ms = a.elapsed_time(b) / steps
        nbytes = 28 * row_floats * rows
        out[name] = {"ms": round(ms, 4), "gaussians": rows, "bytes_per_launch": nbytes,
                     "achieved_GBs": round(nbytes / (ms * 1e-3) / 1e9, 1),
                     "frac": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    out["kept_clusters"] = kept
    out["clusters"] = nc
    out["bound"] = "hbm"
    out["peak_GBs"] = HBM_PEAK_GBS
    return out


def densify_leg(rz, st, stats, steps):
    """Densification round of Sec. 3.3 on the room: the variance metric of the
    statistic the timed steps accumulated, densification of the 5 % largest (half of
    them split: the split bound is the median largest log-scale), the Adam moments
    moved along, the opacity decay and the Morton re-sort of the grown scene. Per-call
    times from HIP events on the launch stream."""
    import torch
    n = st.n
    K = n // 20
    metric = rz.variance(stats["S"], stats["M"], stats["C"])
    split_ls = float(st.log_scales.max(dim=1).values.median().item())
    noise = torch.randn((n, 2, 3), device=rz.device, generator=torch.Generator(device=rz.device).manual_seed(3))
    state = {"exp_avg": torch.zeros_like(st.sh).view(n, -1), "exp_avg_sq": torch.zeros_like(st.sh).view(n, -1)}
    times = {"densify": [], "opacity_decay": [], "morton_resort": []}
    n_out = None
    for it in range(steps + 2):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        ev[0].record()
        grown, _, n_dev = rz.densify(st, metric, noise, 1e-12, K, split_ls, state=state, sync=False)
        ev[1].record()
        if n_out is None:  # the same every round: read once
            n_out = int(n_dev.item())
        cut = [t[:n_out] for t in grown.tensors()]
        ev[2].record()
        rz.opacity_decay(cut[3], 0.5)
        ev[3].record()
        e4 = torch.cuda.Event(enable_timing=True)
        e5 = torch.cuda.Event(enable_timing=True)
        e4.record()
        perm, _ = rz.morton_order(cut[0])
        rz.apply_permutation(perm, cut)
        e5.record()
        e5.synchronize()
        if it >= 2:
            times["densify"].append(ev[0].elapsed_time(ev[1]))
            times["opacity_decay"].append(ev[2].elapsed_time(ev[3]))
            times["morton_resort"].append(e4.elapsed_time(e5))
    out = {k: round(sorted(v)[len(v) // 2], 4) for k, v in times.items()}
    out.update({"n": n, "candidates": K, "n_out": n_out, "state_arrays": 2, "reps": steps})
    return out


def cpu_baseline(scene, cam, repeats, threads, gpu_forms=None):
    """The FP64 oracle's forward + backward of the whole view (the same scene, camera
    and loss as the GPU step; the loss gradient is zeroed on the pixels the oracle
    flags as fragile), timed `repeats` times; the median is reported. With gpu_forms
    (a callable taking that upstream gradient and returning, per GPU form, its image
    and parameter gradients), the error of each form against the oracle's last run:
    image max abs and normwise on non-fragile pixels; per gradient group normwise and
    the largest element error relative to max(|g*|, 1e-3 of the group's largest)."""
    import numpy as np
    import oracle
    from paper_2503_01199_amd import scenes
    oracle.load()
    H, W = cam.height, cam.width
    w, gt = scenes.l1_weights((3, H, W), config=2)
    times = []
    for _ in range(repeats):
        t = time.perf_counter()
        r = oracle.render(scene, cam, mode=1, threads=threads)
        g = oracle.l1_grad(r["image"], w, gt)
        g[:, r["fragile"]] = 0.0
        b = oracle.backward(scene, cam, g, mode=1, threads=threads)
        times.append(time.perf_counter() - t)
    med = sorted(times)[len(times) // 2]
    out = {"value": round(med * 1e3, 1), "unit": "ms/iter", "cores": threads, "kind": "oracle",
           "sample": "FP64 oracle forward + backward of the whole %dx%d view, median of %d runs (%s s)"
                     % (W, H, repeats, ", ".join("%.2f" % x for x in times))}
    errors = None
    if gpu_forms is not None:
        keep = ~r["fragile"]
        errors = {}
        for name, (img, grads) in gpu_forms(g.astype(np.float32)).items():
            d = (np.asarray(img, np.float64) - r["image"])[:, keep]
            e = {"image_max_abs": float(np.abs(d).max()),
                 "image_normwise": float(np.linalg.norm(d) / max(np.linalg.norm(r["image"][:, keep]), 1e-30))}
            for k, ga in grads.items():
                ref = b[k].reshape(ga.shape[0], -1)
                gg = np.asarray(ga, np.float64).reshape(ref.shape)
                floor = 1e-3 * max(np.abs(ref).max(), 1e-30)
                e[k + "_normwise"] = float(np.linalg.norm(gg - ref) / max(np.linalg.norm(ref), 1e-30))
                e[k + "_max_rel"] = float((np.abs(gg - ref) / np.maximum(np.abs(ref), floor)).max())
            errors[name] = {k: float("%.3g" % v) for k, v in e.items()}
        errors["pixels"] = int(keep.sum())
        errors["fragile_pixels"] = int((~keep).sum())
    return out, errors


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--latency-iters", type=int, default=200,
                    help="steps timed one at a time (after 20 warm-up steps) for p50/p99")
    ap.add_argument("--cycle-views", type=int, default=16,
                    help="views of the room cycled through, one per step (0 skips; room workload only)")
    ap.add_argument("--workload", default="room", choices=["room", "spheres", "unbounded", "tiny"])
    ap.add_argument("--n", type=int, default=None, help="override the Gaussian count (testing only)")
    ap.add_argument("--no-cull", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-repeats", type=int, default=5)
    ap.add_argument("--no-serving", action="store_true", help="skip the render-serving stream")
    ap.add_argument("--no-adam", action="store_true", help="skip the cluster-granular Adam leg")
    ap.add_argument("--no-densify", action="store_true", help="skip the densification round")
    ap.add_argument("--schedule-sweep", action="store_true",
                    help="also time the rasters over a sweep of the band-split thresholds")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 1 GiB device to device 3 times (scales the FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--serve-requests", type=int, default=3000)
    ap.add_argument("--serve-rates", default="200,1000,3000",
                    help="arrival rates (req/s) of the serving sweep; the first is the reported stream")
    ap.add_argument("--order", default="morton", choices=["morton", "shuffled"],
                    help="Gaussian order of the scene (shuffled: a random permutation, for cache counters)")
    ap.add_argument("--only-steps", action="store_true",
                    help="warm up, time the steps and stop (for profiler runs)")
    ap.add_argument("--tile-width", type=int, default=0, choices=[0, 4, 8, 16, 32, 64],
                    help="with --only-steps: tiles of 256 pixels this wide (0: 16x16)")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp16", "fp16t"],
                    help="blend precision of the steps of an --only-steps run")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (got --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2503_01199_amd import scenes
    from paper_2503_01199_amd.raster import Rasterizer, SceneTensors, Workspace, new_stats

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a HIP device")
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": src.numel() * 4, "copies": 3}), flush=True)
        return
    log("generating workload %s" % args.workload)
    scene, cams, desc = build_workload(args.workload, args.n)
    cam = cams[0]
    rz = Rasterizer(0)
    dev = rz.device
    st = SceneTensors.from_scene(scene, dev)

    # Morton reorder (Sec. 3.2.1), amortised over epochs: timed on its own
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    perm, _ = rz.morton_order(st.means)
    arrays = rz.apply_permutation(perm, list(st.tensors()))
    t1.record()
    torch.cuda.synchronize()
    morton_cold_ms = t0.elapsed_time(t1)
    # warm: the same reorder again (workspaces in place), median of 10
    warm = []
    for _ in range(0 if args.only_steps else 10):
        t0.record()
        perm, _ = rz.morton_order(st.means)
        arrays = rz.apply_permutation(perm, list(st.tensors()))
        t1.record()
        t1.synchronize()
        warm.append(t0.elapsed_time(t1))
    morton_ms = sorted(warm)[len(warm) // 2] if warm else morton_cold_ms
    if args.order == "shuffled":
        perm = torch.randperm(st.n, device=dev, generator=torch.Generator(device=dev).manual_seed(1))
        arrays = rz.apply_permutation(perm, list(st.tensors()))
    st = SceneTensors(*arrays, st.sh_degree)
    scene_sorted = scene.permuted(perm.cpu().numpy())

    wgt = []
    for v, c in enumerate(cams):
        w_np, gt_np = scenes.l1_weights((3, c.height, c.width), config=2, salt=v)
        wgt.append((torch.as_tensor(w_np, device=dev), torch.as_tensor(gt_np, device=dev)))
    ws = Workspace(dev)
    stats = new_stats(st.n, dev)
    dls = [torch.empty((3, c.height, c.width), dtype=torch.float32, device=dev) for c in cams]
    grads = {k: torch.empty_like(t) for k, t in zip(("means", "log_scales", "quats", "opacity_logits", "sh"),
                                                     st.tensors())}
    cull = not args.no_cull

    from paper_2503_01199_amd import _lib as L

    def step(check=False, precision=L.GSR_FP32, deterministic=False, radius_mode=0, half_reduction=False,
             tile_width=0):
        fr = rz.forward(st, cams, cluster_cull=cull, workspace=ws, check=check, precision=precision,
                        deterministic=deterministic, radius_mode=radius_mode, half_reduction=half_reduction,
                        tile_width=tile_width)
        for img, (w, gt), dl in zip(fr.images, wgt, dls):
            rz.l1_grad(img, w, gt, out=dl)
        rz.backward(fr, dls, grads=grads, stats=stats)
        return fr

    log("warmup %d steps" % args.warmup)
    tw0 = args.tile_width if args.only_steps else 0
    fr = step(check=True, tile_width=tw0)  # sizes the workspace for this frame's instance count
    for _ in range(max(args.warmup - 1, 0)):
        fr = step(tile_width=tw0)
    torch.cuda.synchronize()

    if args.only_steps:  # profiler runs: the timed steps only
        prec = {"fp32": L.GSR_FP32, "fp16": L.GSR_FP16_BLEND, "fp16t": L.GSR_FP16_BLEND_T}[args.precision]
        torch.cuda.synchronize()
        wall0 = time.perf_counter()
        for _ in range(args.steps):
            fr = step(precision=prec, tile_width=tw0)
        torch.cuda.synchronize()
        info = rz.check_frame(fr)
        print(json.dumps({"workload": desc, "order": args.order, "cluster_cull": cull, "precision": args.precision,
                          "ms_per_step":
                          round((time.perf_counter() - wall0) * 1e3 / args.steps, 4), "steps": args.steps,
                          "frames": 1 + max(args.warmup - 1, 0) + args.steps,
                          "instances": info["instances"]}), flush=True)
        return

    # algorithmic work of one step, from the frame state (outside the timed region)
    ins = rz.inspect(fr)
    E = int(ins["pixel_last"].to(torch.int64).sum().item())
    stats1 = new_stats(st.n, dev)
    rz.backward(fr, dls, grads=grads, stats=stats1)
    torch.cuda.synchronize()
    F = int(stats1["C"].to(torch.int64).sum().item())
    info = dict(ins["info"])

    # timed region: K whole steps enqueued back to back (no host wait inside a step)
    log("timing %d steps" % args.steps)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    for _ in range(args.steps):
        fr = step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    rz.check_frame(fr)  # the frame's instances fitted the workspace
    ms_per_step = wall * 1e3 / args.steps

    # per-step latency: each step alone on the device, timed by events around it
    log("latency over %d single steps" % args.latency_iters)
    for _ in range(20):
        step()
    torch.cuda.synchronize()
    times = []
    for _ in range(args.latency_iters):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        step()
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b))

    # per-stage times (HIP events on the launch stream), in a separate pass because
    # the per-stage events and waits cost time of their own
    log("profiling %d steps" % args.steps)
    rz.set_profiling(True)
    stage_acc = {}
    for _ in range(args.steps):
        step()
        for k, v in rz.stage_times().items():
            if v >= 0:
                stage_acc.setdefault(k, []).append(v)
    rz.set_profiling(False)
    stages = {k: round(sum(v) / len(v), 4) for k, v in stage_acc.items()}

    # the packed-FP16 blend variant (Sec. 3.1.2) on the same workload and protocol
    log("timing %d FP16-blend steps" % args.steps)
    for _ in range(max(args.warmup, 1)):
        step(precision=L.GSR_FP16_BLEND)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    for _ in range(args.steps):
        fr16 = step(precision=L.GSR_FP16_BLEND)
    torch.cuda.synchronize()
    fp16_ms = (time.perf_counter() - wall0) * 1e3 / args.steps
    rz.check_frame(fr16)
    rz.set_profiling(True)
    acc16 = {}
    for _ in range(args.steps):
        step(precision=L.GSR_FP16_BLEND)
        for k, v in rz.stage_times().items():
            if v >= 0:
                acc16.setdefault(k, []).append(v)
    rz.set_profiling(False)
    st16 = {k: round(sum(v) / len(v), 4) for k, v in acc16.items()}
    fp16 = {"ms_per_step": round(fp16_ms, 4), "raster_fwd_ms": st16.get("raster_fwd"),
            "raster_bwd_ms": st16.get("raster_bwd")}

    # the FP16 blend with the forward's T in FP16 as well, same protocol
    log("timing %d FP16-T steps" % args.steps)
    for _ in range(max(args.warmup, 1)):
        step(precision=L.GSR_FP16_BLEND_T)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    for _ in range(args.steps):
        fr16t = step(precision=L.GSR_FP16_BLEND_T)
    torch.cuda.synchronize()
    fp16t_ms = (time.perf_counter() - wall0) * 1e3 / args.steps
    rz.check_frame(fr16t)
    rz.set_profiling(True)
    acc16t = {}
    for _ in range(args.steps):
        step(precision=L.GSR_FP16_BLEND_T)
        for k, v in rz.stage_times().items():
            if v >= 0:
                acc16t.setdefault(k, []).append(v)
    rz.set_profiling(False)
    st16t = {k: round(sum(v) / len(v), 4) for k, v in acc16t.items()}
    fp16t = {"ms_per_step": round(fp16t_ms, 4), "raster_fwd_ms": st16t.get("raster_fwd"),
             "raster_bwd_ms": st16t.get("raster_bwd")}

    # the deterministic backward (fixed-point per-tile sums) on the same protocol
    log("timing %d deterministic steps" % args.steps)
    step(check=True, deterministic=True)  # grows the workspace by the fixed-point rows
    for _ in range(max(args.warmup, 1)):
        step(deterministic=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    for _ in range(args.steps):
        step(deterministic=True)
    torch.cuda.synchronize()
    det_ms = (time.perf_counter() - wall0) * 1e3 / args.steps
    rz.set_profiling(True)
    accd = {}
    for _ in range(args.steps):
        step(deterministic=True)
        for k, v in rz.stage_times().items():
            if v >= 0:
                accd.setdefault(k, []).append(v)
    rz.set_profiling(False)
    std = {k: round(sum(v) / len(v), 4) for k, v in accd.items()}
    det = {"ms_per_step": round(det_ms, 4), "raster_bwd_ms": std.get("raster_bwd"),
           "zero_grad_ms": std.get("zero_grad")}

    # the half2-packed colour/opacity gradient reduction (Sec. 3.1.2), same protocol
    log("timing %d steps with the half2 gradient reduction" % args.steps)
    step(check=True, half_reduction=True)
    for _ in range(max(args.warmup, 1)):
        step(half_reduction=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    for _ in range(args.steps):
        step(half_reduction=True)
    torch.cuda.synchronize()
    h_ms = (time.perf_counter() - wall0) * 1e3 / args.steps
    rz.set_profiling(True)
    acch = {}
    for _ in range(args.steps):
        step(half_reduction=True)
        for k, v in rz.stage_times().items():
            if v >= 0:
                acch.setdefault(k, []).append(v)
    rz.set_profiling(False)
    sth = {k: round(sum(v) / len(v), 4) for k, v in acch.items()}
    half_red = {"ms_per_step": round(h_ms, 4), "raster_bwd_ms": sth.get("raster_bwd"),
                "preprocess_bwd_ms": sth.get("preprocess_bwd")}

    # the 3-sigma tile-membership bound instead of the exact alpha >= 1/255 box (a
    # different image: every pixel of a covered tile, and only those, evaluates the
    # Gaussian), same protocol
    log("timing %d steps with the 3-sigma bound" % args.steps)
    fr3 = step(check=True, radius_mode=1)
    inst3 = int(fr3.info["instances"])
    for _ in range(max(args.warmup, 1)):
        step(radius_mode=1)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    for _ in range(args.steps):
        fr3 = step(radius_mode=1)
    torch.cuda.synchronize()
    r3_ms = (time.perf_counter() - wall0) * 1e3 / args.steps
    rz.check_frame(fr3)
    rz.set_profiling(True)
    acc3 = {}
    for _ in range(args.steps):
        step(radius_mode=1)
        for k, v in rz.stage_times().items():
            if v >= 0:
                acc3.setdefault(k, []).append(v)
    rz.set_profiling(False)
    st3 = {k: round(sum(v) / len(v), 4) for k, v in acc3.items()}
    radius3 = {"ms_per_step": round(r3_ms, 4), "instances": inst3, "stages_ms": st3}
    step(check=True)  # back to the default bound's frame

    # tile shapes of 256 pixels other than 16x16 (F4): 4x64, 8x32, 32x8 and 64x4
    # tiles, one wave64 per tile with 4 pixels per lane, same protocol
    shapes = {}
    for tw in (4, 8, 32, 64):
        log("timing %d steps with %dx%d tiles" % (args.steps, tw, 256 // tw))
        frs = step(check=True, tile_width=tw)
        inst_s = int(frs.info["instances"])
        for _ in range(max(args.warmup, 1)):
            step(tile_width=tw)
        torch.cuda.synchronize()
        wall0 = time.perf_counter()
        for _ in range(args.steps):
            frs = step(tile_width=tw)
        torch.cuda.synchronize()
        s_ms = (time.perf_counter() - wall0) * 1e3 / args.steps
        rz.check_frame(frs)
        rz.set_profiling(True)
        accs = {}
        for _ in range(args.steps):
            step(tile_width=tw)
            for k, v in rz.stage_times().items():
                if v >= 0:
                    accs.setdefault(k, []).append(v)
        rz.set_profiling(False)
        sts = {k: round(sum(v) / len(v), 4) for k, v in accs.items()}
        shapes["%dx%d" % (tw, 256 // tw)] = {"ms_per_step": round(s_ms, 4), "instances": inst_s,
                                             "raster_fwd_ms": sts.get("raster_fwd"),
                                             "raster_bwd_ms": sts.get("raster_bwd"),
                                             "tile_sort_ms": sts.get("tile_sort"), "emit_ms": sts.get("emit")}
    step(check=True)  # back to 16x16 tiles

    # raster schedule sweep (F4): the list length above which a tile is rastered as
    # band items, 1 pixel per lane in the forward's four 16x4 bands, 2 in the
    # backward's halves, against whole 16x16 tiles with 4 pixels per lane
    sweep = None
    if args.schedule_sweep:
        never = 0xffffffff
        sweep = {"forward": {}, "backward": {}}
        for key, settings in (("forward", [(never, 0), (1024, 0), (512, 0), (256, 0), (128, 0), (64, 0), (0, 0)]),
                              ("backward", [(0, never), (0, 1024), (0, 512), (0, 256), (0, 128)])):
            for fl, bl in settings:
                rz.set_raster_split(fl, bl)
                step(check=True)
                rz.set_profiling(True)
                acc = {}
                for _ in range(min(args.steps, 20)):
                    f_ = step()
                    for k, v in rz.stage_times().items():
                        if v >= 0:
                            acc.setdefault(k, []).append(v)
                rz.set_profiling(False)
                inf = rz.inspect(f_)["info"]
                stage = "raster_fwd" if key == "forward" else "raster_bwd"
                thr = fl if key == "forward" else bl
                name = "never" if thr == never else ("default" if thr == 0 else str(thr))
                sweep[key][name] = {"ms": round(sorted(acc[stage])[len(acc[stage]) // 2], 4),
                                    "split_tiles": inf["split_tiles" if key == "forward" else "split_tiles_bwd"]}
        rz.set_raster_split(0, 0)

    # a cycle over views of the room, one per step, so that no view's working set
    # stays resident in the caches as it does when one view repeats
    cycle = None
    if args.workload == "room" and args.cycle_views > 0:
        ccams = scenes.room_cycle_cameras(args.cycle_views)
        log("timing a %d-view cycle" % len(ccams))

        def cstep(c, check=False):
            f = rz.forward(st, [c], cluster_cull=cull, workspace=ws, check=check)
            rz.l1_grad(f.images[0], *wgt[0], out=dls[0])
            rz.backward(f, [dls[0]], grads=grads, stats=stats)
            return f

        inst = []
        for c in ccams:  # sizes the workspace for every view of the cycle
            inst.append(rz.inspect(cstep(c, check=True))["info"]["instances"])
        torch.cuda.synchronize()
        nsteps = 2 * len(ccams)
        wall0 = time.perf_counter()
        for i in range(nsteps):
            frc = cstep(ccams[i % len(ccams)])
        torch.cuda.synchronize()
        cyc_ms = (time.perf_counter() - wall0) * 1e3 / nsteps
        rz.check_frame(frc)
        cycle = {"views": len(ccams), "steps": nsteps, "ms_per_step": round(cyc_ms, 4),
                 "instances_min": int(min(inst)), "instances_max": int(max(inst)),
                 "instances_mean": int(sum(inst) / len(inst))}

    # the optimiser step that follows the backward (not part of the metric's step)
    adam = None
    if not args.no_adam:
        log("timing the cluster-granular Adam step")
        fr = step()  # the room view's frame again (the legs above reused the workspace)
        ins = rz.inspect(fr)
        adam = adam_leg(rz, st, grads, ins["cluster_visible"][: ins["info"]["clusters"]].clone(), args.steps)

    # whole training iterations (forward, loss gradient, backward, Adam over the kept
    # clusters), steps enqueued back to back: the backward and the Adam step as two
    # calls, and fused (gsr_backward_adam: no gradient array is written or read)
    train = None
    if not args.no_adam:
        log("timing training iterations with the Adam step")
        keys = ("means", "log_scales", "quats", "opacity_logits", "sh")
        tp = SceneTensors(*[t.clone() for t in st.tensors()], st.sh_degree)
        mom = [{k: torch.zeros_like(t) for k, t in zip(keys, tp.tensors())} for _ in range(2)]
        fr_t = rz.forward(tp, cams, cluster_cull=cull, workspace=ws, check=True)
        vis_view = rz.inspect(fr_t)["cluster_visible"][: fr_t.info["clusters"]]  # the workspace's flags, live
        counter = [0]

        def train_iter(fused):
            counter[0] += 1
            f_ = rz.forward(tp, cams, cluster_cull=cull, workspace=ws, check=False)
            for img, (w, gt), dl in zip(f_.images, wgt, dls):
                rz.l1_grad(img, w, gt, out=dl)
            if fused:
                rz.backward_adam(f_, dls, mom[0], mom[1], ADAM_LR, counter[0], stats=stats)
            else:
                rz.backward(f_, dls, grads=grads, stats=stats)
                rz.sparse_adam(dict(zip(keys, tp.tensors())), grads, mom[0], mom[1], vis_view, ADAM_LR, counter[0])
            return f_
        train = {}
        for name, fused in (("two_calls", False), ("fused", True)):
            for _ in range(3):
                train_iter(fused)
            torch.cuda.synchronize()
            wall0 = time.perf_counter()
            for _ in range(args.steps):
                f_ = train_iter(fused)
            torch.cuda.synchronize()
            train[name + "_ms"] = round((time.perf_counter() - wall0) * 1e3 / args.steps, 4)
            rz.check_frame(f_)

    dens = None
    if not args.no_densify:
        log("timing a densification round")
        dens = densify_leg(rz, st, stats, min(args.steps, 10))

    # roofline of the dominant kernel (each stage below is one kernel launch)
    dom = max(("raster_bwd", "raster_fwd", "preprocess_bwd", "preprocess"), key=lambda k: stages.get(k, 0.0))
    roof_kernel = {"raster_bwd": "k_raster_bwd", "raster_fwd": "k_raster_fwd", "preprocess_bwd": "k_sh_bwd",
                   "preprocess": "k_preprocess_fwd"}[dom]
    dur_s = stages[dom] * 1e-3
    if dom == "raster_bwd":
        work = BWD_FLOP_EVAL * E + BWD_FLOP_FRAG * F
        roof = {"bound": "alu", "achieved": round(work / dur_s / 1e12, 3), "peak": FP32_PEAK_TFLOPS,
                "unit": "TFLOP/s"}
    elif dom == "raster_fwd":
        work = FWD_FLOP_EVAL * E + FWD_FLOP_FRAG * F
        roof = {"bound": "alu", "achieved": round(work / dur_s / 1e12, 3), "peak": FP32_PEAK_TFLOPS,
                "unit": "TFLOP/s"}
    else:
        K = (st.sh_degree + 1) ** 2
        pbytes = 4 * (3 + 3 + 4 + 1 + 3 * K)
        nvis = info["n_visible_slots"]
        if dom == "preprocess_bwd":
            work = st.n * pbytes + nvis * (pbytes + 48 + 4) + st.n * 12
        else:
            work = nvis * (pbytes + 48 + 4 + 4 + 8 + 4)
        roof = {"bound": "hbm", "achieved": round(work / dur_s / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    roof["frac"] = round(roof["achieved"] / roof["peak"], 4)
    roof["traffic"] = measured_traffic(roof_kernel, desc)
    roof.update(recorded_valu(roof_kernel, desc))
    roof["kernel"] = roof_kernel
    roof["launch_ms"] = stages[dom]
    roof["work_per_launch"] = work
    pixels = sum(c.width * c.height for c in cams)
    nbytes = stage_bytes(info, st.n, st.sh_degree, len(cams), pixels)
    step_roof = step_roofline(stages, nbytes, FWD_FLOP_EVAL * E + FWD_FLOP_FRAG * F,
                              BWD_FLOP_EVAL * E + BWD_FLOP_FRAG * F, 48 * pixels, ms_per_step)

    serving = None
    if not args.no_serving:
        from paper_2503_01199_amd.serve import serve_benchmark
        rates = [float(r) for r in args.serve_rates.split(",") if r.strip()]
        # the first rate is the reported stream; the others go past capacity
        serving = serve_benchmark(rz, n_warmup=200, n_measured=args.serve_requests, rate=rates[0], log=log,
                                  more_rates=tuple(rates[1:]))

    cpu = None
    err_report = None
    if not args.no_cpu_baseline and len(cams) == 1:
        threads = min(16, os.cpu_count() or 1)
        log("timing the FP64 oracle on the whole view, %d runs on %d threads" % (args.cpu_repeats, threads))

        def gpu_forms(g):
            """The GPU path's image and gradients for the oracle's upstream gradient, per
            form: FP32, the FP16 blend, the FP16 blend with FP16 T, the half2 reduction."""
            gd = torch.as_tensor(g, device=dev)
            res = {}
            for name, prec, half in (("fp32", L.GSR_FP32, False), ("fp16_blend", L.GSR_FP16_BLEND, False),
                                     ("fp16_blend_t", L.GSR_FP16_BLEND_T, False),
                                     ("half_reduction", L.GSR_FP32, True)):
                f_ = rz.forward(st, cams, cluster_cull=cull, workspace=ws, precision=prec, half_reduction=half)
                gr = rz.backward(f_, [gd])
                torch.cuda.synchronize()
                res[name] = (f_.images[0].cpu().numpy(), {k: v.cpu().numpy() for k, v in gr.items()})
            return res
        cpu, err_report = cpu_baseline(scene_sorted, cam, args.cpu_repeats, threads, gpu_forms)
        cpu["host_cpus"] = os.cpu_count()
        cpu["cpu_model"] = cpu_model()

    out = {
        "metric": METRIC,
        "value": round(ms_per_step, 4),
        "unit": "ms/iter",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "gaussians": st.n, "sh_degree": st.sh_degree, "views": len(cams),
                   "width": cam.width, "height": cam.height, "precision": "fp32", "cluster_cull": cull,
                   "morton_ordered": True},
        "p50_ms": round(percentile(times, 50), 4),
        "p99_ms": round(percentile(times, 99), 4),
        "stages_ms": stages,
        "morton_reorder_ms": round(morton_ms, 3),
        "morton_reorder_cold_ms": round(morton_cold_ms, 3),
        "frame": {"visible_slots": info["n_visible_slots"], "instances": info["instances"],
                  "evaluations_E": E, "fragments_F": F, "tiles": info["tiles"]},
        "fp16_blend": fp16,
        "fp16_blend_t": fp16t,
        "deterministic": det,
        "radius_3sigma": radius3,
        "tile_shapes": shapes,
        "half_reduction": half_red,
        "schedule_sweep": sweep,
        "view_cycle": cycle,
        "sparse_adam": adam,
        "train_iteration": train,
        "densify": dens,
        "serving": serving,
        "roofline": roof,
        "step_roofline": step_roof,
        "cpu_baseline": cpu,
        "error_vs_oracle": err_report,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
