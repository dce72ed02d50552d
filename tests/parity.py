"""GPU-vs-oracle parity helpers shared by the GPU test modules.

Compositing is per pixel, so a discrete decision within rounding of its threshold
(a fragile pixel, flagged by the oracle) can only change that pixel's terms. The
upstream gradient is set to zero on the oracle's fragile pixels for both sides;
then every gradient and the statistic's S and M are compared on every Gaussian,
per element within 1e-3 relative (floor 1e-3 of the group's largest magnitude).
The fragment count C counts blended pairs whatever their gradient, so a flipped
decision at a fragile pixel may move it: the oracle returns, per Gaussian, the
number of fragile pixels at which its count may change (C_slack), and
|C_gpu - C| <= C_slack must hold on every Gaussian (exact equality where the
slack is zero).
"""
from __future__ import annotations

import numpy as np
import torch

import oracle as orc
from helpers import GRAD_TOL, IMAGE_TOL, grad_errors, image_errors, normwise
from paper_2503_01199_amd import scenes

GROUPS = ("means", "log_scales", "quats", "opacity_logits", "sh")


def upstream(scene, cams, salt=0, config=0):
    """dL/dI of the random-weighted L1 loss, from the oracle's image (so both sides
    receive identical upstream gradients), zero on the oracle's fragile pixels.
    Returns (gradients, oracle renders)."""
    gs, refs = [], []
    for v, cam in enumerate(cams):
        ref = orc.render(scene, cam, mode=1)
        w, gt = scenes.l1_weights((3, cam.height, cam.width), config=config, salt=salt + v)
        g = orc.l1_grad(ref["image"], w, gt).astype(np.float32)
        g[:, ref["fragile"]] = 0.0
        gs.append(g)
        refs.append(ref)
    return gs, refs


def run_gpu(rz, scene, cams, gI, cull=True, stats=None, precision=None):
    """Forward + backward on the GPU; returns (frame, gradients, statistic) with
    the gradients and statistic as numpy arrays."""
    from paper_2503_01199_amd import _lib as L
    from paper_2503_01199_amd.raster import SceneTensors, Workspace, new_stats
    print("gpu fwd+bwd n=%d views=%d cull=%s" % (scene.n, len(cams), cull), flush=True)
    st = SceneTensors.from_scene(scene, rz.device)
    fr = rz.forward(st, cams, cluster_cull=cull, workspace=Workspace(rz.device),
                    precision=L.GSR_FP32 if precision is None else precision)
    stats = stats if stats is not None else new_stats(scene.n, rz.device)
    grads = rz.backward(fr, [torch.as_tensor(g, device=rz.device) for g in gI], stats=stats)
    torch.cuda.synchronize()
    return fr, {k: v.cpu().numpy() for k, v in grads.items()}, {k: v.cpu().numpy() for k, v in stats.items()}


def oracle_sum(scene, cams, gI, threads=0):
    """The oracle's backward summed over views (fragile flags OR-ed)."""
    out = None
    for cam, g in zip(cams, gI):
        b = orc.backward(scene, cam, g.astype(np.float64), mode=1, threads=threads)
        if out is None:
            out = b
        else:
            for k in out:
                out[k] = out[k] | b[k] if k == "fragile" else out[k] + b[k]
    return out


def compare_images(fr, refs, what):
    for v, ref in enumerate(refs):
        err, over, nfrag = image_errors(fr.images[v].cpu().numpy(), ref["image"], ref["fragile"])
        print("%s view %d: image max rel %.3g over %d non-fragile pixels (%d fragile)"
              % (what, v, err, ref["fragile"].size - nfrag, nfrag))
        assert err <= IMAGE_TOL, (what, v, err)


def compare_counts(C_gpu, ref, what):
    C_gpu = np.asarray(C_gpu).astype(np.int64)
    d = np.abs(C_gpu - ref["C"])
    slack = ref["C_slack"]
    print("%s: fragment counts equal on %d of %d Gaussians; %d have slack (largest %d), largest |dC| %d"
          % (what, int((d == 0).sum()), d.size, int((slack > 0).sum()), int(slack.max()) if slack.size else 0,
             int(d.max()) if d.size else 0))
    bad = np.flatnonzero(d > slack)
    assert bad.size == 0, (what, bad[:8], C_gpu[bad[:8]], ref["C"][bad[:8]], slack[bad[:8]])


def compare(grads, stats, ref, what, logits=None):
    """Every gradient group and S, M per element on every Gaussian; C within the
    oracle's per-Gaussian slack."""
    none = np.zeros(ref["C"].shape, bool)
    for k in GROUPS:
        e = grad_errors(grads[k], ref[k], none)
        print("  %s %-15s max rel %.3g  normwise %.3g" % (what, k, e, normwise(grads[k], ref[k])))
        assert e <= GRAD_TOL, (what, k, e)
    for k in ("M", "S"):
        e = grad_errors(stats[k], ref[k], none)
        print("  %s statistic %s max rel %.3g" % (what, k, e))
        assert e <= GRAD_TOL, (what, k, e)
    compare_counts(stats["C"], ref, what)
    if logits is not None:
        # M is dL/do summed over fragments, so M o (1 - o) = dL/dlogit
        o = 1 / (1 + np.exp(-np.asarray(logits, np.float64)))
        assert grad_errors(stats["M"] * o * (1 - o), grads["opacity_logits"], none) <= 2 * GRAD_TOL


def gaussians(mean, log_scale, quat, opacity, rgb, degree=0):
    """Scene of the given Gaussians (FP32), colour set through the DC SH coefficient."""
    import math
    mean = np.atleast_2d(np.asarray(mean, np.float64))
    n = mean.shape[0]
    K = (degree + 1) ** 2
    sh = np.zeros((n, K, 3))
    sh[:, 0, :] = (np.atleast_2d(rgb) - 0.5) * (2.0 * math.sqrt(math.pi))
    op = np.atleast_1d(np.asarray(opacity, np.float64))
    logit = np.log(op / (1 - op))
    return scenes.Scene(*(np.ascontiguousarray(np.broadcast_to(a, s), np.float32) for a, s in
                          ((mean, (n, 3)), (log_scale, (n, 3)), (quat, (n, 4)), (logit, (n,)), (sh, (n, K, 3)))),
                        degree)


def camera(W=64, H=48, f=64.0, cx=None, cy=None, bg=(0, 0, 0), near=0.2):
    """Identity-pose pinhole camera looking down +z."""
    return scenes.Camera(W, H, f, f, W / 2 if cx is None else cx, H / 2 if cy is None else cy,
                         np.eye(3, dtype=np.float32), np.zeros(3, np.float32), near, bg)


def full_parity(rz, sc, cams, what, salt=0, cull=True):
    """Image, T and last blended position (non-fragile pixels), every gradient, S, M
    and C (within slack) of a small scene against the oracle. Returns the frame,
    the inspected buffers, the oracle renders and backward."""
    gI, refs = upstream(sc, cams, salt=salt)
    fr, grads, stats = run_gpu(rz, sc, cams, gI, cull=cull)
    compare_images(fr, refs, what)
    ins = rz.inspect(fr)
    T = ins["pixel_T"].cpu().numpy()
    for v, cam in enumerate(cams):
        r2 = orc.render(sc, cam, mode=2)
        keep = ~r2["fragile"]
        base = ins["pixel_base"][v]
        Tv = T[base:base + cam.width * cam.height].reshape(cam.height, cam.width)
        eT = np.abs(Tv - r2["T"])[keep].max()
        last = ins["pixel_last"].cpu().numpy().view(np.uint32)[base:base + cam.width * cam.height]
        lv = last.reshape(cam.height, cam.width)
        print("%s view %d: T max abs err %.3g, last blended position equal on %d of %d non-fragile pixels"
              % (what, v, eT, int((lv == r2["n_contrib"])[keep].sum()), int(keep.sum())))
        assert eT <= IMAGE_TOL
        assert np.array_equal(lv[keep], r2["n_contrib"][keep])
    ref = oracle_sum(sc, cams, gI)
    compare(grads, stats, ref, what, logits=sc.opacity_logits)
    return fr, ins, refs, ref
