"""Shared helpers of the test suite: tolerances, scene conversion and record decoding."""
from __future__ import annotations

import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# Floating-point parity bars (the image bar is relative with a floor of 1 because
# image values are O(1); the gradient bar is per parameter group with a floor of
# 1e-3 of the group's largest gradient, so tiny gradients compare absolutely).
IMAGE_TOL = 1e-5
GRAD_TOL = 1e-3
GRAD_FLOOR = 1e-3


def ensure_built():
    """Builds libgsr.so if it is missing (tests never rebuild an existing library)."""
    lib = os.path.join(ROOT, "paper_2503_01199_amd", "libgsr.so")
    if not os.path.exists(lib):
        subprocess.check_call([sys.executable, "-m", "paper_2503_01199_amd.build"], cwd=ROOT)
    return lib


def image_errors(img, ref, fragile):
    """Per-pixel |I - I*| / max(1, |I*|) over non-fragile pixels; returns (max, count of
    pixels over the bar, fragile pixel count)."""
    img = np.asarray(img, np.float64)
    ref = np.asarray(ref, np.float64)
    keep = ~np.asarray(fragile, bool)
    err = np.abs(img - ref) / np.maximum(1.0, np.abs(ref))
    err = err[:, keep]
    return float(err.max()) if err.size else 0.0, int((err > IMAGE_TOL).sum()), int((~keep).sum())


def grad_errors(g, ref, skip):
    """max over elements of |g - g*| / max(|g*|, floor * max|g*|) on Gaussians not in skip."""
    g = np.asarray(g, np.float64).reshape(len(skip), -1)
    ref = np.asarray(ref, np.float64).reshape(len(skip), -1)
    keep = ~np.asarray(skip, bool)
    if not keep.any():
        return 0.0
    floor = GRAD_FLOOR * max(np.abs(ref[keep]).max(), 1e-30)
    err = np.abs(g[keep] - ref[keep]) / np.maximum(np.abs(ref[keep]), floor)
    return float(err.max())


def normwise(g, ref):
    g = np.asarray(g, np.float64).ravel()
    ref = np.asarray(ref, np.float64).ravel()
    return float(np.linalg.norm(g - ref) / max(np.linalg.norm(ref), 1e-30))


def decode_records(rec):
    """Screen mean (FP64 from the float-float pair) and conic (a, b, c) from records
    f32[R,12] = (u_hi, v_hi, u_lo, v_lo, k1, r, k2, quad4, o, rgb): the exponent in log2
    units is k1 (dx + r dy)^2 + k2 dy^2 = -log2(e)/2 (a dx^2 + 2 b dx dy + c dy^2), and
    quad4 is a quarter of its coefficient of dy^2, -log2(e) c / 8."""
    rec = np.asarray(rec, np.float64)
    u = rec[:, 0] + rec[:, 2]
    v = rec[:, 1] + rec[:, 3]
    ln2 = np.log(2.0)
    a = -2.0 * ln2 * rec[:, 4]
    b = a * rec[:, 5]
    c = -8.0 * ln2 * rec[:, 7]
    return u, v, np.stack([a, b, c], 1), rec[:, 8], rec[:, 9:12]
