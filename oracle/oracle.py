"""ctypes wrapper of the FP64 oracle (``gs_oracle.cpp``). Test infrastructure.

Scenes and cameras are taken by duck typing (attributes ``means``, ``log_scales``,
``quats``, ``opacity_logits``, ``sh``, ``sh_degree``; ``width``, ``height``, ``fx``,
``fy``, ``cx``, ``cy``, ``R``, ``t``, ``near``, ``bg``), so this module imports
nothing from the GPU package.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gs_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

__all__ = ["build", "load", "camera_array", "sh_basis", "preprocess", "render", "backward", "chain",
           "morton", "cluster_bounds", "bin_instances", "count_instances", "variance", "l1_grad",
           "l1_loss", "ADAM_GROUPS", "sparse_adam", "quat_to_rotation", "densify", "opacity_decay"]


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (FP64, no FMA contraction) into liboracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-pthread",
                               "-ffp-contract=off", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = ctypes.CDLL(_LIB)
        _lib.orc_count_instances.restype = ctypes.c_int64
        _lib.orc_bin.restype = ctypes.c_int64
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _scene_args(scene):
    arrs = [np.ascontiguousarray(x, dtype=np.float32) for x in
            (scene.means, scene.log_scales, scene.quats, scene.opacity_logits, scene.sh)]
    return arrs, [ctypes.c_int64(arrs[0].shape[0]), ctypes.c_int(int(scene.sh_degree))] + [_p(a) for a in arrs]


def camera_array(cam, radius_mode: int = 0, tile_width: int = 0) -> np.ndarray:
    """24 doubles: W, H, fx, fy, cx, cy, R (9, row-major), t (3), near, bg (3), the
    tile-membership bound (0: the alpha >= 1/255 ellipse's box, 1: the 3-sigma
    square) and the tile width in pixels (4, 8, 16, 32 or 64, the height 256 / width;
    0: 16). The float fields are rounded to FP32 first, exactly as the GPU library
    receives them."""
    if tile_width not in (0, 4, 8, 16, 32, 64):
        raise ValueError("tile_width must be 0, 4, 8, 16, 32 or 64")
    f32 = lambda x: float(np.float32(x))  # noqa: E731
    R = np.asarray(cam.R, dtype=np.float32).reshape(9).astype(np.float64)
    t = np.asarray(cam.t, dtype=np.float32).reshape(3).astype(np.float64)
    bg = np.asarray(cam.bg, dtype=np.float32).reshape(3).astype(np.float64)
    out = np.array([cam.width, cam.height, f32(cam.fx), f32(cam.fy), f32(cam.cx), f32(cam.cy)]
                   + list(R) + list(t) + [f32(cam.near)] + list(bg) + [int(radius_mode), int(tile_width)],
                   dtype=np.float64)
    return out


def sh_basis(deg: int, direction):
    lib = load()
    K = (deg + 1) ** 2
    d = np.ascontiguousarray(direction, dtype=np.float64)
    Y = np.zeros(K)
    dY = np.zeros((K, 3))
    lib.orc_sh_basis(ctypes.c_int(deg), _p(d), _p(Y), _p(dY))
    return Y, dY


def preprocess(scene, cam, radius_mode: int = 0, tile_width: int = 0) -> dict:
    lib = load()
    arrs, args = _scene_args(scene)
    n = arrs[0].shape[0]
    f = np.zeros((n, 16))
    iv = np.zeros((n, 8), dtype=np.int32)
    db = np.zeros(n, dtype=np.uint32)
    ca = camera_array(cam, radius_mode, tile_width)
    lib.orc_preprocess(*args, _p(ca), _p(f), _p(iv), _p(db))
    return dict(u=f[:, 0], v=f[:, 1], conic=f[:, 2:5], cov=f[:, 5:8], opacity=f[:, 8], rgb=f[:, 9:12],
                depth=f[:, 12], tcam=f[:, 13:16], valid=iv[:, 0].astype(bool), rect=iv[:, 1:5],
                tiles=iv[:, 5], rect_fragile=iv[:, 6].astype(bool), depth_bits=db)


def _window(cam, window):
    if window is None:
        return 0, cam.width, 0, cam.height
    x0, x1, y0, y1 = window
    return int(x0), int(x1), int(y0), int(y1)


def render(scene, cam, mode: int = 1, window=None, threads: int = 0, radius_mode: int = 0,
           tile_width: int = 0) -> dict:
    """Forward render. mode 0 = brute force over all Gaussians, 1 = per-pixel
    footprint filter, 2 = per-tile lists (list positions comparable to a tiled walk).
    Returns image f64[3,H,W], T f64[H,W], n_contrib, n_blended i32[H,W], fragile bool."""
    lib = load()
    arrs, args = _scene_args(scene)
    H, W = cam.height, cam.width
    img = np.zeros((3, H, W))
    T = np.ones((H, W))
    nc = np.zeros((H, W), dtype=np.int32)
    nb = np.zeros((H, W), dtype=np.int32)
    fr = np.zeros((H, W), dtype=np.uint8)
    ca = camera_array(cam, radius_mode, tile_width)
    x0, x1, y0, y1 = _window(cam, window)
    lib.orc_render(*args, _p(ca), ctypes.c_int(mode), ctypes.c_int(x0), ctypes.c_int(x1), ctypes.c_int(y0),
                   ctypes.c_int(y1), ctypes.c_int(threads), _p(img), _p(T), _p(nc), _p(nb), _p(fr))
    return dict(image=img, T=T, n_contrib=nc, n_blended=nb, fragile=fr.astype(bool))


def backward(scene, cam, dL_dI, mode: int = 1, window=None, threads: int = 0, radius_mode: int = 0,
             tile_width: int = 0) -> dict:
    """Analytic FP64 backward of render() for upstream gradient dL_dI [3,H,W].
    Besides the gradients and the statistic (S, M, C), returns `fragile` (the
    Gaussian is in the list of a pixel with a fragile decision) and `C_slack`, the
    number of fragile pixels at which the Gaussian's blend decision may flip in FP32:
    |C_fp32 - C| <= C_slack for every Gaussian."""
    lib = load()
    arrs, args = _scene_args(scene)
    n = arrs[0].shape[0]
    K = (int(scene.sh_degree) + 1) ** 2
    g = np.ascontiguousarray(dL_dI, dtype=np.float64)
    assert g.shape == (3, cam.height, cam.width)
    out = dict(means=np.zeros((n, 3)), log_scales=np.zeros((n, 3)), quats=np.zeros((n, 4)),
               opacity_logits=np.zeros(n), sh=np.zeros((n, K, 3)), g2d=np.zeros((n, 9)),
               S=np.zeros(n), M=np.zeros(n), C=np.zeros(n, dtype=np.int64), fragile=np.zeros(n, dtype=np.uint8),
               C_slack=np.zeros(n, dtype=np.int64))
    ca = camera_array(cam, radius_mode, tile_width)
    x0, x1, y0, y1 = _window(cam, window)
    lib.orc_backward(*args, _p(ca), ctypes.c_int(mode), ctypes.c_int(x0), ctypes.c_int(x1), ctypes.c_int(y0),
                     ctypes.c_int(y1), ctypes.c_int(threads), _p(g), _p(out["means"]), _p(out["log_scales"]),
                     _p(out["quats"]), _p(out["opacity_logits"]), _p(out["sh"]), _p(out["g2d"]), _p(out["S"]),
                     _p(out["M"]), _p(out["C"]), _p(out["fragile"]), _p(out["C_slack"]))
    out["fragile"] = out["fragile"].astype(bool)
    return out


def chain(scene, cam, g2d) -> dict:
    """Chain screen-space gradients g2d f64[n,9] (u, v, a, b, c, o, r, g, b) to the parameters."""
    lib = load()
    arrs, args = _scene_args(scene)
    n = arrs[0].shape[0]
    K = (int(scene.sh_degree) + 1) ** 2
    g = np.ascontiguousarray(g2d, dtype=np.float64)
    out = dict(means=np.zeros((n, 3)), log_scales=np.zeros((n, 3)), quats=np.zeros((n, 4)),
               opacity_logits=np.zeros(n), sh=np.zeros((n, K, 3)))
    ca = camera_array(cam)
    lib.orc_chain(*args, _p(ca), _p(g), _p(out["means"]), _p(out["log_scales"]), _p(out["quats"]),
                  _p(out["opacity_logits"]), _p(out["sh"]))
    return out


def morton(means):
    lib = load()
    m = np.ascontiguousarray(means, dtype=np.float32)
    n = m.shape[0]
    codes = np.zeros(n, dtype=np.uint64)
    perm = np.zeros(n, dtype=np.int64)
    lib.orc_morton(ctypes.c_int64(n), _p(m), _p(codes), _p(perm))
    return codes, perm


def cluster_bounds(means, log_scales, csize: int = 128):
    lib = load()
    m = np.ascontiguousarray(means, dtype=np.float32)
    ls = np.ascontiguousarray(log_scales, dtype=np.float32)
    n = m.shape[0]
    nc = (n + csize - 1) // csize
    out = np.zeros((nc, 8), dtype=np.float32)
    lib.orc_cluster_bounds(ctypes.c_int64(n), ctypes.c_int(csize), _p(m), _p(ls), _p(out))
    return out


def _bin_inputs(views):
    """views: list of (valid bool[n], rect i32[n,4] (x0,x1,y0,y1), depth_bits u32[n], tiles_x, tiles_y)."""
    V = len(views)
    n = views[0][0].shape[0]
    rects = np.zeros((V * n, 5), dtype=np.int32)
    depth = np.zeros(V * n, dtype=np.uint32)
    base = np.zeros(V + 1, dtype=np.int64)
    tx = np.zeros(V, dtype=np.int32)
    for v, (valid, rect, db, tiles_x, tiles_y) in enumerate(views):
        rects[v * n:(v + 1) * n, 0] = valid.astype(np.int32)
        rects[v * n:(v + 1) * n, 1:] = rect
        depth[v * n:(v + 1) * n] = db
        base[v + 1] = base[v] + tiles_x * tiles_y
        tx[v] = tiles_x
    return V, n, rects, depth, base, tx


def count_instances(views) -> int:
    lib = load()
    V, n, rects, depth, base, tx = _bin_inputs(views)
    return int(lib.orc_count_instances(ctypes.c_int64(n), ctypes.c_int(V), _p(rects)))


def bin_instances(views):
    """Stable (tile, depth) binning. Returns keys u64[M], vals i64[M], ranges u32[T,2]."""
    lib = load()
    V, n, rects, depth, base, tx = _bin_inputs(views)
    M = int(lib.orc_count_instances(ctypes.c_int64(n), ctypes.c_int(V), _p(rects)))
    keys = np.zeros(max(M, 1), dtype=np.uint64)
    vals = np.zeros(max(M, 1), dtype=np.int64)
    ranges = np.zeros(2 * int(base[-1]), dtype=np.uint32)
    m2 = lib.orc_bin(ctypes.c_int64(n), ctypes.c_int(V), _p(rects), _p(depth), _p(base), _p(tx), _p(keys),
                     _p(vals), _p(ranges))
    assert m2 == M
    return keys[:M], vals[:M], ranges.reshape(-1, 2)


def variance(S, M, C):
    lib = load()
    S = np.ascontiguousarray(S, dtype=np.float64)
    M = np.ascontiguousarray(M, dtype=np.float64)
    C = np.ascontiguousarray(C, dtype=np.int64)
    out = np.zeros_like(S)
    lib.orc_variance(ctypes.c_int64(S.shape[0]), _p(S), _p(M), _p(C), _p(out))
    return out


def l1_loss(image, w, gt) -> float:
    """Random-weighted L1 loss sum w |I - gt| in FP64."""
    return float(np.sum(np.asarray(w, np.float64) * np.abs(np.asarray(image, np.float64) - gt)))


def l1_grad(image, w, gt):
    """dL/dI of l1_loss: w * sign(I - gt)."""
    return np.asarray(w, np.float64) * np.sign(np.asarray(image, np.float64) - np.asarray(gt, np.float64))


ADAM_GROUPS = ("means", "log_scales", "quats", "opacity_logits", "sh")


def sparse_adam(params, grads, m, v, visible, lr, beta1, beta2, eps, step, csize: int = 128):
    """One Adam step (Kingma and Ba, Algorithm 1) applied at cluster granularity,
    as Sec. 3.2.3 applies the sparse update of the per-view visible primitives to
    whole clusters of ``csize`` consecutive Gaussians. The paper gives neither the
    rates nor the handling of skipped Gaussians; the reading is that of the sparse
    Adam it builds on: the moments and parameters of a cluster that is not visible
    stay as they are, and the bias corrections use the global step count
    ``step`` >= 1.

    params, grads, m, v: dicts over ADAM_GROUPS of arrays with n rows (any trailing
    shape). visible: flags per cluster (nonzero = visible), or None for all.
    lr: dict with a rate per group, the SH group split into 'sh_dc' (the first 3
    floats of each row: the degree-0 coefficient of the 3 colours) and 'sh_rest'.
    Returns new (params, m, v) dicts in FP64; the inputs are not modified.
    """
    n = params["means"].shape[0]
    nc = (n + csize - 1) // csize
    rows = np.ones(n, dtype=bool)
    if visible is not None:
        vis = np.asarray(visible).reshape(-1)[:nc] != 0
        rows = np.repeat(vis, csize)[:n]
    bc1 = 1.0 - beta1 ** step
    bc2 = 1.0 - beta2 ** step
    out_p, out_m, out_v = {}, {}, {}
    for k in ADAM_GROUPS:
        p0 = np.asarray(params[k], np.float64).reshape(n, -1)
        g = np.asarray(grads[k], np.float64).reshape(n, -1)
        m0 = np.asarray(m[k], np.float64).reshape(n, -1)
        v0 = np.asarray(v[k], np.float64).reshape(n, -1)
        if k == "sh":
            rate = np.full(p0.shape[1], lr["sh_rest"], np.float64)
            rate[:3] = lr["sh_dc"]
        else:
            rate = np.full(p0.shape[1], lr[k], np.float64)
        m1 = beta1 * m0 + (1.0 - beta1) * g            # biased first moment
        v1 = beta2 * v0 + (1.0 - beta2) * g * g        # biased second raw moment
        m_hat = m1 / bc1
        v_hat = v1 / bc2
        p1 = p0 - rate[None, :] * m_hat / (np.sqrt(v_hat) + eps)
        shape = np.shape(params[k])
        out_p[k] = np.where(rows[:, None], p1, p0).reshape(shape)
        out_m[k] = np.where(rows[:, None], m1, m0).reshape(shape)
        out_v[k] = np.where(rows[:, None], v1, v0).reshape(shape)
    return out_p, out_m, out_v


def quat_to_rotation(q):
    """Rotation matrices [n,3,3] of quaternions (w, x, y, z) [n,4], normalised first."""
    q = np.asarray(q, np.float64)
    q = q / np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)], -2)


def densify(params, metric, noise, threshold, max_candidates, split_log_scale, split_factor, prune_logit,
            state=None):
    """Densification driven by the opacity-gradient variance metric (Sec. 3.3): the
    Gaussians whose metric C Var (gsr_variance's output) is largest are the ones a
    single primitive no longer represents, and get split or cloned.

    The paper fixes the metric only; the rest follows the densification of 3DGS that
    it modifies, with every threshold an argument:
      * candidates: metric >= threshold (threshold > 0), the max_candidates largest,
        ties to the lower index; the decision compares the FP32 values given;
      * a candidate whose largest log-scale exceeds split_log_scale is split into two
        children at mean + R (exp(s) * z_c), z_c = noise[i, c] (standard normal draws
        passed in), with log-scales s - ln(split_factor) and the parent's other
        parameters; the parent is removed. Any other candidate is cloned (an exact
        copy is appended; the original stays);
      * an original (not a candidate's child or clone) with opacity logit below
        prune_logit is removed.
    Output rows: the kept originals in index order, then per candidate in rank order
    its clone, or its two children. ``state``: dict of per-Gaussian arrays (optimiser
    moments) whose kept rows move with their Gaussians and whose new rows are zero.

    Returns (out_params, out_state, src, kind): src[j] the input row of output row j,
    kind[j] 0 kept original, 1 clone, 2 / 3 first / second child of a split.
    """
    n = params["means"].shape[0]
    m = np.asarray(metric, np.float32)
    thr = np.float32(threshold)
    qual = np.nonzero(m >= thr)[0]
    order = qual[np.argsort(-m[qual], kind="stable")]     # descending metric, ties by index
    cand = order[:max_candidates]
    ls = np.asarray(params["log_scales"], np.float32)
    split = ls[cand].max(axis=1) > np.float32(split_log_scale)
    removed = np.zeros(n, bool)
    removed[cand[split]] = True
    removed |= np.asarray(params["opacity_logits"], np.float32) < np.float32(prune_logit)
    kept = np.nonzero(~removed)[0]
    src, kind = [kept], [np.zeros(len(kept), np.int64)]
    for i, sp in zip(cand, split):
        src.append(np.array([i, i] if sp else [i]))
        kind.append(np.array([2, 3] if sp else [1]))
    src = np.concatenate(src).astype(np.int64)
    kind = np.concatenate(kind).astype(np.int64)
    out = {k: np.asarray(v)[src].copy() for k, v in params.items()}
    child = kind >= 2
    if child.any():
        i = src[child]
        c = kind[child] - 2
        R = quat_to_rotation(np.asarray(params["quats"])[i])
        z = np.asarray(noise, np.float64).reshape(n, 2, 3)[i, c]
        off = np.einsum("nij,nj->ni", R, np.exp(ls[i].astype(np.float64)) * z)
        out["means"][child] = (np.asarray(params["means"], np.float64)[i] + off).astype(np.float32)
        out["log_scales"][child] = (ls[i].astype(np.float64) - np.log(np.float64(np.float32(split_factor)))
                                    ).astype(np.float32)
    out_state = {}
    for k, v in (state or {}).items():
        a = np.asarray(v)[src].copy()
        a[kind != 0] = 0
        out_state[k] = a
    return out, out_state, src, kind


def opacity_decay(logits, factor):
    """Opacity decay (Sec. 3.3), the gentler replacement of the opacity reset: the
    activated opacity o = sigmoid(l) is multiplied by factor (the paper halves it)
    and turned back into a logit, FP64."""
    l = np.asarray(logits, np.float64)
    o = factor / (1.0 + np.exp(-l))
    return (np.log(o) - np.log1p(-o)).astype(np.float32)
