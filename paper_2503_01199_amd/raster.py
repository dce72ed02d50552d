"""Torch-facing binding of libgsr: argument marshalling only.

Every step of the rasterizer runs in the library's HIP kernels; this module turns
torch tensors into device pointers, keeps the caller-owned workspace, and runs on
torch's current HIP stream.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math

import numpy as np
import torch

from . import _lib as L

GRAD_KEYS = ("means", "log_scales", "quats", "opacity_logits", "sh")

_ALIGN = 256


def camera_struct(cam) -> L.GsrCamera:
    c = L.GsrCamera()
    c.width, c.height = int(cam.width), int(cam.height)
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    R = np.asarray(cam.R, dtype=np.float32).reshape(9)
    t = np.asarray(cam.t, dtype=np.float32).reshape(3)
    bg = np.asarray(cam.bg, dtype=np.float32).reshape(3)
    for k in range(9):
        c.R[k] = float(R[k])
    for k in range(3):
        c.t[k] = float(t[k])
        c.bg[k] = float(bg[k])
    c.near_plane = float(cam.near)
    return c


def _ptr(t: torch.Tensor | None) -> int | None:
    return None if t is None else t.data_ptr()


@dataclasses.dataclass
class SceneTensors:
    """The scene's parameter tensors on the device (FP32, contiguous)."""
    means: torch.Tensor
    log_scales: torch.Tensor
    quats: torch.Tensor
    opacity_logits: torch.Tensor
    sh: torch.Tensor
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @staticmethod
    def from_scene(scene, device="cuda") -> "SceneTensors":
        f = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device=device)  # noqa: E731
        return SceneTensors(f(scene.means), f(scene.log_scales), f(scene.quats), f(scene.opacity_logits),
                            f(scene.sh), int(scene.sh_degree))

    def tensors(self):
        return (self.means, self.log_scales, self.quats, self.opacity_logits, self.sh)

    def struct(self) -> L.GsrScene:
        for t in self.tensors():
            if t.dtype != torch.float32 or not t.is_contiguous():
                raise ValueError("scene tensors must be contiguous float32")
        s = L.GsrScene()
        s.n = self.n
        s.sh_degree = self.sh_degree
        s.means, s.log_scales, s.quats, s.opacity_logits, s.sh = (_ptr(t) for t in self.tensors())
        return s


class Workspace:
    """A caller-owned device byte buffer, grown on demand, 256-byte aligned. The
    rasterizer that renders into it is told when the buffer goes away, so that the
    library drops the frame state it keeps for the address."""

    def __init__(self, device):
        self.device = torch.device(device)
        self.buf = None
        self.offset = 0
        self.nbytes = 0
        self.owner = None  # (library, context) of the last forward on this buffer

    def _release(self):
        if self.owner is not None and self.buf is not None:
            lib, ctx = self.owner
            if ctx.value:
                lib.gsr_frame_release(ctx, self.ptr)
        self.owner = None

    def __del__(self):
        try:
            self._release()
        except Exception:  # interpreter shutdown
            pass

    def ensure(self, nbytes: int):
        if self.buf is not None and self.nbytes >= nbytes:
            return
        self._release()
        self.buf = torch.empty(int(nbytes) + _ALIGN, dtype=torch.uint8, device=self.device)
        self.offset = (-self.buf.data_ptr()) % _ALIGN
        self.nbytes = int(nbytes)

    @property
    def ptr(self) -> int:
        return self.buf.data_ptr() + self.offset

    def view(self, dev_ptr: int, count: int, dtype: torch.dtype) -> torch.Tensor:
        """Tensor view of `count` elements at device pointer dev_ptr inside the workspace."""
        start = dev_ptr - self.buf.data_ptr()
        itemsize = torch.empty((), dtype=dtype).element_size()
        assert 0 <= start and start + count * itemsize <= self.buf.numel(), "pointer outside the workspace"
        return self.buf[start:start + count * itemsize].view(dtype)


@dataclasses.dataclass
class Frame:
    """State of one forward: what gsr_backward needs to run on the same workspace."""
    scene: SceneTensors
    cameras: list
    cam_structs: ctypes.Array
    opts: L.GsrOptions
    workspace: Workspace
    images: list
    info: dict


class Rasterizer:
    """One library context on one device (not thread-safe; one per host thread)."""

    def __init__(self, device: int | str | torch.device = 0):
        self.lib = L.load()
        dev = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        if dev.type != "cuda":
            raise ValueError("the rasterizer runs on a HIP device")
        self.device = torch.device("cuda", dev.index if dev.index is not None else torch.cuda.current_device())
        ctx = ctypes.c_void_p()
        st = self.lib.gsr_context_create(self.device.index, ctypes.byref(ctx))
        if st != L.GSR_OK:
            raise L.GsrError(st, "gsr_context_create(%d)" % self.device.index)
        self.ctx = ctx
        self.default_workspace = Workspace(self.device)
        self.morton_workspace = Workspace(self.device)

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx is not None and ctx.value:
            self.lib.gsr_context_destroy(ctx)
            ctx.value = None  # workspaces that still refer to the context see it gone
            self.ctx = None

    def _check(self, st: int, what: str):
        if st != L.GSR_OK:
            msg = self.lib.gsr_last_error(self.ctx)
            raise L.GsrError(st, "%s: %s" % (what, msg.decode() if msg else ""))

    def _stream(self) -> int:
        return torch.cuda.current_stream(self.device).cuda_stream

    @staticmethod
    def options(precision=L.GSR_FP32, cluster_cull=True, stats=True, deterministic=False,
                radius_mode=0, half_reduction=False, tile_width=0) -> L.GsrOptions:
        o = L.GsrOptions()
        o.precision = int(precision)
        o.cluster_cull = 1 if cluster_cull else 0
        o.stats = 1 if stats else 0
        o.deterministic = 1 if deterministic else 0
        o.radius_mode = int(radius_mode)
        o.half_reduction = 1 if half_reduction else 0
        o.tile_width = int(tile_width)
        return o

    # ------------------------------------------------------------------ forward / backward
    def forward(self, scene: SceneTensors, cameras, precision=L.GSR_FP32, cluster_cull=True, stats=True,
                workspace: Workspace | None = None, images=None, check: bool = True,
                deterministic: bool = False, radius_mode: int = 0, half_reduction: bool = False,
                tile_width: int = 0) -> Frame:
        """Renders the views. With check (the default) waits for the frame's counters
        and, when its instances did not fit the workspace, grows it and renders
        again; check=False returns right after enqueueing (info is then empty: call
        check_frame to wait, read the counters and learn whether it fitted).
        deterministic: the frame's backward sums per-tile gradients in fixed point
        (bitwise reproducible gradients). radius_mode: 0 the exact alpha >= 1/255 tile
        membership, 1 the 3-sigma bound. half_reduction: the frame's backward reduces
        colour and opacity gradients as packed FP16 pairs. tile_width: tiles of 256
        pixels, that many wide (4, 8, 16, 32 or 64; 0: 16x16)."""
        V = len(cameras)
        cams = (L.GsrCamera * V)(*[camera_struct(c) for c in cameras])
        opts = self.options(precision, cluster_cull, stats, deterministic, radius_mode, half_reduction, tile_width)
        sc = scene.struct()
        ws = workspace if workspace is not None else self.default_workspace
        if images is None:
            images = [torch.empty((3, c.height, c.width), dtype=torch.float32, device=self.device) for c in cameras]
        img_ptrs = (ctypes.c_void_p * V)(*[t.data_ptr() for t in images])
        if ws.buf is None:
            nbytes = ctypes.c_size_t()
            self._check(self.lib.gsr_workspace_size(self.ctx, ctypes.byref(sc), cams, V, ctypes.byref(opts),
                                                    8 * scene.n + 4096, ctypes.byref(nbytes)), "gsr_workspace_size")
            ws.ensure(nbytes.value)
        for _ in range(4):
            st = self.lib.gsr_forward(self.ctx, ctypes.byref(sc), cams, V, ctypes.byref(opts), ws.ptr, ws.nbytes,
                                      img_ptrs, self._stream())
            if st == L.GSR_ERR_WORKSPACE_TOO_SMALL:
                ws.ensure(self.lib.gsr_required_workspace(self.ctx))
                continue
            self._check(st, "gsr_forward")
            ws.owner = (self.lib, self.ctx)
            frame = Frame(scene, list(cameras), cams, opts, ws, images, {})
            if not check:
                return frame
            st, info = self._inspect(ws, None)
            if st == L.GSR_ERR_WORKSPACE_TOO_SMALL:
                ws.ensure(self.lib.gsr_required_workspace(self.ctx))
                continue
            self._check(st, "gsr_frame_inspect")
            frame.info = info
            return frame
        self._check(st, "gsr_forward")
        raise L.GsrError(L.GSR_ERR_WORKSPACE_TOO_SMALL, "gsr_forward: workspace did not converge")

    def prepare(self, scene: SceneTensors, cameras, cluster_cull=True, stats=True,
                workspace: Workspace | None = None, stream=None, deterministic: bool = False,
                radius_mode: int = 0, tile_width: int = 0) -> Frame:
        """Enqueues every stage before the raster (gsr_prepare) on `stream` (a
        torch.cuda.Stream; default the current stream); render with raster_batch."""
        V = len(cameras)
        cams = (L.GsrCamera * V)(*[camera_struct(c) for c in cameras])
        opts = self.options(L.GSR_FP32, cluster_cull, stats, deterministic, radius_mode, tile_width=tile_width)
        sc = scene.struct()
        ws = workspace if workspace is not None else Workspace(self.device)
        if ws.buf is None:
            nbytes = ctypes.c_size_t()
            self._check(self.lib.gsr_workspace_size(self.ctx, ctypes.byref(sc), cams, V, ctypes.byref(opts),
                                                    8 * scene.n + 4096, ctypes.byref(nbytes)), "gsr_workspace_size")
            ws.ensure(nbytes.value)
        s = self._stream() if stream is None else stream.cuda_stream
        self._check(self.lib.gsr_prepare(self.ctx, ctypes.byref(sc), cams, V, ctypes.byref(opts), ws.ptr, ws.nbytes,
                                         s), "gsr_prepare")
        ws.owner = (self.lib, self.ctx)
        return Frame(scene, list(cameras), cams, opts, ws, None, {})

    def raster_batch(self, frames, precision=L.GSR_FP32, batch_workspace: Workspace | None = None, stream=None,
                     images=None):
        """One gsr_raster_batch launch over prepared frames on `stream`; returns (and
        stores in each frame) the list of its [3, H, W] images."""
        n = len(frames)
        wsp = (ctypes.c_void_p * n)(*[f.workspace.ptr for f in frames])
        if images is None:
            images = [[torch.empty((3, c.height, c.width), dtype=torch.float32, device=self.device) for c in f.cameras]
                      for f in frames]
        rows = [(ctypes.c_void_p * len(im))(*[t.data_ptr() for t in im]) for im in images]
        table = (ctypes.POINTER(ctypes.c_void_p) * n)(*[ctypes.cast(r, ctypes.POINTER(ctypes.c_void_p)) for r in rows])
        nbytes = ctypes.c_size_t()
        self._check(self.lib.gsr_raster_batch_workspace_size(self.ctx, n, wsp, ctypes.byref(nbytes)),
                    "gsr_raster_batch_workspace_size")
        bws = batch_workspace if batch_workspace is not None else Workspace(self.device)
        bws.ensure(max(nbytes.value, _ALIGN))
        s = self._stream() if stream is None else stream.cuda_stream
        self._check(self.lib.gsr_raster_batch(self.ctx, n, wsp, table, int(precision), bws.ptr, bws.nbytes, s),
                    "gsr_raster_batch")
        for f, im in zip(frames, images):
            f.images = im
            f.opts.precision = int(precision)
        return images

    def _inspect(self, ws: Workspace, bufs):
        info = L.GsrFrameInfo()
        st = self.lib.gsr_frame_inspect(self.ctx, ws.ptr, ctypes.byref(info), None if bufs is None else ctypes.byref(bufs))
        return st, {k: getattr(info, k) for k, _ in L.GsrFrameInfo._fields_ if k != "reserved"}

    def check_frame(self, frame: Frame) -> dict:
        """Waits for the frame's counters; raises GsrError if its instances did not
        fit the workspace (GSR_ERR_WORKSPACE_TOO_SMALL) or a device wait gave up."""
        st, info = self._inspect(frame.workspace, None)
        self._check(st, "gsr_frame_inspect")
        frame.info = info
        return info

    def backward(self, frame: Frame, dL_dimages, grads=None, stats=None):
        """Returns the parameter gradients (a dict of tensors shaped like the scene's).
        `stats` is None or a dict with tensors S, M (float32) and C (int32) that are
        accumulated in place."""
        V = len(frame.cameras)
        sc = frame.scene.struct()
        dl = [t.contiguous() for t in dL_dimages]
        for t, c in zip(dl, frame.cameras):
            if t.shape != (3, c.height, c.width) or t.dtype != torch.float32:
                raise ValueError("dL/dimage must be float32 [3, H, W]")
        dl_ptrs = (ctypes.c_void_p * V)(*[t.data_ptr() for t in dl])
        if grads is None:
            grads = {k: torch.empty_like(t) for k, t in zip(("means", "log_scales", "quats", "opacity_logits", "sh"),
                                                            frame.scene.tensors())}
        g = L.GsrGrads()
        g.means, g.log_scales, g.quats, g.opacity_logits, g.sh = (
            _ptr(grads[k]) for k in ("means", "log_scales", "quats", "opacity_logits", "sh"))
        st_ptr = None
        if stats is not None:
            s = L.GsrStats()
            s.S, s.M, s.C = _ptr(stats["S"]), _ptr(stats["M"]), _ptr(stats["C"])
            st_ptr = ctypes.byref(s)
        ws = frame.workspace
        self._check(self.lib.gsr_backward(self.ctx, ctypes.byref(sc), frame.cam_structs, V, ctypes.byref(frame.opts),
                                          ws.ptr, ws.nbytes, dl_ptrs, ctypes.byref(g), st_ptr, self._stream()),
                    "gsr_backward")
        return grads

    def backward_adam(self, frame: Frame, dL_dimages, exp_avg: dict, exp_avg_sq: dict, lr: dict, step: int,
                      beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-15, stats=None):
        """The backward with the Adam step of the frame's kept clusters fused in
        (gsr_backward_adam): the frame's scene tensors are updated in place, with the
        moments; no gradient is returned."""
        V = len(frame.cameras)
        sc = frame.scene.struct()
        dl = [t.contiguous() for t in dL_dimages]
        for t, c in zip(dl, frame.cameras):
            if t.shape != (3, c.height, c.width) or t.dtype != torch.float32:
                raise ValueError("dL/dimage must be float32 [3, H, W]")
        dl_ptrs = (ctypes.c_void_p * V)(*[t.data_ptr() for t in dl])
        sets = []
        for d in (exp_avg, exp_avg_sq):
            g = L.GsrGrads()
            for k, t in zip(GRAD_KEYS, frame.scene.tensors()):
                if d[k].shape != t.shape or d[k].dtype != torch.float32 or not d[k].is_contiguous():
                    raise ValueError("moments must be contiguous float32 tensors shaped like the scene")
                setattr(g, k, d[k].data_ptr())
            sets.append(g)
        st_ptr = None
        if stats is not None:
            s = L.GsrStats()
            s.S, s.M, s.C = _ptr(stats["S"]), _ptr(stats["M"]), _ptr(stats["C"])
            st_ptr = ctypes.byref(s)
        o = L.GsrAdamOptions(lr["means"], lr["log_scales"], lr["quats"], lr["opacity_logits"], lr["sh_dc"],
                             lr["sh_rest"], beta1, beta2, eps, 0, int(step))
        ws = frame.workspace
        self._check(self.lib.gsr_backward_adam(self.ctx, ctypes.byref(sc), frame.cam_structs, V,
                                               ctypes.byref(frame.opts), ws.ptr, ws.nbytes, dl_ptrs,
                                               ctypes.byref(sets[0]), ctypes.byref(sets[1]), ctypes.byref(o), st_ptr,
                                               self._stream()), "gsr_backward_adam")

    # ------------------------------------------------------------------ inspection
    def inspect(self, frame: Frame, allow_overflow: bool = False) -> dict:
        """Tensor views (not copies) of the frame's intermediate buffers in the
        workspace. With allow_overflow, a frame whose instances did not all fit is
        inspected too: its instance lists then hold the kept prefix (info["kept"])."""
        b = L.GsrFrameBuffers()
        ws = frame.workspace
        st, info_d = self._inspect(ws, b)
        if not (allow_overflow and st == L.GSR_ERR_WORKSPACE_TOO_SMALL):
            self._check(st, "gsr_frame_inspect")
        info = L.GsrFrameInfo(**{k: v for k, v in info_d.items()})
        V = len(frame.cameras)
        ncap = info.clusters * L.GSR_CLUSTER
        R = ncap * V
        M = info.instances
        if st == L.GSR_ERR_WORKSPACE_TOO_SMALL:
            ends = ws.view(b.ranges, 2 * info.tiles, torch.int32).view(-1, 2)[:, 1]
            M = int(ends.max().item()) if info.tiles > 0 else 0
        info_d["kept"] = M
        P = info.pixels
        u32, f32, i16 = torch.int32, torch.float32, torch.int16
        out = dict(
            records=ws.view(b.record, 12 * R, f32).view(R, 12),
            depth_key=ws.view(b.depth_key, R, u32),
            tiles=ws.view(b.tiles, R, u32),
            rect=ws.view(b.rect, 4 * R, i16).view(R, 4),
            compact2full=ws.view(b.compact2full, ncap, u32),
            inst_tile=ws.view(b.inst_tile, M, u32) if M > 0 else torch.zeros(0, dtype=u32, device=self.device),
            inst_record=ws.view(b.inst_record, M, u32) if M > 0 else torch.zeros(0, dtype=u32, device=self.device),
            ranges=ws.view(b.ranges, 2 * info.tiles, u32).view(-1, 2),
            pixel_T=ws.view(b.pixel_T, P, f32),
            pixel_last=ws.view(b.pixel_last, P, u32),
            grad2d=ws.view(b.grad2d, 12 * R, f32).view(R, 12),
            cluster_bounds=ws.view(b.cluster_bounds, 8 * max(info.clusters, 1), f32).view(-1, 8),
            cluster_visible=ws.view(b.cluster_visible, max(info.clusters, 1), u32),
            fwd_items=ws.view(b.fwd_items, info.tiles + 3 * info.split_tiles, u32),
            bwd_items=ws.view(b.bwd_items, info.tiles + info.split_tiles_bwd, u32),
            pixel_base=[b.pixel_base[v] for v in range(V)],
            tile_base=[b.tile_base[v] for v in range(V)],
            info=info_d,
        )
        return out

    # ------------------------------------------------------------------ Morton / permutation / variance
    def morton_order(self, means: torch.Tensor):
        """(perm i64[n], codes as i64[n] holding the 63-bit codes) of Sec. 3.2.1."""
        n = int(means.shape[0])
        means = means.contiguous()
        nbytes = ctypes.c_size_t()
        self._check(self.lib.gsr_morton_workspace_size(self.ctx, n, ctypes.byref(nbytes)), "gsr_morton_workspace_size")
        self.morton_workspace.ensure(nbytes.value)
        perm = torch.empty(n, dtype=torch.int64, device=self.device)
        codes = torch.empty(n, dtype=torch.int64, device=self.device)
        self._check(self.lib.gsr_morton_order(self.ctx, means.data_ptr(), n, self.morton_workspace.ptr,
                                              self.morton_workspace.nbytes, perm.data_ptr(), codes.data_ptr(),
                                              self._stream()), "gsr_morton_order")
        return perm, codes

    def sort_u32(self, keys: torch.Tensor, vals: torch.Tensor | None = None, bits: int = 32,
                 workspace: Workspace | None = None):
        """Stable radix sort of 32-bit keys (int32 tensors holding the bits) on their low
        `bits` bits with their values (None: positions), gsr_sort_u32. Keys and values
        may start at any 4-byte offset. Returns (keys, values) and raises if a
        device-wide wait gave up."""
        n = int(keys.numel())
        assert keys.dtype == torch.int32 and keys.is_contiguous()
        assert vals is None or (vals.dtype == torch.int32 and vals.is_contiguous() and vals.numel() == n)
        nbytes = ctypes.c_size_t()
        self._check(self.lib.gsr_sort_workspace_size(self.ctx, n, int(bits), ctypes.byref(nbytes)),
                    "gsr_sort_workspace_size")
        ws = workspace if workspace is not None else Workspace(self.device)
        ws.ensure(nbytes.value)
        out_k = torch.empty(n, dtype=torch.int32, device=self.device)
        out_v = torch.empty(n, dtype=torch.int32, device=self.device)
        self._check(self.lib.gsr_sort_u32(self.ctx, keys.data_ptr(), vals.data_ptr() if vals is not None else None, n,
                                          int(bits), out_k.data_ptr(), out_v.data_ptr(), ws.ptr, ws.nbytes,
                                          self._stream()), "gsr_sort_u32")
        if n > 0 and int(ws.view(ws.ptr, 1, torch.int32).item()) != 0:
            raise L.GsrError(L.GSR_ERR_DEVICE, "gsr_sort_u32: a device-wide wait gave up")
        return out_k, out_v

    def apply_permutation(self, perm: torch.Tensor, arrays):
        """New tensors dst[i] = src[perm[i]] for each array (rows along dim 0)."""
        n = int(perm.shape[0])
        srcs = [a.contiguous() for a in arrays]
        dsts = [torch.empty_like(a) for a in srcs]
        rows = (ctypes.c_int32 * len(srcs))(*[int(a[0].numel()) if a.shape[0] > 0 else 0 for a in srcs])
        sp = (ctypes.c_void_p * len(srcs))(*[a.data_ptr() for a in srcs])
        dp = (ctypes.c_void_p * len(srcs))(*[a.data_ptr() for a in dsts])
        self._check(self.lib.gsr_apply_permutation(self.ctx, perm.contiguous().data_ptr(), n, len(srcs), sp, dp, rows,
                                                   self._stream()), "gsr_apply_permutation")
        return dsts

    def densify(self, scene: SceneTensors, metric: torch.Tensor, noise: torch.Tensor, threshold: float,
                max_candidates: int, split_log_scale: float, split_factor: float = 1.6,
                prune_logit: float = float("-inf"), state: dict | None = None, capacity: int | None = None,
                sync: bool = True):
        """Densification by the variance metric (gsr_densify, Sec. 3.3). Returns
        (scene, state, n_out): new tensors of `capacity` rows (default n + the
        candidates) and the output row count; with sync the count is read back (one
        host wait) and the tensors are cut to it, else n_out is a device int64 tensor."""
        n = scene.n
        K = min(int(max_candidates), n)
        cap = n + K if capacity is None else int(capacity)
        sc = scene.struct()
        if metric.dtype != torch.float32 or metric.numel() != n or noise.dtype != torch.float32 or noise.numel() != 6 * n:
            raise ValueError("metric must be float32 [n], noise float32 [n, 2, 3]")
        out = [torch.empty((cap,) + tuple(t.shape[1:]), dtype=torch.float32, device=self.device)
               for t in scene.tensors()]
        g = L.GsrGrads()
        g.means, g.log_scales, g.quats, g.opacity_logits, g.sh = (t.data_ptr() for t in out)
        names = list(state) if state else []
        s_in = [state[k].contiguous() for k in names]
        s_out = [torch.empty((cap,) + tuple(t.shape[1:]), dtype=torch.float32, device=self.device) for t in s_in]
        for t in s_in:
            if t.dtype != torch.float32 or t.shape[0] != n:
                raise ValueError("state arrays must be float32 with n rows")
        rows = (ctypes.c_int32 * max(1, len(names)))(*[int(t[0].numel()) if n > 0 else 1 for t in s_in])
        sp = (ctypes.c_void_p * max(1, len(names)))(*[t.data_ptr() for t in s_in])
        dp = (ctypes.c_void_p * max(1, len(names)))(*[t.data_ptr() for t in s_out])
        nbytes = ctypes.c_size_t()
        self._check(self.lib.gsr_densify_workspace_size(self.ctx, n, K, ctypes.byref(nbytes)),
                    "gsr_densify_workspace_size")
        self.morton_workspace.ensure(nbytes.value)
        n_out = torch.empty(1, dtype=torch.int64, device=self.device)
        o = L.GsrDensifyOptions(threshold, split_log_scale, split_factor, prune_logit, K)
        self._check(self.lib.gsr_densify(self.ctx, ctypes.byref(sc), metric.contiguous().data_ptr(),
                                         noise.contiguous().data_ptr(), ctypes.byref(o), ctypes.byref(g), cap,
                                         len(names), sp, dp, rows, self.morton_workspace.ptr,
                                         self.morton_workspace.nbytes, n_out.data_ptr(), self._stream()),
                    "gsr_densify")
        if not sync:
            return SceneTensors(*out, scene.sh_degree), dict(zip(names, s_out)), n_out
        rows_out = int(n_out.item())
        if rows_out < 0:
            raise L.GsrError(L.GSR_ERR_DEVICE, "gsr_densify: a device-wide wait gave up")
        cut = lambda t: t[:rows_out]  # noqa: E731
        return (SceneTensors(*[cut(t) for t in out], scene.sh_degree), {k: cut(t) for k, t in zip(names, s_out)},
                rows_out)

    def opacity_decay(self, logits: torch.Tensor, factor: float = 0.5):
        """In place: sigmoid(l) <- factor sigmoid(l) (gsr_opacity_decay, Sec. 3.3)."""
        if logits.dtype != torch.float32 or not logits.is_contiguous():
            raise ValueError("logits must be contiguous float32")
        self._check(self.lib.gsr_opacity_decay(self.ctx, logits.data_ptr(), logits.numel(), factor, self._stream()),
                    "gsr_opacity_decay")

    def l1_grad(self, image: torch.Tensor, w: torch.Tensor, gt: torch.Tensor, out: torch.Tensor | None = None):
        """dL/dI of L = sum w |I - gt| computed by the library's kernel."""
        out = torch.empty_like(image) if out is None else out
        self._check(self.lib.gsr_l1_grad(self.ctx, image.data_ptr(), w.data_ptr(), gt.data_ptr(), image.numel(),
                                         out.data_ptr(), self._stream()), "gsr_l1_grad")
        return out

    def set_raster_split(self, split_len: int = 0, split_len_bwd: int = 0):
        """Lists longer than split_len (forward) / split_len_bwd (backward) are rastered
        as band items in frames prepared from now on; 0 restores the default,
        0xffffffff never splits (gsr_set_raster_split)."""
        self._check(self.lib.gsr_set_raster_split(self.ctx, int(split_len), int(split_len_bwd)),
                    "gsr_set_raster_split")

    def set_fault_injection(self, mode: int):
        """Failure injection of the frames prepared from now on (tests of the error
        path): L.GSR_FAULT_NONE, GSR_FAULT_ABORT_BEFORE_SORT or GSR_FAULT_WITHHOLD_STATUS."""
        self._check(self.lib.gsr_set_fault_injection(self.ctx, int(mode)), "gsr_set_fault_injection")

    def set_profiling(self, enable: bool):
        self._check(self.lib.gsr_set_profiling(self.ctx, 1 if enable else 0), "gsr_set_profiling")

    def stage_times(self) -> dict:
        """Milliseconds per stage of the last profiled forward / backward (waits for them)."""
        ms = (ctypes.c_float * len(L.STAGES))()
        self._check(self.lib.gsr_stage_times(self.ctx, ms), "gsr_stage_times")
        return {name: float(ms[k]) for k, name in enumerate(L.STAGES)}

    def variance(self, S: torch.Tensor, M: torch.Tensor, C: torch.Tensor) -> torch.Tensor:
        n = int(S.shape[0])
        out = torch.empty(n, dtype=torch.float32, device=self.device)
        s = L.GsrStats()
        s.S, s.M, s.C = S.data_ptr(), M.data_ptr(), C.data_ptr()
        self._check(self.lib.gsr_variance(self.ctx, ctypes.byref(s), n, out.data_ptr(), self._stream()), "gsr_variance")
        return out


    def sparse_adam(self, params: dict, grads: dict, exp_avg: dict, exp_avg_sq: dict, visible, lr: dict,
                    step: int, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-15, sh_degree=None):
        """One Adam step in place over the Gaussians of visible clusters (gsr_sparse_adam).
        params / grads / exp_avg / exp_avg_sq: dicts of float32 tensors with the scene
        shapes; visible: u32 (int32) flags per cluster, e.g. inspect(frame)['cluster_visible'],
        or None for every cluster; lr: rates keyed means, log_scales, quats,
        opacity_logits, sh_dc, sh_rest."""
        n = int(params["means"].shape[0])
        if sh_degree is None:
            K = params["sh"].shape[1] if params["sh"].dim() == 3 else params["sh"].shape[1] // 3
            sh_degree = int(round(math.sqrt(K))) - 1
        sets = []
        for d in (params, grads, exp_avg, exp_avg_sq):
            g = L.GsrGrads()
            for k in GRAD_KEYS:
                t = d[k]
                if t.dtype != torch.float32 or not t.is_contiguous() or t.device != self.device or t.shape[0] != n:
                    raise ValueError("sparse_adam: %s must be a contiguous float32 tensor on %s with %d rows"
                                     % (k, self.device, n))
                setattr(g, k, t.data_ptr())
            sets.append(g)
        nc = (n + 127) // 128
        if visible is not None:
            if visible.dtype not in (torch.int32, torch.uint32) or visible.numel() < nc or visible.device != self.device:
                raise ValueError("sparse_adam: visible must hold %d u32 flags on %s" % (nc, self.device))
        o = L.GsrAdamOptions(lr["means"], lr["log_scales"], lr["quats"], lr["opacity_logits"], lr["sh_dc"],
                             lr["sh_rest"], beta1, beta2, eps, 0, int(step))
        self._check(self.lib.gsr_sparse_adam(self.ctx, n, int(sh_degree), _ptr(visible), *[ctypes.byref(g) for g in sets],
                                             ctypes.byref(o), self._stream()), "gsr_sparse_adam")


def new_stats(n: int, device) -> dict:
    """Zeroed statistic accumulators S, M (float32) and C (int32 holding u32 counts)."""
    return dict(S=torch.zeros(n, dtype=torch.float32, device=device), M=torch.zeros(n, dtype=torch.float32, device=device),
                C=torch.zeros(n, dtype=torch.int32, device=device))
