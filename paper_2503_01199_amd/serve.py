"""Render serving over the library: resident scenes, continuous batching, HBM-budget
admission, p50/p99 latency.

A request asks for one novel view of one resident scene. The scheduler runs one
host loop:

- arrivals join a FIFO queue;
- the queue head is admitted when a slot is free and its workspace bound (the
  planner's byte count for the request's view) fits in what is left of the HBM
  budget; admission enqueues the request's preparation (gsr_prepare: cull,
  projection, sorting, binning) on the slot's own stream, so preparations of
  different requests overlap on the device with each other and with rasters;
- every tick, all prepared requests not yet rendered go into ONE batched raster
  launch (gsr_raster_batch) on the raster stream, which waits for their slots;
- completed batches free their slots and bytes at once, so requests that arrived
  meanwhile are admitted while other batches are still on the GPU;
- a frame whose instances outgrew its bound (known only after projection) is
  queued again at the head with the exact byte count it reported.

Latency is arrival to the host's observation of the batch's completion event.

The scheduler only talks to an executor (bytes_needed / start / launch / poll /
finish) and a clock, so the policy is tested on the CPU with a simulated
executor and clock, and runs on the GPU with GpuExecutor.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    scene: str
    camera: object
    arrival: float
    admitted: float | None = None
    done: float | None = None
    nbytes: int = 0
    retries: int = 0
    images: list | None = None
    rejected: bool = False


@dataclasses.dataclass
class ServeStats:
    latencies: list
    admission_waits: list
    slots_in_flight: list
    batches: int
    batch_sizes: list
    max_bytes_in_use: int
    rejected: int
    retries: int
    wall: float

    def summary(self, warmup: int = 0) -> dict:
        lat = np.asarray(self.latencies[warmup:]) * 1e3
        waits = np.asarray(self.admission_waits[warmup:]) * 1e3
        n = len(lat)
        return {
            "requests": n,
            "p50_ms": round(float(np.percentile(lat, 50)), 3) if n else None,
            "p99_ms": round(float(np.percentile(lat, 99)), 3) if n else None,
            "views_per_s": round(len(self.latencies) / self.wall, 1) if self.wall > 0 else None,
            "mean_slots_in_flight": round(float(np.mean(self.slots_in_flight)), 2) if self.slots_in_flight else 0.0,
            "mean_admission_wait_ms": round(float(waits.mean()), 3) if n else None,
            "batches": self.batches,
            "mean_batch": round(float(np.mean(self.batch_sizes)), 2) if self.batch_sizes else 0.0,
            "max_bytes_in_use": int(self.max_bytes_in_use),
            "rejected": self.rejected,
            "retries": self.retries,
        }


class Scheduler:
    """Continuous batching with FIFO admission under a byte budget."""

    def __init__(self, executor, budget_bytes: int, slots: int = 8, max_batch: int = 16, max_views: int = 64):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.slots = int(slots)
        self.max_batch = int(max_batch)
        self.max_views = int(max_views)

    def run(self, requests, clock=time.perf_counter, idle=None) -> ServeStats:
        """Serves `requests` (sorted by arrival, in seconds from the start) to
        completion. `idle(t_next)` is called when nothing can progress before the
        next arrival (default: a short sleep)."""
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        queue = collections.deque()
        prepared = []                 # (request, handle) admitted, preparation enqueued
        batches = []                  # (token, [(request, handle)])
        free_slots = list(range(self.slots))
        used = 0
        lat, waits, inflight, sizes = [], [], [], []
        n_batches = max_used = n_retries = n_rejected = 0
        total = len(pending)
        finished = 0
        t0 = clock()
        while finished < total:
            now = clock() - t0
            while pending and pending[0].arrival <= now:
                queue.append(pending.popleft())
            # completions first: they free slots and bytes for this tick's admissions
            still = []
            for token, members in batches:
                if not self.ex.poll(token):
                    still.append((token, members))
                    continue
                t_done = clock() - t0
                for req, h in members:
                    ok, need = self.ex.finish(h)
                    used -= req.nbytes
                    free_slots.append(h.slot)
                    if ok:
                        req.done = t_done
                        lat.append(req.done - req.arrival)
                        waits.append(req.admitted - req.arrival)
                        finished += 1
                    else:
                        req.nbytes = int(need)
                        req.retries += 1
                        n_retries += 1
                        queue.appendleft(req)
            batches = still
            # admission: FIFO, while a slot and the bytes are free
            while queue and free_slots:
                req = queue[0]
                if req.nbytes == 0:
                    req.nbytes = int(self.ex.bytes_needed(req))
                if req.nbytes > self.budget:
                    queue.popleft()
                    req.rejected = True
                    n_rejected += 1
                    finished += 1
                    continue
                if used + req.nbytes > self.budget:
                    break
                queue.popleft()
                used += req.nbytes
                max_used = max(max_used, used)
                if req.admitted is None:
                    req.admitted = clock() - t0
                prepared.append((req, self.ex.start(req, free_slots.pop())))
            # one batched raster over everything prepared (bounded by the launch limits)
            while prepared:
                take, views = [], 0
                while prepared and len(take) < self.max_batch and views + prepared[0][1].views <= self.max_views:
                    views += prepared[0][1].views
                    take.append(prepared.pop(0))
                batches.append((self.ex.launch([h for _, h in take]), take))
                n_batches += 1
                sizes.append(len(take))
            inflight.append(self.slots - len(free_slots))
            if not batches and not prepared and finished < total:
                nxt = pending[0].arrival if pending else None
                if not queue and nxt is not None:
                    (idle or _sleep_until(clock, t0))(nxt)
            elif batches:
                if idle is not None:
                    idle(None)
        return ServeStats(lat, waits, inflight, n_batches, sizes, max_used, n_rejected, n_retries, clock() - t0)


def _sleep_until(clock, t0):
    def idle(t_next):
        dt = t_next - (clock() - t0)
        if dt > 0:
            time.sleep(min(dt, 1e-3))
    return idle


# --------------------------------------------------------------------------- GPU executor
class _Handle:
    __slots__ = ("req", "frame", "event", "slot", "views", "ws")

    def __init__(self, req, frame, event, slot, views, ws):
        self.req, self.frame, self.event, self.slot, self.views, self.ws = req, frame, event, slot, views, ws


class GpuExecutor:
    """Runs requests through the library: gsr_prepare on per-slot streams, one
    gsr_raster_batch per launch on the raster stream (which first waits for the
    slots' preparations), completion by HIP events."""

    def __init__(self, rasterizer, scenes: dict, precision=None, slots: int = 8, instance_margin: float = 1.5):
        import torch
        from . import _lib as L
        self.torch = torch
        self.L = L
        self.rz = rasterizer
        self.scenes = scenes
        self.precision = L.GSR_FP16_BLEND if precision is None else precision
        self.streams = [torch.cuda.Stream(device=rasterizer.device) for _ in range(slots)]
        self.raster_stream = torch.cuda.Stream(device=rasterizer.device)
        self.margin = instance_margin
        self.max_device_retries = 3
        self.density = {}  # instances per pixel of each scene, from one probe view

    def calibrate(self, name, camera):
        """Instances per pixel of a probe view of the scene (the largest over the
        probes given): the planner's bound for a request is margin x density x pixels
        instances. A frame that outgrows its bound raises its scene's density."""
        fr = self.rz.forward(self.scenes[name], [camera], precision=self.precision)
        d = fr.info["instances"] / float(camera.width * camera.height)
        self.density[name] = max(self.density.get(name, 0.0), d)
        fr.workspace._release()

    def bytes_needed(self, req) -> int:
        import ctypes
        from .raster import camera_struct
        st = self.scenes[req.scene]
        cams = (self.L.GsrCamera * 1)(camera_struct(req.camera))
        opts = self.rz.options(self.precision, True, False)
        m = int(self.margin * self.density.get(req.scene, 8.0) * req.camera.width * req.camera.height) + 4096
        nbytes = ctypes.c_size_t()
        sc = st.struct()
        self.rz._check(self.rz.lib.gsr_workspace_size(self.rz.ctx, ctypes.byref(sc), cams, 1, ctypes.byref(opts), m,
                                                      ctypes.byref(nbytes)), "gsr_workspace_size")
        return int(nbytes.value) + 512

    def start(self, req, slot) -> _Handle:
        from .raster import Workspace
        torch = self.torch
        s = self.streams[slot]
        with torch.cuda.stream(s):
            ws = Workspace(self.rz.device)
            ws.ensure(req.nbytes - 512)
            frame = self.rz.prepare(self.scenes[req.scene], [req.camera], stats=False, workspace=ws, stream=s)
            ev = torch.cuda.Event()
            ev.record(s)
        return _Handle(req, frame, ev, slot, 1, ws)

    def launch(self, handles):
        torch = self.torch
        rs = self.raster_stream
        with torch.cuda.stream(rs):
            for h in handles:
                rs.wait_event(h.event)
                h.ws.buf.record_stream(rs)
            imgs = self.rz.raster_batch([h.frame for h in handles], precision=self.precision, stream=rs)
            ev = torch.cuda.Event()
            ev.record(rs)
        for h, im in zip(handles, imgs):
            h.req.images = im
        return ev

    def poll(self, token) -> bool:
        return token.query()

    def finish(self, h):
        st, info = self.rz._inspect(h.ws, None)
        need = 0
        ok = st == self.L.GSR_OK
        if st == self.L.GSR_ERR_WORKSPACE_TOO_SMALL:
            need = int(self.rz.lib.gsr_required_workspace(self.rz.ctx)) + 512
            cam = h.req.camera
            seen = 1.1 * info["instances"] / float(cam.width * cam.height) / self.margin
            self.density[h.req.scene] = max(self.density.get(h.req.scene, 0.0), seen)
        elif st == self.L.GSR_ERR_DEVICE and h.req.retries < self.max_device_retries:
            # the frame's device-wide waits ran out of time and were abandoned (frames
            # prepared on concurrent streams can starve each other's look-back): render again
            need = h.req.nbytes
        elif st != self.L.GSR_OK:
            self.rz._check(st, "gsr_frame_inspect")
        h.ws._release()
        h.ws.buf = None
        h.frame = None
        return ok, need


# --------------------------------------------------------------------------- workload
RESOLUTIONS = ((256, 256), (512, 512), (1280, 720), (1920, 1080))


def request_stream(scene_radii: dict, n: int, rate: float, seed: int = 7):
    """n requests with Poisson arrivals at `rate` per second: scene uniform over the
    resident ones, orbit azimuth U(0, 360), elevation U(-10, 30) degrees at the
    scene's orbit radius, resolution uniform over RESOLUTIONS (60 degree FoV)."""
    from . import scenes
    rng = np.random.default_rng(seed)
    names = sorted(scene_radii)
    t = 0.0
    out = []
    for i in range(n):
        t += rng.exponential(1.0 / rate)
        name = names[int(rng.integers(0, len(names)))]
        w, h = RESOLUTIONS[int(rng.integers(0, len(RESOLUTIONS)))]
        cam = scenes.orbit_camera(float(rng.uniform(0, 360)), float(rng.uniform(-10, 30)),
                                  radius=scene_radii[name], width=w, height=h, fov_x=60.0)
        out.append(Request(i, name, cam, t))
    return out


def resident_scenes(rasterizer, sizes=(100_000, 500_000, 1_000_000, 2_000_000)):
    """The four serving scenes (SH3): spheres-and-planes at the two smaller sizes,
    the room and the unbounded layout, Morton-ordered on the device. Returns
    ({name: SceneTensors}, {name: orbit radius})."""
    from . import scenes
    from .raster import SceneTensors
    gens = [("spheres-%dk" % (sizes[0] // 1000), lambda: scenes.spheres_planes_scene(sizes[0], seed_salt=11), 7.0),
            ("spheres-%dk" % (sizes[1] // 1000), lambda: scenes.spheres_planes_scene(sizes[1], seed_salt=12), 7.0),
            ("room-%dk" % (sizes[2] // 1000), lambda: scenes.room_scene(sizes[2], seed_salt=13), 3.0),
            ("unbounded-%dk" % (sizes[3] // 1000), lambda: scenes.unbounded_scene(sizes[3], seed_salt=14), 6.0)]
    out, radii = {}, {}
    for name, gen, radius in gens:
        st = SceneTensors.from_scene(gen(), rasterizer.device)
        perm, _ = rasterizer.morton_order(st.means)
        st = SceneTensors(*rasterizer.apply_permutation(perm, list(st.tensors())), st.sh_degree)
        out[name] = st
        radii[name] = radius
    return out, radii


def serve_benchmark(rasterizer, n_warmup=200, n_measured=3000, rate=200.0, budget_bytes=4 << 30, slots=8,
                    sizes=(100_000, 500_000, 1_000_000, 2_000_000), log=None, more_rates=()):
    """The serving stream: resident scenes, Poisson arrivals, FP16-blend forward;
    returns the latency / throughput summary over the measured requests. more_rates:
    further streams over the same resident scenes at other arrival rates (past
    capacity, views/s saturates and batches grow), summarised under "rate_sweep"."""
    from . import scenes as S
    res, radii = resident_scenes(rasterizer, sizes)
    ex = GpuExecutor(rasterizer, res, slots=slots)
    for name in res:
        for az in (0.0, 90.0, 180.0, 270.0):
            ex.calibrate(name, S.orbit_camera(az, 10.0, radius=radii[name], width=512, height=512, fov_x=60.0))
    out = None
    sweep = []
    for r in (rate,) + tuple(more_rates):
        reqs = request_stream(radii, n_warmup + n_measured, r)
        if log:
            log("serving %d requests at %.0f/s over %d scenes (budget %.1f GiB, %d slots)"
                % (len(reqs), r, len(res), budget_bytes / 2 ** 30, slots))
        sched = Scheduler(ex, budget_bytes, slots=slots)
        stats = sched.run(reqs)
        summ = stats.summary(warmup=n_warmup)
        summ["rate_per_s"] = r
        if out is None:
            out = summ
            out["budget_bytes"] = int(budget_bytes)
            out["scenes"] = sorted(res)
        else:
            sweep.append(summ)
    out["rate_sweep"] = sweep
    return out


def percentile(xs, p):
    s = sorted(xs)
    if not s:
        return math.nan
    k = (len(s) - 1) * p / 100.0
    lo, hi = math.floor(k), math.ceil(k)
    return s[lo] + (s[hi] - s[lo]) * (k - lo)
