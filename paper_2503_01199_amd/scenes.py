"""Seeded synthetic inputs: Gaussian scenes, cameras, loss weights and optimiser state.

This module only draws inputs. It holds none of the rasterizer's arithmetic, and it
is the one module that both the GPU path and the test oracle receive data from.
Every generator is deterministic given its seed (``numpy.random.default_rng``).

The paper measures on captured datasets that are not available here. The scenes
below are synthetic stand-ins with the shapes of its workloads: surface-distributed
Gaussians whose footprints overlap the way a trained scene's do, an SH colour
model of degree 0 or 3, and image sizes of the paper's benchmark frames.

Conventions shared by every consumer:
  * means f32[N,3] (world), log_scales f32[N,3], quats f32[N,4] as (w, x, y, z),
    opacity_logits f32[N], sh f32[N,K,3] with K = (degree+1)^2;
  * a camera maps world to camera space by x_cam = R @ x_world + t with x right,
    y down, z forward; pixel (px, py) has its centre at (px + 1/2, py + 1/2).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_BASE = 20250301


@dataclasses.dataclass
class Scene:
    means: np.ndarray
    log_scales: np.ndarray
    quats: np.ndarray
    opacity_logits: np.ndarray
    sh: np.ndarray
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return Scene(self.means[idx].copy(), self.log_scales[idx].copy(), self.quats[idx].copy(),
                     self.opacity_logits[idx].copy(), self.sh[idx].copy(), self.sh_degree)

    def permuted(self, perm) -> "Scene":
        return self.subset(perm)

    def arrays(self):
        return (self.means, self.log_scales, self.quats, self.opacity_logits, self.sh)


@dataclasses.dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray            # f32[3,3] world -> camera
    t: np.ndarray            # f32[3]
    near: float = 0.2
    bg: tuple = (0.0, 0.0, 0.0)

    def tiles(self, tile: int = 16):
        return ((self.width + tile - 1) // tile, (self.height + tile - 1) // tile)


def rng_for(config: int, salt: int = 0) -> np.random.Generator:
    return np.random.default_rng([SEED_BASE, config, salt])


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _finish(means, log_scales, quats, logits, sh, degree) -> Scene:
    return Scene(_f32(means), _f32(log_scales), _f32(quats), _f32(logits), _f32(sh), int(degree))


def random_quats(rng, n):
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def frame_to_quats(t1, t2, nrm):
    """Unit quaternions (w, x, y, z) of the rotations whose columns are (t1, t2, nrm)."""
    m = np.stack([t1, t2, nrm], axis=2)  # [n,3,3], columns
    n = m.shape[0]
    q = np.empty((n, 4))
    tr = m[:, 0, 0] + m[:, 1, 1] + m[:, 2, 2]
    w = np.sqrt(np.maximum(0.0, 1.0 + tr)) / 2
    x = np.sqrt(np.maximum(0.0, 1.0 + m[:, 0, 0] - m[:, 1, 1] - m[:, 2, 2])) / 2
    y = np.sqrt(np.maximum(0.0, 1.0 - m[:, 0, 0] + m[:, 1, 1] - m[:, 2, 2])) / 2
    z = np.sqrt(np.maximum(0.0, 1.0 - m[:, 0, 0] - m[:, 1, 1] + m[:, 2, 2])) / 2
    x = np.copysign(x, m[:, 2, 1] - m[:, 1, 2])
    y = np.copysign(y, m[:, 0, 2] - m[:, 2, 0])
    z = np.copysign(z, m[:, 1, 0] - m[:, 0, 1])
    q[:, 0], q[:, 1], q[:, 2], q[:, 3] = w, x, y, z
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def _tangent_frame(rng, nrm):
    a = np.where(np.abs(nrm[:, :1]) < 0.9, np.array([[1.0, 0, 0]]), np.array([[0, 1.0, 0]]))
    t1 = np.cross(nrm, a)
    t1 /= np.linalg.norm(t1, axis=1, keepdims=True)
    t2 = np.cross(nrm, t1)
    ang = rng.uniform(0, 2 * np.pi, size=(nrm.shape[0], 1))
    c, s = np.cos(ang), np.sin(ang)
    return c * t1 + s * t2, -s * t1 + c * t2


def surface_gaussians(rng, points, normals, area_total, n, degree, sh_sigma=0.2,
                      jitter=0.01, tangential_sigma=0.3):
    """Gaussians lying on surfaces: local z along the normal, flat (10:1) discs whose
    tangential size follows the mean spacing d = sqrt(area / n), so that the surface
    is covered about as densely as in a trained scene."""
    d = math.sqrt(area_total / n)
    pts = points + normals * rng.normal(0.0, jitter, size=(n, 1))
    t1, t2 = _tangent_frame(rng, normals)
    quats = frame_to_quats(t1, t2, normals)
    ls = np.empty((n, 3))
    ls[:, 0] = math.log(0.6 * d) + rng.normal(0, tangential_sigma, n)
    ls[:, 1] = math.log(0.6 * d) + rng.normal(0, tangential_sigma, n)
    ls[:, 2] = math.log(0.06 * d)
    logits = rng.normal(0.0, 1.0, n)
    K = (degree + 1) ** 2
    sh = rng.normal(0.0, sh_sigma, size=(n, K, 3))
    return _finish(pts, ls, quats, logits, sh, degree)


def look_at(eye, target, down=(0.0, 1.0, 0.0)):
    """World->camera (R, t) for a camera at `eye` looking at `target`. The camera
    frame is x right, y down, z forward; `down` is the world direction that
    appears at the bottom of the image (world y points down by default)."""
    eye = np.asarray(eye, dtype=np.float64)
    f = np.asarray(target, dtype=np.float64) - eye
    f /= np.linalg.norm(f)
    dn = np.asarray(down, dtype=np.float64)
    x = np.cross(dn, f)
    if np.linalg.norm(x) < 1e-9:
        x = np.cross(np.array([0.0, 0.0, 1.0]), f)
    x /= np.linalg.norm(x)
    y = np.cross(f, x)
    R = np.stack([x, y, f], axis=0)
    t = -R @ eye
    return _f32(R), _f32(t)


def pinhole(width, height, fov_x_deg, R, t, near=0.2, bg=(0.0, 0.0, 0.0)) -> Camera:
    fx = (width / 2.0) / math.tan(math.radians(fov_x_deg) / 2.0)
    return Camera(int(width), int(height), float(np.float32(fx)), float(np.float32(fx)),
                  width / 2.0, height / 2.0, _f32(R), _f32(t), near, tuple(bg))


# --------------------------------------------------------------------------- C1
def tiny_scene(n=1024, seed_salt=0):
    """1,024 Gaussians uniform in x, y in [-1, 1], z in [2, 6] before an identity
    camera; log-scales N(-3, 0.5); random unit quaternions; logits N(0, 1); SH
    degree 0 whose DC coefficient ~ U(-sqrt(pi), sqrt(pi)) makes the rendered colour
    U(0, 1) (the constant basis function is 1/(2 sqrt(pi)), plus the 1/2 offset)."""
    rng = rng_for(0, seed_salt)
    means = np.stack([rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(2, 6, n)], axis=1)
    ls = rng.normal(-3.0, 0.5, size=(n, 3))
    quats = random_quats(rng, n)
    logits = rng.normal(0.0, 1.0, n)
    sh = rng.uniform(-math.sqrt(math.pi), math.sqrt(math.pi), size=(n, 1, 3))
    return _finish(means, ls, quats, logits, sh, 0)


def tiny_camera(width=128, height=128):
    return Camera(width, height, 128.0, 128.0, width / 2.0, height / 2.0,
                  np.eye(3, dtype=np.float32), np.zeros(3, dtype=np.float32))


# --------------------------------------------------------------------------- C2
def _sample_sphere(rng, c, r, n):
    v = rng.standard_normal((n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return c + r * v, v


def _sample_square(rng, center, u, v, nrm, half, n):
    a = rng.uniform(-half, half, size=(n, 1))
    b = rng.uniform(-half, half, size=(n, 1))
    p = center + a * u + b * v
    return p, np.repeat(np.asarray(nrm, dtype=np.float64)[None], n, axis=0)


def spheres_planes_scene(n=200_000, degree=3, seed_salt=0):
    """Gaussians on 10 random spheres (centres U([-2,2]^3), radii U(0.3, 1)) and 4
    6x6 squares (floor y = 2.5 with y down, back wall z = -3, side walls x = +-3),
    area-weighted, jittered along the normal by N(0, 0.01)."""
    rng = rng_for(1, seed_salt)
    shapes = []
    for _ in range(10):
        shapes.append(("sphere", rng.uniform(-2, 2, 3), rng.uniform(0.3, 1.0)))
    e = np.eye(3)
    shapes.append(("square", np.array([0, 2.5, 0.0]), e[0], e[2], -e[1], 3.0))
    shapes.append(("square", np.array([0, 0, -3.0]), e[0], e[1], e[2], 3.0))
    shapes.append(("square", np.array([-3.0, 0, 0]), e[1], e[2], e[0], 3.0))
    shapes.append(("square", np.array([3.0, 0, 0]), e[1], e[2], -e[0], 3.0))
    areas = np.array([4 * np.pi * s[2] ** 2 if s[0] == "sphere" else (2 * s[5]) ** 2 for s in shapes])
    counts = rng.multinomial(n, areas / areas.sum())
    pts, nrms = [], []
    for s, k in zip(shapes, counts):
        if s[0] == "sphere":
            p, q = _sample_sphere(rng, s[1], s[2], k)
        else:
            p, q = _sample_square(rng, s[1], s[2], s[3], s[4], s[5], k)
        pts.append(p)
        nrms.append(q)
    pts = np.concatenate(pts)
    nrms = np.concatenate(nrms)
    order = rng.permutation(n)  # arrival order unrelated to space
    return surface_gaussians(rng, pts[order], nrms[order], areas.sum(), n, degree)


def spheres_planes_camera():
    R, t = look_at((0.0, -0.5, 7.0), (0.0, 0.0, 0.0))
    return pinhole(800, 800, 50.0, R, t)


# --------------------------------------------------------------------------- C3
def room_scene(n=1_000_000, degree=3, seed_salt=0):
    """A closed room: the 6 inward faces of [-5,5]x[-1.5,1.5]x[-4,4] plus 50
    ellipsoids (centres uniform in the room shrunk by 1 m, semi-axes U(0.1, 0.6),
    random rotations); Gaussians area-weighted on them as for spheres_planes_scene."""
    rng = rng_for(2, seed_salt)
    lo = np.array([-5.0, -1.5, -4.0])
    hi = np.array([5.0, 1.5, 4.0])
    ext = hi - lo
    faces = []
    for ax in range(3):
        o1, o2 = [a for a in range(3) if a != ax]
        for side, sgn in ((lo[ax], 1.0), (hi[ax], -1.0)):
            faces.append((ax, o1, o2, side, sgn))
    face_areas = [ext[f[1]] * ext[f[2]] for f in faces]
    ells = []
    for _ in range(50):
        c = rng.uniform(lo + 1.0, hi - 1.0)
        ax = rng.uniform(0.1, 0.6, 3)
        Rm = _rotmat(random_quats(rng, 1)[0])
        p = 1.6075
        area = 4 * np.pi * (((ax[0] * ax[1]) ** p + (ax[0] * ax[2]) ** p + (ax[1] * ax[2]) ** p) / 3) ** (1 / p)
        ells.append((c, ax, Rm, area))
    areas = np.array(face_areas + [e[3] for e in ells])
    counts = rng.multinomial(n, areas / areas.sum())
    pts, nrms = [], []
    for f, k in zip(faces, counts[:6]):
        ax, o1, o2, side, sgn = f
        p = np.empty((k, 3))
        p[:, ax] = side
        p[:, o1] = rng.uniform(lo[o1], hi[o1], k)
        p[:, o2] = rng.uniform(lo[o2], hi[o2], k)
        q = np.zeros((k, 3))
        q[:, ax] = sgn
        pts.append(p)
        nrms.append(q)
    for (c, ax, Rm, _), k in zip(ells, counts[6:]):
        v = rng.standard_normal((k, 3))
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        p = c + (v * ax) @ Rm.T
        nn = (v / ax) @ Rm.T
        nn /= np.linalg.norm(nn, axis=1, keepdims=True)
        pts.append(p)
        nrms.append(nn)
    pts = np.concatenate(pts)
    nrms = np.concatenate(nrms)
    order = rng.permutation(n)
    return surface_gaussians(rng, pts[order], nrms[order], areas.sum(), n, degree)


def _rotmat(q):
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def room_camera(width=1600, height=1064):
    R, t = look_at((0.0, 0.0, 3.0), (0.0, 0.0, -1.0))
    return pinhole(width, height, 70.0, R, t)


def room_cycle_cameras(k=16, width=1600, height=1064):
    """k views of the room from an ellipse at mid-height (semi-axes 3.5 m along x,
    2.5 m along z), evenly spaced in angle, each looking at the room's centre: a
    cycle over which no view's working set stays cache-resident."""
    cams = []
    for i in range(k):
        a = 2.0 * math.pi * i / k
        R, t = look_at((3.5 * math.sin(a), 0.0, 2.5 * math.cos(a)), (0.0, 0.0, 0.0))
        cams.append(pinhole(width, height, 70.0, R, t))
    return cams


# --------------------------------------------------------------------------- C4
def unbounded_scene(n=3_000_000, degree=3, seed_salt=0):
    """60% of the Gaussians volume-uniform in a ball of radius 10 (log-scales
    ln(0.6 d) + N(0, 0.5), d = (V/N_ball)^(1/3)), 40% on a shell whose radius is
    log-uniform in [10, 100] (scale 0.6 r sqrt(4 pi / N_shell) e^N(0, 0.5)); random
    rotations."""
    rng = rng_for(3, seed_salt)
    nb = int(round(0.6 * n))
    ns = n - nb
    v = rng.standard_normal((nb, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    r = 10.0 * rng.uniform(0, 1, nb) ** (1 / 3)
    pb = v * r[:, None]
    d = (4 / 3 * np.pi * 1000.0 / nb) ** (1 / 3)
    lsb = math.log(0.6 * d) + rng.normal(0, 0.5, size=(nb, 3))
    v = rng.standard_normal((ns, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    rs = np.exp(rng.uniform(math.log(10.0), math.log(100.0), ns))
    ps = v * rs[:, None]
    lss = np.log(0.6 * rs * math.sqrt(4 * np.pi / ns))[:, None] + rng.normal(0, 0.5, size=(ns, 3))
    means = np.concatenate([pb, ps])
    ls = np.concatenate([lsb, lss])
    order = rng.permutation(n)
    K = (degree + 1) ** 2
    return _finish(means[order], ls[order], random_quats(rng, n), rng.normal(0, 1, n),
                   rng.normal(0, 0.2, size=(n, K, 3)), degree)


def orbit_camera(azimuth_deg, elevation_deg=10.0, radius=6.0, width=1920, height=1080, fov_x=60.0):
    az = math.radians(azimuth_deg)
    el = math.radians(elevation_deg)
    eye = (radius * math.cos(el) * math.sin(az), -radius * math.sin(el), radius * math.cos(el) * math.cos(az))
    R, t = look_at(eye, (0.0, 0.0, 0.0))
    return pinhole(width, height, fov_x, R, t)


def orbit_cameras(k=8, **kw):
    return [orbit_camera(360.0 * i / k, **kw) for i in range(k)]


# --------------------------------------------------------------------------- loss
def l1_weights(shape, config=0, salt=0):
    """Per-pixel, per-channel weights w ~ U(0,1) and targets gt ~ U(0,1) of the
    random-weighted L1 loss L = sum w |I - gt|."""
    rng = rng_for(100 + config, salt)
    w = rng.uniform(0, 1, size=shape).astype(np.float32)
    gt = rng.uniform(0, 1, size=shape).astype(np.float32)
    return w, gt


# ------------------------------------------------------------------ optimiser step
ADAM_GROUPS = ("means", "log_scales", "quats", "opacity_logits", "sh")


def adam_inputs(n, degree=3, salt=0, zero_rows=0.1):
    """Parameters, gradients and the two Adam moments of n Gaussians: four dicts
    over ADAM_GROUPS of f32 arrays with the scene shapes. Values span several
    decades, as a trained scene's do: p ~ N(0, 1); g, m ~ N(0, 1) 10^U(-6, -1);
    v = (N(0, 1) 10^U(-6, -1))^2 >= 0; a fraction `zero_rows` of the Gaussians have
    an exact zero gradient (Gaussians that no view blends)."""
    rng = rng_for(300, salt)
    K = (degree + 1) ** 2
    shapes = {"means": (n, 3), "log_scales": (n, 3), "quats": (n, 4), "opacity_logits": (n,), "sh": (n, K, 3)}
    zero = rng.uniform(0, 1, size=n) < zero_rows

    def spread(shape):
        return rng.standard_normal(shape) * 10.0 ** rng.uniform(-6, -1, size=shape)

    P, G, M, V = {}, {}, {}, {}
    for k, sh in shapes.items():
        P[k] = _f32(rng.standard_normal(sh))
        g = spread(sh)
        g[zero] = 0.0
        G[k] = _f32(g)
        M[k] = _f32(spread(sh))
        V[k] = _f32(spread(sh) ** 2)
    return P, G, M, V


def cluster_flags(nc, pattern="random", salt=0):
    """Visibility flags u32[nc] of clusters: 'all', 'none', 'random' (each visible
    with probability 1/2) or 'alternate' (even clusters)."""
    if pattern == "all":
        return np.ones(nc, np.uint32)
    if pattern == "none":
        return np.zeros(nc, np.uint32)
    if pattern == "alternate":
        return (np.arange(nc) % 2 == 0).astype(np.uint32)
    return (rng_for(301, salt).uniform(0, 1, size=nc) < 0.5).astype(np.uint32)


def densify_inputs(n, salt=0, zero_frac=0.2):
    """Densification metric f32[n] (C Var values log-uniform over 10^[-8, -2], a
    fraction zero_frac exactly 0: Gaussians no pixel blended) and the standard
    normal draws f32[n, 2, 3] that place the two children of a split."""
    rng = rng_for(302, salt)
    metric = 10.0 ** rng.uniform(-8, -2, size=n)
    metric[rng.uniform(0, 1, size=n) < zero_frac] = 0.0
    return _f32(metric), _f32(rng.standard_normal((n, 2, 3)))


def scene_by_name(name: str, n: int | None = None):
    if name == "tiny":
        return tiny_scene(n or 1024), [tiny_camera()]
    if name == "spheres":
        return spheres_planes_scene(n or 200_000), [spheres_planes_camera()]
    if name == "room":
        return room_scene(n or 1_000_000), [room_camera()]
    if name == "unbounded":
        return unbounded_scene(n or 3_000_000), orbit_cameras(8)
    raise KeyError(name)
