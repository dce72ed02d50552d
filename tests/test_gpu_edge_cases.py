"""The method's edge cases, GPU against the FP64 oracle on the same inputs.

Each case mirrors an oracle pin (the pin fixes the oracle, this test holds the
GPU path to the oracle): the alpha clamp at 0.99 and its zero derivative, five
stacked Gaussians of alpha 0.95 of which exactly three blend, the clamped EWA
Jacobian beyond 1.3 x the half field of view, a 1:100 needle (a screen
covariance with condition number ~1200), a Gaussian straddling the near plane
and one just in front of it, and the cluster bounds buffer. Bars as in
tests/parity.py: images and T within 1e-5, the last blended position exact on
non-fragile pixels, every gradient and S, M per element within 1e-3, C within
the oracle's per-Gaussian slack.
"""
import math

import numpy as np
import pytest
import torch

import oracle as orc
from helpers import ensure_built
from paper_2503_01199_amd import scenes
from parity import camera, full_parity, gaussians

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rz():
    ensure_built()
    from paper_2503_01199_amd.raster import Rasterizer
    return Rasterizer(0)


def _with_background(sc_front, n=300, salt=0, W=32, H=32):
    """Appends n small random Gaussians behind the case so that tiles carry lists."""
    rng = np.random.default_rng([4242, salt])
    means = np.stack([rng.uniform(-0.8, 0.8, n), rng.uniform(-0.8, 0.8, n), rng.uniform(3.5, 5.0, n)], 1)
    K = (sc_front.sh_degree + 1) ** 2
    sh = np.zeros((n, K, 3))
    sh[:, 0, :] = rng.normal(0, 0.5, (n, 3))
    bg = scenes.Scene(*(np.ascontiguousarray(a, np.float32) for a in
                        (means, rng.normal(-2.5, 0.3, (n, 3)), rng.standard_normal((n, 4)),
                         rng.normal(0, 1, n), sh)), sc_front.sh_degree)
    cat = lambda a, b: np.ascontiguousarray(np.concatenate([a, b]), np.float32)  # noqa: E731
    return scenes.Scene(cat(sc_front.means, bg.means), cat(sc_front.log_scales, bg.log_scales),
                        cat(sc_front.quats, bg.quats), cat(sc_front.opacity_logits, bg.opacity_logits),
                        cat(sc_front.sh, bg.sh), sc_front.sh_degree)


def test_alpha_clamp_forward_and_zero_derivative(rz):
    """A large Gaussian with opacity 0.999 (alpha clamped to 0.99 wherever
    o G > 0.99, about a hundred pixels) and one of opacity 0.7 behind it, in front
    of random ones: at the clamped pixels the front Gaussian's opacity derivative is
    zero on both sides, so its opacity gradient comes only from the rim where the
    clamp does not hold. (Two clamped Gaussians in a row would leave T exactly at
    the 1e-4 stop, a fragile decision.)"""
    cam = camera(W=32, H=32, f=32.0, cx=16.5, cy=16.5, bg=(0.2, 0.3, 0.1))
    front = gaussians([[0, 0, 2.0], [0.3, -0.2, 2.5]], [math.log(3.0), math.log(2.5), math.log(2.8)],
                      [0.9, 0.1, -0.2, 0.3], [0.999, 0.7], [[0.9, 0.2, 0.4], [0.1, 0.8, 0.3]])
    sc = _with_background(front, salt=1)
    pp = orc.preprocess(sc, cam)
    py, px = np.mgrid[0:32, 0:32]
    dx, dy = px + 0.5 - pp["u"][0], py + 0.5 - pp["v"][0]
    a, b, c = pp["conic"][0]
    clamped = pp["opacity"][0] * np.exp(-0.5 * (a * dx * dx + 2 * b * dx * dy + c * dy * dy)) > 0.99
    print("clamped pixels: %d" % clamped.sum())
    assert clamped.sum() > 80
    full_parity(rz, sc, [cam], "alpha clamp", salt=1)


def test_alpha_095_stack_blends_exactly_three(rz):
    cam = camera(W=32, H=32, f=32.0, cx=16.5, cy=16.5)
    n = 5
    sc = gaussians([[0, 0, 2.0 + 0.1 * i] for i in range(n)], math.log(3.0), [1, 0, 0, 0], [0.95] * n,
                   [[0.5, 0.5, 0.5]] * n)
    fr, ins, refs, ref = full_parity(rz, sc, [cam], "alpha 0.95 stack", salt=2)
    T = ins["pixel_T"].cpu().numpy().reshape(32, 32)
    last = ins["pixel_last"].cpu().numpy().view(np.uint32).reshape(32, 32)
    o = 1 / (1 + np.exp(-np.float64(sc.opacity_logits[0])))
    print("centre pixel: T %.9g (expected %.9g), last %d" % (T[16, 16], (1 - o) ** 3, last[16, 16]))
    assert last[16, 16] == 3
    assert abs(T[16, 16] - (1 - o) ** 3) <= 1e-5 * (1 - o) ** 3 + 1e-9
    # every Gaussian but the last two blends at the centre: C counts them
    assert refs[0]["n_blended"][16, 16] == 3


def test_clamped_jacobian_gradients(rz):
    """The three off-axis Gaussians of the oracle's clamp pin (two beyond
    x/z = 0.65), their footprints reaching into the image."""
    cam = camera(W=48, H=40, f=48.0, bg=(0.1, 0.1, 0.1))
    means = [[1.6, 0.1, 2.0], [-1.7, -0.2, 2.1], [0.1, 1.3, 1.9]]
    sc = gaussians(means, [math.log(0.5), math.log(0.3), math.log(0.4)], [0.8, 0.3, -0.2, 0.4], [0.7, 0.8, 0.6],
                   [[0.9, 0.2, 0.4], [0.1, 0.8, 0.3], [0.5, 0.5, 0.9]])
    pp = orc.preprocess(sc, cam)
    assert np.sum(np.abs(pp["tcam"][:, 0] / pp["tcam"][:, 2]) > 1.3 * 48 / 96) == 2 and pp["valid"].all()
    full_parity(rz, sc, [cam], "clamped Jacobian", salt=3)


@pytest.mark.parametrize("angle", [30.0, 73.0])
def test_needle_one_to_hundred(rz, angle):
    """A 1:100 needle 20 px long, rotated in the image plane and tilted out of it,
    over random Gaussians: the screen covariance is ill-conditioned (the FP32
    conditioning case of the projection)."""
    z, f = 3.0, 64.0
    s1 = 20.0 * z / f
    th = math.radians(angle)
    q = np.array([math.cos(th / 2), 0.15, 0.1, math.sin(th / 2)])
    front = gaussians([[0.05, -0.03, z]], [math.log(s1), math.log(s1 / 100), math.log(s1 / 100)], q, 0.9,
                      [0.9, 0.4, 0.2])
    sc = _with_background(front, salt=4, W=64, H=64)
    cam = camera(W=64, H=64, f=f)
    pp = orc.preprocess(sc, cam)
    cov = pp["cov"][0]
    kappa = np.linalg.cond(np.array([[cov[0], cov[1]], [cov[1], cov[2]]]))
    print("needle screen covariance condition number %.0f" % kappa)
    assert kappa > 500
    full_parity(rz, sc, [cam], "needle %g deg" % angle, salt=4)


def test_near_plane_straddle(rz):
    """A Gaussian whose mean lies just beyond the near plane (0.2) but whose extent
    reaches behind it, one just in front of the near plane (culled), and random
    Gaussians behind."""
    cam = camera(W=48, H=48, f=48.0, near=0.2)
    front = gaussians([[0.002, 0.001, 0.23], [0.0, 0.0, 0.19], [0.01, -0.01, 0.4]],
                      [math.log(0.05), math.log(0.02), math.log(0.03)], [0.95, 0.2, 0.1, -0.2],
                      [0.7, 0.8, 0.6], [[0.9, 0.2, 0.4], [0.1, 0.8, 0.3], [0.5, 0.5, 0.9]])
    sc = _with_background(front, salt=5, W=48, H=48)
    pp = orc.preprocess(sc, cam)
    assert pp["valid"][0] and not pp["valid"][1] and pp["valid"][2]
    assert pp["tcam"][0, 2] - 3 * 0.05 < 0.2  # three scales reach behind the near plane
    fr, ins, refs, ref = full_parity(rz, sc, [cam], "near plane", salt=5)
    assert ref["C"][1] == 0


@pytest.mark.parametrize("n", [1024, 1000, 129])
def test_cluster_bounds_buffer(rz, n):
    """The cluster bounds buffer (min and max of the means and the largest
    log-scale per 128 Gaussians, ragged last cluster) equals the oracle's, bit for
    bit."""
    sc = scenes.tiny_scene(n, seed_salt=6)
    from paper_2503_01199_amd.raster import SceneTensors, Workspace
    fr = rz.forward(SceneTensors.from_scene(sc, rz.device), [scenes.tiny_camera()], workspace=Workspace(rz.device))
    ins = rz.inspect(fr)
    got = ins["cluster_bounds"].cpu().numpy()
    ref = orc.cluster_bounds(sc.means, sc.log_scales, 128)
    nc = -(-n // 128)
    assert got.shape[0] >= nc and ref.shape[0] == nc
    assert np.array_equal(got[:nc, :7].view(np.uint32), ref[:, :7].astype(np.float32).view(np.uint32))
