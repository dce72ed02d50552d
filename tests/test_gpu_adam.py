"""Adam at cluster granularity (Sec. 3.2.3) on the GPU against the FP64 oracle.

Parity bar, per float, from the FP32 arithmetic of the kernel (u = 2^-24; the
oracle gets the same FP32 inputs and computes in FP64):
  m' = b1 m + (1 - b1) g        rounding of (1 - b1), of its product with g and of
                                the fused add: |dm| <= 3u (|b1 m| + |(1 - b1) g|)
  v' = b2 v + (1 - b2) g^2      four roundings of non-negative terms: |dv| <= 5u v'
  den = sqrt(v') c + eps        (c = 1 / sqrt(1 - b2^t) rounded once) relative error
                                <= 8u, and the quotient m' / den, the rounded rate
                                lr / (1 - b1^t) and their product 3u more, so the
                                update d = step m' / den is off by at most
                                12u |d| + step |dm| / den
  p' = p - d                    plus u |p'|.
The tests allow twice each bound. A cluster whose flag is 0 must come back bit for
bit (parameters and both moments)."""
import numpy as np
import pytest
import torch

import oracle as orc
from helpers import ensure_built
from paper_2503_01199_amd import scenes

pytestmark = pytest.mark.gpu

U = 2.0 ** -24
LR = {"means": 1.6e-4, "log_scales": 5e-3, "quats": 1e-3, "opacity_logits": 2.5e-2, "sh_dc": 2.5e-3,
      "sh_rest": 1.25e-4}
KEYS = orc.ADAM_GROUPS


@pytest.fixture(scope="module")
def rz():
    ensure_built()
    from paper_2503_01199_amd.raster import Rasterizer
    return Rasterizer(0)


def _dev(d, rz):
    return {k: torch.as_tensor(v, device=rz.device).contiguous() for k, v in d.items()}


def _rates(k, shape):
    if k != "sh":
        return np.full(shape, LR[k])
    r = np.full(shape, LR["sh_rest"])
    r[:, 0, :] = LR["sh_dc"]
    return r


def _bounds(k, g, m_in, ref, b1, b2, eps, t, B_in=(0.0, 0.0, 0.0)):
    """Error bounds (of the module docstring) of one FP32 step whose reference
    outputs are ref = (p', m', v') and whose inputs m_in, g carry the bounds
    B_in = (Bp, Bm, Bv) of earlier steps (0 for exact FP32 inputs)."""
    rp, rm, rv = ref
    Bp_in, Bm_in, Bv_in = B_in
    b1f, b2f = float(np.float32(b1)), float(np.float32(b2))
    Bm = b1f * Bm_in + 3 * U * (np.abs(b1f * m_in) + np.abs((1 - b1f) * g))
    Bv = b2f * Bv_in + 5 * U * rv
    step = _rates(k, rp.shape) / (1 - b1f ** t)
    den = np.sqrt(rv / (1 - b2f ** t)) + float(np.float32(eps))
    d = step * rm / den
    Bp = Bp_in + U * np.abs(rp) + 12 * U * np.abs(d) + step * Bm / den + 0.5 * np.abs(d) * b2f * Bv_in / rv
    return Bp, Bm, Bv


def _assert_within(k, got, ref, bounds):
    for name, a, b, bound in zip("pmv", got, ref, bounds):
        err = np.abs(np.asarray(a, np.float64) - b)
        bad = err > 2 * bound
        assert not bad.any(), "%s.%s: %d floats over the bar, worst %.3g vs bound %.3g" % (
            k, name, int(bad.sum()), float(err[bad].max()), float(2 * bound[bad][np.argmax(err[bad])]))


def _check(k, got, ref, inp, b1, b2, eps, t, rows):
    """got / ref: (p, m, v) of group k (rows = the Gaussians compared); inp: (p, g, m, v)
    FP32 inputs. Asserts twice the bounds of the module docstring."""
    _, g, m0, _ = (np.asarray(x, np.float64)[rows] for x in inp)
    ref = tuple(np.asarray(x, np.float64)[rows] for x in ref)
    got = tuple(np.asarray(x, np.float64)[rows] for x in got)
    _assert_within(k, got, ref, _bounds(k, g, m0, ref, b1, b2, eps, t))


def _run_case(rz, n, degree, flags, t, b1=0.9, b2=0.999, eps=1e-15, salt=0):
    P, G, M, V = scenes.adam_inputs(n, degree, salt=salt)
    dP, dG, dM, dV = _dev(P, rz), _dev(G, rz), _dev(M, rz), _dev(V, rz)
    vis = None if flags is None else torch.as_tensor(flags.astype(np.int32), device=rz.device)
    print("sparse adam n=%d degree=%d t=%d flags=%s" % (n, degree, t, None if flags is None else int(flags.sum())),
          flush=True)
    rz.sparse_adam(dP, dG, dM, dV, vis, LR, t, b1, b2, eps)
    torch.cuda.synchronize()
    rp, rm, rv = orc.sparse_adam(P, G, M, V, flags, LR, float(np.float32(b1)), float(np.float32(b2)),
                                 float(np.float32(eps)), t)
    rows = np.ones(n, bool) if flags is None else np.repeat(flags != 0, 128)[:n]
    for k in KEYS:
        got = (dP[k].cpu().numpy(), dM[k].cpu().numpy(), dV[k].cpu().numpy())
        for a, b in zip(got, (P[k], M[k], V[k])):  # culled clusters: untouched, bit for bit
            assert np.array_equal(a[~rows], b[~rows]), k
        _check(k, got, (rp[k], rm[k], rv[k]), (P[k], G[k], M[k], V[k]), b1, b2, eps, t, rows)
    return dP, dM, dV


@pytest.mark.parametrize("n,degree,pattern,t", [
    (37, 3, "all", 1),               # one partial cluster
    (128 * 9 + 37, 3, "random", 1),  # full clusters and a ragged tail
    (128 * 20, 2, "all", 17),        # 27-float SH rows: float4 units straddle rows
    (1000, 0, "alternate", 250),     # degree 0: the SH row is DC only
    (128 * 50 + 5, 1, "none", 3),    # nothing visible: nothing moves
    (128 * 33 + 100, 3, "random", 10_000),
])
def test_sparse_adam_matches_oracle(rz, n, degree, pattern, t):
    flags = scenes.cluster_flags((n + 127) // 128, pattern, salt=n)
    _run_case(rz, n, degree, flags, t, salt=degree)


def test_dense_adam_when_no_flags(rz):
    _run_case(rz, 128 * 7 + 64, 3, None, 5, b1=0.8, b2=0.95, eps=1e-8, salt=4)


def test_empty_scene_is_a_no_op(rz):
    from paper_2503_01199_amd.raster import GRAD_KEYS
    z = {k: torch.zeros((0, 3) if k != "opacity_logits" else (0,), device=rz.device) for k in GRAD_KEYS}
    z["quats"] = torch.zeros((0, 4), device=rz.device)
    z["sh"] = torch.zeros((0, 16, 3), device=rz.device)
    rz.sparse_adam(z, z, z, z, None, LR, 1, sh_degree=3)  # n = 0 enqueues nothing (aliasing is moot)
    torch.cuda.synchronize()


def test_two_steps_in_a_row(rz):
    """Moments carried on the device across two calls (t = 1, then t = 2 with other
    flags and gradients) equal the oracle's chained steps."""
    n, degree = 128 * 12 + 77, 3
    P, G, M, V = scenes.adam_inputs(n, degree, salt=7)
    _, G2, _, _ = scenes.adam_inputs(n, degree, salt=8)
    f1 = scenes.cluster_flags(13, "random", salt=1)
    f2 = scenes.cluster_flags(13, "random", salt=2)
    dP, dM, dV = _dev(P, rz), _dev(M, rz), _dev(V, rz)
    print("two steps n=%d" % n, flush=True)
    rz.sparse_adam(dP, _dev(G, rz), dM, dV, torch.as_tensor(f1.astype(np.int32), device=rz.device), LR, 1)
    rz.sparse_adam(dP, _dev(G2, rz), dM, dV, torch.as_tensor(f2.astype(np.int32), device=rz.device), LR, 2)
    torch.cuda.synchronize()
    p1, m1, v1 = orc.sparse_adam(P, G, M, V, f1, LR, float(np.float32(0.9)), float(np.float32(0.999)),
                                 float(np.float32(1e-15)), 1)
    p2, m2, v2 = orc.sparse_adam(p1, G2, m1, v1, f2, LR, float(np.float32(0.9)), float(np.float32(0.999)),
                                 float(np.float32(1e-15)), 2)
    for k in KEYS:
        # the first step's rounding enters the second as an input error: the
        # second step's bounds carry the first step's
        B1 = _bounds(k, G[k].astype(np.float64), M[k].astype(np.float64), (p1[k], m1[k], v1[k]), 0.9, 0.999, 1e-15,
                     1)
        live1 = np.repeat(f1 != 0, 128)[:n]
        B1 = tuple(np.where(live1.reshape((n,) + (1,) * (b.ndim - 1)), b, 0.0) for b in B1)
        B2 = _bounds(k, G2[k].astype(np.float64), m1[k], (p2[k], m2[k], v2[k]), 0.9, 0.999, 1e-15, 2, B1)
        live2 = np.repeat(f2 != 0, 128)[:n].reshape((n,) + (1,) * (B1[0].ndim - 1))
        B = tuple(np.where(live2, b2, b1) for b1, b2 in zip(B1, B2))
        _assert_within(k, tuple(d[k].cpu().numpy() for d in (dP, dM, dV)), (p2[k], m2[k], v2[k]), B)
        untouched = np.repeat((f1 == 0) & (f2 == 0), 128)[:n]
        assert np.array_equal(dP[k].cpu().numpy()[untouched], P[k][untouched])


def test_bad_arguments_are_rejected(rz):
    from paper_2503_01199_amd import _lib as L
    n = 300
    P, G, M, V = (_dev(d, rz) for d in scenes.adam_inputs(n, 1, salt=1))
    with pytest.raises(L.GsrError):
        rz.sparse_adam(P, G, M, V, None, LR, 0)  # step must be >= 1
    with pytest.raises(L.GsrError):
        rz.sparse_adam(P, G, M, V, None, LR, 1, beta1=1.0)
    with pytest.raises(L.GsrError):
        rz.sparse_adam(P, G, P, V, None, LR, 1)  # moments alias the parameters
    un = dict(P)
    un["means"] = torch.empty(3 * n + 1, device=rz.device)[1:].view(n, 3)  # 4-byte aligned only
    with pytest.raises(L.GsrError):
        rz.sparse_adam(un, G, M, V, None, LR, 1)


def test_training_step_updates_the_clusters_the_frame_kept(rz):
    """forward, backward, then the update over the frame's cluster_visible flags:
    every Gaussian with a non-zero oracle gradient lies in a kept cluster, culled
    clusters keep their parameters, and the kept ones equal a dense update of the
    same rows."""
    from paper_2503_01199_amd.raster import SceneTensors, Workspace
    sc = scenes.spheres_planes_scene(20_000, seed_salt=3)
    _, perm = orc.morton(sc.means)
    sc = sc.permuted(perm)
    cam = scenes.orbit_camera(30.0, 10.0, radius=4.0, width=160, height=120)
    st = SceneTensors.from_scene(sc, rz.device)
    print("training step n=%d" % sc.n, flush=True)
    fr = rz.forward(st, [cam], cluster_cull=True, workspace=Workspace(rz.device))
    w, gt = scenes.l1_weights((3, cam.height, cam.width), config=0, salt=1)
    dl = torch.empty((3, cam.height, cam.width), device=rz.device)
    rz.l1_grad(fr.images[0], torch.as_tensor(w, device=rz.device), torch.as_tensor(gt, device=rz.device), out=dl)
    grads = rz.backward(fr, [dl])
    vis = rz.inspect(fr)["cluster_visible"][: fr.info["clusters"]].clone()
    torch.cuda.synchronize()
    flags = vis.cpu().numpy().astype(np.uint32)
    assert 0 < flags.sum() < flags.size
    ref = orc.backward(sc, cam, orc.l1_grad(orc.render(sc, cam)["image"], w, gt))
    hot = np.zeros(sc.n, bool)
    for k in KEYS:
        hot |= np.abs(ref[k].reshape(sc.n, -1)).max(axis=1) > 0
    assert np.all(np.repeat(flags != 0, 128)[: sc.n][hot])
    params = dict(zip(KEYS, (t.clone() for t in st.tensors())))
    dense = {k: t.clone() for k, t in params.items()}
    m = {k: torch.zeros_like(t) for k, t in params.items()}
    v = {k: torch.zeros_like(t) for k, t in params.items()}
    m2 = {k: torch.zeros_like(t) for k, t in params.items()}
    v2 = {k: torch.zeros_like(t) for k, t in params.items()}
    rz.sparse_adam(params, grads, m, v, vis, LR, 1)
    rz.sparse_adam(dense, grads, m2, v2, None, LR, 1)
    torch.cuda.synchronize()
    rows = np.repeat(flags != 0, 128)[: sc.n]
    for k, t0 in zip(KEYS, st.tensors()):
        a, b, o = params[k].cpu().numpy(), dense[k].cpu().numpy(), t0.cpu().numpy()
        assert np.array_equal(a[rows], b[rows]) and np.array_equal(a[~rows], o[~rows]), k


def test_room_size_sampled_against_oracle(rz):
    """1M Gaussians of SH degree 3 with seeded flags over the 7,813 clusters, in the
    launch the bench times; 4,096 sampled Gaussians compared with the oracle (the
    update is per float, so the oracle runs on the sampled rows alone)."""
    n, degree, t = 1_000_000, 3, 40
    P, G, M, V = scenes.adam_inputs(n, degree, salt=11)
    flags = scenes.cluster_flags((n + 127) // 128, "random", salt=11)
    dP, dG, dM, dV = _dev(P, rz), _dev(G, rz), _dev(M, rz), _dev(V, rz)
    print("room-size sparse adam n=%d" % n, flush=True)
    rz.sparse_adam(dP, dG, dM, dV, torch.as_tensor(flags.astype(np.int32), device=rz.device), LR, t)
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    idx = np.sort(rng.choice(n, 4096, replace=False))
    idx[-1] = n - 1  # the last Gaussian (a partial cluster: 1M = 7812 x 128 + 64)
    sub = lambda d: {k: d[k][idx] for k in KEYS}
    rows = np.repeat(flags != 0, 128)[:n][idx]
    rp, rm, rv = orc.sparse_adam(sub(P), sub(G), sub(M), sub(V), None, LR, float(np.float32(0.9)),
                                 float(np.float32(0.999)), float(np.float32(1e-15)), t)
    ti = torch.as_tensor(idx, device=rz.device)
    for k in KEYS:
        got = tuple(d[k].index_select(0, ti).cpu().numpy() for d in (dP, dM, dV))
        for a, b in zip(got, (P[k][idx], M[k][idx], V[k][idx])):
            assert np.array_equal(a[~rows], b[~rows]), k
        _check(k, got, (rp[k], rm[k], rv[k]), (P[k][idx], G[k][idx], M[k][idx], V[k][idx]), 0.9, 0.999, 1e-15, t,
               rows)


@pytest.mark.parametrize("which", ["spheres-sh3", "tiny-sh0"])
def test_fused_backward_adam_equals_two_calls(rz, which):
    """gsr_backward_adam against gsr_backward followed by gsr_sparse_adam on the
    frame's cluster flags: bit for bit over two steps with carried moments (frames
    in the deterministic mode, so both paths see the same gradient bits), culled
    clusters untouched, and the statistic identical."""
    from paper_2503_01199_amd.raster import SceneTensors, Workspace, new_stats
    if which == "tiny-sh0":
        sc, cam = scenes.tiny_scene(3000, seed_salt=4), scenes.tiny_camera()
    else:
        sc = scenes.spheres_planes_scene(20_000, seed_salt=6)
        _, perm = orc.morton(sc.means)
        sc = sc.permuted(perm)
        cam = scenes.orbit_camera(60.0, 10.0, radius=4.0, width=200, height=150)
    _, _, M, V = scenes.adam_inputs(sc.n, sc.sh_degree, salt=12)
    M["sh"] = M["sh"].reshape(sc.sh.shape)
    V["sh"] = V["sh"].reshape(sc.sh.shape)
    two = SceneTensors.from_scene(sc, rz.device)
    fused = SceneTensors.from_scene(sc, rz.device)
    m2, v2, mf, vf = _dev(M, rz), _dev(V, rz), _dev(M, rz), _dev(V, rz)
    s2, sf = new_stats(sc.n, rz.device), new_stats(sc.n, rz.device)
    print("fused backward + adam %s n=%d" % (which, sc.n), flush=True)
    for t in (1, 2):
        w, gt = scenes.l1_weights((3, cam.height, cam.width), config=0, salt=t)
        w, gt = torch.as_tensor(w, device=rz.device), torch.as_tensor(gt, device=rz.device)
        fa = rz.forward(two, [cam], workspace=Workspace(rz.device), deterministic=True)
        fb = rz.forward(fused, [cam], workspace=Workspace(rz.device), deterministic=True)
        assert torch.equal(fa.images[0], fb.images[0])
        dl = rz.l1_grad(fa.images[0], w, gt)
        grads = rz.backward(fa, [dl], stats=s2)
        vis = rz.inspect(fa)["cluster_visible"][: fa.info["clusters"]].clone()
        rz.sparse_adam(dict(zip(KEYS, two.tensors())), grads, m2, v2, vis, LR, t)
        rz.backward_adam(fb, [dl], mf, vf, LR, t, stats=sf)
        torch.cuda.synchronize()
        flags = vis.cpu().numpy()
        assert 0 < flags.sum() < flags.size or which == "tiny-sh0"
    rows = np.repeat(flags != 0, 128)[: sc.n]
    for k, a, b, p0 in zip(KEYS, two.tensors(), fused.tensors(), sc.arrays()):
        assert torch.equal(a, b), k
        assert torch.equal(m2[k], mf[k]) and torch.equal(v2[k], vf[k]), k
        if (~rows).any():  # culled in both steps here: untouched (the view is the same)
            assert np.array_equal(b.cpu().numpy()[~rows], np.asarray(p0)[~rows]), k
    for k in ("S", "M", "C"):
        assert torch.equal(s2[k], sf[k]), k
