"""Raster schedules (the forward's and the backward's work-item lists) against the
rule they implement, on a frame of a few thousand tiles (built by one block) and
on one of more than 8,192 tiles (built by several blocks): tiles ordered by list
length clamped at 4,095, longest first; the first ns = min(#lists longer than the
split length, ceil(tiles / 4)) are split (four 16x4 bands forward, two halves
backward), and where the cap cuts through tiles of equal clamped length the ones of
lower index are split. Within a length, other tiles may come in any order, so the
check takes the split set and the length order, which the rule fixes, and that
every tile appears exactly once."""
import numpy as np
import pytest

from helpers import ensure_built
from paper_2503_01199_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rz():
    ensure_built()
    from paper_2503_01199_amd.raster import Rasterizer
    r = Rasterizer(0)
    yield r
    r.set_raster_split(0, 0)


def _check_list(items, lens, split_len, ways):
    T = len(lens)
    clamped = np.minimum(lens, 4095)
    order = np.lexsort((np.arange(T), -clamped))  # longest first, lower index first
    ns = min(int((lens > split_len).sum()), (T + 3) // 4)
    codes = items & 7
    tiles = (items >> 3).astype(np.int64)
    assert len(items) == T + (ways - 1) * ns
    head, tail = items[:ways * ns], items[ways * ns:]
    want = np.arange(ways) if ways == 4 else np.array([5, 6])
    hs = (head >> 3).reshape(-1, ways) if ns else np.zeros((0, ways), np.int64)
    if ns:
        assert (hs == hs[:, :1]).all(), "a split tile's items are consecutive"
        assert ((head & 7).reshape(-1, ways) == want).all()
    split = np.sort(hs[:, 0]) if ns else np.zeros(0, np.int64)
    assert np.array_equal(split, np.sort(order[:ns])), "split set"
    assert ((tail & 7) == 4).all()
    seq = np.concatenate([hs[:, 0], tail >> 3]).astype(np.int64)
    assert np.array_equal(np.sort(seq), np.arange(T)), "every tile exactly once"
    c = clamped[seq]
    assert (np.diff(c[:ns]) <= 0).all() and (np.diff(c[ns:]) <= 0).all(), "length order"
    return ns, tiles, codes


@pytest.mark.parametrize("views,split", [(1, (0, 0)), (1, (2, 3)), (3, (0, 0)), (3, (2, 3))])
def test_schedule_follows_the_rule(rz, views, split):
    from paper_2503_01199_amd.raster import SceneTensors, Workspace
    sc = scenes.spheres_planes_scene(60_000, seed_salt=8)
    cams = [scenes.orbit_camera(20.0 * v, radius=7.0, width=1920, height=1080) for v in range(views)]
    rz.set_raster_split(*split)
    print("schedule views=%d split=%s" % (views, split), flush=True)
    fr = rz.forward(SceneTensors.from_scene(sc, rz.device), cams, workspace=Workspace(rz.device))
    ins = rz.inspect(fr)
    rz.set_raster_split(0, 0)
    rg = ins["ranges"].cpu().numpy().view(np.uint32).astype(np.int64)
    lens = rg[:, 1] - rg[:, 0]
    T = len(lens)
    sl = split[0] or 256
    sb = split[1] or 512
    ns, _, _ = _check_list(ins["fwd_items"].cpu().numpy().view(np.uint32).astype(np.int64), lens, sl, 4)
    nb, _, _ = _check_list(ins["bwd_items"].cpu().numpy().view(np.uint32).astype(np.int64), lens, sb, 2)
    print("tiles %d (%s), split forward %d backward %d, longest list %d"
          % (T, "one block" if T <= 8192 else "several blocks", ns, nb, lens.max()))
    assert (T > 8192) == (views > 1)
    assert ns == fr.info["split_tiles"] and nb == fr.info["split_tiles_bwd"]
    if split != (0, 0):
        assert ns == (T + 3) // 4 and nb > 0, "the cap binds: the rule's edge case is exercised"
