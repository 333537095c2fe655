"""View culling of the cut (v3dg_set_culling) through the C ABI.

Culling must leave the cut (the gid list) and the image unchanged bit for bit,
and may only drop clusters none of whose Gaussians reaches a tile.
"""
import numpy as np
import pytest

import oracle
import paper_2505_06523_amd as v
import scenegen as sg
from tests import helpers as H
from tests.test_gpu_parity import _say, check_image

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a GPU"
    v.lib()
    return _t


def _both(sc, cam, tau, torch):
    """(ids, slots, image) without and with culling."""
    out = []
    for on in (False, True):
        sc.set_culling(on)
        sel = sc.select(cam, tau)
        img = sc.render(cam, sel).clone()
        torch.cuda.synchronize()
        out.append((sel.ids(), sel.slots(), img))
        sel.free()
    sc.set_culling(False)
    return out


def test_culling_keeps_cut_and_image_random_views(torch):
    rng = np.random.default_rng(31)
    a = sg.make_asset(16384, 3, 77)
    T = sg.grid_instances(3, 1.2, 0.2, 4)
    sc = v.Scene(a, T)
    dropped = 0
    for it in range(12):
        cam = H.random_camera_near(rng, int(rng.integers(64, 300)), int(rng.integers(48, 240)), dist=(0.05, 8.0))
        tau = float([0.0, 1.0, 30.0][it % 3])
        (ids0, (r0, i0), img0), (ids1, (r1, i1), img1) = _both(sc, cam, tau, torch)
        assert np.array_equal(ids0, ids1), it
        assert torch.equal(img0, img1), it
        # the kept slots are a subsequence of the full slot stream
        full = r0.astype(np.uint64) | (i0.astype(np.uint64) << np.uint64(32))
        kept = r1.astype(np.uint64) | (i1.astype(np.uint64) << np.uint64(32))
        order = np.argsort(full, kind="stable")
        at = np.searchsorted(full[order], kept)
        assert (at < full.size).all() and np.array_equal(full[order][np.minimum(at, full.size - 1)], kept)
        assert (np.diff(order[at]) > 0).all()
        dropped += r0.size - r1.size
    _say("random views: %d slots culled in total" % dropped)
    assert dropped > 0
    sc.close()


def test_culled_clusters_reach_no_tile(torch):
    """Every Gaussian the cull drops has no tile in the unculled projection."""
    rng = np.random.default_rng(7)
    a = sg.make_asset(16384, 0, 5)
    T = sg.grid_instances(3, 1.3, 0.2, 8)
    sc = v.Scene(a, T)
    checked = 0
    for it in range(8):
        cam = H.random_camera_near(rng, 160, 120, dist=(0.1, 5.0))
        sel = sc.select(cam, 1.0)
        sc.render(cam, sel)
        proj = sc.projection()
        rows, inst = sel.slots()
        sc.set_culling(True)
        sel2 = sc.select(cam, 1.0)
        rows2, inst2 = sel2.slots()
        sc.set_culling(False)
        keep = set(zip(rows2.tolist(), inst2.tolist()))
        culled = np.array([(r, i) not in keep for r, i in zip(rows.tolist(), inst.tolist())])
        assert (proj["tiles"][culled] == 0).all(), it
        checked += int(culled.sum())
        sel.free()
        sel2.free()
    _say("%d culled Gaussians checked for zero tiles" % checked)
    assert checked > 0
    sc.close()


def test_culling_matches_oracle_near_views(torch):
    a = sg.make_asset(16384, 0, 1)
    T = sg.identity_instances(1)
    sc = v.Scene(a, T)
    sc.set_culling(True)
    for eye in [(0.3, 0.1, 0.05), (-0.2, 0.35, 0.1), (0.9, 0.9, 0.2)]:
        cam = sg.look_at(eye, (0.1, 0.0, 0.0), 200, 150, 1.2)
        sel = sc.select(cam, 1.0)
        img = sc.render(cam, sel).cpu().numpy()
        ref, amb, _ = oracle.render(a, T, cam, sel.ids())
        check_image(img, ref, amb, "culled near view %s" % (eye,))
    sc.close()


def test_culling_flythrough_100_instances(torch):
    """100 instances of the 1M-leaf asset; the camera flies inside the grid."""
    a = sg.cached_asset(1 << 20, 3, 2)
    T = sg.grid_instances(10, 1.5, 0.2, 3)
    sc = v.Scene(a, T)
    cams = sg.flythrough_cameras(300, 103)
    for f in [0, 150, 299]:
        (ids0, (r0, _), img0), (ids1, (r1, _), img1) = _both(sc, cams[f], 1.0, torch)
        _say("flythrough frame %d: %d of %d slots kept" % (f, r1.size, r0.size))
        assert np.array_equal(ids0, ids1)
        assert torch.equal(img0, img1)
        assert r1.size < r0.size
    sc.close()
