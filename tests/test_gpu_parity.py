"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Selection: bit-exact gid lists.  Slot stream: equal to the serial expansion.
Projection: FP32 depth bit-equal, splat values within 1e-4 relative.  Sort:
equal to numpy's stable sort.  Images: max |error| <= 2e-3 per channel over
pixels with no threshold decision within 2^-14 of its threshold, and
PSNR >= 50 dB over all pixels, against the FP64 oracle.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import paper_2505_06523_amd as v
import scenegen as sg
from tests import helpers as H

pytestmark = pytest.mark.gpu

MAX_ABS = 2e-3
MIN_PSNR = 50.0


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a GPU"
    v.lib()
    return _t


def psnr(a, b):
    a = np.clip(a[..., :3], 0, 1)
    b = np.clip(b[..., :3], 0, 1)
    mse = float(np.mean((a - b) ** 2))
    return float("inf") if mse == 0 else 10 * math.log10(1.0 / mse)


def check_image(gpu, ref, amb, tag=""):
    ok = amb == 0
    err = np.abs(gpu.astype(np.float64) - ref)
    max_ok = float(err[ok].max()) if ok.any() else 0.0
    p = psnr(gpu.astype(np.float64), ref)
    _say("%s max_abs(non-ambiguous)=%.3g psnr=%.2f ambiguous=%d/%d" % (tag, max_ok, p, int((~ok).sum()), ok.size))
    assert max_ok <= MAX_ABS, tag
    assert p >= MIN_PSNR, tag
    assert (~ok).mean() < 0.05, tag  # sanity: a window of 2^-14 flags ~1% of busy pixels


# ------------------------------------------------------------------------------
# small plain case: 16,384 leaves, SH0, 256x256, fov 60 deg
# ------------------------------------------------------------------------------
@pytest.fixture(scope="module")
def c1(torch):
    a = sg.make_asset(16384, 0, 1)
    sc = v.Scene(a)
    yield a, sc
    sc.close()


def test_select_c1_tau_sweep(c1):
    a, sc = c1
    cam = sg.single_camera_c1()
    T = sg.identity_instances(1)
    sel = None
    for tau in [0.0, 1.0, 10.0, 100.0, 1e3, 3e3, 1e4, 1e5, 1e6, 3e38]:
        sel = sc.select(cam, tau, sel)
        ref = oracle.mask_to_gids(oracle.select_walk(a, T, cam, tau))
        got = sel.ids()
        assert np.array_equal(got, ref), tau
        nc, ng = sel.info()
        assert nc == ref.size and ng == int(a.count[ref % a.n_clusters].sum())


def test_select_random_assets_instances_cameras(torch):
    rng = np.random.default_rng(2024)
    for it in range(4):
        n = int(rng.integers(100, 20000))
        a = sg.make_asset(n, int(rng.integers(0, 4)), int(rng.integers(1 << 30)), n_ellipsoids=int(rng.integers(1, 6)))
        T = np.concatenate([sg.identity_instances(1), sg.grid_instances(3, 1.2, 0.3, it)[: int(rng.integers(1, 9))]])
        T[-1, :, :3] *= 1.7  # a uniformly scaled instance
        sc = v.Scene(a, T)
        sel = None
        for c in range(6):
            cam = H.random_camera_near(rng, int(rng.integers(16, 200)), int(rng.integers(16, 200)), dist=(0.05, 40))
            for tau in [0.0, float(rng.uniform(0, 5)), float(10 ** rng.uniform(1, 6)), 3e38]:
                sel = sc.select(cam, tau, sel)
                ref = oracle.mask_to_gids(oracle.select_walk(a, T, cam, tau))
                assert np.array_equal(sel.ids(), ref), (it, c, tau)
        sc.close()


def test_slot_stream_is_serial_expansion(c1):
    a, sc = c1
    cam = sg.single_camera_c1()
    for tau in [0.0, 2000.0, 5e4]:
        sel = sc.select(cam, tau)
        gids = sel.ids()
        rows, inst = sel.slots()
        er, ei = [], []
        for g in gids:
            k = g % a.n_clusters
            er.extend(range(a.first_row[k], a.first_row[k] + a.count[k]))
            ei.extend([g // a.n_clusters] * a.count[k])
        assert np.array_equal(rows, np.asarray(er, np.uint32))
        assert np.array_equal(inst, np.asarray(ei, np.uint32))
        sel.free()


def _projection_parity(a, T, cam, sc, sel, torch):
    img = sc.render(cam, sel)
    torch.cuda.synchronize()
    gids = sel.ids()
    g = sc.projection()
    r = oracle.project(a, T, cam, gids)
    assert g["depth"].shape[0] == r["depth"].shape[0]
    assert np.array_equal(g["depth"].view(np.uint32), r["depth"].view(np.uint32)), "FP32 depth must be bit-equal"
    vis = g["tiles"] > 0
    # every splat the GPU keeps is valid for the oracle
    assert (r["valid"][vis] == 1).all()
    rel = lambda x, y: np.abs(x - y) / np.maximum(np.abs(y), 1.0)
    assert rel(g["mean2"][vis], r["mean2"][vis]).max() < 1e-4
    ca = np.abs(r["conic"][vis]).max(axis=1, keepdims=True)
    assert (np.abs(g["conic"][vis] - r["conic"][vis]) / ca).max() < 1e-3
    assert np.abs(g["rgb"][vis] - r["rgb"][vis]).max() < 1e-5
    assert np.array_equal(g["opacity"][vis], r["opacity"][vis].astype(np.float32))
    return img


def test_projection_parity_sh0_and_sh3(torch):
    for deg, n in [(0, 16384), (3, 8192)]:
        a = sg.make_asset(n, deg, 31 + deg)
        T = sg.grid_instances(2, 1.0, 0.2, 5)
        sc = v.Scene(a, T)
        cam = sg.look_at((1.5, -2.5, 1.2), (0, 0, 0), 320, 240, 1.0)
        sel = sc.select(cam, 50.0)
        _projection_parity(a, T, cam, sc, sel, torch)
        sc.close()


# ------------------------------------------------------------------------------
# sort primitive
# ------------------------------------------------------------------------------
@pytest.mark.parametrize("n,bits", [(1, 8), (100, 13), (4095, 40), (4096, 45), (4097, 64), (100003, 45),
                                    (2_000_000, 47), (33, 1)])
def test_sort_pairs_matches_numpy_stable(torch, n, bits):
    rng = np.random.default_rng(n + bits)
    hi = np.uint64((1 << bits) - 1) if bits < 64 else np.uint64(0xFFFFFFFFFFFFFFFF)
    keys = rng.integers(0, 1 << 62, n, dtype=np.uint64) * np.uint64(4) + rng.integers(0, 4, n, dtype=np.uint64)
    keys &= hi
    if n > 10:
        keys[: n // 3] = keys[n // 3]  # many duplicates
    vals = np.arange(n, dtype=np.uint32)
    kt = torch.from_numpy(keys.view(np.int64).copy()).cuda()
    vt = torch.from_numpy(vals.view(np.int32).copy()).cuda()
    v.sort_pairs(kt, vt, bits)
    torch.cuda.synchronize()
    order = np.argsort(keys, kind="stable")
    assert np.array_equal(kt.cpu().numpy().view(np.uint64), keys[order])
    assert np.array_equal(vt.cpu().numpy().view(np.uint32), vals[order])


def _check_frame_keys(sc):
    st = sc.frame_stats()
    keys, vals = sc.sorted_keys()
    proj = sc.projection()
    assert keys.size == st["n_keys"] == int(proj["tiles"].sum())
    # ascending keys; equal keys keep ascending slots (stable)
    assert (np.diff(keys.astype(np.float64)) >= 0).all() or np.all(keys[1:] >= keys[:-1])
    same = keys[1:] == keys[:-1]
    assert (vals[1:][same] > vals[:-1][same]).all()
    # each slot appears tiles[t] times with distinct tiles and its own depth bits
    cnt = np.bincount(vals, minlength=proj["tiles"].size)
    assert np.array_equal(cnt, proj["tiles"])
    assert np.array_equal((keys & np.uint64(0xFFFFFFFF)).astype(np.uint32), proj["depth"].view(np.uint32)[vals])
    tk = (keys >> np.uint64(32)) * np.uint64(1 << 32) + vals.astype(np.uint64)
    assert np.unique(tk).size == tk.size
    return st


def test_frame_keys_sorted_stable_and_complete(c1, torch):
    a, sc = c1
    cam = sg.single_camera_c1()
    sel = sc.select(cam, 1.0)
    sc.render(cam, sel)
    _check_frame_keys(sc)


def test_sort_modes_identical(c1, torch):
    """Depth-first binning and 64-bit keys give the same order and image."""
    a, sc = c1
    for cam, tau in [(sg.single_camera_c1(), 1.0), (sg.look_at((0.6, 0.5, 0.4), (0, 0, 0), 333, 250, 1.2), 30.0)]:
        sel = sc.select(cam, tau)
        sc.set_sort_mode(v.V3DG_SORT_KEYS64)
        i64 = sc.render(cam, sel).clone()
        k64, v64 = sc.sorted_keys()
        st64 = sc.frame_stats()
        sc.set_sort_mode(v.V3DG_SORT_DEPTH_FIRST)
        idf = sc.render(cam, sel).clone()
        kdf, vdf = sc.sorted_keys()
        stdf = sc.frame_stats()
        torch.cuda.synchronize()
        assert st64["sort_mode"] == 1 and stdf["sort_mode"] == 0
        assert np.array_equal(k64, kdf) and np.array_equal(v64, vdf)
        assert torch.equal(i64, idf)


def test_tile_coverage_is_conservative(c1, torch):
    """Every pixel where a kept splat reaches alpha >= 1/255 lies in a 32x32
    bin it was binned to."""
    a, sc = c1
    cam = sg.look_at((0.9, -0.7, 0.6), (0, 0, 0), 320, 200, 1.1)
    sel = sc.select(cam, 1.0)
    sc.render(cam, sel)
    keys, vals = sc.sorted_keys()
    pr = sc.projection()
    bins_x = (cam.width + 31) // 32
    binned = {}
    for k, t in zip((keys >> np.uint64(32)).astype(np.int64), vals.astype(np.int64)):
        binned.setdefault(t, set()).add(int(k))
    vis = np.flatnonzero(pr["tiles"] > 0)
    rng = np.random.default_rng(1)
    ys, xs = np.mgrid[0:cam.height, 0:cam.width]
    for t in rng.choice(vis, size=min(1500, vis.size), replace=False):
        mx, my = pr["mean2"][t]
        A, B, Cc = pr["conic"][t].astype(np.float64)
        o = float(pr["opacity"][t])
        dx = mx - (xs + 0.5)
        dy = my - (ys + 0.5)
        power = np.minimum(0.0, -0.5 * (A * dx * dx + Cc * dy * dy) - B * dx * dy)
        alpha = np.minimum(0.99, o * np.exp(power))
        hit = alpha >= (1.0 / 255.0) * (1 - 1e-4)
        need = set(((ys[hit] // 32) * bins_x + xs[hit] // 32).tolist())
        assert need <= binned.get(int(t), set()), int(t)
        assert len(binned[int(t)]) == int(pr["tiles"][t])


# ------------------------------------------------------------------------------
# images
# ------------------------------------------------------------------------------
def test_image_parity_c1(c1, torch):
    a, sc = c1
    cam = sg.single_camera_c1()
    T = sg.identity_instances(1)
    for tau in [1.0, 3000.0]:
        sel = sc.select(cam, tau)
        img = sc.render(cam, sel).cpu().numpy()
        ref, amb, _ = oracle.render(a, T, cam, sel.ids())
        check_image(img, ref, amb, "c1 tau=%g" % tau)


def test_image_parity_sh3_instances_background(torch):
    a = sg.make_asset(16384, 3, 77)
    T = sg.grid_instances(2, 1.1, 0.2, 9)[:3]
    sc = v.Scene(a, T)
    cam = sg.look_at((2.0, -2.2, 1.6), (0, 0, 0), 333, 250, 1.1)  # ragged tiles on both axes
    cam.bg = (0.2, 0.4, 0.1)
    for tau in [0.0, 200.0]:
        sel = sc.select(cam, tau)
        img = sc.render(cam, sel).cpu().numpy()
        ref, amb, _ = oracle.render(a, T, cam, sel.ids())
        check_image(img, ref, amb, "sh3 tau=%g" % tau)
    sc.close()


@pytest.mark.parametrize("opacity,seed", [((0.02, 0.12), 5), ((0.3, 0.95), 6), ((0.05, 0.5), 7)])
def test_long_tile_lists_chunked_blending(torch, opacity, seed):
    """Thousands of splats over a few tiles: lists far longer than one chunk,
    pixels that never saturate, and pixels that stop inside later chunks."""
    a = H.stacked_splats(16000, seed, opacity)
    cam = H.identity_camera(72, 56, 300.0, bg=(0.1, 0.2, 0.3))
    T = sg.identity_instances(1)
    sc = v.Scene(a, T)
    sel = sc.select(cam, 0.0)
    img = sc.render(cam, sel).cpu().numpy()
    st = sc.frame_stats()
    keys, _ = sc.sorted_keys()
    per_tile = np.bincount((keys >> np.uint64(32)).astype(np.int64))
    _say("long lists: keys %d, longest tile list %d" % (st["n_keys"], per_tile.max()))
    first, later = H.blend_chunk_sizes()
    assert per_tile.max() > first + 4 * later  # a first chunk and at least five more
    ref, amb, _ = oracle.render(a, T, cam, sel.ids())
    check_image(img, ref, amb, "stacked o=%s" % (opacity,))
    sc.set_sort_mode(v.V3DG_SORT_KEYS64)
    img2 = sc.render(cam, sel).cpu().numpy()
    assert np.array_equal(img, img2)
    sc.set_sort_mode(v.V3DG_SORT_DEPTH_FIRST)
    # the larger chunks of the serving loop, and the largest allowed
    for ck in (2048, 4096):
        sc.set_chunk_keys(ck)
        assert per_tile.max() > 3 * ck  # a first chunk of 3 ck keys and at least one more
        img3 = sc.render(cam, sel).cpu().numpy()
        check_image(img3, ref, amb, "stacked o=%s, chunks of %d keys" % (opacity, ck))
    sc.close()


def test_tau0_equals_full_detail_bitwise_and_deterministic(c1, torch):
    a, sc = c1
    cam = sg.single_camera_c1()
    sel = sc.select(cam, 0.0)
    i1 = sc.render(cam, sel).clone()
    i2 = sc.render_full(cam).clone()
    i3 = sc.render(cam, sel).clone()
    torch.cuda.synchronize()
    assert torch.equal(i1, i2)
    assert torch.equal(i1, i3)
    for _ in range(5):
        assert torch.equal(sc.render(cam, sel), i1)


def test_empty_and_degenerate_frames(c1, torch):
    a, sc = c1
    # looking away from the asset: nothing visible, image is the background
    cam = sg.look_at((0, 0, 3.0), (0, 0, 6.0), 37, 19, 1.0)
    cam.bg = (0.25, 0.5, 0.75)
    sel = sc.select(cam, 1.0)
    img = sc.render(cam, sel).cpu().numpy()
    assert np.array_equal(img[..., :3], np.broadcast_to(np.float32([0.25, 0.5, 0.75]), img[..., :3].shape))
    assert (img[..., 3] == 0).all()
    assert sc.frame_stats()["n_keys"] == 0
    # a 1x1 image
    cam1 = sg.look_at((1.0, 1.0, 1.0), (0, 0, 0), 1, 1, 0.5)
    sel = sc.select(cam1, 0.0)
    img = sc.render(cam1, sel).cpu().numpy()
    ref, amb, _ = oracle.render(a, sg.identity_instances(1), cam1, sel.ids())
    if amb[0, 0] == 0:
        assert np.abs(img - ref).max() <= MAX_ABS
    # camera inside the asset
    cam2 = sg.look_at((0.05, 0.02, 0.01), (1, 0.3, 0.2), 64, 48, 1.4)
    sel = sc.select(cam2, 10.0)
    img = sc.render(cam2, sel).cpu().numpy()
    ref, amb, _ = oracle.render(a, sg.identity_instances(1), cam2, sel.ids())
    check_image(img, ref, amb, "inside")


def test_invalid_arguments_raise(c1, torch):
    a, sc = c1
    cam = sg.single_camera_c1()
    for bad in [-1.0, float("nan"), float("inf")]:
        with pytest.raises(v.V3DGError) as ei:
            sc.select(cam, bad)
        assert ei.value.code == v.V3DG_ERR_INVALID_ARG
    c2 = sg.single_camera_c1()
    c2.fx = 0.0
    with pytest.raises(v.V3DGError):
        sc.select(c2, 1.0)
    c3 = sg.single_camera_c1()
    c3.world_to_cam = c3.world_to_cam.copy()
    c3.world_to_cam[0, 0] = np.nan
    with pytest.raises(v.V3DGError):
        sc.select(c3, 1.0)


# ------------------------------------------------------------------------------
# full-size workloads: 1M-leaf SH3 asset at 1080p, and 100 instances of it
# ------------------------------------------------------------------------------
@pytest.fixture(scope="module")
def c2(torch):
    _say("generating 1,048,576-leaf SH3 asset")
    a = sg.cached_asset(1 << 20, 3, 2)
    sc = v.Scene(a)
    yield a, sc
    sc.close()


def test_c2_selection_bitexact_all_cameras(c2):
    a, sc = c2
    T = sg.identity_instances(1)
    cams = sg.orbit_cameras(64, 102)
    sel = None
    n = 0
    for ci, cam in enumerate(cams):
        for tau in [0.0, 1.0, 4.0, 16.0, 64.0, 256.0, 1024.0, 4096.0, 3e38]:
            sel = sc.select(cam, tau, sel)
            ref = oracle.mask_to_gids(oracle.select_walk(a, T, cam, tau))
            assert np.array_equal(sel.ids(), ref), (ci, tau)
            n += 1
    _say("c2 selection: %d (camera, tau) cases bit-exact" % n)


def test_c2_frame_keys_wide_partitions(c2, torch):
    """A frame with more than 4M keys: the tile sort then uses its wide (6144-key) partitions."""
    a, sc = c2
    for cam in sg.orbit_cameras(64, 102):
        sel = sc.select(cam, 1.0)
        sc.render(cam, sel)
        k = sc.frame_stats()["n_keys"]
        if (1 << 22) <= k <= 24_000_000:
            break
    st = _check_frame_keys(sc)
    _say("c2 wide-partition frame: %d keys checked" % st["n_keys"])
    assert st["n_keys"] >= 1 << 22


def test_c2_image_full_frame_parity(c2, torch):
    a, sc = c2
    T = sg.identity_instances(1)
    cam = sg.orbit_cameras(64, 102)[3]
    sel = sc.select(cam, 1.0)
    img = sc.render(cam, sel).cpu().numpy()
    ref, amb, _ = oracle.render(a, T, cam, sel.ids())
    check_image(img, ref, amb, "c2 cam 3 tau 1 (1080p)")


def test_c2_image_sampled_parity(c2, torch):
    a, sc = c2
    T = sg.identity_instances(1)
    cams = sg.orbit_cameras(64, 102)
    rng = np.random.default_rng(7)
    for ci, tau in [(0, 0.0), (10, 1024.0), (21, 16.0)]:
        cam = cams[ci]
        sel = sc.select(cam, tau)
        img = sc.render(cam, sel).cpu().numpy()
        pix = np.stack([rng.integers(0, cam.width, 3000), rng.integers(0, cam.height, 3000)], axis=1).astype(np.uint32)
        ref, amb, st = oracle.render_pixels(a, T, cam, sel.ids(), pix)
        got = img[pix[:, 1], pix[:, 0]]
        ok = amb == 0
        err = np.abs(got - ref)[ok].max()
        _say("c2 cam %d tau %g: slots %d keys %d sampled max_abs %.3g amb %d" %
             (ci, tau, sc.frame_stats()["n_slots"], sc.frame_stats()["n_keys"], err, int((~ok).sum())))
        assert err <= MAX_ABS
        assert psnr(got[None], ref[None]) >= MIN_PSNR


@pytest.fixture(scope="module")
def c3(c2):
    """100 instances of the 1M-leaf asset on a 10 x 10 grid (about 105M virtual leaves)."""
    a, _ = c2
    T = sg.grid_instances(10, 1.5, 0.2, 3)
    sc = v.Scene(a, T)
    yield a, T, sc
    sc.close()


def test_c3_selection_bitexact_flythrough(c3, torch):
    a, T, sc = c3
    cams = sg.flythrough_cameras(300, 103)
    sel = None
    for f in [0, 37, 150, 299]:
        sel = sc.select(cams[f], 1.0, sel)
        ref = oracle.mask_to_gids(oracle.select_walk(a, T, cams[f], 1.0))
        assert np.array_equal(sel.ids(), ref), f
        nc, ng = sel.info()
        _say("c3 frame %d: %d clusters, %d Gaussians selected" % (f, nc, ng))


@pytest.mark.parametrize("frame,cull", [(37, False), (150, True)])
def test_c3_image_sampled_parity(c3, torch, frame, cull):
    """Fly-through frames of the composed scene at 1920x1080, tolerance 1:
    sampled pixels against the oracle (which projects all ~105M slots)."""
    a, T, sc = c3
    cam = sg.flythrough_cameras(300, 103)[frame]
    sc.set_culling(cull)
    try:
        sel = sc.select(cam, 1.0)
        img = sc.render(cam, sel).cpu().numpy()
        st = sc.frame_stats()
    finally:
        sc.set_culling(False)
    rng = np.random.default_rng(frame)
    pix = np.stack([rng.integers(0, cam.width, 3000), rng.integers(0, cam.height, 3000)], axis=1).astype(np.uint32)
    ref, amb, ost = oracle.render_pixels(a, T, cam, sel.ids(), pix)
    got = img[pix[:, 1], pix[:, 0]]
    ok = amb == 0
    err = np.abs(got - ref)[ok].max()
    lit = int((ref[:, 3] > 0.01).sum())
    _say("c3 frame %d (culling %s): %d slots projected (oracle %d), %d keys, sampled max_abs %.3g amb %d, "
         "%d sampled pixels covered" % (frame, cull, st["n_slots"], ost["n_slots"], st["n_keys"], err,
                                        int((~ok).sum()), lit))
    assert lit > 300  # the frame shows the scene
    assert err <= MAX_ABS
    assert psnr(got[None], ref[None]) >= MIN_PSNR


def test_large_splats_and_32bit_tile_ids(torch):
    """An 8224 x 8224 image (66,049 bins of 32 x 32 pixels: 32-bit bin ids) of
    the c1-sized asset seen from close by, so that near splats cover thousands
    of bins and go through the large-splat emission: the image and the sorted
    keys equal the 64-bit-key mode (whose emission has no large-splat path) bit
    for bit, and sampled pixels match the oracle."""
    a = sg.make_asset(16384, 3, 41)
    T = sg.identity_instances(1)
    sc = v.Scene(a, T)
    cam = sg.look_at((0.35, -0.3, 0.25), (0, 0, 0), 8224, 8224, 1.4)
    sel = sc.select(cam, 1.0)
    sc.set_sort_mode(v.V3DG_SORT_KEYS64)
    i64 = sc.render(cam, sel).clone()
    k64, v64 = sc.sorted_keys()
    sc.set_sort_mode(v.V3DG_SORT_DEPTH_FIRST)
    idf = sc.render(cam, sel).clone()
    kdf, vdf = sc.sorted_keys()
    st = sc.frame_stats()
    torch.cuda.synchronize()
    assert st["n_bins"] == 257 * 257 and st["n_tiles"] == 514 * 514 and st["key_bits"] > 16
    # splats with more than 2048 bins exist in this frame
    proj = sc.projection()
    tiles = np.asarray(proj["tiles"])
    n_big = int((tiles > 2048).sum())
    assert n_big > 0
    assert np.array_equal(k64, kdf) and np.array_equal(v64, vdf)
    assert torch.equal(i64, idf)
    img = idf.cpu().numpy()
    rng = np.random.default_rng(5)
    pix = np.stack([rng.integers(0, cam.width, 2000), rng.integers(0, cam.height, 2000)], axis=1).astype(np.uint32)
    ref, amb, _ = oracle.render_pixels(a, T, cam, sel.ids(), pix)
    got = img[pix[:, 1], pix[:, 0]]
    ok = amb == 0
    err = np.abs(got - ref)[ok].max()
    _say("8224x8224 close view: %d splats over 2048 bins, %d keys, sampled max_abs %.3g"
         % (n_big, st["n_keys"], err))
    assert err <= MAX_ABS and psnr(got[None], ref[None]) >= MIN_PSNR
    sc.close()


def test_blend_pair_counts_against_the_oracle(c1, torch):
    """The blend kernels' own pair counts on a frame without long tile lists
    (no later chunk is walked speculatively): the pairs they find contributing
    (alpha >= 1/255 while the pixel still composites, the one that ends it
    included) equal the oracle's contributing pairs up to near-threshold
    decisions, and the pairs they evaluate (the unit of the blend roofline)
    are at least those."""
    a, sc = c1
    cam = sg.single_camera_c1()
    T = sg.identity_instances(1)
    first, _ = H.blend_chunk_sizes()
    for tau in (1.0, 16.0, 64.0, 256.0, 3000.0):  # the finest cut whose bin lists fit one chunk
        sel = sc.select(cam, tau)
        sc.render(cam, sel)
        keys, _ = sc.sorted_keys()
        longest = int(np.bincount((keys >> np.uint64(32)).astype(np.int64)).max())
        if longest <= first:
            break
    sc.collect_profile()
    sc.render(cam, sel)
    assert sc.collect_profile()["pairs_taken"] == 0  # counted only when asked for
    sc.set_profiling(False, audit_pairs=True)
    sc.render(cam, sel)
    P = sc.collect_profile()
    sc.set_profiling(False)
    _, amb, st = oracle.render(a, T, cam, sel.ids())
    _say("pairs at tolerance %g: evaluated %d, contributing %d; oracle contributing %d (bucket walk %d); ambiguous "
         "pixels %d; longest bin list %d" % (tau, P["pairs"], P["pairs_taken"], st["n_hits"], st["n_pairs"],
                                            int(amb.sum()), longest))
    assert longest <= first
    assert P["pairs"] >= P["pairs_taken"] > 0
    assert abs(P["pairs_taken"] - st["n_hits"]) <= 1e-4 * st["n_hits"] + 20 * int(amb.sum())


def test_render_capacity_overflow_is_still_exact(torch):
    """v3dg_render sizes the first frame of an image size exactly (one host
    wait); later frames run on a key capacity (at least 2^20 keys, 48 keys per
    pixel and twice the most keys seen) without host waits.  A later frame
    that needs more keys than that is blended from all visible splats in depth
    order: its image still matches the oracle, its sorted keys are
    unavailable, and the next frame runs on a grown capacity with its keys
    sorted."""
    a = H.stacked_splats(16000, 5, (0.05, 0.5), log_scale=-1.0)
    T = np.tile(sg.identity_instances(1), (4, 1, 1))  # 64,000 splats: up to 62 keys per pixel
    sc = v.Scene(a, T)
    far = H.identity_camera(160, 120, 4.0, bg=(0.1, 0.2, 0.3))    # the stack covers a few pixels
    near = H.identity_camera(160, 120, 600.0, bg=(0.1, 0.2, 0.3))  # every splat covers every bin
    s_far = sc.select(far, 0.0)
    sc.render(far, s_far)
    k_far = sc.frame_stats()["n_keys"]
    cap = max(2 * k_far, 48 * 160 * 120, 1 << 20)
    s_near = sc.select(near, 0.0)
    img = sc.render(near, s_near).clone()
    st = sc.frame_stats()
    _say("capacity after a %d-key frame: %d; the next frame needs %d keys" % (k_far, cap, st["n_keys"]))
    assert st["n_keys"] > cap  # this frame overflowed the capacity
    with pytest.raises(v.V3DGError) as ei:
        sc.sorted_keys()
    assert ei.value.code == v.V3DG_ERR_CAPACITY
    ref, amb, _ = oracle.render(a, T, near, s_near.ids())
    check_image(img.cpu().numpy(), ref, amb, "over capacity (all-splat walk)")
    img2 = sc.render(near, s_near).clone()  # capacity grown: sorted and chunked as usual
    keys, _ = sc.sorted_keys()
    assert keys.size == sc.frame_stats()["n_keys"] == st["n_keys"]
    check_image(img2.cpu().numpy(), ref, amb, "after growth")
    # many frames in flight without host waits, then read back in order
    outs = [sc.render(cam, sel) for cam, sel in [(far, s_far), (near, s_near)] * 12]
    torch.cuda.synchronize()
    assert torch.equal(outs[-1], img2) and torch.equal(outs[1], img2)
    sc.close()
