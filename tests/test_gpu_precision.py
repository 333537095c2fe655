"""The narrow storage tiers (FP16 scale/rotation/opacity, BF16 or FP16 SH;
FP32 positions and FP32 arithmetic) through the C ABI.

Storage: the rows the library keeps equal numpy's round-to-nearest-even of
the FP32 input, bit for bit.  Rendering: parity with the FP64 oracle run on
those same rounded attributes, to the bar of the FP32 tier (max |error|
<= 2e-3 on non-ambiguous pixels, PSNR >= 50 dB).  The cost of the rounding
itself (oracle on rounded vs oracle on FP32 attributes) is reported.
"""
import numpy as np
import pytest

import oracle
import paper_2505_06523_amd as v
import scenegen as sg
from tests import helpers as H
from tests.test_gpu_parity import MAX_ABS, MIN_PSNR, _say, check_image, psnr

pytestmark = pytest.mark.gpu

NARROW = ["fp16_bf16sh", "fp16"]


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a GPU"
    v.lib()
    return _t


def _with_ties(a):
    """Put exact rounding ties and FP16 subnormals into a few rows."""
    a.scale[0] = [1 + 2 ** -11, 1 + 3 * 2 ** -11, 3e-6]       # FP16 ties (to even) and a subnormal
    a.scale[1] = [2 ** -24 * 1.5, 65504.0, 0.1]                # subnormal tie, FP16 maximum
    a.opacity[0] = 0.5 + 2 ** -12                              # tie at 0.5 (ulp 2^-11)
    a.opacity[1] = 0.5 + 3 * 2 ** -12
    a.sh[0, 0] = [1 + 2 ** -8, 1 + 3 * 2 ** -8, -(1 + 2 ** -11)]  # BF16 ties, FP16 tie
    a.sh[1, 0] = [1e-30, -3.0e4, 2 ** -20]                    # FP16 underflow, large, exact
    return a


@pytest.mark.parametrize("precision", ["fp32"] + NARROW)
def test_stored_attributes_round_to_nearest_even(torch, precision):
    a = _with_ties(sg.make_asset(8192, 3, 41))
    sc = v.Scene(a, precision=precision)
    got = sc.attributes()
    want = H.quantized_asset(a, precision)
    for k in ["pos", "scale", "rot", "opacity", "sh"]:
        g = np.ascontiguousarray(got[k], np.float32)
        w = np.ascontiguousarray(getattr(want, k), np.float32).reshape(g.shape)
        bad = np.flatnonzero(g.view(np.uint32) != w.view(np.uint32))
        assert bad.size == 0, (k, bad[:5], g.reshape(-1)[bad[:5]], w.reshape(-1)[bad[:5]])
    part = sc.attributes(100, 7)
    assert np.array_equal(part["sh"], got["sh"][100:107])
    with pytest.raises(v.V3DGError):
        sc.attributes(8000, 10 ** 6)
    sc.close()


@pytest.mark.parametrize("precision", NARROW)
def test_narrow_tier_projection_and_image_parity(torch, precision):
    a = sg.make_asset(16384, 3, 77)
    T = sg.grid_instances(2, 1.1, 0.2, 9)[:3]
    aq = H.quantized_asset(a, precision)
    sc = v.Scene(a, T, precision=precision)
    ref_sc = v.Scene(a, T)
    cam = sg.look_at((2.0, -2.2, 1.6), (0, 0, 0), 333, 250, 1.1)  # ragged tiles on both axes
    cam.bg = (0.2, 0.4, 0.1)
    for tau in [0.0, 200.0]:
        sel = sc.select(cam, tau)
        gids = sel.ids()
        # the cut reads only the sphere table, which every tier keeps in FP32
        assert np.array_equal(gids, oracle.mask_to_gids(oracle.select_walk(a, T, cam, tau)))
        img = sc.render(cam, sel).cpu().numpy()
        g = sc.projection()
        r = oracle.project(aq, T, cam, gids)
        assert np.array_equal(g["depth"].view(np.uint32), r["depth"].view(np.uint32))
        vis = g["tiles"] > 0
        assert (r["valid"][vis] == 1).all()
        assert np.abs(g["rgb"][vis] - r["rgb"][vis]).max() < 1e-5
        assert np.array_equal(g["opacity"][vis], r["opacity"][vis].astype(np.float32))
        ref, amb, _ = oracle.render(aq, T, cam, gids)
        check_image(img, ref, amb, "%s tau=%g" % (precision, tau))
        # what the rounding costs, on both sides
        ref32, _, _ = oracle.render(a, T, cam, gids)
        img32 = ref_sc.render(cam, ref_sc.select(cam, tau)).cpu().numpy()
        q_oracle = psnr(ref, ref32)
        q_gpu = psnr(img.astype(np.float64), img32.astype(np.float64))
        _say("%s tau=%g: rounding cost PSNR oracle %.2f dB, GPU %.2f dB" % (precision, tau, q_oracle, q_gpu))
        assert q_oracle >= 40.0 and q_gpu >= 40.0
    sc.close()
    ref_sc.close()


@pytest.mark.parametrize("precision", NARROW)
def test_narrow_tier_long_lists_and_determinism(torch, precision):
    a = H.stacked_splats(16000, 6, (0.3, 0.95))
    aq = H.quantized_asset(a, precision)
    cam = H.identity_camera(72, 56, 300.0, bg=(0.1, 0.2, 0.3))
    T = sg.identity_instances(1)
    sc = v.Scene(a, T, precision=precision)
    sel = sc.select(cam, 0.0)
    img = sc.render(cam, sel).clone()
    img2 = sc.render_full(cam).clone()
    torch.cuda.synchronize()
    assert torch.equal(img, img2)
    ref, amb, _ = oracle.render(aq, T, cam, sel.ids())
    check_image(img.cpu().numpy(), ref, amb, "stacked %s" % precision)
    sc.close()


def test_c2_narrow_tier_sampled_parity(torch):
    """1M-leaf SH3 asset at 1920x1080 in the FP16 + BF16-SH tier."""
    a = sg.cached_asset(1 << 20, 3, 2)
    aq = H.quantized_asset(a, "fp16_bf16sh")
    sc = v.Scene(a, precision="fp16_bf16sh")
    T = sg.identity_instances(1)
    cams = sg.orbit_cameras(64, 102)
    rng = np.random.default_rng(8)
    for ci, tau in [(3, 1.0), (21, 16.0)]:
        cam = cams[ci]
        sel = sc.select(cam, tau)
        img = sc.render(cam, sel).cpu().numpy()
        pix = np.stack([rng.integers(0, cam.width, 3000), rng.integers(0, cam.height, 3000)], axis=1).astype(np.uint32)
        ref, amb, _ = oracle.render_pixels(aq, T, cam, sel.ids(), pix)
        got = img[pix[:, 1], pix[:, 0]]
        ok = amb == 0
        err = np.abs(got - ref)[ok].max()
        _say("c2 fp16_bf16sh cam %d tau %g: sampled max_abs %.3g amb %d" % (ci, tau, err, int((~ok).sum())))
        assert err <= MAX_ABS
        assert psnr(got[None], ref[None]) >= MIN_PSNR
    sc.close()


@pytest.mark.parametrize("precision", ["fp32", "fp16_bf16sh"])
def test_c2_3840x2160_sampled_parity(torch, precision):
    """The 1M-leaf SH3 asset at 3840x2160 (32,400 tiles), FP32 and FP16 +
    BF16-SH storage, against the oracle on the stored attributes."""
    import dataclasses
    a = sg.cached_asset(1 << 20, 3, 2)
    aq = H.quantized_asset(a, precision)
    sc = v.Scene(a, precision=precision)
    T = sg.identity_instances(1)
    cams = sg.orbit_cameras(64, 102)
    rng = np.random.default_rng(9)
    for ci, tau in [(3, 1.0), (40, 4.0)]:
        c = cams[ci]
        cam = dataclasses.replace(c, width=2 * c.width, height=2 * c.height, fx=2 * c.fx, fy=2 * c.fy,
                                  cx=2 * c.cx, cy=2 * c.cy)
        sel = sc.select(cam, tau)
        assert np.array_equal(sel.ids(), oracle.mask_to_gids(oracle.select_walk(a, T, cam, tau)))
        img = sc.render(cam, sel).cpu().numpy()
        st = sc.frame_stats()
        assert st["n_tiles"] == 240 * 135
        pix = np.stack([rng.integers(0, cam.width, 3000), rng.integers(0, cam.height, 3000)], axis=1).astype(np.uint32)
        ref, amb, _ = oracle.render_pixels(aq, T, cam, sel.ids(), pix)
        got = img[pix[:, 1], pix[:, 0]]
        ok = amb == 0
        err = np.abs(got - ref)[ok].max()
        _say("c2 %s 3840x2160 cam %d tau %g: %d keys, sampled max_abs %.3g amb %d, psnr %.1f"
             % (precision, ci, tau, st["n_keys"], err, int((~ok).sum()), psnr(got[None], ref[None])))
        assert err <= MAX_ABS
        assert psnr(got[None], ref[None]) >= MIN_PSNR
    sc.close()
