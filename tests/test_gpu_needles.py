"""Near-degenerate splats: the FP64 redo of the 2D covariance.

With no 2D dilation (paper Sec. 5.1) nothing keeps a thin Gaussian away
from a singular 2D covariance.  A splat whose FP32 determinant falls below
1e-6 px^4 has its covariance and conic redone in FP64 on the GPU; these tests
plant such needles, count the redo on the device and check projection and
image against the FP64 oracle.

Needles lying along a pixel row (or column) through pixel centres draw a
visible line (dy = 0 there, so only the long axis of the conic matters);
rotated needles are checked through their conics.  A needle thinner than
~1e-19 px has a conic entry beyond FP32 range; the library stores it clamped
to +-1e38, which keeps the axis-aligned line and overflows elsewhere.
"""
import numpy as np
import pytest

import oracle
import paper_2505_06523_amd as v
import scenegen as sg
from tests import helpers as H
from tests.test_gpu_parity import _say, check_image

pytestmark = pytest.mark.gpu

W, HH, F = 96, 64, 100.0
CX, CY = 48.5, 32.5  # pixel centres of column 48 and row 32


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a GPU"
    v.lib()
    return _t


def _needle_scene(seed):
    """Normal splats, row and column needles through pixel centres, rotated
    needles, and clamped (extreme) row and column needles.  Returns the asset
    rows and the kinds: 0 normal, 1 needle, 2 extreme needle."""
    rng = np.random.default_rng(seed)
    pos, scale, rot, kind = [], [], [], []
    for _ in range(120):  # normal splats, at least 0.6 px across on every axis
        z = rng.uniform(1.5, 3.0)
        pos.append([rng.uniform(-0.6, 0.6) * z, rng.uniform(-0.4, 0.4) * z, z])
        scale.append(np.exp(rng.uniform(np.log(0.02), np.log(0.06), 3)))
        q = rng.standard_normal(4)
        rot.append(q / np.linalg.norm(q) * np.sign(q[0]))
        kind.append(0)
    for i in range(6):  # along row 32: y = 0 maps to my = CY exactly
        z = 1.5 + 0.25 * i
        pos.append([(-0.3 + 0.12 * i) * z, 0.0, z])
        scale.append([0.08, 1e-7, 1e-7])
        rot.append([1, 0, 0, 0])
        kind.append(1)
    for i in range(4):  # along column 48
        z = 1.6 + 0.3 * i
        pos.append([0.0, (-0.2 + 0.13 * i) * z, z])
        scale.append([1e-7, 0.07, 1e-7])
        rot.append([1, 0, 0, 0])
        kind.append(1)
    for _ in range(10):  # rotated needles: thin enough for the FP64 redo, thick enough for FP64 sums
        z = rng.uniform(1.5, 3.0)
        pos.append([rng.uniform(-0.5, 0.5) * z, rng.uniform(-0.3, 0.3) * z, z])
        scale.append([0.08, 2e-7, 2e-7])
        q = rng.standard_normal(4)
        rot.append(q / np.linalg.norm(q) * np.sign(q[0]))
        kind.append(1)
    for i in range(2):  # extreme: conic entries beyond FP32 range
        z = 2.0 + 0.5 * i
        pos.append([(0.25 + 0.1 * i) * z, 0.0, z] if i == 0 else [0.0, 0.15 * z, z])
        scale.append([0.06, 1e-24, 1e-24] if i == 0 else [1e-24, 0.06, 1e-24])
        rot.append([1, 0, 0, 0])
        kind.append(2)
    n = len(pos)
    opacity = np.where(np.asarray(kind) == 0, rng.uniform(0.2, 0.8, n), 0.8)
    sh = rng.normal(0.0, 0.4, (n, 1, 3))
    a = H.flat_asset(pos, scale, rot, opacity, sh)
    return a, np.asarray(kind)


def test_needles_take_the_fp64_redo_and_match_the_oracle(torch):
    a, kind = _needle_scene(3)
    n = kind.size
    T = sg.identity_instances(1)
    cam = H.identity_camera(W, HH, F, cx=CX, cy=CY, bg=(0.05, 0.1, 0.15))
    sc = v.Scene(a, T)
    sel = sc.select(cam, 0.0)  # tau = 0: the leaves, every row once in stored order
    gids = sel.ids()
    ref_gids = oracle.mask_to_gids(oracle.select_walk(a, T, cam, 0.0))
    assert np.array_equal(gids, ref_gids)
    img = sc.render(cam, sel).cpu().numpy()
    st = sc.frame_stats()
    _say("needles: %d slots, fp64 redo %d, clamped %d" % (st["n_slots"], st["n_fp64_conics"],
                                                           st["n_conics_clamped"]))
    assert st["n_slots"] == n
    assert st["n_fp64_conics"] == int((kind > 0).sum())
    assert st["n_conics_clamped"] == int((kind == 2).sum())

    g = sc.projection()
    r = oracle.project(a, T, cam, gids)
    assert np.array_equal(g["depth"].view(np.uint32), r["depth"].view(np.uint32))
    vis = g["tiles"] > 0
    assert (r["valid"][vis] == 1).all()
    # every needle is in view and kept
    assert vis[kind > 0].all()
    gc = g["conic"].astype(np.float64)
    rc = r["conic"]
    ndl = (kind == 1) & vis
    # conic entries of the FP64 redo against the oracle, entry by entry (the
    # off-diagonal measured against the diagonal's geometric mean)
    scale_b = np.sqrt(np.abs(rc[ndl, 0] * rc[ndl, 2]))
    assert (np.abs(gc[ndl, 0] - rc[ndl, 0]) <= 2e-3 * np.abs(rc[ndl, 0])).all()
    assert (np.abs(gc[ndl, 2] - rc[ndl, 2]) <= 2e-3 * np.abs(rc[ndl, 2])).all()
    assert (np.abs(gc[ndl, 1] - rc[ndl, 1]) <= 2e-3 * np.maximum(np.abs(rc[ndl, 1]), 1e-3 * scale_b)).all()
    # extreme needles: the long axis as the oracle's, the thin axis clamped
    ext = np.flatnonzero(kind == 2)
    row, col = ext[0], ext[1]
    assert rc[row, 2] > 1e38 and gc[row, 2] == np.float32(1e38)
    assert abs(gc[row, 0] - rc[row, 0]) <= 1e-6 * rc[row, 0]
    assert rc[col, 0] > 1e38 and gc[col, 0] == np.float32(1e38)
    assert abs(gc[col, 2] - rc[col, 2]) <= 1e-6 * rc[col, 2]

    assert np.isfinite(img).all()
    ref, amb, _ = oracle.render(a, T, cam, gids)
    check_image(img, ref, amb, "needles")
    # the test draws something: the axis-aligned needles alone cover many
    # pixels of row 32 and column 48 in the oracle's image, and nothing else
    idx = np.flatnonzero((kind > 0) & (np.abs(a.pos[: kind.size, 0]) * np.abs(a.pos[: kind.size, 1]) == 0))
    an = H.flat_asset(a.pos[idx], a.scale[idx], a.rot[idx], a.opacity[idx], a.sh[idx])
    alone, _, _ = oracle.render(an, T, cam, oracle.mask_to_gids(oracle.select_walk(an, T, cam, 0.0)))
    lit = alone[..., 3] > 0.05
    _say("needles alone light %d pixels on row 32 and %d on column 48" % (lit[32].sum(), lit[:, 48].sum()))
    assert lit[32].sum() > 40 and lit[:, 48].sum() > 25
    lit[32, :] = False
    lit[:, 48] = False
    assert not lit.any()
    sc.close()


def test_generic_scene_takes_no_fp64_redo(torch):
    """Ordinary splats (at least a few tenths of a pixel across) never reach the
    FP64 branch, and no conic is clamped."""
    a = sg.make_asset(16384, 0, 1)
    sc = v.Scene(a)
    cam = sg.single_camera_c1()
    sel = sc.select(cam, 1.0)
    sc.render(cam, sel)
    st = sc.frame_stats()
    # the oracle's smallest 2D determinant in this frame is ~9e-3 px^4
    r = oracle.project(a, sg.identity_instances(1), cam, sel.ids())
    c = r["cov2"][r["valid"] == 1]
    assert (c[:, 0] * c[:, 2] - c[:, 1] ** 2).min() > 1e-3
    _say("c1 frame: %d slots, fp64 redo %d" % (st["n_slots"], st["n_fp64_conics"]))
    assert st["n_fp64_conics"] == 0 and st["n_conics_clamped"] == 0
    sc.close()
