"""Offline build on the GPU (v3dg_build_bundle) against the oracle.

Every decision of the build (split axes and orders, kept Gaussians, grouping)
is taken in a fixed arithmetic order, so the GPU bundle equals the oracle's
bit for bit: rows, scales, cluster links and spheres.  The built bundle then
loads and renders like any other asset.
"""
import numpy as np
import pytest

import oracle
from oracle import offline_build as ob
import paper_2505_06523_amd as v
import scenegen as sg
from tests import helpers as H
from tests.test_gpu_parity import _say, check_image

pytestmark = pytest.mark.gpu

FIELDS = ["src", "gen", "first_row", "count", "level", "parent", "first_child", "n_children", "self_sphere",
          "parent_sphere", "pos", "scale", "rot", "opacity", "sh"]


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a GPU"
    v.lib()
    return _t


def _input(n, sh_degree, seed):
    a = sg.make_asset(max(n, 64), sh_degree, seed)
    return a.pos[:n], a.scale[:n], a.rot[:n], a.opacity[:n], a.sh[:n]


def _same(g, r, tag):
    assert g["n_leaf_clusters"] == r["n_leaf_clusters"], tag
    for k in FIELDS:
        a = np.asarray(g[k])
        b = np.asarray(r[k]).astype(a.dtype).reshape(a.shape)
        if a.dtype.kind == "f":
            bad = np.flatnonzero(a.view(np.uint32).reshape(-1) != b.view(np.uint32).reshape(-1))
        else:
            bad = np.flatnonzero(a.reshape(-1) != b.reshape(-1))
        assert bad.size == 0, (tag, k, bad[:5], a.reshape(-1)[bad[:5]], b.reshape(-1)[bad[:5]])


@pytest.mark.parametrize("n,sh_degree,cluster", [(1, 0, 64), (64, 1, 64), (65, 1, 64), (1000, 0, 64),
                                                 (4096, 3, 64), (12345, 1, 64), (5000, 1, 16), (777, 2, 2)])
def test_build_matches_oracle(torch, n, sh_degree, cluster):
    pos, scale, rot, opacity, sh = _input(n, sh_degree, 11 + n)
    g = v.build_bundle(pos, scale, rot, opacity, sh, cluster)
    r = ob.build_bundle(pos, scale, rot, opacity, sh, cluster)
    _same(g, r, (n, cluster))
    _say("build n=%d cluster=%d: %d clusters, %d rows, %d layers" % (n, cluster, len(g["count"]), len(g["src"]),
                                                                    g["n_layers"]))


def test_build_ties_and_signed_zeros(torch):
    """Duplicate positions, -0 / +0 coordinates and equal scores: the stable
    orders of the paper's split and halving decide, as in the oracle."""
    n = 3000
    rng = np.random.default_rng(5)
    pos = rng.integers(-3, 4, size=(n, 3)).astype(np.float32) * np.float32(0.25)
    pos[::7, 1] = -0.0
    scale = np.full((n, 3), 0.01, np.float32)
    scale[::3] = 0.02
    opacity = np.where(rng.random(n) < 0.5, 0.5, 0.25).astype(np.float32)
    rot = np.tile(np.array([1, 0, 0, 0], np.float32), (n, 1))
    sh = rng.standard_normal((n, 4, 3)).astype(np.float32)
    _same(v.build_bundle(pos, scale, rot, opacity, sh, 64), ob.build_bundle(pos, scale, rot, opacity, sh, 64), "ties")


def test_built_bundle_renders_like_the_oracle(torch):
    pos, scale, rot, opacity, sh = _input(20000, 1, 4)
    b = v.build_bundle(pos, scale, rot, opacity, sh, 64)
    a = H.bundle_asset(b, 1)
    T = sg.identity_instances(1)
    sc = v.Scene(a, T)
    cam = sg.look_at((1.8, -1.6, 1.1), (0, 0, 0), 211, 157, 1.0)
    for tau in [0.0, 4.0, 400.0]:
        sel = sc.select(cam, tau)
        gids = sel.ids()
        assert np.array_equal(gids, oracle.mask_to_gids(oracle.select_walk(a, T, cam, tau)))
        img = sc.render(cam, sel).cpu().numpy()
        ref, amb, _ = oracle.render(a, T, cam, gids)
        check_image(img, ref, amb, "built bundle tau=%g" % tau)
        sel.free()
    sc.close()


def test_build_c2_size_sampled(torch):
    """The 1M-Gaussian leaves of the benchmark asset, rebuilt on the GPU: the
    tree invariants hold at full size and a subtree matches the oracle."""
    a = sg.cached_asset(1 << 20, 3, 2)
    L = a.n_leaf_rows
    pos, scale, rot, opacity, sh = a.pos[:L], a.scale[:L], a.rot[:L], a.opacity[:L], a.sh[:L]
    g = v.build_bundle(pos, scale, rot, opacity, sh, 64)
    C = len(g["count"])
    _say("c2 build: %d clusters, %d rows, %d layers" % (C, len(g["src"]), g["n_layers"]))
    nl = g["n_leaf_clusters"]
    leaf_rows = int(g["first_row"][nl - 1]) + int(g["count"][nl - 1])
    assert np.array_equal(np.sort(g["src"][:leaf_rows]), np.arange(L))
    assert list(np.flatnonzero(g["parent"] < 0)) == [C - 1]
    assert g["count"].max() <= 64
    # rows: copies of the input with scales grown gen times
    grow = np.float32(2.0 ** (1.0 / 6.0))
    s = scale[g["src"]].copy()
    for t in range(1, int(g["gen"].max()) + 1):
        sel = g["gen"] >= t
        s[sel] = s[sel] * grow
    np.testing.assert_array_equal(g["scale"], s)
    np.testing.assert_array_equal(g["pos"], pos[g["src"]])
    # the loader accepts it
    sc = v.Scene(H.bundle_asset(g, 3), sg.identity_instances(1))
    sc.close()
