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


# ---- builds with local splatting (Sec. 3.2) ---------------------------------
ROWS = ("pos", "scale", "rot", "opacity", "sh", "src", "gen")
LR = dict(pos=1.6e-5, log_scale=5e-3, quat=1e-3, logit=5e-2, dc=2.5e-3)


def _unit_dirs(n, seed):
    d = np.random.default_rng(seed).standard_normal((n, 3))
    return (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)


def _group_of(b, p):
    """Rows of the cluster group that made cluster p: its children's rows in
    child order, and the children's ids."""
    kids = range(int(b["first_child"][p]), int(b["first_child"][p]) + int(b["n_children"][p]))
    idx = np.concatenate([np.arange(b["first_row"][c], b["first_row"][c] + b["count"][c]) for c in kids])
    return idx, list(kids)


def _halved(b, idx):
    """The group's kept rows before the fit: the ceil(m/2) largest
    ((sx sy) sz) o (ties: the earlier), scales grown once."""
    s, o = b["scale"][idx], b["opacity"][idx]
    score = ((s[:, 0] * s[:, 1]) * s[:, 2]) * o
    keep = np.sort(np.argsort(-score.astype(np.float64), kind="stable")[:(len(idx) + 1) // 2])
    init = {k: b[k][idx][keep].copy() for k in ROWS}
    init["scale"] = init["scale"] * GROW
    return init


GROW = np.float32(2.0 ** (1.0 / 6.0))


def _rows_of(b, idx):
    return {k: b[k][idx] for k in ROWS}


def test_fitted_build_every_group_matches_oracle(torch):
    """Every group of a build with local splatting, taken on the GPU's own
    inputs (its children's rows as built): the kept Gaussians are the top
    half by score, the sphere is the oracle's bit for bit, and the fitted rows
    follow the FP64 local-splatting oracle (differences measured in Adam
    steps of each parameter's learning rate); the leaves equal the
    structural oracle's."""
    from oracle import local_splat as ls
    iters = 6
    dirs = _unit_dirs(iters, 17)
    pos, scale, rot, opacity, sh = _input(1000, 1, 23)
    g = v.build_bundle(pos, scale, rot, opacity, sh, 64, fit_iters=iters, view_dirs=dirs)
    r = ob.build_bundle(pos, scale, rot, opacity, sh, 64)
    nl = g["n_leaf_clusters"]
    assert nl == r["n_leaf_clusters"] and g["n_layers"] == int(r["level"].max()) + 1
    L = int(g["first_row"][nl - 1]) + int(g["count"][nl - 1])
    for k in ROWS + ("first_row", "count", "self_sphere"):
        a, b_ = np.asarray(g[k]), np.asarray(r[k]).astype(np.asarray(g[k]).dtype).reshape(np.asarray(g[k]).shape)
        sel = slice(0, L) if k in ROWS else slice(0, nl)
        np.testing.assert_array_equal(a[sel], b_[sel], err_msg=k)
    assert g["fit_loss"].shape == (g["n_layers"] - 1, iters)
    errs = {k: [] for k in LR}
    for p in range(nl, len(g["count"])):
        idx, kids = _group_of(g, p)
        rows = _rows_of(g, idx)
        init = _halved(g, idx)
        mine = np.arange(g["first_row"][p], g["first_row"][p] + g["count"][p])
        np.testing.assert_array_equal(g["src"][mine], init["src"])
        assert (g["gen"][mine] == g["level"][p]).all()
        sph = ob.group_sphere(rows["pos"], [g["self_sphere"][c] for c in kids])
        np.testing.assert_array_equal(g["self_sphere"][p], sph)
        vs = ob.view_sphere(rows, sph)
        out, _, _ = ls.local_splat(rows, init, vs[:3].astype(np.float64), float(vs[3]), dirs.astype(np.float64),
                                   iters)
        errs["pos"].append(np.abs(g["pos"][mine] - out["pos"]).ravel() / LR["pos"])
        errs["log_scale"].append(np.abs(np.log(g["scale"][mine]) - np.log(out["scale"])).ravel() / LR["log_scale"])
        qd = np.minimum(np.abs(g["rot"][mine] - out["rot"]).max(1), np.abs(g["rot"][mine] + out["rot"]).max(1))
        errs["quat"].append(qd / LR["quat"])
        lo = lambda o: np.log(o / (1 - o))
        errs["logit"].append(np.abs(lo(g["opacity"][mine].astype(np.float64)) - lo(out["opacity"])) / LR["logit"])
        errs["dc"].append(np.abs(g["sh"][mine][:, 0, :] - out["sh"][:, 0, :]).ravel() / LR["dc"])
    for k, e in errs.items():
        e = np.concatenate(e)
        _say("fitted build %-9s |gpu - oracle| in steps of lr: median %.2e  99%% %.2e  max %.2e"
             % (k, np.median(e), np.quantile(e, 0.99), e.max()))
        # within half an Adam step of the parameter everywhere (a step moves it by about lr)
        assert np.median(e) < 0.01 and e.max() < 0.5, (k, np.median(e), e.max())


def test_fitted_build_equals_the_local_splat_entry_point(torch):
    """The build's refinement is v3dg_local_splat on each group's rows: every
    coarse cluster of a 20000-Gaussian build equals, bit for bit, the entry
    point run on its children's rows and its kept rows before the fit, with
    the oracle's view sphere (so the build frames its views bit for bit as
    the oracle does)."""
    iters = 20
    dirs = _unit_dirs(iters, 3)
    pos, scale, rot, opacity, sh = _input(20000, 2, 31)
    g = v.build_bundle(pos, scale, rot, opacity, sh, 64, fit_iters=iters, view_dirs=dirs)
    nl = g["n_leaf_clusters"]
    groups, orig, fit, mine = [], [], [], []
    o0 = f0 = 0
    for p in range(nl, len(g["count"])):
        idx, _ = _group_of(g, p)
        init = _halved(g, idx)
        orig.append(_rows_of(g, idx))
        fit.append(init)
        mine.append(np.arange(g["first_row"][p], g["first_row"][p] + g["count"][p]))
        groups.append((o0, len(idx), f0, len(init["src"]), tuple(ob.view_sphere(_rows_of(g, idx), g["self_sphere"][p]))))
        o0 += len(idx)
        f0 += len(init["src"])
    cat = lambda parts: {k: np.concatenate([q[k] for q in parts]) for k in ROWS}
    o, f = cat(orig), cat(fit)
    o["dc"], f["dc"] = o["sh"][:, 0, :], f["sh"][:, 0, :]
    out, losses, _ = v.local_splat(groups, o, f, dirs, iters)
    rows = np.concatenate(mine)
    for k in ("pos", "scale", "rot", "opacity"):
        np.testing.assert_array_equal(g[k][rows], out[k], err_msg=k)
    np.testing.assert_array_equal(g["sh"][rows][:, 0, :], out["dc"])
    np.testing.assert_array_equal(g["sh"][rows][:, 1:, :], f["sh"][:, 1:, :])
    # the layer means of the losses
    lvl = g["level"][nl:]
    for l in range(1, g["n_layers"]):
        np.testing.assert_allclose(g["fit_loss"][l - 1], losses[lvl == l].astype(np.float64).mean(0), rtol=1e-5)
    _say("fitted build: %d groups, layer-1 loss %.4f -> %.4f" % (len(groups), g["fit_loss"][0, 0],
                                                                 g["fit_loss"][0, -1]))


def test_fitted_build_full_size_sampled(torch):
    """The benchmark asset's 1M leaves built with local splatting (16 views
    per group, the launch shape of the 640-view build): sampled groups of the
    first, a middle and the top layer, taken on the GPU's own inputs, keep the
    oracle's kept set and sphere bit for bit and follow the FP64 oracle's fit
    within half an Adam step."""
    from oracle import local_splat as ls
    iters = 16
    dirs = _unit_dirs(iters, 29)
    a = sg.cached_asset(1 << 20, 3, 2)
    L = a.n_leaf_rows
    g = v.build_bundle(a.pos[:L], a.scale[:L], a.rot[:L], a.opacity[:L], a.sh[:L], 64, fit_iters=iters,
                       view_dirs=dirs)
    nl = g["n_leaf_clusters"]
    lv = g["level"]
    picks = []
    for layer in (1, int(lv.max()) // 2, int(lv.max())):
        ids = np.flatnonzero(lv == layer)
        picks += list(ids[np.linspace(0, len(ids) - 1, 2).astype(int)]) if len(ids) > 1 else list(ids)
    worst = 0.0
    for p in sorted(set(int(x) for x in picks)):
        idx, kids = _group_of(g, p)
        rows = _rows_of(g, idx)
        init = _halved(g, idx)
        mine = np.arange(g["first_row"][p], g["first_row"][p] + g["count"][p])
        np.testing.assert_array_equal(g["src"][mine], init["src"])
        sph = ob.group_sphere(rows["pos"], [g["self_sphere"][c] for c in kids])
        np.testing.assert_array_equal(g["self_sphere"][p], sph)
        vs = ob.view_sphere(rows, sph)
        out, _, _ = ls.local_splat(rows, init, vs[:3].astype(np.float64), float(vs[3]), dirs.astype(np.float64), iters)
        e_pos = np.abs(g["pos"][mine] - out["pos"]).max() / LR["pos"]
        e_ls = np.abs(np.log(g["scale"][mine]) - np.log(out["scale"])).max() / LR["log_scale"]
        lo = lambda o: np.log(o / (1 - o))
        e_op = np.abs(lo(g["opacity"][mine].astype(np.float64)) - lo(out["opacity"])).max() / LR["logit"]
        e_dc = np.abs(g["sh"][mine][:, 0, :] - out["sh"][:, 0, :]).max() / LR["dc"]
        worst = max(worst, e_pos, e_ls, e_op, e_dc)
        assert max(e_pos, e_ls, e_op, e_dc) < 0.5, (p, lv[p], e_pos, e_ls, e_op, e_dc)
    _say("1M fitted build: %d sampled groups (layers 1 .. %d) within %.2e Adam steps of the oracle"
         % (len(set(picks)), int(lv.max()), worst))
