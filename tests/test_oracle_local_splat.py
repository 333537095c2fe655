"""Pins of the local-splatting oracle (paper Sec. 3.2).

* its render equals the pinned renderer oracle (C, FP64) on a pseudo-view;
* its gradients equal central finite differences of its loss;
* fitting the simplified Gaussians lowers the loss, and a set fitted to
  itself has zero loss and does not move.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import local_splat as ls
import scenegen as sg


def _group(m, seed, spread=0.3):
    rng = np.random.default_rng(seed)
    pos = (rng.standard_normal((m, 3)) * spread).astype(np.float32)
    scale = np.exp(rng.uniform(np.log(0.03), np.log(0.12), (m, 3))).astype(np.float32)
    q = rng.standard_normal((m, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    q[q[:, 0] < 0] *= -1
    opacity = rng.uniform(0.2, 0.9, m).astype(np.float32)
    sh = (rng.standard_normal((m, 1, 3)) * 0.8).astype(np.float32)
    return dict(pos=pos, scale=scale, rot=q.astype(np.float32), opacity=opacity, sh=sh)


def _asset(g):
    m = len(g["opacity"])
    k = (m + 63) // 64
    first = np.arange(k, dtype=np.uint32) * 64
    count = np.minimum(64, m - first).astype(np.uint8)
    c = g["pos"].mean(0)
    sph = np.tile(np.array([c[0], c[1], c[2], 0.0], np.float32), (k, 1))
    par = sph.copy()
    par[:, 3] = np.inf
    return sg.Asset(sh_degree=0, pos=g["pos"], scale=g["scale"], rot=g["rot"], opacity=g["opacity"], sh=g["sh"],
                    first_row=first, count=count, level=np.zeros(k, np.uint8), parent=np.full(k, -1, np.int32),
                    first_child=np.full(k, -1, np.int32), n_children=np.zeros(k, np.uint8), self_sphere=sph,
                    parent_sphere=par, n_leaf_clusters=k)


def _cam(center, radius, d):
    d = np.asarray(d, np.float64)
    up = (0.0, 1.0, 0.0) if abs(d[2]) > 0.99 else (0.0, 0.0, 1.0)
    return sg.look_at(np.asarray(center) + 4 * radius * d, center, 64, 64, 2 * math.asin(0.25), up=up)


def _torch_params(g):
    return ls.params_from(g["pos"], g["scale"], g["rot"], g["opacity"], g["sh"])


@pytest.mark.parametrize("m,seed", [(1, 1), (40, 2), (128, 3)])
def test_render_equals_renderer_oracle(m, seed):
    g = _group(m, seed)
    c = g["pos"].mean(0).astype(np.float64)
    r = 0.6
    for d in [(0.3, -0.8, 0.52), (0.0, 0.0, 1.0), (-1.0, 0.0, 0.0)]:
        d = np.asarray(d) / np.linalg.norm(d)
        cam = _cam(c, r, d)
        Rv0, eye0 = ls.view_camera(c, r, d)
        w2c = cam.world_to_cam.astype(np.float64)
        np.testing.assert_allclose(Rv0, w2c[:, :3], atol=1e-6)
        np.testing.assert_allclose(eye0, cam.centre(), atol=1e-5)
        p = _torch_params(g)
        with torch.no_grad():
            rgb, a = ls.render(p["pos"], torch.exp(p["log_scale"]), p["quat"], torch.sigmoid(p["logit"]), p["dc"],
                               w2c[:, :3], cam.centre())
        ref, amb, _ = oracle.render(_asset(g), sg.identity_instances(1), cam,
                                    np.arange((m + 63) // 64, dtype=np.uint32))
        ok = amb == 0
        assert ok.mean() > 0.98
        err = np.abs(rgb.numpy() - ref[..., :3])[ok].max()
        err_a = np.abs(a.numpy() - ref[..., 3])[ok].max()
        assert err < 1e-6 and err_a < 1e-6, (m, d, err, err_a)


def test_gradients_equal_finite_differences():
    orig, simp = _group(24, 7), _group(12, 8)
    c, r = orig["pos"].mean(0), 0.7
    d = np.array([0.2, 0.9, 0.3])
    d /= np.linalg.norm(d)
    Rv, eye = ls.view_camera(c, r, d)
    po, ps = _torch_params(orig), _torch_params(simp)
    with torch.no_grad():
        target = ls.render(po["pos"], torch.exp(po["log_scale"]), po["quat"], torch.sigmoid(po["logit"]), po["dc"],
                           Rv, eye)
    for t in ps.values():
        t.requires_grad_(True)
    ls.loss_of(ps, target, Rv, eye).backward()
    rng = np.random.default_rng(0)
    for k, t in ps.items():
        for _ in range(4):
            idx = tuple(int(rng.integers(0, s)) for s in t.shape)
            h = 1e-6
            with torch.no_grad():
                t[idx] += h
                lp = float(ls.loss_of(ps, target, Rv, eye))
                t[idx] -= 2 * h
                lm = float(ls.loss_of(ps, target, Rv, eye))
                t[idx] += h
            fd = (lp - lm) / (2 * h)
            g = float(t.grad[idx])
            assert abs(fd - g) <= 1e-5 + 1e-3 * abs(g), (k, idx, fd, g)


def test_fitting_lowers_the_loss():
    orig = _group(48, 11)
    keep = np.argsort(-orig["opacity"])[:24]
    simp = {k: v[keep].copy() for k, v in orig.items()}
    simp["scale"] = simp["scale"] * np.float32(2 ** (1 / 6))
    rng = np.random.default_rng(3)
    dirs = rng.standard_normal((60, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    out, losses, _ = ls.local_splat(orig, simp, orig["pos"].mean(0), 0.8, dirs, 60)
    assert np.mean(losses[-10:]) < 0.9 * np.mean(losses[:10]), (losses[:10], losses[-10:])
    assert out["pos"].shape == simp["pos"].shape


def test_a_set_fitted_to_itself_stays():
    g = _group(20, 5)
    dirs = np.array([[0.0, 0.6, 0.8], [1.0, 0.0, 0.0], [0.0, -1.0, 0.0]])
    out, losses, grads = ls.local_splat(g, g, g["pos"].mean(0), 0.7, dirs, 3)
    assert max(losses) == 0.0
    for k in grads:
        assert np.abs(grads[k]).max() == 0.0
    np.testing.assert_allclose(out["pos"], g["pos"], atol=0)
    np.testing.assert_allclose(out["opacity"], g["opacity"].astype(np.float64), rtol=1e-12)
