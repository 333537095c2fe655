"""Pins of the local-splatting oracle (paper Sec. 3.2).

* its render equals the pinned renderer oracle (C, FP64) on a pseudo-view;
* its gradients equal central finite differences of its loss;
* fitting the simplified Gaussians lowers the loss, and a set fitted to
  itself has zero loss and does not move;
* the first iteration makes exactly the first bias-corrected Adam step with
  each parameter's learning rate;
* the loss of one isotropic splat against an empty view equals its closed form.
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


def test_first_step_is_the_bias_corrected_adam_step():
    """Adam's first bias-corrected step (m1 = (1 - b1) g, v1 = (1 - b2) g^2,
    so m1 / (1 - b1) = g and v1 / (1 - b2) = g^2) moves every parameter by
    exactly -lr sign(g) (eps = 1e-15 is far below |g|), with the learning rate
    of its kind: position 1.6e-5, log scale 5e-3, quaternion 1e-3 (then
    normalised), logit opacity 5e-2, dc 2.5e-3 (Sec. 3.2; the last four are the
    3DGS defaults).  A wrong bias correction or learning-rate mapping moves
    some parameter by another amount."""
    orig, simp = _group(30, 21), _group(10, 22)
    d = np.array([[0.3, -0.4, 0.866]])
    d /= np.linalg.norm(d)
    out, losses, g = ls.local_splat(orig, simp, orig["pos"].mean(0), 0.8, d, 1)
    p0 = _torch_params(simp)
    lr = dict(pos=1.6e-5, log_scale=5e-3, quat=1e-3, logit=5e-2, dc=2.5e-3)
    for k in lr:  # a gradient of exactly 0 (or below 1e-15) would not move; none here
        assert (np.abs(g[k]) > 1e-12).mean() > 0.9, k
    live = {k: np.abs(g[k]) > 1e-12 for k in lr}

    def moved(k, after, before):
        step = after - before.numpy()
        want = -lr[k] * np.sign(g[k])
        np.testing.assert_allclose(step[live[k]], want[live[k]], rtol=1e-9, atol=1e-13, err_msg=k)

    moved("pos", out["pos"], p0["pos"])
    moved("log_scale", np.log(out["scale"]), p0["log_scale"])
    moved("logit", np.log(out["opacity"] / (1 - out["opacity"])), p0["logit"])
    moved("dc", out["sh"][:, 0, :], p0["dc"])
    q1 = p0["quat"].numpy() - lr["quat"] * np.sign(g["quat"]) * live["quat"]
    np.testing.assert_allclose(out["rot"], q1 / np.linalg.norm(q1, axis=1, keepdims=True), rtol=1e-9, atol=1e-12)


def test_loss_of_one_splat_against_an_empty_target():
    """The loss is mean |rgb - target| + 0.1 mean |alpha - target alpha| over
    the 64 x 64 view.  Against an empty target (zero colour and alpha), one
    isotropic splat at the group centre, seen on the view axis at distance 4 r,
    has alpha(p) = min(0.99, o exp(-|p - (32, 32)|^2 / (2 sigma^2))) with
    sigma = f s / (4 r) (zero where alpha < 1/255) and colour alpha(p) c with
    c = max(0, C0 dc + 0.5), so the loss is mean(alpha) (mean(c) + 0.1)."""
    c = np.array([0.1, -0.2, 0.3])
    r, s, o = 0.5, 0.03, 0.8
    dc = np.array([0.7, -0.9, 2.5])  # the last channel is clamped at 0 after the shift
    simp = dict(pos=c[None].astype(np.float32), scale=np.full((1, 3), s, np.float32),
                rot=np.array([[0.6, 0.0, 0.8, 0.0]], np.float32), opacity=np.array([o], np.float32),
                sh=dc.reshape(1, 1, 3).astype(np.float32))
    d = np.array([0.48, 0.6, 0.64])
    Rv, eye = ls.view_camera(c, r, d)
    p = _torch_params(simp)
    target = (torch.zeros(64, 64, 3, dtype=torch.float64), torch.zeros(64, 64, dtype=torch.float64))
    got = float(ls.loss_of(p, target, Rv, eye))
    focal = 32.0 / math.tan(math.asin(0.25))  # the view's sphere of radius r at 4 r spans the image
    pc = (np.asarray(simp["pos"][0], np.float64) - eye) @ Rv.T  # on the axis up to rounding
    zc = pc[2]
    u = focal * pc[0] / zc + 32.0
    v = focal * pc[1] / zc + 32.0
    sig2 = (focal * float(np.float32(s)) / zc) ** 2
    ys, xs = np.mgrid[0:64, 0:64] + 0.5
    alpha = np.minimum(0.99, float(np.float32(o)) * np.exp(-((xs - u) ** 2 + (ys - v) ** 2) / (2 * sig2)))
    alpha[alpha < 1 / 255] = 0.0
    y00 = 0.5 / math.sqrt(math.pi)
    col = np.maximum(0.0, y00 * np.asarray(simp["sh"][0, 0], np.float64) + 0.5)
    assert abs(u - 32.0) < 1e-6 and abs(v - 32.0) < 1e-6 and abs(zc - 4 * r) < 1e-6
    assert col[2] > 0 and col.min() >= 0.0
    want = alpha.mean() * (col.mean() + 0.1)
    assert got == pytest.approx(want, rel=1e-6)
