"""CPU oracle of the local splatting of a cluster group (paper Sec. 3.2).

TEST INFRASTRUCTURE ONLY: only ``tests/`` may import it.  It shares no code with
the HIP library.  Plain PyTorch on the CPU in FP64; the gradients come from
autograd.

The simplified Gaussians of a group are fitted to the group's original ones:
for every pseudo-view (facing the group centre from four radii away), both
sets are rendered at 64 x 64, the two renders are compared, and the loss is
back-propagated into the simplified Gaussians; adaptive density control is
off and positions use the learning rate 1.6e-5 (the paper's).  Choices the
paper leaves open are fixed as follows:

* View i looks at the centre c from c + 4 r d_i (d_i: unit directions given
  by the caller), OpenCV axes (x right, y down, z forward), up = +z unless
  |d_z| > 0.99 (then +y); 64 x 64 pixels, f = 32 / tan(asin(1/4)) so that
  the sphere spans the image; pixel centres at +0.5.
* Splatting as in the renderer (EWA, no dilation, Jacobian guard band
  1.3 tan(fov/2), cull det <= 0 and z <= 0.01); alpha = min(0.99, o e^power)
  with power = min(0, quadratic form), skip alpha < 1/255, stop before a
  splat that would take T below 1e-4, depth order (ties: index order).
* Colour of a Gaussian in these renders: max(0, C0 dc + 0.5), its SH degree-0
  term (the paper's assets are degree 0); higher SH bands are left as they are.
* Loss: mean |rgb - rgb_target| + 0.1 mean |alpha - alpha_target| (L1 and the
  paper's alpha supervision; no D-SSIM term).  Background 0.
* Parameters: position, log scale, quaternion (normalised in the render),
  logit opacity, dc; Adam (beta 0.9 / 0.999, eps 1e-15) with learning rates
  1.6e-5, 5e-3, 1e-3, 5e-2, 2.5e-3 (the last four: the 3DGS defaults).  One
  view per iteration, view i at iteration i.
"""
from __future__ import annotations

import math

import numpy as np
import torch

C0 = 0.28209479177387814
RES = 64
FOCAL = 32.0 * math.sqrt(15.0)  # 32 / tan(asin(1/4))
LR = dict(pos=1.6e-5, log_scale=5e-3, quat=1e-3, logit=5e-2, dc=2.5e-3)
ALPHA_W = 0.1


def view_camera(center, radius, d):
    """World-to-camera rotation (rows: x, y, z axes) and eye of a pseudo-view."""
    c = np.asarray(center, np.float64)
    d = np.asarray(d, np.float64)
    eye = c + 4.0 * float(radius) * d
    fwd = -d / np.linalg.norm(d)
    up = np.array([0.0, 1.0, 0.0]) if abs(d[2]) > 0.99 else np.array([0.0, 0.0, 1.0])
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    return np.stack([right, down, fwd]), eye


def quat_mat(q):
    q = q / torch.linalg.norm(q, dim=-1, keepdim=True)
    w, x, y, z = q.unbind(-1)
    return torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)], -2)


def render(pos, scale, quat, opacity, dc, Rv, eye):
    """RGB (64, 64, 3) and alpha (64, 64) of Gaussians (torch FP64 tensors)."""
    Rv = torch.as_tensor(Rv, dtype=torch.float64)
    eye = torch.as_tensor(eye, dtype=torch.float64)
    pc = (pos - eye) @ Rv.T
    x, y, z = pc.unbind(-1)
    valid = z > 0.01
    zs = torch.where(valid, z, torch.ones_like(z))
    u = FOCAL * x / zs + 32.0
    v = FOCAL * y / zs + 32.0
    lim = 1.3 * 32.0 / FOCAL
    tx = torch.clamp(x / zs, -lim, lim) * zs
    ty = torch.clamp(y / zs, -lim, lim) * zs
    zero = torch.zeros_like(zs)
    J = torch.stack([torch.stack([FOCAL / zs, zero, -FOCAL * tx / (zs * zs)], -1),
                     torch.stack([zero, FOCAL / zs, -FOCAL * ty / (zs * zs)], -1)], -2)
    Rq = quat_mat(quat)
    M = Rq * scale.unsqueeze(-2)
    S3 = M @ M.transpose(-1, -2)
    T = J @ Rv.unsqueeze(0)
    S2 = T @ S3 @ T.transpose(-1, -2)
    a, b, c = S2[:, 0, 0], S2[:, 0, 1], S2[:, 1, 1]
    det = a * c - b * b
    valid = valid & (det > 0)
    dets = torch.where(valid, det, torch.ones_like(det))
    ca, cb, cc = c / dets, -b / dets, a / dets
    rgb = torch.clamp(C0 * dc + 0.5, min=0.0)
    zd = z.detach()
    order = sorted(range(len(zd)), key=lambda i: (float(zd[i]), i))
    py, px = torch.meshgrid(torch.arange(RES, dtype=torch.float64) + 0.5,
                            torch.arange(RES, dtype=torch.float64) + 0.5, indexing="ij")
    Tr = torch.ones(RES, RES, dtype=torch.float64)
    col = torch.zeros(RES, RES, 3, dtype=torch.float64)
    live = torch.ones(RES, RES, dtype=torch.bool)
    for i in order:
        if not bool(valid[i]):
            continue
        dx, dy = u[i] - px, v[i] - py
        power = torch.clamp(-0.5 * (ca[i] * dx * dx + cc[i] * dy * dy) - cb[i] * dx * dy, max=0.0)
        alpha = torch.clamp(opacity[i] * torch.exp(power), max=0.99)
        take = live & (alpha >= 1.0 / 255.0)
        Tn = Tr * (1.0 - alpha)
        stop = take & (Tn < 1e-4)
        add = take & ~stop
        col = col + torch.where(add.unsqueeze(-1), (alpha * Tr).unsqueeze(-1) * rgb[i], torch.zeros_like(col))
        Tr = torch.where(add, Tn, Tr)
        live = live & ~stop
    return col, 1.0 - Tr


def params_from(pos, scale, rot, opacity, sh):
    """Trainable parameters of Gaussians given as numpy rows."""
    o = np.clip(np.asarray(opacity, np.float64), 1e-6, 1 - 1e-6)
    return dict(pos=torch.tensor(np.asarray(pos, np.float64)),
                log_scale=torch.tensor(np.log(np.asarray(scale, np.float64))),
                quat=torch.tensor(np.asarray(rot, np.float64)),
                logit=torch.tensor(np.log(o / (1 - o))),
                dc=torch.tensor(np.asarray(sh, np.float64).reshape(len(o), -1, 3)[:, 0, :].copy()))


def loss_of(p, target, Rv, eye):
    rgb, a = render(p["pos"], torch.exp(p["log_scale"]), p["quat"], torch.sigmoid(p["logit"]), p["dc"], Rv, eye)
    return (rgb - target[0]).abs().mean() + ALPHA_W * (a - target[1]).abs().mean()


def local_splat(orig, simp, center, radius, dirs, iters):
    """Fit the simplified Gaussians (dict of numpy rows: pos, scale, rot,
    opacity, sh) to the originals over views dirs[0 .. iters-1].  Returns the
    fitted rows (quaternions as unit quaternions, which rotate as the fitted
    ones do), the loss of every iteration (before its step) and the gradients
    of the first iteration."""
    po = params_from(orig["pos"], orig["scale"], orig["rot"], orig["opacity"], orig["sh"])
    ps = params_from(simp["pos"], simp["scale"], simp["rot"], simp["opacity"], simp["sh"])
    for t in ps.values():
        t.requires_grad_(True)
    m = {k: torch.zeros_like(t) for k, t in ps.items()}
    v = {k: torch.zeros_like(t) for k, t in ps.items()}
    losses, g_first = [], None
    for it in range(iters):
        Rv, eye = view_camera(center, radius, dirs[it])
        with torch.no_grad():
            target = render(po["pos"], torch.exp(po["log_scale"]), po["quat"], torch.sigmoid(po["logit"]), po["dc"],
                            Rv, eye)
        loss = loss_of(ps, target, Rv, eye)
        for t in ps.values():
            t.grad = None
        loss.backward()
        losses.append(float(loss.detach()))
        if g_first is None:
            g_first = {k: t.grad.detach().numpy().copy() for k, t in ps.items()}
        with torch.no_grad():
            step = it + 1
            for k, t in ps.items():
                g = t.grad
                m[k] = 0.9 * m[k] + 0.1 * g
                v[k] = 0.999 * v[k] + 0.001 * g * g
                mh = m[k] / (1 - 0.9 ** step)
                vh = v[k] / (1 - 0.999 ** step)
                t -= LR[k] * mh / (torch.sqrt(vh) + 1e-15)
    with torch.no_grad():
        sh = np.asarray(simp["sh"], np.float64).reshape(len(simp["opacity"]), -1, 3).copy()
        sh[:, 0, :] = ps["dc"].numpy()
        q = ps["quat"].numpy()
        out = dict(pos=ps["pos"].numpy().copy(), scale=np.exp(ps["log_scale"].numpy()),
                   rot=q / np.linalg.norm(q, axis=1, keepdims=True),
                   opacity=1.0 / (1.0 + np.exp(-ps["logit"].numpy())), sh=sh)
    return out, losses, g_first
