"""Small hand-built inputs shared by the tests (no method arithmetic here)."""
from __future__ import annotations

import math

import numpy as np

import scenegen as sg


def single_cluster_asset(pos, scale, rot, opacity, sh, sh_degree=0) -> sg.Asset:
    """One leaf cluster that is also the root: always selected."""
    pos = np.asarray(pos, np.float32).reshape(-1, 3)
    n = pos.shape[0]
    assert 1 <= n <= 64
    nc = (sh_degree + 1) ** 2
    return sg.Asset(
        sh_degree=sh_degree,
        pos=pos,
        scale=np.asarray(scale, np.float32).reshape(n, 3),
        rot=np.asarray(rot, np.float32).reshape(n, 4),
        opacity=np.asarray(opacity, np.float32).reshape(n),
        sh=np.asarray(sh, np.float32).reshape(n, nc, 3),
        first_row=np.array([0], np.uint32), count=np.array([n], np.uint8), level=np.array([0], np.uint8),
        parent=np.array([-1], np.int32), first_child=np.array([-1], np.int32), n_children=np.array([0], np.uint8),
        self_sphere=np.array([[0, 0, 0, 0]], np.float32),
        parent_sphere=np.array([[0, 0, 0, np.inf]], np.float32),
        n_leaf_clusters=1,
    )


def two_level_asset(root_sphere, n_leaves=4) -> sg.Asset:
    """A root (own sphere given) over n_leaves single-row leaf clusters."""
    nl = n_leaves
    rows = nl + 1
    pos = np.zeros((rows, 3), np.float32)
    pos[:, 2] = np.linspace(-0.1, 0.1, rows)
    rs = np.asarray(root_sphere, np.float32)
    self_sphere = np.zeros((nl + 1, 4), np.float32)
    self_sphere[:nl, :3] = pos[:nl]
    self_sphere[nl] = rs
    parent_sphere = np.zeros_like(self_sphere)
    parent_sphere[:nl] = rs
    parent_sphere[nl, :3] = rs[:3]
    parent_sphere[nl, 3] = np.inf
    return sg.Asset(
        sh_degree=0, pos=pos, scale=np.full((rows, 3), 0.01, np.float32),
        rot=np.tile(np.array([1, 0, 0, 0], np.float32), (rows, 1)), opacity=np.full(rows, 0.5, np.float32),
        sh=np.zeros((rows, 1, 3), np.float32),
        first_row=np.arange(nl + 1, dtype=np.uint32), count=np.ones(nl + 1, np.uint8),
        level=np.array([0] * nl + [1], np.uint8),
        parent=np.array([nl] * nl + [-1], np.int32), first_child=np.array([-1] * nl + [0], np.int32),
        n_children=np.array([0] * nl + [nl], np.uint8),
        self_sphere=self_sphere, parent_sphere=parent_sphere, n_leaf_clusters=nl,
    )


def identity_camera(width=64, height=64, f=100.0, cx=None, cy=None, near=0.01, far=1e10, bg=(0.0, 0.0, 0.0)):
    v = np.hstack([np.eye(3), np.zeros((3, 1))]).astype(np.float32)
    return sg.Camera(width, height, float(f), float(f), float(width / 2 if cx is None else cx),
                     float(height / 2 if cy is None else cy), v, near, far, bg)


def leaf_mask(asset) -> np.ndarray:
    m = np.zeros(asset.n_clusters, np.uint8)
    m[: asset.n_leaf_clusters] = 1
    return m


def chains_ok(asset, mask_row) -> bool:
    """Exactly one selected cluster on every leaf-to-root chain."""
    for leaf in range(asset.n_leaf_clusters):
        k, n = leaf, 0
        while k >= 0:
            n += int(mask_row[k])
            k = int(asset.parent[k])
        if n != 1:
            return False
    return True


def random_camera_near(rng, width=64, height=48, dist=(0.05, 30.0)):
    az = rng.uniform(0, 2 * math.pi)
    el = rng.uniform(-1.2, 1.2)
    d = math.exp(rng.uniform(math.log(dist[0]), math.log(dist[1])))
    eye = d * np.array([math.cos(el) * math.cos(az), math.cos(el) * math.sin(az), math.sin(el)])
    tgt = rng.uniform(-0.3, 0.3, 3)
    return sg.look_at(eye, tgt, width, height, rng.uniform(0.3, 1.5))


def flat_asset(pos, scale, rot, opacity, sh, sh_degree=0) -> sg.Asset:
    """Leaf clusters of up to 64 rows under one root (fan-out <= 255)."""
    pos = np.asarray(pos, np.float32).reshape(-1, 3)
    n = pos.shape[0]
    nl = (n + 63) // 64
    assert 1 <= nl <= 255
    nc = (sh_degree + 1) ** 2
    first = np.arange(nl, dtype=np.uint32) * 64
    count = np.minimum(64, n - first).astype(np.uint8)
    p64 = pos.astype(np.float64)
    c = p64.mean(axis=0)
    r = float(np.linalg.norm(p64 - c, axis=1).max()) * 1.01 + 1e-3
    # the root's rows: the first min(64, n) Gaussians again (never selected at tau = 0)
    rows = np.concatenate([np.arange(n), np.arange(min(64, n))])
    self_sphere = np.zeros((nl + 1, 4), np.float32)
    self_sphere[:nl, :3] = p64[first].astype(np.float32)
    self_sphere[nl, :3] = c
    self_sphere[nl, 3] = r
    parent_sphere = np.repeat(self_sphere[nl:nl + 1], nl + 1, axis=0)
    parent_sphere[nl, 3] = np.inf
    return sg.Asset(
        sh_degree=sh_degree, pos=pos[rows], scale=np.asarray(scale, np.float32).reshape(n, 3)[rows],
        rot=np.asarray(rot, np.float32).reshape(n, 4)[rows], opacity=np.asarray(opacity, np.float32).reshape(n)[rows],
        sh=np.asarray(sh, np.float32).reshape(n, nc, 3)[rows],
        first_row=np.append(first, n).astype(np.uint32), count=np.append(count, min(64, n)).astype(np.uint8),
        level=np.array([0] * nl + [1], np.uint8), parent=np.array([nl] * nl + [-1], np.int32),
        first_child=np.array([-1] * nl + [0], np.int32), n_children=np.array([0] * nl + [nl], np.uint8),
        self_sphere=self_sphere, parent_sphere=parent_sphere, n_leaf_clusters=nl,
    )


def stacked_splats(n, seed, opacity_range, spread=0.15, depth=(1.0, 4.0), log_scale=-4.0):
    """n Gaussians stacked in front of the camera over a few tiles."""
    rng = np.random.default_rng(seed)
    z = rng.uniform(depth[0], depth[1], n)
    xy = rng.normal(0.0, spread, (n, 2)) * z[:, None] * 0.1
    pos = np.concatenate([xy, z[:, None]], axis=1)
    scale = np.exp(rng.normal(log_scale, 0.4, (n, 3)))
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    q[q[:, 0] < 0] *= -1
    o = rng.uniform(opacity_range[0], opacity_range[1], n)
    sh = rng.normal(0.0, 0.3, (n, 1, 3))
    return flat_asset(pos, scale, q, o, sh)


def round_fp16(x) -> np.ndarray:
    """FP32 values rounded to binary16 (numpy casts round to nearest even), as FP32."""
    return np.asarray(x, np.float32).astype(np.float16).astype(np.float32)


def round_bf16(x) -> np.ndarray:
    """FP32 values rounded to bfloat16 (8 significant bits, ties to even) by
    FP64 arithmetic: x = m 2^e with m in [0.5, 1), step 2^(e - 8)."""
    x = np.asarray(x, np.float32).astype(np.float64)
    _, e = np.frexp(x)
    step = np.ldexp(1.0, np.maximum(e, -125) - 8)
    return (np.rint(x / step) * step).astype(np.float32)


def quantized_asset(asset, precision: str):
    """The asset with scale, rotation and opacity in FP16 and SH in BF16
    ("fp16_bf16sh") or FP16 ("fp16"), widened back to FP32."""
    import dataclasses
    if precision == "fp32":
        return asset
    sh = round_bf16(asset.sh) if precision == "fp16_bf16sh" else round_fp16(asset.sh)
    return dataclasses.replace(asset, scale=round_fp16(asset.scale), rot=round_fp16(asset.rot),
                               opacity=round_fp16(asset.opacity), sh=sh)


def bundle_asset(b: dict, sh_degree: int) -> sg.Asset:
    """A bundle (offline-build arrays) as a scene-generator Asset."""
    return sg.Asset(sh_degree=sh_degree, pos=b["pos"], scale=b["scale"], rot=b["rot"], opacity=b["opacity"],
                    sh=b["sh"].reshape(len(b["pos"]), (sh_degree + 1) ** 2, 3), first_row=b["first_row"],
                    count=b["count"], level=b["level"], parent=b["parent"], first_child=b["first_child"],
                    n_children=b["n_children"], self_sphere=b["self_sphere"], parent_sphere=b["parent_sphere"],
                    n_leaf_clusters=int(b["n_leaf_clusters"]))


def blend_chunk_sizes(server: bool = False) -> tuple[int, int]:
    """(first, later) chunk sizes in keys of the long-list blending of scene
    renders (server=False) or of the serving loop, as the library's plan
    header defines them: later chunks of 2^shift keys, a first chunk of three."""
    import os
    import re
    h = open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "..", "paper_2505_06523_amd", "csrc",
                          "blend_plan.h")).read()
    name = "kChunkShiftServer" if server else "kChunkShiftRender"
    shift = int(re.search(r"constexpr uint32_t %s = (\d+);" % name, h).group(1))
    return 3 << shift, 1 << shift
