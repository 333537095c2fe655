"""CPU oracle of the offline build (paper Sec. 3.1-3.2, Algorithm 1).

TEST INFRASTRUCTURE ONLY: only ``tests/`` and the benchmark's baseline leg may
import it.  It shares no code with the HIP library.

The paper builds a bundle of clusters from an asset's N Gaussians: a binary
median split cuts them into clusters of n Gaussians (layer C_0); then, while
a layer has at least two clusters, the same split groups its clusters into
cluster groups of n_{C in CG} = 2, every group is simplified to half its
Gaussians (those with the larger product of scale and opacity, scales grown by
2^(1/6)) and the simplified Gaussians form the clusters of the next layer.  A
group's bounding sphere (centre: mean Gaussian position; radius: farthest
Gaussian) becomes the own sphere of the simplified cluster and the parent
sphere of the group's clusters.  Optionally (iters > 0) the simplified
Gaussians of every group are then refined by local splatting (Sec. 3.2, the
local-splatting oracle) against the group's Gaussians, with the same view
directions for every group; the views face the group centre from four times
the group's reach, the farthest 3-sigma extent of its Gaussians.
Every layer is made from the current rows of the layer below (positions for
means and spheres, scales and opacities for the scores).

Where the paper leaves a choice open, this file fixes it (the readings are
listed with the design notes):

* Split of a set larger than n: the axis of the largest FP32 bounding-box
  extent (max - min; the first such axis on ties), the set stably ordered by
  that coordinate (-0 and +0 equal), the first ceil(s/2) items to the left.
  Splitting proceeds layer by layer until no set exceeds n.
* Cluster position for grouping: the FP64 mean of its Gaussians' positions,
  summed in row order, rounded to FP32.
* Simplify: score = ((sx * sy) * sz) * opacity in FP32 with the current
  scales; the ceil(m/2) largest scores are kept (ties: the earlier Gaussian
  in the group), in group order; their scales are multiplied by
  float32(2^(1/6)).
* Group sphere: centre = FP64 mean (row order) rounded to FP32; radius =
  the largest FP64 distance from that FP32 centre, rounded up to FP32; then
  grown, for every child cluster, to (|c_p - c_c| + r_c)(1 + 2^-10) rounded
  up, so that spheres nest (the loader's requirement).  Leaves: centre = the
  cluster's mean, radius 0.  The root's parent sphere has radius +inf.
* Ids are layer-major; within a layer, the clusters are in the order of the
  grouping split, so that every group's clusters are consecutive.  Rows follow
  the cluster ids.
"""
from __future__ import annotations

import math

import numpy as np

SCALE_GROWTH = np.float32(2.0 ** (1.0 / 6.0))
NEST_SLACK = 1.0 + 2.0 ** -10


def round_up32(x: float) -> np.float32:
    """Smallest float32 >= x (x finite, non-negative)."""
    f = np.float32(x)
    if float(f) < x:
        f = np.nextafter(f, np.float32(np.inf))
    return f


def split(points: np.ndarray, items: np.ndarray, n: int) -> list:
    """Algorithm 1's Split: binary median split of ``items`` (indices into
    ``points``, in their current order) into sets of at most n, left to right."""
    sets = [np.asarray(items, dtype=np.int64)]
    while any(len(s) > n for s in sets):
        nxt = []
        for s in sets:
            if len(s) <= n:
                nxt.append(s)
                continue
            p = points[s]
            ext = p.max(axis=0) - p.min(axis=0)  # float32
            axis = int(np.argmax(ext))
            key = p[:, axis] + np.float32(0.0)
            o = np.argsort(key, kind="stable")
            s = s[o]
            h = (len(s) + 1) // 2
            nxt.append(s[:h])
            nxt.append(s[h:])
        sets = nxt
    return sets


def seq_mean64(p: np.ndarray) -> np.ndarray:
    """FP64 mean of the rows of p (float32), summed in row order."""
    return np.cumsum(p.astype(np.float64), axis=0)[-1] / float(len(p))


FIELDS = ("pos", "scale", "rot", "opacity", "sh", "src", "gen")


def take(rows: dict, idx) -> dict:
    return {k: v[idx].copy() for k, v in rows.items()}


def concat(parts: list) -> dict:
    return {k: np.concatenate([p[k] for p in parts]) for k in FIELDS}


def simplify(rows: dict) -> dict:
    """Keep the ceil(m/2) Gaussians with the largest scale product x opacity
    (FP32, ties: the earlier one), in group order, scales grown by 2^(1/6)."""
    m = len(rows["src"])
    s = rows["scale"]
    score = ((s[:, 0] * s[:, 1]) * s[:, 2]) * rows["opacity"]
    order = np.argsort(-score.astype(np.float64), kind="stable")  # descending, ties: earlier first
    keep = np.sort(order[:(m + 1) // 2])
    out = take(rows, keep)
    out["scale"] = out["scale"] * SCALE_GROWTH
    out["gen"] = out["gen"] + 1
    return out


def group_sphere(p, child_sph):
    """Centre, radius of a group of Gaussians at positions p (FP32); grown
    to hold the child spheres."""
    p = np.asarray(p, np.float32)
    c32 = seq_mean64(p).astype(np.float32)
    c = c32.astype(np.float64)
    r = 0.0
    for q in p.astype(np.float64):
        d = q - c
        r = max(r, math.sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]))
    r = float(round_up32(r))
    for ch in child_sph:
        d = ch[:3].astype(np.float64) - c
        need = (math.sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]) + float(ch[3])) * NEST_SLACK
        r = max(r, float(round_up32(need)))
    return np.array([c32[0], c32[1], c32[2], np.float32(r)], dtype=np.float32)


def view_sphere(rows: dict, sph: np.ndarray) -> np.ndarray:
    """Sphere framing a group's pseudo-views: the group centre and the
    farthest 3-sigma reach |p - c| + 3 max(sx, sy, sz) of its Gaussians (FP64,
    rounded up to FP32), so that the views hold the Gaussians' extents."""
    c = sph[:3].astype(np.float64)
    r = 0.0
    for q, s in zip(rows["pos"].astype(np.float64), rows["scale"]):
        d = q - c
        r = max(r, math.sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]) + 3.0 * float(s.max()))
    return np.array([sph[0], sph[1], sph[2], round_up32(r)], np.float32)


def fit(orig: dict, simp: dict, sph: np.ndarray, dirs, iters: int) -> dict:
    """Local splatting of a group's simplified Gaussians; FP32 rows back."""
    from oracle import local_splat as ls
    out, _, _ = ls.local_splat(orig, simp, sph[:3].astype(np.float64), float(sph[3]),
                               np.asarray(dirs, np.float64), iters)
    res = dict(simp)
    for k in ("pos", "scale", "rot", "opacity", "sh"):
        res[k] = np.asarray(out[k], np.float64).astype(np.float32).reshape(simp[k].shape)
    return res


def build_bundle(pos, scale, rot, opacity, sh, n: int = 64, iters: int = 0, dirs=None) -> dict:
    """Algorithm 1 on N Gaussians (local splatting with iters views along
    dirs when iters > 0); returns the bundle arrays."""
    pos = np.ascontiguousarray(pos, np.float32)
    N = pos.shape[0]
    inp = dict(pos=pos, scale=np.asarray(scale, np.float32), rot=np.asarray(rot, np.float32),
               opacity=np.asarray(opacity, np.float32), sh=np.asarray(sh, np.float32).reshape(N, -1, 3),
               src=np.arange(N, dtype=np.int64), gen=np.zeros(N, np.int64))
    # layer C_0
    sets = split(pos, np.arange(N), n)
    cur = [take(inp, s) for s in sets]
    cur_sph = [np.concatenate([seq_mean64(c["pos"]).astype(np.float32), [np.float32(0)]]) for c in cur]
    cur_children = [None] * len(cur)
    layers = []
    while len(cur) >= 2:
        cent = np.array([seq_mean64(c["pos"]).astype(np.float32) for c in cur], dtype=np.float32)
        groups = split(cent, np.arange(len(cur)), 2)
        order = np.concatenate(groups)
        cur = [cur[k] for k in order]
        cur_sph = [cur_sph[k] for k in order]
        cur_children = [cur_children[k] for k in order]
        layers.append((cur, cur_sph, cur_children))
        nxt, nxt_sph, nxt_children = [], [], []
        first = 0
        for g in groups:
            members = list(range(first, first + len(g)))
            first += len(g)
            rows = concat([cur[m] for m in members])
            sph = group_sphere(rows["pos"], [cur_sph[m] for m in members])
            kept = simplify(rows)
            if iters:
                kept = fit(rows, kept, view_sphere(rows, sph), dirs, iters)
            nxt.append(kept)
            nxt_sph.append(sph)
            nxt_children.append((members[0], len(members)))
        cur, cur_sph, cur_children = nxt, nxt_sph, nxt_children
    layers.append((cur, cur_sph, cur_children))

    # ids, rows and links
    base = np.cumsum([0] + [len(l[0]) for l in layers])
    C = int(base[-1])
    first_row = np.zeros(C, np.uint32)
    count = np.zeros(C, np.uint8)
    level = np.zeros(C, np.uint8)
    parent = np.full(C, -1, np.int32)
    first_child = np.full(C, -1, np.int32)
    n_children = np.zeros(C, np.uint8)
    self_sphere = np.zeros((C, 4), np.float32)
    parts = []
    row = 0
    for li, (cl, sph, ch) in enumerate(layers):
        for k, rows in enumerate(cl):
            cid = int(base[li]) + k
            first_row[cid] = row
            count[cid] = len(rows["src"])
            level[cid] = li
            self_sphere[cid] = sph[k]
            if ch[k] is not None:
                first_child[cid] = int(base[li - 1]) + ch[k][0]
                n_children[cid] = ch[k][1]
                for m in range(ch[k][1]):
                    parent[int(base[li - 1]) + ch[k][0] + m] = cid
            parts.append(rows)
            row += len(rows["src"])
    allr = concat(parts)
    parent_sphere = np.zeros((C, 4), np.float32)
    for cid in range(C):
        if parent[cid] < 0:
            parent_sphere[cid] = np.array([self_sphere[cid, 0], self_sphere[cid, 1], self_sphere[cid, 2], np.inf],
                                          np.float32)
        else:
            parent_sphere[cid] = self_sphere[parent[cid]]
    sh_out = allr["sh"].reshape((len(allr["src"]),) + np.asarray(sh).shape[1:])
    return dict(pos=allr["pos"], scale=allr["scale"], rot=allr["rot"], opacity=allr["opacity"], sh=sh_out,
                first_row=first_row, count=count, level=level, parent=parent, first_child=first_child,
                n_children=n_children, self_sphere=self_sphere, parent_sphere=parent_sphere,
                n_leaf_clusters=int(base[1]), src=allr["src"].astype(np.int64), gen=allr["gen"].astype(np.int64))
