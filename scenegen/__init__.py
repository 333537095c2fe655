"""Seeded synthetic inputs for the V3DG per-frame path.

This module builds the *inputs* of the online stage and nothing else:

* an asset of 3D Gaussians (position, scale, rotation quaternion, opacity,
  real-SH colour coefficients; the primitive of paper Sec. 2.1) sampled on
  random ellipsoid surfaces,
* a cluster hierarchy standing in for the offline build stage (paper Sec. 3.1,
  3.2 and Algorithm 1): leaves are runs of 64 Morton-ordered Gaussians, each
  parent merges up to four children by moment matching, and every cluster
  carries its own bounding sphere and a bit-identical copy of its parent's
  (paper Sec. 3.3 and 3.4),
* rigid instance layouts (paper Sec. 4.2 and Appendix A.2/A.3) and pinhole
  cameras (paper Sec. 5.1).

It holds none of the selection or rendering arithmetic: the HIP library and
the CPU oracle each implement that on their own, and both consume the arrays
made here.  All randomness comes from ``numpy.random.default_rng(seed)``.
"""
from __future__ import annotations

import hashlib
import math
import os
from dataclasses import dataclass, field

import numpy as np

CLUSTER_ROWS = 64
FANOUT = 4
NEST_REL = 2.0 ** -10
NEST_ABS = 1e-4


# --------------------------------------------------------------------------
# small helpers
# --------------------------------------------------------------------------
def _quat_to_mat(q: np.ndarray) -> np.ndarray:
    """Rotation matrices for unit quaternions q = (w, x, y, z), shape (..., 3, 3)."""
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    m = np.empty(q.shape[:-1] + (3, 3), dtype=np.float64)
    m[..., 0, 0] = 1 - 2 * (y * y + z * z)
    m[..., 0, 1] = 2 * (x * y - w * z)
    m[..., 0, 2] = 2 * (x * z + w * y)
    m[..., 1, 0] = 2 * (x * y + w * z)
    m[..., 1, 1] = 1 - 2 * (x * x + z * z)
    m[..., 1, 2] = 2 * (y * z - w * x)
    m[..., 2, 0] = 2 * (x * z - w * y)
    m[..., 2, 1] = 2 * (y * z + w * x)
    m[..., 2, 2] = 1 - 2 * (x * x + y * y)
    return m


def _mat_to_quat(m: np.ndarray) -> np.ndarray:
    """Unit quaternions (w >= 0) for proper rotation matrices, shape (..., 4).

    Uses the largest-diagonal branch selection so every branch divides by a
    quantity of at least 1/2.
    """
    m = np.asarray(m, dtype=np.float64)
    n = m.shape[:-2]
    m = m.reshape(-1, 3, 3)
    q = np.empty((m.shape[0], 4))
    tr = m[:, 0, 0] + m[:, 1, 1] + m[:, 2, 2]
    d = np.stack([tr, m[:, 0, 0], m[:, 1, 1], m[:, 2, 2]], axis=1)
    br = np.argmax(d, axis=1)
    # w largest
    s = br == 0
    t = np.sqrt(np.maximum(1.0 + tr[s], 1e-300)) * 2
    q[s, 0] = 0.25 * t
    q[s, 1] = (m[s, 2, 1] - m[s, 1, 2]) / t
    q[s, 2] = (m[s, 0, 2] - m[s, 2, 0]) / t
    q[s, 3] = (m[s, 1, 0] - m[s, 0, 1]) / t
    # x largest
    s = br == 1
    t = np.sqrt(np.maximum(1.0 + m[s, 0, 0] - m[s, 1, 1] - m[s, 2, 2], 1e-300)) * 2
    q[s, 0] = (m[s, 2, 1] - m[s, 1, 2]) / t
    q[s, 1] = 0.25 * t
    q[s, 2] = (m[s, 0, 1] + m[s, 1, 0]) / t
    q[s, 3] = (m[s, 0, 2] + m[s, 2, 0]) / t
    # y largest
    s = br == 2
    t = np.sqrt(np.maximum(1.0 + m[s, 1, 1] - m[s, 0, 0] - m[s, 2, 2], 1e-300)) * 2
    q[s, 0] = (m[s, 0, 2] - m[s, 2, 0]) / t
    q[s, 1] = (m[s, 0, 1] + m[s, 1, 0]) / t
    q[s, 2] = 0.25 * t
    q[s, 3] = (m[s, 1, 2] + m[s, 2, 1]) / t
    # z largest
    s = br == 3
    t = np.sqrt(np.maximum(1.0 + m[s, 2, 2] - m[s, 0, 0] - m[s, 1, 1], 1e-300)) * 2
    q[s, 0] = (m[s, 1, 0] - m[s, 0, 1]) / t
    q[s, 1] = (m[s, 0, 2] + m[s, 2, 0]) / t
    q[s, 2] = (m[s, 1, 2] + m[s, 2, 1]) / t
    q[s, 3] = 0.25 * t
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    q[q[:, 0] < 0] *= -1
    return q.reshape(n + (4,))


def _unit_quats(rng: np.random.Generator, n: int) -> np.ndarray:
    """Uniform random unit quaternions with w >= 0 (normalised 4D Gaussian)."""
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    q[q[:, 0] < 0] *= -1
    return q


def _spread_bits21(v: np.ndarray) -> np.ndarray:
    """Insert two zero bits between each of the low 21 bits of v (uint64)."""
    v = v.astype(np.uint64) & np.uint64(0x1FFFFF)
    v = (v | (v << np.uint64(32))) & np.uint64(0x1F00000000FFFF)
    v = (v | (v << np.uint64(16))) & np.uint64(0x1F0000FF0000FF)
    v = (v | (v << np.uint64(8))) & np.uint64(0x100F00F00F00F00F)
    v = (v | (v << np.uint64(4))) & np.uint64(0x10C30C30C30C30C3)
    v = (v | (v << np.uint64(2))) & np.uint64(0x1249249249249249)
    return v


def morton_order(pos: np.ndarray) -> np.ndarray:
    """Stable argsort of 63-bit Morton codes (21 bits per axis) over the AABB."""
    lo = pos.min(axis=0)
    hi = pos.max(axis=0)
    ext = np.where(hi > lo, hi - lo, 1.0)
    qv = np.floor((pos - lo) / ext * float((1 << 21) - 1)).astype(np.int64)
    qv = np.clip(qv, 0, (1 << 21) - 1).astype(np.uint64)
    code = (_spread_bits21(qv[:, 0]) << np.uint64(2)) | (_spread_bits21(qv[:, 1]) << np.uint64(1)) \
        | _spread_bits21(qv[:, 2])
    return np.argsort(code, kind="stable")


def round_up_f32(x: np.ndarray) -> np.ndarray:
    """Smallest float32 >= x (elementwise, x finite float64)."""
    f = x.astype(np.float32)
    low = f.astype(np.float64) < x
    f[low] = np.nextafter(f[low], np.float32(np.inf))
    return f


# --------------------------------------------------------------------------
# the asset
# --------------------------------------------------------------------------
@dataclass
class Asset:
    """One asset: Gaussian rows (SoA) plus its cluster hierarchy.

    Row layout is cluster-major: leaf clusters first (Morton order), then each
    coarser level; a cluster's rows are ``first_row[k] .. first_row[k]+count[k]``.
    Cluster IDs are level-major: leaves first, the single root last.
    """
    sh_degree: int
    pos: np.ndarray          # (R,3) f32
    scale: np.ndarray        # (R,3) f32, linear
    rot: np.ndarray          # (R,4) f32, unit (w,x,y,z), w >= 0
    opacity: np.ndarray      # (R,)  f32, activated
    sh: np.ndarray           # (R, (d+1)^2, 3) f32
    first_row: np.ndarray    # (C,) u32
    count: np.ndarray        # (C,) u8, <= 64
    level: np.ndarray        # (C,) u8
    parent: np.ndarray       # (C,) i32, -1 for the root
    first_child: np.ndarray  # (C,) i32, -1 for leaves
    n_children: np.ndarray   # (C,) u8
    self_sphere: np.ndarray  # (C,4) f32 (cx,cy,cz,r); r = 0 for leaves
    parent_sphere: np.ndarray  # (C,4) f32; r = +inf for the root
    n_leaf_clusters: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def n_clusters(self) -> int:
        return int(self.first_row.shape[0])

    @property
    def n_rows(self) -> int:
        return int(self.pos.shape[0])

    @property
    def n_leaf_rows(self) -> int:
        k = self.n_leaf_clusters
        return int(self.first_row[k - 1]) + int(self.count[k - 1])

    def digest(self) -> str:
        h = hashlib.sha256()
        for a in (self.pos, self.scale, self.rot, self.opacity, self.sh, self.first_row, self.count,
                  self.parent, self.first_child, self.n_children, self.self_sphere, self.parent_sphere):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()


def _sample_leaves(rng, n_leaves, n_ellipsoids, sh_degree):
    n_coef = (sh_degree + 1) ** 2
    per = np.full(n_ellipsoids, n_leaves // n_ellipsoids)
    per[: n_leaves % n_ellipsoids] += 1
    pts = []
    for e in range(n_ellipsoids):
        a = rng.uniform(0.08, 0.25, 3)
        rm = _quat_to_mat(_unit_quats(rng, 1))[0]
        half = np.sqrt(((rm * a[None, :]) ** 2).sum(axis=1))  # rotated AABB half-extent
        c = rng.uniform(-0.5 + half, 0.5 - half)
        u = rng.standard_normal((per[e], 3))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        pts.append(c[None, :] + (u * a[None, :]) @ rm.T)
    pos = np.concatenate(pts, axis=0)
    scale = np.exp(rng.normal(-4.5, 0.5, (n_leaves, 3)))
    rot = _unit_quats(rng, n_leaves)
    opacity = 1.0 / (1.0 + np.exp(-rng.standard_normal(n_leaves)))
    sh = np.empty((n_leaves, n_coef, 3))
    sh[:, 0, :] = rng.normal(0.0, 0.3, (n_leaves, 3))
    if n_coef > 1:
        sh[:, 1:, :] = rng.normal(0.0, 0.05, (n_leaves, n_coef - 1, 3))
    return pos, scale, rot, opacity, sh


def _merge_groups(starts, pos, scale, rot, opacity, sh):
    """Moment-matching merge of contiguous row groups beginning at ``starts``.

    Weights w = o*sx*sy*sz; mean and covariance (including the spread of the
    means) are w-weighted; the merged covariance is factored by eigh in FP64.
    Opacity and SH are w-weighted means.  This stands in for the paper's
    local-splatting simplification (Sec. 3.2), which is not part of the
    online path.
    """
    w = opacity * scale[:, 0] * scale[:, 1] * scale[:, 2]
    wsum = np.add.reduceat(w, starts)
    mu = np.add.reduceat(w[:, None] * pos, starts) / wsum[:, None]
    gid = np.repeat(np.arange(len(starts)), np.diff(np.append(starts, len(w))))
    d = pos - mu[gid]
    rm = _quat_to_mat(rot)
    cov = np.einsum("nij,nj,nkj->nik", rm, scale * scale, rm)
    cov = cov + d[:, :, None] * d[:, None, :]
    csum = np.add.reduceat(w[:, None, None] * cov, starts) / wsum[:, None, None]
    lam, vec = np.linalg.eigh(csum)
    det = np.linalg.det(vec)
    vec[det < 0, :, 0] *= -1
    s_new = np.sqrt(np.maximum(lam, 1e-12))
    q_new = _mat_to_quat(vec)
    o_new = np.add.reduceat(w * opacity, starts) / wsum
    sh_new = np.add.reduceat(w[:, None, None] * sh, starts) / wsum[:, None, None]
    return mu, s_new, q_new, o_new, sh_new


def make_asset(n_leaves: int, sh_degree: int, seed: int, n_ellipsoids: int = 4,
               cluster_rows: int = CLUSTER_ROWS, fanout: int = FANOUT) -> Asset:
    """Build a seeded asset of ``n_leaves`` Gaussians and its hierarchy."""
    if n_leaves < 1 or cluster_rows < 1 or cluster_rows > 64 or fanout < 2:
        raise ValueError("bad generator parameters")
    rng = np.random.default_rng(seed)
    pos, scale, rot, opacity, sh = _sample_leaves(rng, n_leaves, n_ellipsoids, sh_degree)
    order = morton_order(pos)
    pos, scale, rot, opacity, sh = pos[order], scale[order], rot[order], opacity[order], sh[order]
    # round leaf attributes to their stored precision before anything is derived from them
    pos = pos.astype(np.float32).astype(np.float64)
    scale = scale.astype(np.float32).astype(np.float64)
    rot = rot.astype(np.float32).astype(np.float64)
    opacity = opacity.astype(np.float32).astype(np.float64)
    sh = sh.astype(np.float32).astype(np.float64)

    # ---- levels: per level, cluster row ranges (relative to the level's rows)
    lvl_rows = [(pos, scale, rot, opacity, sh)]
    n0 = (n_leaves + cluster_rows - 1) // cluster_rows
    lvl_first = [np.arange(n0, dtype=np.int64) * cluster_rows]
    lvl_count = [np.minimum(cluster_rows, n_leaves - lvl_first[0])]
    lvl_children = [None]  # per level >= 1: (first child index within previous level, n children)
    while len(lvl_first[-1]) > 1:
        nprev = len(lvl_first[-1])
        npar = (nprev + fanout - 1) // fanout
        fc = np.arange(npar, dtype=np.int64) * fanout
        nc = np.minimum(fanout, nprev - fc)
        prev_first, prev_count = lvl_first[-1], lvl_count[-1]
        # rows of parent j = concatenation of its children's rows, merged 4 at a time
        child_row_start = prev_first[fc]
        child_row_end = prev_first[fc + nc - 1] + prev_count[fc + nc - 1]
        child_rows = child_row_end - child_row_start
        par_count = (child_rows + 3) // 4
        starts = []
        for j in range(npar):
            starts.append(child_row_start[j] + 4 * np.arange(par_count[j]))
        starts = np.concatenate(starts)
        p, s, q, o, c = lvl_rows[-1]
        merged = _merge_groups(starts, p, s, q, o, c)
        merged = tuple(m.astype(np.float32).astype(np.float64) for m in merged)
        # keep quaternions unit-norm after rounding
        lvl_rows.append(merged)
        par_first = np.concatenate([[0], np.cumsum(par_count)[:-1]]).astype(np.int64)
        lvl_first.append(par_first)
        lvl_count.append(par_count)
        lvl_children.append((fc, nc))

    # ---- flatten into level-major cluster IDs and rows
    n_levels = len(lvl_first)
    cl_base = np.concatenate([[0], np.cumsum([len(f) for f in lvl_first])]).astype(np.int64)
    row_base = np.concatenate([[0], np.cumsum([len(r[0]) for r in lvl_rows])]).astype(np.int64)
    n_clusters = int(cl_base[-1])
    first_row = np.concatenate([lvl_first[i] + row_base[i] for i in range(n_levels)]).astype(np.uint32)
    count = np.concatenate(lvl_count).astype(np.uint8)
    level = np.concatenate([np.full(len(lvl_first[i]), i) for i in range(n_levels)]).astype(np.uint8)
    parent = np.full(n_clusters, -1, dtype=np.int32)
    first_child = np.full(n_clusters, -1, dtype=np.int32)
    n_children = np.zeros(n_clusters, dtype=np.uint8)
    for i in range(1, n_levels):
        fc, nc = lvl_children[i]
        ids = cl_base[i] + np.arange(len(fc))
        first_child[ids] = (cl_base[i - 1] + fc).astype(np.int32)
        n_children[ids] = nc.astype(np.uint8)
        for c in range(int(nc.max())):
            m = nc > c
            parent[cl_base[i - 1] + fc[m] + c] = ids[m].astype(np.int32)
    allp = np.concatenate([r[0] for r in lvl_rows])
    alls = np.concatenate([r[1] for r in lvl_rows])
    allq = np.concatenate([r[2] for r in lvl_rows])
    allq /= np.linalg.norm(allq, axis=1, keepdims=True)
    allo = np.concatenate([r[3] for r in lvl_rows])
    allsh = np.concatenate([r[4] for r in lvl_rows])
    pos32 = allp.astype(np.float32)

    # ---- spheres (paper Sec. 3.3): own sphere of a non-leaf cluster is the
    # mean / max-distance sphere of its children's Gaussian positions; leaves
    # have r = 0.  Nesting (parent contains child with slack) is enforced
    # bottom-up so that a parent that fits implies each child fits.
    sphere_c = np.zeros((n_clusters, 3))
    sphere_r = np.zeros(n_clusters)
    p64 = pos32.astype(np.float64)
    # leaves: centre of own rows (not used by selection, since r = 0)
    lf = first_row[: cl_base[1]].astype(np.int64)
    lc = count[: cl_base[1]].astype(np.int64)
    sphere_c[: cl_base[1]] = np.add.reduceat(p64[: int(lf[-1] + lc[-1])], lf) / lc[:, None]
    for i in range(1, n_levels):
        ids = np.arange(cl_base[i], cl_base[i + 1])
        fc = first_child[ids].astype(np.int64)
        nc = n_children[ids].astype(np.int64)
        rs = first_row[fc].astype(np.int64)
        re = first_row[fc + nc - 1].astype(np.int64) + count[fc + nc - 1].astype(np.int64)
        seg = np.concatenate([np.arange(a, b) for a, b in zip(rs, re)])
        seg_starts = np.concatenate([[0], np.cumsum(re - rs)[:-1]])
        cen = np.add.reduceat(p64[seg], seg_starts) / (re - rs)[:, None]
        cen32 = cen.astype(np.float32).astype(np.float64)
        gid = np.repeat(np.arange(len(ids)), re - rs)
        dist = np.linalg.norm(p64[seg] - cen32[gid], axis=1)
        r = np.maximum.reduceat(dist, seg_starts)
        if i >= 2:  # nest around non-leaf children
            for c in range(int(nc.max())):
                m = nc > c
                ch = fc[m] + c
                need = (np.linalg.norm(cen32[m] - sphere_c[ch], axis=1) + sphere_r[ch]) * (1 + NEST_REL) + NEST_ABS
                r[m] = np.maximum(r[m], need)
        sphere_c[ids] = cen32
        sphere_r[ids] = round_up_f32(r).astype(np.float64)
    self_sphere = np.concatenate([sphere_c, sphere_r[:, None]], axis=1).astype(np.float32)
    self_sphere[: cl_base[1], 3] = 0.0
    parent_sphere = np.empty_like(self_sphere)
    has_p = parent >= 0
    parent_sphere[has_p] = self_sphere[parent[has_p]]
    parent_sphere[~has_p, :3] = self_sphere[~has_p, :3]
    parent_sphere[~has_p, 3] = np.inf

    return Asset(
        sh_degree=sh_degree,
        pos=pos32,
        scale=alls.astype(np.float32),
        rot=allq.astype(np.float32),
        opacity=allo.astype(np.float32),
        sh=allsh.astype(np.float32),
        first_row=first_row, count=count, level=level, parent=parent,
        first_child=first_child, n_children=n_children,
        self_sphere=self_sphere, parent_sphere=parent_sphere,
        n_leaf_clusters=int(cl_base[1]),
        meta=dict(n_leaves=n_leaves, seed=seed, n_ellipsoids=n_ellipsoids, levels=n_levels),
    )


_ASSET_CACHE: dict = {}


def cached_asset(n_leaves: int, sh_degree: int, seed: int, n_ellipsoids: int = 4) -> Asset:
    """make_asset with an in-process cache and an optional on-disk cache.

    The disk cache lives under ``$V3DG_ASSET_CACHE`` when that is set.
    """
    key = (n_leaves, sh_degree, seed, n_ellipsoids)
    if key in _ASSET_CACHE:
        return _ASSET_CACHE[key]
    cdir = os.environ.get("V3DG_ASSET_CACHE")
    path = None
    if cdir:
        os.makedirs(cdir, exist_ok=True)
        path = os.path.join(cdir, "asset_%d_%d_%d_%d.npz" % key)
        if os.path.exists(path):
            with np.load(path, allow_pickle=False) as z:
                a = Asset(sh_degree=sh_degree, n_leaf_clusters=int(z["n_leaf_clusters"]),
                          **{f: z[f] for f in _ARRAY_FIELDS})
            _ASSET_CACHE[key] = a
            return a
    a = make_asset(n_leaves, sh_degree, seed, n_ellipsoids)
    if path:
        np.savez(path + ".tmp.npz", n_leaf_clusters=a.n_leaf_clusters, **{f: getattr(a, f) for f in _ARRAY_FIELDS})
        os.replace(path + ".tmp.npz", path)
    _ASSET_CACHE[key] = a
    return a


_ARRAY_FIELDS = ("pos", "scale", "rot", "opacity", "sh", "first_row", "count", "level", "parent",
                 "first_child", "n_children", "self_sphere", "parent_sphere")


# --------------------------------------------------------------------------
# cameras and instances
# --------------------------------------------------------------------------
@dataclass
class Camera:
    """Pinhole camera, OpenCV axes (x right, y down, z forward)."""
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    world_to_cam: np.ndarray  # (3,4) float32
    near: float = 0.01
    far: float = 1e10
    bg: tuple = (0.0, 0.0, 0.0)

    def centre(self) -> np.ndarray:
        v = self.world_to_cam.astype(np.float64)
        return -v[:, :3].T @ v[:, 3]


def look_at(eye, target, width, height, fov_x, up=(0.0, 0.0, 1.0), near=0.01, far=1e10) -> Camera:
    eye = np.asarray(eye, dtype=np.float64)
    f = np.asarray(target, dtype=np.float64) - eye
    f /= np.linalg.norm(f)
    right = np.cross(f, np.asarray(up, dtype=np.float64))
    if np.linalg.norm(right) < 1e-9:
        right = np.cross(f, np.array([0.0, 1.0, 0.0]))
    right /= np.linalg.norm(right)
    down = np.cross(f, right)
    rm = np.stack([right, down, f])
    v = np.concatenate([rm, (-rm @ eye)[:, None]], axis=1)
    fx = (width / 2.0) / math.tan(fov_x / 2.0)
    return Camera(width, height, fx, fx, width / 2.0, height / 2.0, v.astype(np.float32), near, far)


def orbit_cameras(n: int, seed: int, width: int = 1920, height: int = 1080, fov_x: float = math.pi / 4,
                  dist_range=(0.5, 20.0), elevations_deg=(15, 30, 45, 60, 75)):
    """Cameras on orbits around the origin: azimuth U[0,2pi), elevation from a
    fixed set (paper Sec. 5.2 protocol), distance log-uniform in ``dist_range``."""
    rng = np.random.default_rng(seed)
    cams = []
    for _ in range(n):
        az = rng.uniform(0.0, 2 * math.pi)
        el = math.radians(float(rng.choice(np.asarray(elevations_deg))))
        d = math.exp(rng.uniform(math.log(dist_range[0]), math.log(dist_range[1])))
        eye = d * np.array([math.cos(el) * math.cos(az), math.cos(el) * math.sin(az), math.sin(el)])
        cams.append(look_at(eye, (0.0, 0.0, 0.0), width, height, fov_x))
    return cams


def tangent_path_cameras(n: int = 100, radius: float = 0.45, height: float = 0.05, width: int = 1920,
                         heig: int = 1080, fov_x: float = math.pi / 3):
    """A close walk through an asset: n cameras on a horizontal circle of
    ``radius`` around the origin at ``height``, each looking along the circle
    (counter-clockwise), so that every view holds only a part of the asset."""
    cams = []
    for i in range(n):
        th = 2 * math.pi * i / n
        eye = (radius * math.cos(th), radius * math.sin(th), height)
        tgt = (eye[0] - math.sin(th), eye[1] + math.cos(th), height)
        cams.append(look_at(eye, tgt, width, heig, fov_x))
    return cams


def single_camera_c1(seed: int = 101) -> Camera:
    """The small case: 256x256, fov 60 deg, distance 2, elevation 30 deg, seeded azimuth."""
    rng = np.random.default_rng(seed)
    az = rng.uniform(0.0, 2 * math.pi)
    el = math.radians(30.0)
    eye = 2.0 * np.array([math.cos(el) * math.cos(az), math.cos(el) * math.sin(az), math.sin(el)])
    return look_at(eye, (0.0, 0.0, 0.0), 256, 256, math.radians(60.0))


def grid_instances(n_side: int = 10, spacing: float = 1.5, jitter: float = 0.2, seed: int = 3) -> np.ndarray:
    """Rigid instance transforms (N,3,4) float64 on an n_side x n_side grid with
    xy jitter and random yaw (paper Appendix A.2 places assets on a plane with
    2D rotations)."""
    rng = np.random.default_rng(seed)
    out = []
    off = (n_side - 1) * spacing / 2.0
    for iy in range(n_side):
        for ix in range(n_side):
            yaw = rng.uniform(0, 2 * math.pi)
            c, s = math.cos(yaw), math.sin(yaw)
            t = np.array([ix * spacing - off + rng.uniform(-jitter, jitter),
                          iy * spacing - off + rng.uniform(-jitter, jitter), 0.0])
            out.append(np.array([[c, -s, 0, t[0]], [s, c, 0, t[1]], [0, 0, 1, t[2]]]))
    return np.stack(out)


def identity_instances(n: int = 1) -> np.ndarray:
    return np.tile(np.hstack([np.eye(3), np.zeros((3, 1))])[None], (n, 1, 1))


def _catmull_rom(p0, p1, p2, p3, t):
    t2, t3 = t * t, t * t * t
    return 0.5 * ((2 * p1) + (-p0 + p2) * t + (2 * p0 - 5 * p1 + 4 * p2 - p3) * t2 + (-p0 + 3 * p1 - 3 * p2 + p3) * t3)


def flythrough_cameras(n_frames: int = 300, seed: int = 103, width: int = 1920, height: int = 1080,
                       fov_x: float = math.pi / 4, extent: float = 7.5, n_ctrl: int = 6):
    """A Catmull-Rom fly-through over a grid scene: control points at height
    0.5-3, looking along the tangent pitched 15 degrees down."""
    rng = np.random.default_rng(seed)
    ctrl = np.stack([rng.uniform(-extent, extent, n_ctrl), rng.uniform(-extent, extent, n_ctrl),
                     rng.uniform(0.5, 3.0, n_ctrl)], axis=1)
    pts = np.concatenate([ctrl[:1], ctrl, ctrl[-1:]], axis=0)
    cams = []
    nseg = n_ctrl - 1
    for f in range(n_frames):
        u = f / max(1, n_frames - 1) * nseg
        i = min(int(u), nseg - 1)
        t = u - i
        p = _catmull_rom(pts[i], pts[i + 1], pts[i + 2], pts[i + 3], t)
        pn = _catmull_rom(pts[i], pts[i + 1], pts[i + 2], pts[i + 3], min(1.0, t + 1e-3))
        if t + 1e-3 > 1.0:
            pp = _catmull_rom(pts[i], pts[i + 1], pts[i + 2], pts[i + 3], t - 1e-3)
            d = p - pp
        else:
            d = pn - p
        d[2] = 0.0
        nd = np.linalg.norm(d)
        d = d / nd if nd > 1e-12 else np.array([1.0, 0.0, 0.0])
        pitch = math.radians(15.0)
        fwd = np.array([d[0] * math.cos(pitch), d[1] * math.cos(pitch), -math.sin(pitch)])
        cams.append(look_at(p, p + fwd, width, height, fov_x))
    return cams


# ---- serving workload -------------------------------------------------------------
SERVING_LEAVES_M = (1, 2, 4, 6, 8, 12, 16, 20)
SERVING_RESOLUTIONS = ((1280, 720), (1920, 1080), (3840, 2160))
SERVING_TOLERANCES = (1.0, 4.0)


def compose_copies(asset: Asset, T: np.ndarray) -> Asset:
    """One asset made of rigid copies of ``asset``: copy c takes the rows
    ``[c R, (c+1) R)`` and the clusters ``[c C, (c+1) C)`` (copy-major, each with
    its own root), positions, rotations and sphere centres moved by
    ``T[c] = [Rot | t]``.  The rows are physically distinct; scales, opacity and
    SH coefficients are copied as they are (view-dependent colour is not
    rotated with the copy)."""
    T = np.asarray(T, np.float64).reshape(-1, 3, 4)
    n, R, C = T.shape[0], asset.n_rows, asset.n_clusters
    rot_m, t = T[:, :, :3], T[:, :, 3]
    pos = (np.einsum("cij,rj->cri", rot_m, asset.pos.astype(np.float64)) + t[:, None, :]).astype(np.float32)
    qr = _mat_to_quat(rot_m)  # (n, 4) w, x, y, z
    q = asset.rot.astype(np.float64)
    w1, x1, y1, z1 = (qr[:, None, i] for i in range(4))
    w2, x2, y2, z2 = (q[None, :, i] for i in range(4))
    qq = np.stack([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                   w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2], axis=-1)
    qq /= np.linalg.norm(qq, axis=-1, keepdims=True)
    qq[qq[..., 0] < 0] *= -1
    sph = asset.self_sphere.astype(np.float64)
    centres = (np.einsum("cij,kj->cki", rot_m, sph[:, :3]) + t[:, None, :]).astype(np.float32)
    self_sphere = np.concatenate([centres, np.broadcast_to(asset.self_sphere[None, :, 3:], (n, C, 1))], axis=2)
    self_sphere = self_sphere.reshape(-1, 4).astype(np.float32)
    off_c = (np.arange(n, dtype=np.int64) * C)[:, None]
    parent = np.where(asset.parent[None, :] >= 0, asset.parent[None, :] + off_c, -1).astype(np.int32).reshape(-1)
    first_child = np.where(asset.first_child[None, :] >= 0, asset.first_child[None, :] + off_c,
                           -1).astype(np.int32).reshape(-1)
    parent_sphere = np.empty_like(self_sphere)
    inner = parent >= 0
    parent_sphere[inner] = self_sphere[parent[inner]]          # bit-identical copies of the parents' own spheres
    parent_sphere[~inner, :3] = self_sphere[~inner, :3]
    parent_sphere[~inner, 3] = np.inf
    first_row = (asset.first_row[None, :].astype(np.int64) + (np.arange(n, dtype=np.int64) * R)[:, None])
    assert first_row.max() + 64 < (1 << 32)
    return Asset(
        sh_degree=asset.sh_degree, pos=pos.reshape(-1, 3), scale=np.tile(asset.scale, (n, 1)),
        rot=qq.astype(np.float32).reshape(-1, 4), opacity=np.tile(asset.opacity, n),
        sh=np.tile(asset.sh, (n, 1, 1)), first_row=first_row.astype(np.uint32).reshape(-1),
        count=np.tile(asset.count, n), level=np.tile(asset.level, n), parent=parent, first_child=first_child,
        n_children=np.tile(asset.n_children, n), self_sphere=self_sphere, parent_sphere=parent_sphere,
        n_leaf_clusters=asset.n_leaf_clusters * n, meta=dict(asset.meta, copies=n))


def serving_scenes(seed: int = 500, base_leaves: int = 1 << 18):
    """Eight scenes of {1, 2, 4, 6, 8, 12, 16, 20}M leaves.  Scene j is one
    asset of L / base_leaves rigid copies (on a grid with jitter and yaw) of its
    own SH3 base asset with 2 + j ellipsoids, so that every scene's rows are
    distinct and resident.  Yields (asset, identity instance, grid extent), one
    scene at a time, so that a caller can free each after loading it."""
    for j, m in enumerate(SERVING_LEAVES_M):
        n_copies = m * (1 << 20) // base_leaves
        base = cached_asset(base_leaves, 3, seed + j, n_ellipsoids=2 + j)
        side = int(math.ceil(math.sqrt(n_copies)))
        T = grid_instances(side, 1.5, 0.2, seed + 100 + j)[:n_copies]
        yield compose_copies(base, T), identity_instances(1), side * 1.5


def serving_requests(n: int, rate: float, extents, seed: int):
    """n camera requests with Poisson arrivals at `rate` per second (rate 0:
    all at t = 0): scene uniform, resolution uniform over 720p / 1080p / 2160p,
    tolerance uniform over {1, 4}, camera on an orbit around the scene's grid
    (distance log-uniform in [0.35, 2] x extent, elevation 15-75 deg, fov_x pi/4)."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n)) if rate > 0 else np.zeros(n)
    reqs = []
    for i in range(n):
        j = int(rng.integers(0, len(extents)))
        w, h = SERVING_RESOLUTIONS[int(rng.integers(0, len(SERVING_RESOLUTIONS)))]
        tau = SERVING_TOLERANCES[int(rng.integers(0, len(SERVING_TOLERANCES)))]
        L = extents[j]
        d = L * math.exp(rng.uniform(math.log(0.35), math.log(2.0)))
        az = rng.uniform(0.0, 2 * math.pi)
        el = math.radians(float(rng.choice([15, 30, 45, 60, 75])))
        eye = d * np.array([math.cos(el) * math.cos(az), math.cos(el) * math.sin(az), math.sin(el)])
        reqs.append(dict(t=float(t[i]), scene=j, cam=look_at(eye, (0.0, 0.0, 0.0), w, h, math.pi / 4), tau=tau))
    return reqs
