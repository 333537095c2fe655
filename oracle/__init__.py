"""CPU oracle for the V3DG per-frame path (ctypes binding of ``v3dg_oracle.c``).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg may import this package.  It shares no code
with the HIP library: the C source here restates the paper's definitions on
its own (selection: paper Sec. 3.3-3.4; splatting and compositing: Sec. 2.1
with the Sec. 5.1 settings).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "v3dg_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2 -ffp-contract=off -fopenmp, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
               "-Wall", "-Wno-unused-function", _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class OrcAsset(C.Structure):
    _fields_ = [("n_clusters", C.c_uint32), ("n_rows", C.c_uint32), ("sh_degree", C.c_uint32), ("pad0", C.c_uint32),
                ("self_sphere", C.c_void_p), ("parent_sphere", C.c_void_p), ("first_row", C.c_void_p),
                ("count", C.c_void_p), ("parent", C.c_void_p), ("first_child", C.c_void_p),
                ("n_children", C.c_void_p), ("pos", C.c_void_p), ("scale", C.c_void_p), ("rot", C.c_void_p),
                ("opacity", C.c_void_p), ("sh", C.c_void_p)]


class OrcCamera(C.Structure):
    _fields_ = [("width", C.c_uint32), ("height", C.c_uint32), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("V", C.c_float * 12), ("near_plane", C.c_float),
                ("far_plane", C.c_float), ("bg", C.c_float * 3), ("pad0", C.c_float)]


class OrcStats(C.Structure):
    _fields_ = [("n_slots", C.c_uint64), ("n_valid", C.c_uint64), ("n_ambiguous", C.c_uint64),
                ("n_pairs", C.c_uint64), ("n_hits", C.c_uint64)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        _lib = C.CDLL(_LIB_PATH)
        P = C.c_void_p
        _lib.orc_frame_setup.argtypes = [C.c_uint32, P, P, P, P, P, P]
        _lib.orc_frame_setup.restype = None
        _lib.orc_select_walk.argtypes = [P, C.c_uint32, P, P, C.c_float, P]
        _lib.orc_select_walk.restype = C.c_uint64
        _lib.orc_select_predicate.argtypes = [P, C.c_uint32, P, P, C.c_float, P]
        _lib.orc_select_predicate.restype = C.c_uint64
        _lib.orc_footprint.argtypes = [P, P, C.c_float, C.c_float, C.c_float]
        _lib.orc_footprint.restype = C.c_double
        _lib.orc_sh_basis.argtypes = [C.c_int, P, P]
        _lib.orc_sh_basis.restype = None
        _lib.orc_count_slots.argtypes = [P, C.c_uint64, P]
        _lib.orc_count_slots.restype = C.c_uint64
        _lib.orc_project.argtypes = [P, C.c_uint32, P, P, C.c_uint64, P, P, P, P, P, P, P, P]
        _lib.orc_project.restype = None
        _lib.orc_render.argtypes = [P, C.c_uint32, P, P, C.c_uint64, P, C.c_int, C.c_int, P, P, P]
        _lib.orc_render.restype = C.c_int
        _lib.orc_render_pixels.argtypes = [P, C.c_uint32, P, P, C.c_uint64, P, C.c_uint64, P, C.c_int, P, P, P]
        _lib.orc_render_pixels.restype = C.c_int
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class _Bound:
    """Keeps the numpy arrays referenced by an OrcAsset alive."""

    def __init__(self, asset):
        self.asset = asset  # holds the object so its id() cannot be reused while cached
        self.arrays = dict(
            self_sphere=np.ascontiguousarray(asset.self_sphere, np.float32),
            parent_sphere=np.ascontiguousarray(asset.parent_sphere, np.float32),
            first_row=np.ascontiguousarray(asset.first_row, np.uint32),
            count=np.ascontiguousarray(asset.count, np.uint8),
            parent=np.ascontiguousarray(asset.parent, np.int32),
            first_child=np.ascontiguousarray(asset.first_child, np.int32),
            n_children=np.ascontiguousarray(asset.n_children, np.uint8),
            pos=np.ascontiguousarray(asset.pos, np.float32),
            scale=np.ascontiguousarray(asset.scale, np.float32),
            rot=np.ascontiguousarray(asset.rot, np.float32),
            opacity=np.ascontiguousarray(asset.opacity, np.float32),
            sh=np.ascontiguousarray(asset.sh, np.float32),
        )
        s = OrcAsset()
        s.n_clusters = asset.first_row.shape[0]
        s.n_rows = asset.pos.shape[0]
        s.sh_degree = asset.sh_degree
        for k, v in self.arrays.items():
            setattr(s, k, v.ctypes.data)
        self.struct = s


_BOUND_CACHE: dict = {}


def _asset(asset) -> _Bound:
    key = id(asset)
    b = _BOUND_CACHE.get(key)
    if b is None or b.asset is not asset:
        b = _Bound(asset)
        _BOUND_CACHE.clear()
        _BOUND_CACHE[key] = b
    return b


def _camera(cam) -> OrcCamera:
    c = OrcCamera()
    c.width, c.height = int(cam.width), int(cam.height)
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    v = np.asarray(cam.world_to_cam, np.float32).reshape(12)
    for i in range(12):
        c.V[i] = float(v[i])
    c.near_plane, c.far_plane = float(cam.near), float(cam.far)
    for i in range(3):
        c.bg[i] = float(cam.bg[i])
    return c


def _inst(T) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(T, np.float64).reshape(-1, 12))


def frame_setup(T, cam):
    T = _inst(T)
    n = T.shape[0]
    A = np.zeros((n, 12), np.float32)
    s = np.zeros(n, np.float32)
    ch = np.zeros((n, 3), np.float64)
    K = np.zeros(1, np.float32)
    c = _camera(cam)
    lib().orc_frame_setup(n, _ptr(T), C.byref(c), _ptr(A), _ptr(s), _ptr(ch), _ptr(K))
    return A, s, ch, float(K[0])


def select_walk(asset, T, cam, tau: float) -> np.ndarray:
    """Selection mask (n_inst, n_clusters) from the recursive tree walk."""
    T = _inst(T)
    b = _asset(asset)
    mask = np.zeros((T.shape[0], asset.n_clusters), np.uint8)
    c = _camera(cam)
    lib().orc_select_walk(C.byref(b.struct), T.shape[0], _ptr(T), C.byref(c), float(tau), _ptr(mask))
    return mask


def select_predicate(asset, T, cam, tau: float) -> np.ndarray:
    T = _inst(T)
    b = _asset(asset)
    mask = np.zeros((T.shape[0], asset.n_clusters), np.uint8)
    c = _camera(cam)
    lib().orc_select_predicate(C.byref(b.struct), T.shape[0], _ptr(T), C.byref(c), float(tau), _ptr(mask))
    return mask


def mask_to_gids(mask: np.ndarray) -> np.ndarray:
    return np.flatnonzero(mask.reshape(-1)).astype(np.uint32)


def footprint(sphere, A_row2, s, fx, fy) -> float:
    sp = np.ascontiguousarray(sphere, np.float32)
    a2 = np.ascontiguousarray(A_row2, np.float32)
    return lib().orc_footprint(_ptr(sp), _ptr(a2), float(s), float(fx), float(fy))


def sh_basis(degree: int, d) -> np.ndarray:
    d = np.ascontiguousarray(d, np.float64)
    out = np.zeros((degree + 1) ** 2, np.float64)
    lib().orc_sh_basis(int(degree), _ptr(d), _ptr(out))
    return out


def project(asset, T, cam, gids):
    T = _inst(T)
    b = _asset(asset)
    g = np.ascontiguousarray(gids, np.uint32)
    n = int(lib().orc_count_slots(C.byref(b.struct), g.size, _ptr(g)))
    out = dict(valid=np.zeros(n, np.uint8), depth=np.zeros(n, np.float32), mean2=np.zeros((n, 2)),
               conic=np.zeros((n, 3)), rgb=np.zeros((n, 3)), opacity=np.zeros(n), cov2=np.zeros((n, 3)))
    c = _camera(cam)
    lib().orc_project(C.byref(b.struct), T.shape[0], _ptr(T), C.byref(c), g.size, _ptr(g),
                      _ptr(out["valid"]), _ptr(out["depth"]), _ptr(out["mean2"]), _ptr(out["conic"]),
                      _ptr(out["rgb"]), _ptr(out["opacity"]), _ptr(out["cov2"]))
    return out


def render(asset, T, cam, gids, use_index: bool = True, n_threads: int = 0):
    """FP64 image (H,W,4), ambiguous mask (H,W) and stats dict."""
    T = _inst(T)
    b = _asset(asset)
    g = np.ascontiguousarray(gids, np.uint32)
    img = np.zeros((cam.height, cam.width, 4), np.float64)
    amb = np.zeros((cam.height, cam.width), np.uint8)
    st = OrcStats()
    c = _camera(cam)
    lib().orc_render(C.byref(b.struct), T.shape[0], _ptr(T), C.byref(c), g.size, _ptr(g), int(bool(use_index)),
                     int(n_threads), _ptr(img), _ptr(amb), C.byref(st))
    return img, amb, dict(n_slots=st.n_slots, n_valid=st.n_valid, n_ambiguous=st.n_ambiguous, n_pairs=st.n_pairs,
                             n_hits=st.n_hits)


def render_pixels(asset, T, cam, gids, pix_xy, n_threads: int = 0):
    """FP64 RGBA at the listed pixel coordinates (N,2) -> (N,4), ambiguous (N,)."""
    T = _inst(T)
    b = _asset(asset)
    g = np.ascontiguousarray(gids, np.uint32)
    pix = np.ascontiguousarray(pix_xy, np.uint32).reshape(-1, 2)
    out = np.zeros((pix.shape[0], 4), np.float64)
    amb = np.zeros(pix.shape[0], np.uint8)
    st = OrcStats()
    c = _camera(cam)
    lib().orc_render_pixels(C.byref(b.struct), T.shape[0], _ptr(T), C.byref(c), g.size, _ptr(g), pix.shape[0],
                            _ptr(pix), int(n_threads), _ptr(out), _ptr(amb), C.byref(st))
    return out, amb, dict(n_slots=st.n_slots, n_valid=st.n_valid, n_ambiguous=st.n_ambiguous, n_pairs=st.n_pairs,
                             n_hits=st.n_hits)
