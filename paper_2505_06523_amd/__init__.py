"""Python binding of libv3dg (the V3DG per-frame path on MI355X).

The functions ``v3dg_*`` mirror the C ABI in ``include/v3dg.h`` one to one and
only marshal arguments; every step of the frame runs in the library's HIP
kernels.  ``Scene`` and ``Selection`` wrap the handles for convenience.
PyTorch supplies device memory (the image tensor) and the HIP stream.

The library must be built first (``python -m paper_2505_06523_amd.build``);
loading fails loudly when it is missing.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libv3dg.so")

V3DG_OK = 0
V3DG_ERR_INVALID_ARG = -1
V3DG_ERR_OOM = -2
V3DG_ERR_HIP = -3
V3DG_ERR_NOT_MONOTONE = -4
V3DG_ERR_CAPACITY = -5
V3DG_ERR_DEVICE = -6
V3DG_ERR_IO = -7
V3DG_PAGE_FILE_DIRECT = 1
V3DG_PAGE_FILE_KEEP = 2
V3DG_FP32 = 0
V3DG_FP16_BF16SH = 1
V3DG_FP16 = 2
PRECISIONS = {"fp32": V3DG_FP32, "fp16_bf16sh": V3DG_FP16_BF16SH, "fp16": V3DG_FP16}
V3DG_LOAD_REPAIR_NESTING = 1
V3DG_PROFILE_ALL = 0x7FF
V3DG_PROFILE_PAIR_AUDIT = 0x800
V3DG_PROFILE_PAIRS = 0x1000
V3DG_SORT_DEPTH_FIRST = 0
V3DG_SORT_KEYS64 = 1
STAGES = ["setup", "select", "expand", "project", "scan", "emit", "sort_hist", "sort_pass", "ranges", "blend",
          "depth_sort"]


class V3DGError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("v3dg error %d: %s" % (code, msg))
        self.code = code


class v3dg_camera(C.Structure):
    _fields_ = [("width", C.c_uint32), ("height", C.c_uint32), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("world_to_cam", C.c_float * 12),
                ("near_plane", C.c_float), ("far_plane", C.c_float), ("bg", C.c_float * 3), ("pad0", C.c_float)]


class v3dg_hierarchy_desc(C.Structure):
    _fields_ = [("n_clusters", C.c_uint32), ("n_rows", C.c_uint32), ("sh_degree", C.c_uint32),
                ("precision", C.c_uint32), ("self_sphere", C.c_void_p), ("parent_sphere", C.c_void_p),
                ("first_row", C.c_void_p), ("count", C.c_void_p), ("parent", C.c_void_p),
                ("first_child", C.c_void_p), ("n_children", C.c_void_p), ("pos", C.c_void_p),
                ("scale", C.c_void_p), ("rot", C.c_void_p), ("opacity", C.c_void_p), ("sh", C.c_void_p)]


class v3dg_frame_stats(C.Structure):
    _fields_ = [("n_slots", C.c_uint64), ("n_keys", C.c_uint64), ("n_tiles", C.c_uint32),
                ("key_bits", C.c_uint32), ("sort_passes", C.c_uint32), ("sort_mode", C.c_uint32),
                ("n_fp64_conics", C.c_uint32), ("n_conics_clamped", C.c_uint32), ("n_bins", C.c_uint32)]


class v3dg_stream_stats(C.Structure):
    _fields_ = [("frames", C.c_uint64), ("pages_in", C.c_uint64), ("bytes_in", C.c_uint64),
                ("evictions", C.c_uint64), ("last_pages_in", C.c_uint64), ("last_resident_used", C.c_uint32),
                ("pool_clusters", C.c_uint32), ("resident", C.c_uint32), ("tier", C.c_uint32),
                ("file_reads", C.c_uint64)]


class v3dg_profile(C.Structure):
    _fields_ = [("ms", C.c_double * 11), ("launches", C.c_uint64 * 11), ("frames", C.c_uint64),
                ("selects", C.c_uint64), ("tests", C.c_uint64), ("sel_clusters", C.c_uint64),
                ("slots", C.c_uint64), ("visible", C.c_uint64), ("keys", C.c_uint64), ("tiles", C.c_uint64),
                ("pixels", C.c_uint64), ("sort_passes", C.c_uint64), ("depth_sorts", C.c_uint64),
                ("pairs", C.c_uint64), ("pairs_taken", C.c_uint64)]


class v3dg_server_config(C.Structure):
    _fields_ = [("n_contexts", C.c_uint32), ("max_batch", C.c_uint32), ("hbm_budget_bytes", C.c_uint64),
                ("use_graphs", C.c_uint32), ("keys_per_pixel", C.c_uint32), ("cull", C.c_uint32),
                ("chunk_keys", C.c_uint32)]


class v3dg_request_done(C.Structure):
    _fields_ = [("ticket", C.c_uint64), ("status", C.c_int32), ("retries", C.c_uint32), ("n_slots", C.c_uint64),
                ("n_keys", C.c_uint64), ("submit_ms", C.c_double), ("admit_ms", C.c_double),
                ("done_ms", C.c_double)]


class v3dg_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("completed", C.c_uint64), ("failed", C.c_uint64),
                ("retries", C.c_uint64), ("batches", C.c_uint64), ("batched_requests", C.c_uint64),
                ("graph_captures", C.c_uint64), ("graph_launches", C.c_uint64),
                ("workspace_bytes", C.c_uint64), ("peak_workspace_bytes", C.c_uint64),
                ("contexts_live", C.c_uint32), ("queued", C.c_uint32)]


EXPORTS = [
    "v3dg_load_hierarchy", "v3dg_load_hierarchy_streamed", "v3dg_load_hierarchy_streamed_file",
    "v3dg_get_stream_stats", "v3dg_set_instances", "v3dg_select", "v3dg_render", "v3dg_render_full",
    "v3dg_selection_info", "v3dg_selection_copy_ids", "v3dg_selection_copy_slots", "v3dg_selection_free",
    "v3dg_scene_free", "v3dg_get_frame_stats", "v3dg_copy_projection", "v3dg_copy_attributes", "v3dg_copy_sorted_keys",
    "v3dg_set_sort_mode", "v3dg_set_chunk_keys", "v3dg_set_culling", "v3dg_set_profiling", "v3dg_collect_profile", "v3dg_sort_pairs",
    "v3dg_sort_pairs_noalloc", "v3dg_last_error",
    "v3dg_server_create", "v3dg_server_submit", "v3dg_server_submit_full", "v3dg_server_poll", "v3dg_server_get_stats", "v3dg_server_free",
    "v3dg_build_bundle", "v3dg_bundle_sizes", "v3dg_bundle_copy", "v3dg_bundle_fit_loss", "v3dg_bundle_free", "v3dg_local_splat",
]

_lib = None


def lib():
    """Load libv3dg.so (raises when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libv3dg.so is not built: run `python -m paper_2505_06523_amd.build` (needs hipcc)")
    L = C.CDLL(LIB_PATH)
    P, U32, U64, I = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int
    sig = {
        "v3dg_load_hierarchy": ([P, P, U32, P, U32, P], I),
        "v3dg_load_hierarchy_streamed": ([P, P, U32, P, U32, U32, P], I),
        "v3dg_load_hierarchy_streamed_file": ([P, P, U32, P, U32, U32, C.c_char_p, U32, P], I),
        "v3dg_get_stream_stats": ([P, P], I),
        "v3dg_set_instances": ([P, P, U32], I),
        "v3dg_select": ([P, P, C.c_float, P], I),
        "v3dg_render": ([P, P, P, P], I),
        "v3dg_render_full": ([P, P, P], I),
        "v3dg_selection_info": ([P, P, P], I),
        "v3dg_selection_copy_ids": ([P, P, U64, P], I),
        "v3dg_selection_copy_slots": ([P, P, P, U64, P], I),
        "v3dg_selection_free": ([P], None),
        "v3dg_scene_free": ([P], None),
        "v3dg_get_frame_stats": ([P, P], I),
        "v3dg_copy_projection": ([P, P, P, P, P, P, P, U64, P], I),
        "v3dg_copy_attributes": ([P, U64, U64, P, P, P, P, P], I),
        "v3dg_copy_sorted_keys": ([P, P, P, U64, P], I),
        "v3dg_set_sort_mode": ([P, I], I),
        "v3dg_set_chunk_keys": ([P, U32], I),
        "v3dg_set_culling": ([P, I], I),
        "v3dg_set_profiling": ([P, I], I),
        "v3dg_collect_profile": ([P, P], I),
        "v3dg_sort_pairs": ([P, P, U64, U32, P], I),
        "v3dg_sort_pairs_noalloc": ([P, P, U64, U32, P], I),
        "v3dg_last_error": ([], C.c_char_p),
        "v3dg_server_create": ([P, U32, P, P], I),
        "v3dg_server_submit": ([P, U32, P, C.c_float, P, P], I),
        "v3dg_server_submit_full": ([P, U32, P, P, P], I),
        "v3dg_server_poll": ([P, I, P, U32, P], I),
        "v3dg_server_get_stats": ([P, P], I),
        "v3dg_server_free": ([P], None),
        "v3dg_build_bundle": ([P, P, P, P, P, U32, U32, U32, U32, P, P], I),
        "v3dg_bundle_fit_loss": ([P, P], I),
        "v3dg_bundle_sizes": ([P, P, P, P, P], I),
        "v3dg_bundle_copy": ([P] + [P] * 15, I),
        "v3dg_bundle_free": ([P], None),
        "v3dg_local_splat": ([U32] + [P] * 10 + [U32] + [P] * 5 + [U32, P, U32, P, P], I),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def last_error() -> str:
    return lib().v3dg_last_error().decode()


def _check(rc: int):
    if rc != 0:
        raise V3DGError(rc, last_error())


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


# ---- one-to-one wrappers of the C ABI ------------------------------------------
def v3dg_load_hierarchy(desc, instances_3x4, n_instances, hip_stream, flags, pool_clusters: int = 0,
                        page_file: str | None = None, file_flags: int = 0):
    out = C.c_void_p()
    if page_file is not None:
        _check(lib().v3dg_load_hierarchy_streamed_file(C.byref(desc), instances_3x4, n_instances, hip_stream, flags,
                                                       int(pool_clusters), os.fsencode(page_file), int(file_flags),
                                                       C.byref(out)))
    elif pool_clusters:
        _check(lib().v3dg_load_hierarchy_streamed(C.byref(desc), instances_3x4, n_instances, hip_stream, flags,
                                                  int(pool_clusters), C.byref(out)))
    else:
        _check(lib().v3dg_load_hierarchy(C.byref(desc), instances_3x4, n_instances, hip_stream, flags,
                                         C.byref(out)))
    return out


def v3dg_get_stream_stats(scene) -> dict:
    st = v3dg_stream_stats()
    _check(lib().v3dg_get_stream_stats(scene, C.byref(st)))
    return {k: getattr(st, k) for k, _ in st._fields_}


def v3dg_set_instances(scene, instances_3x4, n_instances):
    _check(lib().v3dg_set_instances(scene, instances_3x4, n_instances))


def v3dg_select(scene, cam, tolerance, sel=None):
    h = C.c_void_p(sel.value if isinstance(sel, C.c_void_p) else sel)
    _check(lib().v3dg_select(scene, C.byref(cam), float(tolerance), C.byref(h)))
    return h


def v3dg_render(scene, cam, sel, image_ptr):
    _check(lib().v3dg_render(scene, C.byref(cam), sel, image_ptr))


def v3dg_render_full(scene, cam, image_ptr):
    _check(lib().v3dg_render_full(scene, C.byref(cam), image_ptr))


def v3dg_selection_info(sel):
    nc, ng = C.c_uint64(), C.c_uint64()
    _check(lib().v3dg_selection_info(sel, C.byref(nc), C.byref(ng)))
    return nc.value, ng.value


def v3dg_selection_copy_ids(sel):
    nc, _ = v3dg_selection_info(sel)
    out = np.zeros(max(nc, 1), np.uint32)
    n = C.c_uint64()
    _check(lib().v3dg_selection_copy_ids(sel, _p(out), out.size, C.byref(n)))
    return out[: n.value]


def v3dg_selection_copy_slots(sel):
    _, ng = v3dg_selection_info(sel)
    rows = np.zeros(max(ng, 1), np.uint32)
    inst = np.zeros(max(ng, 1), np.uint32)
    n = C.c_uint64()
    _check(lib().v3dg_selection_copy_slots(sel, _p(rows), _p(inst), rows.size, C.byref(n)))
    return rows[: n.value], inst[: n.value]


def v3dg_selection_free(sel):
    lib().v3dg_selection_free(sel)


def v3dg_scene_free(scene):
    lib().v3dg_scene_free(scene)


def v3dg_get_frame_stats(scene) -> dict:
    st = v3dg_frame_stats()
    _check(lib().v3dg_get_frame_stats(scene, C.byref(st)))
    return dict(n_slots=st.n_slots, n_keys=st.n_keys, n_tiles=st.n_tiles, key_bits=st.key_bits,
                sort_passes=st.sort_passes, sort_mode=st.sort_mode, n_fp64_conics=st.n_fp64_conics,
                n_conics_clamped=st.n_conics_clamped, n_bins=st.n_bins)


def v3dg_copy_projection(scene, n_slots: int) -> dict:
    n = max(int(n_slots), 1)
    out = dict(mean2=np.zeros((n, 2), np.float32), conic=np.zeros((n, 3), np.float32),
               rgb=np.zeros((n, 3), np.float32), opacity=np.zeros(n, np.float32), depth=np.zeros(n, np.float32),
               tiles=np.zeros(n, np.uint32))
    got = C.c_uint64()
    _check(lib().v3dg_copy_projection(scene, _p(out["mean2"]), _p(out["conic"]), _p(out["rgb"]),
                                      _p(out["opacity"]), _p(out["depth"]), _p(out["tiles"]), n, C.byref(got)))
    return {k: v[: got.value] for k, v in out.items()}


def v3dg_copy_attributes(scene, first: int, n: int, sh_degree: int) -> dict:
    m = max(int(n), 1)
    nc = (int(sh_degree) + 1) ** 2
    out = dict(pos=np.zeros((m, 3), np.float32), scale=np.zeros((m, 3), np.float32), rot=np.zeros((m, 4), np.float32),
               opacity=np.zeros(m, np.float32), sh=np.zeros((m, nc, 3), np.float32))
    _check(lib().v3dg_copy_attributes(scene, int(first), int(n), _p(out["pos"]), _p(out["scale"]), _p(out["rot"]),
                                      _p(out["opacity"]), _p(out["sh"])))
    return {k: v[: int(n)] for k, v in out.items()}


def v3dg_copy_sorted_keys(scene, n_keys: int):
    n = max(int(n_keys), 1)
    keys = np.zeros(n, np.uint64)
    vals = np.zeros(n, np.uint32)
    got = C.c_uint64()
    _check(lib().v3dg_copy_sorted_keys(scene, _p(keys), _p(vals), n, C.byref(got)))
    return keys[: got.value], vals[: got.value]


def v3dg_set_sort_mode(scene, mode: int):
    _check(lib().v3dg_set_sort_mode(scene, int(mode)))


def v3dg_set_chunk_keys(scene, keys: int):
    _check(lib().v3dg_set_chunk_keys(scene, int(keys)))


def v3dg_set_culling(scene, on: bool):
    _check(lib().v3dg_set_culling(scene, int(bool(on))))


def v3dg_set_profiling(scene, stage_mask: int):
    _check(lib().v3dg_set_profiling(scene, int(stage_mask)))


def v3dg_collect_profile(scene) -> dict:
    p = v3dg_profile()
    _check(lib().v3dg_collect_profile(scene, C.byref(p)))
    out = {name: getattr(p, name) for name, _ in v3dg_profile._fields_ if name not in ("ms", "launches")}
    out["stages"] = {s: (float(p.ms[i]), int(p.launches[i])) for i, s in enumerate(STAGES)}
    return out


def v3dg_sort_pairs(keys_ptr, vals_ptr, n, key_bits, hip_stream):
    _check(lib().v3dg_sort_pairs(keys_ptr, vals_ptr, int(n), int(key_bits), hip_stream))


V3DG_SORT_NOALLOC_MAX = 1 << 20


def v3dg_sort_pairs_noalloc(keys_ptr, vals_ptr, n, key_bits, hip_stream):
    _check(lib().v3dg_sort_pairs_noalloc(keys_ptr, vals_ptr, int(n), int(key_bits), hip_stream))


def v3dg_server_create(scene_handles, cfg: v3dg_server_config):
    arr = (C.c_void_p * len(scene_handles))(*[h.value for h in scene_handles])
    out = C.c_void_p()
    _check(lib().v3dg_server_create(arr, len(scene_handles), C.byref(cfg), C.byref(out)))
    return out


def v3dg_server_submit(srv, scene: int, cam: v3dg_camera, tau: float, image_ptr) -> int:
    t = C.c_uint64()
    _check(lib().v3dg_server_submit(srv, int(scene), C.byref(cam), float(tau), image_ptr, C.byref(t)))
    return t.value


def v3dg_server_submit_full(srv, scene: int, cam: v3dg_camera, image_ptr) -> int:
    t = C.c_uint64()
    _check(lib().v3dg_server_submit_full(srv, int(scene), C.byref(cam), image_ptr, C.byref(t)))
    return t.value


def v3dg_server_poll(srv, wait: bool, cap: int = 256) -> list:
    arr = (v3dg_request_done * cap)()
    n = C.c_uint32()
    _check(lib().v3dg_server_poll(srv, int(bool(wait)), arr, cap, C.byref(n)))
    return [{name: getattr(arr[i], name) for name, _ in v3dg_request_done._fields_} for i in range(n.value)]


def v3dg_server_get_stats(srv) -> dict:
    st = v3dg_server_stats()
    _check(lib().v3dg_server_get_stats(srv, C.byref(st)))
    return {name: getattr(st, name) for name, _ in v3dg_server_stats._fields_}


def v3dg_server_free(srv):
    lib().v3dg_server_free(srv)


# ---- convenience layer -----------------------------------------------------------
def make_camera(cam) -> v3dg_camera:
    """v3dg_camera from any object with width, height, fx, fy, cx, cy,
    world_to_cam (3x4), near, far and bg attributes."""
    c = v3dg_camera()
    c.width, c.height = int(cam.width), int(cam.height)
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    v = np.asarray(cam.world_to_cam, np.float32).reshape(12)
    for i in range(12):
        c.world_to_cam[i] = float(v[i])
    c.near_plane, c.far_plane = float(cam.near), float(cam.far)
    bg = getattr(cam, "bg", (0.0, 0.0, 0.0))
    for i in range(3):
        c.bg[i] = float(bg[i])
    return c


def _torch():
    import torch
    return torch


def current_stream_ptr():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Selection:
    def __init__(self, scene: "Scene", handle: C.c_void_p):
        self.scene = scene
        self.handle = handle

    def info(self):
        return v3dg_selection_info(self.handle)

    def ids(self) -> np.ndarray:
        return v3dg_selection_copy_ids(self.handle)

    def slots(self):
        return v3dg_selection_copy_slots(self.handle)

    def free(self):
        if self.handle is not None and self.handle.value:
            v3dg_selection_free(self.handle)
        self.handle = None

    def __del__(self):
        try:
            if self.scene is not None and self.scene.handle is not None:
                self.free()
        except Exception:
            pass


class Scene:
    """An asset in HBM with its instance table.  ``precision`` is the
    attribute storage tier: V3DG_FP32, V3DG_FP16_BF16SH or V3DG_FP16 (or its
    name in PRECISIONS).  ``pool_clusters`` > 0 streams the rows from host
    memory through a pool of that many 64-row pages (v3dg_load_hierarchy_streamed);
    with ``page_file`` the page images live in that file on disk instead
    (v3dg_load_hierarchy_streamed_file, ``file_flags`` V3DG_PAGE_FILE_*)."""

    def __init__(self, asset, instances=None, stream=None, flags: int = 0, precision=V3DG_FP32,
                 pool_clusters: int = 0, page_file: str | None = None, file_flags: int = 0):
        arrays = dict(
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
        d = v3dg_hierarchy_desc()
        d.n_clusters = arrays["first_row"].shape[0]
        d.n_rows = arrays["pos"].shape[0]
        d.sh_degree = int(asset.sh_degree)
        d.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        self.precision = int(d.precision)
        self.sh_degree = int(asset.sh_degree)
        self.n_rows = int(d.n_rows)
        for k, v in arrays.items():
            setattr(d, k, v.ctypes.data)
        if instances is None:
            instances = np.hstack([np.eye(3), np.zeros((3, 1))])[None]
        T = np.ascontiguousarray(np.asarray(instances, np.float64).reshape(-1, 12))
        self.n_instances = T.shape[0]
        self.n_clusters = int(d.n_clusters)
        if stream is None:
            stream = current_stream_ptr()
        elif not isinstance(stream, C.c_void_p):
            stream = C.c_void_p(stream)
        self.stream = stream
        self.handle = None
        self.handle = v3dg_load_hierarchy(d, _p(T), T.shape[0], stream, flags, pool_clusters, page_file, file_flags)

    def set_instances(self, instances):
        T = np.ascontiguousarray(np.asarray(instances, np.float64).reshape(-1, 12))
        v3dg_set_instances(self.handle, _p(T), T.shape[0])

    def select(self, cam, tau: float, sel: Selection | None = None) -> Selection:
        c = make_camera(cam)
        h = v3dg_select(self.handle, c, tau, sel.handle if sel is not None else None)
        if sel is not None:
            return sel
        return Selection(self, h)

    def _image(self, cam, out):
        torch = _torch()
        if out is None:
            out = torch.empty((int(cam.height), int(cam.width), 4), dtype=torch.float32, device="cuda")
        if (not out.is_cuda or out.dtype != torch.float32 or not out.is_contiguous()
                or tuple(out.shape) != (int(cam.height), int(cam.width), 4)):
            raise ValueError("image must be a contiguous float32 CUDA tensor of shape (H, W, 4)")
        return out

    def render(self, cam, sel: Selection, out=None):
        out = self._image(cam, out)
        v3dg_render(self.handle, make_camera(cam), sel.handle, C.c_void_p(out.data_ptr()))
        return out

    def render_full(self, cam, out=None):
        out = self._image(cam, out)
        v3dg_render_full(self.handle, make_camera(cam), C.c_void_p(out.data_ptr()))
        return out

    def frame_stats(self) -> dict:
        return v3dg_get_frame_stats(self.handle)

    def stream_stats(self) -> dict:
        return v3dg_get_stream_stats(self.handle)

    def projection(self) -> dict:
        return v3dg_copy_projection(self.handle, self.frame_stats()["n_slots"])

    def attributes(self, first: int = 0, n: int | None = None) -> dict:
        """Stored rows widened to FP32 (what the projection reads)."""
        n = self.n_rows - first if n is None else n
        return v3dg_copy_attributes(self.handle, first, n, self.sh_degree)

    def sorted_keys(self):
        return v3dg_copy_sorted_keys(self.handle, self.frame_stats()["n_keys"])

    def set_sort_mode(self, mode: int):
        v3dg_set_sort_mode(self.handle, mode)

    def set_chunk_keys(self, keys: int):
        """Later-chunk size of long bin lists in later renders (1024, 2048 or 4096)."""
        v3dg_set_chunk_keys(self.handle, keys)

    def set_culling(self, on: bool = True):
        v3dg_set_culling(self.handle, on)

    def set_profiling(self, on=True, pairs: bool = False, audit_pairs: bool = False):
        """True / False, or an iterable of stage names to time; pairs counts
        the pairs blending walks (profile "pairs"), audit_pairs also those it
        takes ("pairs_taken")."""
        if on is True or on is False:
            mask = V3DG_PROFILE_ALL if on else 0
        else:
            mask = sum(1 << STAGES.index(s) for s in on)
        mask |= V3DG_PROFILE_PAIRS if pairs else 0
        mask |= V3DG_PROFILE_PAIR_AUDIT if audit_pairs else 0
        v3dg_set_profiling(self.handle, mask)

    def collect_profile(self) -> dict:
        return v3dg_collect_profile(self.handle)

    def close(self):
        if self.handle is not None and self.handle.value:
            v3dg_scene_free(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_bundle(pos, scale, rot, opacity, sh, cluster_size: int = 64, fit_iters: int = 0, view_dirs=None) -> dict:
    """Offline build on the GPU (v3dg_build_bundle) of n Gaussians given as
    host arrays, with fit_iters local-splatting views along view_dirs
    (fit_iters x 3) per group; returns the bundle arrays (rows, clusters, src
    and gen) and fit_loss ((n_layers - 1) x fit_iters)."""
    f32 = lambda a: np.ascontiguousarray(a, np.float32)
    pos, scale, rot, opacity, sh = f32(pos), f32(scale), f32(rot), f32(opacity), f32(sh)
    n = pos.shape[0]
    k = sh.reshape(n, -1).shape[1] // 3
    sh_degree = int(round(math.sqrt(k))) - 1
    ptr = lambda a: a.ctypes.data_as(C.c_void_p)
    dirs = None
    if fit_iters:
        dirs = f32(view_dirs).reshape(-1, 3)
        if len(dirs) < fit_iters:
            raise ValueError("view_dirs must hold fit_iters directions")
    h = C.c_void_p()
    _check(lib().v3dg_build_bundle(ptr(pos), ptr(scale), ptr(rot), ptr(opacity), ptr(sh), n, sh_degree,
                                   int(cluster_size), int(fit_iters), None if dirs is None else ptr(dirs),
                                   C.byref(h)))
    try:
        nc, nr, nl, ny = C.c_uint32(), C.c_uint32(), C.c_uint32(), C.c_uint32()
        _check(lib().v3dg_bundle_sizes(h, C.byref(nc), C.byref(nr), C.byref(nl), C.byref(ny)))
        Cn, R = nc.value, nr.value
        out = dict(pos=np.empty((R, 3), np.float32), scale=np.empty((R, 3), np.float32),
                   rot=np.empty((R, 4), np.float32), opacity=np.empty(R, np.float32),
                   sh=np.empty((R, k, 3), np.float32), self_sphere=np.empty((Cn, 4), np.float32),
                   parent_sphere=np.empty((Cn, 4), np.float32), first_row=np.empty(Cn, np.uint32),
                   count=np.empty(Cn, np.uint8), level=np.empty(Cn, np.uint8), parent=np.empty(Cn, np.int32),
                   first_child=np.empty(Cn, np.int32), n_children=np.empty(Cn, np.uint8),
                   src=np.empty(R, np.uint32), gen=np.empty(R, np.uint8))
        names = ["pos", "scale", "rot", "opacity", "sh", "self_sphere", "parent_sphere", "first_row", "count",
                 "level", "parent", "first_child", "n_children", "src", "gen"]
        _check(lib().v3dg_bundle_copy(h, *[ptr(out[x]) for x in names]))
        out["n_leaf_clusters"] = nl.value
        out["n_layers"] = ny.value
        out["fit_loss"] = np.zeros((max(ny.value - 1, 0), int(fit_iters)), np.float32)
        _check(lib().v3dg_bundle_fit_loss(h, ptr(out["fit_loss"])))
        return out
    finally:
        lib().v3dg_bundle_free(h)


def local_splat(groups, orig: dict, fit: dict, view_dirs, iters: int):
    """Local splatting on the GPU (v3dg_local_splat).  groups: list of
    (orig_first, orig_count, fit_first, fit_count, (cx, cy, cz, r)); orig /
    fit: dicts of host rows pos, scale, rot, opacity, dc.  Returns the fitted
    rows, losses (groups x iters) and the first view's gradients (rows x 14)."""
    f32 = lambda a: np.ascontiguousarray(a, np.float32)
    u32 = lambda a: np.ascontiguousarray(a, np.uint32)
    ptr = lambda a: a.ctypes.data_as(C.c_void_p)
    G = len(groups)
    of, oc, ff, fc = (u32([g[i] for g in groups]) for i in range(4))
    sph = f32([g[4] for g in groups]).reshape(G, 4)
    o = {k: f32(orig[k]) for k in ("pos", "scale", "rot", "opacity", "dc")}
    f = {k: f32(fit[k]).copy() for k in ("pos", "scale", "rot", "opacity", "dc")}
    dirs = f32(view_dirs).reshape(-1, 3)
    n_o, n_f = len(o["opacity"]), len(f["opacity"])
    losses = np.zeros((G, iters), np.float32)
    grads = np.zeros((n_f, 14), np.float32)
    _check(lib().v3dg_local_splat(G, ptr(of), ptr(oc), ptr(ff), ptr(fc), ptr(sph), ptr(o["pos"]), ptr(o["scale"]),
                                  ptr(o["rot"]), ptr(o["opacity"]), ptr(o["dc"]), n_o, ptr(f["pos"]),
                                  ptr(f["scale"]), ptr(f["rot"]), ptr(f["opacity"]), ptr(f["dc"]), n_f, ptr(dirs),
                                  int(iters), ptr(losses), ptr(grads)))
    return f, losses, grads


def sort_pairs(keys, vals, key_bits: int, stream=None):
    """Stable radix sort of device tensors (int64 keys as u64, int32 values) in place."""
    torch = _torch()
    if keys.dtype != torch.int64 or vals.dtype != torch.int32 or keys.numel() != vals.numel():
        raise ValueError("keys must be int64 and vals int32 of equal length")
    if not (keys.is_cuda and vals.is_cuda and keys.is_contiguous() and vals.is_contiguous()):
        raise ValueError("keys and vals must be contiguous CUDA tensors")
    st = current_stream_ptr() if stream is None else C.c_void_p(stream)
    v3dg_sort_pairs(C.c_void_p(keys.data_ptr()), C.c_void_p(vals.data_ptr()), keys.numel(), key_bits, st)


def sort_pairs_noalloc(keys, vals, key_bits: int, stream=None):
    """sort_pairs through the entry point that allocates nothing (at most
    V3DG_SORT_NOALLOC_MAX pairs)."""
    torch = _torch()
    if keys.dtype != torch.int64 or vals.dtype != torch.int32 or keys.numel() != vals.numel():
        raise ValueError("keys must be int64 and vals int32 of equal length")
    if not (keys.is_cuda and vals.is_cuda and keys.is_contiguous() and vals.is_contiguous()):
        raise ValueError("keys and vals must be contiguous CUDA tensors")
    st = current_stream_ptr() if stream is None else C.c_void_p(stream)
    v3dg_sort_pairs_noalloc(C.c_void_p(keys.data_ptr()), C.c_void_p(vals.data_ptr()), keys.numel(), key_bits, st)


class Server:
    """Continuous-batching renderer over resident scenes (see v3dg_server_*).

    submit() queues a request and keeps the output tensor alive until its
    completion record comes back from poll()."""

    def __init__(self, scenes, n_contexts: int = 8, max_batch: int = 16, hbm_budget_bytes: int = 64 << 30,
                 use_graphs: bool = True, keys_per_pixel: int = 0, cull: bool = False, chunk_keys: int = 0):
        cfg = v3dg_server_config()
        cfg.n_contexts, cfg.max_batch = int(n_contexts), int(max_batch)
        cfg.hbm_budget_bytes, cfg.use_graphs = int(hbm_budget_bytes), int(bool(use_graphs))
        cfg.keys_per_pixel = int(keys_per_pixel)
        cfg.cull = int(bool(cull))
        cfg.chunk_keys = int(chunk_keys)
        self.scenes = list(scenes)  # keeps the scenes alive while the server runs
        self.handle = None
        self.handle = v3dg_server_create([sc.handle for sc in self.scenes], cfg)
        self.outputs = {}

    def submit(self, scene: int, cam, tau: float, out=None, full: bool = False):
        """full: every leaf, no selection (tau is ignored)."""
        torch = _torch()
        if out is None:
            out = torch.empty((int(cam.height), int(cam.width), 4), dtype=torch.float32, device="cuda")
        if (not out.is_cuda or out.dtype != torch.float32 or not out.is_contiguous()
                or tuple(out.shape) != (int(cam.height), int(cam.width), 4)):
            raise ValueError("image must be a contiguous float32 CUDA tensor of shape (H, W, 4)")
        if full:
            t = v3dg_server_submit_full(self.handle, scene, make_camera(cam), C.c_void_p(out.data_ptr()))
        else:
            t = v3dg_server_submit(self.handle, scene, make_camera(cam), tau, C.c_void_p(out.data_ptr()))
        self.outputs[t] = out
        return t, out

    def poll(self, wait: bool = False) -> list:
        recs = v3dg_server_poll(self.handle, wait)
        for r in recs:
            r["image"] = self.outputs.pop(r["ticket"], None)
        return recs

    def drain(self) -> list:
        out = []
        while self.outputs:
            out.extend(self.poll(wait=True))
        return out

    def stats(self) -> dict:
        return v3dg_server_get_stats(self.handle)

    def close(self):
        if self.handle is not None and self.handle.value:
            v3dg_server_free(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
