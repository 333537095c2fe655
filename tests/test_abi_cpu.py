"""The C ABI on the CPU: every declared symbol is exported, and the loader's
host-side validation rejects malformed inputs before touching the device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_2505_06523_amd as v
import scenegen as sg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "v3dg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(v3dg_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    names = _declared()
    assert len(names) >= 15
    L = v.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(v.EXPORTS)


def test_binding_struct_layouts_match_the_header(tmp_path):
    """Every structure the binding passes through the ABI has the size and the
    field offsets of its C declaration in include/v3dg.h (compiled with gcc),
    field for field by name."""
    import subprocess
    structs = [v.v3dg_camera, v.v3dg_hierarchy_desc, v.v3dg_frame_stats, v.v3dg_stream_stats, v.v3dg_profile,
               v.v3dg_server_config, v.v3dg_request_done, v.v3dg_server_stats]
    lines = ['#include "v3dg.h"', "#include <stddef.h>", "#include <stdio.h>", "int main(void)", "{"]
    for S in structs:
        n = S.__name__
        lines.append('    printf("%s %%zu\\n", sizeof(%s));' % (n, n))
        for f in S._fields_:
            lines.append('    printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (n, f[0], n, f[0]))
    lines += ["    return 0;", "}"]
    src, exe = tmp_path / "layout.c", tmp_path / "layout"
    src.write_text("\n".join(lines) + "\n")
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    got = dict(line.rsplit(" ", 1) for line in out.splitlines())
    for S in structs:
        assert int(got[S.__name__]) == C.sizeof(S), S.__name__
        for f in S._fields_:
            assert int(got[S.__name__ + "." + f[0]]) == getattr(S, f[0]).offset, (S.__name__, f[0])


def test_last_error_initially_empty():
    assert isinstance(v.last_error(), str)


@pytest.fixture
def small():
    return sg.make_asset(2048, 1, 4)


def _expect(asset, code, instances=None, flags=0, precision=0):
    with pytest.raises(v.V3DGError) as ei:
        v.Scene(asset, instances, stream=0, flags=flags, precision=precision)
    assert ei.value.code == code, str(ei.value)
    return str(ei.value)


def test_rejects_non_monotone(small):
    a = small
    root = a.n_clusters - 1
    a.self_sphere[root, 3] = np.float32(1e-3)
    a.parent_sphere[a.parent == root, 3] = np.float32(1e-3)
    msg = _expect(a, v.V3DG_ERR_NOT_MONOTONE)
    assert "nest" in msg


def test_rejects_parent_copy_mismatch(small):
    a = small
    k = a.n_leaf_clusters + 1
    a.parent_sphere[k, 0] += np.float32(1e-3)
    _expect(a, v.V3DG_ERR_INVALID_ARG)


def test_rejects_leaf_radius(small):
    a = small
    a.self_sphere[0, 3] = 0.01
    _expect(a, v.V3DG_ERR_INVALID_ARG)


def test_rejects_bad_quaternion(small):
    a = small
    a.rot[5] = [0.9, 0.0, 0.0, 0.0]
    _expect(a, v.V3DG_ERR_INVALID_ARG)


def test_rejects_nan_position(small):
    a = small
    a.pos[7, 1] = np.nan
    _expect(a, v.V3DG_ERR_INVALID_ARG)


def test_rejects_bad_opacity(small):
    a = small
    a.opacity[3] = 0.0
    _expect(a, v.V3DG_ERR_INVALID_ARG)


def test_rejects_bad_count_and_tree(small):
    a = small
    a.count[2] = 0
    _expect(a, v.V3DG_ERR_INVALID_ARG)
    b = sg.make_asset(2048, 1, 4)
    b.parent[3] = 5  # child no longer points back to its parent
    _expect(b, v.V3DG_ERR_INVALID_ARG)


def test_rejects_sheared_or_mirrored_instances(small):
    T = sg.identity_instances(1).copy()
    T[0, 0, 1] = 0.3
    _expect(small, v.V3DG_ERR_INVALID_ARG, T)
    M = sg.identity_instances(1).copy()
    M[0, 0, 0] = -1.0
    _expect(small, v.V3DG_ERR_INVALID_ARG, M)
    N = sg.identity_instances(1).copy()
    N[0, 1, 3] = np.inf
    _expect(small, v.V3DG_ERR_INVALID_ARG, N)


def test_rejects_unknown_precision(small):
    assert "precision" in _expect(small, v.V3DG_ERR_INVALID_ARG, precision=3)


@pytest.mark.parametrize("precision", [v.V3DG_FP16_BF16SH, v.V3DG_FP16])
def test_rejects_values_lost_in_narrow_storage(precision):
    a = sg.make_asset(2048, 1, 4)
    a.scale[5, 1] = np.float32(1e-9)  # below half the smallest FP16 subnormal: rounds to 0
    assert "FP16" in _expect(a, v.V3DG_ERR_INVALID_ARG, precision=precision)
    a = sg.make_asset(2048, 1, 4)
    a.scale[7, 0] = np.float32(7e4)  # beyond the FP16 maximum 65504
    assert "FP16" in _expect(a, v.V3DG_ERR_INVALID_ARG, precision=precision)
    a = sg.make_asset(2048, 1, 4)
    a.opacity[9] = np.float32(2e-8)
    assert "FP16" in _expect(a, v.V3DG_ERR_INVALID_ARG, precision=precision)


def test_sh_overflow_only_in_fp16():
    a = sg.make_asset(2048, 1, 4)
    a.sh[3, 1, 2] = np.float32(1e5)
    assert "overflows" in _expect(a, v.V3DG_ERR_INVALID_ARG, precision=v.V3DG_FP16)


def test_rejects_too_many_tests():
    a = sg.make_asset(64 * 64, 0, 1)  # 85 clusters
    T = np.tile(sg.identity_instances(1), (800000, 1, 1))  # 85 * 8e5 > 2^26
    _expect(a, v.V3DG_ERR_CAPACITY, T)


def test_null_arguments():
    L = v.lib()
    out = C.c_void_p()
    assert L.v3dg_load_hierarchy(None, None, 0, None, 0, C.byref(out)) == v.V3DG_ERR_INVALID_ARG
    assert L.v3dg_select(None, None, C.c_float(1.0), None) == v.V3DG_ERR_INVALID_ARG
    assert L.v3dg_render(None, None, None, None) == v.V3DG_ERR_INVALID_ARG
    assert L.v3dg_sort_pairs(None, None, 10, 0, None) == v.V3DG_ERR_INVALID_ARG
    assert L.v3dg_sort_pairs(None, None, 0, 8, None) == v.V3DG_OK
    L.v3dg_selection_free(None)
    L.v3dg_scene_free(None)


def test_build_bundle_rejects_bad_arguments():
    L = v.lib()
    n = 16
    pos = np.zeros((n, 3), np.float32)
    scale = np.ones((n, 3), np.float32)
    rot = np.tile(np.array([1, 0, 0, 0], np.float32), (n, 1))
    op = np.ones(n, np.float32)
    sh = np.zeros((n, 4, 3), np.float32)
    p = lambda a: a.ctypes.data_as(C.c_void_p)
    h = C.c_void_p()
    args = [p(pos), p(scale), p(rot), p(op), p(sh)]
    assert L.v3dg_build_bundle(*args, n, 1, 64, 0, None, None) == v.V3DG_ERR_INVALID_ARG
    assert L.v3dg_build_bundle(*args, 0, 1, 64, 0, None, C.byref(h)) == v.V3DG_ERR_INVALID_ARG
    assert L.v3dg_build_bundle(*args, n, 4, 64, 0, None, C.byref(h)) == v.V3DG_ERR_INVALID_ARG
    assert L.v3dg_build_bundle(*args, n, 1, 1, 0, None, C.byref(h)) == v.V3DG_ERR_INVALID_ARG
    assert L.v3dg_build_bundle(*args, n, 1, 65, 0, None, C.byref(h)) == v.V3DG_ERR_INVALID_ARG
    assert "cluster_size" in v.last_error()
    assert L.v3dg_build_bundle(None, *args[1:], n, 1, 64, 0, None, C.byref(h)) == v.V3DG_ERR_INVALID_ARG
    # fitting needs its view directions, finite and non-zero
    assert L.v3dg_build_bundle(*args, n, 1, 64, 3, None, C.byref(h)) == v.V3DG_ERR_INVALID_ARG
    dirs = np.array([[0, 0, 1], [0, 0, 0], [1, 0, 0]], np.float32)
    assert L.v3dg_build_bundle(*args, n, 1, 64, 3, p(dirs), C.byref(h)) == v.V3DG_ERR_INVALID_ARG
    assert "view_dirs" in v.last_error()
    dirs[1, 0] = np.nan
    assert L.v3dg_build_bundle(*args, n, 1, 64, 3, p(dirs), C.byref(h)) == v.V3DG_ERR_INVALID_ARG
    assert L.v3dg_build_bundle(*args, n, 1, 64, (1 << 20) + 1, p(dirs), C.byref(h)) == v.V3DG_ERR_INVALID_ARG
    assert not h.value
    assert L.v3dg_bundle_sizes(None, None, None, None, None) == v.V3DG_ERR_INVALID_ARG
    assert L.v3dg_bundle_copy(None, *([None] * 15)) == v.V3DG_ERR_INVALID_ARG
    assert L.v3dg_bundle_fit_loss(None, None) == v.V3DG_ERR_INVALID_ARG
    L.v3dg_bundle_free(None)


def test_streamed_load_rejects_bad_arguments():
    L = v.lib()
    h = C.c_void_p()
    d = v.v3dg_hierarchy_desc()
    assert L.v3dg_load_hierarchy_streamed(None, None, 1, None, 0, 8, C.byref(h)) == v.V3DG_ERR_INVALID_ARG
    assert L.v3dg_load_hierarchy_streamed(C.byref(d), None, 1, None, 0, 1 << 26, C.byref(h)) == v.V3DG_ERR_INVALID_ARG
    assert "pool_clusters" in v.last_error()
    assert not h.value
    assert L.v3dg_get_stream_stats(None, None) == v.V3DG_ERR_INVALID_ARG
