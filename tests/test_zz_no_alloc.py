"""The allocation-free sort (v3dg_sort_pairs_noalloc) through the C ABI.

For callers that cannot allocate: its result must equal v3dg_sort_pairs's
bit for bit (and numpy's stable sort), on consecutive calls that reuse the
GPU's fixed scratch array, the second with fewer pairs; sizes beyond its
maximum are refused with nothing sorted."""
import numpy as np
import pytest

import paper_2505_06523_amd as v

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a GPU"
    v.lib()
    return _t


def _pairs(n, bits, seed):
    rng = np.random.default_rng(seed)
    hi = np.uint64((1 << bits) - 1) if bits < 64 else np.uint64(0xFFFFFFFFFFFFFFFF)
    keys = (rng.integers(0, 1 << 62, n, dtype=np.uint64) * np.uint64(4) + rng.integers(0, 4, n, dtype=np.uint64)) & hi
    keys[: n // 4] = keys[n // 4]  # duplicates: stability matters
    return keys, np.arange(n, dtype=np.uint32)


def _dev(torch, keys, vals):
    return (torch.from_numpy(keys.view(np.int64).copy()).cuda(), torch.from_numpy(vals.view(np.int32).copy()).cuda())


def test_noalloc_equals_allocating_sort_on_consecutive_calls(torch):
    # the largest size first, then a smaller one with an odd number of passes
    # (the result comes back from the scratch array), then a ragged tiny one
    for n, bits, seed in [(v.V3DG_SORT_NOALLOC_MAX, 45, 1), (300_001, 17, 2), (4097, 64, 3), (1, 8, 4)]:
        keys, vals = _pairs(n, bits, seed)
        k0, v0 = _dev(torch, keys, vals)
        k1, v1 = _dev(torch, keys, vals)
        v.sort_pairs(k0, v0, bits)
        v.sort_pairs_noalloc(k1, v1, bits)
        torch.cuda.synchronize()
        assert torch.equal(k0, k1) and torch.equal(v0, v1), (n, bits)
        order = np.argsort(keys, kind="stable")
        assert np.array_equal(k1.cpu().numpy().view(np.uint64), keys[order]), (n, bits)
        assert np.array_equal(v1.cpu().numpy().view(np.uint32), vals[order]), (n, bits)


def test_noalloc_refuses_sizes_beyond_its_maximum(torch):
    n = v.V3DG_SORT_NOALLOC_MAX + 1
    keys, vals = _pairs(n, 32, 5)
    k, vv = _dev(torch, keys, vals)
    with pytest.raises(v.V3DGError) as ei:
        v.sort_pairs_noalloc(k, vv, 32)
    assert ei.value.code == v.V3DG_ERR_CAPACITY
    torch.cuda.synchronize()
    assert np.array_equal(k.cpu().numpy().view(np.uint64), keys)  # untouched
    with pytest.raises(v.V3DGError):
        v.sort_pairs_noalloc(k[:10], vv[:10], 0)
