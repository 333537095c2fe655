"""The serving path (v3dg_server_*) through the C ABI.

Every request's image must equal, bit for bit, what v3dg_select +
v3dg_render produce for it alone, whatever the mix of scenes, image sizes and
tolerances in flight, with and without graph replay, and after key-capacity
retries.  Served images are also checked against the oracle directly: whole
small frames, and sampled pixels of mixed-resolution requests (up to
3840x2160) on scenes shaped like the serving workload's.
"""
import numpy as np
import pytest

import oracle
import paper_2505_06523_amd as v
import scenegen as sg
from tests import helpers as H
from tests.test_gpu_parity import MAX_ABS, MIN_PSNR, _say, check_image, psnr

pytestmark = pytest.mark.gpu

# the serving loop's chunk size of long bin lists: the standalone references
# render with the same plan, so that images agree bit for bit
SRV_CHUNK = H.blend_chunk_sizes(server=True)[1]


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a GPU"
    v.lib()
    return _t


@pytest.fixture(scope="module")
def worlds():
    return [(sg.make_asset(16384, 0, 1), sg.identity_instances(1)),
            (sg.make_asset(8192, 3, 31), sg.grid_instances(2, 1.0, 0.2, 5)),
            (H.stacked_splats(6000, 5, (0.05, 0.5)), sg.identity_instances(1))]


@pytest.fixture(scope="module")
def scenes(torch, worlds):
    out = [v.Scene(a, T) for a, T in worlds]
    for sc in out:
        sc.set_chunk_keys(SRV_CHUNK)
    yield out
    for sc in out:
        sc.close()


def _requests(rng, n):
    shapes = [(200, 150), (333, 250), (640, 360)]
    reqs = []
    for i in range(n):
        k = int(rng.integers(0, 3))
        w, h = shapes[int(rng.integers(0, 3))]
        if k == 2:
            cam = H.identity_camera(w, h, 300.0 * w / 200.0, bg=(0.1, 0.2, 0.3))
        else:
            cam = H.random_camera_near(rng, w, h, dist=(0.8, 6.0))
        tau = [0.0, 1.0, 50.0][int(rng.integers(0, 3))]
        reqs.append((k, cam, tau))
    return reqs


def _standalone(scenes, torch, reqs):
    ref = []
    for k, cam, tau in reqs:
        sc = scenes[k]
        sel = sc.select(cam, tau)
        img = sc.render(cam, sel).clone()
        ref.append((img, sel.info()[1]))
        sel.free()
    torch.cuda.synchronize()
    return ref


@pytest.mark.parametrize("use_graphs", [True, False])
def test_server_images_equal_standalone(scenes, torch, use_graphs):
    rng = np.random.default_rng(11 + int(use_graphs))
    reqs = _requests(rng, 30)
    ref = _standalone(scenes, torch, reqs)
    srv = v.Server(scenes, n_contexts=4, max_batch=8, use_graphs=use_graphs)
    tickets = {}
    done = []
    # submit in waves with eager work on the default stream in between, so
    # that graphs replay several times interleaved with other launches
    for wave in range(3):
        for i in range(wave * 10, wave * 10 + 10):
            k, cam, tau = reqs[i]
            t, _ = srv.submit(k, cam, tau)
            tickets[t] = i
        done.extend(srv.poll())
        scenes[0].render(reqs[0][1], scenes[0].select(reqs[0][1], 1.0))
        torch.cuda.synchronize()
    done.extend(srv.drain())
    st = srv.stats()
    _say("server graphs=%s: %s" % (use_graphs, st))
    assert len(done) == len(reqs)
    for r in done:
        i = tickets[r["ticket"]]
        assert r["status"] == 0, r
        img, n_slots = ref[i]
        assert r["n_slots"] == n_slots, i
        assert torch.equal(r["image"], img), (i, reqs[i][0], reqs[i][2])
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["batches"] >= 3 and st["batched_requests"] == len(reqs) + st["retries"]
    if use_graphs:
        assert st["graph_launches"] == len(reqs) + st["retries"]
        assert 0 < st["graph_captures"] <= st["graph_launches"]
    else:
        assert st["graph_launches"] == 0
    srv.close()


@pytest.mark.parametrize("use_graphs", [True, False])
def test_server_full_detail_requests(scenes, torch, use_graphs):
    """Full-detail requests (every leaf, no selection) mixed with selected
    ones in one stream of requests: each equals v3dg_render_full (or select +
    render) of the same camera alone, bit for bit."""
    rng = np.random.default_rng(41 + int(use_graphs))
    reqs = _requests(rng, 16)
    full = [i % 2 == 0 for i in range(len(reqs))]
    ref, slots = [], []
    for (k, cam, tau), f in zip(reqs, full):
        sc = scenes[k]
        if f:
            ref.append(sc.render_full(cam).clone())
        else:
            sel = sc.select(cam, tau)
            ref.append(sc.render(cam, sel).clone())
            sel.free()
        slots.append(sc.frame_stats()["n_slots"])
    torch.cuda.synchronize()
    srv = v.Server(scenes, n_contexts=3, max_batch=8, use_graphs=use_graphs)
    tickets = {}
    for i, ((k, cam, tau), f) in enumerate(zip(reqs, full)):
        t, _ = srv.submit(k, cam, tau, full=f)
        tickets[t] = i
    done = srv.drain()
    st = srv.stats()
    _say("server full-detail mix graphs=%s: %s" % (use_graphs, st))
    assert len(done) == len(reqs)
    for r in done:
        i = tickets[r["ticket"]]
        assert r["status"] == 0, r
        assert torch.equal(r["image"], ref[i]), (i, full[i], reqs[i][0])
        assert r["n_slots"] == slots[i], (i, full[i])
    assert st["completed"] == len(reqs) and st["failed"] == 0
    # only the selected requests go through the batched selection
    assert st["batched_requests"] == len(reqs) - sum(full) + st["retries"]
    srv.close()


def test_server_retries_after_key_overflow(scenes, torch):
    """A capacity of one key per pixel (at least 65,536) at first: requests that
    need more are retried on grown buffers.  A fourth scene of 6,000 large
    splats, seen from in front, covers every bin of its images (~6,000 keys
    per bin), so its requests overflow whatever the mix."""
    rng = np.random.default_rng(5)
    dense = v.Scene(H.stacked_splats(6000, 5, (0.05, 0.5), log_scale=-1.0), sg.identity_instances(1))
    dense.set_chunk_keys(SRV_CHUNK)
    all_scenes = list(scenes) + [dense]
    reqs = _requests(rng, 12) + [(3, H.identity_camera(w, h, 300.0 * w / 200.0, bg=(0.1, 0.2, 0.3)), 0.0)
                                 for w, h in [(200, 150), (333, 250), (640, 360)]]
    ref = _standalone(all_scenes, torch, reqs)
    srv = v.Server(all_scenes, n_contexts=3, max_batch=4, keys_per_pixel=1)  # too few keys at first
    tickets = {}
    for i, (k, cam, tau) in enumerate(reqs):
        t, _ = srv.submit(k, cam, tau)
        tickets[t] = i
    done = srv.drain()
    st = srv.stats()
    _say("retries: %s" % st)
    assert st["retries"] > 0
    assert sum(r["retries"] for r in done) == st["retries"]
    for r in done:
        i = tickets[r["ticket"]]
        assert r["status"] == 0
        assert torch.equal(r["image"], ref[i][0]), i
    srv.close()
    dense.close()


def test_server_budget_limits_contexts(scenes, torch):
    rng = np.random.default_rng(9)
    reqs = [r for r in _requests(rng, 60) if r[1].width == 640][:8]
    ref = _standalone(scenes, torch, reqs)
    probe = v.Server(scenes, n_contexts=1, max_batch=1)
    base = probe.stats()["workspace_bytes"]
    probe.submit(*reqs[0])
    probe.drain()
    one = probe.stats()["workspace_bytes"]  # one context holding a 640x360 frame
    probe.close()
    with pytest.raises(v.V3DGError) as ei:
        v.Server(scenes, n_contexts=4, max_batch=4, hbm_budget_bytes=base // 2)
    assert ei.value.code == v.V3DG_ERR_OOM
    budget = one + base // 2  # room for one such context, not for a second one
    srv = v.Server(scenes, n_contexts=8, max_batch=8, hbm_budget_bytes=budget)
    tickets = {}
    for i, (k, cam, tau) in enumerate(reqs):
        t, _ = srv.submit(k, cam, tau)
        tickets[t] = i
    done = srv.drain()
    st = srv.stats()
    _say("budget %d (one context %d): %s" % (budget, one, st))
    assert st["contexts_live"] == 1
    assert st["peak_workspace_bytes"] <= budget
    assert len(done) == len(reqs)
    for r in done:
        assert r["status"] == 0
        assert torch.equal(r["image"], ref[tickets[r["ticket"]]][0])
    srv.close()


def test_server_invalid_arguments(scenes, torch):
    srv = v.Server(scenes, n_contexts=2, max_batch=2)
    cam = H.identity_camera(64, 48, 100.0)
    with pytest.raises(v.V3DGError):
        srv.submit(7, cam, 1.0)
    with pytest.raises(v.V3DGError):
        srv.submit(0, cam, -1.0)
    with pytest.raises(v.V3DGError):
        srv.submit(0, cam, float("nan"))
    bad = H.identity_camera(64, 48, 100.0)
    bad.fx = 0.0
    with pytest.raises(v.V3DGError):
        srv.submit(0, bad, 1.0)
    assert srv.poll() == []
    # a waiting poll with no room for a record is refused (it could never return one)
    with pytest.raises(v.V3DGError) as ei:
        v.v3dg_server_poll(srv.handle, True, cap=0)
    assert ei.value.code == v.V3DG_ERR_INVALID_ARG
    assert v.v3dg_server_poll(srv.handle, False, cap=0) == []
    srv.close()
    with pytest.raises(v.V3DGError):
        v.Server(scenes, n_contexts=0)
    for ck in (512, 3000, 8192):  # chunk sizes: 1024, 2048 or 4096 keys (0: the default)
        with pytest.raises(v.V3DGError):
            v.Server(scenes, n_contexts=1, chunk_keys=ck)
        with pytest.raises(v.V3DGError):
            scenes[0].set_chunk_keys(ck)


@pytest.mark.parametrize("chunk_keys", [1024, 2048])
def test_server_chunk_sizes_equal_standalone(scenes, torch, chunk_keys):
    """Servers with other chunk sizes than the default equal standalone renders
    of the same chunk size bit for bit, long lists included (the stacked scene,
    ~6,000 keys per bin)."""
    rng = np.random.default_rng(40 + chunk_keys)
    reqs = _requests(rng, 9) + [(2, H.identity_camera(w, h, 300.0 * w / 200.0, bg=(0.1, 0.2, 0.3)), 0.0)
                                for w, h in [(200, 150), (640, 360)]]
    try:
        for sc in scenes:
            sc.set_chunk_keys(chunk_keys)
        ref = _standalone(scenes, torch, reqs)
        srv = v.Server(scenes, n_contexts=3, max_batch=4, use_graphs=True, chunk_keys=chunk_keys)
        tickets = {}
        for i, (k, cam, tau) in enumerate(reqs):
            t, _ = srv.submit(k, cam, tau)
            tickets[t] = i
        done = srv.drain()
        assert len(done) == len(reqs)
        for r in done:
            i = tickets[r["ticket"]]
            assert r["status"] == 0, r
            assert torch.equal(r["image"], ref[i][0]), (i, reqs[i][0], reqs[i][2])
        srv.close()
    finally:
        for sc in scenes:
            sc.set_chunk_keys(SRV_CHUNK)


def test_served_images_match_the_oracle(scenes, worlds, torch):
    """Whole served frames (three scenes, three image sizes, three tolerances,
    graph replay) against the FP64 oracle."""
    rng = np.random.default_rng(23)
    reqs = _requests(rng, 12)
    srv = v.Server(scenes, n_contexts=4, max_batch=8, use_graphs=True)
    tickets = {}
    for i, (k, cam, tau) in enumerate(reqs):
        t, _ = srv.submit(k, cam, tau)
        tickets[t] = i
    done = srv.drain()
    assert len(done) == len(reqs)
    for r in done:
        i = tickets[r["ticket"]]
        k, cam, tau = reqs[i]
        a, T = worlds[k]
        assert r["status"] == 0
        gids = oracle.mask_to_gids(oracle.select_walk(a, T, cam, tau))
        ref, amb, _ = oracle.render(a, T, cam, gids)
        check_image(r["image"].cpu().numpy(), ref, amb, "served %d (scene %d, %dx%d, tau %g)"
                    % (i, k, cam.width, cam.height, tau))
    srv.close()


def test_served_mixed_resolutions_sampled_against_the_oracle(torch):
    """The first two scenes of the serving workload (1M and 2M leaves: rigid
    copies of 262,144-leaf SH3 bases), Poisson-style requests at 1280x720,
    1920x1080 and 3840x2160 with tolerances 1 and 4, all in flight together:
    sampled pixels of every served image against the oracle."""
    gen = sg.serving_scenes()
    worlds = [next(gen) for _ in range(2)]
    gen.close()
    scs = [v.Scene(a) for a, _, _ in worlds]
    extents = [L for _, _, L in worlds]
    reqs = sg.serving_requests(8, 0.0, extents, seed=77)
    srv = v.Server(scs, n_contexts=4, max_batch=8, use_graphs=True)
    tickets = {}
    for i, r in enumerate(reqs):
        t, _ = srv.submit(r["scene"], r["cam"], r["tau"])
        tickets[t] = i
    done = srv.drain()
    assert len(done) == len(reqs)
    sizes = set()
    rng = np.random.default_rng(78)
    for d in done:
        i = tickets[d["ticket"]]
        r = reqs[i]
        cam, a = r["cam"], worlds[r["scene"]][0]
        T = sg.identity_instances(1)
        assert d["status"] == 0
        sizes.add((cam.width, cam.height))
        gids = oracle.mask_to_gids(oracle.select_walk(a, T, cam, r["tau"]))
        pix = np.stack([rng.integers(0, cam.width, 2000), rng.integers(0, cam.height, 2000)], axis=1).astype(np.uint32)
        ref, amb, _ = oracle.render_pixels(a, T, cam, gids, pix)
        got = d["image"].cpu().numpy()[pix[:, 1], pix[:, 0]]
        ok = amb == 0
        err = np.abs(got - ref)[ok].max()
        _say("served %d: scene %d %dx%d tau %g, %d slots, sampled max_abs %.3g psnr %.1f"
             % (i, r["scene"], cam.width, cam.height, r["tau"], d["n_slots"], err, psnr(got[None], ref[None])))
        assert d["n_slots"] == int(a.count[gids % a.n_clusters].sum())
        assert err <= MAX_ABS and psnr(got[None], ref[None]) >= MIN_PSNR
    assert len(sizes) >= 2
    srv.close()
    for sc in scs:
        sc.close()
