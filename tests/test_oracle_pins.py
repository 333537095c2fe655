"""Pins of the CPU oracle against what the paper and mathematics fix.

None of these compares the oracle with itself: each expected value is a hand
closed form, a library routine on a special case, a brute-force evaluation,
or an invariant the paper states.
"""
import math
import os

import numpy as np
import pytest
from scipy.spatial.transform import Rotation
from scipy.special import sph_harm_y

import scenegen as sg
from tests import helpers as H

HERE = os.path.dirname(os.path.abspath(__file__))


# --------------------------------------------------------------------------
# footprint (Sec. 3.3) and the selection rule (Sec. 3.4)
# --------------------------------------------------------------------------
def _golden_footprints():
    rows = []
    with open(os.path.join(HERE, "golden", "footprint_cases.txt")) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([float(x) for x in line.split()])
    return rows


@pytest.mark.parametrize("case", _golden_footprints())
def test_footprint_closed_form(oracle_lib, case):
    cx, cy, cz, r, fx, fy, F, tau_fit, tau_no = case
    a2 = np.array([0, 0, 1, 0], np.float32)  # identity camera: z_v = cz
    got = oracle_lib.footprint([cx, cy, cz, r], a2, 1.0, fx, fy)
    assert got == pytest.approx(F, rel=1e-6)
    # the FP32 predicate inside selection agrees with F <= tau on both sides of F
    asset = H.two_level_asset([cx, cy, cz, r])
    cam = H.identity_camera(f=fx)
    cam.fy = fy
    T = sg.identity_instances(1)
    m_fit = oracle_lib.select_walk(asset, T, cam, tau_fit)[0]
    m_no = oracle_lib.select_walk(asset, T, cam, tau_no)[0]
    assert m_fit.tolist() == [0, 0, 0, 0, 1]  # root fits: render the coarse cluster
    assert m_no.tolist() == [1, 1, 1, 1, 0]   # root too big on screen: its children


def test_footprint_inverse_square(oracle_lib):
    a2 = np.array([0, 0, 1, 0], np.float32)
    f1 = oracle_lib.footprint([0, 0, 7, 0.3], a2, 1.0, 500, 500)
    f2 = oracle_lib.footprint([0, 0, 14, 0.3], a2, 1.0, 500, 500)
    assert f1 == pytest.approx(4 * f2, rel=1e-12)
    # camera plane inside the sphere: infinite footprint
    assert math.isinf(oracle_lib.footprint([0, 0, 0.2, 0.3], a2, 1.0, 500, 500))


def test_camera_inside_root_selects_leaves(oracle_lib):
    asset = H.two_level_asset([0, 0, 0.5, 1.0])
    cam = H.identity_camera()
    m = oracle_lib.select_walk(asset, sg.identity_instances(1), cam, 3e38)[0]
    assert m.tolist() == [1, 1, 1, 1, 0]


def test_uniform_scale_scales_radius(oracle_lib):
    # scale 2 doubles both the distance and the radius: F is unchanged
    asset = H.two_level_asset([0, 0, 5, 0.5])
    cam = H.identity_camera(f=100.0)
    T = np.array([[[2.0, 0, 0, 0], [0, 2.0, 0, 0], [0, 0, 2.0, 0]]])
    F = math.pi * 0.25 * 1e4 / 25.0  # 314.159...
    assert oracle_lib.select_walk(asset, T, cam, math.ceil(F))[0].tolist() == [0, 0, 0, 0, 1]
    assert oracle_lib.select_walk(asset, T, cam, math.floor(F))[0].tolist() == [1, 1, 1, 1, 0]


@pytest.fixture(scope="module")
def c1_asset():
    return sg.make_asset(16384, 0, 1)


def test_tau_zero_selects_exactly_leaves(oracle_lib, c1_asset):
    a = c1_asset
    for seed in range(8):
        cam = H.random_camera_near(np.random.default_rng(seed))
        m = oracle_lib.select_walk(a, sg.identity_instances(1), cam, 0.0)[0]
        assert np.array_equal(m, H.leaf_mask(a))


def test_huge_tau_far_camera_selects_root(oracle_lib, c1_asset):
    a = c1_asset
    cam = sg.look_at((60.0, 20.0, 30.0), (0, 0, 0), 64, 64, 1.0)
    m = oracle_lib.select_walk(a, sg.identity_instances(1), cam, 3e38)[0]
    roots = (a.parent < 0).astype(np.uint8)
    assert np.array_equal(m, roots)


@pytest.mark.parametrize("seed", range(6))
def test_cut_invariants_random(oracle_lib, seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(64, 4097))
    a = sg.make_asset(n, 0, int(rng.integers(0, 1 << 30)), n_ellipsoids=int(rng.integers(1, 5)))
    T = np.concatenate([sg.identity_instances(1), sg.grid_instances(2, 1.0, 0.3, seed)[:2]])
    prev = None
    for tau in [0.0, 1e-3, 1.0, 30.0, 1e3, 3e4, 1e6, 3e38]:
        for c in range(3):
            cam = H.random_camera_near(rng)
            w = oracle_lib.select_walk(a, T, cam, tau)
            p = oracle_lib.select_predicate(a, T, cam, tau)
            assert np.array_equal(w, p), "walk and parallel predicate disagree"
            for i in range(T.shape[0]):
                assert H.chains_ok(a, w[i])
        # selected Gaussian count is non-increasing in tau for a fixed camera
        cam = sg.look_at((2.0, 1.0, 0.7), (0, 0, 0), 64, 64, 1.0)
        cnt = int((oracle_lib.select_walk(a, T, cam, tau) * a.count[None, :]).sum())
        if prev is not None:
            assert cnt <= prev
        prev = cnt


def test_walk_matches_bruteforce_footprints(oracle_lib, c1_asset):
    """Independent check of the cut with FP64 footprints away from ties."""
    a = c1_asset
    cam = sg.look_at((1.5, -0.8, 0.9), (0, 0, 0), 200, 150, 1.0)
    T = sg.identity_instances(1)
    A, s, _, K = oracle_lib.frame_setup(T, cam)
    tau = 2000.0
    m = oracle_lib.select_walk(a, T, cam, tau)[0]
    F_self = np.array([oracle_lib.footprint(a.self_sphere[k], A[0, 8:12], s[0], cam.fx, cam.fy)
                       for k in range(a.n_clusters)])
    F_par = np.array([oracle_lib.footprint(a.parent_sphere[k], A[0, 8:12], s[0], cam.fx, cam.fy)
                      for k in range(a.n_clusters)])
    F_self[a.self_sphere[:, 3] == 0] = 0.0
    clear = (np.abs(F_self - tau) > 1e-3 * tau) & (np.abs(F_par - tau) > 1e-3 * tau)
    expect = ((F_self <= tau) & (tau < F_par)).astype(np.uint8)
    assert clear.mean() > 0.9
    assert np.array_equal(m[clear], expect[clear])


# --------------------------------------------------------------------------
# frame set-up
# --------------------------------------------------------------------------
def test_frame_setup_identity_and_inverse(oracle_lib):
    cam = sg.look_at((1.0, 2.0, 3.0), (0.1, 0, 0), 100, 100, 1.0)
    A, s, ch, K = oracle_lib.frame_setup(sg.identity_instances(1), cam)
    assert np.array_equal(A[0], cam.world_to_cam.reshape(12))
    assert s[0] == 1.0
    assert np.allclose(ch[0], cam.centre(), atol=1e-6)
    fx32, fy32 = float(np.float32(cam.fx)), float(np.float32(cam.fy))
    assert K == np.float32(math.pi * fx32 * fy32)
    T = sg.grid_instances(2, 1.5, 0.2, 4)
    A, s, ch, K = oracle_lib.frame_setup(T, cam)
    for i in range(T.shape[0]):
        M = np.vstack([T[i], [0, 0, 0, 1]])
        V = np.vstack([cam.world_to_cam.astype(np.float64), [0, 0, 0, 1]])
        assert np.allclose(A[i].reshape(3, 4), (V @ M)[:3], rtol=1e-6, atol=1e-6)
        # chat maps back onto the camera centre
        assert np.allclose(T[i][:, :3] @ ch[i] + T[i][:, 3], cam.centre(), atol=1e-9)


# --------------------------------------------------------------------------
# spherical harmonics (colour of a Gaussian, Sec. 2.1)
# --------------------------------------------------------------------------
def test_sh_matches_scipy_complex_sh(oracle_lib):
    rng = np.random.default_rng(7)
    for _ in range(20):
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        theta = math.acos(d[2])
        phi = math.atan2(d[1], d[0])
        got = oracle_lib.sh_basis(3, d)
        for l in range(4):
            for m in range(-l, l + 1):
                y = sph_harm_y(l, abs(m), theta, phi)
                if m > 0:
                    ref = math.sqrt(2) * y.real
                elif m < 0:
                    ref = math.sqrt(2) * y.imag
                else:
                    ref = y.real
                assert got[l * l + l + m] == pytest.approx(ref, abs=1e-12)


def test_sh_closed_forms_and_orthonormality(oracle_lib):
    d = np.array([0.3, -0.5, 0.8])
    n = d / np.linalg.norm(d)
    y = oracle_lib.sh_basis(1, d)
    c1 = math.sqrt(3 / (4 * math.pi))
    assert y[0] == pytest.approx(1 / (2 * math.sqrt(math.pi)), abs=1e-15)
    assert y[1:] == pytest.approx([-c1 * n[1], c1 * n[2], -c1 * n[0]], abs=1e-14)
    # orthonormality over the sphere (Gauss-Legendre in cos(theta), uniform phi)
    xs, ws = np.polynomial.legendre.leggauss(12)
    phis = np.linspace(0, 2 * math.pi, 24, endpoint=False)
    G = np.zeros((16, 16))
    for x, w in zip(xs, ws):
        st = math.sqrt(1 - x * x)
        for p in phis:
            Y = oracle_lib.sh_basis(3, np.array([st * math.cos(p), st * math.sin(p), x]))
            G += w * (2 * math.pi / len(phis)) * np.outer(Y, Y)
    assert np.allclose(G, np.eye(16), atol=1e-12)


# --------------------------------------------------------------------------
# projection (EWA splat, Sec. 2.1; no dilation, Sec. 5.1)
# --------------------------------------------------------------------------
def test_onaxis_isotropic_projection(oracle_lib):
    f, s, z = 300.0, 0.05, 4.0
    q = Rotation.random(random_state=3).as_quat()  # (x,y,z,w)
    asset = H.single_cluster_asset([[0, 0, z]], [[s, s, s]], [[q[3], q[0], q[1], q[2]]], [0.7],
                                   [[[0.2, -0.1, 0.4]]])
    cam = H.identity_camera(64, 48, f)
    out = oracle_lib.project(asset, sg.identity_instances(1), cam, [0])
    sig = (f * s / z) ** 2
    assert out["valid"][0] == 1
    assert out["mean2"][0] == pytest.approx([32.0, 24.0], abs=1e-12)
    # the FP32-stored quaternion is unit only to ~1e-7, hence the tolerance
    assert out["cov2"][0] == pytest.approx([sig, 0.0, sig], rel=1e-6, abs=1e-6 * sig)
    assert out["conic"][0] == pytest.approx([1 / sig, 0.0, 1 / sig], rel=1e-6, abs=1e-6 / sig)
    y00 = 1 / (2 * math.sqrt(math.pi))
    assert out["rgb"][0] == pytest.approx([y00 * 0.2 + 0.5, y00 * -0.1 + 0.5, y00 * 0.4 + 0.5], abs=1e-7)
    assert out["depth"][0] == np.float32(z)


def test_onaxis_anisotropic_matches_scipy_rotation(oracle_lib):
    f, z = 250.0, 3.0
    rng = np.random.default_rng(11)
    for _ in range(5):
        rot = Rotation.random(random_state=int(rng.integers(1 << 30)))
        q = rot.as_quat()
        s = rng.uniform(0.01, 0.1, 3)
        asset = H.single_cluster_asset([[0, 0, z]], [s], [[q[3], q[0], q[1], q[2]]], [0.5], [[[0, 0, 0]]])
        cam = H.identity_camera(64, 64, f)
        out = oracle_lib.project(asset, sg.identity_instances(1), cam, [0])
        Rm = rot.as_matrix()
        S = Rm @ np.diag(np.asarray(s, np.float32).astype(np.float64) ** 2) @ Rm.T
        ref = (f / z) ** 2 * S[:2, :2]  # on axis J = diag(f/z, f/z) padded with zeros
        got = out["cov2"][0]
        assert got == pytest.approx([ref[0, 0], ref[0, 1], ref[1, 1]], rel=2e-6, abs=1e-6)


def test_nonunit_quaternion_is_normalised(oracle_lib):
    """The covariance uses the rotation of q / |q| (scipy normalises too), so
    a quaternion stored off unit length (narrow storage) stays a rotation."""
    f, z = 250.0, 3.0
    rng = np.random.default_rng(17)
    for k in range(4):
        q = rng.standard_normal(4) * (0.5 + k)  # (x, y, z, w) for scipy
        s = rng.uniform(0.01, 0.1, 3)
        q32 = np.asarray(q, np.float32)
        asset = H.single_cluster_asset([[0, 0, z]], [s], [[q32[3], q32[0], q32[1], q32[2]]], [0.5], [[[0, 0, 0]]])
        out = oracle_lib.project(asset, sg.identity_instances(1), H.identity_camera(64, 64, f), [0])
        Rm = Rotation.from_quat(q32.astype(np.float64)).as_matrix()
        S = Rm @ np.diag(np.asarray(s, np.float32).astype(np.float64) ** 2) @ Rm.T
        ref = (f / z) ** 2 * S[:2, :2]
        assert out["cov2"][0] == pytest.approx([ref[0, 0], ref[0, 1], ref[1, 1]], rel=1e-9, abs=1e-9)


def test_offaxis_jacobian_matches_finite_difference(oracle_lib):
    """Sigma2 = J Sigma J^T with J the derivative of the pinhole map (no guard clamp active)."""
    f = 200.0
    p = np.array([0.3, -0.2, 2.5])
    s = np.array([0.05, 0.02, 0.08])
    rot = Rotation.from_euler("xyz", [0.3, -0.7, 1.1])
    q = rot.as_quat()
    asset = H.single_cluster_asset([p], [s], [[q[3], q[0], q[1], q[2]]], [0.5], [[[0, 0, 0]]])
    cam = H.identity_camera(128, 128, f)
    out = oracle_lib.project(asset, sg.identity_instances(1), cam, [0])
    pf = np.asarray(p, np.float32).astype(np.float64)

    def proj(x):
        return np.array([f * x[0] / x[2] + 64.0, f * x[1] / x[2] + 64.0])

    h = 1e-6
    J = np.stack([(proj(pf + h * e) - proj(pf - h * e)) / (2 * h) for e in np.eye(3)], axis=1)
    Rm = Rotation.from_quat(np.asarray(q, np.float32).astype(np.float64)).as_matrix()
    S = Rm @ np.diag(np.asarray(s, np.float32).astype(np.float64) ** 2) @ Rm.T
    ref = J @ S @ J.T
    assert out["cov2"][0] == pytest.approx([ref[0, 0], ref[0, 1], ref[1, 1]], rel=1e-6)
    assert out["mean2"][0] == pytest.approx(proj(pf), abs=1e-9)


def test_near_plane_culls(oracle_lib):
    asset = H.single_cluster_asset([[0, 0, 0.005], [0, 0, -1.0], [0, 0, 1.0]], [[0.01] * 3] * 3,
                                   [[1, 0, 0, 0]] * 3, [0.5] * 3, [[[0, 0, 0]]] * 3)
    out = oracle_lib.project(asset, sg.identity_instances(1), H.identity_camera(), [0])
    assert out["valid"].tolist() == [0, 0, 1]


# --------------------------------------------------------------------------
# compositing (Sec. 2.1)
# --------------------------------------------------------------------------
def _iso_alpha(o, f, s, z, mx, my, W, Hh):
    sig2 = (f * s / z) ** 2
    ys, xs = np.mgrid[0:Hh, 0:W]
    d2 = (xs + 0.5 - mx) ** 2 + (ys + 0.5 - my) ** 2
    a = np.minimum(0.99, o * np.exp(-d2 / (2 * sig2)))
    a[a < 1 / 255] = 0.0
    return a


def test_single_isotropic_splat_closed_form(oracle_lib):
    f, s, z, o = 120.0, 0.04, 2.0, 0.8
    col = np.array([0.9, 0.2, 0.4])
    y00 = 1 / (2 * math.sqrt(math.pi))
    dc = (col - 0.5) / y00
    bg = (0.1, 0.3, 0.05)
    # on the optical axis the EWA splat is exactly isotropic; a principal point
    # off the pixel grid puts the mean between pixel centres
    cx, cy = 24.39, 19.71
    asset = H.single_cluster_asset([[0.0, 0.0, z]], [[s, s, s]], [[1, 0, 0, 0]], [o], [dc[None, :]])
    cam = H.identity_camera(48, 40, f, cx=cx, cy=cy, bg=bg)
    img, amb, st = oracle_lib.render(asset, sg.identity_instances(1), cam, [0], use_index=True)
    a = _iso_alpha(o, f, s, z, float(np.float32(cx)), float(np.float32(cy)), 48, 40)
    rgb_exp = a[..., None] * col + (1 - a[..., None]) * np.asarray(bg)
    ok = amb == 0
    assert ok.mean() > 0.95
    # one contributing (pixel, splat) pair per pixel where alpha >= 1/255
    assert abs(st["n_hits"] - int((a > 0).sum())) <= int((~ok).sum())
    assert np.abs(img[..., :3] - rgb_exp)[ok].max() < 1e-6
    assert np.abs(img[..., 3] - a)[ok].max() < 1e-6
    assert (img[..., 3][a == 0] == 0).all()


def test_two_splats_front_to_back(oracle_lib):
    f = 100.0
    y00 = 1 / (2 * math.sqrt(math.pi))
    c1 = np.array([1.0, 0.0, 0.0])
    c2 = np.array([0.0, 1.0, 0.0])
    # stored back-to-front so the depth sort has to reorder them
    asset = H.single_cluster_asset([[0, 0, 3.0], [0, 0, 2.0]], [[0.05] * 3, [0.03] * 3], [[1, 0, 0, 0]] * 2,
                                   [0.9, 0.6], [((c2 - 0.5) / y00)[None], ((c1 - 0.5) / y00)[None]])
    cam = H.identity_camera(40, 40, f)
    img, amb, _ = oracle_lib.render(asset, sg.identity_instances(1), cam, [0])
    a1 = _iso_alpha(0.6, f, 0.03, 2.0, 20, 20, 40, 40)  # nearer
    a2 = _iso_alpha(0.9, f, 0.05, 3.0, 20, 20, 40, 40)
    exp = a1[..., None] * c1 + (a2 * (1 - a1))[..., None] * c2
    ok = amb == 0
    assert np.abs(img[..., :3] - exp)[ok].max() < 1e-5
    assert np.abs(img[..., 3] - (1 - (1 - a1) * (1 - a2)))[ok].max() < 1e-5


def test_opaque_stack_stops(oracle_lib):
    """Three 0.99 splats: after two, T would drop below 1e-4 only with the third."""
    y00 = 1 / (2 * math.sqrt(math.pi))
    cols = [np.array([1.0, 0, 0]), np.array([0, 1.0, 0]), np.array([0, 0, 1.0])]
    asset = H.single_cluster_asset([[0, 0, 1.0], [0, 0, 1.5], [0, 0, 2.0]], [[1.0] * 3] * 3, [[1, 0, 0, 0]] * 3,
                                   [1.0, 1.0, 1.0], [((c - 0.5) / y00)[None] for c in cols])
    cam = H.identity_camera(8, 8, 10.0)
    img, amb, _ = oracle_lib.render(asset, sg.identity_instances(1), cam, [0])
    # pixel near the centre: alpha ~ 0.99 for each splat
    px = img[4, 4]
    # first: 0.99*red; second: T=0.01 -> adds 0.99*0.01 green, T=1e-4 (not below); third would push
    # T to 1e-6 < 1e-4: stop without adding blue
    assert px[0] == pytest.approx(0.99, abs=1e-4)
    _, _, st1 = oracle_lib.render_pixels(asset, sg.identity_instances(1), cam, [0], np.array([[4, 4]], np.uint32))
    assert st1["n_hits"] == 3  # two composited splats and the one that ends the pixel
    assert px[1] == pytest.approx(0.0099, abs=1e-5)
    assert px[2] == pytest.approx(0.0, abs=1e-9)


def test_index_equals_bruteforce_and_alpha_range(oracle_lib):
    rng = np.random.default_rng(5)
    a = sg.make_asset(2048, 3, 77)
    T = sg.identity_instances(1)
    for c in range(3):
        cam = H.random_camera_near(rng, 80, 60, dist=(0.6, 4.0))
        cam.bg = (0.2, 0.1, 0.0)
        gids = oracle_lib.mask_to_gids(oracle_lib.select_walk(a, T, cam, float(rng.choice([0.0, 50.0, 500.0]))))
        i1, m1, s1 = oracle_lib.render(a, T, cam, gids, use_index=True)
        i2, m2, s2 = oracle_lib.render(a, T, cam, gids, use_index=False)
        assert np.array_equal(i1, i2)
        assert np.array_equal(m1, m2)
        assert (i1[..., 3] >= 0).all() and (i1[..., 3] < 1).all()
        assert s1["n_pairs"] < s2["n_pairs"] or s2["n_pairs"] == 0


def test_render_pixels_matches_full(oracle_lib):
    a = sg.make_asset(4096, 0, 9)
    cam = sg.look_at((1.2, -1.0, 0.8), (0, 0, 0), 96, 72, 1.0)
    T = sg.identity_instances(1)
    gids = oracle_lib.mask_to_gids(oracle_lib.select_walk(a, T, cam, 10.0))
    full, amb, _ = oracle_lib.render(a, T, cam, gids)
    pix = np.array([[0, 0], [95, 71], [40, 30], [50, 33], [7, 60]], np.uint32)
    got, gamb, _ = oracle_lib.render_pixels(a, T, cam, gids, pix)
    for i, (x, y) in enumerate(pix):
        assert np.array_equal(got[i], full[y, x])
        assert gamb[i] == amb[y, x]


def test_anisotropic_offaxis_splat_image(oracle_lib):
    """alpha(p) = o exp(-1/2 d^T Sigma2^{-1} d) with Sigma2 from a finite-difference Jacobian."""
    f, W, Hh = 150.0, 64, 48
    p = np.array([0.21, -0.13, 2.2])
    s = np.array([0.06, 0.015, 0.03])
    rot = Rotation.from_euler("zyx", [0.8, 0.2, -0.4])
    q = rot.as_quat()
    o = 0.7
    asset = H.single_cluster_asset([p], [s], [[q[3], q[0], q[1], q[2]]], [o], [[[0, 0, 0]]])
    cam = H.identity_camera(W, Hh, f)
    img, amb, _ = oracle_lib.render(asset, sg.identity_instances(1), cam, [0])
    pf = np.asarray(p, np.float32).astype(np.float64)

    def proj(x):
        return np.array([f * x[0] / x[2] + W / 2, f * x[1] / x[2] + Hh / 2])

    h = 1e-6
    J = np.stack([(proj(pf + h * e) - proj(pf - h * e)) / (2 * h) for e in np.eye(3)], axis=1)
    Rm = Rotation.from_quat(np.asarray(q, np.float32).astype(np.float64)).as_matrix()
    S = Rm @ np.diag(np.asarray(s, np.float32).astype(np.float64) ** 2) @ Rm.T
    Si = np.linalg.inv(J @ S @ J.T)
    mu = proj(pf)
    ys, xs = np.mgrid[0:Hh, 0:W]
    d = np.stack([xs + 0.5 - mu[0], ys + 0.5 - mu[1]], axis=-1)
    q2 = np.einsum("...i,ij,...j->...", d, Si, d)
    a = np.minimum(0.99, np.float32(o) * np.exp(-0.5 * q2))
    a[a < 1 / 255] = 0
    ok = amb == 0
    assert (a > 0.1).sum() > 20
    assert np.abs(img[..., 3] - a)[ok].max() < 1e-6
    # the conic is the inverse of the projected covariance
    out = oracle_lib.project(asset, sg.identity_instances(1), cam, [0])
    ca, cb, cc = out["conic"][0]
    sa, sb, sc = out["cov2"][0]
    assert np.allclose(np.array([[ca, cb], [cb, cc]]) @ np.array([[sa, sb], [sb, sc]]), np.eye(2), atol=1e-9)


def test_guard_band_clamps_the_jacobian(oracle_lib):
    """Sec. 2.1 EWA splat with the 3DGS guard band: beyond |x/z| = 1.3 (W/2)/fx
    (and |y/z| = 1.3 (H/2)/fy) the Jacobian is taken at the clamped point.
    For an isotropic Gaussian of scale s under the identity camera,
    J J^T = (f/z)^2 [[1 + ux^2, ux uy], [ux uy, 1 + uy^2]] with (ux, uy) the
    clamped (x/z, y/z), so Sigma2 = s^2 (f/z)^2 [[1 + ux^2, ux uy], [ux uy, 1 + uy^2]]."""
    f, W, Hh, z, s = 100.0, 64, 48, 2.0, 0.03
    limx = 1.3 * (W / 2) / f  # 0.416
    limy = 1.3 * (Hh / 2) / f  # 0.312
    # (x/z, y/z): both clamped; x clamped on the negative side only; neither clamped
    cases = [(0.6, -0.5), (-0.9, 0.1), (0.2, -0.25)]
    pos = [[u * z, v * z, z] for u, v in cases]
    asset = H.single_cluster_asset(pos, [[s] * 3] * 3, [[1, 0, 0, 0]] * 3, [0.5] * 3, [[[0, 0, 0]]] * 3)
    out = oracle_lib.project(asset, sg.identity_instances(1), H.identity_camera(W, Hh, f), [0])
    s32 = float(np.float32(s))
    for i, (u, v) in enumerate(cases):
        p = np.asarray(pos[i], np.float32).astype(np.float64)
        ux = min(max(p[0] / p[2], -limx), limx)
        uy = min(max(p[1] / p[2], -limy), limy)
        k = s32 * s32 * (f / p[2]) ** 2
        assert out["valid"][i] == 1
        assert out["cov2"][i] == pytest.approx([k * (1 + ux * ux), k * ux * uy, k * (1 + uy * uy)], rel=1e-9)
        # the mean is not clamped: it is the pinhole projection of the centre
        assert out["mean2"][i] == pytest.approx([f * p[0] / p[2] + W / 2, f * p[1] / p[2] + Hh / 2], rel=1e-12)
    # the first case really is outside the band on both axes, the last inside
    assert abs(cases[0][0]) > limx and abs(cases[0][1]) > limy
    assert abs(cases[2][0]) < limx and abs(cases[2][1]) < limy


def test_far_plane_culls(oracle_lib):
    """A splat is kept only for near < z < far (FP32 depth), so z = far and
    beyond are culled while z just in front of the far plane is kept."""
    far = 50.0
    zs = [49.0, 50.0, 51.0, 1.0]
    asset = H.single_cluster_asset([[0, 0, z] for z in zs], [[0.5] * 3] * 4, [[1, 0, 0, 0]] * 4, [0.5] * 4,
                                   [[[0, 0, 0]]] * 4)
    out = oracle_lib.project(asset, sg.identity_instances(1), H.identity_camera(far=far), [0])
    assert out["valid"].tolist() == [1, 0, 0, 1]


def _sh1_asset(coef_m_neg1, coef_m_pos1):
    """One Gaussian at the origin, SH degree 1 with DC 0 and two l = 1
    coefficients: index 1 (m = -1, the y term) and index 3 (m = +1, the x term)."""
    sh = np.zeros((1, 4, 3), np.float32)
    sh[0, 1] = coef_m_neg1
    sh[0, 3] = coef_m_pos1
    return H.single_cluster_asset([[0, 0, 0]], [[0.05] * 3], [[1, 0, 0, 0]], [0.6], sh, sh_degree=1)


def test_sh_view_direction_and_asset_frame(oracle_lib):
    """View-dependent colour (Sec. 2.1): the SH are evaluated at the unit
    direction from the camera centre to the Gaussian, p - c, in the asset's
    own frame.  With Y_1,-1 = -c1 y and Y_1,1 = -c1 x (c1 = sqrt(3 / 4 pi)):
      camera at +5 x, identity instance: d = (-1, 0, 0), so only the m = +1
        term is lit, with Y = +c1;
      the same camera, asset yawed by +90 deg about z: the camera sits at
        (0, -5, 0) in the asset frame, d = (0, 1, 0), so only the m = -1
        term is lit, with Y = -c1."""
    c1 = math.sqrt(3.0 / (4.0 * math.pi))
    a = 0.4
    asset = _sh1_asset([a, 0, 0], [0, a, 0])
    cam = sg.look_at((5.0, 0.0, 0.0), (0.0, 0.0, 0.0), 64, 64, 1.0)
    out = oracle_lib.project(asset, sg.identity_instances(1), cam, [0])
    assert out["valid"][0] == 1
    assert out["rgb"][0] == pytest.approx([0.5, 0.5 + a * c1, 0.5], abs=1e-7)
    yaw = np.array([[[0.0, -1.0, 0.0, 0.0], [1.0, 0.0, 0.0, 0.0], [0.0, 0.0, 1.0, 0.0]]])
    out = oracle_lib.project(asset, yaw, cam, [0])
    assert out["valid"][0] == 1
    assert out["rgb"][0] == pytest.approx([0.5 - a * c1, 0.5, 0.5], abs=1e-7)
