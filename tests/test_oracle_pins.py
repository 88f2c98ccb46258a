"""Pins of the CPU oracle against closed forms, invariants and library routines.

Each test checks the oracle against something other than itself: scipy's
rotations and spherical harmonics, numpy's eigen-solver and lexsort, exact
quadrature, an analytic ray cast of the room box, closed-form single- and
two-Gaussian pixels, and finite differences of the oracle's own forward pass.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
from paper_2506_06988_amd import scenes

P = oracle.default_params()
F32 = lambda v: float(np.float32(v))
LP = F32(0.3)


def one_cam(w=64, h=64, f=64.0):
    return scenes.Camera(w, h, f, f, w / 2.0, h / 2.0, np.eye(3), np.zeros(3))


def gauss(means, log_scales=None, quats=None, logits=None, colours=None, degree=0, sh=None):
    means = np.atleast_2d(np.asarray(means, np.float64))
    n = means.shape[0]
    ls = np.full((n, 3), -3.0) if log_scales is None else np.asarray(log_scales, np.float64)
    q = np.tile([1.0, 0, 0, 0], (n, 1)) if quats is None else np.asarray(quats, np.float64)
    lg = np.zeros(n) if logits is None else np.asarray(logits, np.float64)
    if sh is None:
        k = (degree + 1) ** 2
        sh = np.zeros((n, k, 3))
        col = np.full((n, 3), 0.7) if colours is None else np.asarray(colours, np.float64)
        sh[:, 0, :] = (col - 0.5) / scenes.Y00
    return scenes.make_gaussians(means, ls, q, lg, sh, degree)


# ------------------------------------------------------------ projection --
def test_quaternion_rotation_matches_scipy():
    rng = np.random.default_rng(1)
    for _ in range(50):
        q = rng.standard_normal(4) * rng.uniform(0.1, 3.0)
        R = oracle.quat_to_rot(q)
        ref = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()  # scipy is scalar-last
        np.testing.assert_allclose(R, ref, atol=1e-14)


def test_centred_isotropic_gaussian_closed_form():
    # identity camera, Gaussian on the axis: Sigma' = ((f s / z)^2 + 0.3) I, mean2D = (cx, cy)
    cam = one_cam()
    for z, ls in ((2.0, -3.0), (3.5, -2.2), (5.0, -4.0)):
        g = gauss([[0, 0, z]], log_scales=[[ls] * 3])
        pr = oracle.project(g, cam)
        s = math.exp(float(np.float32(ls)))
        var = (64.0 * s / z) ** 2 + LP
        np.testing.assert_allclose(pr["cov2d"][0], [var, 0.0, var], rtol=1e-13, atol=1e-15)
        np.testing.assert_allclose(pr["mean2d"][0], [32.0, 32.0], atol=1e-13)
        np.testing.assert_allclose(pr["conic"][0], [1 / var, 0.0, 1 / var], rtol=1e-13, atol=1e-15)
        # isotropic: the eigenvalue gap is 0, so lambda_max = var + sqrt(0.1)
        assert pr["radius"][0] == math.ceil(3.0 * math.sqrt(var + math.sqrt(0.1)))


def test_rotated_anisotropic_on_axis_uses_R_S_S_R():
    # on the axis J = diag(f/z, f/z) on x, y, so Sigma' = (f/z)^2 [R S^2 R^T]_xy + 0.3 I
    rng = np.random.default_rng(2)
    cam = one_cam()
    for _ in range(20):
        q = rng.standard_normal(4)
        ls = rng.uniform(-4, -1.5, 3)
        z = rng.uniform(1, 6)
        g = gauss([[0, 0, z]], log_scales=[ls], quats=[q])
        pr = oracle.project(g, cam)
        qq = g.quats[0].astype(np.float64)
        R = Rotation.from_quat([qq[1], qq[2], qq[3], qq[0]]).as_matrix()
        S2 = np.diag(np.exp(g.log_scales[0].astype(np.float64)) ** 2)
        Sig = R @ S2 @ R.T
        zz = float(g.means[0, 2])
        ref = (64.0 / zz) ** 2 * Sig[:2, :2] + LP * np.eye(2)
        np.testing.assert_allclose(pr["cov2d"][0], [ref[0, 0], ref[0, 1], ref[1, 1]], rtol=1e-11)
        # Sigma's eigenvalues are the squared scales
        np.testing.assert_allclose(np.sort(np.linalg.eigvalsh(Sig)), np.sort(np.diag(S2)), rtol=1e-10)


def _pinhole(cam, p):
    pc = cam.R @ p + cam.t
    return np.array([cam.fx * pc[0] / pc[2] + cam.cx, cam.fy * pc[1] / pc[2] + cam.cy])


def test_ewa_covariance_is_the_linearised_projection():
    # Sigma' - 0.3 I == Jfd Sigma Jfd^T with Jfd the finite-difference Jacobian of
    # the full world -> pixel map (independent of the oracle's J formula)
    rng = np.random.default_rng(3)
    for _ in range(30):
        cam = scenes.random_room_camera(rng, 320, 240)
        mu = cam.centre + cam.R.T @ np.array([rng.uniform(-0.6, 0.6), rng.uniform(-0.4, 0.4), 1.0]) * rng.uniform(0.5, 3)
        q = rng.standard_normal(4)
        ls = rng.uniform(-4, -2, 3)
        g = gauss([mu], log_scales=[ls], quats=[q])
        mu64 = g.means[0].astype(np.float64)
        pr = oracle.project(g, cam)
        assert pr["radius"][0] > 0
        h = 1e-6
        Jfd = np.zeros((2, 3))
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            Jfd[:, k] = (_pinhole(cam, mu64 + e) - _pinhole(cam, mu64 - e)) / (2 * h)
        qq = g.quats[0].astype(np.float64)
        R = Rotation.from_quat([qq[1], qq[2], qq[3], qq[0]]).as_matrix()
        Sig = R @ np.diag(np.exp(g.log_scales[0].astype(np.float64)) ** 2) @ R.T
        ref = Jfd @ Sig @ Jfd.T + LP * np.eye(2)
        np.testing.assert_allclose(pr["cov2d"][0], [ref[0, 0], ref[0, 1], ref[1, 1]], rtol=2e-7, atol=1e-9)
        np.testing.assert_allclose(pr["mean2d"][0], _pinhole(cam, mu64), atol=1e-9)
        cov = np.array([[pr["cov2d"][0, 0], pr["cov2d"][0, 1]], [pr["cov2d"][0, 1], pr["cov2d"][0, 2]]])
        inv = np.linalg.inv(cov)
        np.testing.assert_allclose(pr["conic"][0], [inv[0, 0], inv[0, 1], inv[1, 1]], rtol=1e-12)
        lam = np.linalg.eigvalsh(cov)
        if (lam[1] - lam[0]) ** 2 / 4 > 0.1:
            assert pr["radius"][0] == math.ceil(3 * math.sqrt(lam[1]))
        assert pr["depth_bits"][0] == np.float32((cam.R @ mu64 + cam.t)[2]).view(np.uint32)


def test_jacobian_clamp_outside_the_view():
    # beyond 1.3 x the half field of view the Jacobian is taken at the clamped
    # direction: Sigma' equals the linearisation at x/z = 1.3 tan(fov/2)
    cam = one_cam(64, 64, 64.0)
    lim = F32(1.3) * 64 / (2 * 64.0)
    z = 2.0
    g = gauss([[0.7 * z, 0.0, z]], log_scales=[[-1.0, -1.0, -1.0]])
    pr = oracle.project(g, cam)
    assert pr["radius"][0] > 0 and pr["mean2d"][0, 0] > 64  # centre off screen, footprint on it
    s2 = math.exp(2 * -1.0)
    J = np.array([[64 / z, 0, -64 * lim / z], [0, 64 / z, 0]])
    ref = J @ (s2 * np.eye(3)) @ J.T + LP * np.eye(2)
    np.testing.assert_allclose(pr["cov2d"][0], [ref[0, 0], ref[0, 1], ref[1, 1]], rtol=1e-12)


def test_rect_is_the_tile_cover_of_the_3sigma_box():
    rng = np.random.default_rng(4)
    cam = one_cam(100, 70, 80.0)
    g = gauss(np.column_stack([rng.uniform(-1.5, 1.5, 300), rng.uniform(-1, 1, 300), rng.uniform(1, 4, 300)]),
              log_scales=rng.uniform(-4, -1, (300, 3)), quats=rng.standard_normal((300, 4)))
    pr = oracle.project(g, cam)
    TX, TY = 7, 5
    for i in range(300):
        r = pr["radius"][i]
        u, v = pr["mean2d"][i]
        xs = [t for t in range(TX) if t * 16 <= u + r and (t + 1) * 16 > u - r]
        ys = [t for t in range(TY) if t * 16 <= v + r and (t + 1) * 16 > v - r]
        if r == 0:
            assert (not xs or not ys) or pr["depth"][i] <= 0.2
            continue
        x0, x1, y0, y1 = pr["rect"][i]
        assert (x0, x1) == (min(xs), max(xs) + 1)
        assert (y0, y1) == (min(ys), max(ys) + 1)
        assert pr["tiles"][i] == len(xs) * len(ys)


def test_culling_near_plane_and_non_finite():
    cam = one_cam()
    g = gauss([[0, 0, 0.1], [0, 0, F32(0.2)], [0, 0, 0.25], [0, 0, 2.0], [0, 0, 2.0]])
    g.means[4, 0] = np.nan
    pr = oracle.project(g, cam)
    assert list(pr["radius"] > 0) == [False, False, True, True, False]


# --------------------------------------------------------------------- SH --
def _quadrature(nt=12, nphi=24):
    x, w = np.polynomial.legendre.leggauss(nt)
    phi = np.arange(nphi) * 2 * np.pi / nphi
    ct, ph = np.meshgrid(x, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    dirs = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    wts = (w[:, None] * np.full(nphi, 2 * np.pi / nphi)[None]).reshape(-1)
    return dirs, wts


def test_sh_basis_orthonormal_by_exact_quadrature():
    dirs, wts = _quadrature()
    Y = oracle.sh_basis(3, dirs)
    gram = (Y * wts[:, None]).T @ Y
    np.testing.assert_allclose(gram, np.eye(16), atol=1e-12)


def test_sh_basis_matches_scipy_real_combination():
    from scipy.special import sph_harm_y
    rng = np.random.default_rng(5)
    d = rng.standard_normal((200, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    theta = np.arccos(np.clip(d[:, 2], -1, 1))
    phi = np.arctan2(d[:, 1], d[:, 0])
    Y = oracle.sh_basis(3, d)
    for l in range(4):
        for m in range(-l, l + 1):
            c = sph_harm_y(l, abs(m), theta, phi)
            if m > 0:
                ref = math.sqrt(2) * (-1) ** m * c.real
            elif m < 0:
                ref = math.sqrt(2) * (-1) ** m * c.imag
            else:
                ref = c.real
            np.testing.assert_allclose(Y[:, l * l + l + m], ref, atol=1e-12)


def test_sh_colour_offset_and_clamp():
    cam = one_cam()
    # DC only: colour = Y00 * k + 0.5, negative values clamp to 0
    g = gauss([[0, 0, 2.0], [0.1, 0, 2.0]], colours=[[0.2, 0.9, -0.3], [1.4, 0.0, 0.5]])
    pr = oracle.project(g, cam)
    np.testing.assert_allclose(pr["rgb"], [[0.2, 0.9, 0.0], [1.4, 0.0, 0.5]], atol=1e-7)


# -------------------------------------------------------------- sorting --
def test_keys_match_brute_force_lexsort():
    sc = scenes.config1()
    cam = sc.cameras[0]
    k, v, r = oracle.keys(sc.gaussians, cam)
    pr = oracle.project(sc.gaussians, cam)
    TX = 4
    tile_l, dbits_l, gid_l = [], [], []
    for gi in np.nonzero(pr["radius"] > 0)[0]:
        x0, x1, y0, y1 = pr["rect"][gi]
        for ty in range(y0, y1):
            for tx in range(x0, x1):
                tile_l.append(ty * TX + tx)
                dbits_l.append(pr["depth_bits"][gi])
                gid_l.append(gi)
    tile_a, db_a, gid_a = map(np.asarray, (tile_l, dbits_l, gid_l))
    order = np.lexsort((gid_a, db_a, tile_a))
    ref_keys = (tile_a[order].astype(np.uint64) << np.uint64(32)) | db_a[order].astype(np.uint64)
    np.testing.assert_array_equal(k, ref_keys)
    np.testing.assert_array_equal(v, gid_a[order])
    assert len(k) == pr["tiles"].sum()
    # ranges partition [0, K) in tile order
    assert r[0, 0] == 0 and r[-1, 1] == len(k)
    np.testing.assert_array_equal(r[1:, 0], r[:-1, 1])
    counts = np.bincount(tile_a, minlength=r.shape[0])
    np.testing.assert_array_equal(r[:, 1] - r[:, 0], counts)


# ---------------------------------------------------------------- blend --
def quad(z=5.0, half=2.5, tex=None, rng=None):
    rng = rng or np.random.default_rng(0)
    m = scenes.quad_mesh(rng, z=z, half=half, tex_size=8)
    if tex is not None:
        m.tex = tex
    return m


def test_single_gaussian_pixel_closed_form():
    cam = one_cam(32, 32, 32.0)
    z, ls, logit = 2.0, -2.5, 0.8
    g = gauss([[0, 0, z]], log_scales=[[ls] * 3], logits=[logit], colours=[[0.9, 0.3, 0.6]])
    mesh = quad(z=4.0, half=3.0)
    out = oracle.render(g, mesh, cam)
    o = 1 / (1 + math.exp(-float(np.float32(logit))))
    var = (32.0 * math.exp(float(np.float32(ls))) / z) ** 2 + LP
    ii, jj = np.meshgrid(np.arange(32) + 0.5, np.arange(32) + 0.5)
    d2 = (ii - 16.0) ** 2 + (jj - 16.0) ** 2
    a = np.minimum(F32(0.99), np.float32(o) * np.exp(-0.5 * d2 * np.float32(1 / var)))
    r = math.ceil(3 * math.sqrt(var))
    inside = (np.abs(ii - 16) <= 16) & (np.abs(jj - 16) <= 16)  # all tiles of a 32x32 image
    a = np.where((a >= F32(1 / 255)) & inside, a, 0.0)
    col = np.float32(np.array([0.9, 0.3, 0.6]))
    expect = col[:, None, None] * a + (1 - a) * out["mesh_rgb"]
    np.testing.assert_allclose(out["image"], expect, atol=2e-7)
    np.testing.assert_allclose(out["final_T"], 1 - a, atol=2e-7)
    assert r > 0


def test_anisotropic_gaussian_pixel_values():
    # one rotated, anisotropic Gaussian seen off-axis: alpha(p) from Eq. 1 with
    # Sigma' built independently (scipy rotation, finite-difference Jacobian)
    rng = np.random.default_rng(14)
    cam = scenes.Camera(48, 40, 45.0, 44.0, 24.3, 19.7, np.eye(3), np.zeros(3))
    for _ in range(5):
        mu = np.array([rng.uniform(-0.3, 0.3), rng.uniform(-0.3, 0.3), rng.uniform(1.5, 3.0)])
        q = rng.standard_normal(4)
        ls = rng.uniform(-2.8, -1.6, 3)
        g = gauss([mu], log_scales=[ls], quats=[q], logits=[rng.normal()], colours=[[1.0, 0.5, 0.25]])
        mu64 = g.means[0].astype(np.float64)
        qq = g.quats[0].astype(np.float64)
        R = Rotation.from_quat([qq[1], qq[2], qq[3], qq[0]]).as_matrix()
        Sig = R @ np.diag(np.exp(g.log_scales[0].astype(np.float64)) ** 2) @ R.T
        h = 1e-6
        Jfd = np.zeros((2, 3))
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            Jfd[:, k] = (_pinhole(cam, mu64 + e) - _pinhole(cam, mu64 - e)) / (2 * h)
        cov = Jfd @ Sig @ Jfd.T + LP * np.eye(2)
        Q = np.linalg.inv(cov)
        m2 = _pinhole(cam, mu64)
        o = 1 / (1 + np.exp(-float(g.opacity_logits[0])))
        out = oracle.render(g, None, cam, params=oracle.default_params(flags=oracle.FP64_RECORDS))
        pr = oracle.project(g, cam)
        x0, x1, y0, y1 = pr["rect"][0]
        for _ in range(40):
            i, j = int(rng.integers(0, 48)), int(rng.integers(0, 40))
            d = np.array([i + 0.5, j + 0.5]) - m2
            a = min(F32(0.99), o * np.exp(-0.5 * d @ Q @ d))
            inside = x0 <= i // 16 < x1 and y0 <= j // 16 < y1
            a = a if (a >= F32(1 / 255) and inside) else 0.0
            np.testing.assert_allclose(out["image"][0, j, i], a, rtol=2e-6, atol=1e-9)


def test_zero_gaussians_give_the_mesh():
    cam = one_cam(32, 32, 32.0)
    g = gauss(np.zeros((0, 3)))
    mesh = quad(z=4.0, half=3.0, rng=np.random.default_rng(7))
    out = oracle.render(g, mesh, cam)
    np.testing.assert_array_equal(out["image"], out["mesh_rgb"])
    np.testing.assert_array_equal(out["final_T"], 1.0)
    assert out["n_contrib"].max() == 0


def test_gaussians_behind_the_mesh_contribute_nothing():
    sc = scenes.config1()
    g = sc.gaussians
    sel = g.means[:, 2] >= 5.0
    out_all = oracle.render(g.subset(sel), sc.mesh, sc.cameras[0])
    np.testing.assert_array_equal(out_all["image"], out_all["mesh_rgb"])
    assert out_all["n_blended"].max() == 0
    # removing them from the full scene leaves the image unchanged
    full = oracle.render(g, sc.mesh, sc.cameras[0])
    front = oracle.render(g.subset(~sel), sc.mesh, sc.cameras[0])
    np.testing.assert_array_equal(full["image"], front["image"])
    np.testing.assert_array_equal(full["n_blended"], front["n_blended"])


def test_weights_plus_transmittance_sum_to_one():
    sc = scenes.config1()
    g = sc.gaussians
    sh = np.zeros_like(g.sh, dtype=np.float64)
    sh[:, 0, :] = 0.5 / scenes.Y00  # colour exactly 1
    g1 = scenes.make_gaussians(g.means, g.log_scales, g.quats, g.opacity_logits, sh, 0)
    out = oracle.render(g1, None, sc.cameras[0])
    for c in range(3):
        np.testing.assert_allclose(out["image"][c] + out["final_T"], 1.0, atol=1e-12)


def test_two_gaussians_front_to_back():
    cam = one_cam(16, 16, 16.0)
    c1, c2 = [0.9, 0.1, 0.2], [0.2, 0.8, 0.4]
    g = gauss([[0, 0, 3.0], [0, 0, 2.0]], log_scales=[[-1.5] * 3, [-1.8] * 3], logits=[1.0, 0.3],
              colours=[c1, c2])
    out = oracle.render(g, None, cam)
    pr = oracle.project(g, cam)
    ii, jj = np.meshgrid(np.arange(16) + 0.5, np.arange(16) + 0.5)

    def alpha(k):
        o = np.float32(pr["opacity"][k])
        var = pr["cov2d"][k, 0]
        a = np.minimum(F32(0.99), o * np.exp(-0.5 * ((ii - 8) ** 2 + (jj - 8) ** 2) * np.float32(1 / var)))
        return np.where(a >= F32(1 / 255), a, 0.0)

    a_front, a_back = alpha(1), alpha(0)  # Gaussian 1 is nearer
    col = lambda c: np.float32(np.array(c))[:, None, None]
    expect = col(c2) * a_front + col(c1) * a_back * (1 - a_front)
    np.testing.assert_allclose(out["image"], expect, atol=1e-6)


# ------------------------------------- transmittance stop and pixel counts --
# A stack of Gaussians on the optical axis of a camera whose principal point
# is the centre of pixel (16, 16): there every Gaussian has G = 1, so its
# alpha is its record opacity (clamped at 0.99) whatever its depth and size,
# and the list of that pixel's tile is the stack in depth order.
def _axis_stack(logits, depths, colours=None, mesh=None):
    cam = scenes.Camera(32, 32, 32.0, 32.0, 16.5, 16.5, np.eye(3), np.zeros(3))
    n = len(logits)
    means = np.column_stack([np.zeros(n), np.zeros(n), np.asarray(depths, np.float64)])
    col = np.tile([0.8, 0.4, 0.2], (n, 1)) if colours is None else colours
    g = gauss(means, log_scales=[[-2.5] * 3] * n, logits=logits, colours=col)
    out = oracle.render(g, mesh, cam)
    return out, g


def _record_alpha(logit):
    """alpha of a Gaussian seen at its centre: the FP32 record opacity
    sigmoid(logit), clamped at alpha_max"""
    o = F32(1.0 / (1.0 + math.exp(-float(np.float32(logit)))))
    return min(o, F32(0.99))


@pytest.mark.parametrize("offset", [+1e-3, -1e-3])
def test_identical_stack_stops_where_transmittance_would_cross_t_min(offset):
    # k identical Gaussians of alpha a leave T_n = (1 - a)^n after n blends. A
    # pixel stops before the first Gaussian that would take T under t_min:
    # n* = floor(ln t_min / ln(1 - a)) + 1 is that Gaussian's 1-based index,
    # n* - 1 Gaussians blend and T = (1 - a)^(n* - 1). Here (1 - a)^4 sits
    # 1e-3 above (4 blend, the 5th stops) or below (3 blend, the 4th stops)
    # t_min.
    t_min = F32(1e-4)
    a_want = 1.0 - (t_min * (1.0 + offset)) ** 0.25
    logit = math.log(a_want / (1.0 - a_want))
    a = _record_alpha(logit)
    k = 8
    out, g = _axis_stack([logit] * k, 2.0 + 0.25 * np.arange(k))
    n_star = math.floor(math.log(t_min) / math.log(1.0 - a)) + 1
    assert n_star == (5 if offset > 0 else 4)
    j = i = 16
    assert out["n_blended"][j, i] == n_star - 1
    assert out["n_contrib"][j, i] == n_star - 1
    assert out["n_processed"][j, i] == n_star
    T = (1.0 - a) ** (n_star - 1)
    assert T >= t_min and T * (1.0 - a) < t_min
    np.testing.assert_allclose(out["final_T"][j, i], T, rtol=1e-12)
    # the colour of a stack of identical colours c: c (1 - T), no mesh: bg = 0
    col = np.float32([0.8, 0.4, 0.2]).astype(np.float64)
    np.testing.assert_allclose(out["image"][:, j, i], col * (1.0 - T), rtol=1e-6)


def test_clamped_stack_stops_at_the_second_gaussian():
    # alpha clamps at fp32(0.99): (1 - 0.99)^2 is just under fp32(1e-4), so
    # the second Gaussian stops the pixel after one blend
    a = _record_alpha(8.0)
    assert a == F32(0.99)
    assert (1.0 - a) ** 2 < F32(1e-4) <= 1.0 - a
    out, _ = _axis_stack([8.0] * 5, [2.0, 2.5, 3.0, 3.5, 4.0])
    assert (out["n_blended"][16, 16], out["n_contrib"][16, 16], out["n_processed"][16, 16]) == (1, 1, 2)
    np.testing.assert_allclose(out["final_T"][16, 16], 1.0 - a, rtol=1e-12)
    # the decision is within the FP32 slack of t_min: tagged ambiguous
    assert out["amb"][16, 16] & oracle.AMB_T


def test_n_contrib_is_the_list_index_of_the_last_blended_gaussian():
    # entries with alpha < 1/255 are skipped but still take a list position:
    # stack [A s A s s A s s] (A: alpha 0.5, s: alpha ~1e-3): blended
    # positions 1, 3, 6, so n_contrib = 6, n_blended = 3, and the list runs
    # out without a stop, so n_processed = 8 and T = 0.5^3
    A, s_ = 0.0, -7.0
    out, _ = _axis_stack([A, s_, A, s_, s_, A, s_, s_], 2.0 + 0.25 * np.arange(8))
    a = _record_alpha(A)
    assert a == 0.5 and _record_alpha(s_) < F32(1 / 255)
    assert (out["n_contrib"][16, 16], out["n_blended"][16, 16], out["n_processed"][16, 16]) == (6, 3, 8)
    np.testing.assert_allclose(out["final_T"][16, 16], 0.125, rtol=1e-14)


def test_mesh_depth_stop_is_strict_and_counts_the_stopping_entry():
    # Sec. 3.4: Gaussians blend only while D_gs < D_m. A quad at z = 5 has
    # D_m = 5 exactly; a Gaussian at exactly 5 stops the pixel (and is the
    # n_processed-th entry), one at the next smaller FP32 depth blends.
    mesh = quad(z=5.0, half=3.0, rng=np.random.default_rng(4))
    below = float(np.nextafter(np.float32(5.0), np.float32(0.0)))
    a = _record_alpha(0.0)
    for z2, nb, npro in ((5.0, 1, 2), (below, 2, 3)):
        out, _ = _axis_stack([0.0, 0.0, 0.0], [4.0, z2, 6.0], mesh=mesh)
        assert out["mesh_depth"][16, 16] == 5.0
        assert (out["n_blended"][16, 16], out["n_contrib"][16, 16], out["n_processed"][16, 16]) == (nb, nb, npro)
        T = (1.0 - a) ** nb
        np.testing.assert_allclose(out["final_T"][16, 16], T, rtol=1e-14)
        Im = out["mesh_rgb"][:, 16, 16]
        col = np.float32([0.8, 0.4, 0.2]).astype(np.float64)
        np.testing.assert_allclose(out["image"][:, 16, 16], col * (1.0 - T) + T * Im, rtol=1e-6)


def test_ambiguous_decisions_enumerate_both_outcomes():
    # the clamped stack's stop is within the slack: the alternative outcome is
    # the second Gaussian blended (T = (1 - a)^2, 2e-6 under t_min), after
    # which the third stops the pixel far from the threshold
    a = _record_alpha(8.0)
    cam = scenes.Camera(32, 32, 32.0, 32.0, 16.5, 16.5, np.eye(3), np.zeros(3))
    g = gauss(np.column_stack([np.zeros(5), np.zeros(5), [2.0, 2.5, 3.0, 3.5, 4.0]]),
              log_scales=[[-2.5] * 3] * 5, logits=[8.0] * 5)
    out = oracle.render(g, None, cam, alts=True)
    assert out["n_alt"][16, 16] == 2
    first, second = out["alts"][16, 16, 0], out["alts"][16, 16, 1]
    np.testing.assert_array_equal(first[3:], [1.0 - a, 1, 1, 2])
    np.testing.assert_allclose(second[3], (1.0 - a) ** 2, rtol=1e-14)
    np.testing.assert_array_equal(second[4:], [2, 2, 3])
    # a pixel without ambiguous decisions has one outcome, the render itself
    assert out["n_alt"][0, 0] == 1
    np.testing.assert_array_equal(out["alts"][0, 0, 0, :3], out["image"][:, 0, 0])


def test_permuting_gaussians_with_distinct_depths():
    sc = scenes.config1()
    g = sc.gaussians
    perm = np.random.default_rng(9).permutation(g.n)
    a = oracle.render(g, sc.mesh, sc.cameras[0])
    b = oracle.render(g.subset(perm), sc.mesh, sc.cameras[0])
    assert len(np.unique(oracle.project(g, sc.cameras[0])["depth_bits"])) == g.n
    np.testing.assert_array_equal(a["image"], b["image"])
    np.testing.assert_array_equal(a["n_contrib"], b["n_contrib"])


def test_window_matches_full_frame():
    sc = scenes.config1()
    full = oracle.render(sc.gaussians, sc.mesh, sc.cameras[0])
    win = oracle.render(sc.gaussians, sc.mesh, sc.cameras[0], window=(16, 8, 48, 40))
    np.testing.assert_array_equal(win["image"], full["image"][:, 8:40, 16:48])
    np.testing.assert_array_equal(win["n_processed"], full["n_processed"][8:40, 16:48])


# ----------------------------------------------------------------- mesh --
def test_config1_quad_depth_and_bilinear_block_mean():
    sc = scenes.config1()
    out = oracle.render(scenes.make_gaussians(np.zeros((0, 3)), np.zeros((0, 3)), np.zeros((0, 4)),
                                              np.zeros(0), np.zeros((0, 1, 3)), 0), sc.mesh, sc.cameras[0])
    assert np.all(out["mesh_depth"] == 5.0)
    tex = sc.mesh.tex[0].astype(np.float64)
    blocks = tex[1:-1].reshape(63, 4, 254 // 1 // 63 if False else 4, 3) if False else None
    for j in range(64):
        for i in range(64):
            ref = tex[4 * j + 1:4 * j + 3, 4 * i + 1:4 * i + 3].mean(axis=(0, 1))
            np.testing.assert_allclose(out["mesh_rgb"][:, j, i], ref, atol=1e-12)


def test_shared_diagonal_is_owned_by_exactly_one_triangle():
    # the quad's diagonal passes through the pixel centres (i+1/2, i+1/2)
    sc = scenes.config1()
    g0 = gauss(np.zeros((0, 3)))
    cov = []
    for f in range(2):
        m = scenes.Mesh(sc.mesh.verts, sc.mesh.faces[f:f + 1], sc.mesh.uvs[f:f + 1],
                        sc.mesh.face_tex[f:f + 1], sc.mesh.tex)
        cov.append(oracle.render(g0, m, sc.cameras[0])["tri_id"] >= 0)
    assert not np.any(cov[0] & cov[1])
    assert np.all(cov[0] | cov[1])


def _box_raycast(cam, mesh_tex, tex_fn=None):
    """Analytic ray cast of the room box: depth and bilinear colour per pixel."""
    H, W = cam.height, cam.width
    ii, jj = np.meshgrid(np.arange(W) + 0.5, np.arange(H) + 0.5)
    dcam = np.stack([(ii - cam.cx) / cam.fx, (jj - cam.cy) / cam.fy, np.ones_like(ii)], -1)
    dw = dcam @ cam.R  # R^T d as rows
    o = cam.centre
    best_t = np.full((H, W), np.inf)
    uv = np.zeros((H, W, 2))
    texid = np.zeros((H, W), int)
    # (axis, value, texture, other axes)
    planes = [(1, 1.5, 0), (1, -1.5, 1), (0, -3.0, 2), (0, 3.0, 2), (2, -2.0, 3), (2, 2.0, 3)]
    for ax, val, tid in planes:
        with np.errstate(divide="ignore", invalid="ignore"):
            t = (val - o[ax]) / dw[..., ax]
        p = o + t[..., None] * dw
        a, b = [d for d in range(3) if d != ax]
        ok = (t > 0) & (t < best_t)
        best_t = np.where(ok, t, best_t)
        u = (p[..., a] - scenes.ROOM_MIN[a]) / (scenes.ROOM_MAX[a] - scenes.ROOM_MIN[a])
        v = (p[..., b] - scenes.ROOM_MIN[b]) / (scenes.ROOM_MAX[b] - scenes.ROOM_MIN[b])
        uv = np.where(ok[..., None], np.stack([u, v], -1), uv)
        texid = np.where(ok, tid, texid)
    return best_t, uv, texid  # t along dcam (z = 1) is the view depth


def test_room_mesh_matches_analytic_raycast():
    rng = np.random.default_rng(11)
    # large triangles: vertices are snapped to 1/256 px, which tilts a small
    # triangle's plane by up to (1/512 px) / (its size in px)
    mesh = scenes.room_mesh(rng, 400, 32)
    # an affine texture: bilinear filtering reproduces it exactly inside the texture
    n_tex, T = 4, 32
    jj, ii = np.meshgrid(np.arange(T), np.arange(T), indexing="ij")
    tex = np.zeros((n_tex, T, T, 3), np.float32)
    for t in range(n_tex):
        for c in range(3):
            tex[t, :, :, c] = 0.1 + 0.02 * (t + 1) * ii / T + 0.015 * (c + 1) * jj / T
    mesh.tex = tex
    g0 = gauss(np.zeros((0, 3)))
    for v in range(4):
        cam = scenes.random_room_camera(np.random.default_rng(100 + v), 160, 120)
        out = oracle.render(g0, mesh, cam)
        depth, uv, texid = _box_raycast(cam, tex)
        assert np.all(out["tri_id"] >= 0)  # the closed box covers every pixel
        # snapping error is ~2e-5 here; affine instead of perspective-correct
        # interpolation would be off by ~1e-3
        np.testing.assert_allclose(out["mesh_depth"], depth, rtol=1e-4)
        x = uv[..., 0] * T - 0.5
        y = uv[..., 1] * T - 0.5
        interior = (x > 0.01) & (x < T - 1.01) & (y > 0.01) & (y < T - 1.01)
        for c in range(3):
            ref = 0.1 + 0.02 * (texid + 1) * (x / T) + 0.015 * (c + 1) * (y / T)
            np.testing.assert_allclose(out["mesh_rgb"][c][interior], ref[interior], atol=2e-5)


def test_bilinear_texel_centre_and_clamp():
    # a quad whose UV maps pixel centres onto texel centres returns the texels
    cam = one_cam(8, 8, 8.0)
    m = scenes.quad_mesh(np.random.default_rng(3), z=1.0, half=0.5, tex_size=8)
    out = oracle.render(gauss(np.zeros((0, 3))), m, cam)
    np.testing.assert_allclose(out["mesh_rgb"], np.transpose(m.tex[0], (2, 0, 1)), atol=1e-12)


# ----------------------------------------------------------------- loss --
def test_loss_mask_values_and_gradient():
    rng = np.random.default_rng(12)
    H, W = 6, 7
    img, tgt, Im = (rng.uniform(0, 1, (3, H, W)) for _ in range(3))
    T = rng.uniform(0, 1, (H, W))
    T[0, 0] = 0.5
    tri = np.where(rng.uniform(size=(H, W)) < 0.7, 3, -1)
    tri[0, 0] = 1
    L, gi, gt, gm = oracle.loss(img, T, Im, tri, tgt)
    MT = 1 / (1 + np.exp(-20 * (T - 0.5)))
    assert MT[0, 0] == 0.5
    # L_t is 0 where no triangle covers the pixel
    assert np.all(gm[:, tri < 0] == 0) and np.all(gt[tri < 0] == 0)
    h = 1e-6
    for arr, g in ((img, gi), (T, gt), (Im, gm)):
        for idx in [tuple(rng.integers(0, s) for s in arr.shape) for _ in range(10)]:
            a0 = arr[idx]
            arr[idx] = a0 + h
            Lp = oracle.loss(img, T, Im, tri, tgt)[0]
            arr[idx] = a0 - h
            Lm = oracle.loss(img, T, Im, tri, tgt)[0]
            arr[idx] = a0
            np.testing.assert_allclose((Lp - Lm) / (2 * h), g[idx], rtol=1e-5, atol=1e-10)


# ------------------------------------------------------------ gradients --
def tiny_scene(seed, n=12, deg=3, with_mesh=True):
    rng = np.random.default_rng(seed)
    means = np.column_stack([rng.uniform(-0.5, 0.5, n), rng.uniform(-0.5, 0.5, n), rng.uniform(1.5, 3.0, n)])
    g = scenes.make_gaussians(means, rng.uniform(-3.0, -1.8, (n, 3)), rng.standard_normal((n, 4)),
                              rng.normal(0, 1, n), np.concatenate(
                                  [((rng.uniform(0, 1, (n, 1, 3)) - 0.5) / scenes.Y00),
                                   rng.normal(0, 0.2, (n, (deg + 1) ** 2 - 1, 3))], 1), deg)
    mesh = None
    if with_mesh:
        mesh = scenes.quad_mesh(rng, z=2.6, half=1.2, tex_size=8)
    cam = scenes.Camera(32, 32, 30.0, 30.0, 16.0, 16.0, np.eye(3), np.zeros(3))
    return g, mesh, cam


@pytest.mark.parametrize("seed", [21, 22])
def test_oracle_gradient_matches_finite_differences(seed):
    _fd_check(seed, oracle.default_params(flags=oracle.FP64_RECORDS), None)


def _fd_check(seed, pr64, filter3d):
    g, mesh, cam = tiny_scene(seed)
    rng = np.random.default_rng(seed + 1)
    gi = rng.normal(size=(3, 32, 32))
    gt = rng.normal(size=(32, 32))
    gm = rng.normal(size=(3, 32, 32))

    def F(over):
        o = oracle.render(g, mesh, cam, params=pr64, overrides=over, filter3d=filter3d)
        return (np.sum(gi * o["image"]) + np.sum(gt * o["final_T"]) + np.sum(gm * o["mesh_rgb"]),
                o["trace"])

    an = oracle.backward(g, mesh, cam, gi, gt, gm, params=pr64, filter3d=filter3d)
    base = dict(means=g.means.astype(np.float64), log_scales=g.log_scales.astype(np.float64),
                quats=g.quats.astype(np.float64), opacity_logits=g.opacity_logits.astype(np.float64),
                sh=g.sh.astype(np.float64))
    checked = 0
    for name, arr in base.items():
        flat = arr.reshape(-1)
        for idx in rng.choice(flat.size, size=min(flat.size, 25), replace=False):
            h = 1e-6 * max(1.0, abs(flat[idx]))
            over = {k: v.copy() for k, v in base.items()}
            over[name].reshape(-1)[idx] = flat[idx] + h
            fp, tp = F(over)
            over[name].reshape(-1)[idx] = flat[idx] - h
            fm, tm = F(over)
            if tp != tm:
                continue  # a decision flipped between the two evaluations
            fd = (fp - fm) / (2 * h)
            ref = an[name].reshape(-1)[idx]
            assert abs(fd - ref) <= 1e-6 * max(1.0, abs(ref)), (name, idx, fd, ref)
            checked += 1
    assert checked > 80
    # the image is linear in the texture: exact differences with a large step
    tex = mesh.tex.copy()
    for idx in rng.choice(tex.size, 20, replace=False):
        t2 = tex.copy()
        t2.reshape(-1)[idx] += 0.25
        fp, _ = F(dict(base, tex=t2))
        t2.reshape(-1)[idx] -= 0.5
        fm, _ = F(dict(base, tex=t2))
        assert abs((fp - fm) / 0.5 - an["tex"].reshape(-1)[idx]) < 1e-9


def test_texture_gradient_mass_equals_mesh_gradient_mass():
    # bilinear weights sum to 1, so sum(dL/dtex) = sum over pixels of dL/dI_m
    g, mesh, cam = tiny_scene(31)
    rng = np.random.default_rng(5)
    gm = rng.normal(size=(3, 32, 32))
    an = oracle.backward(g, mesh, cam, np.zeros((3, 32, 32)), None, gm)
    out = oracle.render(g, mesh, cam)
    has = out["tri_id"] >= 0
    for c in range(3):
        np.testing.assert_allclose(an["tex"][..., c].sum(), gm[c][has].sum(), rtol=1e-12)


def test_single_gaussian_opacity_derivative_closed_form():
    # dC/do = G (c - I_m) for one unclamped Gaussian over the mesh
    cam = one_cam(16, 16, 16.0)
    g = gauss([[0, 0, 2.0]], log_scales=[[-1.2] * 3], logits=[-1.0], colours=[[0.8, 0.2, 0.5]])
    mesh = quad(z=4.0, half=3.0, rng=np.random.default_rng(2))
    pr64 = oracle.default_params(flags=oracle.FP64_RECORDS)
    out = oracle.render(g, mesh, cam, params=pr64)
    pr = oracle.project(g, cam)
    j, i = 9, 7
    gi = np.zeros((3, 16, 16))
    gi[1, j, i] = 1.0
    an = oracle.backward(g, mesh, cam, gi, None, None, params=pr64)
    var = pr["cov2d"][0, 0]
    G = math.exp(-0.5 * ((i + 0.5 - 8) ** 2 + (j + 0.5 - 8) ** 2) / var)
    o = pr["opacity"][0]
    dC_do = G * (pr["rgb"][0, 1] - out["mesh_rgb"][1, j, i])
    np.testing.assert_allclose(an["opacity_logits"][0], dC_do * o * (1 - o), rtol=1e-10)


# ------------------------------------------------------- full loss (Eq. 3) --
def _ssim_scipy(x, y, c1=0.01 ** 2, c2=0.03 ** 2):
    from scipy.ndimage import correlate
    w = oracle.ssim_window()
    out = []
    for c in range(3):
        cv = lambda z: correlate(z, w, mode="constant", cval=0.0)
        mx, my = cv(x[c]), cv(y[c])
        sxx = cv(x[c] * x[c]) - mx * mx
        syy = cv(y[c] * y[c]) - my * my
        sxy = cv(x[c] * y[c]) - mx * my
        out.append(((2 * mx * my + c1) * (2 * sxy + c2)) / ((mx * mx + my * my + c1) * (sxx + syy + c2)))
    return np.stack(out)


def test_full_loss_ssim_pins():
    rng = np.random.default_rng(40)
    H, W = 23, 31
    x, y = rng.uniform(0, 1, (3, H, W)), rng.uniform(0, 1, (3, H, W))
    T = rng.uniform(0, 1, (H, W))
    tri = -np.ones((H, W), np.int32)
    Im = np.zeros((3, H, W))
    # identical images: SSIM = 1 everywhere, the loss is 0
    L, gi, gt, gm = oracle.full_loss([x], [T], [Im], [tri], [x])
    assert abs(L) < 1e-12
    # against an independent correlation (scipy), zero padding
    L, gi, gt, gm = oracle.full_loss([x], [T], [Im], [tri], [y], mask_mode="none")
    s = _ssim_scipy(x, y)
    ref = 0.8 * np.abs(x - y).mean() + 0.2 * (1 - s.mean())
    np.testing.assert_allclose(L, ref, rtol=1e-12)
    # constant images a, b: SSIM = (2ab + C1) / (a^2 + b^2 + C1) away from the borders
    a, b = 0.3, 0.7
    s = _ssim_scipy(np.full((3, H, W), a), np.full((3, H, W), b))
    np.testing.assert_allclose(s[:, 5:-5, 5:-5], (2 * a * b + 1e-4) / (a * a + b * b + 1e-4), rtol=1e-12)
    # window: normalised, symmetric, sigma 1.5
    w = oracle.ssim_window()
    assert abs(w.sum() - 1) < 1e-15 and np.allclose(w, w.T) and np.allclose(w, w[::-1])


def test_full_loss_gradient_and_mask_variants():
    rng = np.random.default_rng(41)
    H, W = 14, 17
    x, y, Im = (rng.uniform(0, 1, (3, H, W)) for _ in range(3))
    T = rng.uniform(0, 1, (H, W))
    tri = np.where(rng.uniform(size=(H, W)) < 0.6, 1, -1).astype(np.int32)
    for mode in oracle.MASK_MODES:
        L, gi, gt, gm = oracle.full_loss([x], [T], [Im], [tri], [y], mask_mode=mode)
        h = 1e-6
        for arr, g in ((x, gi[0]), (T, gt[0]), (Im, gm[0])):
            for idx in [tuple(rng.integers(0, s) for s in arr.shape) for _ in range(6)]:
                a0 = arr[idx]
                arr[idx] = a0 + h
                lp = oracle.full_loss([x], [T], [Im], [tri], [y], mask_mode=mode)[0]
                arr[idx] = a0 - h
                lm = oracle.full_loss([x], [T], [Im], [tri], [y], mask_mode=mode)[0]
                arr[idx] = a0
                np.testing.assert_allclose((lp - lm) / (2 * h), g[idx], rtol=1e-5, atol=1e-10)
    # L_t reduces to the paper's sigmoid mask: M_T(0.5) = 1/2 and no term without a triangle
    Ls = oracle.full_loss([x], [np.full((H, W), 0.5)], [Im], [tri], [y], mask_mode="sigmoid")[0]
    L0 = oracle.full_loss([x], [np.full((H, W), 0.5)], [Im], [tri], [y], mask_mode="none")[0]
    d = np.where(tri >= 0, y - Im, 0)
    np.testing.assert_allclose(Ls - L0, 0.1 * 0.5 * (d * d).sum() / x.size, rtol=1e-12)


# ------------------------------------------------- training-step oracles --
def test_mean2d_gradient_is_the_principal_point_derivative():
    # shifting (cx, cy) moves every projected mean by the same amount and
    # changes nothing else of a Gaussians-only frame, so dF/dcx = sum_g dF/du_g
    g, _, cam = tiny_scene(41, n=6, with_mesh=False)
    rng = np.random.default_rng(4)
    pr64 = oracle.default_params(flags=oracle.FP64_RECORDS)
    gi = rng.normal(size=(3, 32, 32))
    gt = rng.normal(size=(32, 32))
    an = oracle.backward(g, None, cam, gi, gt, None, params=pr64)

    def F(gs, dcx, dcy):
        c = scenes.Camera(cam.width, cam.height, cam.fx, cam.fy, cam.cx + dcx, cam.cy + dcy,
                          cam.R, cam.t)
        o = oracle.render(gs, None, c, params=pr64)
        return np.sum(gi * o["image"]) + np.sum(gt * o["final_T"]), o["trace"]

    h = 1e-6
    for gs, ref in [(g, an["mean2d"].sum(0))] + [
            (g.subset(np.array([j])), None) for j in range(3)]:
        if ref is None:
            ref = oracle.backward(gs, None, cam, gi, gt, None, params=pr64)["mean2d"][0]
        for axis in range(2):
            d = [0.0, 0.0]
            d[axis] = h
            fp, tp = F(gs, *d)
            fm, tm = F(gs, -d[0], -d[1])
            assert tp == tm
            fd = (fp - fm) / (2 * h)
            assert abs(fd - ref[axis]) <= 1e-6 * max(1.0, abs(ref[axis])), (axis, fd, ref[axis])


def test_adam_matches_torch_optim_and_the_first_step_closed_form():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(8)
    K3 = 12  # one SH row of degree 1: 4 coefficients x 3 channels
    p0 = rng.normal(size=5 * K3)
    grads = [rng.normal(size=p0.size) * s for s in (1.0, 1e-3, 10.0, 0.5)]
    lr, lr_dc = 1e-2, 3e-2
    # torch reference: the head columns form their own parameter group
    head = (np.arange(p0.size) % K3) < 3
    t_dc = torch.tensor(p0[head], dtype=torch.float64, requires_grad=True)
    t_rest = torch.tensor(p0[~head], dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([{"params": [t_dc], "lr": lr_dc}, {"params": [t_rest], "lr": lr}],
                           betas=(0.9, 0.999), eps=1e-15)
    p, m, v = p0.copy(), np.zeros_like(p0), np.zeros_like(p0)
    for step, gr in enumerate(grads, 1):
        p, m, v = oracle.adam(p, gr, m, v, lr, step, lr_head=lr_dc, head=3, row=K3)
        t_dc.grad = torch.tensor(gr[head])
        t_rest.grad = torch.tensor(gr[~head])
        opt.step()
        np.testing.assert_allclose(p[head], t_dc.detach().numpy(), rtol=0, atol=1e-13)
        np.testing.assert_allclose(p[~head], t_rest.detach().numpy(), rtol=0, atol=1e-13)
        if step == 1:
            # bias correction makes the first step lr * g / (|g| + eps)
            rate = np.where(head, lr_dc, lr)
            np.testing.assert_allclose(p, p0 - rate * gr / (np.abs(gr) + 1e-15), rtol=0, atol=1e-15)


def test_lambda_t_schedule_boundaries():
    # Alg. 1: L_t only strictly after the warm-up and strictly before the end of densification
    assert oracle.lambda_t_schedule(0) == 0.0
    assert oracle.lambda_t_schedule(3000) == 0.0
    assert oracle.lambda_t_schedule(3001) == 0.1
    assert oracle.lambda_t_schedule(14999) == 0.1
    assert oracle.lambda_t_schedule(15000) == 0.0
    assert oracle.lambda_t_schedule(29999) == 0.0


# ------------------------------------------------- mesh-depth culling --
def _cull_scene(seed):
    rng = np.random.default_rng(seed)
    n = 80
    means = np.column_stack([rng.uniform(-1.2, 1.2, n), rng.uniform(-0.9, 0.9, n), rng.uniform(1.5, 3.2, n)])
    g = scenes.make_gaussians(means, rng.uniform(-3.0, -1.8, (n, 3)), rng.standard_normal((n, 4)),
                              rng.normal(0, 1, n), ((rng.uniform(0, 1, (n, 1, 3)) - 0.5) / scenes.Y00), 0)
    # a tilted quad that covers the whole view, so every tile is covered
    mesh = scenes.quad_mesh(rng, z=2.6, half=3.0, tex_size=8)
    mesh.verts[:, 2] += 0.2 * mesh.verts[:, 0]
    cam = scenes.Camera(64, 48, 40.0, 40.0, 32.0, 24.0, np.eye(3), np.zeros(3))
    return g, mesh, cam


def test_mesh_depth_culling_keeps_the_image_and_drops_only_stopped_pairs():
    g, mesh, cam = _cull_scene(51)
    base = oracle.render(g, mesh, cam)
    pc = oracle.default_params(flags=oracle.CULL_MESH)
    cut = oracle.render(g, mesh, cam, params=pc)
    assert (base["tri_id"] >= 0).all()
    for k in ("image", "final_T", "n_contrib", "n_blended", "tri_id", "mesh_rgb"):
        np.testing.assert_array_equal(cut[k], base[k])
    dp = base["n_processed"] - cut["n_processed"]
    assert dp.min() >= 0 and dp.max() <= 1 and dp.sum() > 0
    # the key sets: the uncut keys minus the pairs whose depth is not below the
    # tile's largest mesh depth (from the rendered depth map)
    k0, v0, _ = oracle.keys(g, cam)
    k1, v1, r1 = oracle.keys(g, cam, params=pc, mesh=mesh)
    TX = 4
    dmax = base["mesh_depth"].reshape(3, 16, TX, 16).max(axis=(1, 3)).reshape(-1).astype(np.float32)
    tile = (k0 >> np.uint64(32)).astype(np.int64)
    depth = (k0 & np.uint64(0xffffffff)).astype(np.uint32).view(np.float32)
    keep = depth < dmax[tile]
    assert 0 < (~keep).sum() < keep.size
    np.testing.assert_array_equal(k1, k0[keep])
    np.testing.assert_array_equal(v1, v0[keep])
    counts = np.bincount(tile[keep], minlength=12)
    np.testing.assert_array_equal(r1[:, 1] - r1[:, 0], counts)


def test_mesh_depth_culling_leaves_tiles_with_an_uncovered_pixel():
    g, _, cam = _cull_scene(52)
    rng = np.random.default_rng(3)
    small = scenes.quad_mesh(rng, z=2.6, half=0.5, tex_size=8)  # covers only part of the view
    pc = oracle.default_params(flags=oracle.CULL_MESH)
    base = oracle.render(g, small, cam)
    cut = oracle.render(g, small, cam, params=pc)
    for k in ("image", "final_T", "n_contrib", "n_blended", "n_processed"):
        np.testing.assert_array_equal(cut[k], base[k])
    k0, _, _ = oracle.keys(g, cam)
    k1, _, _ = oracle.keys(g, cam, params=pc, mesh=small)
    np.testing.assert_array_equal(k0, k1)



# ------------------------------------------- Mip-Splatting filters (host method) --
def test_mip_filters_on_a_centred_isotropic_gaussian():
    # 3D smoothing adds f3 to every variance and scales the opacity by
    # (s^2 / (s^2 + f3))^(3/2); the 2D filter keeps low_pass as the pixel
    # filter and scales the opacity by sqrt(det / det_filtered) = v / (v + k)
    cam = one_cam()
    k = F32(0.1)
    pm = oracle.default_params(low_pass=0.1, flags=oracle.MIP_2D)
    for z, ls, f3 in ((2.0, -3.0, 2e-3), (3.5, -2.2, 1e-2), (5.0, -4.0, 0.0)):
        g = gauss([[0, 0, z]], log_scales=[[ls] * 3], logits=[0.7])
        pr = oracle.project(g, cam, params=pm, filter3d=np.array([f3]))
        s2 = math.exp(float(np.float32(ls))) ** 2
        v = (64.0 / z) ** 2 * (s2 + f3)
        np.testing.assert_allclose(pr["cov2d"][0], [v + k, 0.0, v + k], rtol=1e-13, atol=1e-15)
        op = 1 / (1 + math.exp(-float(np.float32(0.7))))
        want = op * (s2 / (s2 + f3)) ** 1.5 * v / (v + k)
        np.testing.assert_allclose(pr["opacity"][0], want, rtol=1e-13)


def test_mip_2d_filter_preserves_the_unfiltered_mass():
    # the compensated opacity makes the filtered footprint carry the mass of
    # the unfiltered one: sum over pixels of alpha = 2 pi o sqrt(det Sigma'_0),
    # less the tail under alpha_min (2 pi alpha_min sqrt(det Sigma')); a
    # footprint of variance ~0.3 px^2 sampled on the pixel grid sums to its
    # integral within ~1e-3 (Poisson summation)
    cam = one_cam()
    pm = oracle.default_params(low_pass=0.1, flags=oracle.MIP_2D)
    for ls, u0 in ((-3.5, 0.3), (-3.3, 0.71), (-3.66, 0.5)):
        g = gauss([[u0 * 3.0 / 64, -0.2 * 3.0 / 64, 3.0]], log_scales=[[ls] * 3], logits=[3.0],
                  colours=[[1.0, 1.0, 1.0]])
        out = oracle.render(g, None, cam, params=pm)
        v0 = (64.0 / 3.0 * math.exp(float(np.float32(ls)))) ** 2
        k = F32(0.1)
        op = 1 / (1 + math.exp(-3.0))
        want = 2 * math.pi * (op * v0 - F32(1 / 255) * (v0 + k))
        got = out["image"][0].sum()
        assert abs(got / want - 1) < 1e-2, (ls, got, want)


def test_mip_3d_filter_is_the_highest_sampling_rate_over_the_views():
    # A at the origin; B one unit further back; C facing away. fx = 100, 64x64.
    mk = lambda R, t: scenes.Camera(64, 64, 100.0, 100.0, 32.0, 32.0, np.asarray(R, float), np.asarray(t, float))
    A = mk(np.eye(3), [0, 0, 0])
    B = mk(np.eye(3), [0, 0, 2.0])
    C = mk(np.diag([-1.0, 1.0, -1.0]), [0, 0, 0])
    g = gauss([[0, 0, 4.0], [10.0, 0, 4.0], [0.5, 0, 8.0], [0.0, 0.0, -4.0]])
    f3 = oracle.mip_filter3d(g, [A, B, C], s=0.2)
    nu1 = 100.0 / 4.0        # A sees it at depth 4, B at 6, C not at all
    nu3 = 100.0 / 8.0        # A at depth 8, B at 10
    nu4 = 100.0 / 4.0        # only C sees it (at depth 4)
    np.testing.assert_allclose(f3[0], 0.2 / nu1 ** 2, rtol=1e-12)
    np.testing.assert_allclose(f3[2], 0.2 / nu3 ** 2, rtol=1e-12)
    np.testing.assert_allclose(f3[3], 0.2 / nu4 ** 2, rtol=1e-12)
    # outside every view (u = 282 in A): the largest variance of the seen ones
    np.testing.assert_allclose(f3[1], 0.2 / nu3 ** 2, rtol=1e-12)


@pytest.mark.parametrize("seed", [23, 24])
def test_oracle_gradient_with_mip_filters_matches_finite_differences(seed):
    g, _, _ = tiny_scene(seed)
    f3 = np.random.default_rng(seed).uniform(0.2, 1.0, g.n) * np.exp(2 * g.log_scales.astype(np.float64)).mean(1)
    pm = oracle.default_params(low_pass=0.1, flags=oracle.FP64_RECORDS | oracle.MIP_2D)
    _fd_check(seed, pm, f3)


# ---------------------------------------------------- tile-ellipse culling --
def _ellipse_scene(seed, n=120):
    rng = np.random.default_rng(seed)
    means = np.column_stack([rng.uniform(-1.2, 1.2, n), rng.uniform(-0.9, 0.9, n), rng.uniform(1.5, 4.0, n)])
    ls = rng.uniform(-4.0, -1.8, (n, 3))
    ls[:, 0] += rng.uniform(0, 1.5, n)  # elongated
    g = scenes.make_gaussians(means, ls, rng.standard_normal((n, 4)), rng.normal(-1.0, 2.0, n),
                              ((rng.uniform(0, 1, (n, 1, 3)) - 0.5) / scenes.Y00), 0)
    cam = scenes.Camera(96, 80, 60.0, 60.0, 48.0, 40.0, np.eye(3), np.zeros(3))
    return g, cam


def test_tile_ellipse_keeps_every_pair_a_pixel_blends_and_the_image():
    g, cam = _ellipse_scene(71)
    pe = oracle.default_params(flags=oracle.TILE_ELLIPSE)
    base = oracle.render(g, None, cam)
    cut = oracle.render(g, None, cam, params=pe)
    for k in ("image", "final_T", "n_blended"):
        np.testing.assert_array_equal(cut[k], base[k])
    # positions in the shorter lists
    assert (cut["n_processed"] <= base["n_processed"]).all()
    assert (cut["n_contrib"] <= base["n_contrib"]).all()
    k0, v0, _ = oracle.keys(g, cam)
    k1, v1, _ = oracle.keys(g, cam, params=pe)
    assert len(k1) < 0.7 * len(k0)
    kept = set(zip((k1 >> np.uint64(32)).tolist(), v1.tolist()))
    assert kept <= set(zip((k0 >> np.uint64(32)).tolist(), v0.tolist()))
    # brute force: every dropped (Gaussian, tile) pair has alpha < alpha_min
    # at all of the tile's pixel centres (records as the blend reads them)
    pr = oracle.project(g, cam)
    amin = F32(1 / 255)
    TX = 6
    dropped = 0
    for key, gi in zip(k0.tolist(), v0.tolist()):
        t = key >> 32
        if (t, gi) in kept:
            continue
        dropped += 1
        tx, ty = t % TX, t // TX
        xs = np.arange(tx * 16, min(tx * 16 + 16, cam.width)) + 0.5
        ys = np.arange(ty * 16, min(ty * 16 + 16, cam.height)) + 0.5
        dx = xs[None, :] - F32(pr["mean2d"][gi, 0])
        dy = ys[:, None] - F32(pr["mean2d"][gi, 1])
        a, b, c = (F32(x) for x in pr["conic"][gi])
        power = -0.5 * (a * dx * dx + c * dy * dy) - b * dx * dy
        alpha = F32(pr["opacity"][gi]) * np.exp(power)
        assert alpha.max() < amin, (t, gi, alpha.max())
    assert dropped > 100


def _box_min_quadratic(a, b, c, x0, x1, y0, y1):
    """min of a x^2 + 2 b x y + c y^2 (positive definite) over [x0,x1] x [y0,y1]:
    0 when the origin is inside, else the least of the four edge minima (each
    a 1-D quadratic minimised at its clamped vertex)."""
    if x0 <= 0.0 <= x1 and y0 <= 0.0 <= y1:
        return 0.0
    f = lambda x, y: a * x * x + 2 * b * x * y + c * y * y
    best = math.inf
    for x in (x0, x1):
        y = min(max(-b * x / c, y0), y1)
        best = min(best, f(x, y))
    for y in (y0, y1):
        x = min(max(-b * y / a, x0), x1)
        best = min(best, f(x, y))
    return best


def test_tile_ellipse_key_set_is_the_grown_ellipse_meeting_the_tile():
    # The cut keeps a (Gaussian, tile) pair of the 3-sigma rectangle exactly
    # when the tile's 16x16 pixel-centre box meets the ellipse d^T Q d <= R'
    # around the record's mean (Q its conic), R' = 1.01 R + 0.1 + 1e-5 (a+c)
    # ext^2 grown from R = 2 ln(opacity / alpha_min) (ext: the rectangle's
    # longer side in pixels). Recomputed here by minimising the quadratic form
    # over each box, independent of the oracle's row-by-row x-extent method.
    g, cam = _ellipse_scene(72, n=160)
    pe = oracle.default_params(flags=oracle.TILE_ELLIPSE)
    k0, v0, _ = oracle.keys(g, cam)
    k1, v1, _ = oracle.keys(g, cam, params=pe)
    kept = set(zip((k1 >> np.uint64(32)).tolist(), v1.tolist()))
    pr = oracle.project(g, cam)
    TX = 6
    amin = F32(1 / 255)
    n_keep = n_drop = 0
    for key, gi in zip(k0.tolist(), v0.tolist()):
        t = key >> 32
        tx, ty = t % TX, t // TX
        a, b, c = (F32(x) for x in pr["conic"][gi])
        u, v = (F32(x) for x in pr["mean2d"][gi])
        o = F32(pr["opacity"][gi])
        x0r, x1r, y0r, y1r = pr["rect"][gi]
        if not (a > 0 and c > 0 and a * c - b * b > 0):
            want = True
        elif o <= amin:
            want = False
        else:
            R = 2.0 * (math.log(o) - math.log(amin))
            ext = 16.0 * max(x1r - x0r, y1r - y0r)
            Rp = 1.01 * R + 0.1 + 1e-5 * (a + c) * ext * ext
            m = _box_min_quadratic(a, b, c, 16 * tx + 0.5 - u, 16 * tx + 15.5 - u,
                                   16 * ty + 0.5 - v, 16 * ty + 15.5 - v)
            if abs(m - Rp) <= 1e-9 * Rp:
                continue  # on the boundary: either answer is right
            want = m <= Rp
        assert ((t, gi) in kept) == want, (t, gi)
        n_keep += want
        n_drop += not want
    assert n_keep > 100 and n_drop > 100
    # nothing outside the rectangle's pairs is kept
    assert kept <= set(zip((k0 >> np.uint64(32)).tolist(), v0.tolist()))


def test_tile_ellipse_counts_are_positions_in_the_cut_lists():
    # Every pair the cut drops is skipped by every pixel of its tile, so a
    # pixel of the cut render blends the same Gaussians as the uncut one and
    # stops at the same entry, or - when that entry (a mesh-depth stop) was
    # dropped - at the next kept one, which lies behind the mesh too. Hence
    # n_contrib = kept entries among the first n_contrib of the uncut list;
    # n_processed = kept entries among the first n_processed, plus one when the
    # terminating entry was dropped and kept entries follow it.
    rng = np.random.default_rng(73)
    g, cam = _ellipse_scene(73, n=140)
    mesh = scenes.quad_mesh(rng, z=2.9, half=3.0, tex_size=8)  # stops some pixels
    pe = oracle.default_params(flags=oracle.TILE_ELLIPSE)
    base = oracle.render(g, mesh, cam)
    cut = oracle.render(g, mesh, cam, params=pe)
    for k in ("image", "final_T", "n_blended"):
        np.testing.assert_array_equal(cut[k], base[k])
    k0, v0, r0 = oracle.keys(g, cam)
    k1, v1, _ = oracle.keys(g, cam, params=pe)
    kept = set(zip((k1 >> np.uint64(32)).tolist(), v1.tolist()))
    TX = 6
    stopped_on_dropped = 0
    for t in range(r0.shape[0]):
        lst = v0[r0[t, 0]:r0[t, 1]].tolist()
        keep = np.array([(t, gi) in kept for gi in lst], bool)
        csum = np.concatenate([[0], np.cumsum(keep)])
        tx, ty = t % TX, t // TX
        for j in range(16 * ty, min(16 * ty + 16, cam.height)):
            for i in range(16 * tx, min(16 * tx + 16, cam.width)):
                nc, npro = base["n_contrib"][j, i], base["n_processed"][j, i]
                assert cut["n_contrib"][j, i] == csum[nc]
                extra = int(npro > 0 and not keep[npro - 1] and csum[-1] > csum[npro])
                stopped_on_dropped += extra
                assert cut["n_processed"][j, i] == csum[npro] + extra, (t, j, i)
    assert stopped_on_dropped > 0
