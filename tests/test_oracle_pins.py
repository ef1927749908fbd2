"""Pins of the CPU oracle against facts the paper and mathematics fix
independently of the oracle's own code: brute-force minimisation along rays,
closed forms, the propositions of the appendix, invariants, an independent
library for the SH basis, and brute-force rendering of tiny scenes."""
import math

import numpy as np
import pytest
from scipy import special

import oracle
import scenegen

OPTS = scenegen.default_options()


def _rot(rng):
    a = rng.standard_normal((3, 3))
    q, r = np.linalg.qr(a)
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    return q


def _sigma_inv(Rp, s):
    # independent route: invert the covariance R S^2 R^T numerically
    return np.linalg.inv(Rp @ np.diag(np.asarray(s) ** 2) @ Rp.T)


def _brute_min_along_ray(mu, Sinv, x):
    """min over alpha of (alpha x - mu)^T Sinv (alpha x - mu) by dense sampling
    plus golden-section refinement (no closed form used)."""
    f = lambda a: (a * x - mu) @ Sinv @ (a * x - mu)  # noqa: E731
    scale = np.linalg.norm(mu) / np.linalg.norm(x)
    grid = np.linspace(-4 * scale, 4 * scale, 20001)
    vals = np.array([f(a) for a in grid])
    k = int(np.argmin(vals))
    lo, hi = grid[max(k - 1, 0)], grid[min(k + 1, len(grid) - 1)]
    g = (math.sqrt(5) - 1) / 2
    for _ in range(200):
        c, d = hi - g * (hi - lo), lo + g * (hi - lo)
        if f(c) < f(d):
            hi = d
        else:
            lo = c
    a = 0.5 * (lo + hi)
    return f(a), a


# ----------------------------------------------------------------- D_ray, eq. (5)
def test_divergence_matches_brute_force_minimum(oracle_lib):
    """Prop. A.1: tau(x) x is the point of maximum density along the ray and
    D_ray is the Mahalanobis distance there."""
    rng = np.random.default_rng(1)
    for _ in range(40):
        Rp = _rot(rng)
        s = np.exp(rng.normal(-1.0, 0.7, 3))
        mu = rng.normal(0, 1, 3) + np.array([0, 0, 4.0])
        x = np.array([rng.uniform(-0.6, 0.6), rng.uniform(-0.6, 0.6), 1.0])
        D, tau, e = oracle.divergence(mu, Rp.reshape(-1), s, x)
        Db, ab = _brute_min_along_ray(mu, _sigma_inv(Rp, s), x)
        assert abs(D - Db) <= 1e-9 * max(1.0, Db)
        assert abs(tau - ab) <= 1e-6 * max(1.0, abs(ab))
        np.testing.assert_allclose(e, tau * x - mu, rtol=0, atol=1e-12 * np.linalg.norm(mu))


def test_divergence_isotropic_closed_form(oracle_lib):
    """Sigma = s^2 I, unit ray x: D = (|mu|^2 - (x.mu)^2) / s^2."""
    rng = np.random.default_rng(2)
    for _ in range(50):
        s = math.exp(rng.normal(-2, 0.5))
        mu = rng.normal(0, 1, 3) + [0, 0, 3.0]
        x = rng.normal(0, 1, 3)
        x /= np.linalg.norm(x)
        D, _, _ = oracle.divergence(mu, np.eye(3).reshape(-1), [s, s, s], x)
        ref = (mu @ mu - (x @ mu) ** 2) / s**2
        assert abs(D - ref) <= 1e-9 * max(1.0, ref)


def test_divergence_on_axis_anisotropic_closed_form(oracle_lib):
    """mu = (0,0,d), Sigma = diag(sx^2, sy^2, sz^2), x = (px, py, 1):
    D = d^2 q / (1 + sz^2 q) with q = px^2/sx^2 + py^2/sy^2; tends to the
    linearised (GS) divergence d^2 q as sz -> 0 (Sec. 3.1)."""
    rng = np.random.default_rng(3)
    for _ in range(50):
        d = rng.uniform(1, 10)
        sx, sy, sz = np.exp(rng.normal(-2, 0.5, 3))
        px, py = rng.uniform(-0.3, 0.3, 2)
        q = px**2 / sx**2 + py**2 / sy**2
        D, _, _ = oracle.divergence([0, 0, d], np.eye(3).reshape(-1), [sx, sy, sz], [px, py, 1.0])
        ref = d * d * q / (1 + sz * sz * q)
        assert abs(D - ref) <= 1e-10 * max(1.0, ref)
    D, _, _ = oracle.divergence([0, 0, 5.0], np.eye(3).reshape(-1), [0.1, 0.2, 1e-9], [0.01, 0.02, 1.0])
    assert abs(D - 25 * (0.01**2 / 0.01 + 0.02**2 / 0.04)) < 1e-9


def test_full_support_when_camera_inside(oracle_lib):
    """Prop. A.2: c^2 <= kappa implies omega >= p_min on every ray, and the
    oracle skips such a Gaussian (eq. 6)."""
    rng = np.random.default_rng(4)
    mu = np.array([0.1, -0.05, 0.5])
    s = np.array([0.4, 0.3, 0.5])
    o = 0.9
    kappa = -2 * math.log(OPTS["p_min"] / o)
    c2 = mu @ _sigma_inv(np.eye(3), s) @ mu
    assert c2 <= kappa
    for _ in range(200):
        x = rng.normal(0, 1, 3)
        D, _, _ = oracle.divergence(mu, np.eye(3).reshape(-1), s, x)
        assert o * math.exp(-D / 2) >= OPTS["p_min"]
    scene = dict(means=mu[:, None].astype(np.float32), log_scales=np.log(s)[:, None].astype(np.float32),
                 quats=np.array([[1.0], [0], [0], [0]], np.float32),
                 opacity_logits=np.array([math.log(o / (1 - o))], np.float32),
                 sh=np.zeros((1, 3, 1), np.float32), sh_degree=0)
    cam = scenegen.pinhole(np.concatenate([np.eye(3), np.zeros((3, 1))], 1), 16, 16, 60)
    sp = oracle.preprocess(scene, cam, OPTS)
    assert sp["cull"][0] == oracle.CULL["inside"]


# ------------------------------------------------------- quad of Sec. 4.1 / App. A
def _visible_splats(seed, n=200):
    sc = scenegen.tiny_scene(seed, n, sh_degree=0, log_scale_mean=-2.5, log_scale_std=0.8)
    cam = scenegen.pinhole(scenegen.look_at((0, 0, -3.5)), 96, 80, 70)
    sp = oracle.preprocess(sc, cam, OPTS)
    return sc, cam, sp[sp["cull"] == 0]


def test_rotation_aligning_v_to_mu_hat(oracle_lib):
    """App. A.1: R v = mu^, R in SO(3), for mu^_z >= 0 and < 0 (incl. mu^ = -v)."""
    rng = np.random.default_rng(5)
    cases = [rng.normal(0, 1, 3) for _ in range(100)] + [np.array([0, 0, -1.0]), np.array([0, 0, 1.0])]
    for m in cases:
        m = m / np.linalg.norm(m)
        R = oracle.rot_mu_v(m)
        np.testing.assert_allclose(R @ [0, 0, 1.0], m, atol=1e-14)
        np.testing.assert_allclose(R @ R.T, np.eye(3), atol=1e-14)
        assert abs(np.linalg.det(R) - 1) < 1e-13


def test_quad_geometry_identities(oracle_lib):
    """eq. (8) / Prop. A.5: points e = Phi^-1(u) of the ellipse satisfy
    e^T Sinv e = e^T Sinv mu = c^2 - kappa, tau(e) = 1 (Prop. A.4) and
    D(e) = kappa.  App. A.3: V_ray = c^2/(c^2-kappa) Phi^-1(U O).  eq. (14):
    u1 is the top eigenvector of B.  The quad is a rectangle on the plane
    p^T Sinv mu = c^2."""
    O = np.array([[-1, -1, 1, 1], [-1, 1, 1, -1]], float)
    for seed in (6, 7):
        _, _, sp = _visible_splats(seed)
        assert len(sp) > 50
        for r in sp:
            Rp, s, mu = r["Rp"].reshape(3, 3), r["s"], r["mu"]
            Sinv = _sigma_inv(Rp, s)
            c2 = mu @ Sinv @ mu
            kappa = r["kappa"]
            assert abs(c2 - r["c2"]) <= 1e-10 * c2
            c = math.sqrt(c2)
            a = math.sqrt(kappa / (c2 - kappa))
            Q = Rp @ np.diag(s) @ r["Rv"].reshape(3, 3)
            phi_inv = lambda u: (c2 - kappa) / c * Q @ np.array([a * u[0], a * u[1], 1.0])  # noqa: E731
            for th in np.linspace(0, 2 * math.pi, 7):
                e = phi_inv([math.cos(th), math.sin(th)])
                assert abs(e @ Sinv @ e - (c2 - kappa)) <= 1e-8 * c2
                assert abs(e @ Sinv @ mu - (c2 - kappa)) <= 1e-8 * c2
                D, tau, _ = oracle.divergence(mu, Rp.reshape(-1), s, e)
                assert abs(tau - 1) <= 1e-9
                assert abs(D - kappa) <= 1e-7 * max(1, kappa)
            U = r["U"].reshape(2, 2)
            B = Q[:, :2].T @ Q[:, :2]
            w, v = np.linalg.eigh(B)
            if w[1] - w[0] > 1e-5 * w[1]:
                assert abs(abs(U[:, 1] @ v[:, 1]) - 1) < 1e-9
            assert abs(U[:, 0] @ U[:, 1]) < 1e-14
            V = r["quad"].reshape(4, 3).T
            uo = U @ O
            # App. A.3: V_ray = c^2 / (c^2 - kappa) * Phi^-1(U O), column by column
            Vref = np.stack([c2 / (c2 - kappa) * phi_inv(uo[:, k]) for k in range(4)], 1)
            np.testing.assert_allclose(V, Vref, atol=1e-9 * np.abs(Vref).max())
            for k in range(4):
                assert abs(V[:, k] @ Sinv @ mu - c2) <= 1e-8 * c2
            e01, e12 = V[:, 1] - V[:, 0], V[:, 2] - V[:, 1]
            assert abs(e01 @ e12) <= 1e-9 * (e01 @ e01 + e12 @ e12)


def test_isotropic_on_axis_worked_example(oracle_lib):
    """Worked example (derived from Sec. 4.1, stored in tests/golden): an
    isotropic Gaussian on the optical axis; its support radius in pixels,
    f * tan(asin(s sqrt(kappa) / d)), equals the half-side of the projected
    quad: the support disk is inscribed in the quad."""
    import os

    golden = {}
    path = os.path.join(os.path.dirname(__file__), "golden", "isotropic_on_axis.txt")
    for line in open(path):
        line = line.split("#")[0].strip()
        if line:
            k, v = line.split("=")
            golden[k.strip()] = float(v)
    s, d, o, W = golden["s"], golden["d"], golden["o"], int(golden["width"])
    cam = scenegen.pinhole(np.concatenate([np.eye(3), np.zeros((3, 1))], 1), W, W, golden["fov_deg"])
    scene = dict(means=np.array([[0], [0], [d]], np.float32), log_scales=np.full((3, 1), math.log(s), np.float32),
                 quats=np.array([[1.0], [0], [0], [0]], np.float32),
                 opacity_logits=np.array([math.log(o / (1 - o))], np.float32),
                 sh=np.zeros((1, 3, 1), np.float32), sh_degree=0)
    sp = oracle.preprocess(scene, cam, OPTS)[0]
    half = 0.5 * (sp["bbox"][1] - sp["bbox"][0])
    s32, d32, o32 = float(np.float32(s)), float(np.float32(d)), 1 / (1 + math.exp(-float(np.float32(math.log(o / (1 - o))))))
    kappa = 2 * math.log(o32 / OPTS["p_min"])
    r = cam["fx"] * math.tan(math.asin(math.exp(float(np.float32(math.log(s)))) * math.sqrt(kappa) / d32))
    assert abs(half - r) < 1e-9
    assert abs(half - golden["radius_px"]) < 5e-4
    # brute force: largest pixel radius along +u with omega >= p_min
    rr = np.linspace(0, 2 * r, 200001)
    xs = np.stack([rr / cam["fx"], 0 * rr, 1 + 0 * rr], 1)
    Dv = np.array([oracle.divergence([0, 0, d32], np.eye(3).reshape(-1), [math.exp(float(np.float32(math.log(s))))] * 3, x)[0] for x in xs[::50]])
    inside = rr[::50][o32 * np.exp(-Dv / 2) >= OPTS["p_min"]]
    assert abs(inside.max() - r) < 2 * (rr[50] - rr[0])


def test_quad_encloses_support(oracle_lib):
    """Every pixel centre with omega >= p_min lies inside its Gaussian's
    projected quad and pixel box (Sec. 4.1); brute force over all pixels with
    an independent D (c^2 - L^2/Q from a numerically inverted covariance)."""
    for seed in (8, 9, 10):
        sc, cam, sp = _visible_splats(seed, 300)
        H, W = cam["height"], cam["width"]
        ys, xs = np.mgrid[0:H, 0:W]
        rays = np.stack([(xs + 0.5 - cam["cx"]) / cam["fx"], (ys + 0.5 - cam["cy"]) / cam["fy"], np.ones_like(xs, float)], -1)
        hits = 0
        for r in sp:
            Sinv = _sigma_inv(r["Rp"].reshape(3, 3), r["s"])
            L = rays @ (Sinv @ r["mu"])
            Qd = np.einsum("hwi,ij,hwj->hw", rays, Sinv, rays)
            D = r["c2"] - L * L / Qd
            sup = (r["o"] * np.exp(-D / 2) >= OPTS["p_min"] * (1 + 1e-9)) & (L > 0)
            if not sup.any():
                continue
            hits += 1
            py, px = np.nonzero(sup)
            assert px.min() >= r["px0"] and px.max() <= r["px1"] and py.min() >= r["py0"] and py.max() <= r["py1"]
            if r["all_front"]:
                V = r["quad"].reshape(4, 3)
                P = np.stack([cam["fx"] * V[:, 0] / V[:, 2] + cam["cx"], cam["fy"] * V[:, 1] / V[:, 2] + cam["cy"]], 1)
                pts = np.stack([px + 0.5, py + 0.5], 1)
                sgn = []
                for k in range(4):
                    a, b = P[k], P[(k + 1) % 4]
                    sgn.append((b[0] - a[0]) * (pts[:, 1] - a[1]) - (b[1] - a[1]) * (pts[:, 0] - a[0]))
                sgn = np.stack(sgn, 1)
                tol = 1e-9 * np.abs(sgn).max()
                assert np.all((sgn >= -tol).all(1) | (sgn <= tol).all(1))
        assert hits > 30


# --------------------------------------------------------- compositing, eq. (1)
def _one_gaussian_scene(mus, scales, opac, rgbs):
    n = len(mus)
    sh = np.zeros((1, 3, n))
    sh[0] = (np.asarray(rgbs, float).T - 0.5) * 2 * math.sqrt(math.pi)
    return dict(means=np.asarray(mus, np.float32).T.copy(), log_scales=np.log(np.asarray(scales, float)).T.astype(np.float32).copy(),
                quats=np.tile(np.array([[1.0], [0], [0], [0]], np.float32), (1, n)),
                opacity_logits=np.array([math.log(o / (1 - o)) for o in opac], np.float32), sh=sh.astype(np.float32), sh_degree=0)


def _ident_cam(W=32, H=32, fov=60):
    return scenegen.pinhole(np.concatenate([np.eye(3), np.zeros((3, 1))], 1), W, H, fov)


def test_compositing_closed_forms(oracle_lib):
    cam = _ident_cam()
    px, py = 16, 16
    x = np.array([(px + 0.5 - cam["cx"]) / cam["fx"], (py + 0.5 - cam["cy"]) / cam["fy"], 1.0])

    def alpha(mu, s, o):
        xn = x / np.linalg.norm(x)
        D = (mu @ mu - (xn @ mu) ** 2) / s**2
        return min(o * math.exp(-D / 2), OPTS["alpha_max"])

    f32 = lambda v: float(np.float32(v))  # noqa: E731
    m1, m2 = np.array([0.0, 0.0, 3.0]), np.array([0.02, -0.01, 5.0])
    s1, s2 = 0.2, 0.3
    sc = _one_gaussian_scene([m1], [[s1] * 3], [0.7], [[0.2, 0.5, 0.9]])
    out = oracle.render(sc, cam, OPTS)
    o1 = 1 / (1 + math.exp(-f32(math.log(0.7 / 0.3))))
    rgb1 = np.float32((np.array([0.2, 0.5, 0.9]) - 0.5) * 2 * math.sqrt(math.pi)).astype(float) / (2 * math.sqrt(math.pi)) + 0.5
    a1 = alpha(m1, math.exp(f32(math.log(s1))), o1)
    np.testing.assert_allclose(out["rgb"][:, py, px], a1 * rgb1, atol=1e-12)
    assert abs(out["T"][py, px] - (1 - a1)) < 1e-12
    sc = _one_gaussian_scene([m2, m1], [[s2] * 3, [s1] * 3], [0.6, 0.7], [[1, 0, 0], [0.2, 0.5, 0.9]])
    out = oracle.render(sc, cam, OPTS)
    o2 = 1 / (1 + math.exp(-f32(math.log(0.6 / 0.4))))
    a2 = alpha(np.array([f32(v) for v in m2]), math.exp(f32(math.log(s2))), o2)
    rgb2 = np.float32((np.array([1.0, 0, 0]) - 0.5) * 2 * math.sqrt(math.pi)).astype(float) / (2 * math.sqrt(math.pi)) + 0.5
    np.testing.assert_allclose(out["rgb"][:, py, px], a1 * rgb1 + (1 - a1) * a2 * rgb2, atol=1e-12)
    # an opaque front Gaussian (alpha clamped at alpha_max) leaks at most 1 - alpha_max
    sc = _one_gaussian_scene([m1, m2], [[0.5] * 3, [s2] * 3], [0.999999, 0.9], [[0, 0, 0], [1, 1, 1]])
    out = oracle.render(sc, cam, OPTS)
    assert out["rgb"][:, py, px].max() <= 1 - OPTS["alpha_max"] + 1e-12


def test_order_is_by_depth_not_input(oracle_lib):
    """eq. (1): permuting the input (distinct depths) leaves the image unchanged."""
    sc = scenegen.tiny_scene(11, 60, sh_degree=2)
    cam = scenegen.pinhole(scenegen.look_at((0.3, 0.2, -3.0)), 40, 36, 60)
    a = oracle.render(sc, cam, OPTS)
    perm = np.random.default_rng(0).permutation(60)
    sc2 = {k: (v[..., perm] if isinstance(v, np.ndarray) else v) for k, v in sc.items()}
    b = oracle.render(sc2, cam, OPTS)
    assert np.array_equal(a["rgb"], b["rgb"]) and np.array_equal(a["T"], b["T"])


def _brute_render(sc, cam, opts):
    """All pixels x all Gaussians, no boxes: independent rendering of eq. (1)-(2)."""
    n = sc["opacity_logits"].shape[0]
    W_ = np.asarray(cam["w2c"])
    H, Wd = cam["height"], cam["width"]
    m = sc["means"].astype(np.float64).T
    mu = m @ W_[:, :3].T + W_[:, 3]
    q = sc["quats"].astype(np.float64).T
    s = np.exp(sc["log_scales"].astype(np.float64).T)
    o = 1 / (1 + np.exp(-sc["opacity_logits"].astype(np.float64)))
    Cw = -W_[:, :3].T @ W_[:, 3]
    ys, xs = np.mgrid[0:H, 0:Wd]
    rays = np.stack([(xs + 0.5 - cam["cx"]) / cam["fx"], (ys + 0.5 - cam["cy"]) / cam["fy"], np.ones((H, Wd))], -1)
    keys = np.array([np.float32(z).view(np.uint32) for z in mu[:, 2]])
    order = sorted(range(n), key=lambda i: (keys[i], i))
    C = np.zeros((H, Wd, 3))
    T = np.ones((H, Wd))
    alive = np.ones((H, Wd), bool)
    deg = sc["sh_degree"]
    for i in order:
        qn = q[i] / np.linalg.norm(q[i])
        w, x, y, z = qn
        R = np.array([[w * w + x * x - y * y - z * z, 2 * (x * y - w * z), 2 * (x * z + w * y)],
                      [2 * (x * y + w * z), w * w - x * x + y * y - z * z, 2 * (y * z - w * x)],
                      [2 * (x * z - w * y), 2 * (y * z + w * x), w * w - x * x - y * y + z * z]])
        Rp = W_[:, :3] @ R
        Sinv = np.linalg.inv(Rp @ np.diag(s[i] ** 2) @ Rp.T)
        if mu[i, 2] <= opts["near_z"]:
            continue
        kappa = -2 * math.log(opts["p_min"] / o[i])
        if kappa <= 0 or mu[i] @ Sinv @ mu[i] <= kappa:
            continue
        L = rays @ (Sinv @ mu[i])
        Qd = np.einsum("hwi,ij,hwj->hw", rays, Sinv, rays)
        tau = L / Qd
        e = tau[..., None] * rays - mu[i]
        D = np.einsum("hwi,ij,hwj->hw", e, Sinv, e)
        om = o[i] * np.exp(-D / 2)
        take = alive & (tau > 0) & (om >= opts["p_min"])
        a = np.minimum(om, opts["alpha_max"])
        Tn = T * (1 - a)
        stop = take & (Tn < opts["t_eps"])
        alive &= ~stop
        take &= ~stop
        d = m[i] - Cw
        d /= np.linalg.norm(d)
        Y = _scipy_real_sh(deg, d)
        col = np.maximum(Y @ sc["sh"][:, :, i].astype(np.float64) + 0.5, 0)
        C[take] += (T[take] * a[take])[:, None] * col
        T = np.where(take, Tn, T)
    return C.transpose(2, 0, 1) + T * np.asarray(opts["background"])[:, None, None], T


def test_brute_force_rendering_tiny_scenes(oracle_lib):
    for seed, deg, eye in ((12, 0, (0, 0, -3.0)), (13, 3, (0.5, 0.4, -2.5)), (14, 1, (-0.2, 1.0, -2.2))):
        sc = scenegen.tiny_scene(seed, 40, sh_degree=deg, log_scale_mean=-2.2, log_scale_std=0.6)
        cam = scenegen.pinhole(scenegen.look_at(eye), 30, 26, 65)
        opts = scenegen.default_options(tile_w=8, tile_h=8, background=(0.1, 0.2, 0.3))
        out = oracle.render(sc, cam, opts)
        C, T = _brute_render(sc, cam, opts)
        np.testing.assert_allclose(out["rgb"], C, atol=1e-10)
        np.testing.assert_allclose(out["T"], T, atol=1e-12)


# ---------------------------------------------------------------- SH basis
def _scipy_real_sh(deg, d):
    """Real SH from scipy's complex Y_l^m (which carries the Condon-Shortley
    phase): for m > 0 sqrt2 (-1)^m Re Y_l^m, m < 0 sqrt2 (-1)^m Im Y_l^|m|;
    the colour-model convention used here is that basis times (-1)^m."""
    x, y, z = d
    theta = math.acos(max(-1.0, min(1.0, z)))
    phi = math.atan2(y, x)
    out = []
    for l in range(deg + 1):
        for m in range(-l, l + 1):
            Y = special.sph_harm_y(l, abs(m), theta, phi)
            if m > 0:
                v = math.sqrt(2) * (-1) ** m * Y.real
            elif m < 0:
                v = math.sqrt(2) * (-1) ** m * Y.imag
            else:
                v = Y.real
            out.append(v * (-1) ** m)
    return np.array(out)


def test_sh_basis_against_scipy(oracle_lib):
    rng = np.random.default_rng(15)
    for _ in range(50):
        d = rng.normal(0, 1, 3)
        d /= np.linalg.norm(d)
        Y, _ = oracle.sh_basis(3, d)
        np.testing.assert_allclose(Y, _scipy_real_sh(3, d), atol=1e-12)


def test_sh_basis_orthonormal_and_gradient(oracle_lib):
    # Lebedev-free check: Monte Carlo with many points gives orthonormality to ~1e-2
    rng = np.random.default_rng(16)
    d = rng.normal(0, 1, (40000, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    Ys = np.array([oracle.sh_basis(3, v)[0] for v in d[:8000]])
    G = 4 * math.pi * Ys.T @ Ys / len(Ys)
    assert np.abs(G - np.eye(16)).max() < 0.12
    for v in d[:20]:
        Y, dY = oracle.sh_basis(3, v)
        for j in range(3):
            h = np.zeros(3)
            h[j] = 1e-6
            fd = (oracle.sh_basis(3, v + h)[0] - oracle.sh_basis(3, v - h)[0]) / 2e-6
            np.testing.assert_allclose(dY[:, j], fd, atol=1e-8)


# --------------------------------------------------------- binning and sort
def _support_mask(r, cam, xs, ys):
    """omega >= p_min and tau > 0 at pixel positions (xs, ys), with D from a
    numerically inverted covariance (independent of the oracle's conic)."""
    Sinv = _sigma_inv(r["Rp"].reshape(3, 3), r["s"])
    x = np.stack([(xs - cam["cx"]) / cam["fx"], (ys - cam["cy"]) / cam["fy"], np.ones_like(xs, float)], -1)
    L = x @ (Sinv @ r["mu"])
    Q = np.einsum("...i,ij,...j->...", x, Sinv, x)
    D = r["c2"] - L * L / Q
    return (L > 0) & (r["o"] * np.exp(-D / 2) >= OPTS["p_min"]), D


def _min_D_over_rect(r, cam, x0, x1, y0, y1):
    from scipy.optimize import minimize

    Sinv = _sigma_inv(r["Rp"].reshape(3, 3), r["s"])

    def D(p):
        x = np.array([(p[0] - cam["cx"]) / cam["fx"], (p[1] - cam["cy"]) / cam["fy"], 1.0])
        L = x @ Sinv @ r["mu"]
        return r["c2"] - L * L / (x @ Sinv @ x) if L > 0 else r["c2"]

    best = np.inf
    for sx in np.linspace(x0, x1, 3):
        for sy in np.linspace(y0, y1, 3):
            res = minimize(D, [sx, sy], bounds=[(x0, x1), (y0, y1)], method="L-BFGS-B")
            best = min(best, res.fun)
    return best


def test_tile_lists_by_definition(oracle_lib):
    """A tile is listed for a Gaussian iff the rectangle spanned by its pixel
    centres inside the Gaussian's pixel box meets the support: checked from
    below by pixel centres inside the support, from above by minimising D over
    that rectangle; the list of a tile is ordered by (float32 depth, index)."""
    sc = scenegen.tiny_scene(17, 150, sh_degree=0, log_scale_mean=-2.5, log_scale_std=0.7)
    cam = scenegen.pinhole(scenegen.look_at((0.1, -0.2, -3.0)), 53, 41, 60)
    opts = scenegen.default_options(tile_w=16, tile_h=8)
    sp = oracle.preprocess(sc, cam, opts)
    tiles, keys, idx = oracle.tile_lists(sp, cam, opts)
    tx_n = -(-53 // 16)
    listed = set(zip(tiles.tolist(), idx.tolist()))
    checked_above = 0
    for i in np.nonzero(sp["cull"] == 0)[0]:
        r = sp[i]
        ys, xs = np.mgrid[r["py0"]:r["py1"] + 1, r["px0"]:r["px1"] + 1]
        sup, _ = _support_mask(r, cam, xs + 0.5, ys + 0.5)
        for y, x in zip(ys[sup], xs[sup]):
            assert ((y // 8) * tx_n + x // 16, i) in listed
        mine = [t for (t, j) in listed if j == i]
        for t in mine[:6]:
            ty, tx = divmod(t, tx_n)
            r0, r1 = max(ty * 8, r["py0"]), min(ty * 8 + 7, r["py1"])
            c0, c1 = max(tx * 16, r["px0"]), min(tx * 16 + 15, r["px1"])
            assert r0 <= r1 and c0 <= c1
            assert _min_D_over_rect(r, cam, c0 + 0.5, c1 + 0.5, r0 + 0.5, r1 + 0.5) <= r["kappa"] + 1e-7, (i, t)
            checked_above += 1
    assert checked_above > 100
    # every listed tile lies in the Gaussian's tile rectangle, lists are (depth, index) ordered
    for t, k, i in zip(tiles, keys, idx):
        ty, tx = divmod(int(t), tx_n)
        assert sp["tx0"][i] <= tx <= sp["tx1"][i] and sp["ty0"][i] <= ty <= sp["ty1"][i]
        assert k == np.float32(sp["mu"][i][2]).view(np.uint32)
    for t in np.unique(tiles):
        sel = tiles == t
        pairs = list(zip(keys[sel].tolist(), idx[sel].tolist()))
        assert pairs == sorted(pairs)
    assert len(listed) == len(tiles)


def test_pixel_box_is_centres_inside_bbox(oracle_lib):
    _, cam, sp = _visible_splats(18, 300)
    for r in sp[sp["all_front"] == 1]:
        xs = np.arange(cam["width"]) + 0.5
        inside = np.nonzero((xs >= r["bbox"][0]) & (xs <= r["bbox"][1]))[0]
        assert inside.min() == r["px0"] and inside.max() == r["px1"]


def _support_extent(r, cam, axis):
    """Extent of the support D <= kappa along image axis `axis` (0: u, 1: v)
    by the discriminant route: in homogeneous pixel coordinates the support is
    p^T M p <= 0 with M = (c^2 - kappa) K^T Sinv K - (K^T Sinv mu)(K^T Sinv mu)^T
    (Sinv inverted numerically, K: pixel -> ray); at an extreme value of one
    coordinate the quadratic in the other has a double root, a quadratic
    condition whose two roots are the extent (no centre or radius used)."""
    Sinv = _sigma_inv(r["Rp"].reshape(3, 3), r["s"])
    K = np.array([[1 / cam["fx"], 0, -cam["cx"] / cam["fx"]], [0, 1 / cam["fy"], -cam["cy"] / cam["fy"]], [0, 0, 1.0]])
    a = K.T @ Sinv @ r["mu"]
    M = (r["c2"] - r["kappa"]) * (K.T @ Sinv @ K) - np.outer(a, a)
    i, j = (0, 1) if axis == 0 else (1, 0)
    # row j of the quadratic in the other coordinate: M_jj t^2 + 2 (M_ij s + M_j2) t + (M_ii s^2 + 2 M_i2 s + M_22)
    A2 = M[i, j] ** 2 - M[j, j] * M[i, i]
    A1 = 2 * (M[i, j] * M[j, 2] - M[j, j] * M[i, 2])
    A0 = M[j, 2] ** 2 - M[j, j] * M[2, 2]
    roots = np.sort(np.roots([A2, A1, A0]).real)
    return roots[0], roots[1]


@pytest.mark.parametrize("mip", [0, 1, 2])
def test_binning_box_is_centres_inside_the_support_ellipse_box(oracle_lib, mip):
    """The binning box holds exactly the pixel-box pixels whose centres lie in
    the support ellipse's bounding box; that box equals the extent of D <=
    kappa found by an independent route; every support pixel lies in the
    binning box, and a Gaussian whose box holds no such centre is culled
    (nobin), with no support pixel.  With eq. (17) the ellipse is the widened
    Gaussian's, with the exact MIP the bounding Gaussian's (the splat's s,
    kappa and c2 are those)."""
    opts = dict(OPTS, mip=mip, mip_sigma2_px=1.0)
    checked = 0
    for seed in (18, 19):
        sc = scenegen.tiny_scene(seed, 300, sh_degree=0, log_scale_mean=-2.5, log_scale_std=0.8)
        cam = scenegen.pinhole(scenegen.look_at((0, 0, -3.5)), 96, 80, 70)
        sp = oracle.preprocess(sc, cam, opts)
        tighter = 0
        for r in sp[(sp["cull"] == 0) & (sp["bounded"] == 1)]:
            for axis, (k0, k1) in enumerate(((0, 1), (2, 3))):
                lo, hi = _support_extent(r, cam, axis)
                np.testing.assert_allclose([r["ebox"][k0], r["ebox"][k1]], [lo, hi], rtol=1e-9, atol=1e-9)
            xs = np.arange(r["px0"], r["px1"] + 1)
            ys = np.arange(r["py0"], r["py1"] + 1)
            bx = xs[(xs + 0.5 >= r["ebox"][0]) & (xs + 0.5 <= r["ebox"][1])]
            by = ys[(ys + 0.5 >= r["ebox"][2]) & (ys + 0.5 <= r["ebox"][3])]
            assert (bx.min(), bx.max(), by.min(), by.max()) == (r["bx0"], r["bx1"], r["by0"], r["by1"])
            assert (r["tx0"], r["tx1"], r["ty0"], r["ty1"]) == (r["bx0"] // 16, r["bx1"] // 16, r["by0"] // 16, r["by1"] // 16)
            yy, xx = np.mgrid[r["py0"]:r["py1"] + 1, r["px0"]:r["px1"] + 1]
            sup = _support_mask(r, cam, xx + 0.5, yy + 0.5)[0] if mip == 0 else \
                (_support_mask(r, cam, xx + 0.5, yy + 0.5)[1] <= r["kappa"])
            assert np.all((xx[sup] >= r["bx0"]) & (xx[sup] <= r["bx1"]) & (yy[sup] >= r["by0"]) & (yy[sup] <= r["by1"]))
            tighter += (r["bx1"] - r["bx0"] < r["px1"] - r["px0"]) or (r["by1"] - r["by0"] < r["py1"] - r["py0"])
            checked += 1
        assert tighter > 20
        for r in sp[sp["cull"] == oracle.CULL["nobin"]]:
            yy, xx = np.mgrid[r["py0"]:r["py1"] + 1, r["px0"]:r["px1"] + 1]
            assert not (_support_mask(r, cam, xx + 0.5, yy + 0.5)[1] <= r["kappa"]).any()
    assert checked > 200


# --------------------------------------------------------------------- culls
def test_culls_and_degenerate_inputs(oracle_lib):
    cam = _ident_cam()
    mus = [[0, 0, 0.1], [0, 0, -2], [0, 0, 3], [0, 0, 3], [0, 0, 3], [0, 0, 3], [5, 0, 3]]
    sc = _one_gaussian_scene(mus, [[0.1] * 3] * 7, [0.5, 0.5, 0.5, 0.002, 0.5, 0.5, 0.5], [[0.5] * 3] * 7)
    sc["quats"][:, 4] = 0.0
    sc["means"][0, 5] = np.nan
    sp = oracle.preprocess(sc, cam, OPTS)
    C = oracle.CULL
    assert list(sp["cull"]) == [C["near"], C["near"], C["visible"], C["kappa"], C["invalid"], C["invalid"], C["offscreen"]]


def _sampled_quad_box(quad, cam, n=1201):
    """Box (umin, umax, vmin, vmax) of the projections of a dense grid of
    points on the quad (a rectangle: corners V0, V1, V2, V3 in order) that lie
    in front of the camera and project into the view; None when none does."""
    V = quad.reshape(4, 3)
    s = np.linspace(0.0, 1.0, n)
    S, T = np.meshgrid(s, s, indexing="ij")
    P = V[0] + S[..., None] * (V[3] - V[0]) + T[..., None] * (V[1] - V[0])
    z = P[..., 2]
    front = z > 1e-9
    u = cam["fx"] * P[..., 0] / np.where(front, z, 1.0) + cam["cx"]
    v = cam["fy"] * P[..., 1] / np.where(front, z, 1.0) + cam["cy"]
    inside = front & (u >= 0) & (u <= cam["width"]) & (v >= 0) & (v <= cam["height"])
    if not inside.any():
        return None
    return u[inside].min(), u[inside].max(), v[inside].min(), v[inside].max()


def test_quad_crossing_camera_plane_box_is_clipped(oracle_lib):
    """A large Gaussian just beyond the near plane whose quad crosses z <= 0:
    its box is that of the part of the quad inside the view frustum (the quad
    itself is drawn unclipped, Sec. 4.1), which dense sampling of the quad's
    surface reproduces; a second crossing quad lies wholly outside the view
    and is culled.  The image still matches brute force, which evaluates
    every pixel for every Gaussian, so the clipped box drops no pixel."""
    cam = _ident_cam(24, 20, 90)
    sc = _one_gaussian_scene([[0.3, 0.1, 0.6], [0, 0, 2.0]], [[0.05, 0.5, 0.05], [0.2] * 3], [0.8, 0.6], [[1, 0, 0], [0, 1, 0]])
    sc["quats"][:, 0] = np.array([0.9, 0.3, 0.2, 0.1], np.float32)
    sp = oracle.preprocess(sc, cam, OPTS)
    assert sp["cull"][0] == 0 and sp["all_front"][0] == 0
    ref = _sampled_quad_box(sp["quad"][0], cam)
    assert ref is not None
    # samples lie inside the clipped polygon, and the grid spacing bounds how
    # far inside its extreme points they can stay
    bb = sp["bbox"][0]
    assert bb[0] <= ref[0] + 1e-9 and bb[1] >= ref[1] - 1e-9 and bb[2] <= ref[2] + 1e-9 and bb[3] >= ref[3] - 1e-9
    assert np.abs(bb - np.array(ref)).max() < 0.1
    assert (sp["px0"][0], sp["px1"][0], sp["py0"][0], sp["py1"][0]) == (12, 23, 0, 19)
    out = oracle.render(sc, cam, OPTS)
    C, T = _brute_render(sc, cam, OPTS)
    np.testing.assert_allclose(out["rgb"], C, atol=1e-10)

    side = _one_gaussian_scene([[2.5, 0.1, 0.6], [0, 0, 2.0]], [[0.05, 0.5, 0.05], [0.2] * 3], [0.8, 0.6],
                               [[1, 0, 0], [0, 1, 0]])
    side["quats"][:, 0] = np.array([0.9, 0.3, 0.2, 0.1], np.float32)
    sp = oracle.preprocess(side, cam, OPTS)
    assert sp["all_front"][0] == 0 and _sampled_quad_box(sp["quad"][0], cam) is None
    assert sp["cull"][0] == oracle.CULL["offscreen"]
    C, T = _brute_render(side, cam, OPTS)
    np.testing.assert_allclose(oracle.render(side, cam, OPTS)["rgb"], C, atol=1e-10)


# ----------------------------------------------------------------- MIP, eq. (17)
def test_mip_zero_sigma_is_plain(oracle_lib):
    sc = scenegen.tiny_scene(19, 80, sh_degree=1)
    cam = scenegen.pinhole(scenegen.look_at((0, 0, -3)), 40, 40, 60)
    a = oracle.render(sc, cam, scenegen.default_options(mip=0))
    b = oracle.render(sc, cam, scenegen.default_options(mip=1, mip_sigma2_px=0.0))
    assert np.array_equal(a["rgb"], b["rgb"])


def test_mip_modulation_matches_determinant_form(oracle_lib):
    """Opacity after MIP = o sqrt(|Sigma| c^2 / (|Sigma^| c^^2)) with
    Sigma^ = Sigma + sigma^2 |mu|^2 I (eq. 17, pixel-invariant tau = |mu|);
    for an isotropic Gaussian this is the area ratio s^2 / (s^2 + sigma^2 |mu|^2)."""
    sc = scenegen.tiny_scene(20, 100, sh_degree=0, log_scale_mean=-4.0, log_scale_std=1.0)
    cam = scenegen.pinhole(scenegen.look_at((0, 0, -3)), 64, 64, 60)
    opts = scenegen.default_options(mip=1)
    plain = oracle.preprocess(sc, cam, scenegen.default_options())
    mip = oracle.preprocess(sc, cam, opts)
    sig2 = opts["mip_sigma2_px"] / (cam["fx"] * cam["fy"])
    checked = 0
    for p, m in zip(plain, mip):
        if p["cull"] == 1 or p["cull"] == 2:
            continue
        Sig = p["Rp"].reshape(3, 3) @ np.diag(p["s"] ** 2) @ p["Rp"].reshape(3, 3).T
        Sh = Sig + sig2 * (p["mu"] @ p["mu"]) * np.eye(3)
        c2 = p["mu"] @ np.linalg.solve(Sig, p["mu"])
        ch2 = p["mu"] @ np.linalg.solve(Sh, p["mu"])
        ref = p["o"] * math.sqrt(np.linalg.det(Sig) * c2 / (np.linalg.det(Sh) * ch2))
        assert abs(m["o"] - ref) <= 1e-9 * ref
        np.testing.assert_allclose(m["s"] ** 2, p["s"] ** 2 + sig2 * (p["mu"] @ p["mu"]), rtol=1e-12)
        checked += 1
    assert checked > 50
    iso = _one_gaussian_scene([[0.1, 0.0, 4.0]], [[0.01] * 3], [0.8], [[1, 1, 1]])
    p = oracle.preprocess(iso, _ident_cam(64, 64), scenegen.default_options())[0]
    m = oracle.preprocess(iso, _ident_cam(64, 64), opts)[0]
    f = _ident_cam(64, 64)["fx"]
    s2 = p["s"][0] ** 2
    assert abs(m["o"] / p["o"] - s2 / (s2 + opts["mip_sigma2_px"] / f**2 * (p["mu"] @ p["mu"]))) < 1e-12


# ------------------------------------------------- exact MIP (Sec. 5, App. A.5)
def _tangent_frame(x):
    """Orthonormal F (3x2) with F^T x = 0, from the SVD of x^T."""
    _, _, vt = np.linalg.svd(x[None, :])
    return vt[1:].T


def _pixel_solid_angle(cam, px, py):
    """Solid angle of pixel (px, py) from its four corners on the unit sphere
    (two spherical triangles, Van Oosterom-Strackee formula)."""
    def ray(u, v):
        r = np.array([(u - cam["cx"]) / cam["fx"], (v - cam["cy"]) / cam["fy"], 1.0])
        return r / np.linalg.norm(r)

    a, b, c, d = ray(px, py), ray(px + 1, py), ray(px + 1, py + 1), ray(px, py + 1)

    def tri(p, q, r):
        num = abs(p @ np.cross(q, r))
        den = 1 + p @ q + q @ r + r @ p
        return 2 * math.atan2(num, den)

    return tri(a, b, c) + tri(a, c, d)


def _mip_exact_by_tangent_plane(mu, Rp, s, o, sig2_px, cam, px, py):
    """The per-ray MIP weight from the tangent-plane Gaussian of App. A.5,
    before any of its identities: tau(x) by brute-force minimisation along the
    unit ray, sigma_x^2 = sigma_px^2 times the pixel's solid angle (the area it
    subtends at unit distance), Sigma^ = Sigma + sigma_x^2 tau^2 I, the exponent
    mu^T F (F^T Sigma^ F)^-1 F^T mu and the modulation
    sqrt(det(F^T Sigma F) / det(F^T Sigma^ F)) (the 2D density's normaliser
    with and without the smoothing)."""
    xb = np.array([(px + 0.5 - cam["cx"]) / cam["fx"], (py + 0.5 - cam["cy"]) / cam["fy"], 1.0])
    x = xb / np.linalg.norm(xb)
    Sig = Rp @ np.diag(np.asarray(s) ** 2) @ Rp.T
    _, tau = _brute_min_along_ray(mu, np.linalg.inv(Sig), x)
    sx2 = sig2_px * _pixel_solid_angle(cam, px, py)
    Sh = Sig + sx2 * tau * tau * np.eye(3)
    F = _tangent_frame(x)
    A, A0 = F.T @ Sh @ F, F.T @ Sig @ F
    e = F.T @ mu
    D = e @ np.linalg.solve(A, e)
    return o * math.sqrt(np.linalg.det(A0) / np.linalg.det(A)) * math.exp(-0.5 * D)


def test_mip_exact_weight_matches_tangent_plane_form(oracle_lib):
    """The oracle's per-ray exact MIP weight (Rp^T-frame scales, D_ray of the
    widened covariance, determinant-identity modulation) equals the weight
    written on the ray's tangent plane (App. A.5 before equalities (a)-(d)),
    with tau found by search and the pixel footprint as a solid angle."""
    rng = np.random.default_rng(31)
    # a long focal length keeps the pixel-centre footprint within ~1e-6 of
    # the pixel's solid angle (their difference is second order in 1/f)
    cam = scenegen.pinhole(np.concatenate([np.eye(3), np.zeros((3, 1))], 1), 480, 400, 50)
    sig2_px = 2.0
    sig2 = sig2_px / (cam["fx"] * cam["fy"])
    checked = 0
    for _ in range(40):
        Rp = _rot(rng)
        s = np.exp(rng.normal(-5.0, 0.8, 3))
        mu = np.array([rng.uniform(-0.5, 0.5), rng.uniform(-0.4, 0.4), 1.0]) * rng.uniform(1.5, 6.0)
        o = rng.uniform(0.2, 0.95)
        u0 = cam["fx"] * mu[0] / mu[2] + cam["cx"]
        v0 = cam["fy"] * mu[1] / mu[2] + cam["cy"]
        for _ in range(3):
            px = int(np.clip(u0 + rng.normal(0, 3), 0, cam["width"] - 1))
            py = int(np.clip(v0 + rng.normal(0, 3), 0, cam["height"] - 1))
            xb = [(px + 0.5 - cam["cx"]) / cam["fx"], (py + 0.5 - cam["cy"]) / cam["fy"], 1.0]
            w, tau_h = oracle.mip_exact_weight(mu, Rp.reshape(-1), s, o, sig2, xb)
            ref = _mip_exact_by_tangent_plane(mu, Rp, s, o, sig2_px, cam, px, py)
            assert tau_h > 0
            # relative error of the exponent's size (D about 30 in the far tail)
            assert abs(math.log(w / ref)) <= 2e-6 * (1 + abs(math.log(ref / o))), (w, ref)
            checked += ref > 1e-3
    assert checked > 30


def test_mip_exact_on_axis_ray_matches_eq17(oracle_lib):
    """On the ray through the centre of a Gaussian on the optical axis the
    exact weight is the opacity of eq. (17): tau = |mu| there, the footprint is
    the principal point's, and x^T Sigma^-1 x / x^T Sigma^^-1 x = c^2 / c^^2."""
    rng = np.random.default_rng(32)
    for _ in range(10):
        z = rng.uniform(2.0, 8.0)
        q = rng.standard_normal(4)
        q /= np.linalg.norm(q)
        sc = dict(means=np.array([[0.0], [0.0], [z]], np.float32),
                  log_scales=rng.normal(-3.5, 0.7, (3, 1)).astype(np.float32),
                  quats=q.reshape(4, 1).astype(np.float32), opacity_logits=np.array([1.3], np.float32),
                  sh=np.zeros((1, 3, 1), np.float32), sh_degree=0)
        cam = _ident_cam(64, 64)
        opts = scenegen.default_options(mip=1, mip_sigma2_px=3.0)
        approx = oracle.preprocess(sc, cam, opts)[0]
        plain = oracle.preprocess(sc, cam, scenegen.default_options())[0]
        sig2 = opts["mip_sigma2_px"] / (cam["fx"] * cam["fy"])
        w, _ = oracle.mip_exact_weight(plain["mu"], plain["Rp"], plain["s"], plain["o"], sig2, [0.0, 0.0, 1.0])
        assert abs(w - approx["o"]) <= 1e-12 * approx["o"]


def test_mip_exact_zero_sigma_is_plain(oracle_lib):
    sc = scenegen.tiny_scene(33, 80, sh_degree=1)
    cam = scenegen.pinhole(scenegen.look_at((0, 0, -3)), 40, 36, 60)
    a = oracle.render(sc, cam, scenegen.default_options(mip=0))
    b = oracle.render(sc, cam, scenegen.default_options(mip=2, mip_sigma2_px=0.0))
    assert np.array_equal(a["rgb"], b["rgb"]) and np.array_equal(a["n_contrib"], b["n_contrib"])
    assert a["counters"] == b["counters"]


def _exact_weights_all_pixels(r, cam, sig2_px):
    """Exact MIP weight and tau^ at every pixel centre, vectorised: plain tau
    in closed form, then D_ray of the per-pixel widened covariance as
    mu^T S^-1 mu - (mu^T S^-1 x)^2 / x^T S^-1 x."""
    H, W = cam["height"], cam["width"]
    ys, xs = np.mgrid[0:H, 0:W]
    xb = np.stack([(xs + 0.5 - cam["cx"]) / cam["fx"], (ys + 0.5 - cam["cy"]) / cam["fy"], np.ones((H, W))], -1)
    nrm = np.linalg.norm(xb, axis=-1)
    x = xb / nrm[..., None]
    Rp = r["Rp"].reshape(3, 3)
    xl = x @ Rp
    ml = Rp.T @ r["mu"]
    s2 = r["s0"] ** 2
    tau = (xl * (ml / s2)).sum(-1) / (xl * xl / s2).sum(-1)
    a = sig2_px / (cam["fx"] * cam["fy"]) / nrm**3 * tau**2
    sh2 = s2 + a[..., None]
    L = (xl * (ml / sh2)).sum(-1)
    Q = (xl * xl / sh2).sum(-1)
    D = (ml * ml / sh2).sum(-1) - L * L / Q
    m2 = np.prod(s2) * (xl * xl / s2).sum(-1) / (np.prod(sh2, -1) * Q)
    return r["o"] * np.sqrt(m2) * np.exp(-0.5 * D), L / Q


def test_mip_exact_support_inside_listed_tiles(oracle_lib):
    """Every pixel whose exact MIP weight reaches p_min lies in a listed tile
    of its Gaussian (the bound of the widened Gaussian is conservative), over
    scenes with strongly anisotropic Gaussians and a footprint large enough
    that some have no bound (whole view)."""
    sig2_px = 1.5
    opts = scenegen.default_options(mip=2, mip_sigma2_px=sig2_px, tile_w=8, tile_h=8)
    whole = bounded_hits = widened = 0
    for seed in (34, 35):
        sc = scenegen.tiny_scene(seed, 150, log_scale_mean=-4.0, log_scale_std=1.0)
        cam = scenegen.pinhole(scenegen.look_at((0, 0, -2.5)), 72, 56, 60)
        sp = oracle.preprocess(sc, cam, opts)
        plain = oracle.preprocess(sc, cam, scenegen.default_options(tile_w=8, tile_h=8))
        tiles, _, ids = oracle.tile_lists(sp, cam, opts)
        tiles_x = -(-cam["width"] // 8)
        for i, r in enumerate(sp):
            if r["cull"] in (1, 2, 3):
                continue
            w, th = _exact_weights_all_pixels(r, cam, sig2_px)
            sup = (w >= opts["p_min"] * (1 + 1e-9)) & (th > 0)
            if not sup.any():
                continue
            assert r["cull"] == 0, (seed, i, r["cull"])
            py, px = np.nonzero(sup)
            listed = set(tiles[ids == i].tolist())
            need = set(((py // 8) * tiles_x + px // 8).tolist())
            assert need <= listed, (seed, i)
            if r["whole"]:
                whole += 1
                assert len(listed) == tiles_x * (-(-cam["height"] // 8))
            else:
                bounded_hits += 1
                widened += plain[i]["cull"] != 0 or np.any(px < plain[i]["px0"]) or np.any(px > plain[i]["px1"])
    assert whole > 0 and bounded_hits > 50 and widened > 5


# ------------------------------------------- linearised divergence (Sec. 3.1)
GS = scenegen.default_options(divergence=1, tile_w=8, tile_h=8)


def _numeric_sigma_pi(mu, Sig, cam, h=1e-6):
    """J Sigma J^T with J from central differences of the pinhole projection."""
    def pi(p):
        return np.array([cam["fx"] * p[0] / p[2] + cam["cx"], cam["fy"] * p[1] / p[2] + cam["cy"]])

    J = np.stack([(pi(mu + h * e) - pi(mu - h * e)) / (2 * h) for e in np.eye(3)], 1)
    return J @ Sig @ J.T, pi(mu)


def test_gs_on_axis_isotropic_closed_form(oracle_lib):
    """An isotropic Gaussian of scale s on the optical axis at depth z
    projects to the pixel-space Gaussian of standard deviation f s / z."""
    cam = _ident_cam(40, 40, 60)
    z, s, o = 4.0, 0.05, 0.8
    sc = _one_gaussian_scene([[0.0, 0.0, z]], [[s] * 3], [o], [[0.9, 0.5, 0.2]])
    out = oracle.render(sc, cam, GS)
    ys, xs = np.mgrid[0:40, 0:40]
    d2 = (xs + 0.5 - cam["cx"]) ** 2 + (ys + 0.5 - cam["cy"]) ** 2
    w = o * np.exp(-0.5 * d2 / (cam["fx"] * s / z) ** 2)
    a = np.where(w >= GS["p_min"], np.minimum(w, GS["alpha_max"]), 0.0)
    np.testing.assert_allclose(out["T"], 1 - a, atol=1e-12)
    np.testing.assert_allclose(out["rgb"][0], 0.9 * a, atol=1e-6)  # colour stored as float32 SH


def test_gs_projected_covariance_and_support(oracle_lib):
    """Sigma_pi^-1 of the oracle equals the inverse of J Sigma J^T with J by
    central differences of the projection, and every pixel whose D_gs (from
    that independent Sigma_pi) gives omega >= p_min lies in a listed tile."""
    hits = 0
    for seed in (42, 43):
        sc = scenegen.tiny_scene(seed, 200, log_scale_mean=-2.8, log_scale_std=0.7)
        cam = scenegen.pinhole(scenegen.look_at((0.3, -0.2, -3.0)), 72, 56, 70)
        sp = oracle.preprocess(sc, cam, GS)
        tiles, _, ids = oracle.tile_lists(sp, cam, GS)
        tiles_x = -(-cam["width"] // 8)
        ys, xs = np.mgrid[0:cam["height"], 0:cam["width"]]
        for i, r in enumerate(sp):
            if r["cull"] in (1, 2, 3):
                continue
            Rp = r["Rp"].reshape(3, 3)
            Sp, c = _numeric_sigma_pi(r["mu"], Rp @ np.diag(r["s"] ** 2) @ Rp.T, cam)
            A = np.linalg.inv(Sp)
            np.testing.assert_allclose(r["gs_A"], [A[0, 0], A[0, 1], A[1, 1]], rtol=1e-6, atol=1e-9 * abs(A).max())
            du, dv = xs + 0.5 - c[0], ys + 0.5 - c[1]
            D = A[0, 0] * du * du + 2 * A[0, 1] * du * dv + A[1, 1] * dv * dv
            sup = r["o"] * np.exp(-0.5 * D) >= GS["p_min"] * (1 + 1e-6)
            if not sup.any():
                continue
            assert r["cull"] == 0
            hits += 1
            py, px = np.nonzero(sup)
            need = set(((py // 8) * tiles_x + px // 8).tolist())
            assert need <= set(tiles[ids == i].tolist()), (seed, i)
    assert hits > 50


def test_gs_approaches_ray_for_small_gaussians(oracle_lib):
    """The linearisation error vanishes with the Gaussian's angular size: the
    D_gs and D_ray images of a scene converge as the scales shrink."""
    cam = scenegen.pinhole(scenegen.look_at((0, 0, -4)), 64, 64, 40)
    errs = []
    for lsm in (-3.0, -4.5, -6.0):
        sc = scenegen.tiny_scene(44, 60, log_scale_mean=lsm, log_scale_std=0.3)
        sc["opacity_logits"][:] = 3.0  # bright enough to stay above p_min when small
        a = oracle.render(sc, cam, scenegen.default_options(tile_w=8, tile_h=8))
        b = oracle.render(sc, cam, GS)
        errs.append(np.abs(a["rgb"] - b["rgb"]).max())
    assert errs[0] > errs[1] > errs[2] and errs[2] < 0.05 * errs[0], errs


def test_mip_dilation_only_widens_without_modulation(oracle_lib):
    """mip = 3 (the dilation-only ablation): the scales of eq. (17) with the
    prior opacity unchanged."""
    sc = scenegen.tiny_scene(48, 100, sh_degree=0, log_scale_mean=-4.0, log_scale_std=1.0)
    cam = scenegen.pinhole(scenegen.look_at((0, 0, -3)), 64, 64, 60)
    plain = oracle.preprocess(sc, cam, scenegen.default_options())
    full = oracle.preprocess(sc, cam, scenegen.default_options(mip=1))
    dil = oracle.preprocess(sc, cam, scenegen.default_options(mip=3))
    ok = (plain["cull"] != 1) & (plain["cull"] != 2)
    assert ok.sum() > 50
    np.testing.assert_array_equal(dil["s"][ok], full["s"][ok])
    np.testing.assert_array_equal(dil["o"][ok], plain["o"][ok])
    assert np.all(dil["o"][ok] >= full["o"][ok])
