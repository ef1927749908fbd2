"""Pins of the oracle's decisions at rounding distance (hazards) and of the
results it accepts there.

Where a decision of the per-pixel compositing (omega >= p_min, eqs. 2-3;
the stop before T' < t_eps, eq. 1; the sign of tau, Prop. A.3) or of the
per-Gaussian stage (the float32 depth key; a pixel-box edge on a pixel
centre) lies within rounding distance of its threshold, both outcomes are
correct results.  These tests build scenes that put a decision exactly at
such a point, in double precision, and check that the oracle flags it and
that the values it returns for both outcomes equal closed forms written here
from eq. (1) -- not from the oracle's code.  A last test pins the fragment
counter (pixel centres inside a projected quad) against a half-plane test of
the projected quadrilateral."""
import math

import numpy as np

import oracle
import scenegen

OPTS = scenegen.default_options(background=(0.2, 0.1, 0.05))
Y00 = 0.5 / math.sqrt(math.pi)


def _scene(mus, scales, opacities, rgbs):
    """Isotropic SH0 Gaussians in double precision (the oracle widens its
    inputs to float64, so these values reach it exactly)."""
    n = len(mus)
    o = np.asarray(opacities, float)
    return dict(means=np.asarray(mus, float).T.copy(), log_scales=np.log(np.asarray(scales, float)).T.copy(),
                quats=np.tile(np.array([[1.0], [0.0], [0.0], [0.0]]), (1, n)),
                opacity_logits=np.log(o / (1.0 - o)),
                sh=((np.asarray(rgbs, float).T - 0.5) / Y00)[None].copy(), sh_degree=0)


def _cam(W=32, H=32, fov=60.0):
    return scenegen.pinhole(np.concatenate([np.eye(3), np.zeros((3, 1))], 1), W, H, fov)


def _ray(cam, px, py):
    return np.array([(px + 0.5 - cam["cx"]) / cam["fx"], (py + 0.5 - cam["cy"]) / cam["fy"], 1.0])


def _isotropic_D(mu, s, x):
    """D_ray of an isotropic Gaussian: |mu|^2 sin^2(angle(x, mu)) / s^2."""
    xn = x / np.linalg.norm(x)
    return (mu @ mu - (xn @ mu) ** 2) / (s * s)


def _leaf_set(leaves):
    return sorted(tuple(np.round(lv, 12)) for lv in leaves)


def test_omega_at_p_min_is_flagged_with_both_results():
    """omega = p_min (1 +- 1e-7) at one pixel: flagged, and the two correct
    results are 'contributes' (C = omega rgb + (1 - omega) bg, T = 1 - omega)
    and 'does not' (C = bg, T = 1), the computed one first.  At 1 +- 1e-3 the
    decision is clear: one result, no flag."""
    cam = _cam()
    px, py = 20, 13
    x = _ray(cam, px, py)
    mu, s, rgb = np.array([0.05, -0.02, 3.0]), 0.25, np.array([0.8, 0.3, 0.1])
    D = _isotropic_D(mu, s, x)
    bg = np.array(OPTS["background"])
    for eta in (1e-7, -1e-7, 1e-3, -1e-3):
        w = OPTS["p_min"] * (1.0 + eta)
        o = w * math.exp(D / 2.0)
        assert o < 0.5
        sc = _scene([mu], [[s] * 3], [o], [rgb])
        ref = oracle.render_pixels(sc, cam, OPTS, [px], [py])
        take = np.concatenate([w * rgb + (1 - w) * bg, [1 - w]])
        skip = np.concatenate([bg, [1.0]])
        lv = ref["leaves"][0]
        first = take if eta > 0 else skip
        np.testing.assert_allclose(lv[0], first, rtol=0, atol=1e-12)
        if abs(eta) < 1e-4:
            assert ref["hazard"][0] == 1 and len(lv) == 2, eta
            np.testing.assert_allclose(lv[1], skip if eta > 0 else take, rtol=0, atol=1e-12)
        else:
            assert ref["hazard"][0] == 0 and len(lv) == 1, eta
        # the full render flags the pixel too, and lists both results for it
        full = oracle.render(sc, cam, OPTS)
        assert full["hazard"][py, px] == (abs(eta) < 1e-4)
        if abs(eta) < 1e-4:
            k = int(np.nonzero((full["branches"]["px"] == px) & (full["branches"]["py"] == py))[0][0])
            assert _leaf_set(full["branches"]["leaves"][k]) == _leaf_set(lv)


def test_termination_at_t_eps_is_flagged_with_both_results():
    """Three Gaussians on one pixel's ray (D = 0, so omega = o): after the
    first two, T = (1 - o1)(1 - o2); the third takes T to
    T' = t_eps (1 +- 1e-7).  Both 'taken' and 'stopped before it' are correct
    results, in closed form from eq. (1)."""
    cam = _cam()
    px, py = 9, 22
    x = _ray(cam, px, py)
    t_eps = OPTS["t_eps"]
    o1 = o2 = 0.95
    rgbs = [np.array([0.9, 0.1, 0.2]), np.array([0.1, 0.8, 0.3]), np.array([0.3, 0.3, 0.9])]
    bg = np.array(OPTS["background"])
    for eta in (1e-7, -1e-7, 1e-2):
        o3 = 1.0 - t_eps * (1.0 + eta) / ((1 - o1) * (1 - o2))
        assert o3 < OPTS["alpha_max"]
        # input order differs from depth order: the oracle sorts by depth
        sc = _scene([3.0 * x, 2.0 * x, 4.0 * x], [[0.05] * 3] * 3, [o2, o1, o3], [rgbs[1], rgbs[0], rgbs[2]])
        ref = oracle.render_pixels(sc, cam, OPTS, [px], [py])
        T2 = (1 - o1) * (1 - o2)
        C2 = o1 * rgbs[0] + (1 - o1) * o2 * rgbs[1]
        stopped = np.concatenate([C2 + T2 * bg, [T2]])
        T3 = T2 * (1 - o3)
        taken = np.concatenate([C2 + T2 * o3 * rgbs[2] + T3 * bg, [T3]])
        lv = ref["leaves"][0]
        np.testing.assert_allclose(lv[0], taken if eta > 0 else stopped, rtol=0, atol=1e-12)
        if abs(eta) < 1e-3:
            assert ref["hazard"][0] == 1 and len(lv) == 2, eta
            np.testing.assert_allclose(lv[1], stopped if eta > 0 else taken, rtol=0, atol=1e-12)
        else:
            assert ref["hazard"][0] == 0 and len(lv) == 1


def test_two_decisions_at_one_pixel_give_every_combination():
    """Two Gaussians on one ray, each with omega = p_min (1 + 1e-7): the four
    combinations of contributing or not are all correct results."""
    cam = _cam()
    px, py = 14, 17
    x = _ray(cam, px, py)
    bg = np.array(OPTS["background"])
    mus = [np.array([0.03, 0.01, 2.5]), np.array([-0.02, 0.04, 3.5])]
    rgbs = [np.array([1.0, 0.2, 0.0]), np.array([0.0, 0.5, 1.0])]
    s = 0.12
    w = OPTS["p_min"] * (1 + 1e-7)
    ops = [w * math.exp(_isotropic_D(m, s, x) / 2) for m in mus]
    sc = _scene(mus, [[s] * 3] * 2, ops, rgbs)
    ref = oracle.render_pixels(sc, cam, OPTS, [px], [py])
    want = []
    for a in (0, 1):
        for b in (0, 1):
            C, T = np.zeros(3), 1.0
            for on, rgb in ((a, rgbs[0]), (b, rgbs[1])):
                if on:
                    C, T = C + T * w * rgb, T * (1 - w)
            want.append(np.concatenate([C + T * bg, [T]]))
    assert ref["hazard"][0] == 1
    assert _leaf_set(ref["leaves"][0]) == _leaf_set(want)


def test_depth_key_at_a_float32_midpoint_is_flagged():
    """The depth key is the float32 rounding of mu_z (ties by index).  A
    centre within rounding of a float32 midpoint is flagged; one exactly on
    it (computed without rounding) or clearly off it is not; the key is the
    round-to-nearest-even float32."""
    cam = _cam()
    base = np.float32(3.0)
    up = np.nextafter(base, np.float32(np.inf))
    mid = (float(base) + float(up)) / 2.0
    f32bits = lambda v: int(np.array([v], np.float32).view(np.uint32)[0])  # noqa: E731
    cases = [(mid, False, f32bits(base)),  # exact midpoint: ties to even (3.0)
             (mid + 2.0 ** -47, True, f32bits(up)), (mid - 2.0 ** -47, True, f32bits(base)),
             (mid + 2.0 ** -40, False, f32bits(up)), (mid - 2.0 ** -40, False, f32bits(base))]
    for z, flagged, key in cases:
        sc = _scene([[0.0, 0.0, z]], [[0.1] * 3], [0.7], [[0.5, 0.5, 0.5]])
        sp = oracle.preprocess(sc, cam, OPTS)[0]
        assert bool(sp["hazard"] & oracle.HAZARD["key"]) == flagged, z - mid
        assert int(sp["depth_key"]) == key


def test_equal_depth_keys_are_ordered_by_index():
    """Two Gaussians whose centres round to the same float32 depth: the one
    with the lower index is composited first even when it is farther (ties
    broken by index), and no hazard is flagged."""
    cam = _cam()
    px, py = 16, 16
    x = _ray(cam, px, py)
    far, near = 3.0 + 2.0 ** -25, 3.0
    assert np.float32(far) == np.float32(near)
    mus = [far * x / x[2], near * x / x[2]]
    rgbs = [np.array([1.0, 0.0, 0.0]), np.array([0.0, 0.0, 1.0])]
    sc = _scene(mus, [[0.1] * 3] * 2, [0.6, 0.5], rgbs)
    sp = oracle.preprocess(sc, cam, OPTS)
    assert sp["depth_key"][0] == sp["depth_key"][1] and (sp["hazard"] == 0).all()
    ref = oracle.render_pixels(sc, cam, OPTS, [px], [py])
    a0, a1 = 0.6, 0.5  # on the ray: D = 0
    bg = np.array(OPTS["background"])
    want = a0 * rgbs[0] + (1 - a0) * a1 * rgbs[1] + (1 - a0) * (1 - a1) * bg
    np.testing.assert_allclose(ref["rgb"][0], want, rtol=0, atol=1e-9)


def test_box_edge_on_a_pixel_centre_is_flagged():
    """A pixel-box edge (A12: the box holds the pixel centres inside the
    projected quad's bounding box) within rounding of a pixel centre is
    flagged; moved 1e-6 px off it, it is not, and the box takes or leaves that
    pixel column by the pixel-centre rule."""
    cam = _cam(40, 40, 60.0)
    sc = _scene([[0.0, 0.0, 4.0]], [[0.05] * 3], [0.8], [[0.5, 0.5, 0.5]])
    umin = oracle.preprocess(sc, cam, OPTS)[0]["bbox"][0]
    target = math.floor(umin - 0.5) + 0.5  # a pixel-centre boundary: centre of column target - 0.5
    col = int(round(target - 0.5))
    for shift, flagged, px0 in ((0.0, True, None), (1e-6, False, col + 1), (-1e-6, False, col)):
        c = dict(cam, cx=cam["cx"] + (target - umin) + shift)
        sp = oracle.preprocess(sc, c, OPTS)[0]
        assert abs(sp["bbox"][0] - (target + shift)) < 1e-9
        assert bool(sp["hazard"] & oracle.HAZARD["rect"]) == flagged, shift
        if px0 is not None:
            assert sp["px0"] == px0


def test_binning_box_edge_on_a_pixel_centre_is_flagged():
    """A binning-box edge (the pixels of the box whose centres lie in the
    support ellipse's bounding box) within rounding of a pixel centre is
    flagged; moved 1e-6 px off it, it is not, and the binning box takes or
    leaves that pixel column by the pixel-centre rule."""
    cam = _cam(40, 40, 60.0)
    sc = _scene([[0.0, 0.0, 4.0]], [[0.3, 0.1, 0.1]], [0.8], [[0.5, 0.5, 0.5]])
    c, h = math.cos(math.pi / 8), math.sin(math.pi / 8)  # 45 degrees about the optical axis
    sc["quats"][:, 0] = [c, 0.0, 0.0, h]
    sp0 = oracle.preprocess(sc, cam, OPTS)[0]
    umin = sp0["ebox"][0]
    assert umin > sp0["bbox"][0] + 1.0  # the quad's box is wider than the ellipse's
    target = math.floor(umin - 0.5) + 0.5
    col = int(round(target - 0.5))
    for shift, flagged, bx0 in ((0.0, True, None), (1e-6, False, col + 1), (-1e-6, False, col)):
        c = dict(cam, cx=cam["cx"] + (target - umin) + shift)
        sp = oracle.preprocess(sc, c, OPTS)[0]
        assert abs(sp["ebox"][0] - (target + shift)) < 1e-9
        assert bool(sp["hazard"] & oracle.HAZARD["rect"]) == flagged, shift
        if bx0 is not None:
            assert sp["bx0"] == bx0 and sp["px0"] < bx0


def test_fragment_count_equals_pixel_centres_inside_projected_quads():
    """The fragment counter (pixel centres whose ray hits a Gaussian's 3D quad
    in front of the camera: what a rasteriser shades for the quad, Sec. 4)
    equals the number of pixel centres inside each projected quadrilateral,
    counted with a half-plane test of its four edges, summed over the
    Gaussians (low opacities, so no pixel stops early)."""
    for seed in (21, 22):
        sc = scenegen.tiny_scene(seed, 250, sh_degree=0, log_scale_mean=-2.5, log_scale_std=0.8)
        sc["opacity_logits"][:] = -4.0
        cam = scenegen.pinhole(scenegen.look_at((0.0, 0.0, -3.5)), 96, 80, 70)
        opts = scenegen.default_options()
        sp = oracle.preprocess(sc, cam, opts)
        vis = sp[sp["cull"] == 0]
        assert vis["all_front"].all() and len(vis) > 100
        ref = oracle.render(sc, cam, opts)
        assert ref["T"].min() > opts["t_eps"] * 10
        ys, xs = np.mgrid[0:80, 0:96]
        pts = np.stack([xs.ravel() + 0.5, ys.ravel() + 0.5], 1)
        total = 0
        for r in vis:
            V = r["quad"].reshape(4, 3)
            P = np.stack([cam["fx"] * V[:, 0] / V[:, 2] + cam["cx"], cam["fy"] * V[:, 1] / V[:, 2] + cam["cy"]], 1)
            side = np.stack([(P[(k + 1) % 4, 0] - P[k, 0]) * (pts[:, 1] - P[k, 1])
                             - (P[(k + 1) % 4, 1] - P[k, 1]) * (pts[:, 0] - P[k, 0]) for k in range(4)], 1)
            total += int(((side >= 0).all(1) | (side <= 0).all(1)).sum())
        assert ref["counters"]["fragments"] == total, (seed, ref["counters"]["fragments"], total)
