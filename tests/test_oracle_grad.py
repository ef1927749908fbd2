"""Pin of the oracle's analytic gradient against FP64 central finite
differences (h = 1e-6) of the oracle's own forward render, on the 64-Gaussian
32x32 SH3 subcase.  The loss is linear in the image, L = sum(w * C), so dL/dC = w;
any loss enters the backward only through dL/dC."""
import numpy as np
import pytest
import oracle
import scenegen

KEYS = ("means", "log_scales", "quats", "opacity_logits", "sh")


def _loss(scene, cam, opts, w):
    return float((oracle.render(scene, cam, opts, threads=1)["rgb"] * w).sum())


def _fd_check(scene, cam, opts, w, h=1e-6, stride=1):
    base = {k: np.asarray(scene[k], np.float64).copy() for k in KEYS}
    sc = dict(base, sh_degree=scene["sh_degree"])
    g = oracle.backward(sc, cam, opts, w)
    worst = 0.0
    count = 0
    for k in KEYS:
        flat = sc[k].reshape(-1)
        gflat = g[k].reshape(-1)
        gmax = np.abs(g[k]).max() + 1e-12
        for j in range(0, flat.size, stride):
            v = flat[j]
            flat[j] = v + h
            lp = _loss(sc, cam, opts, w)
            flat[j] = v - h
            lm = _loss(sc, cam, opts, w)
            flat[j] = v
            fd = (lp - lm) / (2 * h)
            err = abs(fd - gflat[j]) / (abs(gflat[j]) + 1e-3 * gmax)
            worst = max(worst, err)
            count += 1
            assert err < 2e-4, (k, j, fd, gflat[j])
    return worst, count


def test_gradient_matches_central_differences(oracle_lib):
    scene, cam = scenegen.fd_subcase()
    opts = scenegen.default_options()
    out = oracle.render(scene, cam, opts)
    assert out["hazard"].sum() == 0
    assert out["counters"]["contributions"] > 1000
    w = np.random.default_rng(7).normal(0, 1, (3, 32, 32))
    worst, count = _fd_check(scene, cam, opts, w)
    assert count == 64 * 59


def test_gradient_with_background_and_sparse_pixels(oracle_lib):
    scene, cam = scenegen.fd_subcase(seed=2003)
    opts = scenegen.default_options(background=(0.3, 0.1, 0.6))
    w = np.zeros((3, 32, 32))
    rng = np.random.default_rng(8)
    ys, xs = rng.integers(0, 32, 40), rng.integers(0, 32, 40)
    w[:, ys, xs] = rng.normal(0, 1, (3, 40))
    _fd_check(scene, cam, opts, w, stride=3)


def test_mip_gradient_matches_central_differences(oracle_lib):
    """With the MIP transform (eq. 17) the rendered scales and opacity depend
    on the scales, the opacity, the rotation and the mean (through |mu|); a
    large pixel filter makes every one of those paths matter."""
    scene, cam = scenegen.fd_subcase(seed=2004)
    opts = scenegen.default_options(mip=1, mip_sigma2_px=4.0)
    out = oracle.render(scene, cam, opts)
    assert out["hazard"].sum() == 0
    plain = oracle.render(scene, cam, scenegen.default_options())
    assert np.abs(out["rgb"] - plain["rgb"]).max() > 1e-2  # the transform changes the image
    w = np.random.default_rng(9).normal(0, 1, (3, 32, 32))
    worst, count = _fd_check(scene, cam, opts, w)
    assert count == 64 * 59


def test_exact_mip_gradient_matches_central_differences(oracle_lib):
    """The exact MIP weight (mip = 2): gradients through the per-ray widening
    (tau of the ray, the footprint) and the per-ray modulation; a footprint of
    4 px^2 makes the widening matter everywhere."""
    scene, cam = scenegen.fd_subcase(seed=2008)  # a seed with no pixel at a threshold (hazard)
    opts = scenegen.default_options(mip=2, mip_sigma2_px=4.0)
    out = oracle.render(scene, cam, opts)
    assert out["hazard"].sum() == 0
    plain = oracle.render(scene, cam, scenegen.default_options())
    assert np.abs(out["rgb"] - plain["rgb"]).max() > 1e-2
    w = np.random.default_rng(13).normal(0, 1, (3, 32, 32))
    worst, count = _fd_check(scene, cam, opts, w)
    assert count == 64 * 59


def test_dilation_only_backward_is_rejected(oracle_lib):
    sc, cam = scenegen.fd_subcase(2004)
    opts = scenegen.default_options(mip=3)
    dl = np.ones((3, cam["height"], cam["width"]))
    with pytest.raises(ValueError):
        oracle.backward(sc, cam, opts, dl)


def test_gs_gradient_matches_central_differences(oracle_lib):
    """The linearised divergence of Sec. 3.1: gradients through pi(mu), the
    Jacobian J(mu) and Sigma = R_p S^2 R_p^T."""
    scene, cam = scenegen.fd_subcase(seed=2005)
    opts = scenegen.default_options(divergence=1)
    out = oracle.render(scene, cam, opts)
    assert out["hazard"].sum() == 0
    w = np.random.default_rng(10).normal(0, 1, (3, 32, 32))
    worst, count = _fd_check(scene, cam, opts, w)
    assert count == 64 * 59
