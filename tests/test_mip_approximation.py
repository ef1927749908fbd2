"""Error of the approximate MIP of eq. (17) against the exact per-ray MIP
weight of Sec. 5 / App. A.5 (both from the oracle).  The paper argues that the
approximation holds for Gaussians whose rays gather near the mean and is
least accurate for thin primitives stretched over a wide cone of rays; these
checks measure that on single Gaussians at the paper's footprint (0.1 px^2)
and assert its direction.  The rendered mass (the sum of omega over a dense
grid of rays) is compared, since the two weights also differ pointwise through
the ray-dependent footprint that eq. (17) takes as constant."""
import math

import numpy as np

import oracle

F = 1000.0
SIG2 = 0.1 / (F * F)


def _rot(rng):
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    return q


def _mass_difference(rng, scales_px, n=10):
    """Median and max over n random Gaussians of |mass(eq. 17) / mass(exact) - 1|."""
    rel = []
    for _ in range(n):
        d = rng.uniform(3.0, 10.0)
        mu = np.array([rng.uniform(-0.2, 0.2), rng.uniform(-0.2, 0.2), 1.0]) * d
        Rp, s, o = _rot(rng), np.asarray(scales_px) * d / F, 0.9
        # eq. (17): one widening sigma^2 |mu|^2 and one modulation for every ray
        sh2 = s**2 + SIG2 * (mu @ mu)
        ml = Rp.T @ mu
        om = o * math.sqrt(np.prod(s**2) * (ml**2 / s**2).sum() / (np.prod(sh2) * (ml**2 / sh2).sum()))
        u0, v0 = mu[0] / mu[2] * F, mu[1] / mu[2] * F
        ext = 3 * max(scales_px) + 3
        grid = np.linspace(-ext, ext, 41)
        wa = we = 0.0
        for a in grid:
            for b in grid:
                x = np.array([(u0 + a) / F, (v0 + b) / F, 1.0])
                D, tau, _ = oracle.divergence(mu, Rp.reshape(-1), np.sqrt(sh2), x)
                wa += om * math.exp(-0.5 * D) if tau > 0 else 0.0
                we += oracle.mip_exact_weight(mu, Rp.reshape(-1), s, o, SIG2, x)[0]
        rel.append(abs(wa / we - 1.0))
    return float(np.median(rel)), float(np.max(rel))


def test_eq17_error_small_for_compact_gaussians_and_larger_for_long_needles(oracle_lib):
    rng = np.random.default_rng(41)
    compact = _mass_difference(rng, [0.3, 0.3, 0.3])
    needle = _mass_difference(rng, [200.0, 0.1, 0.1])
    print(f"eq. 17 rendered-mass error: sub-pixel Gaussian median {compact[0]:.1e} max {compact[1]:.1e}; "
          f"200 x 0.1 px needle median {needle[0]:.1e} max {needle[1]:.1e}")
    assert compact[1] < 1e-4
    assert needle[0] > 30 * compact[1] and needle[1] > 1e-2
