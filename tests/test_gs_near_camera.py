"""The linearised divergence of Sec. 3.1 against the ray-based one of
Sec. 3.2 as the camera approaches scene content (Sec. 6.2 shows the
linearised renderer's spikes on such a trajectory), on the oracle alone.

A camera walks towards a wall of flattened Gaussians.  Far away every
Gaussian subtends a small angle, the projection is nearly linear over its
support and the two images agree; close up the linearisation at the mean
misplaces and stretches the supports.  The test checks that direction on the
oracle's FP64 images: the linearised image drifts monotonically away from
the ray-based one, and its listed supports blow up near the camera while the
ray-based ones stay bounded."""
import math

import numpy as np
import pytest

import oracle
import scenegen

DISTANCES = (6.0, 3.0, 1.5, 0.8, 0.5, 0.35)


def _psnr(a, b):
    mse = float(((a - b) ** 2).mean())
    return math.inf if mse == 0 else 10.0 * math.log10(1.0 / mse)


def test_linearised_divergence_drifts_from_ray_based_near_the_camera():
    sc = scenegen.wall_scene(72, 800)
    cams = scenegen.approach_cameras(DISTANCES, 128, 96)
    opts = scenegen.default_options()
    psnr, listed = [], []
    for cam in cams:
        ray = oracle.render(sc, cam, dict(opts, divergence=0), branches=False)
        gs = oracle.render(sc, cam, dict(opts, divergence=1), branches=False)
        psnr.append(_psnr(gs["rgb"], ray["rgb"]))
        listed.append((ray["counters"]["instances"], gs["counters"]["instances"]))
    print("psnr", [round(p, 2) for p in psnr], "listed (ray, gs)", listed)
    assert all(a > b for a, b in zip(psnr, psnr[1:])), psnr
    assert psnr[0] > 45.0 and psnr[-1] < 20.0
    # far: the same supports to a few percent; near: the linearised ones
    # several times larger
    assert abs(listed[0][1] - listed[0][0]) <= 0.05 * listed[0][0]
    assert listed[-1][1] >= 4 * listed[-1][0]
