"""Seeded generators for the synthetic workloads.

Layout of a scene (all float32, structure of arrays, N Gaussians):
  means          [3][N]   world-frame centres
  log_scales     [3][N]   s = exp(log_scales) per local axis
  quats          [4][N]   (w, x, y, z), unit norm as drawn (renderers normalise again)
  opacity_logits [N]      prior opacity o = sigmoid(logit)
  sh             [(d+1)^2][3][N]  colour coefficients, degree d in {0..3}

A camera is a dict: w2c (3x4 float64, OpenCV axes: x right, y down, z forward),
fx, fy, cx, cy (float64, pixels), width, height (int).  The field of view is
horizontal; fx = fy; the principal point is the image centre.

Workloads (numpy default_rng(1000 + k) for workload k):
  c0  1,000 Gaussians, means U[-1,1]^3, log-scales N(-3,0.5), SH0 colours U[0,1],
      one 128x128 camera at distance 4, 60 deg FOV.
  c1  500k Gaussians in 64 anisotropic clusters (centres U[-5,5]^3, std 0.5),
      log-scales N(-4.5,0.7), logits N(0,1.5), SH3; 1920x1080, 50 deg FOV,
      16 orbit poses at radius 8.
  c2  3M Gaussians, 256 clusters in [-10,10]^3, otherwise as c1; 4 stereo pairs
      (63 mm baseline, parallel axes) at 2064x2208 per eye times a per-pair scale
      drawn from {0.5, 1, 2}, 90 deg FOV.
  c3  1M Gaussians as c1; 4 random orbit views at 1600x1060, 50 deg FOV;
      seeded U[0,1] target images.
  c4  6M Gaussians, 512 clusters in [-20,20]^3, log-scales N(-5,0.8); 16 cameras
      of random resolution (W in 256..2560, H in 256..1440) and FOV 40-90 deg.
"""
from __future__ import annotations

import math

import numpy as np

WORKLOADS = ("c0", "c1", "c2", "c3", "c4")


def default_options(**kw):
    """Renderer options shared by both implementations (see the header docs)."""
    opts = dict(
        p_min=1.0 / 255.0,
        alpha_max=0.99,
        t_eps=1e-4,
        near_z=0.2,
        mip=0,
        mip_sigma2_px=0.1,
        background=(0.0, 0.0, 0.0),
        tile_w=16,
        tile_h=16,
        divergence=0,
    )
    opts.update(kw)
    return opts


# --------------------------------------------------------------------------- cameras
def look_at(eye, target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0)):
    """World-to-camera [R | t] (3x4, float64) for a camera at `eye` looking at
    `target`, OpenCV axes (x right, y down, z forward), world `up` on screen up."""
    eye = np.asarray(eye, np.float64)
    z = np.asarray(target, np.float64) - eye
    z /= np.linalg.norm(z)
    down = -np.asarray(up, np.float64)
    y = down - z * np.dot(down, z)
    y /= np.linalg.norm(y)
    x = np.cross(y, z)
    R = np.stack([x, y, z])  # rows: camera axes in world coordinates
    t = -R @ eye
    return np.concatenate([R, t[:, None]], axis=1)


def pinhole(w2c, width, height, fov_x_deg):
    fx = (width / 2.0) / math.tan(math.radians(fov_x_deg) / 2.0)
    return dict(
        w2c=np.asarray(w2c, np.float64).reshape(3, 4).copy(),
        fx=float(fx),
        fy=float(fx),
        cx=width / 2.0,
        cy=height / 2.0,
        width=int(width),
        height=int(height),
    )


def _orbit_eye(radius, azimuth_deg, elevation_deg=0.0):
    az, el = math.radians(azimuth_deg), math.radians(elevation_deg)
    return np.array(
        [radius * math.cos(el) * math.sin(az), radius * math.sin(el), -radius * math.cos(el) * math.cos(az)]
    )


# --------------------------------------------------------------------------- scenes
def _random_rotations(rng, k):
    """Uniform random rotations from the QR factorisation of Gaussian matrices."""
    a = rng.standard_normal((k, 3, 3))
    q, r = np.linalg.qr(a)
    q = q * np.sign(np.diagonal(r, axis1=1, axis2=2))[:, None, :]
    flip = np.linalg.det(q) < 0
    q[flip, :, 0] *= -1.0
    return q


def _clustered_means(rng, n, n_clusters, half_extent, std=0.5):
    """Gaussian i belongs to cluster i mod K; cluster covariance
    R_k diag(std^2, (std a)^2, (std b)^2) R_k^T with a, b ~ U[0.2, 1]."""
    centres = rng.uniform(-half_extent, half_extent, (n_clusters, 3))
    rots = _random_rotations(rng, n_clusters)
    ab = rng.uniform(0.2, 1.0, (n_clusters, 2))
    sig = std * np.concatenate([np.ones((n_clusters, 1)), ab], axis=1)  # [K][3]
    k = np.arange(n) % n_clusters
    z = rng.standard_normal((n, 3)) * sig[k]
    return centres[k] + np.einsum("nij,nj->ni", rots[k], z)


def make_scene(
    rng,
    n,
    *,
    sh_degree=3,
    clusters=0,
    half_extent=1.0,
    log_scale_mean=-3.0,
    log_scale_std=0.5,
    logit_std=1.0,
):
    """Draw one scene.  clusters == 0 means centres uniform in [-h, h]^3."""
    if clusters:
        means = _clustered_means(rng, n, clusters, half_extent)
    else:
        means = rng.uniform(-half_extent, half_extent, (n, 3))
    log_scales = rng.normal(log_scale_mean, log_scale_std, (n, 3))
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    logits = rng.normal(0.0, logit_std, n)
    nk = (sh_degree + 1) ** 2
    sh = np.empty((nk, 3, n))
    # The DC coefficient is scaled so that a degree-0 colour equals the drawn
    # U[0,1] value under the orthonormal real SH basis (Y_00 = 1 / (2 sqrt(pi))).
    sh[0] = (rng.uniform(0.0, 1.0, (3, n)) - 0.5) * (2.0 * math.sqrt(math.pi))
    if nk > 1:
        sh[1:] = rng.normal(0.0, 0.1, (nk - 1, 3, n))
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)  # noqa: E731
    return dict(
        means=f32(means.T),
        log_scales=f32(log_scales.T),
        quats=f32(q.T),
        opacity_logits=f32(logits),
        sh=f32(sh),
        sh_degree=int(sh_degree),
    )


def tiny_scene(seed, n, *, sh_degree=0, half_extent=1.0, log_scale_mean=-2.0, log_scale_std=0.3, logit_std=1.0):
    """Small uniform scenes for unit tests."""
    rng = np.random.default_rng(seed)
    return make_scene(
        rng,
        n,
        sh_degree=sh_degree,
        half_extent=half_extent,
        log_scale_mean=log_scale_mean,
        log_scale_std=log_scale_std,
        logit_std=logit_std,
    )


def thin_structure_scene(seed, n, *, half_extent=1.0, long_log_scale=-2.5, thin_log_scale=-6.5, sh_degree=0):
    """Thin elongated Gaussians (grass- or wire-like: one axis ~e^-2.5, two
    ~e^-6.5, i.e. a few pixels long and well under a pixel wide at the
    evaluation views), the structures on which rendering at a coarser scale
    than training aliases."""
    rng = np.random.default_rng(seed)
    sc = make_scene(rng, n, sh_degree=sh_degree, half_extent=half_extent, log_scale_mean=0.0, log_scale_std=0.3,
                    logit_std=0.5)
    ls = sc["log_scales"].astype(np.float64)
    ls[0] += long_log_scale
    ls[1:] += thin_log_scale
    sc["log_scales"] = np.ascontiguousarray(ls, dtype=np.float32)
    sc["opacity_logits"] = np.ascontiguousarray(sc["opacity_logits"] + 1.5, dtype=np.float32)
    return sc


def wall_scene(seed, n, *, half_extent=2.0, depth_std=0.05, log_scale_mean=-2.0, log_scale_std=0.5, flatten=2.0):
    """Flattened Gaussians on a wall (the plane z = 0, square of half size
    half_extent, depths N(0, depth_std)): the third log-scale is lowered by
    `flatten`, so most Gaussians are disks of a few centimetres, randomly
    oriented.  A camera walking towards the wall (approach_cameras) brings
    them close to it, where the linearised projection of Sec. 3.1 misplaces
    their supports."""
    rng = np.random.default_rng(seed)
    sc = make_scene(rng, n, sh_degree=0, half_extent=half_extent, log_scale_mean=log_scale_mean,
                    log_scale_std=log_scale_std, logit_std=1.0)
    means = sc["means"].astype(np.float64)
    means[2] = rng.normal(0.0, depth_std, n)
    ls = sc["log_scales"].astype(np.float64)
    ls[2] -= flatten
    sc["means"] = np.ascontiguousarray(means, dtype=np.float32)
    sc["log_scales"] = np.ascontiguousarray(ls, dtype=np.float32)
    return sc


def approach_cameras(distances, width, height, fov_x_deg=90.0, offset=(0.3, 0.2)):
    """Cameras on a straight line towards the wall of wall_scene: the eye at
    (offset, -d) for each distance d, looking along +z (OpenCV axes), so the
    wall fills more of the view and its Gaussians come closer as d shrinks."""
    cams = []
    for d in distances:
        w2c = np.array([[1.0, 0.0, 0.0, -offset[0]], [0.0, 1.0, 0.0, -offset[1]], [0.0, 0.0, 1.0, float(d)]])
        cams.append(pinhole(w2c, width, height, fov_x_deg))
    return cams


def make_cameras(name, rng):
    if name == "c0":
        return [pinhole(look_at((0.0, 0.0, -4.0)), 128, 128, 60.0)]
    if name == "c1":
        return [pinhole(look_at(_orbit_eye(8.0, 22.5 * k)), 1920, 1080, 50.0) for k in range(16)]
    if name == "c2":
        cams = []
        for p, az in enumerate((0.0, 90.0, 180.0, 270.0)):
            scale = float(rng.choice([0.5, 1.0, 2.0]))
            w, h = int(round(2064 * scale)), int(round(2208 * scale))
            head = look_at(_orbit_eye(16.0, az))
            for side in (-1.0, 1.0):
                w2c = head.copy()
                # parallel axes: shift the eye by +-31.5 mm along its own x axis
                w2c[0, 3] -= side * 0.0315
                cams.append(pinhole(w2c, w, h, 90.0))
        return cams
    if name == "c3":
        cams = []
        for _ in range(4):
            az, el = rng.uniform(0.0, 360.0), rng.uniform(-30.0, 30.0)
            cams.append(pinhole(look_at(_orbit_eye(8.0, az, el)), 1600, 1060, 50.0))
        return cams
    if name == "c4":
        cams = []
        for _ in range(16):
            az, el = rng.uniform(0.0, 360.0), rng.uniform(-30.0, 30.0)
            w, h = int(rng.integers(256, 2561)), int(rng.integers(256, 1441))
            cams.append(pinhole(look_at(_orbit_eye(32.0, az, el)), w, h, rng.uniform(40.0, 90.0)))
        return cams
    raise ValueError(name)


_SCENE_ARGS = {
    "c0": dict(n=1000, sh_degree=0, clusters=0, half_extent=1.0, log_scale_mean=-3.0, log_scale_std=0.5, logit_std=1.0),
    "c1": dict(n=500_000, sh_degree=3, clusters=64, half_extent=5.0, log_scale_mean=-4.5, log_scale_std=0.7, logit_std=1.5),
    "c2": dict(n=3_000_000, sh_degree=3, clusters=256, half_extent=10.0, log_scale_mean=-4.5, log_scale_std=0.7, logit_std=1.5),
    "c3": dict(n=1_000_000, sh_degree=3, clusters=64, half_extent=5.0, log_scale_mean=-4.5, log_scale_std=0.7, logit_std=1.5),
    "c4": dict(n=6_000_000, sh_degree=3, clusters=512, half_extent=20.0, log_scale_mean=-5.0, log_scale_std=0.8, logit_std=1.5),
}


def make_workload(name, *, n=None):
    """(scene, cameras, options[, targets]) for workload `name`; `n` overrides the
    Gaussian count (same recipe, smaller scene) for quick tests."""
    k = WORKLOADS.index(name)
    rng = np.random.default_rng(1000 + k)
    args = dict(_SCENE_ARGS[name])
    if n is not None:
        args["n"] = int(n)
    count = args.pop("n")
    scene = make_scene(rng, count, **args)
    cams = make_cameras(name, rng)
    opts = default_options(mip=1 if name == "c2" else 0)
    out = dict(scene=scene, cameras=cams, options=opts)
    if name in ("c3", "c4"):
        out["targets"] = [rng.uniform(0.0, 1.0, (3, c["height"], c["width"])).astype(np.float32) for c in cams]
    return out


def fd_subcase(seed=1003):
    """64 Gaussians at 32x32 for finite-difference gradient checks: means
    U[-1,1]^3, log-scales N(-2,0.3), SH3, camera at distance 4, 60 deg FOV."""
    rng = np.random.default_rng(seed)
    scene = make_scene(rng, 64, sh_degree=3, clusters=0, half_extent=1.0, log_scale_mean=-2.0, log_scale_std=0.3, logit_std=1.0)
    cam = pinhole(look_at((0.0, 0.0, -4.0)), 32, 32, 60.0)
    return scene, cam
