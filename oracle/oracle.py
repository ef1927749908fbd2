"""ctypes wrapper of the C oracle (raygs_oracle.c) plus the oracle's tile
binning, written directly from its definition with numpy's sort.

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "raygs_oracle.c")
# RAYGS_SANITIZE=1 builds and loads a copy instrumented with AddressSanitizer
# and UndefinedBehaviorSanitizer (load it with gcc's libasan preloaded; see
# tests/run_sanitized.sh)
_SANITIZE = os.environ.get("RAYGS_SANITIZE") == "1"
_LIB = os.path.join(_HERE, "liboracle_san.so" if _SANITIZE else "liboracle.so")
_SAN_FLAGS = ["-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]

CULL = dict(visible=0, invalid=1, near=2, kappa=3, inside=4, offscreen=5, notile=6, nobin=7)
HAZARD = dict(key=1, rect=2, eigen=4, cull=8, front=16)


def build_library(force=True):
    """Compile the oracle with gcc (no FMA contraction, IEEE double)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp"
    subprocess.check_call(
        ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fno-fast-math", "-shared", "-fPIC",
         *(_SAN_FLAGS if _SANITIZE else []), "-o", tmp, _SRC, "-lm", "-lpthread"]
    )
    os.replace(tmp, _LIB)
    return _LIB


class Camera(C.Structure):
    _fields_ = [("w2c", C.c_double * 12), ("fx", C.c_double), ("fy", C.c_double), ("cx", C.c_double),
                ("cy", C.c_double), ("width", C.c_int32), ("height", C.c_int32)]


class Options(C.Structure):
    _fields_ = [("p_min", C.c_double), ("alpha_max", C.c_double), ("t_eps", C.c_double), ("near_z", C.c_double),
                ("mip", C.c_int32), ("mip_sigma2_px", C.c_double), ("background", C.c_double * 3),
                ("tile_w", C.c_int32), ("tile_h", C.c_int32), ("divergence", C.c_int32)]


class Scene(C.Structure):
    _fields_ = [("means", C.c_void_p), ("log_scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacity_logits", C.c_void_p), ("sh", C.c_void_p), ("n", C.c_int64), ("sh_degree", C.c_int32)]


SPLAT_DTYPE = np.dtype(
    [("cull", np.int32), ("hazard", np.int32), ("mu", np.float64, 3), ("Rp", np.float64, 9), ("s", np.float64, 3),
     ("o", np.float64), ("kappa", np.float64), ("c2", np.float64), ("mu_w", np.float64, 3), ("b", np.float64),
     ("Rv", np.float64, 9), ("U", np.float64, 4), ("quad", np.float64, 12), ("bbox", np.float64, 4),
     ("ebox", np.float64, 4),
     ("all_front", np.int32), ("px0", np.int32), ("px1", np.int32), ("py0", np.int32), ("py1", np.int32),
     ("bx0", np.int32), ("bx1", np.int32), ("by0", np.int32), ("by1", np.int32),
     ("tx0", np.int32), ("tx1", np.int32), ("ty0", np.int32), ("ty1", np.int32), ("depth_key", np.uint32),
     ("pad", np.int32), ("rgb", np.float64, 3), ("rgb_raw", np.float64, 3), ("dir", np.float64, 3),
     ("dist", np.float64), ("cq", np.float64, 6), ("bounded", np.int32), ("listed", np.int32),
     ("s0", np.float64, 3), ("sig2", np.float64), ("exact", np.int32), ("whole", np.int32), ("gs", np.int32),
     ("pad2", np.int32), ("gs_A", np.float64, 3), ("gs_c", np.float64, 2)],
    align=True,
)

_lib = None


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build_library()
        lib = C.CDLL(_LIB)
        P = C.c_void_p
        lib.orc_preprocess.argtypes = [P, P, P, P, C.c_int]
        lib.orc_render.argtypes = [P, P, P, C.c_int, C.c_int, C.c_int, P, P, P, P, P]
        lib.orc_render_pixels.argtypes = [P, P, P, P, P, C.c_int64, C.c_int, P, P, P, P, P, C.c_int]
        lib.orc_support_cells.argtypes = [P, P, P, C.c_int32, P, P, C.c_int64, C.c_int32, C.c_int32, P, C.c_int]
        lib.orc_support_cells.restype = C.c_int
        lib.orc_backward.argtypes = [P, P, P, P, P, P, P, P, P]
        lib.orc_sh_basis.argtypes = [C.c_int, P, P, P]
        lib.orc_divergence.argtypes = [P, P, P, P, P, P]
        lib.orc_divergence.restype = C.c_double
        lib.orc_rot_mu_v.argtypes = [P, P]
        lib.orc_mip_exact_weight.argtypes = [P, P, P, C.c_double, C.c_double, P, P]
        lib.orc_mip_exact_weight.restype = C.c_double
        lib.orc_splat_size.restype = C.c_int
        lib.orc_list_tiles.argtypes = [P, C.c_int64, P, C.c_int32, P, P, C.c_int64]
        lib.orc_list_tiles.restype = C.c_int64
        if lib.orc_splat_size() != SPLAT_DTYPE.itemsize:
            raise RuntimeError("oracle splat layout mismatch")
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


class _SceneF64:
    """Keeps float64 copies of the scene alive for the duration of a call."""

    def __init__(self, scene):
        self.arrays = {k: np.ascontiguousarray(scene[k], dtype=np.float64)
                       for k in ("means", "log_scales", "quats", "opacity_logits", "sh")}
        n = self.arrays["opacity_logits"].shape[0]
        self.struct = Scene(*(_ptr(self.arrays[k]) for k in ("means", "log_scales", "quats", "opacity_logits", "sh")),
                            n, int(scene["sh_degree"]))
        self.n = n


def _camera(cam):
    c = Camera()
    c.w2c[:] = [float(v) for v in np.asarray(cam["w2c"], np.float64).reshape(-1)]
    c.fx, c.fy, c.cx, c.cy = float(cam["fx"]), float(cam["fy"]), float(cam["cx"]), float(cam["cy"])
    c.width, c.height = int(cam["width"]), int(cam["height"])
    return c


def _options(opts):
    o = Options()
    o.p_min, o.alpha_max, o.t_eps, o.near_z = (float(opts[k]) for k in ("p_min", "alpha_max", "t_eps", "near_z"))
    o.mip = int(opts["mip"])
    o.mip_sigma2_px = float(opts["mip_sigma2_px"])
    o.background[:] = [float(v) for v in opts["background"]]
    o.tile_w, o.tile_h = int(opts["tile_w"]), int(opts["tile_h"])
    o.divergence = int(opts.get("divergence", 0))
    return o


def _threads(n):
    return int(n) if n else (os.cpu_count() or 1)


def preprocess(scene, cam, opts, threads=None):
    """Per-Gaussian quantities for one view (structured array, SPLAT_DTYPE)."""
    lib = load()
    s = _SceneF64(scene)
    out = np.zeros(s.n, SPLAT_DTYPE)
    c, o = _camera(cam), _options(opts)
    lib.orc_preprocess(C.byref(s.struct), C.byref(c), C.byref(o), _ptr(out), _threads(threads))
    return out


# Most correct results kept per pixel (combinations of decisions taken within
# rounding distance, see walk_pixel in raygs_oracle.c).
MAX_LEAVES = 64


def render(scene, cam, opts, rows=None, threads=None, branches=True):
    """Full view (or rows [a, b)): dict(rgb [3][H][W], T [H][W], hazard [H][W],
    n_contrib [H][W], counters) and, with `branches`, branches = dict(px, py,
    leaves): every correct result of each hazard pixel (see render_pixels)."""
    lib = load()
    s = _SceneF64(scene)
    H, W = int(cam["height"]), int(cam["width"])
    a, b = rows if rows is not None else (0, H)
    rgb = np.zeros((3, H, W))
    T = np.ones((H, W))
    hz = np.zeros((H, W), np.uint8)
    nc = np.zeros((H, W), np.int32)
    cnt = np.zeros(5, np.int64)
    c, o = _camera(cam), _options(opts)
    lib.orc_render(C.byref(s.struct), C.byref(c), C.byref(o), int(a), int(b), _threads(threads), _ptr(rgb), _ptr(T),
                   _ptr(hz), _ptr(nc), _ptr(cnt))
    out = dict(rgb=rgb, T=T, hazard=hz, n_contrib=nc,
               counters=dict(visible=int(cnt[0]), instances=int(cnt[1]), fragments=int(cnt[2]),
                             box_pairs=int(cnt[3]), contributions=int(cnt[4])))
    if branches:
        py, px = np.nonzero(hz)
        leaves = render_pixels(scene, cam, opts, px, py, threads)["leaves"] if len(px) else []
        out["branches"] = dict(px=px, py=py, leaves=leaves)
    return out


def render_pixels(scene, cam, opts, px, py, threads=None):
    """Selected pixels: dict(rgb [K][3], T [K], hazard [K], leaves).  leaves[k]
    is an array [n_k][4] of (r, g, b, T): every correct result of pixel k,
    i.e. the result of every combination of outcomes of the decisions taken
    within rounding distance (omega vs p_min, the termination test, the sign
    of tau), the computed one first; n_k = 1 for a pixel without hazard.  A
    pixel with more than MAX_LEAVES such results gets None."""
    lib = load()
    s = _SceneF64(scene)
    px = np.ascontiguousarray(px, np.int32)
    py = np.ascontiguousarray(py, np.int32)
    k = px.shape[0]
    rgb = np.zeros((k, 3))
    T = np.zeros(k)
    hz = np.zeros(k, np.uint8)
    lv = np.zeros((max(k, 1), MAX_LEAVES, 4))
    nl = np.zeros(max(k, 1), np.int32)
    c, o = _camera(cam), _options(opts)
    lib.orc_render_pixels(C.byref(s.struct), C.byref(c), C.byref(o), _ptr(px), _ptr(py), k, _threads(threads),
                          _ptr(rgb), _ptr(T), _ptr(hz), _ptr(lv), _ptr(nl), MAX_LEAVES)
    leaves = [lv[i, :nl[i]].copy() if nl[i] > 0 else None for i in range(k)]
    return dict(rgb=rgb, T=T, hazard=hz, leaves=leaves)


def support_cells(splats, cam, opts, tiles, ids, cell_w, cell_h, threads=None):
    """For each (tile, Gaussian index) pair of one view, the bit mask of the
    tile's cells of cell_w x cell_h pixels (bit cy * (tile_w / cell_w) + cx)
    that hold a pixel centre of the Gaussian's support: inside its pixel box,
    omega >= p_min and tau > 0, both clear of their rounding margins."""
    lib = load()
    sp = np.ascontiguousarray(splats)
    tiles = np.ascontiguousarray(tiles, np.int64)
    ids = np.ascontiguousarray(ids, np.int64)
    cells = np.zeros(max(len(tiles), 1), np.uint32)
    tiles_x = -(-int(cam["width"]) // int(opts["tile_w"]))
    c, o = _camera(cam), _options(opts)
    rc = lib.orc_support_cells(_ptr(sp), C.byref(c), C.byref(o), tiles_x, _ptr(tiles), _ptr(ids), len(tiles),
                               int(cell_w), int(cell_h), _ptr(cells), _threads(threads))
    if rc != 0:
        raise ValueError("cells must divide the tile, at most 32 of them")
    return cells[:len(tiles)]


def backward(scene, cam, opts, dL_dC):
    """Gradients (float64, input shapes) for a given dL/dC [3][H][W]."""
    lib = load()
    s = _SceneF64(scene)
    g = {k: np.zeros_like(v) for k, v in s.arrays.items()}
    dl = np.ascontiguousarray(dL_dC, np.float64)
    c, o = _camera(cam), _options(opts)
    rc = lib.orc_backward(C.byref(s.struct), C.byref(c), C.byref(o), _ptr(dl), _ptr(g["means"]),
                          _ptr(g["log_scales"]), _ptr(g["quats"]), _ptr(g["opacity_logits"]), _ptr(g["sh"]))
    if rc != 0:
        raise ValueError(f"oracle backward failed ({rc})")
    return g


def tile_lists(splats, cam, opts, tile_base=0):
    """Tile binning by definition: for every visible Gaussian and every listed
    tile (the rectangle of the tile's pixel centres inside the Gaussian's pixel
    box meets the support ellipse, see raygs_oracle.c), the pair (tile id, Gaussian index), ordered by
    (tile, depth key, Gaussian index).  Returns (tile ids int64, depth keys
    uint32, Gaussian indices int64)."""
    lib = load()
    tiles_x = -(-int(cam["width"]) // int(opts["tile_w"]))
    sp = np.ascontiguousarray(splats)
    total = int(sp["listed"][sp["cull"] == CULL["visible"]].sum())
    tiles = np.zeros(max(total, 1), np.int64)
    ids = np.zeros(max(total, 1), np.int64)
    o = _options(opts)
    w = lib.orc_list_tiles(_ptr(sp), sp.shape[0], C.byref(o), tiles_x, _ptr(tiles), _ptr(ids), total)
    assert w == total
    tiles, ids = tiles[:w] + tile_base, ids[:w]
    key = sp["depth_key"][ids]
    order = np.lexsort((ids, key, tiles))
    return tiles[order], key[order], ids[order]


def sh_basis(degree, d):
    lib = load()
    d = np.ascontiguousarray(d, np.float64)
    Y = np.zeros(16)
    dY = np.zeros((16, 3))
    lib.orc_sh_basis(int(degree), _ptr(d), _ptr(Y), _ptr(dY))
    nk = (degree + 1) ** 2
    return Y[:nk], dY[:nk]


def divergence(mu, Rp, s, x):
    """(D_ray, tau, e = tau x - mu) from the oracle's definition."""
    lib = load()
    mu, Rp, s, x = (np.ascontiguousarray(a, np.float64) for a in (mu, Rp, s, x))
    tau = np.zeros(1)
    e = np.zeros(3)
    D = lib.orc_divergence(_ptr(mu), _ptr(Rp), _ptr(s), _ptr(x), _ptr(tau), _ptr(e))
    return D, float(tau[0]), e


def mip_exact_weight(mu, Rp, s, o, sig2, xbar):
    """(omega, tau^) of the exact MIP density for the ray through xbar =
    (u, v, 1) (normalised camera coordinates); sig2 is the pixel area at unit
    distance at the principal point."""
    lib = load()
    mu, Rp, s, xbar = (np.ascontiguousarray(a, np.float64) for a in (mu, Rp, s, xbar))
    tau = np.zeros(1)
    w = lib.orc_mip_exact_weight(_ptr(mu), _ptr(Rp), _ptr(s), float(o), float(sig2), _ptr(xbar), _ptr(tau))
    return w, float(tau[0])


def rot_mu_v(muh):
    lib = load()
    muh = np.ascontiguousarray(muh, np.float64)
    R = np.zeros(9)
    lib.orc_rot_mu_v(_ptr(muh), _ptr(R))
    return R.reshape(3, 3)
