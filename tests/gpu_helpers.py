"""Shared helpers of the GPU parity tests (device transfer, workspace reads,
hazard-aware image comparison)."""
import sys

import numpy as np
import torch

import oracle

PARAM_KEYS = ("means", "log_scales", "quats", "opacity_logits", "sh")
IMAGE_TOL = 2e-4


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(scene, requires_grad=False):
    g = {k: torch.from_numpy(np.ascontiguousarray(scene[k])).cuda() for k in PARAM_KEYS}
    if requires_grad:
        for k in PARAM_KEYS:
            g[k].requires_grad_(True)
    g["sh_degree"] = int(scene["sh_degree"])
    return g


def read(buf, offset, count, dtype):
    itemsize = np.dtype(dtype).itemsize
    raw = buf[offset: offset + count * itemsize].cpu().numpy()
    return raw.view(dtype)


def render_with_ws(r, scene, cams, opts, capacity=None, flags=0, to_host=True):
    """Render through the C ABI with an explicit workspace; returns
    (outs as numpy dicts (device tensors with to_host=False), workspace
    buffer, ws struct, layout, status)."""
    g = to_dev(scene)
    n = int(scene["opacity_logits"].shape[0])
    cap = capacity or r.default_capacity(n, len(cams))
    buf, ws = r.new_workspace(n, cams, cap, flags, opts)
    outs = r.allocate_outputs(cams)
    r.render_into(g, cams, outs, ws, opts)
    ok, need = r.status(ws)
    if not ok and capacity is None:  # grow once, as the renderer does
        cap = need
        buf, ws = r.new_workspace(n, cams, cap, flags, opts)
        r.render_into(g, cams, outs, ws, opts)
        ok, need = r.status(ws)
    lay = r.layout(n, cams, cap, flags, opts)
    host = [{k: v.cpu().numpy() for k, v in o.items()} for o in outs] if to_host else outs
    return host, buf, ws, lay, (ok, need)


ID_MASK = (1 << 28) - 1


def listed_count(buf, lay):
    """Instances left after the tile sort (box tiles whose pixel-centre
    rectangle misses the support leave the sort)."""
    return int(read(buf, lay.counters, 8, np.int64)[3])


def instance_lists(buf, lay, with_bands=False):
    """Sorted listed instances (tile ids, Gaussian-view ids[, slot bits])."""
    m = listed_count(buf, lay)
    tiles = read(buf, lay.inst_tiles, m, np.uint32).astype(np.int64)
    raw = read(buf, lay.inst_ids, m, np.uint32).astype(np.int64)
    ids = raw & ID_MASK
    if with_bands:
        return tiles, ids, raw >> 28
    return tiles, ids


def oracle_box_tiles(sp):
    """(kept, tiles): the Gaussians the GPU keeps -- the oracle's visible ones
    plus those whose support meets no tile, whose instances the GPU marks
    empty -- and the tile count of each one's pixel box (0 if not kept)."""
    kept = np.isin(sp["cull"], [oracle.CULL["visible"], oracle.CULL["notile"]])
    tiles = (sp["tx1"].astype(np.int64) - sp["tx0"] + 1) * (sp["ty1"].astype(np.int64) - sp["ty0"] + 1)
    return kept, np.where(kept, tiles, 0)


def hazard_pixel_errors(g_rgb, g_T, leaves):
    """Error of each hazard pixel against the nearest of its correct results:
    g_rgb [K][3], g_T [K], leaves[k] an array [n_k][4] of (r, g, b, T) or None
    (more correct results than the oracle keeps; reported as an infinite
    error).  Returns the per-pixel max-abs error over r, g, b and T."""
    err = np.full(len(leaves), np.inf)
    for k, lv in enumerate(leaves):
        if lv is None:
            continue
        got = np.concatenate([g_rgb[k], [g_T[k]]])
        err[k] = np.abs(lv - got[None, :]).max(axis=1).min()
    return err


def assert_pixels_close(g_rgb, g_T, ref, tol=IMAGE_TOL, label=""):
    """Sampled pixels (g_rgb [K][3], g_T [K]) against oracle.render_pixels:
    every pixel within tol of the oracle; a pixel with a decision taken within
    rounding distance within tol of one of its correct results."""
    hz = ref["hazard"] != 0
    err = np.abs(np.concatenate([g_rgb - ref["rgb"], (g_T - ref["T"])[:, None]], 1)).max(1)
    if hz.any():
        err[hz] = hazard_pixel_errors(g_rgb[hz], g_T[hz], [ref["leaves"][k] for k in np.nonzero(hz)[0]])
    say(f"  {label}: max error {err.max():.3e} over {len(err)} pixels ({int(hz.sum())} with a decision at rounding "
        f"distance, worst of those {err[hz].max() if hz.any() else 0.0:.3e})")
    assert err.max() <= tol, f"{label}: error {err.max()}"
    return err.max()


def assert_image_close(rgb, T, ref, tol=IMAGE_TOL, label=""):
    """Every pixel of a GPU image against oracle.render: within tol of the
    oracle, or, where a decision lies within rounding distance (the hazard
    mask), within tol of one of the pixel's correct results."""
    ok = ref["hazard"] == 0
    err = np.abs(rgb - ref["rgb"])[:, ok].max() if ok.any() else 0.0
    terr = np.abs(T - ref["T"])[ok].max() if ok.any() else 0.0
    br = ref["branches"]
    herr = hazard_pixel_errors(rgb[:, br["py"], br["px"]].T, T[br["py"], br["px"]], br["leaves"])
    say(f"  {label}: max|rgb-oracle|={err:.3e} max|T-oracle|={terr:.3e}; {len(herr)} pixels with a decision at "
        f"rounding distance, worst {herr.max() if len(herr) else 0.0:.3e} from a correct result")
    assert err <= tol, f"{label}: rgb error {err}"
    assert terr <= tol, f"{label}: T error {terr}"
    assert len(herr) == 0 or herr.max() <= tol, f"{label}: hazard pixel error {herr.max()}"
    return max(err, terr)


def oracle_lists_without_hazards(sp, cam, opts, tile_base=0, id_base=0):
    tiles, keys, ids = oracle.tile_lists(sp, cam, opts, tile_base)
    bad = np.nonzero(sp["hazard"] != 0)[0]
    keep = ~np.isin(ids, bad)
    return tiles[keep], keys[keep], ids[keep] + id_base, set((bad + id_base).tolist())
