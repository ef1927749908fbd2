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


def render_with_ws(r, scene, cams, opts, capacity=None, flags=0):
    """Render through the C ABI with an explicit workspace; returns
    (outs as numpy dicts, workspace buffer, ws struct, layout, status)."""
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
    host = [{k: v.cpu().numpy() for k, v in o.items()} for o in outs]
    return host, buf, ws, lay, (ok, need)


ID_MASK = (1 << 28) - 1


def listed_count(buf, lay):
    """Instances left after the tile sort (box tiles whose row bands all miss
    the support leave the sort)."""
    return int(read(buf, lay.counters, 8, np.int64)[3])


def instance_lists(buf, lay, with_bands=False):
    """Sorted listed instances (tile ids, Gaussian-view ids[, band bits])."""
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


def assert_image_close(rgb, T, ref, tol=IMAGE_TOL, max_hazard_frac=0.01, label=""):
    ok = ref["hazard"] == 0
    frac = 1.0 - ok.mean()
    assert frac <= max_hazard_frac, f"{label}: hazard fraction {frac}"
    err = np.abs(rgb - ref["rgb"])[:, ok].max() if ok.any() else 0.0
    terr = np.abs(T - ref["T"])[ok].max() if ok.any() else 0.0
    say(f"  {label}: max|rgb-oracle|={err:.3e} max|T-oracle|={terr:.3e} hazard px={int((~ok).sum())}")
    assert err <= tol, f"{label}: rgb error {err}"
    assert terr <= tol, f"{label}: T error {terr}"
    if (~ok).any():
        assert np.abs(rgb - ref["rgb"])[:, ~ok].max() <= 0.02
    return err


def oracle_lists_without_hazards(sp, cam, opts, tile_base=0, id_base=0):
    tiles, keys, ids = oracle.tile_lists(sp, cam, opts, tile_base)
    bad = np.nonzero(sp["hazard"] != 0)[0]
    keep = ~np.isin(ids, bad)
    return tiles[keep], keys[keep], ids[keep] + id_base, set((bad + id_base).tolist())
