"""Anti-aliasing evaluation harness (Sec. 6.2 compares plain rendering,
4-ray multisampling, MIP dilation without modulation and the full MIP).

Every variant of a view is rendered at several render scales (the camera's
size, focal lengths and principal point multiplied by the scale) and
compared with a supersampled reference of the same pixel grid: the plain
renderer at `ref_factor` x `ref_factor` rays per pixel on an ordered grid,
box-averaged by the library's downsampling kernel.  The reference
approximates the pixel-area integral of the plain (unfiltered) image, which is
what the MIP filter of Sec. 5 aims at.

Variants: plain (mip 0), msaa4 (mip 0 at 2x2 rays per pixel), dilation
(mip 3: eq. 17's widening without the opacity modulation), mip (mip 1,
eq. 17) and mip_exact (mip 2, the per-ray weight).
"""
from __future__ import annotations

import math
from typing import Dict, Sequence

import torch

VARIANTS = ("plain", "msaa4", "dilation", "mip", "mip_exact")


def scaled_camera(cam: dict, scale: float) -> dict:
    """The same view on a pixel grid `scale` times as fine."""
    out = dict(cam)
    out["width"] = int(round(cam["width"] * scale))
    out["height"] = int(round(cam["height"] * scale))
    for k in ("fx", "fy", "cx", "cy"):
        out[k] = float(cam[k]) * scale
    return out


def _render(renderer, g, cam, opts) -> torch.Tensor:
    outs = renderer.render(g, [cam], opts)
    return outs[0]["rgb"]


def supersampled(renderer, g, cam, opts, factor: int) -> torch.Tensor:
    """rgb [3][H][W] from factor x factor rays per pixel."""
    hi = scaled_camera(cam, factor)
    assert hi["width"] == cam["width"] * factor and hi["height"] == cam["height"] * factor
    return renderer.downsample(_render(renderer, g, hi, opts), factor)


def variant_image(renderer, g, cam, base_opts, variant: str) -> torch.Tensor:
    o = dict(base_opts)
    if variant == "plain":
        return _render(renderer, g, cam, dict(o, mip=0))
    if variant == "msaa4":
        return supersampled(renderer, g, cam, dict(o, mip=0), 2)
    mode = {"dilation": 3, "mip": 1, "mip_exact": 2}[variant]
    return _render(renderer, g, cam, dict(o, mip=mode))


def image_errors(img: torch.Tensor, ref: torch.Tensor) -> Dict[str, float]:
    d = (img - ref).float()
    mse = float((d * d).mean())
    return {"mae": float(d.abs().mean()), "max": float(d.abs().max()),
            "psnr": float("inf") if mse == 0 else 10.0 * math.log10(1.0 / mse)}


def evaluate(renderer, g, cam: dict, base_opts: dict, scales: Sequence[float] = (0.5, 1.0, 2.0),
             ref_factor: int = 4, variants: Sequence[str] = VARIANTS) -> Dict[float, Dict[str, Dict[str, float]]]:
    """{scale: {variant: {mae, max, psnr}}} against the supersampled reference."""
    res = {}
    for s in scales:
        c = scaled_camera(cam, s)
        ref = supersampled(renderer, g, c, dict(base_opts, mip=0), ref_factor)
        res[s] = {v: image_errors(variant_image(renderer, g, c, base_opts, v), ref) for v in variants}
    return res


def main():
    """python -m paper_2503_18682_amd.aa_eval [--n N] [--width W --height H] [--ref F]
    prints one JSON line of the errors on a seeded thin-structure scene."""
    import argparse
    import json

    import numpy as np

    import scenegen
    from . import renderer as R

    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=100_000)
    ap.add_argument("--width", type=int, default=640)
    ap.add_argument("--height", type=int, default=480)
    ap.add_argument("--ref", type=int, default=8, help="reference rays per pixel side")
    ap.add_argument("--seed", type=int, default=61)
    a = ap.parse_args()
    sc = scenegen.thin_structure_scene(a.seed, a.n, half_extent=1.5)
    cam = scenegen.pinhole(scenegen.look_at((0.0, 0.4, -4.0)), a.width, a.height, 60.0)
    g = {k: torch.from_numpy(np.ascontiguousarray(sc[k])).cuda() for k in R.PARAM_KEYS}
    g["sh_degree"] = int(sc["sh_degree"])
    r = R.Renderer(0)
    res = evaluate(r, g, cam, scenegen.default_options(tile_w=8, tile_h=16), ref_factor=a.ref)
    print(json.dumps({"scene": f"thin structures: {a.n} Gaussians, seed {a.seed}", "view": [a.width, a.height],
                      "reference_rays_per_pixel": a.ref * a.ref,
                      "errors": {str(s): v for s, v in res.items()}}))
    r.close()


if __name__ == "__main__":
    main()
