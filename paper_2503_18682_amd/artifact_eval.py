"""Near-camera comparison of the two divergences in one pipeline: the
linearised one of Gaussian splatting (Sec. 3.1) and the ray-based one
(Sec. 3.2, eq. 5).

Sec. 3.1 notes that linearising the projection at the mean misplaces a
Gaussian's support, and Sec. 6.2 shows the resulting spikes on a camera
moving close to scene content.  Here a camera walks on a straight line
towards a wall of flattened Gaussians (scenegen.wall_scene,
scenegen.approach_cameras); at each position both divergences render the
same model with the same threshold, clamp and compositing, and the
linearised image is compared with the ray-based one, which takes the
density's maximum along each ray exactly.  Reported per distance:
  psnr            the linearised image against the ray-based one
  max_dT          the largest transmittance difference (coverage change)
  kept            Gaussians kept for drawing by each divergence
  listed          listed (Gaussian, tile) instances of each divergence: the
                  linearised supports grow without bound near the camera
"""
from __future__ import annotations

import math
from typing import Dict, Sequence

import numpy as np
import torch

DIVERGENCES = {"ray": 0, "gs": 1}


def _counters(renderer, n, cam, opts, buf) -> np.ndarray:
    lay = renderer.layout(n, [cam], 1, 0, opts)
    return buf[lay.counters: lay.counters + 64].cpu().numpy().view(np.int64)


def render_pair(renderer, g, cam: dict, opts: dict):
    """{divergence: (rgb [3][H][W], final_T [H][W], counters)} for one camera."""
    n = int(g["opacity_logits"].shape[0])
    out = {}
    for name, div in DIVERGENCES.items():
        o = dict(opts, divergence=div, mip=0)
        outs, (buf, _) = renderer.render(g, [cam], o, keep_workspace=True)
        out[name] = (outs[0]["rgb"], outs[0]["final_T"], _counters(renderer, n, cam, renderer.resolve_options(n, [cam], o), buf))
    return out


def compare(pair) -> Dict[str, float]:
    (rgb_r, T_r, c_r), (rgb_g, T_g, c_g) = pair["ray"], pair["gs"]
    d = (rgb_g - rgb_r).double()
    mse = float((d * d).mean())
    return {"psnr": float("inf") if mse == 0 else 10.0 * math.log10(1.0 / mse),
            "max_dT": float((T_g - T_r).abs().max()),
            "kept_ray": int(c_r[4]), "kept_gs": int(c_g[4]),
            "listed_ray": int(c_r[3]), "listed_gs": int(c_g[3])}


def evaluate(renderer, g, cams: Sequence[dict], distances: Sequence[float], opts: dict):
    """{distance: compare(...)} along the trajectory."""
    return {float(d): compare(render_pair(renderer, g, c, opts)) for d, c in zip(distances, cams)}


DISTANCES = (6.0, 3.0, 1.5, 0.8, 0.5, 0.35)


def main():
    """python -m paper_2503_18682_amd.artifact_eval [--n N] [--width W --height H]
    prints one JSON line with the comparison along the trajectory."""
    import argparse
    import json

    import scenegen
    from . import renderer as R

    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=20_000)
    ap.add_argument("--width", type=int, default=1280)
    ap.add_argument("--height", type=int, default=960)
    ap.add_argument("--seed", type=int, default=72)
    a = ap.parse_args()
    sc = scenegen.wall_scene(a.seed, a.n)
    cams = scenegen.approach_cameras(DISTANCES, a.width, a.height)
    g = {k: torch.from_numpy(np.ascontiguousarray(sc[k])).cuda() for k in R.PARAM_KEYS}
    g["sh_degree"] = int(sc["sh_degree"])
    r = R.Renderer(0)
    res = evaluate(r, g, cams, DISTANCES, scenegen.default_options(tile_w=8, tile_h=16))
    print(json.dumps({"scene": f"wall of {a.n} flattened Gaussians, seed {a.seed}", "view": [a.width, a.height, 90.0],
                      "by_distance": {str(d): v for d, v in res.items()}}))
    r.close()


if __name__ == "__main__":
    main()
