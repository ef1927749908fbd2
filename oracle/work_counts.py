"""Write the algorithmic work counts of the benchmark frames, computed by the
CPU oracle only (TEST / MEASUREMENT INFRASTRUCTURE).

For each view of a workload it records, from a full oracle render:
  visible        Gaussians passing every cull
  instances      listed (Gaussian, tile) pairs at the recorded tile shape
  fragments      pixel centres inside a projected quad (what a rasteriser
                 would shade for the paper's quads), along each pixel's
                 depth order up to the entry at which compositing stops
  box_pairs      pixel centres inside a Gaussian's pixel box, counted the
                 same way
  contributions  fragments that were composited (omega >= p_min, before
                 early termination)
These are the denominators of the roofline figures (work per launch).

    python -m oracle.work_counts c1 [--tile 8x16] [--divergence ray|gs] [--out tests/golden/work_counts_c1.json]

The benchmark's tile shape is 8x16; c2 and c3 are counted with it as well
(python -m oracle.work_counts c2 --tile 8x16).

With --divergence gs the frames are rendered with the linearised divergence
(written to work_counts_<workload>_gs.json); its fragments are the pixel
centres inside each splat's box.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import scenegen  # noqa: E402


def counts(name: str, views=None, tile=None, divergence="ray"):
    w = scenegen.make_workload(name)
    sc, cams, opts = w["scene"], w["cameras"], dict(w["options"])
    if divergence == "gs":
        opts["divergence"], opts["mip"] = 1, 0
    if tile:
        opts["tile_w"], opts["tile_h"] = (int(x) for x in tile.lower().split("x"))
    out = []
    for v, cam in enumerate(cams):
        if views is not None and v not in views:
            continue
        t = time.time()
        r = oracle.render(sc, cam, opts, branches=False)
        c = dict(r["counters"], view=v, width=cam["width"], height=cam["height"])
        out.append(c)
        print(f"{name} view {v}: {c} ({time.time() - t:.1f} s)", flush=True)
    return dict(workload=name, n=int(sc["opacity_logits"].shape[0]), options=opts, views=out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", default="c1", nargs="?")
    ap.add_argument("--out", default=None)
    ap.add_argument("--tile", default=None, help="tile shape WxH (default: the workload's)")
    ap.add_argument("--divergence", default="ray", choices=["ray", "gs"])
    a = ap.parse_args()
    res = counts(a.workload, tile=a.tile, divergence=a.divergence)
    suffix = "_gs" if a.divergence == "gs" else ""
    path = a.out or os.path.join(ROOT, "tests", "golden", f"work_counts_{a.workload}{suffix}.json")
    with open(path, "w") as f:
        json.dump(res, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
