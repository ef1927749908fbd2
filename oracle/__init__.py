"""CPU FP64 oracle for ray-based Gaussian splatting -- TEST INFRASTRUCTURE ONLY.

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It shares no code with the HIP renderer.
"""
from .oracle import (  # noqa: F401
    build_library,
    load,
    preprocess,
    render,
    render_pixels,
    support_cells,
    backward,
    tile_lists,
    sh_basis,
    divergence,
    rot_mu_v,
    mip_exact_weight,
    CULL,
    HAZARD,
)
