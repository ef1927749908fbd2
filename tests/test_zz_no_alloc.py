"""The no-allocation render entry point (rgs_render_noalloc) against the
workspace entry point (rgs_render) through the C ABI: two calls in a row,
the second with a smaller scene and image, give the same images bit for bit
and the same instance count; a frame too large for the scratch is rejected
before any GPU work."""
import ctypes as C

import numpy as np
import pytest
import torch

import scenegen
from gpu_helpers import render_with_ws, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def r():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_18682_amd import renderer as R

    rr = R.Renderer(0)
    yield rr
    rr.close()


def _noalloc(r, g, cams, opts):
    from paper_2503_18682_amd import _lib
    from paper_2503_18682_amd import renderer as R

    outs = r.allocate_outputs(cams)
    need = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    G = R.make_gaussians(g)
    o = R.make_options(opts)
    st = r.lib.rgs_render_noalloc(r.ctx, C.byref(G), R.make_cameras(cams), len(cams), C.byref(o),
                                  R.Renderer._view_outs(outs), C.c_void_p(need.data_ptr()), R._stream(r.device))
    msg = r.lib.rgs_last_error(r.ctx)
    assert st == _lib.RGS_OK, msg
    torch.cuda.synchronize()
    return [{k: v.cpu().numpy() for k, v in x.items()} for x in outs], int(need.item())


def test_noalloc_matches_the_workspace_entry_point_on_two_calls(r):
    cases = [
        ("c0 1000 Gaussians 128x128", scenegen.make_workload("c0")["scene"],
         [scenegen.pinhole(scenegen.look_at((0.0, 0.0, -4.0)), 128, 128, 60.0)], dict(mip=0)),
        ("300 Gaussians, 2 views 96x64 and 40x52, MIP", scenegen.tiny_scene(71, 300, sh_degree=2),
         [scenegen.pinhole(scenegen.look_at((0.2, 0.1, -3.5)), 96, 64, 60.0),
          scenegen.pinhole(scenegen.look_at((-1.0, 0.3, -3.0)), 40, 52, 70.0)], dict(mip=1)),
    ]
    for label, sc, cams, mode in cases:
        say(f"case no-alloc render: {label}")
        opts = scenegen.default_options(tile_w=8, tile_h=16, background=(0.1, 0.2, 0.3), **mode)
        g = to_dev(sc)
        got, need = _noalloc(r, g, cams, opts)
        want, _, _, _, (ok, m) = render_with_ws(r, sc, cams, opts)
        assert ok and need == m, (need, m)
        for v in range(len(cams)):
            for k in ("rgb", "final_T", "n_contrib"):
                assert np.array_equal(got[v][k], want[v][k]), (label, v, k)
        say(f"  {len(cams)} view(s) bit-identical to rgs_render, {need} instances")


def test_noalloc_rejects_a_frame_larger_than_its_scratch(r):
    from paper_2503_18682_amd import _lib
    from paper_2503_18682_amd import renderer as R

    n = 2_000_000  # about 360 MB of per-Gaussian-view state: more than the 256 MiB scratch
    g = {k: torch.zeros(shape, dtype=torch.float32, device="cuda")
         for k, shape in (("means", (3, n)), ("log_scales", (3, n)), ("quats", (4, n)), ("opacity_logits", (n,)),
                          ("sh", (1, 3, n)))}
    g["sh_degree"] = 0
    cams = [scenegen.pinhole(scenegen.look_at((0.0, 0.0, -4.0)), 64, 64, 60.0)]
    outs = r.allocate_outputs(cams)
    G = R.make_gaussians(g)
    o = R.make_options(scenegen.default_options())
    st = r.lib.rgs_render_noalloc(r.ctx, C.byref(G), R.make_cameras(cams), 1, C.byref(o), R.Renderer._view_outs(outs),
                                  None, R._stream(r.device))
    msg = r.lib.rgs_last_error(r.ctx).decode()
    say(f"  rejected: {msg}")
    assert st == _lib.RGS_EINVAL and "scratch" in msg
