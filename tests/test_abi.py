"""Host-only checks of the C ABI: the library loads without a GPU, exports every
function include/raygs.h declares, the ctypes mirrors match the C layouts, and
the host-side validation and workspace layout behave as documented."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

import scenegen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "raygs.h")


@pytest.fixture(scope="module")
def lib():
    from paper_2503_18682_amd import _lib

    if not os.path.exists(_lib.LIB_PATH):
        import __graft_entry__

        __graft_entry__.build()
    return _lib.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rgs_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name
    from paper_2503_18682_amd import _lib

    assert set(names) == set(_lib.EXPORTS)


def test_ctypes_layouts_match_the_header(tmp_path, lib):
    from paper_2503_18682_amd import _lib

    structs = dict(rgs_gaussians=_lib.Gaussians, rgs_camera=_lib.Camera, rgs_options=_lib.Options,
                   rgs_view_out=_lib.ViewOut, rgs_gaussian_grads=_lib.GaussianGrads, rgs_workspace=_lib.Workspace,
                   rgs_workspace_layout=_lib.WorkspaceLayout)
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "raygs.h"', "int main(void){"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = dict(line.split() for line in subprocess.check_output([str(exe)]).decode().splitlines())
    for cname, py in structs.items():
        assert int(out[cname]) == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(out[f"{cname}.{f}"]) == getattr(py, f).offset, (cname, f)


def _args(n=100, cams=None, **opt):
    from paper_2503_18682_amd import renderer

    cams = cams or [scenegen.pinhole(scenegen.look_at((0, 0, -4)), 64, 48, 60)]
    return n, renderer.make_cameras(cams), len(cams), renderer.make_options(dict(scenegen.default_options(), **opt))


def _size(lib, n, arr, nv, opts, capacity=1000, flags=0):
    out = C.c_size_t()
    st = lib.rgs_workspace_size(None, n, arr, nv, C.byref(opts), capacity, flags, C.byref(out))
    return st, out.value


def test_workspace_size_validation(lib):
    from paper_2503_18682_amd import _lib

    n, arr, nv, opts = _args()
    assert _size(lib, n, arr, nv, opts)[0] == _lib.RGS_OK
    assert _size(lib, -1, arr, nv, opts)[0] == _lib.RGS_EINVAL
    assert _size(lib, n, arr, 0, opts)[0] == _lib.RGS_EINVAL
    assert _size(lib, n, arr, nv, opts, capacity=0)[0] == _lib.RGS_EINVAL
    assert _size(lib, n, arr, nv, opts, flags=8)[0] == _lib.RGS_EINVAL
    for bad in (dict(p_min=0.0), dict(p_min=1.0), dict(alpha_max=0.001), dict(alpha_max=1.0), dict(t_eps=-1.0),
                dict(mip=4), dict(mip=-1), dict(mip_sigma2_px=-0.1), dict(divergence=2), dict(divergence=1, mip=1), dict(tile_w=12, tile_h=12), dict(tile_w=64, tile_h=64),
                dict(near_z=float("nan")), dict(near_z=0.0), dict(near_z=-0.5), dict(near_z=float("inf")),
                dict(background=(0, float("inf"), 0))):
        _, a2, _, o2 = _args(**bad)
        assert _size(lib, n, a2, nv, o2)[0] == _lib.RGS_EINVAL, bad
    # exact MIP records are 112 B instead of 64 B per Gaussian-view
    st0, b0 = _size(lib, n, arr, nv, opts)
    _, a3, _, o3 = _args(mip=2)
    st2, b2 = _size(lib, n, a3, nv, o3)
    assert st0 == st2 == _lib.RGS_OK and b2 > b0
    for cam_bad in (dict(width=0), dict(height=20000), dict(fx=0.0), dict(fy=-1.0), dict(cx=float("nan"))):
        c = scenegen.pinhole(scenegen.look_at((0, 0, -4)), 64, 48, 60)
        c.update(cam_bad)
        _, a2, _, o2 = _args(cams=[c])
        assert _size(lib, n, a2, 1, o2)[0] == _lib.RGS_EINVAL, cam_bad
    w = scenegen.look_at((0, 0, -4))
    w[1, 2] = np.inf
    _, a2, _, o2 = _args(cams=[scenegen.pinhole(w, 64, 48, 60)])
    assert _size(lib, n, a2, 1, o2)[0] == _lib.RGS_EINVAL
    # n * n_views must stay below 2^28
    assert _size(lib, 2**27, arr, nv, opts)[0] == _lib.RGS_OK
    cams = [scenegen.pinhole(scenegen.look_at((0, 0, -4)), 64, 48, 60)] * 2
    _, a2, _, o2 = _args(cams=cams)
    assert _size(lib, 2**27, a2, 2, o2)[0] == _lib.RGS_EINVAL


def test_workspace_layout(lib):
    from paper_2503_18682_amd import _lib

    cams = [scenegen.pinhole(scenegen.look_at((0, 0, -4)), 131, 77, 60),
            scenegen.pinhole(scenegen.look_at((1, 0, -4)), 40, 33, 60)]
    n, arr, nv, opts = _args(n=1000, cams=cams)
    lay = _lib.WorkspaceLayout()
    assert lib.rgs_get_workspace_layout(None, n, arr, nv, C.byref(opts), 5000, 0, C.byref(lay)) == 0
    assert lay.n_records == 2000 and lay.capacity == 5000
    assert lay.total_tiles == 9 * 5 + 3 * 3 and lay.tile_bits == 6
    assert lay.record_grads == 0
    offs = [getattr(lay, k) for k in ("counters", "views", "records", "depth_keys", "boxes", "bin_boxes", "conics",
                                      "tile_counts",
                                      "order", "offsets", "inst_tiles", "inst_ids", "tile_ranges")]
    assert all(o % 256 == 0 for o in offs) and len(set(offs)) == len(offs)
    assert max(offs) < lay.total_bytes
    assert _size(lib, n, arr, nv, opts, 5000)[1] == lay.total_bytes
    lay2 = _lib.WorkspaceLayout()
    lib.rgs_get_workspace_layout(None, n, arr, nv, C.byref(opts), 5000, 1, C.byref(lay2))
    assert lay2.record_grads >= lay.total_bytes - 256 and lay2.total_bytes >= lay.total_bytes + 2000 * 64
    big = _size(lib, n, arr, nv, opts, 50000)[1]
    assert big - lay.total_bytes >= 45000 * 16
    # tile shape (0, 0) with no tuned shape (no context) is the default 8x16
    _, a3, _, o3 = _args(n=10, tile_w=0, tile_h=0)
    lay3 = _lib.WorkspaceLayout()
    lib.rgs_get_workspace_layout(None, 10, a3, 1, C.byref(o3), 100, 0, C.byref(lay3))
    assert (lay3.tile_w, lay3.tile_h, lay3.total_tiles) == (8, 16, 8 * 3)


def test_create_without_gpu_fails_cleanly(lib):
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = C.c_void_p()
    assert lib.rgs_create(0, C.byref(h)) != 0
    assert not h.value


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_2503_18682_amd import _lib

    with pytest.raises(ImportError):
        _lib.load(str(tmp_path / "missing.so"))
