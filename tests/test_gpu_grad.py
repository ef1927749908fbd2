"""GPU backward pass against the oracle's analytic gradient (itself pinned to
FP64 central differences on the CPU).  Bar per parameter tensor:
max|g_gpu - g_oracle| <= 1e-3 max|g_oracle| + 1e-7 and cosine >= 0.9999."""
import numpy as np
import pytest
import torch

import oracle
import scenegen
from gpu_helpers import PARAM_KEYS, assert_image_close, assert_pixels_close, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def r():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_18682_amd import renderer as R

    rr = R.Renderer(0)
    yield rr
    rr.close()


def _compare(g_gpu, g_ref, label, rel=1e-3):
    for k in PARAM_KEYS:
        a = g_gpu[k].double().cpu().numpy().reshape(-1)
        b = np.asarray(g_ref[k], np.float64).reshape(-1)
        scale = np.abs(b).max()
        err = np.abs(a - b).max()
        cos = float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-300)) if scale > 0 else 1.0
        say(f"  {label} {k}: max err {err:.3e} (scale {scale:.3e}) cosine {cos:.7f}")
        assert err <= rel * scale + 1e-7, (label, k)
        assert cos >= 0.9999 or scale == 0, (label, k)


def _l1_grad(img, target, n_total):
    return np.sign(img - target) / n_total


def test_fd_subcase_l1(r):
    """64 Gaussians, 32x32, SH3, L1 loss against a seeded noise target."""
    from paper_2503_18682_amd import _lib

    scene, cam = scenegen.fd_subcase()
    opts = scenegen.default_options()
    say("case grad fd-subcase 64 Gaussians 32x32")
    g = to_dev(scene)
    outs, (buf, ws) = r.render(g, [cam], opts, flags=_lib.RGS_WS_BACKWARD, keep_workspace=True)
    img = outs[0]["rgb"].cpu().numpy()
    target = np.random.default_rng(3).uniform(0, 1, img.shape)
    dl = _l1_grad(img, target, img.size).astype(np.float32)
    grads = r.backward(g, [cam], outs, [torch.from_numpy(dl).cuda()], ws, opts)
    ref = oracle.backward(scene, cam, opts, dl.astype(np.float64))
    _compare(grads, ref, "fd-subcase")


@pytest.mark.parametrize("extra", [dict(alpha_max=0.3), dict(p_min=0.05)], ids=["alpha_max_0.3", "p_min_0.05"])
def test_clamp_and_support_threshold_extremes(r, extra):
    """The FD subcase with most fragments clamped at alpha_max (which then
    pass no gradient to omega), and with a support threshold p_min 13 times
    the default (eqs. 2-3): image and gradients against the oracle."""
    from paper_2503_18682_amd import _lib

    scene, cam = scenegen.fd_subcase()
    opts = scenegen.default_options(**extra)
    say(f"case grad fd-subcase {extra}")
    g = to_dev(scene)
    outs, (buf, ws) = r.render(g, [cam], opts, flags=_lib.RGS_WS_BACKWARD, keep_workspace=True)
    assert_image_close(outs[0]["rgb"].cpu().numpy(), outs[0]["final_T"].cpu().numpy(),
                       oracle.render(scene, cam, opts), label=str(extra))
    img = outs[0]["rgb"].cpu().numpy()
    target = np.random.default_rng(4).uniform(0, 1, img.shape)
    dl = _l1_grad(img, target, img.size).astype(np.float32)
    grads = r.backward(g, [cam], outs, [torch.from_numpy(dl).cuda()], ws, opts)
    ref = oracle.backward(scene, cam, opts, dl.astype(np.float64))
    _compare(grads, ref, f"fd-subcase {extra}")


def test_multi_view_sparse_pixels(r):
    """Two views in one batch; dL/dC nonzero on sampled pixels only."""
    from paper_2503_18682_amd import _lib

    sc = scenegen.tiny_scene(41, 20000, sh_degree=3, half_extent=1.5, log_scale_mean=-3.5, log_scale_std=0.6)
    cams = [scenegen.pinhole(scenegen.look_at((0, 0.5, -4)), 320, 212, 50),
            scenegen.pinhole(scenegen.look_at((2.5, 0.0, -3)), 160, 240, 60)]
    opts = scenegen.default_options(background=(0.05, 0.1, 0.2))
    say("case grad 2 views, 20000 Gaussians, sparse pixels")
    g = to_dev(sc)
    outs, (buf, ws) = r.render(g, cams, opts, flags=_lib.RGS_WS_BACKWARD, keep_workspace=True)
    rng = np.random.default_rng(4)
    dls = []
    ref = {k: np.zeros(sc[k].shape) for k in PARAM_KEYS}
    for v, cam in enumerate(cams):
        H, W = cam["height"], cam["width"]
        dl = np.zeros((3, H, W), np.float32)
        ys, xs = rng.integers(0, H, 300), rng.integers(0, W, 300)
        dl[:, ys, xs] = rng.normal(0, 1, (3, 300)).astype(np.float32)
        dls.append(torch.from_numpy(dl).cuda())
        rv = oracle.backward(sc, cam, opts, dl.astype(np.float64))
        for k in PARAM_KEYS:
            ref[k] += rv[k]
    grads = r.backward(g, cams, outs, dls, ws, opts)
    _compare(grads, ref, "2-view sparse", rel=2e-3)


def test_long_tile_lists(r):
    """Dense cluster with tile lists of ~1,500 entries (split into half-tile
    work items in the forward; the backward composites each tile whole)."""
    from paper_2503_18682_amd import _lib

    sc = scenegen.tiny_scene(36, 4000, sh_degree=1, half_extent=0.35, log_scale_mean=-3.2, log_scale_std=0.5)
    # low opacity keeps every pixel's transmittance far above T_eps (no
    # termination decision near its threshold)
    sc["opacity_logits"][:] = -3.0 + 0.3 * np.random.default_rng(0).standard_normal(4000).astype(np.float32)
    cam = scenegen.pinhole(scenegen.look_at((0.0, 0.0, -4.0)), 96, 80, 30)
    opts = scenegen.default_options(tile_w=8, tile_h=16, background=(0.1, 0.2, 0.3))
    say("case grad long lists, 4000 Gaussians 96x80")
    g = to_dev(sc)
    outs, (buf, ws) = r.render(g, [cam], opts, flags=_lib.RGS_WS_BACKWARD, keep_workspace=True)
    rng = np.random.default_rng(7)
    dl = (rng.normal(0, 1, (3, 80, 96)) * (rng.uniform(size=(80, 96)) < 0.3)).astype(np.float32)
    grads = r.backward(g, [cam], outs, [torch.from_numpy(dl).cuda()], ws, opts)
    ref = oracle.backward(sc, cam, opts, dl.astype(np.float64))
    _compare(grads, ref, "long lists", rel=2e-3)


def test_autograd_function_matches_direct_backward(r):
    from paper_2503_18682_amd import _lib
    from paper_2503_18682_amd import renderer as R

    scene, cam = scenegen.fd_subcase(seed=2005)
    opts = scenegen.default_options()
    say("case autograd function")
    g = to_dev(scene, requires_grad=True)
    img = R.render(r, g, [cam], opts)[0]
    target = torch.rand(img.shape, device=img.device, generator=torch.Generator(device=img.device).manual_seed(0))
    loss = (img - target).abs().mean()
    loss.backward()
    g2 = to_dev(scene)
    outs, (buf, ws) = r.render(g2, [cam], opts, flags=_lib.RGS_WS_BACKWARD, keep_workspace=True)
    dl = torch.sign(outs[0]["rgb"] - target) / img.numel()
    direct = r.backward(g2, [cam], outs, [dl], ws, opts)
    for k in PARAM_KEYS:
        a, b = g[k].grad, direct[k]
        assert torch.allclose(a, b, rtol=1e-4, atol=1e-7 * float(b.abs().max() + 1e-30)), k


def test_mip_fd_subcase_l1(r):
    """MIP on (eq. 17) with a large pixel filter: gradients through the
    widening and the opacity modulation against the oracle's (pinned to
    finite differences)."""
    from paper_2503_18682_amd import _lib

    scene, cam = scenegen.fd_subcase(seed=2004)
    opts = scenegen.default_options(mip=1, mip_sigma2_px=4.0)
    say("case grad MIP fd-subcase 64 Gaussians 32x32")
    g = to_dev(scene)
    outs, (buf, ws) = r.render(g, [cam], opts, flags=_lib.RGS_WS_BACKWARD, keep_workspace=True)
    img = outs[0]["rgb"].cpu().numpy()
    target = np.random.default_rng(6).uniform(0, 1, img.shape)
    dl = _l1_grad(img, target, img.size).astype(np.float32)
    grads = r.backward(g, [cam], outs, [torch.from_numpy(dl).cuda()], ws, opts)
    ref = oracle.backward(scene, cam, opts, dl.astype(np.float64))
    _compare(grads, ref, "MIP fd-subcase")


def test_mip_multi_view_sparse_pixels(r):
    """Two views with MIP at the default pixel filter (0.1 px^2)."""
    from paper_2503_18682_amd import _lib

    sc = scenegen.tiny_scene(42, 20000, sh_degree=2, half_extent=1.5, log_scale_mean=-4.0, log_scale_std=0.6)
    cams = [scenegen.pinhole(scenegen.look_at((0, 0.5, -4)), 320, 212, 50),
            scenegen.pinhole(scenegen.look_at((2.5, 0.0, -3)), 160, 240, 60)]
    opts = scenegen.default_options(mip=1)
    say("case grad MIP 2 views, 20000 Gaussians, sparse pixels")
    g = to_dev(sc)
    outs, (buf, ws) = r.render(g, cams, opts, flags=_lib.RGS_WS_BACKWARD, keep_workspace=True)
    rng = np.random.default_rng(5)
    dls = []
    ref = {k: np.zeros(sc[k].shape) for k in PARAM_KEYS}
    for v, cam in enumerate(cams):
        H, W = cam["height"], cam["width"]
        dl = np.zeros((3, H, W), np.float32)
        ys, xs = rng.integers(0, H, 300), rng.integers(0, W, 300)
        dl[:, ys, xs] = rng.normal(0, 1, (3, 300)).astype(np.float32)
        dls.append(torch.from_numpy(dl).cuda())
        rv = oracle.backward(sc, cam, opts, dl.astype(np.float64))
        for k in PARAM_KEYS:
            ref[k] += rv[k]
    grads = r.backward(g, cams, outs, dls, ws, opts)
    _compare(grads, ref, "MIP 2-view sparse", rel=2e-3)


def test_c3_full_size_sampled_gradients(r):
    """1M Gaussians, 4 views at 1600x1060 (the training-style workload): the
    L1 upstream gradient kept on every pixel of a 64-row band of view 0
    (102,400 pixels through the middle of the scene) and on 200 sampled pixels
    of each view."""
    from paper_2503_18682_amd import _lib

    w = scenegen.make_workload("c3")
    sc, cams, opts = w["scene"], w["cameras"], w["options"]
    say("case grad c3 full size: 1M Gaussians, 4 x 1600x1060")
    g = to_dev(sc)
    outs, (buf, ws) = r.render(g, cams, opts, flags=_lib.RGS_WS_BACKWARD, keep_workspace=True)
    rng = np.random.default_rng(6)
    dls = []
    ref = {k: np.zeros(sc[k].shape) for k in PARAM_KEYS}
    total = 3 * 1600 * 1060 * 4
    for v, cam in enumerate(cams):
        img = outs[v]["rgb"].cpu().numpy()
        full = np.sign(img - w["targets"][v]) / total
        mask = np.zeros(img.shape[1:], bool)
        mask[rng.integers(0, 1060, 200), rng.integers(0, 1600, 200)] = True
        if v == 0:
            mask[500:564, :] = True
        dl = np.where(mask[None], full, 0).astype(np.float32)
        dls.append(torch.from_numpy(dl).cuda())
        rv = oracle.backward(sc, cam, opts, dl.astype(np.float64))
        for k in PARAM_KEYS:
            ref[k] += rv[k]
    grads = r.backward(g, cams, outs, dls, ws, opts)
    _compare(grads, ref, "c3 sampled", rel=2e-3)


def test_c4_full_size_autotuned_forward_backward(r):
    """6M Gaussians, 16 cameras of random size (256..2560 x 256..1440) and
    FOV (40..90 deg) in one batch with the autotuned tile shape: every pixel
    of a 493x689 view and sampled pixels of a 2434x1264 one against the
    oracle, then the gradients of an upstream
    gradient on 200 pixels of one view (zero on the other 15)."""
    from paper_2503_18682_amd import _lib

    w = scenegen.make_workload("c4")
    sc, cams, opts0 = w["scene"], w["cameras"], w["options"]
    n = int(sc["opacity_logits"].shape[0])
    say("case c4 full size: 6M Gaussians, 16 uneven cameras, autotuned, forward + backward")
    g = to_dev(sc)
    _, (buf, ws) = r.render(g, cams, opts0, keep_workspace=True)
    need = r.status(ws)[1]
    del buf, ws
    buf, ws = r.new_workspace(n, cams, int(need * 3) + 4096, 0, opts0)
    outs = r.allocate_outputs(cams)
    best, ms = r.autotune(g, cams, ws, outs, reps=1)
    say(f"  autotuned tile {best['tile_w']}x{best['tile_h']} ({ms:.2f} ms per batch)")
    del buf, ws
    outs, (buf, ws) = r.render(g, cams, best, flags=_lib.RGS_WS_BACKWARD, keep_workspace=True)
    rng = np.random.default_rng(10)
    # every pixel of view 0 (493x689), sampled pixels of view 7 (2434x1264)
    host0 = {k: t.cpu().numpy() for k, t in outs[0].items()}
    assert_image_close(host0["rgb"], host0["final_T"], oracle.render(sc, cams[0], best),
                       label=f"c4 view 0 {cams[0]['width']}x{cams[0]['height']}, every pixel")
    cam = cams[7]
    px, py = rng.integers(0, cam["width"], 2000), rng.integers(0, cam["height"], 2000)
    ref = oracle.render_pixels(sc, cam, best, px, py)
    g_rgb = outs[7]["rgb"].cpu().numpy()[:, py, px].T
    g_T = outs[7]["final_T"].cpu().numpy()[py, px]
    assert_pixels_close(g_rgb, g_T, ref, label=f"c4 view 7 {cam['width']}x{cam['height']} sampled")
    v = 7
    dls = [torch.zeros_like(o["rgb"]) for o in outs]
    H, W = cams[v]["height"], cams[v]["width"]
    dl = np.zeros((3, H, W), np.float32)
    dl[:, rng.integers(0, H, 200), rng.integers(0, W, 200)] = rng.normal(0, 1, (3, 200)).astype(np.float32)
    dls[v] = torch.from_numpy(dl).cuda()
    grads = r.backward(g, cams, outs, dls, ws, best)
    ref = oracle.backward(sc, cams[v], best, dl.astype(np.float64))
    _compare(grads, ref, "c4 view 7 sampled", rel=2e-3)


def test_backward_takes_the_tile_shape_of_the_frame_in_its_workspace(r):
    """The backward pass of a workspace uses the tile shape of the frame last
    rendered into it when the options leave the shape open (0, 0), even when
    the context would now resolve (0, 0) to another shape (here the 8x16
    default against a 16x16 frame); an explicit shape that differs from the
    frame's is rejected before any GPU work."""
    from paper_2503_18682_amd import _lib

    say("case backward tile shape of the workspace's frame")
    sc = scenegen.tiny_scene(38, 1500, sh_degree=1)
    cams = [scenegen.pinhole(scenegen.look_at((0, 0, -4)), 120, 100, 60)]
    g = to_dev(sc)
    o16 = scenegen.default_options(tile_w=16, tile_h=16)
    assert (r.layout(1500, cams, 1, 0, dict(o16, tile_w=0, tile_h=0)).tile_w,
            r.layout(1500, cams, 1, 0, dict(o16, tile_w=0, tile_h=0)).tile_h) == (8, 16)
    buf, ws = r.new_workspace(1500, cams, 500000, _lib.RGS_WS_BACKWARD, o16)
    outs = r.allocate_outputs(cams)
    dl = [torch.from_numpy(np.random.default_rng(3).normal(0, 1, (3, 100, 120)).astype(np.float32)).cuda()]
    r.render_into(g, cams, outs, ws, o16)
    want = r.backward(g, cams, outs, dl, ws, o16)
    r.render_into(g, cams, outs, ws, o16)
    got = r.backward(g, cams, outs, dl, ws, dict(o16, tile_w=0, tile_h=0))
    for k in PARAM_KEYS:
        a, b = want[k].cpu().numpy(), got[k].cpu().numpy()
        assert np.abs(a - b).max() <= 1e-5 * max(np.abs(a).max(), 1e-6), k
    with pytest.raises(RuntimeError, match="differs from the 16x16"):
        r.backward(g, cams, outs, dl, ws, dict(o16, tile_w=8, tile_h=16))
    with pytest.raises(RuntimeError):
        r.backward(g, cams, outs, dl, ws, dict(o16, mip=1))
