"""GPU parity of the exact MIP path (mip = 2: the per-ray widening and
modulation of Sec. 5 without its approximations) against the CPU oracle,
through the C ABI.  Same bars as the other parity tests: images within 2e-4
outside the oracle's hazard mask, tile lists bit-exact."""
import numpy as np
import pytest
import torch

import oracle
import scenegen
from gpu_helpers import (assert_image_close, assert_pixels_close, instance_lists, oracle_box_tiles,
                         oracle_lists_without_hazards,
                         render_with_ws, say, to_dev)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def r():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_18682_amd import renderer as R

    rr = R.Renderer(0)
    yield rr
    rr.close()


def _lists_match(buf, lay, sp, cam, opts, label):
    tiles, ids = instance_lists(buf, lay)
    ot, _, oi, bad = oracle_lists_without_hazards(sp, cam, opts)
    keep = ~np.isin(ids, list(bad)) if bad else np.ones_like(ids, bool)
    say(f"  {label}: {len(ids)} listed, {len(bad)} hazard Gaussians excluded")
    assert np.array_equal(tiles[keep], ot) and np.array_equal(ids[keep], oi)


@pytest.mark.parametrize("shape", [(8, 8), (8, 16), (32, 32)])
def test_exact_mip_ragged_image_and_lists(r, shape):
    """A ragged view with strongly anisotropic Gaussians and a footprint
    large enough that some Gaussians get no bound (the whole view): image,
    box tile counts and tile lists, and tile-shape independence."""
    say(f"case exact MIP ragged 131x77 tile {shape}")
    sc = scenegen.tiny_scene(36, 400, sh_degree=2, half_extent=1.2, log_scale_mean=-3.5, log_scale_std=1.0)
    cam = scenegen.pinhole(scenegen.look_at((-0.3, 0.5, -3.0)), 131, 77, 70)
    opts = scenegen.default_options(mip=2, mip_sigma2_px=1.5, tile_w=shape[0], tile_h=shape[1],
                                    background=(0.2, 0.1, 0.05))
    outs, buf, ws, lay, (ok, m) = render_with_ws(r, sc, [cam], opts)
    assert ok
    ref = oracle.render(sc, cam, opts)
    assert_image_close(outs[0]["rgb"], outs[0]["final_T"], ref, label=f"exact MIP {shape}")
    sp = oracle.preprocess(sc, cam, opts)
    whole = int(sp["whole"][sp["cull"] == 0].sum())
    say(f"  {whole} Gaussians listed in the whole view")
    assert whole > 0
    assert m == oracle_box_tiles(sp)[1].sum()
    _lists_match(buf, lay, sp, cam, opts, f"exact MIP {shape} lists")
    base = dict(opts, tile_w=16, tile_h=16)
    b_outs = render_with_ws(r, sc, [cam], base)[0]
    assert np.array_equal(outs[0]["rgb"], b_outs[0]["rgb"]) and np.array_equal(outs[0]["final_T"], b_outs[0]["final_T"])


def test_exact_mip_small_footprint_and_zero_footprint(r):
    """The paper's footprint (0.1 px^2) on a denser scene, and sigma = 0,
    where the exact path lists exactly the plain path's tiles and renders the
    plain image (the oracle's mode-0 image)."""
    sc = scenegen.tiny_scene(37, 3000, sh_degree=3, half_extent=1.5, log_scale_mean=-4.0, log_scale_std=0.8)
    cam = scenegen.pinhole(scenegen.look_at((0.2, -0.4, -4.0)), 203, 141, 60)
    say("case exact MIP, sigma^2 = 0.1 px^2, 3000 Gaussians, 203x141")
    opts = scenegen.default_options(mip=2, mip_sigma2_px=0.1)
    outs, buf, ws, lay, (ok, m) = render_with_ws(r, sc, [cam], opts)
    assert ok
    assert_image_close(outs[0]["rgb"], outs[0]["final_T"], oracle.render(sc, cam, opts), label="exact MIP 0.1")
    _lists_match(buf, lay, oracle.preprocess(sc, cam, opts), cam, opts, "exact MIP 0.1 lists")
    say("case exact MIP, sigma = 0")
    zero = scenegen.default_options(mip=2, mip_sigma2_px=0.0)
    plain = scenegen.default_options()
    z_outs, z_buf, _, z_lay, (ok_z, m_z) = render_with_ws(r, sc, [cam], zero)
    p_outs, p_buf, _, p_lay, (ok_p, m_p) = render_with_ws(r, sc, [cam], plain)
    assert ok_z and ok_p and m_z == m_p
    zt, zi = instance_lists(z_buf, z_lay)
    pt, pi = instance_lists(p_buf, p_lay)
    assert np.array_equal(zt, pt) and np.array_equal(zi, pi)
    assert_image_close(z_outs[0]["rgb"], z_outs[0]["final_T"], oracle.render(sc, cam, plain), label="exact MIP sigma=0")


def test_exact_mip_batch_graph_replays(r):
    """Uneven views in one batch, replayed from a captured graph: equal to
    eager renders bit for bit and to the oracle."""
    from paper_2503_18682_amd import renderer as R

    sc = scenegen.tiny_scene(38, 3000, sh_degree=2, half_extent=1.5, log_scale_mean=-3.5, log_scale_std=0.8)
    cams = [scenegen.pinhole(scenegen.look_at((0, 0, -4)), 160, 120, 60),
            scenegen.pinhole(scenegen.look_at((2, 1, -3.5)), 97, 211, 75)]
    opts = scenegen.default_options(mip=2, mip_sigma2_px=0.5)
    g = to_dev(sc)
    say("case exact MIP graph plan: 2 uneven views, 3 replays")
    br = R.BatchRenderer(r, 3000, 2, cams, capacity=400000, options=opts)
    for rep in range(3):
        moved = []
        for c in cams:
            c2 = dict(c)
            c2["w2c"] = c["w2c"].copy()
            c2["w2c"][1, 3] += 0.04 * rep
            moved.append(c2)
        outs = br.launch(g, moved)
        ok, _ = br.status()
        assert ok
        eager = render_with_ws(r, sc, moved, opts)[0]
        for v in range(2):
            assert np.array_equal(outs[v]["rgb"].cpu().numpy(), eager[v]["rgb"]), (rep, v)
            assert np.array_equal(outs[v]["final_T"].cpu().numpy(), eager[v]["final_T"]), (rep, v)
        if rep == 0:
            for v in range(2):
                assert_image_close(eager[v]["rgb"], eager[v]["final_T"], oracle.render(sc, moved[v], opts),
                                   label=f"exact MIP batch view {v}")
    br.close()


def test_exact_mip_c2_full_size_sampled_pixels(r):
    """The stereo workload (3M Gaussians, 8 views up to 4128x4416) with the
    exact MIP in one graph replay: sampled pixels of the largest and the
    smallest eye against the oracle."""
    from paper_2503_18682_amd import renderer as R

    w = scenegen.make_workload("c2")
    sc, cams = w["scene"], w["cameras"]
    opts = dict(w["options"], mip=2, tile_w=8, tile_h=16)
    n = int(sc["opacity_logits"].shape[0])
    say("case exact MIP c2 full size: 3M Gaussians, 8 stereo views, one graph replay")
    g = to_dev(sc)
    _, (buf, ws) = r.render(g, cams, opts, keep_workspace=True)
    need = r.status(ws)[1]
    del buf, ws
    br = R.BatchRenderer(r, n, sc["sh_degree"], cams, int(need * 1.1) + 4096, options=opts)
    outs = br.launch(g, cams)
    ok, _ = br.status()
    assert ok
    rng = np.random.default_rng(9)
    for v in (2, 5):
        cam = cams[v]
        host = {k: t.cpu().numpy() for k, t in outs[v].items()}
        px = rng.integers(0, cam["width"], 150)
        py = rng.integers(0, cam["height"], 150)
        ref = oracle.render_pixels(sc, cam, opts, px, py)
        assert_pixels_close(host["rgb"][:, py, px].T, host["final_T"][py, px], ref,
                            label=f"exact MIP view {v} {cam['width']}x{cam['height']} sampled")
    br.close()


def test_exact_mip_gradients_match_oracle(r):
    """The backward of the exact MIP weight (per-ray widening and modulation)
    against the oracle's analytic gradient, which central differences pin:
    the finite-difference subcase at a 4 px^2 footprint, and two views with
    sparse pixels at 0.5 px^2."""
    from paper_2503_18682_amd import _lib
    from test_gpu_grad import _compare

    scene, cam = scenegen.fd_subcase(seed=2008)
    opts = scenegen.default_options(mip=2, mip_sigma2_px=4.0)
    say("case exact MIP grad fd-subcase 64 Gaussians 32x32")
    g = to_dev(scene)
    outs, (buf, ws) = r.render(g, [cam], opts, flags=_lib.RGS_WS_BACKWARD, keep_workspace=True)
    img = outs[0]["rgb"].cpu().numpy()
    target = np.random.default_rng(14).uniform(0, 1, img.shape)
    dl = (np.sign(img - target) / img.size).astype(np.float32)
    grads = r.backward(g, [cam], outs, [torch.from_numpy(dl).cuda()], ws, opts)
    _compare(grads, oracle.backward(scene, cam, opts, dl.astype(np.float64)), "exact MIP fd-subcase")

    sc = scenegen.tiny_scene(54, 20000, sh_degree=2, half_extent=1.5, log_scale_mean=-4.0, log_scale_std=0.6)
    cams = [scenegen.pinhole(scenegen.look_at((0, 0.5, -4)), 320, 212, 50),
            scenegen.pinhole(scenegen.look_at((2.5, 0.0, -3)), 160, 240, 60)]
    opts = scenegen.default_options(mip=2, mip_sigma2_px=0.5)
    say("case exact MIP grad 2 views, 20000 Gaussians, sparse pixels")
    g = to_dev(sc)
    outs, (buf, ws) = r.render(g, cams, opts, flags=_lib.RGS_WS_BACKWARD, keep_workspace=True)
    rng = np.random.default_rng(15)
    dls, ref = [], {k: 0.0 for k in ("means", "log_scales", "quats", "opacity_logits", "sh")}
    for cam in cams:
        H, W = cam["height"], cam["width"]
        dl = np.zeros((3, H, W), np.float32)
        idx = rng.choice(H * W, 400, replace=False)
        dl.reshape(3, -1)[:, idx] = rng.normal(0, 1, (3, 400))
        dls.append(torch.from_numpy(dl).cuda())
        o = oracle.backward(sc, cam, opts, dl.astype(np.float64))
        ref = {k: ref[k] + o[k] for k in ref}
    grads = r.backward(g, cams, outs, dls, ws, opts)
    _compare(grads, ref, "exact MIP 2 views", rel=2e-3)


def test_dilation_only_backward_is_unsupported(r):
    from paper_2503_18682_amd import _lib
    from paper_2503_18682_amd import renderer as R

    sc = scenegen.tiny_scene(39, 200, sh_degree=1)
    cam = scenegen.pinhole(scenegen.look_at((0, 0, -3)), 48, 40, 60)
    g = to_dev(sc, requires_grad=True)
    img = R.render(r, g, [cam], scenegen.default_options(mip=3))[0]
    with pytest.raises(_lib.RayGSError) as ei:
        img.sum().backward()
    assert ei.value.status == _lib.RGS_EUNSUPPORTED
