"""GPU parity of the HIP renderer (through the C ABI) against the CPU oracle.

Images: every pixel within 2e-4 max-abs in [0, 1] of the oracle; a pixel where
a decision (omega vs p_min, the termination test, the sign of tau) lies within
rounding distance within 2e-4 of one of its correct results, which the oracle
enumerates.  Depth keys, pixel boxes, box tile counts and tile lists:
bit-exact, excluding Gaussians the oracle flags as hazards (expected count
~0).  The slot bits of each listed instance: a superset of the tile's pixel
slots that hold a pixel of the Gaussian's support."""
import numpy as np
import pytest
import torch

import oracle
import scenegen
from gpu_helpers import (assert_image_close, assert_pixels_close, instance_lists, oracle_box_tiles,
                         oracle_lists_without_hazards, read,
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


def _check_lists(buf, lay, m, sp, cam, opts, label):
    tiles, ids = instance_lists(buf, lay)
    ot, ok_, oi, bad = oracle_lists_without_hazards(sp, cam, opts)
    keep = ~np.isin(ids, list(bad)) if bad else np.ones_like(ids, bool)
    say(f"  {label}: {m} box instances, {len(ids)} listed, {len(bad)} hazard Gaussians excluded")
    assert np.array_equal(tiles[keep], ot) and np.array_equal(ids[keep], oi)


def slot_layout(tw, th):
    """The compositing kernels' pixel slots of a tw x th tile (64 pixels a
    wave evaluates or skips together): 8 x 8 blocks for a tile wider than 8
    pixels with at most 4 of them, else full-width row bands of 64 / tw rows.
    Returns (slot width, slot height, slots across, slots, culling bits per
    instance)."""
    if tw >= 16 and (tw // 8) * (th // 8) <= 4:
        return 8, 8, tw // 8, (tw // 8) * (th // 8), True
    ly = 64 // tw
    return tw, ly, 1, th // ly, th // ly <= 4


def _check_bands(buf, lay, sp, cam, opts, label):
    """The slot culling bits of every listed instance (top 4 bits of its id,
    bit k for slot k) cover every slot that holds a pixel of the Gaussian's
    support, found pixel by pixel by the oracle."""
    tw, th = int(opts["tile_w"]), int(opts["tile_h"])
    cw, ch, bx, slots, bits = slot_layout(tw, th)
    if not bits:
        return
    tiles, ids, bands = instance_lists(buf, lay, with_bands=True)
    keep = sp["hazard"][ids] == 0
    tiles, ids, bands = tiles[keep], ids[keep], bands[keep]
    # oracle cells of the slot size are numbered row-major, as the slots are
    need = oracle.support_cells(sp, cam, opts, tiles, ids, cw, ch).astype(np.int64)
    assert (need >> slots).max(initial=0) == 0
    missing = (need & ~bands) != 0
    set_bits = sum(int(((bands >> k) & 1).sum()) for k in range(4))
    need_bits = sum(int(((need >> k) & 1).sum()) for k in range(4))
    say(f"  {label}: {len(ids)} instances, {need_bits} slots hold support, {set_bits} slot bits set")
    assert not missing.any(), f"{label}: {int(missing.sum())} instances miss a slot that holds support"


def _check_keys_boxes_counts(buf, lay, sp, n):
    """Depth keys and order (kept views, sorted), pixel boxes, binning boxes
    and their tile counts, bit-exact outside the oracle's hazard set."""
    kept, box_tiles = oracle_box_tiles(sp)
    n_kept = int(kept.sum())  # culled views sort last (key 0xffffffff)
    keys = read(buf, lay.depth_keys, n_kept, np.uint32)
    order = read(buf, lay.order, n_kept, np.uint32)
    want = np.nonzero(kept)[0]
    want = want[np.lexsort((want, sp["depth_key"][want]))]
    assert np.array_equal(order, want) and np.array_equal(keys, sp["depth_key"][want])
    boxes = read(buf, lay.boxes, 4 * n, np.uint16).reshape(n, 4)
    good = kept & (sp["hazard"] == 0)
    bins = read(buf, lay.bin_boxes, 4 * n, np.uint16).reshape(n, 4)
    for f, col in (("px0", 0), ("px1", 1), ("py0", 2), ("py1", 3)):
        assert np.array_equal(boxes[good, col], sp[f][good])
    for f, col in (("bx0", 0), ("bx1", 1), ("by0", 2), ("by1", 3)):
        assert np.array_equal(bins[good, col], sp[f][good])
    counts = read(buf, lay.tile_counts, n, np.uint32)
    assert np.array_equal(counts[good], box_tiles[good])
    tighter = int(((sp["bx1"] - sp["bx0"] < sp["px1"] - sp["px0"]) | (sp["by1"] - sp["by0"] < sp["py1"] - sp["py0"]))[good].sum())
    say(f"  keys, order, boxes, binning boxes ({tighter} tighter than the box) and tile counts of {n_kept} kept "
        f"Gaussians bit-exact "
        f"({int((kept & ~good).sum())} hazard Gaussians excluded from boxes)")


def test_c0_image_keys_and_lists(r):
    say("case c0: 1000 Gaussians, 128x128")
    w = scenegen.make_workload("c0")
    sc, cam, opts = w["scene"], w["cameras"][0], w["options"]
    outs, buf, ws, lay, (ok, m) = render_with_ws(r, sc, [cam], opts)
    assert ok
    ref = oracle.render(sc, cam, opts)
    assert_image_close(outs[0]["rgb"], outs[0]["final_T"], ref, label="c0")
    sp = oracle.preprocess(sc, cam, opts)
    assert (sp["hazard"] & oracle.HAZARD["cull"]).sum() == 0
    assert m == oracle_box_tiles(sp)[1].sum()
    _check_keys_boxes_counts(buf, lay, sp, sc["opacity_logits"].shape[0])
    _check_lists(buf, lay, m, sp, cam, opts, "c0 lists")
    _check_bands(buf, lay, sp, cam, opts, "c0 bands")


def test_lists_are_consistent_with_gpu_counts_boxes_and_keys(r):
    """The integer stages are exact functions of the GPU's own outputs: every
    Gaussian is listed in at most its counted number of box tiles, all inside
    its box's tile rectangle and each with slot bits; the kept views and the
    listed instances are counted right; re-sorting the GPU's instances on the
    host by (tile, depth key, id) reproduces its order; tile ranges bracket
    exactly the runs of each tile."""
    say("case consistency: 2000 Gaussians, 200x150, 8x16 tiles")
    sc = scenegen.tiny_scene(31, 2000, sh_degree=1, half_extent=1.5, log_scale_mean=-3.0, log_scale_std=0.8)
    cam = scenegen.pinhole(scenegen.look_at((0.4, 0.3, -4.0)), 200, 150, 55)
    opts = scenegen.default_options(tile_w=8, tile_h=16)
    outs, buf, ws, lay, (ok, m) = render_with_ws(r, sc, [cam], opts)
    assert ok
    n = 2000
    counts = read(buf, lay.tile_counts, n, np.uint32).astype(np.int64)
    n_kept = int((counts > 0).sum())  # culled views sort last (key 0xffffffff)
    keys = read(buf, lay.depth_keys, n_kept, np.uint32)
    order = read(buf, lay.order, n_kept, np.uint32).astype(np.int64)
    boxes = read(buf, lay.boxes, 4 * n, np.uint16).reshape(n, 4).astype(np.int64)
    bins = read(buf, lay.bin_boxes, 4 * n, np.uint16).reshape(n, 4).astype(np.int64)
    kept_ids = order
    # the binning box lies in the pixel box, and the tile count is its tiles
    assert np.all((bins[kept_ids, 0] >= boxes[kept_ids, 0]) & (bins[kept_ids, 1] <= boxes[kept_ids, 1]) &
                  (bins[kept_ids, 2] >= boxes[kept_ids, 2]) & (bins[kept_ids, 3] <= boxes[kept_ids, 3]))
    assert np.array_equal(counts[kept_ids], (bins[kept_ids, 1] // 8 - bins[kept_ids, 0] // 8 + 1) *
                          (bins[kept_ids, 3] // 16 - bins[kept_ids, 2] // 16 + 1))
    assert np.all(counts[order] > 0)
    assert np.all(np.diff(keys.astype(np.int64)) >= 0)
    key_of = np.zeros(n, np.uint32)
    key_of[order] = keys
    c = read(buf, lay.counters, 8, np.int64)
    assert c[4] == n_kept and m == counts.sum()
    tiles, ids, bands = instance_lists(buf, lay, with_bands=True)
    assert c[3] == len(ids) and np.all(np.bincount(ids, minlength=n) <= counts)
    assert np.all(tiles < lay.total_tiles)
    srt = np.lexsort((ids, key_of[ids], tiles))
    assert np.array_equal(srt, np.arange(len(ids)))
    say(f"  {m} binning-box instances, {len(ids)} listed")
    tx_n = -(-200 // 8)
    ty, tx = tiles // tx_n, tiles % tx_n
    b = bins[ids]
    assert np.all((tx >= b[:, 0] // 8) & (tx <= b[:, 1] // 8) & (ty >= b[:, 2] // 16) & (ty <= b[:, 3] // 16))
    # 2 slots per 8x16 tile; a listed tile whose support meets only the gap
    # between the slots' pixel rows has no slot bit (rare)
    assert (bands >> 2).max() == 0 and (bands == 0).mean() < 0.01
    rng = read(buf, lay.tile_ranges, 2 * lay.total_tiles, np.uint32).reshape(-1, 2)
    for t in np.unique(tiles):
        idx = np.nonzero(tiles == t)[0]
        assert rng[t, 0] == idx[0] and rng[t, 1] == idx[-1] + 1


@pytest.mark.parametrize("shape", [(8, 8), (8, 16), (8, 32), (16, 8), (16, 16), (16, 32), (32, 8), (32, 16), (32, 32)])
def test_ragged_image_all_tile_shapes(r, shape):
    say(f"case ragged 131x77 tile {shape}")
    sc = scenegen.tiny_scene(32, 400, sh_degree=2, half_extent=1.2, log_scale_mean=-2.8, log_scale_std=0.7)
    cam = scenegen.pinhole(scenegen.look_at((-0.3, 0.5, -3.5)), 131, 77, 70)
    opts = scenegen.default_options(tile_w=shape[0], tile_h=shape[1], background=(0.2, 0.1, 0.05))
    outs, buf, ws, lay, (ok, m) = render_with_ws(r, sc, [cam], opts)
    assert ok
    ref = oracle.render(sc, cam, opts)
    assert_image_close(outs[0]["rgb"], outs[0]["final_T"], ref, label=f"ragged {shape}")
    sp = oracle.preprocess(sc, cam, opts)
    assert m == oracle_box_tiles(sp)[1].sum()
    _check_lists(buf, lay, m, sp, cam, opts, f"ragged {shape} lists")
    _check_bands(buf, lay, sp, cam, opts, f"ragged {shape} bands")
    base = scenegen.default_options(tile_w=16, tile_h=16, background=(0.2, 0.1, 0.05))
    b_outs = render_with_ws(r, sc, [cam], base)[0]
    # per-pixel arithmetic does not depend on the tiling
    assert np.array_equal(outs[0]["rgb"], b_outs[0]["rgb"]) and np.array_equal(outs[0]["final_T"], b_outs[0]["final_T"])


@pytest.mark.parametrize("logit", [-3.0, 1.0])
def test_long_tile_lists_are_split_by_rows(r, logit):
    """A dense cluster whose tile lists reach ~1,500-2,000 entries: tiles this
    heavy are composited as two half-tile work items.  The image matches the
    oracle, and is bit-identical across tile shapes (8x8 is never split).
    logit -3: transmittance stays above T_eps (whole lists); logit 1: pixels
    terminate early inside split tiles."""
    say(f"case long lists, opacity logit {logit}")
    sc = scenegen.tiny_scene(36, 4000, sh_degree=1, half_extent=0.35, log_scale_mean=-3.2, log_scale_std=0.5)
    sc["opacity_logits"][:] = logit + 0.3 * np.random.default_rng(0).standard_normal(4000).astype(np.float32)
    cam = scenegen.pinhole(scenegen.look_at((0.0, 0.0, -4.0)), 96, 80, 30)
    ref = None
    images = []
    for shape in ((8, 16), (16, 16), (8, 8)):
        opts = scenegen.default_options(tile_w=shape[0], tile_h=shape[1])
        outs, buf, ws, lay, (ok, m) = render_with_ws(r, sc, [cam], opts)
        assert ok
        if ref is None:
            ref = oracle.render(sc, cam, opts)
            sp = oracle.preprocess(sc, cam, opts)
            tiles, _, _ = oracle.tile_lists(sp, cam, opts)
            assert np.bincount(tiles).max() >= 1000
        assert_image_close(outs[0]["rgb"], outs[0]["final_T"], ref, label=f"long lists {shape}")
        images.append(outs[0])
    for o in images[1:]:
        assert np.array_equal(o["rgb"], images[0]["rgb"]) and np.array_equal(o["final_T"], images[0]["final_T"])


def _mk(mus, scales, opac, rgbs, quats=None):
    n = len(mus)
    sh = np.zeros((1, 3, n))
    sh[0] = (np.asarray(rgbs, float).T - 0.5) * 2 * np.sqrt(np.pi)
    q = np.tile(np.array([[1.0], [0], [0], [0]]), (1, n)) if quats is None else np.asarray(quats, float).T
    return dict(means=np.asarray(mus, np.float32).T.copy(), log_scales=np.log(np.asarray(scales, float)).T.astype(np.float32).copy(),
                quats=q.astype(np.float32).copy(), opacity_logits=np.log(np.asarray(opac) / (1 - np.asarray(opac))).astype(np.float32),
                sh=sh.astype(np.float32), sh_degree=0)


@pytest.mark.parametrize("mode", [dict(), dict(mip=1), dict(mip=2, mip_sigma2_px=1.0), dict(mip=3), dict(divergence=1)],
                         ids=["ray", "mip", "exact_mip", "dilation", "gs"])
def test_edge_cases(r, mode):
    cam = scenegen.pinhole(np.concatenate([np.eye(3), np.zeros((3, 1))], 1), 48, 40, 90)
    opts = scenegen.default_options(background=(0.1, 0.2, 0.3), **mode)
    cases = {
        "empty": _mk(np.zeros((0, 3)), np.zeros((0, 3)) + 1, np.zeros(0) + 0.5, np.zeros((0, 3))),
        "single": _mk([[0.1, 0.05, 2.0]], [[0.1, 0.2, 0.05]], [0.8], [[0.9, 0.3, 0.1]]),
        "all_culled": _mk([[0, 0, -1.0], [0, 0, 0.1], [0, 0, 3.0]], [[0.1] * 3] * 3, [0.5, 0.5, 0.002], [[1, 1, 1]] * 3),
        "camera_inside": _mk([[0.05, 0.0, 0.4], [0.0, 0.0, 3.0]], [[0.5] * 3, [0.2] * 3], [0.9, 0.7], [[1, 0, 0], [0, 1, 0]]),
        "quad_crossing_camera_plane": _mk([[0.3, 0.1, 0.6], [0, 0, 2.0]], [[0.05, 0.5, 0.05], [0.2] * 3], [0.8, 0.6],
                                          [[1, 0, 0], [0, 1, 0]], quats=[[0.9, 0.3, 0.2, 0.1], [1, 0, 0, 0]]),
        "offscreen": _mk([[30.0, 0.0, 2.0]], [[0.1] * 3], [0.9], [[1, 1, 1]]),
        # centres outside the image whose supports reach into it (their
        # colour is evaluated after the geometry, the others' before it)
        "centre_outside_support_inside": _mk([[2.5, 0.0, 2.0], [-0.2, -2.3, 2.0], [0.1, 0.0, 2.2]],
                                             [[0.5, 0.4, 0.3], [0.3, 0.6, 0.4], [0.2] * 3], [0.8, 0.7, 0.6],
                                             [[0.9, 0.2, 0.1], [0.1, 0.8, 0.3], [0.2, 0.3, 0.9]]),
    }
    bad = _mk([[0.0, 0.0, 2.0], [0.1, 0.0, 2.5], [0.0, 0.1, 3.0], [-0.1, -0.05, 2.2]], [[0.2] * 3] * 4, [0.7] * 4,
              [[1, 0, 0]] * 4)
    bad["means"][0, 0] = np.nan
    bad["quats"][:, 1] = 0.0  # the fourth Gaussian stays valid
    bad["sh"][0, 1, 2] = np.inf
    cases["non_finite_and_zero_quat"] = bad
    for name, sc in cases.items():
        say(f"case edge/{name} {mode}")
        outs, buf, ws, lay, (ok, m) = render_with_ws(r, sc, [cam], opts)
        assert ok
        ref = oracle.render(sc, cam, opts)
        kept, box_tiles = oracle_box_tiles(oracle.preprocess(sc, cam, opts))
        assert m == box_tiles.sum(), name
        assert_image_close(outs[0]["rgb"], outs[0]["final_T"], ref, label=name)
        if name == "non_finite_and_zero_quat":
            # a non-finite colour coefficient culls like any other cull: no
            # depth position, tile count 0, not counted as kept
            n = sc["opacity_logits"].shape[0]
            assert list(np.nonzero(kept)[0]) == [3]
            assert read(buf, lay.counters, 8, np.int64)[4] == 1
            assert np.array_equal(read(buf, lay.tile_counts, n, np.uint32), box_tiles)
            assert read(buf, lay.order, 1, np.uint32)[0] == 3
    assert np.allclose(render_with_ws(r, cases["empty"], [cam], opts)[0][0]["rgb"][2], 0.3)


@pytest.mark.parametrize("t_eps", [0.0, 0.5, 0.99999999])
def test_termination_threshold_extremes(r, t_eps):
    """Early termination (eq. 1) at the ends of its range: never (t_eps 0),
    after about half the light is absorbed, and at the first composited
    Gaussian (0.99999999, which is 1 in FP32: no pixel takes a colour), in
    every compositing mode, against the oracle.  A pixel's transmittance
    never falls below t_eps before it stops, so a Gaussian that misses the
    pixel cannot stop it."""
    sc = scenegen.tiny_scene(36, 2000, sh_degree=1, half_extent=1.2, log_scale_mean=-2.6, log_scale_std=0.5,
                             logit_std=2.0)
    cam = scenegen.pinhole(scenegen.look_at((0.3, 0.2, -3.5)), 96, 80, 60)
    for mode in (dict(), dict(mip=1), dict(mip=2, mip_sigma2_px=1.0)):
        opts = scenegen.default_options(t_eps=t_eps, background=(0.2, 0.1, 0.3), **mode)
        say(f"case t_eps {t_eps} {mode}")
        outs, buf, ws, lay, (ok, m) = render_with_ws(r, sc, [cam], opts)
        assert ok
        assert_image_close(outs[0]["rgb"], outs[0]["final_T"], oracle.render(sc, cam, opts),
                           label=f"t_eps {t_eps} {mode}")
        if t_eps > 0.9:
            assert np.all(outs[0]["final_T"] == 1.0)


def _crossing_scene(seed, n):
    """Large Gaussians close to a camera at the origin: many quads cross the
    camera plane z = 0."""
    sc = scenegen.tiny_scene(seed, n, sh_degree=1, half_extent=1.0, log_scale_mean=-1.8, log_scale_std=0.6)
    sc["means"][2, :] = np.random.default_rng(seed).uniform(0.25, 2.5, n).astype(np.float32)
    return sc


@pytest.mark.parametrize("mode", [dict(), dict(mip=1), dict(mip=2, mip_sigma2_px=1.0)], ids=["ray", "mip", "exact_mip"])
def test_crossing_quads_are_clipped_to_the_frustum(r, mode):
    """Quads with a vertex at z <= 0: the box is that of the part of the quad
    inside the view frustum, bit-exact against the oracle (outside its hazard
    set), quads wholly outside the view are culled, every crossing quad is
    counted, and the tile lists and image match the oracle."""
    cam = scenegen.pinhole(np.concatenate([np.eye(3), np.zeros((3, 1))], 1), 97, 61, 90)
    opts = scenegen.default_options(**mode)
    sc = _crossing_scene(61, 300)
    say(f"case crossing quads {mode}: 300 Gaussians near the camera, 97x61")
    outs, buf, ws, lay, (ok, m) = render_with_ws(r, sc, [cam], opts)
    assert ok
    sp = oracle.preprocess(sc, cam, opts)
    C = oracle.CULL
    crossing = (sp["all_front"] == 0) & (sp["whole"] == 0) & np.isin(sp["cull"], [0, C["offscreen"], C["notile"],
                                                                                   C["nobin"]])
    clipped_away = crossing & (sp["cull"] == C["offscreen"])
    say(f"  {int(crossing.sum())} crossing quads, {int(clipped_away.sum())} wholly outside the view")
    assert crossing.sum() > 20 and clipped_away.sum() > 0
    assert int(read(buf, lay.counters, 8, np.int64)[5]) == crossing.sum()
    n = 300
    good = sp["hazard"] == 0
    # a box with no listed tile (notile) still has its tiles counted
    counts = read(buf, lay.tile_counts, n, np.uint32)
    assert np.array_equal(counts[good] == 0, ~np.isin(sp["cull"][good], [0, C["notile"]]))
    kept = (sp["cull"] == 0) & good
    boxes = read(buf, lay.boxes, 2 * n, np.uint32).reshape(n, 2)
    bins = read(buf, lay.bin_boxes, 2 * n, np.uint32).reshape(n, 2)
    for f, col, sh in (("px0", 0, 0), ("px1", 0, 16), ("py0", 1, 0), ("py1", 1, 16)):
        assert np.array_equal((boxes[kept, col] >> sh) & 0xFFFF, sp[f][kept]), f
    for f, col, sh in (("bx0", 0, 0), ("bx1", 0, 16), ("by0", 1, 0), ("by1", 1, 16)):
        assert np.array_equal((bins[kept, col] >> sh) & 0xFFFF, sp[f][kept]), f
    assert m == oracle_box_tiles(sp)[1].sum()
    tiles, ids = instance_lists(buf, lay)
    ot, _, oi, bad = oracle_lists_without_hazards(sp, cam, opts)
    keep = ~np.isin(ids, list(bad)) if bad else np.ones_like(ids, bool)
    assert np.array_equal(tiles[keep], ot) and np.array_equal(ids[keep], oi)
    assert_image_close(outs[0]["rgb"], outs[0]["final_T"], oracle.render(sc, cam, opts), label=f"crossing {mode}")


def test_crossing_quads_graph_replays_and_gradients(r):
    """The crossing list in a captured graph: its counter restarts with every
    replay, so replays of moving cameras equal eager renders bit for bit and
    the oracle; and the backward over the crossing scene (clipped boxes,
    clip-culled views with no gradient) matches the oracle's gradient."""
    from paper_2503_18682_amd import _lib
    from paper_2503_18682_amd import renderer as R
    from test_gpu_grad import _compare

    sc = _crossing_scene(61, 300)
    base = np.concatenate([np.eye(3), np.zeros((3, 1))], 1)
    cams = [scenegen.pinhole(base, 97, 61, 90), scenegen.pinhole(base, 64, 80, 80)]
    opts = scenegen.default_options()
    g = to_dev(sc)
    say("case crossing quads graph plan: 2 views, 3 replays")
    br = R.BatchRenderer(r, 300, 1, cams, capacity=200000, options=opts)
    for rep in range(3):
        moved = []
        for c in cams:
            c2 = dict(c)
            c2["w2c"] = c["w2c"].copy()
            c2["w2c"][0, 3] += 0.03 * rep
            moved.append(c2)
        outs = br.launch(g, moved)
        assert br.status()[0]
        eager = render_with_ws(r, sc, moved, opts)[0]
        for v in range(2):
            assert np.array_equal(outs[v]["rgb"].cpu().numpy(), eager[v]["rgb"]), (rep, v)
            assert np.array_equal(outs[v]["final_T"].cpu().numpy(), eager[v]["final_T"]), (rep, v)
        if rep == 2:
            for v in range(2):
                assert_image_close(eager[v]["rgb"], eager[v]["final_T"], oracle.render(sc, moved[v], opts),
                                   label=f"crossing graph view {v}")
    br.close()

    say("case crossing quads gradients: 300 Gaussians, 97x61, dense upstream gradient")
    cam = cams[0]
    outs, (buf, ws) = r.render(g, [cam], opts, flags=_lib.RGS_WS_BACKWARD, keep_workspace=True)
    ref_img = oracle.render(sc, cam, opts)
    dl = np.random.default_rng(64).normal(0, 1, (3, 61, 97))
    dl[:, ref_img["hazard"] != 0] = 0.0  # no gradient through pixels at a decision boundary
    dl = dl.astype(np.float32)
    grads = r.backward(g, [cam], outs, [torch.from_numpy(dl).cuda()], ws, opts)
    _compare(grads, oracle.backward(sc, cam, opts, dl.astype(np.float64)), "crossing", rel=2e-3)


def test_crossing_list_beyond_its_cap_keeps_the_whole_view(r):
    """More crossing quads than the list holds (65536 per launch): every one
    is counted, those beyond the cap keep the whole view (more instances than
    the oracle's clipped boxes need), and the image still matches the oracle
    at every pixel."""
    n = 170000
    sc = scenegen.tiny_scene(62, n, sh_degree=0, half_extent=1.0, log_scale_mean=-1.2, log_scale_std=0.4)
    sc["means"][2, :] = np.random.default_rng(62).uniform(0.25, 1.5, n).astype(np.float32)
    cam = scenegen.pinhole(np.concatenate([np.eye(3), np.zeros((3, 1))], 1), 64, 48, 90)
    opts = scenegen.default_options()
    say("case crossing list overflow: 170000 Gaussians near the camera, 64x48")
    outs, buf, ws, lay, (ok, m) = render_with_ws(r, sc, [cam], opts)
    assert ok
    sp = oracle.preprocess(sc, cam, opts)
    C = oracle.CULL
    crossing = (sp["all_front"] == 0) & np.isin(sp["cull"], [0, C["offscreen"], C["notile"]])
    got = int(read(buf, lay.counters, 8, np.int64)[5])
    say(f"  {got} crossing quads counted, oracle {int(crossing.sum())}")
    assert got == crossing.sum() and got > 65536
    assert m > oracle_box_tiles(sp)[1].sum()
    assert_image_close(outs[0]["rgb"], outs[0]["final_T"], oracle.render(sc, cam, opts), label="crossing overflow")


def test_overflow_is_reported_and_recovers(r):
    say("case overflow: capacity 16")
    w = scenegen.make_workload("c0")
    sc, cam, opts = w["scene"], w["cameras"][0], w["options"]
    outs, buf, ws, lay, (ok, m) = render_with_ws(r, sc, [cam], opts, capacity=16)
    assert not ok and m > 16
    assert np.all(outs[0]["rgb"] == 0.0) and np.all(outs[0]["final_T"] == 1.0)
    outs2, _, _, _, (ok2, m2) = render_with_ws(r, sc, [cam], opts, capacity=m)
    assert ok2 and m2 == m
    assert_image_close(outs2[0]["rgb"], outs2[0]["final_T"], oracle.render(sc, cam, opts), label="after regrow")


def test_batch_plan_overflow_is_reported_by_batch_status(r):
    """A plan whose capacity is too small: rgs_batch_status reports
    RGS_EOVERFLOW with the instance count the frame needed, and the views are
    background; a plan with that capacity then renders the oracle's image."""
    from paper_2503_18682_amd import renderer as R

    say("case batch plan overflow: capacity 16")
    w = scenegen.make_workload("c0")
    sc, cam, opts = w["scene"], w["cameras"][0], w["options"]
    g = to_dev(sc)
    n = int(sc["opacity_logits"].shape[0])
    br = R.BatchRenderer(r, n, sc["sh_degree"], [cam], 16, options=opts)
    outs = br.launch(g, [cam])
    ok, need = br.status()
    assert not ok and need > 16
    assert torch.all(outs[0]["rgb"] == 0.0) and torch.all(outs[0]["final_T"] == 1.0)
    br.close()
    br = R.BatchRenderer(r, n, sc["sh_degree"], [cam], need, options=opts)
    outs = br.launch(g, [cam])
    ok2, need2 = br.status()
    assert ok2 and need2 == need
    host = {k: t.cpu().numpy() for k, t in outs[0].items()}
    br.close()
    assert_image_close(host["rgb"], host["final_T"], oracle.render(sc, cam, opts), label="batch after regrow")


@pytest.mark.parametrize("pose,tile,graph", [(0, (8, 16), True), (8, (16, 16), False)],
                         ids=["pose0-8x16-graph", "pose8-16x16-eager"])
def test_c1_full_frame(r, pose, tile, graph):
    """500k Gaussians at 1920x1080 (the benchmark frame), two of its 16 orbit
    poses: every pixel against the oracle, depth keys, order, pixel boxes and
    box tile counts of every Gaussian, the full tile list bit-exact and the
    slot bits of every listed instance.  Pose 0 runs in the benchmark's launch
    configuration (8x16 tiles, one HIP-graph replay of a batch plan); pose 8
    as an eager render at 16x16 tiles."""
    from paper_2503_18682_amd import renderer as R

    say(f"case c1 full frame: 500k Gaussians, 1920x1080, pose {pose}, tile {tile}, {'graph' if graph else 'eager'}")
    w = scenegen.make_workload("c1")
    sc, cam = w["scene"], w["cameras"][pose]
    opts = dict(w["options"], tile_w=tile[0], tile_h=tile[1])
    n = int(sc["opacity_logits"].shape[0])
    outs, buf, ws, lay, (ok, m) = render_with_ws(r, sc, [cam], opts)
    assert ok
    if graph:
        br = R.BatchRenderer(r, n, sc["sh_degree"], [cam], int(ws.capacity), options=opts)
        g = to_dev(sc)
        for _ in range(2):  # the capture, then a replay
            gouts = br.launch(g, [cam])
        assert br.status()[0]
        for k in ("rgb", "final_T", "n_contrib"):
            assert np.array_equal(gouts[0][k].cpu().numpy(), outs[0][k]), k
        buf = br.buf
        br.close()
    sp = oracle.preprocess(sc, cam, opts)
    assert (sp["hazard"] & oracle.HAZARD["cull"]).sum() == 0
    assert m == oracle_box_tiles(sp)[1].sum()
    _check_keys_boxes_counts(buf, lay, sp, n)
    _check_lists(buf, lay, m, sp, cam, opts, "c1 lists")
    _check_bands(buf, lay, sp, cam, opts, "c1 bands")
    assert_image_close(outs[0]["rgb"], outs[0]["final_T"], oracle.render(sc, cam, opts), label=f"c1 pose {pose}")


def test_maximum_view_size(r):
    """The largest view the ABI takes (16384 x 16384) at the finest tiles
    (8 x 8: 4.2M tiles, 23-bit tile ids): keys, boxes, box tile counts, the
    full tile list and slot bits bit-exact, and 6000 sampled pixels against
    the oracle; then a 16384 x 40 view (widest, ragged last tile row) on
    every pixel."""
    sc = scenegen.tiny_scene(57, 3000, sh_degree=1, half_extent=1.5, log_scale_mean=-4.5, log_scale_std=0.6)
    cam = scenegen.pinhole(scenegen.look_at((0.3, -0.2, -3.0)), 16384, 16384, 90)
    opts = scenegen.default_options(tile_w=8, tile_h=8)
    say("case maximum view size: 3000 Gaussians, 16384x16384, 8x8 tiles")
    outs, buf, ws, lay, (ok, m) = render_with_ws(r, sc, [cam], opts, to_host=False)
    assert ok
    assert int(lay.total_tiles) == 2048 * 2048
    sp = oracle.preprocess(sc, cam, opts)
    assert m == oracle_box_tiles(sp)[1].sum()
    _check_keys_boxes_counts(buf, lay, sp, sc["opacity_logits"].shape[0])
    _check_lists(buf, lay, m, sp, cam, opts, "16384x16384 lists")
    _check_bands(buf, lay, sp, cam, opts, "16384x16384 slot bits")
    rng = np.random.default_rng(12)
    px = torch.from_numpy(rng.integers(0, 16384, 6000))
    py = torch.from_numpy(rng.integers(0, 16384, 6000))
    o = outs[0]
    g_rgb = o["rgb"][:, py.cuda(), px.cuda()].T.cpu().numpy()
    g_T = o["final_T"][py.cuda(), px.cuda()].cpu().numpy()
    del outs, o, buf, ws
    ref = oracle.render_pixels(sc, cam, opts, px.numpy(), py.numpy())
    assert_pixels_close(g_rgb, g_T, ref, label="16384x16384 sampled")
    cam = scenegen.pinhole(scenegen.look_at((0.3, -0.2, -3.0)), 16384, 40, 90)
    say("case maximum view width: 3000 Gaussians, 16384x40, 8x8 tiles")
    outs, buf, ws, lay, (ok, m) = render_with_ws(r, sc, [cam], opts)
    assert ok
    _check_lists(buf, lay, m, oracle.preprocess(sc, cam, opts), cam, opts, "16384x40 lists")
    assert_image_close(outs[0]["rgb"], outs[0]["final_T"], oracle.render(sc, cam, opts), label="16384x40")


def _sampled_pixels(outs_v, sc, cam, opts, n_px, rng, label):
    """GPU pixels against the oracle's per-pixel evaluation at n_px random pixels."""
    px = rng.integers(0, cam["width"], n_px)
    py = rng.integers(0, cam["height"], n_px)
    ref = oracle.render_pixels(sc, cam, opts, px, py)
    assert_pixels_close(outs_v["rgb"][:, py, px].T, outs_v["final_T"][py, px], ref, label=label)


def test_c2_full_size_stereo_batch(r):
    """3M Gaussians, 4 stereo pairs (8 views from 1032x1104 to 4128x4416 per
    eye), MIP on, all 8 views in one HIP-graph replay with the benchmark's
    8x16 tiles: every pixel of a 1032x1104 eye, sampled pixels of a 4128x4416
    eye."""
    from paper_2503_18682_amd import renderer as R

    w = scenegen.make_workload("c2")
    sc, cams = w["scene"], w["cameras"]
    opts = dict(w["options"], tile_w=8, tile_h=16)
    n = int(sc["opacity_logits"].shape[0])
    say("case c2 full size: 3M Gaussians, 8 stereo views, MIP, one graph replay")
    g = to_dev(sc)
    _, (buf, ws) = r.render(g, cams, opts, keep_workspace=True)
    need = r.status(ws)[1]
    del buf, ws
    br = R.BatchRenderer(r, n, sc["sh_degree"], cams, int(need * 1.1) + 4096, options=opts)
    outs = br.launch(g, cams)
    ok, _ = br.status()
    assert ok
    host = {v: {k: t.cpu().numpy() for k, t in outs[v].items()} for v in (2, 5)}
    br.close()
    assert (cams[5]["width"], cams[5]["height"]) == (1032, 1104)
    assert_image_close(host[5]["rgb"], host[5]["final_T"], oracle.render(sc, cams[5], opts),
                       label="c2 view 5 1032x1104, every pixel")
    assert (cams[2]["width"], cams[2]["height"]) == (4128, 4416)
    _sampled_pixels(host[2], sc, cams[2], opts, 3000, np.random.default_rng(8), "c2 view 2 4128x4416 sampled")


def test_batched_views_match_single_views_and_oracle(r):
    """Views of different sizes in one batch (MIP on) equal the same views
    rendered one at a time, bit for bit, and match the oracle."""
    sc = scenegen.tiny_scene(33, 3000, sh_degree=3, half_extent=1.5, log_scale_mean=-3.5, log_scale_std=0.8)
    cams = [scenegen.pinhole(scenegen.look_at((0, 0, -4)), 160, 120, 60),
            scenegen.pinhole(scenegen.look_at((2, 1, -3.5)), 97, 211, 75),
            scenegen.pinhole(scenegen.look_at((-3, 0.5, -2)), 64, 64, 40)]
    opts = scenegen.default_options(mip=1)
    say("case batch of 3 uneven views, MIP on")
    outs, buf, ws, lay, (ok, m) = render_with_ws(r, sc, cams, opts)
    assert ok
    for v, cam in enumerate(cams):
        single = render_with_ws(r, sc, [cam], opts)[0][0]
        assert np.array_equal(outs[v]["rgb"], single["rgb"]), v
        assert np.array_equal(outs[v]["final_T"], single["final_T"]), v
        assert_image_close(outs[v]["rgb"], outs[v]["final_T"], oracle.render(sc, cam, opts), label=f"batch view {v}")


@pytest.mark.parametrize("n_views", [12, 14])
def test_many_view_batches_match_single_views(r, n_views):
    """A batch whose workspace header (counters and a 224-byte entry per
    view) goes to the device as kernel arguments (12 views) or by a copy (14
    views) renders every view as a single-view render does, bit for bit."""
    sc = scenegen.tiny_scene(34, 1500, sh_degree=1, half_extent=1.5, log_scale_mean=-3.0, log_scale_std=0.5)
    rng = np.random.default_rng(35)
    cams = [scenegen.pinhole(scenegen.look_at((rng.uniform(-2, 2), rng.uniform(-1, 1), -4.0)),
                             int(rng.integers(24, 72)), int(rng.integers(24, 72)), 55) for _ in range(n_views)]
    opts = scenegen.default_options()
    say(f"case batch of {n_views} small views")
    outs, buf, ws, lay, (ok, m) = render_with_ws(r, sc, cams, opts)
    assert ok
    header = lay.views + 224 * n_views
    assert (header <= 3072) == (n_views == 12), header
    for v, cam in enumerate(cams):
        single = render_with_ws(r, sc, [cam], opts)[0][0]
        assert np.array_equal(outs[v]["rgb"], single["rgb"]), v
        assert np.array_equal(outs[v]["n_contrib"], single["n_contrib"]), v


def test_graph_plan_replays_match_eager(r):
    from paper_2503_18682_amd import renderer as R

    sc = scenegen.tiny_scene(34, 3000, sh_degree=2, half_extent=1.5, log_scale_mean=-3.5, log_scale_std=0.8)
    cams = [scenegen.pinhole(scenegen.look_at((0, 0, -4)), 160, 120, 60),
            scenegen.pinhole(scenegen.look_at((0.063, 0, -4)), 160, 120, 60),
            scenegen.pinhole(scenegen.look_at((1, 1, -3)), 80, 90, 70)]
    opts = scenegen.default_options(mip=1)
    g = to_dev(sc)
    say("case graph plan: 3 views, 4 replays with moving cameras")
    br = R.BatchRenderer(r, 3000, 2, cams, capacity=200000, options=opts)
    for rep in range(4):
        moved = []
        for c in cams:
            c2 = dict(c)
            c2["w2c"] = c["w2c"].copy()
            c2["w2c"][0, 3] += 0.05 * rep
            moved.append(c2)
        outs = br.launch(g, moved)
        ok, _ = br.status()
        assert ok
        eager = render_with_ws(r, sc, moved, opts)[0]
        for v in range(3):
            assert np.array_equal(outs[v]["rgb"].cpu().numpy(), eager[v]["rgb"]), (rep, v)
            assert np.array_equal(outs[v]["final_T"].cpu().numpy(), eager[v]["final_T"]), (rep, v)
    br.close()


def test_autotune_picks_a_supported_shape(r):
    sc = scenegen.tiny_scene(35, 2000, sh_degree=1)
    cams = [scenegen.pinhole(scenegen.look_at((0, 0, -4)), 200, 160, 60)]
    g = to_dev(sc)
    say("case autotune")
    buf, ws = r.new_workspace(2000, cams, 500000, 0, r.options)
    outs = r.allocate_outputs(cams)
    best, ms = r.autotune(g, cams, ws, outs, reps=2)
    assert best["tile_w"] in (8, 16, 32) and best["tile_h"] in (8, 16, 32)
    assert ms > 0


@pytest.mark.parametrize("mode", [dict(), dict(mip=1), dict(mip=2, mip_sigma2_px=0.5), dict(divergence=1)],
                         ids=["ray", "mip", "exact_mip", "gs"])
def test_training_autotune_picks_a_supported_shape_and_keeps_gradients_valid(r, mode):
    """The render + backward autotuner returns a supported shape, and a
    backward pass at that shape still matches the default shape's, for every
    differentiable divergence and MIP mode."""
    from paper_2503_18682_amd import _lib

    sc = scenegen.tiny_scene(37, 2000, sh_degree=1)
    cams = [scenegen.pinhole(scenegen.look_at((0, 0, -4)), 120, 100, 60)]
    g = to_dev(sc)
    say(f"case training autotune {mode}")
    opts = scenegen.default_options(**mode)
    buf, ws = r.new_workspace(2000, cams, 500000, _lib.RGS_WS_BACKWARD, opts)
    outs = r.allocate_outputs(cams)
    rng = np.random.default_rng(5)
    dl = [torch.from_numpy(rng.normal(0, 1, (3, 100, 120)).astype(np.float32)).cuda()]
    r.render_into(g, cams, outs, ws, opts)
    best, ms = r.autotune_training(g, cams, ws, outs, dl, reps=2, options=opts)
    assert best["tile_w"] in (8, 16, 32) and best["tile_h"] in (8, 16, 32) and ms > 0
    # tile (0, 0) now resolves to the tuned shape on this context
    lay = r.layout(2000, cams, 500000, _lib.RGS_WS_BACKWARD, dict(opts, tile_w=0, tile_h=0))
    assert (lay.tile_w, lay.tile_h) == (best["tile_w"], best["tile_h"])
    grads = {}
    for label, o in (("default", opts), ("tuned", best)):
        r.render_into(g, cams, outs, ws, o)
        grads[label] = r.backward(g, cams, outs, dl, ws, o)
    for k in grads["default"]:
        a, b = grads["default"][k].cpu().numpy(), grads["tuned"][k].cpu().numpy()
        assert np.abs(a - b).max() <= 1e-4 * max(np.abs(a).max(), 1e-6), k


def test_view_clocks_leave_images_unchanged_and_order_in_time(r):
    """Per-view completion clocks: enabling them changes no output bit; every
    view's clock lies after the frame start and within the frame's host-side
    duration; a batch with more views than the clock buffer is rejected."""
    import time

    sc = scenegen.tiny_scene(36, 3000, sh_degree=1, half_extent=1.5, log_scale_mean=-3.5, log_scale_std=0.8)
    cams = [scenegen.pinhole(scenegen.look_at((0, 0, -4)), 160, 120, 60),
            scenegen.pinhole(scenegen.look_at((1, 0.5, -3.5)), 96, 200, 70)]
    opts = scenegen.default_options()
    say("case view clocks: 2 uneven views")
    g = to_dev(sc)
    buf, ws = r.new_workspace(3000, cams, 200000, 0, opts)
    plain = r.allocate_outputs(cams)
    r.render_into(g, cams, plain, ws, opts)
    stamps = torch.zeros(len(cams) + 1, dtype=torch.int64, device="cuda")
    r.set_view_clocks(stamps)
    try:
        clocked = r.allocate_outputs(cams)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r.render_into(g, cams, clocked, ws, opts)
        torch.cuda.synchronize()
        host_ms = (time.perf_counter() - t0) * 1e3
        lat = r.view_latencies_ms(stamps, len(cams))
        s = stamps.cpu().numpy()
        say(f"  latencies {[round(x, 4) for x in lat]} ms, host {host_ms:.3f} ms")
        assert s[0] > 0 and all(s[1:] >= s[0])
        assert all(0.0 < x <= host_ms + 1.0 for x in lat)
        for v in range(len(cams)):
            for key in ("rgb", "final_T", "n_contrib"):
                assert torch.equal(plain[v][key], clocked[v][key]), (v, key)
        small = torch.zeros(2, dtype=torch.int64, device="cuda")
        r.set_view_clocks(small)  # room for one view only
        with pytest.raises(RuntimeError):
            r.render_into(g, cams, clocked, ws, opts)
    finally:
        r.set_view_clocks(None)
