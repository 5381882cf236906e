"""GPU parity of the rasterizer forward pass against the float64 oracle:
projection records, tile lists (bit-exact), images (1e-4 max-abs outside the
oracle's ambiguity margins), plus the invariances the batch-parallel design
promises (tile size, chunk depth, batch composition, run-to-run)."""
import numpy as np
import pytest

from oracle import blendshape as bs
from oracle import raster
from paper_2503_12886_amd import gbr, synth
from gpu_util import IMAGE_TOL, MASK_FRAC_MAX, compare_image, dev, host, make_ctx, render

pytestmark = pytest.mark.gpu


def tiny_case():
    """The tiny workload: N=2000, K=8, one 128x128 frame at z=0.5, fx=fy=150, weights U[0,1]."""
    bases = synth.make_scene(2000, 8, seed=0)
    w = synth.make_weights(1, 8, seed=2)
    cam = synth.fixed_camera(128, 128, 150.0, 0.5, bg=(0.2, 0.3, 0.4))
    raw = bs.blend(bases, w).astype(np.float32)[0]
    return raw, cam


def batch_case(B=5, N=3000, seed=0, res=((64, 48), (96, 96), (80, 72))):
    bases = synth.make_scene(N, 6, seed=seed)
    w = synth.make_weights(B, 6, seed=seed + 1)
    cams = synth.make_cameras(B, seed=seed + 2, resolutions=list(res), dist=(0.4, 0.7))
    raw = bs.blend(bases, w).astype(np.float32).reshape(B * N, 16)
    return raw, cams, N


def test_tiny_image_parity():
    raw, cam = tiny_case()
    ctx = make_ctx()
    imgs, _, _ = render(ctx, raw, [cam])
    ref, Te, nc, fl = raster.render(raw, cam)
    err, masked = compare_image(imgs[0], ref, fl, tag="tiny image")
    assert err <= IMAGE_TOL, err
    assert masked <= MASK_FRAC_MAX, masked
    tfin = gbr.gbr_inspect(ctx, "t_final", 128 * 128).reshape(128, 128)
    assert np.abs(tfin - Te)[fl == 0].max() <= 1e-4


def test_projection_records_and_rects():
    raw, cams, N = batch_case()
    ctx = make_ctx(tile=16)
    render(ctx, raw, cams)
    rec = gbr.gbr_inspect(ctx, "records", raw.shape[0])
    rect = gbr.gbr_inspect(ctx, "rects", raw.shape[0])
    log2e = 1.0 / np.log(2.0)
    for b, cam in enumerate(cams):
        p = raster.project(raw[b * N:(b + 1) * N], cam)
        r = rec[b * N:(b + 1) * N]
        rc = rect[b * N:(b + 1) * N]
        v = p["valid"] > 0
        # integer decisions: identical
        exp_rect = raster.tile_rects(p, cam.width, cam.height, 16)
        assert np.array_equal(rc[v], exp_rect[v].astype(np.int32))
        assert np.all(rc[~v][:, 2] < rc[~v][:, 0])           # culled: empty rect
        # depth key: the binary32 rounding of the camera-space depth
        assert np.array_equal(r[v, 9], p["key"][v].astype(np.float32))
        # float32 records of float64 quantities
        for col, ref in ((0, p["mx"]), (1, p["my"]), (2, -0.5 * log2e * p["A"]), (3, -log2e * p["B"]),
                         (4, -0.5 * log2e * p["C"]), (5, np.log2(p["opacity"]))):
            assert np.allclose(r[v, col], ref[v], rtol=2e-7, atol=1e-30), col


def test_tile_lists_bit_exact():
    """Each context first renders another scene, so bitmap segments that
    have set bits there and none here hold stale words: the lists must not
    see them."""
    raw, cams, N = batch_case(B=4, N=2500, seed=3)
    other, _, _ = batch_case(B=4, N=2500, seed=11)
    for tile in (8, 16, 32):
        ctx = make_ctx(tile=tile)
        render(ctx, other, cams)
        render(ctx, raw, cams)
        projs = [raster.project(raw[b * N:(b + 1) * N], c) for b, c in enumerate(cams)]
        ranges, sf, sg, tile_base = raster.bin_and_sort(projs, cams, tile)
        n_tiles = len(ranges)
        ts = gbr.gbr_inspect(ctx, "tile_start", n_tiles + 1)
        assert np.array_equal(ts[:-1].astype(np.int64), ranges[:, 0])
        assert np.array_equal(ts[1:].astype(np.int64), ranges[:, 1])
        srt = gbr.gbr_inspect(ctx, "sorted", len(sg)).astype(np.int64)
        assert np.array_equal(srt, sf * N + sg)
        ctx.close()


def test_batch_images_with_uneven_sizes_and_gaussian_sets():
    # frames with their own Gaussian sets and resolutions, one pass
    rng = np.random.default_rng(0)
    sizes = [1200, 37, 2500, 0, 900]
    cams = synth.make_cameras(5, seed=4, resolutions=[(64, 48), (50, 70), (96, 96), (33, 17)], dist=(0.45, 0.6))
    raws, offs = [], [0]
    for i, n in enumerate(sizes):
        bases = synth.make_scene(max(n, 1), 4, seed=10 + i)[:, :n]
        raws.append(bs.blend(bases, synth.make_weights(1, 4, seed=i)).astype(np.float32)[0])
        offs.append(offs[-1] + n)
    raw = np.concatenate(raws, axis=0)
    ctx = make_ctx()
    imgs, _, _ = render(ctx, raw, cams, offs)
    for b, cam in enumerate(cams):
        ref, _, _, fl = raster.render(raw[offs[b]:offs[b + 1]], cam)
        err, masked = compare_image(imgs[b], ref, fl, tag=f"uneven-sets frame {b}")
        assert err <= IMAGE_TOL, (b, err)
        assert masked <= MASK_FRAC_MAX, (b, masked)


def test_tile_size_and_chunk_invariance_bit_exact():
    raw, cams, N = batch_case(B=3, N=3000, seed=5)
    base = None
    for tile in (8, 16, 32):
        for chunk in (64, 128, 256):
            ctx = make_ctx(tile=tile, chunk=chunk)
            imgs, _, _ = render(ctx, raw, cams)
            flat = np.concatenate([i.ravel() for i in imgs])
            if base is None:
                base = flat
            assert np.array_equal(flat, base), (tile, chunk)
            ctx.close()


def test_frame_alone_equals_frame_in_batch():
    raw, cams, N = batch_case(B=6, N=2000, seed=6)
    ctx = make_ctx()
    imgs, _, _ = render(ctx, raw, cams)
    for b in (0, 3, 5):
        one, _, _ = render(ctx, raw[b * N:(b + 1) * N], [cams[b]])
        assert np.array_equal(one[0], imgs[b])


def test_run_to_run_deterministic():
    raw, cams, N = batch_case(B=4, N=4000, seed=7)
    ctx = make_ctx()
    a, _, _ = render(ctx, raw, cams)
    b, _, _ = render(ctx, raw, cams)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_degenerate_inputs():
    ctx = make_ctx()
    cam = synth.fixed_camera(37, 21, 60.0, 0.5, bg=(0.1, 0.7, 0.3))
    # every Gaussian behind the camera -> background everywhere
    r = np.zeros((10, 16), np.float32)
    r[:, 2] = -1.0; r[:, 3] = 1.0
    imgs, _, _ = render(ctx, r, [cam])
    assert np.array_equal(imgs[0], np.broadcast_to(np.float32([0.1, 0.7, 0.3])[:, None, None], (3, 21, 37)))
    # a single Gaussian far off screen, and a 1x1 image
    r = np.zeros((1, 16), np.float32)
    r[0, 0] = 5.0; r[0, 3] = 1.0; r[0, 7:10] = -5.0
    imgs, _, _ = render(ctx, r, [cam])
    assert np.allclose(imgs[0][1], 0.7)
    cam1 = synth.fixed_camera(1, 1, 60.0, 0.5, bg=(0, 0, 0))
    r = np.zeros((1, 16), np.float32)
    r[0, 3] = 1.0; r[0, 7:10] = -4.0; r[0, 10] = 3.0; r[0, 11:14] = 1.0
    imgs, _, _ = render(ctx, r, [cam1])
    ref, _, _, _ = raster.render(r, cam1)
    assert np.abs(imgs[0] - ref).max() <= IMAGE_TOL


def test_overflow_is_reported_and_recoverable():
    raw, cams, N = batch_case(B=2, N=3000, seed=8)
    import torch
    ctx = make_ctx(max_entries=1000)
    rw = dev(raw)
    out = torch.zeros(gbr.image_numel(cams), device="cuda")
    gbr.gbr_render(ctx, rw, [0, N, 2 * N], cams, out)
    st = gbr.gbr_query_status(ctx)
    assert st.overflow and st.entries > 1000
    gbr.gbr_reserve(ctx, st.entries)
    gbr.gbr_render(ctx, rw, [0, N, 2 * N], cams, out)
    st2 = gbr.gbr_query_status(ctx)
    assert not st2.overflow and st2.entries == st.entries
    ref_ctx = make_ctx()
    ref, _, _ = render(ref_ctx, raw, cams)
    assert np.array_equal(host(out), np.concatenate([i.ravel() for i in ref]))


def test_per_frame_scheme_matches_batched():
    """preprocess -> host sync on the entry count -> rasterize (Fig. 5a)."""
    import torch
    raw, cams, N = batch_case(B=3, N=2000, seed=9)
    ctx = make_ctx(max_entries=64)
    rw = dev(raw)
    outs = []
    for b in range(3):
        out = torch.zeros(gbr.image_numel([cams[b]]), device="cuda")
        gbr.gbr_preprocess(ctx, rw[b * N:(b + 1) * N], [0, N], [cams[b]])
        e = gbr.gbr_entry_count(ctx)
        assert e > 64
        gbr.gbr_rasterize(ctx, out)
        outs.append(host(out))
    ref_ctx = make_ctx()
    ref, _, _ = render(ref_ctx, raw, cams)
    assert np.array_equal(np.concatenate(outs), np.concatenate([i.ravel() for i in ref]))


def test_invalid_arguments_are_rejected():
    ctx = make_ctx(max_frames=2)
    import torch
    raw = torch.zeros(32, device="cuda")
    cams = synth.make_cameras(3, 16, 16)
    out = torch.zeros(gbr.image_numel(cams), device="cuda")
    with pytest.raises(gbr.GbrError) as e:
        gbr.gbr_render(ctx, raw, [0, 1, 2, 2], cams, out)
    assert e.value.code == -2
    with pytest.raises(gbr.GbrError) as e:
        gbr.gbr_render(ctx, raw, [0, 2, 1], cams[:2], out)      # decreasing offsets
    assert e.value.code == -1
    bad = synth.make_cameras(1, 16, 16)
    bad[0].width = 0
    with pytest.raises(gbr.GbrError):
        gbr.gbr_render(ctx, raw, [0, 1], bad, out)
    fresh = make_ctx()
    with pytest.raises(gbr.GbrError) as e:
        gbr.gbr_render_backward(fresh, out, raw)
    assert e.value.code == -5


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_contribution_masks_match_reference_contributors(tile):
    """The forward pass's per-entry contribution bits (one per wave quadrant)
    are exactly 'some pixel of the quadrant has this Gaussian among its
    contributors' in the reference, on quadrants with no ambiguous pixel;
    no reference contributor lies past a quadrant's last used list position,
    and a tile's last position is the largest of its quadrants'."""
    raw, cams, N = batch_case(B=3, N=2500, seed=7)
    ctx = make_ctx(tile=tile)
    render(ctx, raw, cams)
    ntiles = [((c.width + tile - 1) // tile) * ((c.height + tile - 1) // tile) for c in cams]
    tile_base = np.concatenate([[0], np.cumsum(ntiles)])
    ts = gbr.gbr_inspect(ctx, "tile_start", int(tile_base[-1]) + 1).astype(np.int64)
    srt = gbr.gbr_inspect(ctx, "sorted", int(ts[-1])).astype(np.int64)
    cm = gbr.gbr_inspect(ctx, "cmask", int(ts[-1]))
    last = gbr.gbr_inspect(ctx, "tile_last", int(tile_base[-1])).astype(np.int64)
    ql = gbr.gbr_inspect(ctx, "quad_last", int(tile_base[-1])).astype(np.int64)
    q = tile // 2 if tile > 8 else tile          # quadrant side
    nq = 4 if tile > 8 else 1
    assert np.array_equal(last, ql.max(axis=1))   # the tile's last position is its quadrants' largest
    if nq == 1:
        assert not ql[:, 1:].any()
    checked = 0
    for b, cam in enumerate(cams):
        r = raw[b * N:(b + 1) * N]
        lists, cnt = raster.contributors(r, cam, cap=1024)
        _, _, _, fl = raster.render(r, cam)
        ntx = (cam.width + tile - 1) // tile
        for lt in range(ntiles[b]):
            g = tile_base[b] + lt
            tx, ty = lt % ntx, lt // ntx
            sets, ambiguous = [], []
            for w in range(nq):
                x0, y0 = tx * tile + (w & 1) * q, ty * tile + (w >> 1) * q
                ys = slice(y0, min(y0 + q, cam.height))
                xs = slice(x0, min(x0 + q, cam.width))
                sub = lists[ys, xs]
                sets.append(set(sub[sub >= 0].tolist()))
                ambiguous.append(bool(fl[ys, xs].any()))
            for i in range(ts[g], ts[g + 1]):
                n = srt[i] - b * N
                want = [n in sets[w] for w in range(nq)]
                if i - ts[g] >= last[g]:
                    assert not any(want[w] and not ambiguous[w] for w in range(nq)), (b, lt, i)
                    continue
                for w in range(nq):
                    if not ambiguous[w]:
                        # past its own last position a quadrant has no contributor and no bit
                        if i - ts[g] >= ql[g, w]:
                            assert not want[w] and not (cm[i] >> w) & 1, (b, lt, i, w)
                        assert bool((cm[i] >> w) & 1) == want[w], (b, lt, i, w)
                        checked += 1
    assert checked > 1000
    ctx.close()


def test_pass_order_is_a_prefix_of_the_complete_lists():
    """The forward pass orders each tile's list only as far as it composites;
    what it left must be the leading part of the complete sorted list."""
    raw, cams, N = batch_case(B=3, N=3000, seed=11)
    ctx = make_ctx()
    render(ctx, raw, cams)
    n_tiles = sum(((c.width + 15) // 16) * ((c.height + 15) // 16) for c in cams)
    ts = gbr.gbr_inspect(ctx, "tile_start", n_tiles + 1).astype(np.int64)
    last = gbr.gbr_inspect(ctx, "tile_last", n_tiles).astype(np.int64)
    part = gbr.gbr_inspect(ctx, "sorted_pass", int(ts[-1])).astype(np.int64)
    full = gbr.gbr_inspect(ctx, "sorted", int(ts[-1])).astype(np.int64)
    used = 0
    for g in range(n_tiles):
        k = ts[g] + last[g]
        assert np.array_equal(part[ts[g]:k], full[ts[g]:k]), g
        used += last[g]
    assert used > 0
    ctx.close()


def test_large_frame_orders_tiles_in_a_separate_pass():
    """Frames with more visible splats than the lazy in-kernel ordering holds
    (its bitmap) take the separate per-tile sort; same images, same lists."""
    N = 300_000
    bases = synth.make_scene(N, 2, seed=12)
    w = synth.make_weights(1, 2, seed=13)
    cam = synth.fixed_camera(64, 64, 75.0, 0.5, bg=(0.3, 0.2, 0.1))
    raw = bs.blend(bases, w).astype(np.float32)[0]
    ctx = make_ctx(max_splats=N, max_entries=1 << 24)
    imgs, _, _ = render(ctx, raw, [cam])
    ref, _, _, fl = raster.render(raw, cam)
    err, masked = compare_image(imgs[0], ref, fl, tag="300k-Gaussian frame")
    # 300,000 Gaussians over 64 x 64 pixels: thousands of contributors per
    # pixel, 5 of the 4096 pixels flagged
    assert err <= IMAGE_TOL and masked <= 2 * MASK_FRAC_MAX, (err, masked)
    proj = raster.project(raw, cam)
    ranges, sf, sg, _ = raster.bin_and_sort([proj], [cam], 16)
    srt = gbr.gbr_inspect(ctx, "sorted", len(sg)).astype(np.int64)
    assert np.array_equal(srt, sg)
    ctx.close()


@pytest.mark.parametrize("W,H", [(400, 360), (320, 320)])
def test_frames_with_many_tiles_build_rows_in_memory(W, H):
    """A frame with more tiles than the workgroup's LDS copy of its bitmap
    words holds (tile 8, 400 x 360 = 2250 tiles) sets its rows' bits in
    memory; one of 1600 tiles still builds them in LDS, with 8-word
    segments.  Lists and image as the reference."""
    N = 3000
    bases = synth.make_scene(N, 2, seed=14)
    w = synth.make_weights(1, 2, seed=15)
    cam = synth.fixed_camera(W, H, 400.0, 0.5, bg=(0.5, 0.4, 0.3))
    raw = bs.blend(bases, w).astype(np.float32)[0]
    ctx = make_ctx(tile=8)
    imgs, _, _ = render(ctx, raw, [cam])
    ref, _, _, fl = raster.render(raw, cam)
    err, masked = compare_image(imgs[0], ref, fl, tag=f"{W}x{H} frame, tile 8")
    assert err <= IMAGE_TOL and masked <= MASK_FRAC_MAX, (err, masked)
    proj = raster.project(raw, cam)
    ranges, sf, sg, _ = raster.bin_and_sort([proj], [cam], 8)
    assert len(ranges) == (W // 8) * (H // 8)
    ts = gbr.gbr_inspect(ctx, "tile_start", len(ranges) + 1).astype(np.int64)
    assert np.array_equal(ts[:-1], ranges[:, 0]) and np.array_equal(ts[1:], ranges[:, 1])
    srt = gbr.gbr_inspect(ctx, "sorted", len(sg)).astype(np.int64)
    assert np.array_equal(srt, sg)
    ctx.close()


@pytest.mark.parametrize("N", [100, 1500, 5000])
def test_equal_depths_rank_by_index(N):
    """Gaussians all at one depth fall in one depth bucket, which is ranked
    in LDS by comparison (100 keys), by the large-bucket workgroups'
    comparison (1500) or by their radix passes (5000); equal depths go by
    Gaussian index, so the tile lists equal the reference's bit for bit and
    the image agrees."""
    rng = np.random.default_rng(N)
    r = np.zeros((N, 16), np.float32)
    r[:, 0] = rng.uniform(-0.08, 0.08, N)
    r[:, 1] = rng.uniform(-0.07, 0.07, N)
    r[:, 3] = 1.0                                  # identity rotation: every mean at camera depth 0.5
    r[:, 7:10] = rng.normal(-5.0, 0.3, (N, 3))
    r[:, 10] = rng.normal(0.0, 1.0, N)
    r[:, 11:14] = rng.uniform(0.0, 1.0, (N, 3))
    cam = synth.fixed_camera(96, 80, 150.0, 0.5, bg=(0.2, 0.3, 0.4))
    ctx = make_ctx(tile=16)
    imgs, _, _ = render(ctx, r, [cam])
    proj = raster.project(r, cam)
    v = proj["valid"] > 0
    assert v.sum() > 0.9 * N and np.unique(proj["depth"][v].astype(np.float32)).size == 1
    ranges, sf, sg, _ = raster.bin_and_sort([proj], [cam], 16)
    ts = gbr.gbr_inspect(ctx, "tile_start", len(ranges) + 1).astype(np.int64)
    assert np.array_equal(ts[:-1], ranges[:, 0]) and np.array_equal(ts[1:], ranges[:, 1])
    srt = gbr.gbr_inspect(ctx, "sorted", len(sg)).astype(np.int64)
    assert np.array_equal(srt, sg)
    ref, _, _, fl = raster.render(r, cam)
    err, masked = compare_image(imgs[0], ref, fl, tag=f"equal depths, N={N}")
    assert err <= IMAGE_TOL and masked <= MASK_FRAC_MAX, (err, masked)
    ctx.close()


def test_frame_without_gaussians_in_a_batch():
    """A frame whose Gaussian range is empty renders its background; the
    frames around it are unaffected (bit-equal to rendering them alone), and
    the backward gives them the same gradient."""
    import torch
    raw, cams, N = batch_case(B=2, N=2000, seed=21)
    cam_e = synth.fixed_camera(40, 24, 60.0, 0.5, bg=(0.6, 0.1, 0.9))
    cams3 = [cams[0], cam_e, cams[1]]
    ctx = make_ctx()
    imgs, rt, _ = render(ctx, raw, cams3, gauss_offsets=[0, N, N, 2 * N])
    assert np.array_equal(imgs[1], np.broadcast_to(np.float32([0.6, 0.1, 0.9])[:, None, None], (3, 24, 40)))
    rng = np.random.default_rng(22)
    dimg = [rng.normal(size=(3, c.height, c.width)).astype(np.float32) for c in cams3]
    draw3 = torch.zeros(2 * N, 16, device="cuda")
    gbr.gbr_render_backward(ctx, dev(np.concatenate([d.ravel() for d in dimg])), draw3)
    torch.cuda.synchronize()
    ctx2 = make_ctx()
    imgs2, rt2, _ = render(ctx2, raw, [cams[0], cams[1]])
    assert np.array_equal(imgs[0], imgs2[0]) and np.array_equal(imgs[2], imgs2[1])
    draw2 = torch.zeros(2 * N, 16, device="cuda")
    gbr.gbr_render_backward(ctx2, dev(np.concatenate([dimg[0].ravel(), dimg[2].ravel()])), draw2)
    torch.cuda.synchronize()
    assert torch.equal(draw3, draw2)
    ctx.close()
    ctx2.close()
