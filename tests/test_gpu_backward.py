"""GPU parity of the backward pass against the float64 adjoint: render
backward (dL/d blended Gaussians) and the full chain to the bases and
weights, on the tiny workload and on small batches."""
import numpy as np
import pytest

from oracle import blendshape as bs
from oracle import raster
from paper_2503_12886_amd import gbr, synth
from gpu_util import MASK_FRAC_MAX, dev, grad_check, host, make_ctx, render, report, zero_flagged

pytestmark = pytest.mark.gpu


def _render_grad_case(raw, cams, N, seed=0, tile=16, chunk=128, flags=None):
    """GPU render adjoint of a random image gradient; with the reference's
    flags, the gradient is zero at the ambiguous pixels."""
    import torch
    ctx = make_ctx(tile=tile, chunk=chunk)
    imgs, rw, images = render(ctx, raw, cams)
    rng = np.random.default_rng(seed)
    dimg = [rng.normal(size=(3, c.height, c.width)).astype(np.float32) for c in cams]
    if flags is not None:
        dimg = zero_flagged(dimg, flags)
    draw = torch.zeros(raw.shape[0] * 16, device="cuda")
    gbr.gbr_render_backward(ctx, dev(np.concatenate([d.ravel() for d in dimg])), draw)
    return host(draw).reshape(-1, 16), dimg


def test_tiny_render_backward():
    bases = synth.make_scene(2000, 8, seed=0)
    w = synth.make_weights(1, 8, seed=2)
    cam = synth.fixed_camera(128, 128, 150.0, 0.5, bg=(0.2, 0.3, 0.4))
    raw = bs.blend(bases, w).astype(np.float32)[0]
    _, _, nc, fl = raster.render(raw, cam)
    report("tiny backward", masked_frac=float((fl != 0).mean()), max_contributors=int(nc.max()))
    assert (fl != 0).mean() <= MASK_FRAC_MAX
    got, dimg = _render_grad_case(raw, [cam], 2000, flags=[fl])
    ref, _ = raster.render_grad(raw, cam, dimg[0])
    mag = raster.adjoint_magnitude(raw, cam, dimg[0])
    rel, worst = grad_check(got[:, :14], ref[:, :14], tag="tiny backward draw", mag=mag[:, :14], n_max=nc.max())
    assert rel <= 1e-3, rel
    assert worst <= 1.0, worst
    assert np.all(got[:, 14:] == 0)


@pytest.mark.parametrize("tile,chunk", [(8, 64), (16, 256), (32, 128)])
def test_batch_render_backward_all_tilings(tile, chunk):
    B, N = 3, 1500
    bases = synth.make_scene(N, 4, seed=1)
    w = synth.make_weights(B, 4, seed=3)
    cams = synth.make_cameras(B, seed=5, resolutions=[(72, 64), (96, 80)], dist=(0.45, 0.6))
    raw = bs.blend(bases, w).astype(np.float32).reshape(B * N, 16)
    refs = [raster.render(raw[b * N:(b + 1) * N], cam) for b, cam in enumerate(cams)]
    flags = [r[3] for r in refs]
    for b, fl in enumerate(flags):
        report(f"batch backward frame {b}", masked_frac=float((fl != 0).mean()), max_contributors=int(refs[b][2].max()))
        assert (fl != 0).mean() <= MASK_FRAC_MAX
    got, dimg = _render_grad_case(raw, cams, N, seed=1, tile=tile, chunk=chunk, flags=flags)
    for b, cam in enumerate(cams):
        r = raw[b * N:(b + 1) * N]
        ref, _ = raster.render_grad(r, cam, dimg[b])
        mag = raster.adjoint_magnitude(r, cam, dimg[b])
        rel, worst = grad_check(got[b * N:(b + 1) * N, :14], ref[:, :14],
                                tag=f"batch backward draw frame {b} tile {tile} chunk {chunk}", mag=mag[:, :14],
                                n_max=refs[b][2].max())
        assert rel <= 1e-3, (b, rel)
        assert worst <= 1.0, (b, worst)


def test_backward_deterministic_and_tiling_independent():
    B, N = 2, 2500
    bases = synth.make_scene(N, 4, seed=2)
    w = synth.make_weights(B, 4, seed=4)
    cams = synth.make_cameras(B, 80, 80, seed=6)
    raw = bs.blend(bases, w).astype(np.float32).reshape(B * N, 16)
    a, _ = _render_grad_case(raw, cams, N, seed=2)
    b, _ = _render_grad_case(raw, cams, N, seed=2)
    assert np.array_equal(a, b)


def test_full_chain_to_bases_and_weights():
    """Tiny workload end to end: L2 loss vs a random target -> dL/dbases, dL/dweights."""
    import torch
    N, K = 2000, 8
    bases = synth.make_scene(N, K, seed=0)
    w = synth.make_weights(1, K, seed=2)
    cam = synth.fixed_camera(128, 128, 150.0, 0.5, bg=(0.2, 0.3, 0.4))
    target = synth.make_targets([cam])[0]
    ctx = make_ctx()
    Bt, Wt = dev(bases), dev(w)
    raw = torch.zeros(N * 16, device="cuda")
    gbr.gbr_blend(ctx, Bt, Wt, raw.view(1, N, 16))
    images = torch.zeros(3 * 128 * 128, device="cuda")
    gbr.gbr_render(ctx, raw, [0, N], [cam], images)
    dimages = torch.zeros_like(images)
    gbr.gbr_loss(ctx, images, dev(target.ravel()), 2, dimages)
    dB = torch.zeros_like(Bt)
    dW = torch.zeros_like(Wt)
    gbr.gbr_backward(ctx, dimages, Bt, Wt, dB, dW)
    # reference chain in float64
    raw_ref = bs.blend(bases, w).astype(np.float32)[0]
    img_ref, _, _, fl = raster.render(raw_ref, cam)
    L, G = bs.loss_l2([img_ref], [target])
    draw_ref, _ = raster.render_grad(raw_ref, cam, G[0])
    dB_ref, dW_ref = bs.blend_adjoint(draw_ref[None], bases, w)
    st = gbr.gbr_query_status(ctx)
    assert st.loss == pytest.approx(L, rel=1e-4)
    rel, _ = grad_check(host(dB)[..., :14].reshape(-1, 14), dB_ref[..., :14].reshape(-1, 14))
    assert rel <= 1e-3, rel
    relw, _ = grad_check(host(dW).ravel(), dW_ref.ravel())
    assert relw <= 1e-3, relw
