"""The autograd wrapper: images and gradients through torch.autograd equal
the float64 reference (blend, render, adjoint) on a small two-frame batch."""
import numpy as np
import pytest

from oracle import blendshape as bs
from oracle import raster
from paper_2503_12886_amd import synth
from gpu_util import IMAGE_TOL, compare_image, dev, grad_check, host, make_ctx, masked_gaussians, split_images

pytestmark = pytest.mark.gpu


def test_blend_render_autograd_matches_reference():
    import torch
    from paper_2503_12886_amd.autograd import blend_render
    B, N, K = 2, 1500, 6
    bases = synth.make_scene(N, K, seed=7)
    w = synth.make_weights(B, K, seed=8)
    cams = synth.make_cameras(B, 96, 80, seed=9)
    rng = np.random.default_rng(10)
    g = [rng.normal(size=(3, c.height, c.width)) for c in cams]
    ctx = make_ctx(max_entries=1024)           # forces the overflow-and-grow path
    Bt = dev(bases).requires_grad_(True)
    Wt = dev(w).requires_grad_(True)
    images = blend_render(Bt, Wt, cams, ctx)
    gflat = dev(np.concatenate([x.ravel() for x in g]).astype(np.float32))
    (images * gflat).sum().backward()
    torch.cuda.synchronize()

    raw = bs.blend(bases, w).astype(np.float32)
    draw_ref = np.zeros((B, N, 16))
    bad = np.zeros((B, N), dtype=bool)
    for b, (cam, img) in enumerate(zip(cams, split_images(host(images), cams))):
        ref, _, _, fl = raster.render(raw[b], cam)
        err, masked = compare_image(img, ref, fl)
        assert err <= IMAGE_TOL and masked < 0.02, (b, err, masked)
        draw_ref[b], _ = raster.render_grad(raw[b], cam, g[b])
        bad[b] = masked_gaussians(raster.project(raw[b], cam), fl)
    dbases_ref, dw_ref = bs.blend_adjoint(draw_ref, bases, w)
    rel, _ = grad_check(host(Bt.grad)[..., :14], dbases_ref[..., :14])
    assert rel <= 1e-3, rel
    rel, _ = grad_check(host(Wt.grad), dw_ref)
    assert rel <= 1e-3, rel
    ctx.close()
