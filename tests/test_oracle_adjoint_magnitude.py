"""Pins of the reference's projection adjoint applied on its own and of the
adjoint magnitudes (the sums of per-pixel term magnitudes that bound a
binary32 implementation's cancellation error): the projection adjoint of the
render's projected-quantity gradients is the render's adjoint; a magnitude
bounds the gradient it belongs to, scales with |dL/dimage| and ignores its
sign, and reduces to |gradient| where a single pixel contributes."""
import numpy as np

from oracle import blendshape as bs
from oracle import raster
from paper_2503_12886_amd import synth


def _scene(seed=0, N=300, W=48):
    bases = synth.make_scene(N, 2, seed=seed)
    w = synth.make_weights(1, 2, seed=seed + 1)
    raw = bs.blend(bases, w)[0]
    cam = synth.fixed_camera(W, W, 150.0 * W / 128.0, 0.5, bg=(0.3, 0.2, 0.1))
    return raw, cam


def test_projection_adjoint_alone_equals_render_adjoint():
    raw, cam = _scene()
    g = np.random.default_rng(1).normal(size=(3, cam.height, cam.width))
    draw, dproj = raster.render_grad(raw, cam, g)
    again = raster.project_adjoint(raw, cam, dproj)
    assert np.allclose(again, draw, rtol=1e-12, atol=1e-15 * np.abs(draw).max())


def test_magnitude_bounds_gradient_and_scales():
    raw, cam = _scene(seed=2)
    g = np.random.default_rng(3).normal(size=(3, cam.height, cam.width))
    draw, _ = raster.render_grad(raw, cam, g)
    mag = raster.adjoint_magnitude(raw, cam, g)
    assert np.all(mag >= np.abs(draw) * (1 - 1e-12))
    assert (mag[:, :14] > 2 * np.abs(draw[:, :14])).any()       # cancellation exists, and is seen
    assert np.allclose(raster.adjoint_magnitude(raw, cam, -g), mag, rtol=1e-12)
    assert np.allclose(raster.adjoint_magnitude(raw, cam, 2.5 * g), 2.5 * mag, rtol=1e-12)


def test_single_pixel_single_quantity_magnitude_is_exact():
    """One pixel of one channel: every projected-quantity gradient is a single
    term, so the colour magnitudes equal |dL/dcolour| exactly."""
    raw, cam = _scene(seed=4)
    g = np.zeros((3, cam.height, cam.width))
    g[1, cam.height // 2, cam.width // 2] = 0.7
    draw, dproj = raster.render_grad(raw, cam, g)
    mag = raster.adjoint_magnitude(raw, cam, g)
    assert np.count_nonzero(dproj[:, 7]) > 0
    assert np.allclose(mag[:, 12], np.abs(draw[:, 12]), rtol=1e-12, atol=0)
    assert np.all(mag[:, 11] == 0) and np.all(mag[:, 13] == 0)
