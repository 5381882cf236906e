"""The allocation-free blend adjoint (gbr_blend_backward_noalloc) against the
context entry point gbr_blend_backward: two calls in a row, the second on a
smaller input, bit for bit; accumulation; a shape beyond its fixed scratch
is refused."""
import numpy as np
import pytest

from paper_2503_12886_amd import gbr, synth
from gpu_util import dev, make_ctx

pytestmark = pytest.mark.gpu


def _case(B, K, N, seed):
    rng = np.random.default_rng(seed)
    bases = synth.make_scene(N, K, seed=seed)
    w = synth.make_weights(B, K, seed=seed + 1)
    draw = rng.normal(size=(B, N, 16)).astype(np.float32)
    draw[..., 14:] = 0.0
    return dev(bases), dev(w), dev(draw)


def _pair(ctx, bases, w, draw, accumulate=False, init=None):
    import torch
    K1, N, _ = bases.shape
    B = draw.shape[0]
    outs = []
    for fn in ("ctx", "noalloc"):
        dB = torch.zeros_like(bases) if init is None else init[0].clone()
        dW = torch.zeros(B, K1 - 1, device="cuda") if init is None else init[1].clone()
        if fn == "ctx":
            gbr.gbr_blend_backward(ctx, draw, bases, w, dB, dW, accumulate)
        else:
            gbr.gbr_blend_backward_noalloc(draw, bases, w, dB, dW, accumulate)
        torch.cuda.synchronize()
        outs.append((dB.cpu().numpy(), dW.cpu().numpy()))
    return outs


def test_noalloc_blend_backward_equals_context_entry_point():
    import torch
    ctx = make_ctx(max_frames=16, max_splats=16 * 50_000)
    # the training batch's shape, then a smaller ragged one (N not a multiple of 64)
    for B, K, N, seed in ((16, 20, 50_000, 1), (3, 7, 1_234, 2)):
        print(f"noalloc case B={B} K={K} N={N}", flush=True)
        bases, w, draw = _case(B, K, N, seed)
        (b0, w0), (b1, w1) = _pair(ctx, bases, w, draw)
        assert np.array_equal(b0, b1) and np.array_equal(w0, w1), (B, K, N)
        assert np.abs(w1).max() > 0
    # accumulate into existing outputs
    init = (torch.ones_like(bases), torch.ones(draw.shape[0], bases.shape[0] - 1, device="cuda"))
    (b0, w0), (b1, w1) = _pair(ctx, bases, w, draw, accumulate=True, init=init)
    assert np.array_equal(b0, b1) and np.array_equal(w0, w1)
    ctx.close()


def test_noalloc_refuses_shapes_beyond_its_scratch():
    import torch
    B, K, N = 64, 40, 20_000          # 4 * ceil(N*16/1024) * B * K partials > 2^20
    bases = torch.zeros(K + 1, N, 16, device="cuda")
    w = torch.zeros(B, K, device="cuda")
    draw = torch.zeros(B, N, 16, device="cuda")
    dW = torch.zeros(B, K, device="cuda")
    with pytest.raises(gbr.GbrError) as e:
        gbr.gbr_blend_backward_noalloc(draw, bases, w, None, dW)
    assert e.value.code == -2
