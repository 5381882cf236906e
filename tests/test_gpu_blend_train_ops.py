"""GPU parity of the dense pieces: blend (Eq. 1) and its adjoint, the weight
MLP (Eq. 2), the photometric loss and Adam, against the float64 oracle."""
import numpy as np
import pytest

from oracle import blendshape as bs
from paper_2503_12886_amd import gbr, synth
from gpu_util import dev, host, make_ctx

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("B,K,N", [(1, 8, 2000), (3, 20, 4133), (17, 20, 37), (16, 20, 1000), (5, 0, 100),
                                   (33, 63, 130)])
def test_blend_matches_float64_rounded_once(B, K, N):
    bases = synth.make_scene(N, K, seed=B + K)
    w = synth.make_weights(B, K, seed=7) if K else np.zeros((B, 0), np.float32)
    ref = bs.blend(bases, w.astype(np.float64)).astype(np.float32)
    ctx = make_ctx()
    raw = dev(np.zeros((B, N, 16), np.float32))
    gbr.gbr_blend(ctx, dev(bases), dev(w if K else np.zeros((B, 1), np.float32)), raw)
    got = host(raw)
    ref[..., 14:] = 0.0
    # float64 accumulation rounded once: equal except where the two float64
    # sums straddle a float32 rounding boundary (then 1 ulp apart)
    diff = got.view(np.int32).astype(np.int64) - ref.view(np.int32).astype(np.int64)
    assert np.abs(diff).max() <= 1
    assert (diff != 0).mean() < 1e-4


def test_blend_is_independent_of_batch():
    B, K, N = 19, 20, 3000
    bases = dev(synth.make_scene(N, K, seed=1))
    w = synth.make_weights(B, K, seed=3)
    ctx = make_ctx()
    full = dev(np.zeros((B, N, 16), np.float32))
    gbr.gbr_blend(ctx, bases, dev(w), full)
    for b in (0, 7, 18):
        one = dev(np.zeros((1, N, 16), np.float32))
        gbr.gbr_blend(ctx, bases, dev(w[b:b + 1]), one)
        assert np.array_equal(host(one)[0], host(full)[b])


@pytest.mark.parametrize("B,K,N", [(1, 8, 2000), (16, 20, 3000), (17, 20, 517), (40, 40, 300)])
def test_blend_backward(B, K, N):
    rng = np.random.default_rng(11)
    bases = synth.make_scene(N, K, seed=2)
    w = synth.make_weights(B, K, seed=4)
    draw = rng.normal(size=(B, N, 16)).astype(np.float32)
    draw[..., 14:] = 0.0
    dB_ref, dw_ref = bs.blend_adjoint(draw, bases, w)
    ctx = make_ctx()
    dB = dev(np.zeros_like(bases))
    dw = dev(np.zeros((B, K), np.float32))
    gbr.gbr_blend_backward(ctx, dev(draw), dev(bases), dev(w), dB, dw)
    dB_ref[..., 14:] = 0.0
    assert np.abs(host(dB) - dB_ref).max() <= 1e-5 * np.abs(dB_ref).max()
    assert np.linalg.norm(host(dw) - dw_ref) <= 1e-5 * np.linalg.norm(dw_ref)
    # accumulate adds into the outputs
    gbr.gbr_blend_backward(ctx, dev(draw), dev(bases), dev(w), dB, dw, accumulate=True)
    assert np.allclose(host(dB), 2 * dB_ref, rtol=1e-5, atol=1e-5 * np.abs(dB_ref).max())


def _mlp_pack(p):
    return np.concatenate([p["W1"].ravel(), p["b1"], p["W2"].ravel(), p["b2"], p["W3"].ravel(), p["b3"]])


@pytest.mark.parametrize("B,d_in,hidden,K", [(1, 56, 256, 20), (16, 56, 256, 20), (37, 56, 256, 20),
                                            (5, 100, 128, 40), (3, 7, 300, 64)])
def test_mlp_forward_backward(B, d_in, hidden, K):
    """The training shape (56 -> 256 -> 256 -> 20) and others: hidden sizes
    that split unevenly over the backward's four workgroups per frame, and
    the largest K."""
    p = synth.make_mlp(K=K, seed=5, d_in=d_in, hidden=hidden)
    rng = np.random.default_rng(2)
    theta = synth.make_tracking(B, seed=2) if d_in == 56 else rng.normal(size=(B, d_in)).astype(np.float32)
    psi_ref, cache = bs.mlp_forward(p, theta)
    g = np.random.default_rng(0).normal(size=psi_ref.shape).astype(np.float32)
    grads = bs.mlp_backward(p, cache, g)
    ctx = make_ctx()
    P = dev(_mlp_pack(p))
    th = dev(theta)
    psi = dev(np.zeros((B, K), np.float32))
    gbr.gbr_mlp_forward(ctx, P, th, d_in, hidden, K, psi)
    assert np.abs(host(psi) - psi_ref).max() <= 1e-5 * max(1.0, np.abs(psi_ref).max())
    dP = dev(np.zeros_like(_mlp_pack(p)))
    gbr.gbr_mlp_backward(ctx, P, dev(g), dP)
    ref = _mlp_pack(grads)
    assert np.linalg.norm(host(dP) - ref) <= 1e-5 * np.linalg.norm(ref)


def test_adam_matches_reference():
    rng = np.random.default_rng(3)
    n = 21 * 1000 * 16
    p0 = rng.normal(size=n).astype(np.float32)
    lr = bs.feature_lrs(20)
    split = 1000 * 16
    lr_flat = np.concatenate([np.tile(lr[0], 1000), np.tile(lr[1], 20 * 1000)])
    table = list(lr[0]) + list(lr[1])
    ctx = make_ctx()
    P = dev(p0); M = dev(np.zeros(n, np.float32)); V = dev(np.zeros(n, np.float32))
    pr, mr, vr = p0.astype(np.float64), np.zeros(n), np.zeros(n)
    for step in range(1, 4):
        g = rng.normal(size=n).astype(np.float32)
        gbr.gbr_adam_step(ctx, 0, P, dev(g), M, V, split, table)
        pr, mr, vr = bs.adam_step(pr, g, mr, vr, step, lr_flat)
    assert np.abs(host(P) - pr).max() <= 1e-6 + 1e-6 * np.abs(pr).max()
    assert gbr.gbr_query_status(ctx).adam_steps[0] == 3


def test_adam_step_count_across_grid_shapes():
    """Each update advances its group's step count once: over updates of one
    workgroup, of 1313, of the 8192-workgroup grid-stride cap and of no
    element, the counts equal the number of updates per group, and every
    element follows the reference with the bias correction of the step it was
    updated at."""
    rng = np.random.default_rng(11)
    n_big = 8192 * 256 + 1000
    table = [1e-3] * 32
    ctx = make_ctx()
    p0 = rng.normal(size=n_big).astype(np.float32)
    P = dev(p0); M = dev(np.zeros(n_big, np.float32)); V = dev(np.zeros(n_big, np.float32))
    pr, mr, vr = p0.astype(np.float64), np.zeros(n_big), np.zeros(n_big)
    sizes = [n_big, 1, 21 * 1000 * 16, 0, n_big, 777, 64]
    for step, k in enumerate(sizes, start=1):
        g = rng.normal(size=k).astype(np.float32)
        gbr.gbr_adam_step(ctx, 2, P[:k], dev(g), M[:k], V[:k], 0, table)
        if k:
            pr[:k], mr[:k], vr[:k] = bs.adam_step(pr[:k], g, mr[:k], vr[:k], step, 1e-3)
        gbr.gbr_adam_step(ctx, 3, P[:0], P[:0], P[:0], P[:0], 0, table)   # another group, no elements
        st = gbr.gbr_query_status(ctx)
        assert st.adam_steps[2] == step and st.adam_steps[3] == step and st.adam_steps[0] == 0
    assert np.abs(host(P) - pr).max() <= 1e-6 + 1e-6 * np.abs(pr).max()


def test_loss_l1_l2():
    cams = synth.make_cameras(3, 40, 24, seed=1)
    imgs = [np.random.default_rng(i).uniform(size=(3, c.height, c.width)).astype(np.float32) for i, c in enumerate(cams)]
    tg = synth.make_targets(cams)
    ctx = make_ctx()
    # a loss needs a pass to know the frame layout: render an empty scene
    r = np.zeros((3, 16), np.float32)
    r[:, 2] = -1.0                      # behind every camera: culled
    r[:, 3] = 1.0
    raw = dev(r)
    out = dev(np.zeros(gbr.image_numel(cams), np.float32))
    gbr.gbr_render(ctx, raw, [0, 1, 2, 3], cams, out)
    for kind, fn in ((1, bs.loss_l1), (2, bs.loss_l2)):
        d = dev(np.zeros(gbr.image_numel(cams), np.float32))
        x = np.concatenate([i.ravel() for i in imgs]); y = np.concatenate([t.ravel() for t in tg])
        gbr.gbr_loss(ctx, dev(x), dev(y), kind, d)
        L, G = fn(imgs, tg)
        st = gbr.gbr_query_status(ctx)
        assert st.loss == pytest.approx(L, rel=1e-6)
        assert np.allclose(host(d), np.concatenate([gg.ravel() for gg in G]), rtol=1e-6, atol=1e-12)
