"""Pins of the reference's ambiguity margins (the flags that mark pixels where
a binary32 renderer may take another discrete decision than the float64
reference: alpha against 1/255 and 0.99, the transmittance stop at 1e-4).

The margins are first-order bounds on a binary32 evaluation's error.  They
are checked here against binary32 evaluations written independently in
numpy (two different formulations of alpha, every operation rounded to
binary32, the exponential correctly rounded), against the binary32 product
of a pixel's transmittance factors, and on scenes built so that a decision
sits exactly on its threshold (flagged) or clearly off it (not flagged).
"""
import numpy as np
import pytest

from oracle import raster
from paper_2503_12886_amd import synth

F = np.float32
U = 2.0 ** -24


def _scene_and_samples(seed=0, N=400, W=512, per=24):
    bases = synth.make_scene(N, 0, seed=seed)
    raw = bases[0].astype(np.float64)
    cam = synth.fixed_camera(W, W, 150.0 * W / 128.0, 0.5, bg=(0.1, 0.2, 0.3))
    p = raster.project(raw, cam)
    rng = np.random.default_rng(seed + 1)
    g, x, y = [], [], []
    for n in np.nonzero(p["valid"] > 0)[0]:
        g.append(np.full(per, n))
        x.append(rng.integers(p["px0"][n], p["px1"][n] + 1, size=per) + 0.5)
        y.append(rng.integers(p["py0"][n], p["py1"][n] + 1, size=per) + 0.5)
    return raw, cam, p, np.concatenate(g), np.concatenate(x), np.concatenate(y)


def _alpha_f32_natural(p, g, x, y):
    """o * exp(-q/2), q = A dx^2 + 2 B dx dy + C dy^2, every step in binary32."""
    mx, my = p["mx"][g].astype(F), p["my"][g].astype(F)
    A, B, C = p["A"][g].astype(F), p["B"][g].astype(F), p["C"][g].astype(F)
    o = p["opacity"][g].astype(F)
    dx, dy = x.astype(F) - mx, y.astype(F) - my
    q = A * dx * dx + F(2) * B * dx * dy + C * dy * dy
    q = np.maximum(q, F(0))
    e = np.exp((F(-0.5) * q).astype(np.float64)).astype(F)     # correctly rounded exponential
    return o * e


def _alpha_f32_log2(p, g, x, y):
    """2^(log2 o + a dx^2 + b dx dy + c dy^2) with the conic pre-scaled by
    -log2(e)/2, every step in binary32, the power clamped at log2 o."""
    l2e = 1.0 / np.log(2.0)
    mx, my = p["mx"][g].astype(F), p["my"][g].astype(F)
    ca = (-0.5 * l2e * p["A"][g]).astype(F)
    cb = (-l2e * p["B"][g]).astype(F)
    cc = (-0.5 * l2e * p["C"][g]).astype(F)
    lo = np.log2(p["opacity"][g]).astype(F)
    dx, dy = x.astype(F) - mx, y.astype(F) - my
    pw = ca * dx * dx + lo
    pw = cb * dx * dy + pw
    pw = cc * dy * dy + pw
    pw = np.minimum(pw, lo)
    return np.exp2(pw.astype(np.float64)).astype(F)


@pytest.mark.parametrize("seed", [0, 1])
def test_alpha_bound_covers_binary32_evaluations(seed):
    raw, cam, p, g, x, y = _scene_and_samples(seed)
    a64, eb = raster.alpha_bounds(raw, cam, g, x, y)
    keep = a64 >= 1e-3
    assert keep.sum() > 2000
    worst = 0.0
    for fn in (_alpha_f32_natural, _alpha_f32_log2):
        a32 = fn(p, g, x, y).astype(np.float64)
        ratio = np.abs(a32 - a64)[keep] / (eb[keep] * a64[keep])
        assert ratio.max() <= 1.0, (fn.__name__, ratio.max())
        worst = max(worst, float(ratio.max()))
    # the bound is a worst case, not a vacuous one: some evaluation comes within 20x of it
    assert worst >= 0.05, worst
    # and it reflects the rounded mean: larger on the far side of a 512-px frame
    assert eb.max() > 50 * U


def test_transmittance_bound_covers_binary32_products():
    raw, cam, p, *_ = _scene_and_samples(2, N=3000, W=128)
    cam = synth.fixed_camera(128, 128, 150.0, 0.5, bg=(0.1, 0.2, 0.3))
    lists, cnt = raster.contributors(raw, cam)
    rng = np.random.default_rng(3)
    ys, xs = np.nonzero(cnt >= 8)
    assert len(ys) > 200
    pick = rng.choice(len(ys), size=200, replace=False)
    checked = 0
    for i, j in zip(ys[pick], xs[pick]):
        idx = lists[i, j, :cnt[i, j]]
        px, py = np.full(len(idx), j + 0.5), np.full(len(idx), i + 0.5)
        a64, eb = raster.alpha_bounds(raw, cam, idx, px, py)
        al64 = np.minimum(a64, 0.99)
        pr = raster.project(raw, cam)
        a32 = _alpha_f32_log2(pr, idx, px, py)
        al32 = np.minimum(a32, F(0.99))
        T64, T32, rho = 1.0, F(1.0), 0.0
        for k in range(len(idx)):
            T64 *= 1.0 - al64[k]
            T32 = T32 * (F(1.0) - al32[k])
            e = U if a64[k] >= 0.99 else eb[k]
            rho += al64[k] / (1.0 - al64[k]) * e + 2 * U
            assert abs(float(T32) - T64) <= rho * T64, (i, j, k)
        checked += 1
    assert checked == 200


def _stack(n, logit, ls=-4.0):
    r = np.zeros((n, 16))
    r[:, 0] = 0.0
    r[:, 1] = 0.0
    r[:, 2] = np.linspace(-0.02, 0.02, n)        # distinct depths, same screen position
    r[:, 3] = 1.0
    r[:, 7:10] = ls
    r[:, 10] = logit
    r[:, 11:14] = 0.5
    return r


def test_stop_on_the_threshold_is_flagged():
    # two clamped Gaussians at a pixel centre: T = (1 - 0.99)^2 = 1e-4 up to
    # double rounding, so the stop decision is on its threshold
    cam = synth.fixed_camera(32, 32, 150.0, 0.5, bg=(0.0, 0.0, 0.0))
    _, Te, nc, fl = raster.render(_stack(2, 8.0, ls=-2.0), cam)
    assert fl[15, 15] & 2 and fl[16, 16] & 2
    # opacity 0.985 instead: T after two is 2.25e-4, well clear of 1e-4
    logit = np.log(0.985 / 0.015)
    _, Te, nc, fl = raster.render(_stack(2, logit, ls=-2.0), cam)
    assert fl[16, 16] == 0 and nc[16, 16] == 2


def test_alpha_on_the_skip_threshold_is_flagged():
    # one isotropic Gaussian at the image centre, opacity chosen so that alpha
    # at the pixel centre (16.5, 16.5) is 1/255 up to double rounding
    cam = synth.fixed_camera(32, 32, 150.0, 0.5, bg=(0.0, 0.0, 0.0))
    ls = -4.0
    sig2 = (150.0 * np.exp(ls) / 0.5) ** 2 + 0.3
    o = np.exp(0.5 * 0.5 / sig2) / 255.0
    r = _stack(1, np.log(o / (1 - o)), ls=ls)
    r[0, 2] = 0.0
    _, _, _, fl = raster.render(r, cam)
    assert fl[16, 16] & 1
    assert fl[16, 16] == fl[15, 15] == fl[15, 16] == fl[16, 15]       # the four pixels at 0.5 px
    r[0, 10] += 0.01                                                  # 1 % more opacity
    _, _, _, fl = raster.render(r, cam)
    assert fl[16, 16] == 0


def test_clamp_on_the_threshold_is_flagged():
    cam = synth.fixed_camera(32, 32, 150.0, 0.5, bg=(0.0, 0.0, 0.0))
    ls = -2.0
    sig2 = (150.0 * np.exp(ls) / 0.5) ** 2 + 0.3
    o = 0.99 * np.exp(0.5 * 0.5 / sig2)
    r = _stack(1, np.log(o / (1 - o)), ls=ls)
    r[0, 2] = 0.0
    _, _, _, fl = raster.render(r, cam)
    assert fl[16, 16] & 4


def test_fixed_margins_flag_a_superset():
    raw, cam, *_ = _scene_and_samples(4, N=2000, W=128)
    cam = synth.fixed_camera(128, 128, 150.0, 0.5, bg=(0.1, 0.2, 0.3))
    d = raster.render(raw, cam)[3]
    wide = raster.render(raw, cam, 1e-3, 1e-2)[3]
    assert np.all(wide[d != 0] != 0)
