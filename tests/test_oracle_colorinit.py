"""Pins of the colour-initialisation reference (Eq. 3): the splatting-weight
sums against a brute-force per-pixel composite, closed forms (a constant
image gives its colour; a ramp seen by a centred isotropic Gaussian gives
the ramp's centre value), and the first-visible-frame and threshold rules."""
import numpy as np

from oracle import colorinit, raster
from paper_2503_12886_amd import synth

from test_oracle_pins import _random_scene, cam_eye, one_gaussian


def brute_force_sums(raw, cam, target):
    """Per pixel, every Gaussian in depth order: w = alpha T of each taken one."""
    p = raster.project(raw, cam)
    N = raw.shape[0]
    idx = [n for n in range(N) if p["tz"][n] > cam.near]
    order = sorted(idx, key=lambda n: (np.float32(p["key"][n]), n))
    wi, w = np.zeros((N, 3)), np.zeros(N)
    for i in range(cam.height):
        for j in range(cam.width):
            T = 1.0
            for n in order:
                dx, dy = j + 0.5 - p["mx"][n], i + 0.5 - p["my"][n]
                S = np.array([[p["S00"][n], p["S01"][n]], [p["S01"][n], p["S11"][n]]])
                d = np.array([dx, dy])
                q = max(0.0, d @ np.linalg.solve(S, d))
                a = min(0.99, p["opacity"][n] * np.exp(-0.5 * q))
                if a < 1 / 255:
                    continue
                if T * (1 - a) < 1e-4:
                    break
                w[n] += a * T
                wi[n] += a * T * target[:, i, j]
                T *= 1 - a
    return wi, w


def test_sums_match_brute_force():
    rng = np.random.default_rng(0)
    for seed in range(2):
        raw = _random_scene(30, 20 + seed, spread=0.03)
        cam = cam_eye(W=16, H=16, f=60.0)
        target = rng.uniform(size=(3, 16, 16))
        wi, w = colorinit.frame_color_sums(raw, cam, target)
        bwi, bw = brute_force_sums(raw, cam, target)
        assert np.allclose(w, bw, atol=1e-10) and np.allclose(wi, bwi, atol=1e-10)
        assert (w > colorinit.DELTA).sum() > 5


def test_constant_image_gives_its_colour():
    raw = _random_scene(200, 5)
    cam = cam_eye(W=48, H=48)
    c = np.array([0.2, 0.7, 0.45])
    target = np.broadcast_to(c[:, None, None], (3, 48, 48))
    cols, done, _ = colorinit.color_init(raw[None], [cam], target[None], np.zeros((200, 3)), np.zeros(200, bool))
    assert done.sum() > 20
    assert np.allclose(cols[done], c, atol=1e-12)
    assert not cols[~done].any()


def test_centred_isotropic_gaussian_sees_the_ramp_centre():
    cam = cam_eye(W=48, H=40, bg=(0.0, 0.0, 0.0))
    r = one_gaussian((0.0, 0.0, 0.0), log_s=(-4.0, -4.0, -4.0), logit=1.0)
    x = np.arange(48) + 0.5
    target = np.zeros((3, 40, 48))
    target[0] = 0.1 + 0.01 * x[None, :]          # linear in x, symmetric weights about x = 24
    target[1] = 0.3
    target[2] = 0.9 - 0.02 * (np.arange(40) + 0.5)[:, None]
    cols, done, _ = colorinit.color_init(r[None], [cam], target[None], np.zeros((1, 3)), np.zeros(1, bool))
    assert done[0]
    assert np.allclose(cols[0], [0.1 + 0.01 * 24.0, 0.3, 0.9 - 0.02 * 20.0], atol=1e-12)


def test_first_visible_frame_and_threshold():
    cams = [cam_eye(W=32, H=32), cam_eye(W=32, H=32), cam_eye(W=32, H=32)]
    raw = np.vstack([one_gaussian((0.0, 0.0, 0.0), log_s=(-4, -4, -4), logit=1.0),
                     one_gaussian((0.0, 0.0, 0.0), log_s=(-7, -7, -7), logit=-4.0)])   # tiny and faint
    raws = np.stack([raw.copy(), raw.copy(), raw.copy()])
    raws[0, 0, 0] = 5.0                          # frame 0: the first Gaussian is far off screen
    targets = np.stack([np.full((3, 32, 32), v) for v in (0.1, 0.5, 0.9)])
    cols, done, sums = colorinit.color_init(raws, cams, targets, np.full((2, 3), -1.0), np.zeros(2, bool))
    assert sums[0][1][0] == 0.0 and sums[1][1][0] > colorinit.DELTA
    assert done[0] and np.allclose(cols[0], 0.5)          # frame 1: the first frame that shows it
    assert sums[1][1][1] < colorinit.DELTA and not done[1] and (cols[1] == -1.0).all()
    # an initialised Gaussian keeps its colour
    cols2, done2, _ = colorinit.color_init(raws[2:], cams[2:], targets[2:], cols, done)
    assert np.array_equal(cols2, cols) and np.array_equal(done2, done)
