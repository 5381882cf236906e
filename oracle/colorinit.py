"""Float64 reference for the colour initialisation of Eq. 3 (Sec. 3.1,
"Initialization").

TEST INFRASTRUCTURE ONLY (see the package docstring).

A Gaussian's initial colour is the splatting-weight average of the observed
pixel colours, c = sum_p w_p I_p / sum_p w_p, where w_p is the weight with
which the Gaussian enters pixel p's composite (alpha times the transmittance
in front of it).  It is applied once per Gaussian, the first time its total
weight sum_p w_p exceeds delta = 0.1; less visible Gaussians wait.

Readings:
* the visibility test compares the Gaussian's total weight over the frame
  (the denominator of Eq. 3) with delta;
* within a batch the first frame (lowest index) that passes the test
  provides the colour;
* the colour written is the base model's (G_0's colour features), whose
  blendshape deltas start at zero.

The sums are the adjoint of the colour attributes with the target image as
the cotangent: d out_p / d c = w_p per channel, so the renderer reference's
colour gradient under dL/dout = I gives sum_p w_p I_p, and under
dL/dout = 1 gives sum_p w_p.
"""
from __future__ import annotations

import numpy as np

from . import raster

DELTA = 0.1


def frame_color_sums(raw, cam, target):
    """One frame: (sum_p w_p I_p [N, 3], sum_p w_p [N]) in float64."""
    target = np.asarray(target, dtype=np.float64).reshape(3, cam.height, cam.width)
    d_i, _ = raster.render_grad(raw, cam, target)
    d_1, _ = raster.render_grad(raw, cam, np.ones_like(target))
    return d_i[:, 11:14], d_1[:, 11]


def color_init(raws, cams, targets, colors, done, delta: float = DELTA):
    """raws [B][N][16] (the batch's blended Gaussians), targets [B][3][H][W],
    colors [N][3] (G_0's colours), done [N] bool -> (colors, done, sums) with
    the not-yet-initialised Gaussians of sufficient weight set from the first
    frame that shows them; sums = per frame (wI [N, 3], w [N])."""
    colors = np.array(colors, dtype=np.float64, copy=True)
    done = np.array(done, dtype=bool, copy=True)
    sums = [frame_color_sums(raws[b], cams[b], targets[b]) for b in range(len(cams))]
    for n in range(colors.shape[0]):
        if done[n]:
            continue
        for wi, w in sums:
            if w[n] > delta:
                colors[n] = wi[n] / w[n]
                done[n] = True
                break
    return colors, done, sums
