"""Float64 reference for blending, the weight MLP, losses and Adam.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Each function is the plain definition from the paper:

* blend: G^psi = G_0 + sum_k psi_k dG_k (Eq. 1), summed in k order;
* blend adjoint: dG_0 = sum_b draw_b, dG_k = sum_b psi[b,k] draw_b,
  dpsi[b,k] = <dG_k, draw_b>;
* MLP psi = F(theta) (Eq. 2): three linear layers, ReLU between them, linear
  output (the paper names a three-layer MLP, Sec. A.3, and leaves the
  activation open: ReLU is a reading of it);
* L1 colour loss (Sec. 3.2, "Loss Function") and an L2 variant, both as
  means over every channel of every pixel of every frame;
* Adam (Sec. A.3) with bias correction, one learning rate per parameter.
"""
from __future__ import annotations

import numpy as np


def blend(bases: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """bases [(K+1), N, F], psi [B, K] -> raw [B, N, F] (float64)."""
    bases = np.asarray(bases, dtype=np.float64)
    psi = np.asarray(psi, dtype=np.float64)
    B, K = psi.shape
    out = np.empty((B,) + bases.shape[1:], dtype=np.float64)
    for b in range(B):
        acc = bases[0].copy()
        for k in range(K):
            acc += psi[b, k] * bases[k + 1]
        out[b] = acc
    return out


def blend_adjoint(draw: np.ndarray, bases: np.ndarray, psi: np.ndarray):
    """draw [B, N, F] -> (dbases [(K+1), N, F], dpsi [B, K])."""
    draw = np.asarray(draw, dtype=np.float64)
    bases = np.asarray(bases, dtype=np.float64)
    psi = np.asarray(psi, dtype=np.float64)
    B, K = psi.shape
    dbases = np.zeros_like(bases)
    dbases[0] = draw.sum(axis=0)
    for k in range(K):
        dbases[k + 1] = np.tensordot(psi[:, k], draw, axes=(0, 0))
    dpsi = np.einsum("knf,bnf->bk", bases[1:], draw)
    return dbases, dpsi


def mlp_forward(params: dict, theta: np.ndarray):
    """theta [B, H] -> psi [B, K], cache for the backward pass."""
    x = np.asarray(theta, dtype=np.float64)
    W1, b1, W2, b2, W3, b3 = (np.asarray(params[k], dtype=np.float64) for k in ("W1", "b1", "W2", "b2", "W3", "b3"))
    z1 = x @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    psi = h2 @ W3.T + b3
    return psi, (x, z1, h1, z2, h2)


def mlp_backward(params: dict, cache, dpsi: np.ndarray) -> dict:
    x, z1, h1, z2, h2 = cache
    W2, W3 = (np.asarray(params[k], dtype=np.float64) for k in ("W2", "W3"))
    g = np.asarray(dpsi, dtype=np.float64)
    grads = {"W3": g.T @ h2, "b3": g.sum(axis=0)}
    dh2 = g @ W3
    dz2 = dh2 * (z2 > 0.0)
    grads["W2"] = dz2.T @ h1
    grads["b2"] = dz2.sum(axis=0)
    dh1 = dz2 @ W2
    dz1 = dh1 * (z1 > 0.0)
    grads["W1"] = dz1.T @ x
    grads["b1"] = dz1.sum(axis=0)
    return grads


def loss_l2(images, targets):
    """Mean squared error over all channels/pixels/frames -> (loss, dL/dimages)."""
    n = sum(np.asarray(i).size for i in images)
    loss = 0.0
    grads = []
    for im, tg in zip(images, targets):
        d = np.asarray(im, dtype=np.float64) - np.asarray(tg, dtype=np.float64)
        loss += float((d * d).sum())
        grads.append(2.0 * d / n)
    return loss / n, grads


def loss_l1(images, targets):
    """Mean absolute error -> (loss, dL/dimages); the derivative of |0| is taken as 0."""
    n = sum(np.asarray(i).size for i in images)
    loss = 0.0
    grads = []
    for im, tg in zip(images, targets):
        d = np.asarray(im, dtype=np.float64) - np.asarray(tg, dtype=np.float64)
        loss += float(np.abs(d).sum())
        grads.append(np.sign(d) / n)
    return loss / n, grads


def adam_step(p, g, m, v, step: int, lr, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-15):
    """One Adam update at 1-based `step`; `lr` may be an array broadcast against p."""
    p = np.asarray(p, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    p = p - lr * mhat / (np.sqrt(vhat) + eps)
    return p, m, v


# Per-feature learning rates of the base model and the blendshape deltas
# (Sec. A.3): position 8e-4, opacity 0.25, scale 0.025, rotation 5e-3,
# colour 0.0125; the deltas of position, rotation and colour use 0.05, 0.5
# and 0.5 of those.  The paper blends neither opacity nor scale; where this
# build does blend them (all 14 features), the delta rates equal the base ones.
BASE_LR = {"pos": 8e-4, "rot": 5e-3, "scale": 0.025, "opacity": 0.25, "color": 0.0125}
DELTA_SCALE = {"pos": 0.05, "rot": 0.5, "scale": 1.0, "opacity": 1.0, "color": 0.5}
FEATURE_GROUP = ["pos"] * 3 + ["rot"] * 4 + ["scale"] * 3 + ["opacity"] + ["color"] * 3
MLP_LR = 1e-3


def feature_lrs(K: int, nfeat: int = 16) -> np.ndarray:
    """[(K+1), nfeat] learning rate of every stored feature of every slice (pads 0)."""
    lr = np.zeros((K + 1, nfeat))
    for f, grp in enumerate(FEATURE_GROUP):
        lr[0, f] = BASE_LR[grp]
        lr[1:, f] = BASE_LR[grp] * DELTA_SCALE[grp]
    return lr
