"""Seeded synthetic inputs for the blendshape-avatar rendering path.

This module only draws random numbers into arrays of the right shapes.  It
holds none of the method's arithmetic (no blending, projection, compositing or
optimisation), so both the GPU path and the CPU reference may consume what it
produces.

The shapes follow the paper's workloads (Sec. 4.1: 512x512 frames; Sec. A.3:
about 60k Gaussians, K = 20 blendshapes, batches of ~10 frames); the value
recipes are the synthetic stand-ins used because the captured videos, FLAME
tracks and trained avatars are not available:

* Gaussian means uniform in an ellipsoid of radii (0.08, 0.10, 0.09) around
  the origin, log-scales N(-5, 0.3), unit quaternions (w, x, y, z) from
  normalised N(0, 1)^4, opacity logits N(0, 1), RGB U[0, 1];
* blendshape deltas N(0, delta_std) on every feature (pads stay zero);
* tracking vectors: 50 expression coefficients N(0, 1) + 6 jaw/neck pose
  values N(0, 0.1);
* cameras: pinhole, fx = fy = 150 * W / 128, principal point at the image
  centre, world->camera = translate(0, 0, d) * rot_y(yaw), yaw U[-10, 10]
  degrees, d = 0.5 (or U[lo, hi]); near plane 0.2; background U[0, 1]^3.

Seeds: scene 0, cameras 1, tracking 2, targets/backgrounds 3, request stream 4.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

NFEAT = 16          # stored floats per Gaussian (14 used + 2 pad)
FEAT_USED = 14
THETA_DIM = 56      # 50 expression + 6 jaw/neck pose
MLP_HIDDEN = 256


@dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray            # (3, 3) world -> camera, row-major
    t: np.ndarray            # (3,)
    near: float = 0.2
    bg: np.ndarray = field(default_factory=lambda: np.zeros(3))

    def __post_init__(self):
        # Every camera value is a binary32 number: the renderer's interface is fp32.
        f = lambda v: float(np.float32(v))
        self.fx, self.fy, self.cx, self.cy, self.near = map(f, (self.fx, self.fy, self.cx, self.cy, self.near))
        self.R = np.asarray(self.R, dtype=np.float32).reshape(3, 3)
        self.t = np.asarray(self.t, dtype=np.float32).reshape(3)
        self.bg = np.asarray(self.bg, dtype=np.float32).reshape(3)


def make_scene(N: int, K: int, seed: int = 0, delta_std: float = 1e-3) -> np.ndarray:
    """Bases [(K+1), N, 16] float32; slice 0 is the base model, 1..K deltas."""
    rng = np.random.default_rng(seed)
    bases = np.zeros((K + 1, N, NFEAT), dtype=np.float64)
    d = rng.normal(size=(N, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = rng.uniform(size=(N, 1)) ** (1.0 / 3.0)
    bases[0, :, 0:3] = d * r * np.array([0.08, 0.10, 0.09])
    q = rng.normal(size=(N, 4))
    bases[0, :, 3:7] = q / np.linalg.norm(q, axis=1, keepdims=True)
    bases[0, :, 7:10] = rng.normal(-5.0, 0.3, size=(N, 3))
    bases[0, :, 10] = rng.normal(0.0, 1.0, size=N)
    bases[0, :, 11:14] = rng.uniform(0.0, 1.0, size=(N, 3))
    if K > 0:
        bases[1:, :, :FEAT_USED] = rng.normal(0.0, delta_std, size=(K, N, FEAT_USED))
    return bases.astype(np.float32)


def rot_y(deg: float) -> np.ndarray:
    a = np.deg2rad(deg)
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])


def make_cameras(B: int, width: int = 512, height: int = 512, seed: int = 1, yaw_deg: float = 10.0,
                 dist=(0.5, 0.5), resolutions=None, bg_seed: int = 3) -> list:
    """B cameras; `resolutions` (list of (W, H)) draws each frame's size uniformly."""
    rng = np.random.default_rng(seed)
    bg_rng = np.random.default_rng(bg_seed)
    cams = []
    for _ in range(B):
        if resolutions is not None:
            w, h = resolutions[rng.integers(len(resolutions))]
        else:
            w, h = width, height
        yaw = rng.uniform(-yaw_deg, yaw_deg) if yaw_deg > 0 else 0.0
        d = rng.uniform(dist[0], dist[1]) if dist[1] > dist[0] else dist[0]
        f = 150.0 * w / 128.0
        cams.append(Camera(width=int(w), height=int(h), fx=f, fy=f, cx=w / 2.0, cy=h / 2.0,
                           R=rot_y(yaw), t=np.array([0.0, 0.0, d]), near=0.2,
                           bg=bg_rng.uniform(0.0, 1.0, size=3)))
    return cams


def fixed_camera(width: int, height: int, fx: float, dist: float, bg=(0.0, 0.0, 0.0)) -> Camera:
    """Unrotated camera at distance `dist` (the tiny workload uses fx = 150, 128x128, z = 0.5)."""
    return Camera(width=width, height=height, fx=fx, fy=fx, cx=width / 2.0, cy=height / 2.0,
                  R=np.eye(3), t=np.array([0.0, 0.0, dist]), near=0.2, bg=np.asarray(bg, dtype=np.float64))


def make_weights(B: int, K: int, seed: int = 2) -> np.ndarray:
    return np.random.default_rng(seed).uniform(0.0, 1.0, size=(B, K)).astype(np.float32)


def make_tracking(B: int, seed: int = 2) -> np.ndarray:
    rng = np.random.default_rng(seed)
    th = np.empty((B, THETA_DIM))
    th[:, :50] = rng.normal(0.0, 1.0, size=(B, 50))
    th[:, 50:] = rng.normal(0.0, 0.1, size=(B, 6))
    return th.astype(np.float32)


def make_mlp(K: int = 20, seed: int = 5, d_in: int = THETA_DIM, hidden: int = MLP_HIDDEN) -> dict:
    """Layer weights (out, in) and biases drawn U(-1/sqrt(fan_in), 1/sqrt(fan_in))."""
    rng = np.random.default_rng(seed)
    p = {}
    dims = [(hidden, d_in), (hidden, hidden), (K, hidden)]
    for li, (o, i) in enumerate(dims, start=1):
        b = 1.0 / np.sqrt(i)
        p[f"W{li}"] = rng.uniform(-b, b, size=(o, i)).astype(np.float32)
        p[f"b{li}"] = rng.uniform(-b, b, size=(o,)).astype(np.float32)
    return p


def make_targets(cams: list, seed: int = 3) -> list:
    rng = np.random.default_rng(seed + 1000)
    return [rng.uniform(0.0, 1.0, size=(3, c.height, c.width)).astype(np.float32) for c in cams]


def perturb_scene(bases: np.ndarray, seed: int = 6, pos_std: float = 2e-3, rot_std: float = 0.05,
                  logscale_std: float = 0.1, logit_std: float = 0.3, rgb_std: float = 0.05) -> np.ndarray:
    """A starting point for fitting: the base model of `bases` with Gaussian
    noise on every attribute (deltas unchanged)."""
    rng = np.random.default_rng(seed)
    out = bases.astype(np.float64).copy()
    N = bases.shape[1]
    out[0, :, 0:3] += rng.normal(0.0, pos_std, size=(N, 3))
    out[0, :, 3:7] += rng.normal(0.0, rot_std, size=(N, 4))
    out[0, :, 7:10] += rng.normal(0.0, logscale_std, size=(N, 3))
    out[0, :, 10] += rng.normal(0.0, logit_std, size=N)
    out[0, :, 11:14] += rng.normal(0.0, rgb_std, size=(N, 3))
    return out.astype(np.float32)


def make_request_stream(n: int, rate_per_s: float, n_avatars: int, seed: int = 4):
    """Poisson arrivals: (arrival times in s, avatar ids, tracking vectors, yaw degrees)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=n)
    t = np.cumsum(gaps)
    av = rng.integers(0, n_avatars, size=n)
    th = np.empty((n, THETA_DIM), dtype=np.float32)
    th[:, :50] = rng.normal(0.0, 1.0, size=(n, 50))
    th[:, 50:] = rng.normal(0.0, 0.1, size=(n, 6))
    yaw = rng.uniform(-10.0, 10.0, size=n)
    return t, av, th, yaw


# ---------------------------------------------------------------- head mesh (tangent-space binding)
def make_head_mesh(n_lat: int = 24, n_lon: int = 48, radii=(0.08, 0.10, 0.09)):
    """A closed-cap-free ellipsoidal band mesh standing in for a tracked head
    mesh: latitude rows between the poles, quads split in two.  Returns
    (verts [V,3] f32, faces [F,3] i32, face_uv [F,3,2] f32) with UVs
    u = longitude / 2 pi (the seam column repeated at u = 1 per face) and
    v = row / (n_lat - 1)."""
    lat = np.linspace(0.15 * np.pi, 0.85 * np.pi, n_lat)
    lon = np.linspace(0.0, 2.0 * np.pi, n_lon, endpoint=False)
    th, ph = np.meshgrid(lat, lon, indexing="ij")
    verts = np.stack([np.sin(th) * np.cos(ph) * radii[0], np.cos(th) * radii[1], np.sin(th) * np.sin(ph) * radii[2]],
                     axis=-1).reshape(-1, 3)
    faces, uvs = [], []
    for i in range(n_lat - 1):
        for j in range(n_lon):
            j2 = (j + 1) % n_lon
            a, b, c, d = i * n_lon + j, i * n_lon + j2, (i + 1) * n_lon + j, (i + 1) * n_lon + j2
            ua, ub = j / n_lon, (j + 1) / n_lon
            va, vc = i / (n_lat - 1), (i + 1) / (n_lat - 1)
            faces += [(a, b, c), (b, d, c)]          # counter-clockwise seen from outside
            uvs += [((ua, va), (ub, va), (ua, vc)), ((ub, va), (ub, vc), (ua, vc))]
    return verts.astype(np.float32), np.array(faces, dtype=np.int32), np.array(uvs, dtype=np.float32)


def deform_mesh(verts: np.ndarray, B: int, seed: int = 21, amp: float = 2e-3) -> np.ndarray:
    """B per-frame deformations of the mesh: smooth displacements along the
    radial direction plus a small per-frame rotation and translation."""
    rng = np.random.default_rng(seed)
    v = np.asarray(verts, dtype=np.float64)
    out = np.zeros((B,) + v.shape)
    rad = v / np.linalg.norm(v, axis=1, keepdims=True)
    for b in range(B):
        w = rng.normal(size=3)
        w /= np.linalg.norm(w)
        disp = amp * np.sin(40.0 * v @ w + rng.uniform(0, 2 * np.pi))[:, None] * rad
        a = np.deg2rad(rng.uniform(-5, 5))
        Q = np.array([[np.cos(a), -np.sin(a), 0.0], [np.sin(a), np.cos(a), 0.0], [0.0, 0.0, 1.0]])
        out[b] = (v + disp) @ Q.T + rng.normal(0.0, 2e-3, size=3)
    return out.astype(np.float32)


def bind_gaussians(faces: np.ndarray, verts: np.ndarray, N: int, seed: int = 22):
    """Triangle (area-weighted) and uniform barycentric coordinates per Gaussian."""
    rng = np.random.default_rng(seed)
    v = np.asarray(verts, dtype=np.float64)
    e1 = v[faces[:, 1]] - v[faces[:, 0]]
    e2 = v[faces[:, 2]] - v[faces[:, 0]]
    area = 0.5 * np.linalg.norm(np.cross(e1, e2), axis=1)
    tri = rng.choice(len(faces), size=N, p=area / area.sum()).astype(np.int32)
    r1, r2 = rng.uniform(size=N), rng.uniform(size=N)
    s1 = np.sqrt(r1)
    bary = np.stack([1 - s1, s1 * (1 - r2), s1 * r2], axis=1)
    return tri, bary.astype(np.float32)


def make_tangent_scene(N: int, K: int, seed: int = 0, offset_std: float = 5e-3, delta_std: float = 1e-3):
    """Bases like make_scene, with positions as small tangent-space offsets
    (UV units along T and B, and along N) from the bound triangle's point."""
    bases = make_scene(N, K, seed=seed, delta_std=delta_std).astype(np.float64)
    rng = np.random.default_rng(seed + 100)
    bases[0, :, 0:3] = rng.normal(0.0, offset_std, size=(N, 3)) * np.array([1.0, 1.0, 0.2])
    if K > 0:
        bases[1:, :, 0:3] *= 0.5
    return bases.astype(np.float32)
