"""ctypes front end of the double-precision renderer reference (gs_ref.c),
plus the tile binning / ordering reference.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Binning reference (Sec. 3.2: the rasterize stage's memory depends on the
per-tile lists that preprocess produces).  A projected Gaussian covers the
pixels whose centres lie in the axis-aligned box of its alpha >= 1/255
ellipse (plus a 0.01 px pad); it is listed in every T x T tile that box
meets.  Entries are emitted frame by frame, Gaussian by Gaussian, tiles in
row-major order, and then stably ordered by (global tile, binary32 depth):
equal depths keep Gaussian index order.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

NPROJ = 24
PROJ_FIELDS = ["valid", "mx", "my", "S00", "S01", "S11", "A", "B", "C", "depth", "key", "opacity",
               "r", "g", "b", "px0", "px1", "py0", "py1", "ex", "ey", "tx", "ty", "tz"]


def build(force: bool = False) -> str:
    """Compile gs_ref.c into liboracle (gcc, -ffp-contract=off)."""
    src = os.path.join(_HERE, "gs_ref.c")
    out = os.path.join(_HERE, "libgs_ref.so")
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        import subprocess
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared", src,
                               "-o", out, "-lm"])
    return out


def _lib():
    global _LIB
    if _LIB is None:
        path = build()
        lib = ctypes.CDLL(path)
        d = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.c_int64
        lib.oracle_project.argtypes = [i64, d, d, ctypes.c_int, ctypes.c_int, d]
        lib.oracle_render.argtypes = [i64, d, d, ctypes.c_int, ctypes.c_int, d, d,
                                      ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_uint8),
                                      ctypes.c_double, ctypes.c_double]
        lib.oracle_render_grad.argtypes = [i64, d, d, ctypes.c_int, ctypes.c_int, d, d, d, d]
        lib.oracle_project_adjoint.argtypes = [i64, d, d, ctypes.c_int, ctypes.c_int, d, d]
        lib.oracle_alpha_bounds.argtypes = [i64, d, d, ctypes.c_int, ctypes.c_int, i64,
                                            ctypes.POINTER(ctypes.c_int64), d, d, d, d]
        lib.oracle_contributors.argtypes = [i64, d, d, ctypes.c_int, ctypes.c_int, ctypes.c_int32,
                                            ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32)]
        _LIB = lib
    return _LIB


def _ptr(a, ct=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def cam_record(cam) -> np.ndarray:
    """fx fy cx cy R[9] t[3] near bg[3] as float64 (values are binary32 numbers)."""
    return np.concatenate([[cam.fx, cam.fy, cam.cx, cam.cy], np.asarray(cam.R, np.float64).ravel(),
                           np.asarray(cam.t, np.float64).ravel(), [cam.near],
                           np.asarray(cam.bg, np.float64).ravel()]).astype(np.float64)


def _raw64(raw):
    r = np.ascontiguousarray(np.asarray(raw, dtype=np.float64))
    assert r.ndim == 2 and r.shape[1] == 16, r.shape
    return r


def project(raw, cam) -> dict:
    """Per-Gaussian projection of one frame: dict of float64 arrays (PROJ_FIELDS)."""
    r = _raw64(raw)
    N = r.shape[0]
    out = np.zeros((max(N, 1), NPROJ))
    c = cam_record(cam)
    _lib().oracle_project(N, _ptr(r), _ptr(c), cam.width, cam.height, _ptr(out))
    out = out[:N]
    return {k: out[:, i] for i, k in enumerate(PROJ_FIELDS)}


# Ambiguity margins.  By default (None) each decision's margin is the
# first-order bound on a binary32 implementation's error for that very
# decision, per entry for alpha and accumulated per pixel for the
# transmittance (derivation in gs_ref.c, "ambiguity margins").  Fixed relative
# margins can be given instead (e.g. 1e-5 for both).


def render(raw, cam, eps_a: float | None = None, eps_t: float | None = None):
    """-> image [3, H, W], T_end [H, W], n_contrib [H, W], flags [H, W] (uint8 bits:
    1 alpha near 1/255, 2 transmittance stop near 1e-4, 4 alpha near 0.99)."""
    if (eps_a is None) != (eps_t is None):
        raise ValueError("give both fixed margins or neither")
    if eps_a is None:
        eps_a, eps_t = -1.0, -1.0
    r = _raw64(raw)
    H, W = cam.height, cam.width
    img = np.zeros((3, H, W))
    Te = np.zeros((H, W))
    nc = np.zeros((H, W), dtype=np.int32)
    fl = np.zeros((H, W), dtype=np.uint8)
    c = cam_record(cam)
    rc = _lib().oracle_render(r.shape[0], _ptr(r), _ptr(c), W, H, _ptr(img), _ptr(Te),
                              _ptr(nc, ctypes.c_int32), _ptr(fl, ctypes.c_uint8), eps_a, eps_t)
    if rc != 0:
        raise MemoryError("oracle_render failed")
    return img, Te, nc, fl


def render_grad(raw, cam, dimage):
    """dL/dimage [3, H, W] -> (draw [N, 16], dproj [N, 9]) with dproj columns
    (mx, my, Q00, Q01, Q11, opacity, r, g, b); Q01 is the coefficient B of
    q = Q00 dx^2 + 2 B dx dy + Q11 dy^2."""
    r = _raw64(raw)
    N = r.shape[0]
    g = np.ascontiguousarray(np.asarray(dimage, dtype=np.float64))
    assert g.shape == (3, cam.height, cam.width)
    draw = np.zeros((max(N, 1), 16))
    dproj = np.zeros((max(N, 1), 9))
    c = cam_record(cam)
    rc = _lib().oracle_render_grad(N, _ptr(r), _ptr(c), cam.width, cam.height, _ptr(g), _ptr(draw), _ptr(dproj),
                                   None)
    if rc != 0:
        raise MemoryError("oracle_render_grad failed")
    return draw[:N], dproj[:N]


def project_adjoint(raw, cam, dproj):
    """The projection's adjoint alone: dproj [N, 9] (columns as render_grad
    returns them) -> draw [N, 16]."""
    r = _raw64(raw)
    N = r.shape[0]
    dp = np.ascontiguousarray(np.asarray(dproj, dtype=np.float64).reshape(N, 9))
    draw = np.zeros((max(N, 1), 16))
    c = cam_record(cam)
    _lib().oracle_project_adjoint(N, _ptr(r), _ptr(c), cam.width, cam.height, _ptr(dp), _ptr(draw))
    return draw[:N]


def adjoint_magnitude(raw, cam, dimage):
    """Per Gaussian and blended feature, the magnitude that its gradient is
    summed from: the sum over pixels of the magnitudes of the per-pixel terms
    of each projected-quantity gradient, carried to the blended features
    through the magnitudes of the projection adjoint's coefficients,
    sum_c |d raw_f / d proj_c| * sum_p |term_{p,c}|  -> [N, 16]."""
    r = _raw64(raw)
    N = r.shape[0]
    g = np.ascontiguousarray(np.asarray(dimage, dtype=np.float64))
    draw = np.zeros((max(N, 1), 16))
    dproj = np.zeros((max(N, 1), 9))
    mag = np.zeros((max(N, 1), 9))
    c = cam_record(cam)
    rc = _lib().oracle_render_grad(N, _ptr(r), _ptr(c), cam.width, cam.height, _ptr(g), _ptr(draw), _ptr(dproj),
                                   _ptr(mag))
    if rc != 0:
        raise MemoryError("oracle_render_grad failed")
    out = np.zeros((N, 16))
    for k in range(9):
        e = np.zeros((N, 9))
        e[:, k] = 1.0
        out += np.abs(project_adjoint(r, cam, e)) * mag[:N, k:k + 1]
    return out


def alpha_bounds(raw, cam, gidx, px, py):
    """Unclamped alpha of Gaussian gidx[m] at (px[m], py[m]) and the bound on
    the relative error of a binary32 evaluation of it that the ambiguity
    margins use -> (alpha [M], rel_bound [M])."""
    r = _raw64(raw)
    g = np.ascontiguousarray(np.asarray(gidx, dtype=np.int64))
    x = np.ascontiguousarray(np.asarray(px, dtype=np.float64))
    y = np.ascontiguousarray(np.asarray(py, dtype=np.float64))
    M = g.shape[0]
    a = np.zeros(max(M, 1))
    e = np.zeros(max(M, 1))
    c = cam_record(cam)
    rc = _lib().oracle_alpha_bounds(r.shape[0], _ptr(r), _ptr(c), cam.width, cam.height, M,
                                    _ptr(g, ctypes.c_int64), _ptr(x), _ptr(y), _ptr(a), _ptr(e))
    if rc != 0:
        raise IndexError("Gaussian index out of range")
    return a[:M], e[:M]


def contributors(raw, cam, cap: int = 4096):
    """Per-pixel contributor index lists in compositing order -> (lists [H, W, cap], counts [H, W])."""
    r = _raw64(raw)
    H, W = cam.height, cam.width
    lists = np.full((H, W, cap), -1, dtype=np.int64)
    cnt = np.zeros((H, W), dtype=np.int32)
    c = cam_record(cam)
    over = _lib().oracle_contributors(r.shape[0], _ptr(r), _ptr(c), W, H, cap, _ptr(lists, ctypes.c_int64),
                                      _ptr(cnt, ctypes.c_int32))
    if over:
        raise ValueError("contributor cap exceeded")
    return lists, cnt


def tile_rects(proj: dict, width: int, height: int, tile: int):
    """Per Gaussian inclusive tile rect (tx0, ty0, tx1, ty1) from the pixel box; -1 rows where culled."""
    valid = proj["valid"] > 0
    rect = np.full((valid.shape[0], 4), -1, dtype=np.int64)
    rect[valid, 0] = proj["px0"][valid].astype(np.int64) // tile
    rect[valid, 1] = proj["py0"][valid].astype(np.int64) // tile
    rect[valid, 2] = proj["px1"][valid].astype(np.int64) // tile
    rect[valid, 3] = proj["py1"][valid].astype(np.int64) // tile
    return rect


def bin_and_sort(projs: list, cams: list, tile: int):
    """Tile lists of a batch of frames.

    projs[b] is ``project`` of frame b.  Returns (ranges [n_tiles, 2] int64 of
    [start, end) into the sorted list, sorted_frame [P], sorted_gauss [P],
    tile_base [B+1]).  Tiles are numbered frame by frame, row-major within a
    frame (ceil(W/T) x ceil(H/T) per frame).
    """
    tile_base = [0]
    tiles, keys, frames, gauss = [], [], [], []
    for b, (p, cam) in enumerate(zip(projs, cams)):
        ntx = -(-cam.width // tile)
        nty = -(-cam.height // tile)
        rect = tile_rects(p, cam.width, cam.height, tile)
        key = p["key"].astype(np.float32)
        for n in np.nonzero(p["valid"] > 0)[0]:
            tx0, ty0, tx1, ty1 = rect[n]
            for ty in range(ty0, ty1 + 1):
                for tx in range(tx0, tx1 + 1):
                    tiles.append(tile_base[-1] + ty * ntx + tx)
                    keys.append(key[n])
                    frames.append(b)
                    gauss.append(n)
        tile_base.append(tile_base[-1] + ntx * nty)
    tiles = np.asarray(tiles, dtype=np.int64)
    keys = np.asarray(keys, dtype=np.float32)
    frames = np.asarray(frames, dtype=np.int64)
    gauss = np.asarray(gauss, dtype=np.int64)
    order = np.lexsort((keys, tiles))          # stable: equal (tile, depth) keep emission order
    st = tiles[order]
    n_tiles = tile_base[-1]
    starts = np.searchsorted(st, np.arange(n_tiles), side="left")
    ends = np.searchsorted(st, np.arange(n_tiles), side="right")
    return np.stack([starts, ends], axis=1), frames[order], gauss[order], np.asarray(tile_base)
