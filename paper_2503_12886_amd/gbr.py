"""ctypes binding of libgbr (include/gbr.h).

Argument marshalling only: every function here checks the tensors it is given
(device, dtype, contiguity, sizes), turns them into raw pointers and calls the
C entry point of the same name.  All computation happens in the library's HIP
kernels.  Loading fails loudly if libgbr.so has not been built: there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgbr.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "gbr.h")
_LIB = None

GBR_OK = 0
ERRORS = {-1: "GBR_ERR_INVALID_ARG", -2: "GBR_ERR_CAPACITY", -3: "GBR_ERR_OOM", -4: "GBR_ERR_HIP",
          -5: "GBR_ERR_STATE", -6: "GBR_ERR_OVERFLOW"}


class GbrError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = lib().gbr_strerror(code).decode() if _LIB is not None else str(code)
        super().__init__(f"{where}: {ERRORS.get(code, code)} ({msg})")


class gbr_camera(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("fx", ctypes.c_float),
                ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("R", ctypes.c_float * 9), ("t", ctypes.c_float * 3), ("near_z", ctypes.c_float),
                ("bg", ctypes.c_float * 3)]


class gbr_config(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("chunk", ctypes.c_int32), ("device", ctypes.c_int32),
                ("max_frames", ctypes.c_int32), ("max_splats", ctypes.c_int64), ("max_pixels", ctypes.c_int64),
                ("max_entries", ctypes.c_int64)]


class gbr_status(ctypes.Structure):
    _fields_ = [("entries", ctypes.c_int64), ("entries_capacity", ctypes.c_int64), ("overflow", ctypes.c_int32),
                ("adam_steps", ctypes.c_int32 * 4), ("loss", ctypes.c_float)]


_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_f32 = ctypes.c_float
_SIGS = {
    "gbr_strerror": ([ctypes.c_int], ctypes.c_char_p),
    "gbr_create": ([ctypes.POINTER(gbr_config), ctypes.POINTER(_vp)], ctypes.c_int),
    "gbr_destroy": ([_vp], ctypes.c_int),
    "gbr_reserve": ([_vp, _i64], ctypes.c_int),
    "gbr_set_tiling": ([_vp, _i32, _i32], ctypes.c_int),
    "gbr_memory": ([_vp, ctypes.POINTER(_i64)], ctypes.c_int),
    "gbr_plan_bytes": ([ctypes.POINTER(gbr_config), _i32, ctypes.POINTER(_i64), ctypes.POINTER(_i32),
                        ctypes.POINTER(_i32), _i64, ctypes.POINTER(_i64)], ctypes.c_int),
    "gbr_blend": ([_vp, _vp, _vp, _i32, _i32, _i64, _vp, _vp], ctypes.c_int),
    "gbr_render": ([_vp, _vp, ctypes.POINTER(_i64), ctypes.POINTER(gbr_camera), _i32, _vp, _vp], ctypes.c_int),
    "gbr_preprocess": ([_vp, _vp, ctypes.POINTER(_i64), ctypes.POINTER(gbr_camera), _i32, _vp], ctypes.c_int),
    "gbr_entry_count": ([_vp, _vp, ctypes.POINTER(_i64)], ctypes.c_int),
    "gbr_rasterize": ([_vp, _vp, _vp], ctypes.c_int),
    "gbr_render_backward": ([_vp, _vp, _vp, _vp], ctypes.c_int),
    "gbr_blend_backward": ([_vp, _vp, _vp, _vp, _i32, _i32, _i64, _vp, _vp, _i32, _vp], ctypes.c_int),
    "gbr_blend_backward_noalloc": ([_vp, _vp, _vp, _i32, _i32, _i64, _vp, _vp, _i32, _vp], ctypes.c_int),
    "gbr_backward": ([_vp, _vp, _vp, _vp, _i32, _vp, _vp, _vp], ctypes.c_int),
    "gbr_color_init": ([_vp, _vp, _vp, ctypes.c_float, _vp, _vp], ctypes.c_int),
    "gbr_tangent_frames": ([_vp, _vp, _vp, _vp, _i32, _i32, _i32, _vp, _vp], ctypes.c_int),
    "gbr_tangent_transform": ([_vp, _vp, _vp, _vp, _vp, _vp, _vp, _i32, _i64, _i32, _i32, _vp, _vp], ctypes.c_int),
    "gbr_tangent_backward": ([_vp, _vp, _vp, _vp, _i32, _i64, _i32, _vp, _vp], ctypes.c_int),
    "gbr_render_tangent": ([_vp, _vp, _vp, _vp, _vp, _vp, _vp, _i64, _i32, _i32, ctypes.POINTER(gbr_camera), _i32,
                            _vp, _vp], ctypes.c_int),
    "gbr_loss": ([_vp, _vp, _vp, _i32, _vp, _vp], ctypes.c_int),
    "gbr_mlp_forward": ([_vp, _vp, _vp, _i32, _i32, _i32, _i32, _vp, _vp], ctypes.c_int),
    "gbr_mlp_backward": ([_vp, _vp, _vp, _vp, _vp], ctypes.c_int),
    "gbr_adam_step": ([_vp, _i32, _vp, _vp, _vp, _vp, _i64, _i64, ctypes.POINTER(_f32), _f32, _f32, _f32, _vp],
                      ctypes.c_int),
    "gbr_blend_adam_step": ([_vp, _i32, _vp, _vp, _i32, _i32, _i64, _vp, _vp, _vp, ctypes.POINTER(_f32), _f32, _f32,
                             _f32, _vp], ctypes.c_int),
    "gbr_query_status": ([_vp, _vp, ctypes.POINTER(gbr_status)], ctypes.c_int),
    "gbr_status_post": ([_vp, _vp], ctypes.c_int),
    "gbr_status_posts": ([_vp, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "gbr_status_wait": ([_vp, ctypes.c_int64, ctypes.POINTER(gbr_status)], ctypes.c_int),
    "gbr_stage_frames": ([_vp, ctypes.POINTER(_i64), ctypes.POINTER(gbr_camera), _i32], ctypes.c_int),
    "gbr_graph_begin": ([_vp, _vp], ctypes.c_int),
    "gbr_graph_end": ([_vp, _vp, ctypes.POINTER(_vp)], ctypes.c_int),
    "gbr_graph_launch": ([_vp, _vp], ctypes.c_int),
    "gbr_graph_destroy": ([_vp], ctypes.c_int),
    "gbr_autotune": ([_vp, _vp, ctypes.POINTER(_i64), ctypes.POINTER(gbr_camera), _i32, _vp, _vp, _vp, _vp,
                      ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_f32)], ctypes.c_int),
    "gbr_inspect": ([_vp, _i32, _vp, ctypes.POINTER(_i64)], ctypes.c_int),
    "gbr_timing": ([_vp, _i32, _i32], ctypes.c_int),
    "gbr_timing_read": ([_vp, _i32, ctypes.POINTER(_f32)], ctypes.c_int),
    "gbr_timing_accum": ([_vp, _i32, _i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)],
                         ctypes.c_int),
}

# kernel ids of gbr_timing (GBR_K_*)
K_BLEND, K_PREPROCESS, K_BINNING, K_TILE_SORT, K_COMPOSITE_FWD, K_COMPOSITE_BWD, K_GATHER_BWD, K_BLEND_BWD, \
    K_ADAM, K_LOSS, K_MLP, K_TILE_SCAN, K_DEPTH_ORDER = range(13)
KERNEL_NAMES = ["blend", "preprocess", "binning", "tile_sort", "composite_fwd", "composite_bwd", "gather_bwd",
                "blend_bwd", "adam", "loss", "mlp", "tile_scan", "depth_order"]


def header_symbols() -> list:
    """Names of every function declared in include/gbr.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gbr_[a-z_]+)\s*\(", text)))


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _LIB = L
    return _LIB


def _check(rc: int, where: str) -> None:
    if rc != GBR_OK:
        raise GbrError(rc, where)


def _ptr(t) -> int:
    """Device pointer of a contiguous float32/int CUDA tensor."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


def _f32dev(t, name: str, numel: Optional[int] = None):
    import torch
    if t.dtype != torch.float32:
        raise ValueError(f"{name}: expected float32, got {t.dtype}")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name}: expected at least {numel} elements, got {t.numel()}")
    return _ptr(t)


def _stream(stream) -> int:
    import torch
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def cameras_c(cams: Sequence) -> "ctypes.Array":
    """Pack camera records (objects with width, height, fx, fy, cx, cy, R, t, near, bg)."""
    arr = (gbr_camera * len(cams))()
    for i, c in enumerate(cams):
        a = arr[i]
        a.width, a.height = int(c.width), int(c.height)
        a.fx, a.fy, a.cx, a.cy = float(c.fx), float(c.fy), float(c.cx), float(c.cy)
        R = np.asarray(c.R, dtype=np.float32).ravel()
        t = np.asarray(c.t, dtype=np.float32).ravel()
        bg = np.asarray(c.bg, dtype=np.float32).ravel()
        for k in range(9):
            a.R[k] = float(R[k])
        for k in range(3):
            a.t[k] = float(t[k])
            a.bg[k] = float(bg[k])
        a.near_z = float(c.near)
    return arr


def offsets_c(offsets: Sequence[int]):
    arr = (_i64 * len(offsets))()
    for i, v in enumerate(offsets):
        arr[i] = int(v)
    return arr


def image_numel(cams: Sequence) -> int:
    return int(sum(3 * int(c.width) * int(c.height) for c in cams))


def image_offsets(cams: Sequence) -> list:
    out, o = [], 0
    for c in cams:
        out.append(o)
        o += 3 * int(c.width) * int(c.height)
    return out


class Context:
    """Owns one gbr_ctx (workspace sized from the capacities)."""

    def __init__(self, tile: int = 16, chunk: int = 64, device: int = 0, max_frames: int = 64,
                 max_splats: int = 1 << 20, max_pixels: int = 1 << 22, max_entries: int = 1 << 24):
        self.cfg = gbr_config(tile, chunk, device, max_frames, max_splats, max_pixels, max_entries)
        h = _vp()
        _check(lib().gbr_create(ctypes.byref(self.cfg), ctypes.byref(h)), "gbr_create")
        self.handle = h
        self.tile, self.chunk = tile, chunk
        # forward passes started on this context (gbr_render, gbr_preprocess,
        # gbr_autotune): the state a backward reads is the latest pass's
        self.passes = 0

    def close(self) -> None:
        if getattr(self, "handle", None):
            lib().gbr_destroy(self.handle)
            self.handle = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- entry points (same names as the C ABI)
def gbr_reserve(ctx: Context, max_entries: int) -> None:
    _check(lib().gbr_reserve(ctx.handle, int(max_entries)), "gbr_reserve")


def gbr_memory(ctx: Context) -> int:
    """Device bytes the context's workspace holds now."""
    n = _i64()
    _check(lib().gbr_memory(ctx.handle, ctypes.byref(n)), "gbr_memory")
    return int(n.value)


def gbr_plan_bytes(tile: int, chunk: int, max_frames: int, max_splats: int, max_pixels: int, max_entries: int,
                   gauss_offsets, widths, heights, entries: int = 0) -> int:
    """Device bytes a context of this configuration would hold after one pass
    over frames of these Gaussian counts and sizes (host only, no GPU)."""
    cfg = gbr_config(tile, chunk, 0, max_frames, max_splats, max_pixels, max_entries)
    B = len(widths)
    w = (_i32 * B)(*[int(x) for x in widths])
    h = (_i32 * B)(*[int(x) for x in heights])
    n = _i64()
    _check(lib().gbr_plan_bytes(ctypes.byref(cfg), B, offsets_c(gauss_offsets), w, h, int(entries), ctypes.byref(n)),
           "gbr_plan_bytes")
    return int(n.value)


def gbr_set_tiling(ctx: Context, tile: int, chunk: int) -> None:
    _check(lib().gbr_set_tiling(ctx.handle, int(tile), int(chunk)), "gbr_set_tiling")
    ctx.tile, ctx.chunk = tile, chunk


def gbr_blend(ctx: Context, bases, weights, raw, stream=None) -> None:
    K1, N, F = bases.shape
    B = raw.shape[0]
    K = K1 - 1
    if F != 16 or raw.shape[1:] != (N, 16) or (K > 0 and tuple(weights.shape) != (B, K)):
        raise ValueError("gbr_blend: shape mismatch")
    _check(lib().gbr_blend(ctx.handle, _f32dev(bases, "bases"), _f32dev(weights, "weights") if K > 0 else None,
                           B, K, N, _f32dev(raw, "raw"), _stream(stream)), "gbr_blend")


def _frames(raw, gauss_offsets, cams):
    B = len(cams)
    if len(gauss_offsets) != B + 1:
        raise ValueError("gauss_offsets must have B+1 entries")
    if raw.numel() < int(gauss_offsets[-1]) * 16:
        raise ValueError("raw is smaller than gauss_offsets[-1] * 16")
    return B, offsets_c(gauss_offsets), cameras_c(cams)


def gbr_render(ctx: Context, raw, gauss_offsets, cams, images, stream=None) -> None:
    B, off, cc = _frames(raw, gauss_offsets, cams)
    _f32dev(images, "images", image_numel(cams))
    ctx.passes += 1
    _check(lib().gbr_render(ctx.handle, _f32dev(raw, "raw"), off, cc, B, _ptr(images), _stream(stream)),
           "gbr_render")


def gbr_preprocess(ctx: Context, raw, gauss_offsets, cams, stream=None) -> None:
    B, off, cc = _frames(raw, gauss_offsets, cams)
    ctx.passes += 1
    _check(lib().gbr_preprocess(ctx.handle, _f32dev(raw, "raw"), off, cc, B, _stream(stream)), "gbr_preprocess")


def gbr_entry_count(ctx: Context, stream=None) -> int:
    e = _i64()
    _check(lib().gbr_entry_count(ctx.handle, _stream(stream), ctypes.byref(e)), "gbr_entry_count")
    return int(e.value)


def gbr_rasterize(ctx: Context, images, stream=None) -> None:
    _check(lib().gbr_rasterize(ctx.handle, _f32dev(images, "images"), _stream(stream)), "gbr_rasterize")


def gbr_render_backward(ctx: Context, dimages, draw, stream=None) -> None:
    _check(lib().gbr_render_backward(ctx.handle, _f32dev(dimages, "dimages"), _f32dev(draw, "draw"),
                                     _stream(stream)), "gbr_render_backward")


def gbr_blend_backward(ctx: Context, draw, bases, weights, dbases, dweights, accumulate: bool = False,
                       stream=None) -> None:
    """dbases may be None: only dweights is formed."""
    K1, N, _ = bases.shape
    K = K1 - 1
    B = draw.shape[0]
    _check(lib().gbr_blend_backward(ctx.handle, _f32dev(draw, "draw"), _f32dev(bases, "bases"),
                                    _f32dev(weights, "weights") if K > 0 else None, B, K, N,
                                    _f32dev(dbases, "dbases") if dbases is not None else None,
                                    _f32dev(dweights, "dweights") if K > 0 else None,
                                    int(bool(accumulate)), _stream(stream)), "gbr_blend_backward")


def gbr_blend_backward_noalloc(draw, bases, weights, dbases, dweights, accumulate: bool = False,
                               stream=None) -> None:
    """gbr_blend_backward without a context and without allocating (see
    include/gbr.h); dbases may be None."""
    K1, N, _ = bases.shape
    K = K1 - 1
    B = draw.shape[0]
    _check(lib().gbr_blend_backward_noalloc(_f32dev(draw, "draw"), _f32dev(bases, "bases"),
                                            _f32dev(weights, "weights") if K > 0 else None, B, K, N,
                                            _f32dev(dbases, "dbases") if dbases is not None else None,
                                            _f32dev(dweights, "dweights") if K > 0 else None,
                                            int(bool(accumulate)), _stream(stream)), "gbr_blend_backward_noalloc")


def gbr_blend_adam_step(ctx: Context, group: int, draw, weights, bases, m, v, lr_table: Sequence[float],
                        beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-15, stream=None) -> None:
    """Adam on bases [(K+1)][N][16] with the blend adjoint of draw [B][N][16] as the gradient."""
    K1, N, _ = bases.shape
    K = K1 - 1
    B = draw.shape[0]
    for t, nm in ((m, "m"), (v, "v")):
        if t.numel() != bases.numel():
            raise ValueError(f"gbr_blend_adam_step: {nm} size mismatch")
    tab = (_f32 * 32)(*[float(x) for x in lr_table])
    _check(lib().gbr_blend_adam_step(ctx.handle, int(group), _f32dev(draw, "draw"),
                                     _f32dev(weights, "weights") if K > 0 else None, B, K, N,
                                     _f32dev(bases, "bases"), _f32dev(m, "m"), _f32dev(v, "v"), tab, beta1, beta2,
                                     eps, _stream(stream)), "gbr_blend_adam_step")


def gbr_backward(ctx: Context, dimages, bases, weights, dbases, dweights, stream=None) -> None:
    K = bases.shape[0] - 1
    _check(lib().gbr_backward(ctx.handle, _f32dev(dimages, "dimages"), _f32dev(bases, "bases"),
                              _f32dev(weights, "weights") if K > 0 else None, K,
                              _f32dev(dbases, "dbases") if dbases is not None else None,
                              _f32dev(dweights, "dweights") if K > 0 else None, _stream(stream)), "gbr_backward")


def _i32dev(t, name: str):
    import torch
    if t.dtype != torch.int32:
        raise ValueError(f"{name}: expected int32, got {t.dtype}")
    return _ptr(t)


def gbr_tangent_frames(ctx: Context, verts, faces, face_uv, frames, stream=None) -> None:
    """verts [B][V][3], faces [F][3] int32, face_uv [F][3][2] -> frames [B][F][16] (device tensors)."""
    B, V, _ = verts.shape
    F = faces.shape[0]
    _check(lib().gbr_tangent_frames(ctx.handle, _f32dev(verts, "verts"), _i32dev(faces, "faces"),
                                    _f32dev(face_uv, "face_uv"), B, V, F, _f32dev(frames, "frames", B * F * 16),
                                    _stream(stream)), "gbr_tangent_frames")


def gbr_tangent_transform(ctx: Context, raw_t, tri, bary, verts, faces, frames, raw_d, stream=None) -> None:
    """raw_t [B][N][16] tangent-space Gaussians -> raw_d [B][N][16] deformed-space ones."""
    B, N, _ = raw_t.shape
    V, F = verts.shape[1], faces.shape[0]
    _check(lib().gbr_tangent_transform(ctx.handle, _f32dev(raw_t, "raw_t"), _i32dev(tri, "tri"),
                                       _f32dev(bary, "bary"), _f32dev(verts, "verts"), _i32dev(faces, "faces"),
                                       _f32dev(frames, "frames"), B, N, V, F, _f32dev(raw_d, "raw_d", B * N * 16),
                                       _stream(stream)), "gbr_tangent_transform")


def gbr_tangent_backward(ctx: Context, draw_d, tri, frames, draw_t, stream=None) -> None:
    """dL/draw_d [B][N][16] -> dL/draw_t [B][N][16]."""
    B, N, _ = draw_d.shape
    F = frames.shape[1]
    _check(lib().gbr_tangent_backward(ctx.handle, _f32dev(draw_d, "draw_d"), _i32dev(tri, "tri"),
                                      _f32dev(frames, "frames"), B, N, F, _f32dev(draw_t, "draw_t", B * N * 16),
                                      _stream(stream)), "gbr_tangent_backward")


def gbr_render_tangent(ctx: Context, raw_t, tri, bary, verts, faces, frames, cams, images, stream=None) -> None:
    """gbr_render of tangent-space Gaussians raw_t [B][N][16], carried to
    each frame's mesh (verts [B][V][3]) inside the pass; the backward then
    returns tangent-space gradients."""
    B, N, _ = raw_t.shape
    if len(cams) != B or verts.shape[0] != B or frames.shape[0] != B:
        raise ValueError("gbr_render_tangent: one camera, mesh and frame table per frame")
    V, F = verts.shape[1], faces.shape[0]
    _f32dev(images, "images", image_numel(cams))
    ctx.passes += 1
    _check(lib().gbr_render_tangent(ctx.handle, _f32dev(raw_t, "raw_t"), _i32dev(tri, "tri"), _f32dev(bary, "bary"),
                                    _f32dev(verts, "verts"), _i32dev(faces, "faces"),
                                    _f32dev(frames, "frames", B * F * 16), N, V, F, cameras_c(cams), B, _ptr(images),
                                    _stream(stream)), "gbr_render_tangent")


def gbr_color_init(ctx: Context, targets, bases, done, delta: float = 0.1, stream=None) -> None:
    """Eq. 3 colour initialisation after a render (see include/gbr.h); done is a
    device uint8 tensor [N], updated in place, as are the base colours."""
    import torch
    if done.dtype != torch.uint8 or not done.is_cuda or not done.is_contiguous():
        raise ValueError("done must be a contiguous uint8 device tensor")
    _check(lib().gbr_color_init(ctx.handle, _f32dev(targets, "targets"), _f32dev(bases, "bases"), float(delta),
                                _ptr(done), _stream(stream)), "gbr_color_init")


def gbr_loss(ctx: Context, images, targets, kind: int, dimages, stream=None) -> None:
    _check(lib().gbr_loss(ctx.handle, _f32dev(images, "images"), _f32dev(targets, "targets"), int(kind),
                          _f32dev(dimages, "dimages"), _stream(stream)), "gbr_loss")


def gbr_mlp_forward(ctx: Context, params, theta, d_in: int, hidden: int, K: int, psi, stream=None) -> None:
    B = theta.shape[0]
    n = hidden * d_in + hidden + hidden * hidden + hidden + K * hidden + K
    _check(lib().gbr_mlp_forward(ctx.handle, _f32dev(params, "params", n), _f32dev(theta, "theta", B * d_in), B,
                                 d_in, hidden, K, _f32dev(psi, "psi", B * K), _stream(stream)), "gbr_mlp_forward")


def gbr_mlp_backward(ctx: Context, params, dpsi, dparams, stream=None) -> None:
    _check(lib().gbr_mlp_backward(ctx.handle, _f32dev(params, "params"), _f32dev(dpsi, "dpsi"),
                                  _f32dev(dparams, "dparams"), _stream(stream)), "gbr_mlp_backward")


def gbr_adam_step(ctx: Context, group: int, params, grads, m, v, split: int, lr_table: Sequence[float],
                  beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-15, stream=None) -> None:
    n = params.numel()
    for t, nm in ((grads, "grads"), (m, "m"), (v, "v")):
        if t.numel() != n:
            raise ValueError(f"gbr_adam_step: {nm} size mismatch")
    tab = (_f32 * 32)(*[float(x) for x in lr_table])
    _check(lib().gbr_adam_step(ctx.handle, int(group), _f32dev(params, "params"), _f32dev(grads, "grads"),
                               _f32dev(m, "m"), _f32dev(v, "v"), n, int(split), tab, beta1, beta2, eps,
                               _stream(stream)), "gbr_adam_step")


def gbr_query_status(ctx: Context, stream=None) -> gbr_status:
    st = gbr_status()
    _check(lib().gbr_query_status(ctx.handle, _stream(stream), ctypes.byref(st)), "gbr_query_status")
    return st


def gbr_status_post(ctx: Context, stream=None) -> None:
    _check(lib().gbr_status_post(ctx.handle, _stream(stream)), "gbr_status_post")


def gbr_status_posts(ctx: Context) -> int:
    n = ctypes.c_int64()
    _check(lib().gbr_status_posts(ctx.handle, ctypes.byref(n)), "gbr_status_posts")
    return int(n.value)


def gbr_status_wait(ctx: Context, n: int) -> gbr_status:
    st = gbr_status()
    _check(lib().gbr_status_wait(ctx.handle, int(n), ctypes.byref(st)), "gbr_status_wait")
    return st


def gbr_stage_frames(ctx: Context, gauss_offsets, cams) -> None:
    _check(lib().gbr_stage_frames(ctx.handle, offsets_c(gauss_offsets), cameras_c(cams), len(cams)),
           "gbr_stage_frames")


def gbr_graph_begin(ctx: Context, stream=None) -> None:
    _check(lib().gbr_graph_begin(ctx.handle, _stream(stream)), "gbr_graph_begin")


def gbr_graph_end(ctx: Context, stream=None):
    g = _vp()
    _check(lib().gbr_graph_end(ctx.handle, _stream(stream), ctypes.byref(g)), "gbr_graph_end")
    return g


def gbr_graph_launch(graph, stream=None) -> None:
    _check(lib().gbr_graph_launch(graph, _stream(stream)), "gbr_graph_launch")


def gbr_graph_destroy(graph) -> None:
    _check(lib().gbr_graph_destroy(graph), "gbr_graph_destroy")


def gbr_autotune(ctx: Context, raw, gauss_offsets, cams, images, dimages, draw, stream=None):
    B, off, cc = _frames(raw, gauss_offsets, cams)
    bt, bc = _i32(), _i32()
    times = (_f32 * 9)()
    ctx.passes += 1
    _check(lib().gbr_autotune(ctx.handle, _f32dev(raw, "raw"), off, cc, B, _f32dev(images, "images"),
                              _f32dev(dimages, "dimages"), _f32dev(draw, "draw"), _stream(stream), ctypes.byref(bt),
                              ctypes.byref(bc), times), "gbr_autotune")
    ctx.tile, ctx.chunk = bt.value, bc.value
    return bt.value, bc.value, list(times)


INSPECT = {"records": (1, np.float32, 12), "rects": (2, np.int32, 4), "tile_start": (3, np.uint32, 1),
           "sorted": (4, np.uint32, 1), "n_iter": (5, np.uint32, 1), "t_final": (6, np.float32, 1),
           "tile_last": (7, np.uint32, 1), "n_contrib": (8, np.uint32, 1), "cmask": (9, np.uint8, 1),
           "sorted_pass": (10, np.uint32, 1), "quad_last": (11, np.uint32, 4)}


def gbr_timing(ctx: Context, which: int, enable: bool) -> None:
    _check(lib().gbr_timing(ctx.handle, int(which), int(bool(enable))), "gbr_timing")


def gbr_timing_read(ctx: Context, which: int) -> float:
    ms = _f32()
    _check(lib().gbr_timing_read(ctx.handle, int(which), ctypes.byref(ms)), "gbr_timing_read")
    return float(ms.value)


def gbr_timing_accum(ctx: Context, which: int, reset: bool = False) -> tuple:
    """(total ms, launches) of one kernel accumulated on the device since its
    timing was enabled (or last reset); counts graph replays too."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(lib().gbr_timing_accum(ctx.handle, int(which), int(bool(reset)), ctypes.byref(ms), ctypes.byref(n)),
           "gbr_timing_accum")
    return float(ms.value), int(n.value)


def gbr_inspect(ctx: Context, what: str, count: int) -> np.ndarray:
    """Copy an internal buffer of the last pass to the host (count = rows)."""
    code, dt, width = INSPECT[what]
    out = np.zeros(max(count, 1) * width, dtype=dt)
    nb = _i64(out.nbytes)
    _check(lib().gbr_inspect(ctx.handle, code, out.ctypes.data_as(_vp), ctypes.byref(nb)), "gbr_inspect")
    n = nb.value // out.itemsize
    out = out[:n]
    return out.reshape(-1, width) if width > 1 else out
