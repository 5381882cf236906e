"""Helpers shared by the GPU tests: tensor upload, running the library on a
batch, and the oracle-side comparison rules."""
from __future__ import annotations

import numpy as np

from paper_2503_12886_amd import gbr, synth

IMAGE_TOL = 1e-4        # max-abs image error against the float64 reference
GRAD_RTOL = 1e-3        # relative gradient error (per tensor, and per entry above a floor)


def dev(a, dtype=None):
    import torch
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda().contiguous()


def host(t) -> np.ndarray:
    return t.detach().cpu().numpy()


def make_ctx(tile=16, chunk=128, max_frames=64, max_splats=1 << 20, max_pixels=1 << 22, max_entries=1 << 24):
    return gbr.Context(tile=tile, chunk=chunk, max_frames=max_frames, max_splats=max_splats,
                       max_pixels=max_pixels, max_entries=max_entries)


def render(ctx, raw_np, cams, gauss_offsets=None):
    """Render packed raw [S,16] for the given cameras; returns (images list, raw tensor, images tensor)."""
    import torch
    raw = dev(raw_np.astype(np.float32))
    if gauss_offsets is None:
        n = raw_np.shape[0] // len(cams)
        gauss_offsets = [b * n for b in range(len(cams) + 1)]
    images = torch.empty(gbr.image_numel(cams), device="cuda", dtype=torch.float32)
    gbr.gbr_render(ctx, raw, gauss_offsets, cams, images)
    torch.cuda.synchronize()
    st = gbr.gbr_query_status(ctx)
    if st.overflow:
        gbr.gbr_reserve(ctx, st.entries + st.entries // 4 + 1024)
        gbr.gbr_render(ctx, raw, gauss_offsets, cams, images)
        torch.cuda.synchronize()
    return split_images(host(images), cams), raw, images


def split_images(flat: np.ndarray, cams) -> list:
    out, o = [], 0
    for c in cams:
        n = 3 * c.width * c.height
        out.append(flat[o:o + n].reshape(3, c.height, c.width))
        o += n
    return out


def pack_images(imgs) -> np.ndarray:
    return np.concatenate([np.asarray(i, dtype=np.float32).ravel() for i in imgs])


def compare_image(gpu_img, ref_img, flags, tol=IMAGE_TOL):
    """Max-abs error on pixels whose threshold decisions are not within the
    reference's ambiguity margins; returns (max_err, masked_fraction)."""
    ok = flags == 0
    err = np.abs(gpu_img.astype(np.float64) - ref_img)
    m = float(err[:, ok].max()) if ok.any() else 0.0
    return m, 1.0 - ok.mean()


def masked_gaussians(proj, flags) -> np.ndarray:
    """Gaussians whose pixel box contains a flagged pixel (excluded from per-entry gradient checks)."""
    ys, xs = np.nonzero(flags)
    bad = np.zeros(len(proj["valid"]), dtype=bool)
    if len(ys) == 0:
        return bad
    v = proj["valid"] > 0
    for y, x in zip(ys, xs):
        bad |= v & (proj["px0"] <= x) & (proj["px1"] >= x) & (proj["py0"] <= y) & (proj["py1"] >= y)
    return bad


def grad_check(gpu, ref, exclude_rows=None, rtol=GRAD_RTOL, floor=1e-3):
    """Per-tensor relative L2 error and per-entry error with a per-column floor.
    Returns (rel_norm_err, worst_entry_ratio) where ratio <= 1 passes."""
    g = np.asarray(gpu, dtype=np.float64)
    r = np.asarray(ref, dtype=np.float64)
    rel = np.linalg.norm(g - r) / max(np.linalg.norm(r), 1e-30)
    g2 = g.reshape(g.shape[0], -1) if g.ndim > 1 else g[:, None]
    r2 = r.reshape(r.shape[0], -1) if r.ndim > 1 else r[:, None]
    if exclude_rows is not None:
        keep = ~np.asarray(exclude_rows)
        g2, r2 = g2[keep], r2[keep]
    colmax = np.abs(r2).max(axis=0, keepdims=True) + 1e-30
    bound = rtol * np.maximum(np.abs(r2), floor * colmax)
    worst = float((np.abs(g2 - r2) / bound).max()) if g2.size else 0.0
    return rel, worst
