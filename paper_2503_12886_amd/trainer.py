"""Training-step driver: the sequence of library calls that makes one
optimisation step of the reduced-Gaussian-blendshape avatar, in two schemes.

* batched (Sec. 3.2, Fig. 5c): B frames per step -- weights MLP (Eq. 2),
  blend (Eq. 1), one batch-parallel render, L1 loss with random backgrounds
  (Sec. 3.2), backward to bases and MLP, Adam with per-attribute learning
  rates (Sec. A.3); one host synchronisation (the status read) per step.
  The whole step can be captured once as a graph and replayed.
* per-frame (Fig. 5a, "w/o batch parallel"): one frame per optimisation
  step, preprocess -> host synchronisation to size the tile lists ->
  rasterize, and an Adam step per frame.
* naive batch-parallel (Fig. 5b, Table 4 middle row): one optimisation step
  per batch (batched MLP, blend, blend adjoint, MLP adjoint, Adam), but the
  frames are rasterised one after another, each with its own host
  synchronisation between preprocess and rasterize.

This module only sequences calls into libgbr and owns the device buffers;
every step of the computation runs in the library's kernels.
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np

from . import gbr

# Adam learning rates of Sec. A.3: position 8e-4, opacity 0.25, scale 0.025,
# rotation 5e-3, colour 0.0125; blendshape deltas of position, rotation and
# colour at 0.05x, 0.5x and 0.5x of those (deltas of scale and opacity, which
# the paper does not blend, keep the base rate here); MLP 1e-3.
_BASE = {"pos": 8e-4, "rot": 5e-3, "scale": 0.025, "opacity": 0.25, "color": 0.0125}
_DELTA = {"pos": 0.05, "rot": 0.5, "scale": 1.0, "opacity": 1.0, "color": 0.5}
_GROUPS = ["pos"] * 3 + ["rot"] * 4 + ["scale"] * 3 + ["opacity"] + ["color"] * 3 + [None, None]
MLP_LR = 1e-3
ADAM_BETAS = (0.9, 0.999)
ADAM_EPS = 1e-15


# Features the paper leaves out of the blend (Sec. A.3): scale and opacity.
UNBLENDED = (7, 8, 9, 10)


def bases_lr_table(paper_mask: bool = False) -> list:
    """32-entry Adam rate table: 16 per-feature rates of G_0, then 16 of the
    deltas.  With paper_mask the deltas of scale and opacity get rate 0 (they
    stay at zero: those attributes are not blended)."""
    base = [(_BASE[g] if g else 0.0) for g in _GROUPS]
    delta = [(_BASE[g] * _DELTA[g] if g else 0.0) for g in _GROUPS]
    if paper_mask:
        for f in UNBLENDED:
            delta[f] = 0.0
    return base + delta


@dataclass
class StepConfig:
    N: int = 50_000
    K: int = 20
    B: int = 16
    width: int = 512
    height: int = 512
    d_in: int = 56
    hidden: int = 256
    loss: int = 1            # 1 = L1 (paper), 2 = L2
    tile: int = 16
    chunk: int = 64
    paper_mask: bool = False  # scale and opacity not blended (their deltas held at zero)
    fused_adam: bool = True   # the bases' Adam step forms dbases itself (gbr_blend_adam_step)


def mlp_numel(d_in: int, hidden: int, K: int) -> int:
    return hidden * d_in + hidden + hidden * hidden + hidden + K * hidden + K


class Trainer:
    def __init__(self, cfg: StepConfig, bases: np.ndarray, mlp_params: np.ndarray, max_entries: int = 0,
                 device: int = 0):
        import torch
        self.cfg = cfg
        self.torch = torch
        N, K, B = cfg.N, cfg.K, cfg.B
        dev = torch.device("cuda", device)
        f32 = dict(device=dev, dtype=torch.float32)
        self.bases = torch.from_numpy(np.ascontiguousarray(bases, dtype=np.float32)).to(dev)
        assert tuple(self.bases.shape) == (K + 1, N, 16)
        self._mask_deltas()
        self.bases_m = torch.zeros_like(self.bases)
        self.bases_v = torch.zeros_like(self.bases)
        self.dbases = torch.zeros_like(self.bases)
        nm = mlp_numel(cfg.d_in, cfg.hidden, K)
        self.mlp = torch.from_numpy(np.ascontiguousarray(mlp_params, dtype=np.float32)).to(dev)
        assert self.mlp.numel() == nm
        self.mlp_m = torch.zeros_like(self.mlp)
        self.mlp_v = torch.zeros_like(self.mlp)
        self.dmlp = torch.zeros_like(self.mlp)
        self.theta = torch.zeros(B, cfg.d_in, **f32)
        self.psi = torch.zeros(B, K, **f32)
        self.dpsi = torch.zeros(B, K, **f32)
        self.raw = torch.zeros(B, N, 16, **f32)
        self.draw = torch.zeros(B, N, 16, **f32)
        npix = cfg.width * cfg.height
        self.images = torch.zeros(B * 3 * npix, **f32)
        self.dimages = torch.zeros_like(self.images)
        self.targets = torch.zeros_like(self.images)
        if max_entries <= 0:
            max_entries = max(1 << 20, 40 * B * N)
        self.ctx = gbr.Context(tile=cfg.tile, chunk=cfg.chunk, device=device, max_frames=max(B, 1),
                               max_splats=B * N, max_pixels=B * npix, max_entries=max_entries)
        self.lr_bases = bases_lr_table(cfg.paper_mask)
        self.lr_mlp = [MLP_LR] * 32
        self.cams = None
        self.graph = None
        self.steps_launched = 0     # batched steps enqueued, retries included
        self.offsets = [b * N for b in range(B + 1)]
        # a stream of its own (default priority): the legacy null stream cannot be captured
        self.stream = torch.cuda.Stream(device=dev)

    # ---------------------------------------------------------------- inputs
    def bind_mesh(self, faces: np.ndarray, face_uv: np.ndarray, tri: np.ndarray, bary: np.ndarray,
                  n_verts: int) -> None:
        """Tangent-space Gaussians (Sec. 3.1, Eq. 4): Gaussian n is bound to
        triangle tri[n] at barycentric coordinates bary[n]; every batch then
        carries one deformed mesh per frame (set_batch(..., verts=...)) and the
        step transforms the blended Gaussians to it before rendering."""
        torch, cfg = self.torch, self.cfg
        assert self.graph is None, "bind the mesh before capturing"
        dev = self.bases.device
        self.faces = torch.from_numpy(np.ascontiguousarray(faces, dtype=np.int32)).to(dev)
        self.face_uv = torch.from_numpy(np.ascontiguousarray(face_uv, dtype=np.float32)).to(dev)
        self.tri = torch.from_numpy(np.ascontiguousarray(tri, dtype=np.int32)).to(dev)
        self.bary = torch.from_numpy(np.ascontiguousarray(bary, dtype=np.float32)).to(dev)
        F = self.faces.shape[0]
        self.verts = torch.zeros(cfg.B, n_verts, 3, device=dev, dtype=torch.float32)
        self.frames = torch.zeros(cfg.B, F, 16, device=dev, dtype=torch.float32)

    def set_batch(self, theta: np.ndarray, targets: np.ndarray, cams: list, verts=None) -> None:
        """Copy one batch of (tracking vector, target image, camera[, deformed mesh])
        into the step's buffers."""
        assert len(cams) == self.cfg.B
        assert (verts is None) == (getattr(self, "verts", None) is None), "verts go with a bound mesh"
        self.torch.cuda.synchronize()
        self.theta.copy_(self.torch.from_numpy(np.ascontiguousarray(theta, dtype=np.float32)))
        self.targets.copy_(self.torch.from_numpy(np.ascontiguousarray(targets, dtype=np.float32).ravel()))
        if verts is not None:
            self.verts.copy_(self.torch.from_numpy(np.ascontiguousarray(verts, dtype=np.float32)))
        self.torch.cuda.synchronize()
        self.cams = list(cams)
        if self.graph is not None:
            gbr.gbr_stage_frames(self.ctx, self.offsets, self.cams)

    def set_batch_device(self, theta, targets, cams: list) -> None:
        """The same from device tensors (theta [B][d_in], targets [B][3 H W]),
        ordered on the trainer's stream."""
        assert len(cams) == self.cfg.B
        self._no_mesh("streaming batches")
        cur = self.torch.cuda.current_stream()
        self.stream.wait_stream(cur)
        with self.torch.cuda.stream(self.stream):
            self.theta.copy_(theta)
            self.targets.copy_(targets.reshape(-1))
        theta.record_stream(self.stream)      # the sources stay allocated until the copies ran
        targets.record_stream(self.stream)
        self.cams = list(cams)
        if self.graph is not None:
            gbr.gbr_stage_frames(self.ctx, self.offsets, self.cams)

    def render_targets(self) -> None:
        """Targets = this model's own renders of the current batch (used to make
        a ground-truth avatar's frames the training targets)."""
        c, cfg = self.ctx, self.cfg
        with self.torch.cuda.stream(self.stream):
            gbr.gbr_mlp_forward(c, self.mlp, self.theta, cfg.d_in, cfg.hidden, cfg.K, self.psi)
            gbr.gbr_blend(c, self.bases, self.psi, self.raw)
            self._render(self.targets)
            st = gbr.gbr_query_status(c, self.stream)
        if st.overflow:
            self._grow(st.entries)
            self.render_targets()

    def _mask_deltas(self) -> None:
        if self.cfg.paper_mask:
            self.bases[1:, :, list(UNBLENDED)] = 0.0

    def load_bases(self, bases: np.ndarray) -> None:
        """Replace the blendshape bases (Adam state restarts)."""
        self.torch.cuda.synchronize()
        self.bases.copy_(self.torch.from_numpy(np.ascontiguousarray(bases, dtype=np.float32)))
        self._mask_deltas()
        self.bases_m.zero_()
        self.bases_v.zero_()
        self.torch.cuda.synchronize()

    # ---------------------------------------------------------------- one step
    def enqueue_step(self) -> None:
        """Every kernel of one batched optimisation step, enqueued on the trainer's stream."""
        with self.torch.cuda.stream(self.stream):
            self._enqueue_step()

    def batch_grads(self) -> None:
        """The batched step's gradients (dbases, dpsi, dmlp) without the update."""
        with self.torch.cuda.stream(self.stream):
            self._enqueue_grads()

    def _render(self, images) -> None:
        """The batch's render of the blended Gaussians (enqueued on the
        current stream).  With a bound mesh they live in tangent space: the
        per-(frame, triangle) frames are formed, and the pass carries every
        Gaussian to its frame's mesh inside the projection; its backward then
        returns tangent-space gradients."""
        c = self.ctx
        if getattr(self, "verts", None) is None:
            gbr.gbr_render(c, self.raw, self.offsets, self.cams, images)
            return
        gbr.gbr_tangent_frames(c, self.verts, self.faces, self.face_uv, self.frames)
        gbr.gbr_render_tangent(c, self.raw, self.tri, self.bary, self.verts, self.faces, self.frames, self.cams,
                               images)

    def _enqueue_grads(self, fused: bool = False):
        """Forward, loss and backward. With fused, dbases is left to the
        update (gbr_blend_adam_step); returns the draw that update needs."""
        c, cfg = self.ctx, self.cfg
        gbr.gbr_mlp_forward(c, self.mlp, self.theta, cfg.d_in, cfg.hidden, cfg.K, self.psi)
        gbr.gbr_blend(c, self.bases, self.psi, self.raw)
        self._render(self.images)
        gbr.gbr_loss(c, self.images, self.targets, cfg.loss, self.dimages)
        dbases = None if fused else self.dbases
        gbr.gbr_render_backward(c, self.dimages, self.draw)     # tangent space when a mesh is bound
        gbr.gbr_blend_backward(c, self.draw, self.bases, self.psi, dbases, self.dpsi)
        gbr.gbr_mlp_backward(c, self.mlp, self.dpsi, self.dmlp)
        return self.draw

    def _enqueue_step(self) -> None:
        c, cfg = self.ctx, self.cfg
        draw = self._enqueue_grads(cfg.fused_adam)
        if cfg.fused_adam:
            gbr.gbr_blend_adam_step(c, 0, draw, self.psi, self.bases, self.bases_m, self.bases_v, self.lr_bases,
                                    ADAM_BETAS[0], ADAM_BETAS[1], ADAM_EPS)
        else:
            gbr.gbr_adam_step(c, 0, self.bases, self.dbases, self.bases_m, self.bases_v, cfg.N * 16, self.lr_bases,
                              ADAM_BETAS[0], ADAM_BETAS[1], ADAM_EPS)
        gbr.gbr_adam_step(c, 1, self.mlp, self.dmlp, self.mlp_m, self.mlp_v, self.mlp.numel(), self.lr_mlp,
                          ADAM_BETAS[0], ADAM_BETAS[1], ADAM_EPS)

    def step(self) -> gbr.gbr_status:
        """One batched step (graph replay if captured) and its single status read.
        On entry overflow the step did not update anything: grow and replay."""
        for _ in range(3):
            if self.graph is not None:
                self._replay()
            else:
                self.enqueue_step()
            self.steps_launched += 1
            st = gbr.gbr_query_status(self.ctx, self.stream)
            if not st.overflow:
                return st
            self._grow(st.entries)
        raise RuntimeError("tile-entry overflow persists after growing the capacity")

    def run_steps(self, n: int, depth: int = 2, record: list | None = None) -> gbr.gbr_status:
        """n steps on the current batch from the captured graph, each replay
        enqueued before the host waits for the status of the step before it:
        still one status read per step, but the GPU does not idle while the
        host reads it and launches the next replay.  The captured step ends
        with its own status post, so nothing is enqueued between replays.  A
        step that overflowed updated nothing: the steps in flight are
        drained, the capacity grows, the graph is captured again and the
        missing steps run. Returns the last step's status.  With record,
        appends (host time when the step's status arrived, its tile entries)
        for every completed step."""
        assert self.graph is not None, "capture the step first"
        assert 1 <= depth <= 4                     # the status ring holds 4 posts
        done, inflight, retries = 0, [], 0
        last = None
        while done < n:
            while len(inflight) < depth and done + len(inflight) < n:
                self._replay()
                inflight.append(gbr.gbr_status_posts(self.ctx))   # this replay's post
                self.steps_launched += 1
            st = gbr.gbr_status_wait(self.ctx, inflight.pop(0))
            if not st.overflow:
                done, last, retries = done + 1, st, 0
                if record is not None:
                    record.append((time.perf_counter(), int(st.entries)))
                continue
            need = st.entries
            for post in inflight:                 # drain the replays in flight
                s2 = gbr.gbr_status_wait(self.ctx, post)
                if s2.overflow:
                    need = max(need, s2.entries)
                else:
                    done, last = done + 1, s2
                    if record is not None:
                        record.append((time.perf_counter(), int(s2.entries)))
            inflight = []
            retries += 1
            if retries > 3:
                raise RuntimeError("tile-entry overflow persists after growing the capacity")
            self._grow(need)
        return last

    def _grow(self, entries: int) -> None:
        gbr.gbr_reserve(self.ctx, entries + entries // 4 + 4096)
        if self.graph is not None:      # buffers moved: capture again
            self._recapture()

    def _recapture(self) -> None:
        gbr.gbr_graph_destroy(self.graph)
        self.graph = None
        self.capture()

    def _replay(self) -> None:
        """Launch the captured step; if the context reallocated a buffer the
        graph uses since it was captured (e.g. an entry count of the
        per-frame scheme grew the capacity), the library refuses the launch
        and the step is captured again."""
        try:
            gbr.gbr_graph_launch(self.graph, self.stream)
        except gbr.GbrError as e:
            if e.code != -5:
                raise
            self._recapture()
            gbr.gbr_graph_launch(self.graph, self.stream)

    def capture(self) -> None:
        """Capture one step as a graph (after a warm-up step sized the buffers),
        ending with a post of its status (gbr_status_post)."""
        self.torch.cuda.synchronize()
        gbr.gbr_graph_begin(self.ctx, self.stream)
        try:
            self.enqueue_step()
            gbr.gbr_status_post(self.ctx, self.stream)
        finally:
            g = gbr.gbr_graph_end(self.ctx, self.stream)
        self.graph = g

    # ---------------------------------------------------------------- per-frame scheme
    def per_frame_steps(self, frames) -> None:
        """One optimisation step per frame (frames: indices into the current batch)."""
        with self.torch.cuda.stream(self.stream):
            self._per_frame_steps(frames)

    def _no_mesh(self, what: str) -> None:
        if getattr(self, "verts", None) is not None:
            raise NotImplementedError(f"{what} runs on world-space Gaussians only (no bound mesh)")

    def _per_frame_steps(self, frames) -> None:
        self._no_mesh("the per-frame scheme")
        c, cfg = self.ctx, self.cfg
        npix = cfg.width * cfg.height
        for b in frames:
            th = self.theta[b:b + 1]
            psi = self.psi[b:b + 1]
            raw = self.raw[0:1]
            img = self.images[:3 * npix]
            dimg = self.dimages[:3 * npix]
            tgt = self.targets[b * 3 * npix:(b + 1) * 3 * npix]
            gbr.gbr_mlp_forward(c, self.mlp, th, cfg.d_in, cfg.hidden, cfg.K, psi)
            gbr.gbr_blend(c, self.bases, psi, raw)
            gbr.gbr_preprocess(c, raw, [0, cfg.N], [self.cams[b]])
            gbr.gbr_entry_count(c)                      # the per-frame host synchronisation (Sec. 3.2)
            gbr.gbr_rasterize(c, img)
            gbr.gbr_loss(c, img, tgt, cfg.loss, dimg)
            gbr.gbr_backward(c, dimg, self.bases, psi, self.dbases, self.dpsi[b:b + 1])
            gbr.gbr_mlp_backward(c, self.mlp, self.dpsi[b:b + 1], self.dmlp)
            gbr.gbr_adam_step(c, 0, self.bases, self.dbases, self.bases_m, self.bases_v, cfg.N * 16,
                              self.lr_bases, ADAM_BETAS[0], ADAM_BETAS[1], ADAM_EPS)
            gbr.gbr_adam_step(c, 1, self.mlp, self.dmlp, self.mlp_m, self.mlp_v, self.mlp.numel(), self.lr_mlp,
                              ADAM_BETAS[0], ADAM_BETAS[1], ADAM_EPS)
            st = gbr.gbr_query_status(c)
            if st.overflow:
                raise RuntimeError("unexpected overflow in the per-frame scheme")

    # ---------------------------------------------------------------- colour initialisation
    def color_init(self, delta: float = 0.1) -> int:
        """Eq. 3 on the current batch: render it, then set the base colour of every
        not-yet-initialised Gaussian whose total splatting weight in some frame
        exceeds delta.  Returns how many Gaussians are initialised so far."""
        c, cfg = self.ctx, self.cfg
        if getattr(self, "ci_done", None) is None:
            self.ci_done = self.torch.zeros(cfg.N, dtype=self.torch.uint8, device=self.bases.device)
        for _ in range(3):
            with self.torch.cuda.stream(self.stream):
                gbr.gbr_mlp_forward(c, self.mlp, self.theta, cfg.d_in, cfg.hidden, cfg.K, self.psi)
                gbr.gbr_blend(c, self.bases, self.psi, self.raw)
                self._render(self.images)
                st = gbr.gbr_query_status(c, self.stream)
                if not st.overflow:
                    gbr.gbr_color_init(c, self.targets, self.bases, self.ci_done, delta)
                    gbr.gbr_query_status(c, self.stream)
                    return int(self.ci_done.sum().item())
            self._grow(st.entries)
        raise RuntimeError("tile-entry overflow persists after growing the capacity")

    # ---------------------------------------------------------------- naive batch-parallel scheme
    def naive_batch_grads(self) -> None:
        """Gradients of one batch, rasterising frame by frame with a host
        synchronisation per frame (Fig. 5b).  Each frame's loss is normalised
        over that frame alone: the gradients are B times the batched step's
        (a constant factor that Adam's update does not see)."""
        with self.torch.cuda.stream(self.stream):
            self._naive_batch_grads()

    def _naive_batch_grads(self) -> None:
        self._no_mesh("the naive batch-parallel scheme")
        c, cfg = self.ctx, self.cfg
        npix = cfg.width * cfg.height
        if getattr(self, "draw", None) is None:
            self.draw = self.torch.zeros_like(self.raw)
        gbr.gbr_mlp_forward(c, self.mlp, self.theta, cfg.d_in, cfg.hidden, cfg.K, self.psi)
        gbr.gbr_blend(c, self.bases, self.psi, self.raw)
        for b in range(cfg.B):
            img = self.images[b * 3 * npix:(b + 1) * 3 * npix]
            dimg = self.dimages[b * 3 * npix:(b + 1) * 3 * npix]
            tgt = self.targets[b * 3 * npix:(b + 1) * 3 * npix]
            gbr.gbr_preprocess(c, self.raw[b:b + 1], [0, cfg.N], [self.cams[b]])
            gbr.gbr_entry_count(c)                      # the synchronisation of each frame (Fig. 5b)
            gbr.gbr_rasterize(c, img)
            gbr.gbr_loss(c, img, tgt, cfg.loss, dimg)
            gbr.gbr_render_backward(c, dimg, self.draw[b:b + 1])
        gbr.gbr_blend_backward(c, self.draw, self.bases, self.psi, self.dbases, self.dpsi)
        gbr.gbr_mlp_backward(c, self.mlp, self.dpsi, self.dmlp)

    def naive_batch_steps(self, n: int) -> None:
        """n optimisation steps of the naive batch-parallel scheme."""
        c, cfg = self.ctx, self.cfg
        with self.torch.cuda.stream(self.stream):
            for _ in range(n):
                self._naive_batch_grads()
                gbr.gbr_adam_step(c, 0, self.bases, self.dbases, self.bases_m, self.bases_v, cfg.N * 16,
                                  self.lr_bases, ADAM_BETAS[0], ADAM_BETAS[1], ADAM_EPS)
                gbr.gbr_adam_step(c, 1, self.mlp, self.dmlp, self.mlp_m, self.mlp_v, self.mlp.numel(),
                                  self.lr_mlp, ADAM_BETAS[0], ADAM_BETAS[1], ADAM_EPS)
                st = gbr.gbr_query_status(c)
                if st.overflow:
                    raise RuntimeError("unexpected overflow in the naive batch-parallel scheme")

    def close(self) -> None:
        if self.graph is not None:
            gbr.gbr_graph_destroy(self.graph)
            self.graph = None
        self.ctx.close()


def mlp_pack(p: dict) -> np.ndarray:
    return np.concatenate([p["W1"].ravel(), p["b1"], p["W2"].ravel(), p["b2"], p["W3"].ravel(), p["b3"]]).astype(
        np.float32)
