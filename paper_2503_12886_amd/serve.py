"""Continuous-batching animation server for resident avatars.

Runtime animation in the paper (Sec. 4.2, Table 2) maps a tracking vector
through the avatar's weight MLP (Eq. 2), blends its Gaussian blendshapes
(Eq. 1) and renders the frame.  Serving many such requests at once:

* several avatars stay resident on the GPU, each with its own Gaussian count,
  bases and MLP;
* requests arrive continuously; a batch is formed at least every `window_s`
  seconds (or as soon as `max_batch` requests wait) from the queue in arrival
  order, for any free execution slot;
* admission is by HBM footprint: the executor holds `budget_bytes` of device
  workspace, split over its slots (each slot's library context is sized so
  that the bytes it holds, by the library's own accounting, fit its share);
  a request joins a batch only while the batch fits its slot's capacity
  (frames, Gaussians, pixels, tile entries) and the footprint of all work in
  flight stays within the budget; requests held back by either limit are
  counted as deferred;
* each slot has its own stream and library context, so batches launched
  while others are still on the GPU overlap with them;
* a batch holds frames of different avatars: per avatar, one MLP call and
  one blend into the packed batch buffer, then a single render of all frames
  with per-frame Gaussian sets (the library's per-frame offsets).

The host-side policy (`Batcher`) has no GPU dependency and is tested with a
fake clock and a fake executor; `GpuExecutor` issues the library calls.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np


@dataclass
class Request:
    rid: int
    avatar: int
    theta: np.ndarray
    cam: object
    t_arrival: float
    t_done: Optional[float] = None
    slot: Optional[int] = None
    frame: Optional[int] = None


@dataclass
class AvatarSpec:
    N: int
    K: int


ENTRIES_PER_SPLAT = 32   # tile entries a frame's Gaussian is planned for (measured 18 at 512 x 512, distance 0.5)


def _plan(ns, width, height, tile=16, entries_per_splat=ENTRIES_PER_SPLAT) -> int:
    """Device bytes of a library context sized exactly for one pass over
    frames of these Gaussian counts (the library's own accounting)."""
    from . import gbr
    B = len(ns)
    offs = [0]
    for n in ns:
        offs.append(offs[-1] + int(n))
    total = max(offs[-1], 1)
    return gbr.gbr_plan_bytes(tile, 64, B, total, B * width * height, max(1, total * entries_per_splat), offs,
                              [width] * B, [height] * B, total * entries_per_splat)


def frame_footprint(N: int, width: int, height: int, n_max: int | None = None, tile: int = 16,
                    entries_per_splat: int = ENTRIES_PER_SPLAT) -> int:
    """Device bytes one frame of an avatar of N Gaussians adds to a pass: the
    library's per-splat, per-pixel, per-tile and per-entry workspace, the tile
    bitmap rows sized by the largest avatar in a batch (n_max), as the
    difference of two planned contexts."""
    n_max = max(N, n_max or N)
    return (_plan([n_max, N], width, height, tile, entries_per_splat)
            - _plan([n_max], width, height, tile, entries_per_splat))


@dataclass
class SlotSpec:
    """Capacities of one execution slot's library context."""
    max_frames: int
    max_splats: int
    max_pixels: int
    max_entries: int
    tile: int = 16
    bytes: int = 0          # device bytes a context of these capacities holds after a full pass


def slot_spec_for_budget(budget_bytes: int, n_slots: int, avatars_n, width: int, height: int, max_batch: int,
                         tile: int = 16, entries_per_splat: int = ENTRIES_PER_SPLAT) -> SlotSpec:
    """The largest Gaussian capacity S per slot whose context fits
    budget / n_slots after its most demanding pass: max_batch frames (the
    most tiles) holding S Gaussians, one of them of the largest avatar (the
    longest tile bitmap rows)."""
    from . import gbr
    share = budget_bytes // n_slots
    n_max = max(avatars_n)
    W, H, mb = width, height, max_batch

    def plan(S):
        rest = S - n_max
        k = mb - 1
        ns = [n_max] + [max(1, rest // k + (1 if i < rest % k else 0)) for i in range(k)] if k else [n_max]
        offs = [0]
        for n in ns:
            offs.append(offs[-1] + n)
        return gbr.gbr_plan_bytes(tile, 64, mb, offs[-1], mb * W * H, offs[-1] * entries_per_splat, offs,
                                  [W] * len(ns), [H] * len(ns), offs[-1] * entries_per_splat)

    lo, hi = n_max, mb * n_max
    if plan(lo) > share:
        raise ValueError("the memory budget cannot hold a full batch with one frame of the largest avatar per slot")
    while lo < hi:                               # the largest S with plan(S) <= share
        mid = (lo + hi + 1) // 2
        if plan(mid) <= share:
            lo = mid
        else:
            hi = mid - 1
    return SlotSpec(mb, lo, mb * W * H, lo * entries_per_splat, tile, plan(lo))


@dataclass
class Batcher:
    """Queue, batch formation and admission (host policy only)."""
    avatars: List[AvatarSpec]
    budget_bytes: int
    max_batch: int = 16
    window_s: float = 0.002
    slot: Optional[SlotSpec] = None          # capacity of a slot's context (None: the budget alone)
    queue: collections.deque = field(default_factory=collections.deque)
    inflight_bytes: int = 0
    deferred: int = 0                        # times the head request waited for budget or slot capacity
    _fp: dict = field(default_factory=dict)

    def footprint(self, r: Request) -> int:
        key = (r.avatar, r.cam.width, r.cam.height)
        if key not in self._fp:
            n_max = max(a.N for a in self.avatars)
            self._fp[key] = frame_footprint(self.avatars[r.avatar].N, r.cam.width, r.cam.height, n_max)
        return self._fp[key]

    def add(self, r: Request) -> None:
        if self.footprint(r) > self.budget_bytes or (self.slot is not None and (
                self.avatars[r.avatar].N > self.slot.max_splats or
                r.cam.width * r.cam.height > self.slot.max_pixels)):
            raise ValueError("request larger than the whole memory budget")
        self.queue.append(r)

    def due(self, now: float) -> bool:
        """A batch should be formed now: the oldest request waited a window or a batch is full."""
        return bool(self.queue) and (len(self.queue) >= self.max_batch or now - self.queue[0].t_arrival >= self.window_s)

    def take(self) -> List[Request]:
        """Requests for one batch, in arrival order, within the free budget and
        the slot's capacity."""
        batch, used, splats, pixels = [], 0, 0, 0
        while self.queue and len(batch) < self.max_batch:
            r = self.queue[0]
            f = self.footprint(r)
            n = self.avatars[r.avatar].N
            px = r.cam.width * r.cam.height
            over = self.inflight_bytes + used + f > self.budget_bytes
            if self.slot is not None:
                over = over or splats + n > self.slot.max_splats or pixels + px > self.slot.max_pixels
            if over:
                self.deferred += 1
                break
            batch.append(self.queue.popleft())
            used += f
            splats += n
            pixels += px
        self.inflight_bytes += used
        return batch

    def release(self, batch: List[Request]) -> None:
        self.inflight_bytes -= sum(self.footprint(r) for r in batch)
        assert self.inflight_bytes >= 0


class Server:
    """Drives a Batcher and an executor over a stream of requests."""

    def __init__(self, batcher: Batcher, executor, clock: Callable[[], float] = time.perf_counter,
                 sleep: Callable[[float], None] = time.sleep):
        self.b = batcher
        self.ex = executor
        self.clock = clock
        self.sleep = sleep
        self.inflight = {}          # slot -> (batch, handle)
        self.done: List[Request] = []
        self.max_inflight_bytes = 0

    def _poll(self) -> None:
        for slot in list(self.inflight):
            batch, handle = self.inflight[slot]
            if self.ex.is_done(handle):
                now = self.clock()
                self.ex.finish(handle)
                for r in batch:
                    r.t_done = now
                self.b.release(batch)
                self.done.extend(batch)
                del self.inflight[slot]

    def _launch(self) -> None:
        free = [s for s in range(self.ex.n_slots) if s not in self.inflight]
        while free and self.b.due(self.clock()):
            batch = self.b.take()
            if not batch:
                break
            slot = free.pop(0)
            for i, r in enumerate(batch):
                r.slot, r.frame = slot, i
            self.inflight[slot] = (batch, self.ex.launch(slot, batch))
            self.max_inflight_bytes = max(self.max_inflight_bytes, self.b.inflight_bytes)

    def run(self, requests: List[Request], t0: Optional[float] = None, drain_timeout_s: float = 30.0) -> dict:
        """Feed requests at their arrival times (relative to t0) and serve them all."""
        pending = collections.deque(sorted(requests, key=lambda r: r.t_arrival))
        t0 = self.clock() if t0 is None else t0
        for r in pending:
            r.t_arrival += t0
        deadline = None
        while pending or self.b.queue or self.inflight:
            now = self.clock()
            while pending and pending[0].t_arrival <= now:
                self.b.add(pending.popleft())
            self._poll()
            self._launch()
            if not pending and deadline is None:
                deadline = now + drain_timeout_s
            if deadline is not None and now > deadline:
                raise TimeoutError("requests not drained")
            # wait for the next event: an arrival, a batch window, a completion
            nxt = pending[0].t_arrival if pending else now + 1e-4
            if self.b.queue:
                nxt = min(nxt, self.b.queue[0].t_arrival + self.b.window_s)
            wait = min(max(nxt - self.clock(), 0.0), 1e-4 if self.inflight else 1e-3)
            self.sleep(max(wait, 2e-5))
        lat = np.array([(r.t_done - r.t_arrival) * 1e3 for r in self.done])
        span = max(r.t_done for r in self.done) - min(r.t_arrival for r in self.done)
        return {"requests": len(self.done), "frames_per_s": len(self.done) / span if span > 0 else 0.0,
                "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "mean_ms": float(lat.mean()), "max_inflight_bytes": int(self.max_inflight_bytes),
                "deferred": int(self.b.deferred)}


class GpuExecutor:
    """Executes batches with libgbr: one stream, context and buffer set per slot."""

    def __init__(self, avatars_bases, avatars_mlp, n_slots: int = 3, max_batch: int = 16, width: int = 512,
                 height: int = 512, d_in: int = 56, hidden: int = 256, tile: int = 16, chunk: int = 64,
                 device: int = 0, slot: Optional[SlotSpec] = None):
        """With slot, every slot's context gets those capacities (a memory
        budget's share, slot_spec_for_budget); without, room for max_batch
        frames of the largest avatar."""
        import torch

        from . import gbr
        self.torch, self.gbr = torch, gbr
        dev = torch.device("cuda", device)
        self.dev = dev
        self.bases = [torch.from_numpy(np.ascontiguousarray(b, np.float32)).to(dev) for b in avatars_bases]
        self.mlp = [torch.from_numpy(np.ascontiguousarray(m, np.float32)).to(dev) for m in avatars_mlp]
        self.N = [b.shape[1] for b in self.bases]
        self.K = [b.shape[0] - 1 for b in self.bases]
        self.d_in, self.hidden = d_in, hidden
        self.n_slots = n_slots
        maxN = max(self.N)
        if slot is None:
            slot = SlotSpec(max_batch, max_batch * maxN, max_batch * width * height,
                            max_batch * maxN * ENTRIES_PER_SPLAT, tile)
        self.spec = slot
        max_splats = slot.max_splats
        self.overflows = 0
        self.slots = []
        for _ in range(n_slots):
            ctx = gbr.Context(tile=slot.tile, chunk=chunk, device=device, max_frames=slot.max_frames,
                              max_splats=max_splats, max_pixels=slot.max_pixels, max_entries=slot.max_entries)
            self.slots.append({
                "ctx": ctx, "stream": torch.cuda.Stream(device=dev),
                "theta_h": torch.zeros(max_batch, d_in, dtype=torch.float32).pin_memory(),
                "theta": torch.zeros(max_batch, d_in, device=dev),
                "psi": torch.zeros(max_batch, max(self.K), device=dev),
                "raw": torch.zeros(max_splats, 16, device=dev),
                "images": torch.zeros(max_batch * 3 * width * height, device=dev),
                "event": torch.cuda.Event(),
            })

    def enqueue(self, slot: int, batch: List[Request]):
        """Every kernel of one batch on the slot's stream; returns the image offsets."""
        gbr, S = self.gbr, self.slots[slot]
        order = sorted(range(len(batch)), key=lambda i: batch[i].avatar)   # group frames by avatar (stable)
        frames = [batch[i] for i in order]
        with self.torch.cuda.stream(S["stream"]):
            for i, r in enumerate(frames):
                S["theta_h"][i].copy_(self.torch.from_numpy(np.asarray(r.theta, np.float32)))
            S["theta"][:len(frames)].copy_(S["theta_h"][:len(frames)], non_blocking=True)
            offsets = [0]
            i = 0
            while i < len(frames):
                a = frames[i].avatar
                j = i
                while j < len(frames) and frames[j].avatar == a:
                    j += 1
                n, N, K = j - i, self.N[a], self.K[a]
                kmax = S["psi"].shape[1]
                psi = S["psi"].view(-1)[i * kmax:i * kmax + n * K].view(n, K)   # disjoint per group
                gbr.gbr_mlp_forward(S["ctx"], self.mlp[a], S["theta"][i:j], self.d_in, self.hidden, K, psi)
                raw = S["raw"].view(-1)[offsets[-1] * 16:(offsets[-1] + n * N) * 16].view(n, N, 16)
                gbr.gbr_blend(S["ctx"], self.bases[a], psi, raw)
                for _ in range(n):
                    offsets.append(offsets[-1] + N)
                i = j
            gbr.gbr_render(S["ctx"], S["raw"], offsets, [r.cam for r in frames], S["images"])
            S["event"].record(S["stream"])
        out = {}
        o = 0
        for r in frames:
            npx = 3 * r.cam.width * r.cam.height
            out[r.rid] = (o, npx)
            o += npx
        return out

    def launch(self, slot: int, batch: List[Request]):
        return (slot, self.enqueue(slot, batch), batch)

    def is_done(self, handle) -> bool:
        return self.slots[handle[0]]["event"].query()

    def finish(self, handle) -> None:
        """Reads the batch's status; a batch that overflowed the slot's tile
        entries (more than planned) grows them and renders again."""
        slot, _, batch = handle
        S = self.slots[slot]
        st = self.gbr.gbr_query_status(S["ctx"], S["stream"])
        if st.overflow:
            self.overflows += 1
            self.gbr.gbr_reserve(S["ctx"], st.entries + st.entries // 4 + 4096)
            self.enqueue(slot, batch)
            if self.gbr.gbr_query_status(S["ctx"], S["stream"]).overflow:
                raise RuntimeError("tile-entry overflow persists while serving")

    def memory(self) -> int:
        """Device bytes the slots' contexts hold (the library's accounting)."""
        return sum(self.gbr.gbr_memory(S["ctx"]) for S in self.slots)

    def image(self, slot: int, offsets: dict, rid: int):
        o, n = offsets[rid]
        return self.slots[slot]["images"][o:o + n]

    def close(self) -> None:
        for S in self.slots:
            S["ctx"].close()
