"""On-the-fly reconstruction from a frame stream (Sec. 3.3, "Online
Reconstruction Process"; Alg. 2 of the appendix).

Incoming frames enter a local pool in first-in-first-out order; a frame
leaving the full local pool enters a global pool by reservoir sampling, so
that every frame of the stream is equally likely to be retained there.  Each
optimisation step trains on a batch drawn from both pools: a fraction eta of
it from the local pool (recent, under-fitted frames), the rest from the
global pool (history, against forgetting).  The paper uses eta = 0.7,
|M_l| = 150, |M_g| = 1000 at a 25 FPS stream.

Readings where the text is silent:
* the reservoir index of an evicted frame is its position in the stream
  (frames are evicted in arrival order, so it is also the number of frames
  evicted before it) and the replacement draw is uniform over 0..j
  inclusive, which makes the retention probability |M_g| / (frames evicted);
* the local share of a batch is round(eta B); a pool with fewer frames than
  its share gives what it has and the other pool fills the rest; draws within
  a pool are without replacement while the pool is large enough, with
  replacement otherwise (only at the very start of a stream).

Frames live in a device-resident store (HBM holds |M_l| + |M_g| frames of
targets easily), addressed by slot; a step gathers its batch on the device.
"""
from __future__ import annotations

from collections import deque

import numpy as np


class SamplingPools:
    """The local FIFO pool and the global reservoir pool of Alg. 2, over
    arbitrary items (here: store slots)."""

    def __init__(self, local_cap: int = 150, global_cap: int = 1000, eta: float = 0.7, seed: int = 4):
        if local_cap < 1 or global_cap < 0 or not 0.0 <= eta <= 1.0:
            raise ValueError("bad pool sizes or ratio")
        self.local_cap, self.global_cap, self.eta = local_cap, global_cap, eta
        self.local: deque = deque()
        self.glob: list = []
        self.seen = 0            # frames pushed so far
        self.rng = np.random.default_rng(seed)

    def push(self, item):
        """Add an incoming frame.  Returns the items that left both pools (their
        storage can be reused): the evicted frame when the reservoir rejects it,
        or the global frame it replaced."""
        dropped = []
        if len(self.local) == self.local_cap:
            j = self.seen - self.local_cap          # stream position of the evicted frame
            old = self.local.popleft()
            if len(self.glob) < self.global_cap:
                self.glob.append(old)
            else:
                k = int(self.rng.integers(0, j + 1))  # uniform over 0..j
                if k < self.global_cap:
                    dropped.append(self.glob[k])
                    self.glob[k] = old
                else:
                    dropped.append(old)
        self.local.append(item)
        self.seen += 1
        return dropped

    def _draw(self, pool, n: int) -> list:
        if n <= 0 or not pool:
            return []
        idx = self.rng.choice(len(pool), size=n, replace=len(pool) < n)
        return [pool[i] for i in idx]

    def sample(self, B: int) -> list:
        """A batch of B items: round(eta B) from the local pool, the rest from the
        global pool; a short pool's share goes to the other."""
        if not self.local and not self.glob:
            raise RuntimeError("no frames yet")
        n_l = int(round(self.eta * B))
        n_g = B - n_l
        if len(self.glob) < n_g:
            n_l += n_g - len(self.glob)
            n_g = len(self.glob)
        if len(self.local) < n_l and self.glob:
            extra = min(n_l - len(self.local), max(len(self.glob) - n_g, 0))
            n_l -= extra
            n_g += extra
        return self._draw(list(self.local), n_l) + self._draw(self.glob, n_g)


class OnlineTrainer:
    """Streams frames into a device-resident store and trains on batches drawn
    from the two pools, with the batched (graph-captured) training step."""

    def __init__(self, trainer, local_cap: int = 150, global_cap: int = 1000, eta: float = 0.7, seed: int = 4):
        import torch
        self.tr, self.torch = trainer, torch
        cfg = trainer.cfg
        self.pools = SamplingPools(local_cap, global_cap, eta, seed)
        cap = local_cap + global_cap + 1   # the incoming frame takes a slot before the eviction frees one
        dev = trainer.theta.device
        npix = cfg.width * cfg.height
        self.theta = torch.zeros(cap, cfg.d_in, device=dev, dtype=torch.float32)
        self.targets = torch.zeros(cap, 3 * npix, device=dev, dtype=torch.float32)
        self.cams = [None] * cap
        self.frame_id = [-1] * cap        # stream position of the frame in each slot
        self.free = list(range(cap - 1, -1, -1))
        self.captured = False

    def add_frame(self, theta: np.ndarray, target: np.ndarray, cam) -> None:
        """One incoming frame (tracking vector, target image CHW, camera)."""
        slot = self.free.pop()
        self.theta[slot].copy_(self.torch.from_numpy(np.ascontiguousarray(theta, dtype=np.float32)))
        self.targets[slot].copy_(self.torch.from_numpy(np.ascontiguousarray(target, dtype=np.float32).ravel()))
        self.cams[slot] = cam
        self.frame_id[slot] = self.pools.seen
        for s in self.pools.push(slot):
            self.free.append(s)

    def step(self):
        """One optimisation step on a batch drawn from the pools."""
        tr = self.tr
        slots = self.pools.sample(tr.cfg.B)
        idx = self.torch.tensor(slots, device=self.theta.device, dtype=self.torch.long)
        tr.set_batch_device(self.theta.index_select(0, idx), self.targets.index_select(0, idx),
                            [self.cams[s] for s in slots])
        st = tr.step()
        if not self.captured:
            tr.capture()
            self.captured = True
        return st, slots
