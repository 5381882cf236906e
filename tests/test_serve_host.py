"""Serving policy without a GPU: fake clock, fake executor that completes a
batch after a scripted delay."""
import numpy as np
import pytest

from paper_2503_12886_amd import synth
from paper_2503_12886_amd.serve import AvatarSpec, Batcher, Request, Server, frame_footprint


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-5)


class FakeExecutor:
    """Completes a batch `base + per_frame * len(batch)` seconds after launch."""

    def __init__(self, clock, n_slots=2, base=1e-3, per_frame=2e-4):
        self.clock, self.n_slots, self.base, self.per_frame = clock, n_slots, base, per_frame
        self.launched = []
        self.busy_slots = set()

    def launch(self, slot, batch):
        assert slot not in self.busy_slots
        self.busy_slots.add(slot)
        self.launched.append((self.clock(), slot, [r.rid for r in batch]))
        return (slot, self.clock() + self.base + self.per_frame * len(batch))

    def is_done(self, h):
        return self.clock() >= h[1]

    def finish(self, h):
        self.busy_slots.discard(h[0])


def make_requests(n, rate, avatars, seed=0):
    t, av, th, yaw = synth.make_request_stream(n, rate, len(avatars), seed=seed)
    cam = synth.make_cameras(1, 64, 64, seed=1)[0]
    return [Request(rid=i, avatar=int(av[i]), theta=th[i], cam=cam, t_arrival=float(t[i])) for i in range(n)]


AV = [AvatarSpec(N=n, K=20) for n in (2000, 4000, 6000, 8000)]


def test_every_request_served_once_and_budget_respected():
    clock = FakeClock()
    budget = 3 * frame_footprint(8000, 64, 64)
    b = Batcher(AV, budget_bytes=budget, max_batch=8, window_s=0.002)
    ex = FakeExecutor(clock, n_slots=3)
    srv = Server(b, ex, clock=clock, sleep=clock.sleep)
    reqs = make_requests(400, 2000.0, AV)
    stats = srv.run(reqs, t0=0.0)
    assert stats["requests"] == 400
    assert sorted(r.rid for r in srv.done) == list(range(400))
    assert srv.max_inflight_bytes <= budget
    assert b.inflight_bytes == 0
    # batches never exceed the size limit, and a request waits in the queue at
    # most a window beyond the moment a slot and budget were free
    assert all(len(ids) <= 8 for _, _, ids in ex.launched)
    assert stats["p99_ms"] >= stats["p50_ms"] > 0


def test_continuous_batching_overlaps_batches():
    clock = FakeClock()
    b = Batcher(AV, budget_bytes=1 << 40, max_batch=4, window_s=0.002)
    ex = FakeExecutor(clock, n_slots=3, base=5e-3, per_frame=1e-3)
    srv = Server(b, ex, clock=clock, sleep=clock.sleep)
    srv.run(make_requests(200, 4000.0, AV), t0=0.0)
    # some batch was launched while an earlier one was still running
    spans = []
    for t, slot, ids in ex.launched:
        spans.append((t, t + 5e-3 + 1e-3 * len(ids)))
    overlaps = sum(1 for i in range(1, len(spans)) if spans[i][0] < spans[i - 1][1])
    assert overlaps > 0


def test_window_bounds_queueing_when_idle():
    clock = FakeClock()
    b = Batcher(AV, budget_bytes=1 << 40, max_batch=16, window_s=0.002)
    ex = FakeExecutor(clock, n_slots=4, base=1e-4, per_frame=1e-5)
    srv = Server(b, ex, clock=clock, sleep=clock.sleep)
    reqs = make_requests(50, 100.0, AV)            # sparse arrivals: slots always free
    srv.run(reqs, t0=0.0)
    for t, _, ids in ex.launched:
        for rid in ids:
            r = next(x for x in srv.done if x.rid == rid)
            assert t - r.t_arrival <= 0.002 + 2e-4


def test_admission_rejects_oversized_and_waits_for_budget():
    b = Batcher(AV, budget_bytes=frame_footprint(8000, 64, 64), max_batch=8)
    cam = synth.make_cameras(1, 64, 64)[0]
    big = Request(0, 3, np.zeros(56), cam, 0.0)
    b.add(big)
    b.add(Request(1, 3, np.zeros(56), cam, 0.0))
    first = b.take()
    assert [r.rid for r in first] == [0]            # the second does not fit while the first is in flight
    assert b.take() == []
    b.release(first)
    assert [r.rid for r in b.take()] == [1]
    huge = Batcher(AV, budget_bytes=10, max_batch=8)
    with pytest.raises(ValueError):
        huge.add(Request(2, 0, np.zeros(56), cam, 0.0))


def test_slot_capacity_from_the_memory_budget():
    """A slot's Gaussian capacity is the largest whose planned workspace (the
    library's accounting, its most demanding pass) fits the slot's share."""
    from paper_2503_12886_amd import gbr
    from paper_2503_12886_amd.serve import slot_spec_for_budget
    ns = (20_000, 100_000, 50_000)
    spec = slot_spec_for_budget(2 << 30, 3, ns, 512, 512, 8)
    assert spec.bytes <= (2 << 30) // 3
    assert 100_000 <= spec.max_splats < 8 * 100_000
    with pytest.raises(ValueError):
        slot_spec_for_budget(64 << 20, 3, ns, 512, 512, 8)
    # the footprint of a frame grows with its Gaussians and includes the tile entries (57 B each)
    assert frame_footprint(100_000, 512, 512) - frame_footprint(50_000, 512, 512, 100_000) > 50_000 * 32 * 57


def test_batches_fit_the_slot_and_deferrals_are_counted():
    from paper_2503_12886_amd.serve import SlotSpec
    clock = FakeClock()
    spec = SlotSpec(max_frames=8, max_splats=12_000, max_pixels=8 * 64 * 64, max_entries=12_000 * 32)
    b = Batcher(AV, budget_bytes=1 << 40, max_batch=8, window_s=0.002, slot=spec)
    ex = FakeExecutor(clock, n_slots=2, base=2e-3, per_frame=5e-4)
    srv = Server(b, ex, clock=clock, sleep=clock.sleep)
    stats = srv.run(make_requests(300, 4000.0, AV), t0=0.0)
    assert stats["requests"] == 300
    n_of = {i: a.N for i, a in enumerate(AV)}
    done = {r.rid: r for r in srv.done}
    for _, _, ids in ex.launched:
        assert sum(n_of[done[i].avatar] for i in ids) <= spec.max_splats
    assert stats["deferred"] > 0
