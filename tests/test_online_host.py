"""Host logic of on-the-fly reconstruction (Alg. 2): the local pool is a
FIFO of the latest frames, the global pool a reservoir in which every frame
that left the local pool is retained with the same probability (checked
statistically against |M_g| / evicted), and batches split eta : 1 - eta."""
import numpy as np

from paper_2503_12886_amd.online import SamplingPools


def test_local_pool_is_a_fifo_of_the_latest_frames():
    p = SamplingPools(local_cap=150, global_cap=1000, seed=0)
    for i in range(200):
        p.push(i)
    assert list(p.local) == list(range(50, 200))
    assert sorted(p.glob) == list(range(50))          # the reservoir is not full yet: all kept


def test_every_frame_is_kept_exactly_once_somewhere_or_dropped():
    p = SamplingPools(local_cap=7, global_cap=11, seed=1)
    dropped = []
    for i in range(500):
        dropped += p.push(i)
    held = list(p.local) + p.glob
    assert len(set(held)) == len(held)
    assert sorted(held + dropped) == list(range(500))
    assert len(p.glob) == 11 and len(p.local) == 7


def test_reservoir_retains_every_evicted_frame_with_equal_probability():
    # 205 frames through a local pool of 5: frames 0..199 are evicted, and a
    # reservoir of 20 must keep each with probability 20 / 200
    trials, n_ev, cap = 3000, 200, 20
    counts = np.zeros(n_ev)
    for t in range(trials):
        p = SamplingPools(local_cap=5, global_cap=cap, seed=1000 + t)
        for i in range(n_ev + 5):
            p.push(i)
        counts[np.array(p.glob)] += 1
    expected = trials * cap / n_ev
    chi2 = float(((counts - expected) ** 2 / expected).sum())
    # chi-square with 199 degrees of freedom: mean 199, sd 20
    assert chi2 < 199 + 5 * 20, chi2
    # no drift between early and late frames
    assert abs(counts[:100].mean() - counts[100:].mean()) < 0.05 * expected


def test_batches_split_between_the_pools():
    p = SamplingPools(local_cap=150, global_cap=1000, eta=0.7, seed=2)
    for i in range(1300):
        p.push(i)
    loc, glob = set(p.local), set(p.glob)
    for _ in range(50):
        b = p.sample(16)
        assert len(b) == 16
        l, g = b[:11], b[11:]                              # round(0.7 * 16) = 11
        assert set(l) <= loc and set(g) <= glob
        assert len(set(l)) == 11 and len(set(g)) == 5     # without replacement


def test_short_pools_lend_their_share():
    p = SamplingPools(local_cap=150, global_cap=1000, eta=0.7, seed=3)
    for i in range(3):
        p.push(i)
    b = p.sample(16)                   # only 3 frames: all from the local pool, with replacement
    assert len(b) == 16 and set(b) <= {0, 1, 2}
    p2 = SamplingPools(local_cap=4, global_cap=100, eta=0.7, seed=3)
    for i in range(60):
        p2.push(i)
    b = p2.sample(16)                  # local has 4 < 11: global fills the rest
    assert len(b) == 16
    assert sum(x in set(p2.local) for x in b) == 4
