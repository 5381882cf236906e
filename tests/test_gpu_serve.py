"""Serving on the GPU: a frame rendered alone equals the same frame rendered
inside a mixed batch of several avatars (bit for bit), and a short Poisson
stream is served completely with overlapping batches."""
import numpy as np
import pytest

from paper_2503_12886_amd import synth
from paper_2503_12886_amd.serve import AvatarSpec, Batcher, GpuExecutor, Request, Server
from paper_2503_12886_amd.trainer import mlp_pack

pytestmark = pytest.mark.gpu

NS = (3000, 5000, 2000)


def executor(n_slots=2, W=128):
    bases = [synth.make_scene(n, 20, seed=10 + i) for i, n in enumerate(NS)]
    mlps = [mlp_pack(synth.make_mlp(K=20, seed=20 + i)) for i in range(len(NS))]
    return GpuExecutor(bases, mlps, n_slots=n_slots, max_batch=16, width=W, height=W)


def requests(n, W=128, seed=0):
    t, av, th, yaw = synth.make_request_stream(n, 2000.0, len(NS), seed=seed)
    cams = synth.make_cameras(n, W, W, seed=seed + 1)
    return [Request(rid=i, avatar=int(av[i]), theta=th[i], cam=cams[i], t_arrival=float(t[i])) for i in range(n)]


def test_alone_equals_in_mix():
    import torch
    ex = executor()
    reqs = requests(12)
    mixed = ex.enqueue(0, reqs)
    torch.cuda.synchronize()
    for r in reqs:
        alone = ex.enqueue(1, [r])
        torch.cuda.synchronize()
        a = ex.image(1, alone, r.rid).cpu().numpy()
        m = ex.image(0, mixed, r.rid).cpu().numpy()
        assert np.array_equal(a, m), r.rid
    ex.close()


def test_stream_is_served_with_overlap():
    ex = executor(n_slots=3)
    b = Batcher([AvatarSpec(N=n, K=20) for n in NS], budget_bytes=1 << 30, max_batch=8, window_s=0.002)
    srv = Server(b, ex)
    stats = srv.run(requests(300, seed=3))
    assert stats["requests"] == 300
    assert stats["p99_ms"] < 1000.0
    ex.close()
