"""The training step: graph replay equals eager execution bit for bit (over
several replays with eager work and synchronisations in between), re-staged
cameras reach the replay, overflow is recovered, the per-frame scheme runs
the same kernels one frame per step, and the naive batch-parallel scheme
(frames rasterised one by one, a synchronisation each) gives the batched
step's gradients."""
import numpy as np
import pytest

from paper_2503_12886_amd import gbr, synth
from paper_2503_12886_amd.trainer import StepConfig, Trainer, mlp_pack

pytestmark = pytest.mark.gpu


def small(seed=0, B=4, N=3000, K=8, W=96, H=80):
    cfg = StepConfig(N=N, K=K, B=B, width=W, height=H)
    bases = synth.make_scene(N, K, seed=seed)
    mlp = mlp_pack(synth.make_mlp(K=K, seed=5))
    theta = synth.make_tracking(B, seed=2)
    cams = synth.make_cameras(B, W, H, seed=1)
    targets = np.stack(synth.make_targets(cams, seed=3))
    return cfg, bases, mlp, theta, cams, targets


def state(tr):
    return [t.detach().cpu().numpy().copy() for t in (tr.bases, tr.bases_m, tr.bases_v, tr.mlp, tr.mlp_m, tr.mlp_v)]


def test_graph_replay_equals_eager():
    cfg, bases, mlp, theta, cams, targets = small()
    a = Trainer(cfg, bases, mlp)
    a.set_batch(theta, targets, cams)
    b = Trainer(cfg, bases, mlp)
    b.set_batch(theta, targets, cams)
    la = [a.step().loss for _ in range(4)]
    lb = [b.step().loss]
    b.capture()
    for _ in range(3):
        lb.append(b.step().loss)
        # eager work and a synchronisation between replays
        x = b.torch.ones(1000, device="cuda").sum()
        b.torch.cuda.synchronize()
        assert float(x) == 1000.0
    assert la == lb
    for x, y in zip(state(a), state(b)):
        assert np.array_equal(x, y)
    assert a.step().adam_steps[0] == b.step().adam_steps[0] == 5
    a.close(); b.close()


def test_restaged_cameras_reach_the_replay():
    cfg, bases, mlp, theta, cams, targets = small(seed=1)
    cams2 = synth.make_cameras(cfg.B, cfg.width, cfg.height, seed=9)
    a = Trainer(cfg, bases, mlp)
    a.set_batch(theta, targets, cams)
    a.step()
    a.set_batch(theta, targets, cams2)
    a.step()
    b = Trainer(cfg, bases, mlp)
    b.set_batch(theta, targets, cams)
    b.step()
    b.capture()
    b.set_batch(theta, targets, cams2)     # re-stages the captured frame table
    b.step()
    for x, y in zip(state(a), state(b)):
        assert np.array_equal(x, y)
    a.close(); b.close()


def test_step_recovers_from_entry_overflow():
    cfg, bases, mlp, theta, cams, targets = small(seed=2)
    a = Trainer(cfg, bases, mlp, max_entries=2000)
    a.set_batch(theta, targets, cams)
    st = a.step()
    assert not st.overflow and st.entries > 2000 and st.adam_steps[0] == 1
    b = Trainer(cfg, bases, mlp)
    b.set_batch(theta, targets, cams)
    b.step()
    for x, y in zip(state(a), state(b)):
        assert np.array_equal(x, y)
    a.close(); b.close()


def test_per_frame_scheme_runs_one_step_per_frame():
    cfg, bases, mlp, theta, cams, targets = small(seed=3, B=3)
    a = Trainer(cfg, bases, mlp, max_entries=1000)
    a.set_batch(theta, targets, cams)
    a.per_frame_steps(range(3))
    st = gbr.gbr_query_status(a.ctx)
    assert st.adam_steps[0] == 3 and st.adam_steps[1] == 3
    assert np.isfinite(a.bases.cpu().numpy()).all()
    a.close()


def test_naive_batch_scheme_gives_the_batched_gradients():
    """Rasterising the frames one after another (Fig. 5b) changes when the
    work runs, not what it computes: with each frame's loss normalised over
    that frame alone, every gradient is exactly B (= 4, a power of two) times
    the batched step's."""
    cfg, bases, mlp, theta, cams, targets = small(seed=4, B=4)
    a = Trainer(cfg, bases, mlp)
    a.set_batch(theta, targets, cams)
    a.batch_grads()
    gbr.gbr_query_status(a.ctx, a.stream)
    ref = [t.detach().cpu().numpy().copy() for t in (a.dbases, a.dpsi, a.dmlp)]
    a.naive_batch_grads()
    gbr.gbr_query_status(a.ctx, a.stream)
    got = [t.detach().cpu().numpy().copy() for t in (a.dbases, a.dpsi, a.dmlp)]
    for r, g in zip(ref, got):
        assert np.abs(r).max() > 0
        assert np.array_equal(g, np.float32(cfg.B) * r)
    a.naive_batch_steps(2)
    assert gbr.gbr_query_status(a.ctx).adam_steps[0] == 2
    a.close()


def test_paper_feature_mask_keeps_scale_and_opacity_unblended():
    """With the paper's feature mask (Sec. A.3: scale and opacity are not
    blended) their delta slices stay exactly zero through training while the
    base model and the other deltas move.  From the same start (those slices
    zero) one masked step equals one unmasked step bit for bit everywhere
    but there: the mask withholds exactly their update and nothing else (the
    gradients, and so the Adam moments, are the same)."""
    from dataclasses import replace
    from paper_2503_12886_amd.trainer import UNBLENDED
    cfg, bases, mlp, theta, cams, targets = small(seed=5)
    masked = list(UNBLENDED)
    start = bases.copy()
    start[1:][:, :, masked] = 0.0
    a = Trainer(replace(cfg, paper_mask=True), start, mlp)
    b = Trainer(cfg, start, mlp)
    for tr in (a, b):
        tr.set_batch(theta, targets, cams)
    b0 = a.bases.cpu().numpy().copy()
    assert not b0[1:][:, :, masked].any()
    a.step()
    b.step()
    sa, sb = state(a), state(b)
    keep = np.ones(sa[0].shape, bool)
    keep[1:, :, masked] = False
    assert np.array_equal(sa[0][keep], sb[0][keep])          # bases outside the masked slices
    assert not sa[0][~keep].any() and sb[0][~keep].any()     # masked: held in a, moved in b
    for x, y in zip(sa[1:], sb[1:]):                          # Adam moments and the MLP: identical
        assert np.array_equal(x, y)
    for _ in range(2):
        a.step()
    b1 = a.bases.cpu().numpy()
    assert not b1[1:][:, :, masked].any()
    assert not np.array_equal(b1[0], b0[0])
    assert not np.array_equal(b1[1:][:, :, :3], b0[1:][:, :, :3])
    a.close(); b.close()


def test_online_trainer_streams_frames_through_the_pools():
    """On-the-fly training (Alg. 2): frames stream into a device store through
    the two pools; every step trains on frames the pools hold (the gathered
    tracking vectors are those frames'), slots are reused only once a frame
    left both pools, and the captured step replays with each batch's cameras."""
    from paper_2503_12886_amd.online import OnlineTrainer
    cfg, bases, mlp, theta, cams, targets = small(seed=6, B=4)
    n = 30
    th = synth.make_tracking(n, seed=7)
    cm = synth.make_cameras(n, cfg.width, cfg.height, seed=8)
    tg = np.stack(synth.make_targets(cm, seed=9))
    tr = Trainer(cfg, bases, mlp)
    on = OnlineTrainer(tr, local_cap=6, global_cap=10, eta=0.75, seed=1)
    for i in range(n):
        on.add_frame(th[i], tg[i], cm[i])
        st, slots = on.step()
        assert not st.overflow and np.isfinite(st.loss)
        held = list(on.pools.local) + on.pools.glob
        assert set(slots) <= set(held)
        assert len(set(held)) == len(held) and not set(held) & set(on.free)
        got = tr.theta.cpu().numpy()
        want = np.stack([th[on.frame_id[s]] for s in slots]).astype(np.float32)
        assert np.array_equal(got, want)
    assert on.captured and tr.graph is not None
    assert list(on.pools.local) and len(on.pools.glob) == 10
    tr.close()


def test_color_init_then_training():
    """Colour initialisation on the batch (Eq. 3) sets the base colours of the
    visible Gaussians once, and training proceeds from there."""
    cfg, bases, mlp, theta, cams, targets = small(seed=7)
    a = Trainer(cfg, bases, mlp)
    a.set_batch(theta, targets, cams)
    n1 = a.color_init()
    assert 0 < n1 < cfg.N
    c1 = a.bases[0, :, 11:14].cpu().numpy().copy()
    assert not np.array_equal(c1, bases[0, :, 11:14])
    n2 = a.color_init()
    assert n2 == n1 and np.array_equal(a.bases[0, :, 11:14].cpu().numpy(), c1)
    l0 = a.step().loss
    for _ in range(3):
        l1 = a.step().loss
    assert np.isfinite(l1) and l1 < l0
    a.close()


def test_kernel_timing_brackets_count_graph_replays():
    """The wall-clock brackets of a timed kernel run in eager steps and again
    on every replay of a graph captured with timing on, and leave the step's
    results untouched."""
    cfg, bases, mlp, theta, cams, targets = small(seed=4)
    a = Trainer(cfg, bases, mlp)
    a.set_batch(theta, targets, cams)
    b = Trainer(cfg, bases, mlp)
    b.set_batch(theta, targets, cams)
    k = gbr.KERNEL_NAMES.index("composite_bwd")
    la = [a.step().loss for _ in range(6)]
    lb = [b.step().loss]
    gbr.gbr_timing(b.ctx, k, True)
    lb += [b.step().loss for _ in range(2)]
    ev_ms = gbr.gbr_timing_read(b.ctx, k)
    tot, n = gbr.gbr_timing_accum(b.ctx, k, reset=True)
    assert n == 2 and tot > 0.0 and ev_ms > 0.0
    assert 0.2 < (tot / n) / ev_ms < 5.0
    b.capture()
    lb += [b.step().loss for _ in range(3)]
    tot, n = gbr.gbr_timing_accum(b.ctx, k)
    assert n == 3 and tot > 0.0
    gbr.gbr_timing(b.ctx, k, False)
    assert la == lb
    for x, y in zip(state(a), state(b)):
        assert np.array_equal(x, y)
    a.close(); b.close()


@pytest.mark.parametrize("K,paper_mask", [(8, False), (30, True)])
def test_fused_blend_adam_equals_separate_steps(K, paper_mask):
    """The bases' Adam step with the blend adjoint formed inside it
    (gbr_blend_adam_step) leaves every parameter and moment bit for bit where
    the blend adjoint followed by the plain Adam step does, over several
    steps, eagerly and replayed (K = 30 takes the wider slice template)."""
    cfg, bases, mlp, theta, cams, targets = small(seed=6, K=K)
    cfg.paper_mask = paper_mask
    cfg_sep = StepConfig(**{**cfg.__dict__, "fused_adam": False})
    a = Trainer(cfg, bases, mlp)
    b = Trainer(cfg_sep, bases, mlp)
    for tr in (a, b):
        tr.set_batch(theta, targets, cams)
    la = [a.step().loss for _ in range(2)]
    lb = [b.step().loss for _ in range(2)]
    a.capture(); b.capture()
    la += [a.step().loss for _ in range(3)]
    lb += [b.step().loss for _ in range(3)]
    assert la == lb
    for x, y in zip(state(a), state(b)):
        assert np.array_equal(x, y)
    sa, sb = a.step(), b.step()
    assert sa.adam_steps[0] == sb.adam_steps[0] == 6
    a.close(); b.close()


def test_pipelined_steps_equal_one_by_one_and_recover_from_overflow():
    """run_steps enqueues each replay before reading the previous step's
    status: the same updates as one step at a time; with a capacity too
    small for the batch, the overflowed replays update nothing and are run
    again after the capacity grows."""
    cfg, bases, mlp, theta, cams, targets = small(seed=7)
    a = Trainer(cfg, bases, mlp, max_entries=2000)
    b = Trainer(cfg, bases, mlp)
    for tr in (a, b):
        tr.set_batch(theta, targets, cams)
    a.enqueue_step()                    # sizes the other buffers; the entries overflow, nothing updates
    assert gbr.gbr_query_status(a.ctx, a.stream).overflow
    a.capture()                         # captured at the small capacity: its replays overflow
    st = a.run_steps(4)
    assert not st.overflow and st.entries > 2000 and st.adam_steps[0] == 4
    b.step()
    b.capture()
    lb = [b.step().loss for _ in range(3)]
    for x, y in zip(state(a), state(b)):
        assert np.array_equal(x, y)
    assert st.loss == lb[-1]
    st2 = a.run_steps(3, depth=3)
    lb += [b.step().loss for _ in range(3)]
    assert st2.adam_steps[0] == 7 and st2.loss == lb[-1]
    for x, y in zip(state(a), state(b)):
        assert np.array_equal(x, y)
    a.close(); b.close()


def test_replay_after_an_eager_render_uploads_the_captured_frames():
    """A captured step reads its own frame table: an eager render of other
    cameras on the same context leaves the device holding that render's
    table, and the next replay uploads the captured one again (the steps
    equal those of a trainer that rendered nothing in between)."""
    cfg, bases, mlp, theta, cams, targets = small(seed=11)
    cams2 = synth.make_cameras(cfg.B, cfg.width, cfg.height, seed=9)
    a = Trainer(cfg, bases, mlp)
    b = Trainer(cfg, bases, mlp)
    for tr in (a, b):
        tr.set_batch(theta, targets, cams)
        tr.step()
        tr.capture()
        tr.step()
    other = a.torch.zeros(gbr.image_numel(cams2), device="cuda")
    gbr.gbr_render(a.ctx, a.raw, a.offsets, cams2, other)     # same sizes, other poses; b renders nothing
    gbr.gbr_query_status(a.ctx, a.stream)
    assert float(other.abs().sum()) > 0
    la = [a.step().loss for _ in range(2)]
    lb = [b.step().loss for _ in range(2)]
    assert la == lb
    for x, y in zip(state(a), state(b)):
        assert np.array_equal(x, y)
    a.close(); b.close()


def test_status_ring_eager_and_captured_posts():
    """Status posts land in a ring of 4 host records numbered by the device:
    an eager post and the posts at the end of captured steps read back what
    a synchronous read gives; a graph's post counts at each launch; a wait
    for a post never enqueued, or for one that newer posts overwrote, is
    refused."""
    cfg, bases, mlp, theta, cams, targets = small(seed=8)
    a = Trainer(cfg, bases, mlp)
    a.set_batch(theta, targets, cams)
    a.step()
    n0 = gbr.gbr_status_posts(a.ctx)
    gbr.gbr_status_post(a.ctx, a.stream)
    assert gbr.gbr_status_posts(a.ctx) == n0 + 1
    st = gbr.gbr_status_wait(a.ctx, n0 + 1)
    ref = gbr.gbr_query_status(a.ctx, a.stream)
    assert (st.entries, st.loss, list(st.adam_steps)) == (ref.entries, ref.loss, list(ref.adam_steps))
    with pytest.raises(gbr.GbrError):
        gbr.gbr_status_wait(a.ctx, n0 + 2)          # never enqueued
    a.capture()
    assert gbr.gbr_status_posts(a.ctx) == n0 + 1    # capturing runs nothing
    posts = []
    for _ in range(3):
        a._replay()
        posts.append(gbr.gbr_status_posts(a.ctx))
    assert posts == [n0 + 2, n0 + 3, n0 + 4]
    got = [gbr.gbr_status_wait(a.ctx, p) for p in posts]
    assert [g.adam_steps[0] for g in got] == [2, 3, 4]
    final = gbr.gbr_query_status(a.ctx, a.stream)
    assert got[-1].loss == final.loss and got[-1].entries == final.entries and not got[-1].overflow
    for _ in range(5):                              # posts n0+5 .. n0+9: n0+4's record is rewritten
        gbr.gbr_status_post(a.ctx, a.stream)
    a.torch.cuda.synchronize()
    with pytest.raises(gbr.GbrError):
        gbr.gbr_status_wait(a.ctx, n0 + 4)
    assert gbr.gbr_status_wait(a.ctx, n0 + 9).adam_steps[0] == 4
    a.close()


def test_graph_refuses_to_launch_after_its_buffers_moved():
    """A graph keeps the buffer addresses of its capture: after the entry
    capacity grows, launching it returns GBR_ERR_STATE with nothing enqueued,
    and the trainer captures its step again and goes on."""
    import torch
    cfg, bases, mlp, theta, cams, targets = small(seed=4)
    tr = Trainer(cfg, bases, mlp)
    tr.set_batch(theta, targets, cams)
    tr.step()
    tr.capture()
    tr.step()
    st = gbr.gbr_query_status(tr.ctx)
    gbr.gbr_reserve(tr.ctx, st.entries_capacity * 2)
    with pytest.raises(gbr.GbrError) as e:
        gbr.gbr_graph_launch(tr.graph, tr.stream)
    assert e.value.code == -5
    st2 = tr.step()                       # the trainer captures again
    assert tr.graph is not None and not st2.overflow
    torch.cuda.synchronize()
    tr.close()


def test_timing_read_without_a_launch_leaves_no_error():
    """Reading the timer of a kernel that has not run since its timing was
    enabled is refused, and the refusal leaves nothing behind for the next
    call to report."""
    cfg, bases, mlp, theta, cams, targets = small(seed=9)
    a = Trainer(cfg, bases, mlp)
    a.set_batch(theta, targets, cams)
    k = gbr.KERNEL_NAMES.index("composite_bwd")
    gbr.gbr_timing(a.ctx, k, True)
    with pytest.raises(gbr.GbrError):
        gbr.gbr_timing_read(a.ctx, k)
    assert np.isfinite(a.step().loss)
    assert gbr.gbr_timing_read(a.ctx, k) > 0.0
    gbr.gbr_timing(a.ctx, k, False)
    a.close()
