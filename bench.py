"""Training-throughput benchmark of the batch-parallel blendshape-avatar step.

Workload (one step): N = 50,000 Gaussians, K = 20 blendshapes, B = 16 frames
of 512 x 512, weight MLP 56 -> 256 -> 256 -> 20, L1 loss with random
backgrounds, full backward to the bases and the MLP, Adam on both -- in
float32.  Synthetic inputs (see paper_2503_12886_amd/synth.py): the targets
are a ground-truth synthetic avatar's renders of the batch, and training
starts from a perturbed copy of it, as in fitting a captured head.

Reports the batched, graph-captured step (one host synchronisation per
step) in images/s, next to the per-frame scheme (one frame per optimisation
step, host synchronisation between preprocess and rasterize) and the naive
batch-parallel scheme (one update per batch, frames rasterised one by one
with a synchronisation each) on the same GPU, the dominant kernel's roofline
position measured with HIP events over the timed region, a per-kernel time
breakdown, the float64 CPU reference timed on a bounded sample, and the
same step with the Gaussians in a mesh's tangent space.  With --k-sweep,
also the graph-captured step time at other blendshape counts.

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")   # the CPU reference leg is single-threaded
ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "train img/s (fwd+bwd, 50k Gaussians, 512²) batched vs per-frame; serve p99 ms"
HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3   # 256 CU x 2.4 GHz x 256 FLOP/clk (packed dual FMA)

# Algorithmic work per contributing (pixel, Gaussian) pair, FP32 operations
# with a fused multiply-add counted as 2:
#  forward: alpha = o * exp(-q/2) with q the conic quadratic form of the
#   offset (12), clamp, 1 - alpha, T (1 - alpha), alpha T (4), colour
#   accumulation (6)  -> 22
#  backward: alpha recomputed (12), T_i recovered (2), w_i = alpha_i T_i (1),
#   dL/dc (3), residual colour update (6), <g, c> and <g, R> (10), dL/dalpha
#   (3), dL/do and dL/dq (3), conic gradient (9), mean gradient (10) -> 59
#  (the cross-lane reduction over a tile's pixels is not counted)
WORKLOAD_TAG = "train_n50k_k20_b16_512"      # names the profiles/ summaries of this workload
FWD_FLOP_PER_PAIR = 22
BWD_FLOP_PER_PAIR = 59


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--per-frame-frames", type=int, default=48)
    ap.add_argument("--naive-steps", type=int, default=4, help="timed steps of the naive batch-parallel scheme")
    ap.add_argument("--k-sweep", type=str, default="",
                    help="comma-separated blendshape counts: graph-captured ms per step at each K")
    ap.add_argument("--tile", type=int, default=16)
    ap.add_argument("--chunk", type=int, default=64)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--quick", action="store_true", help="few steps, no per-frame/CPU legs (for profilers)")
    ap.add_argument("--timed-only", action="store_true",
                    help="the timed region at full length, no other legs (for a profiler's per-kernel averages)")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=2.0)
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="after the run, copy a buffer of this many MiB on the device (a known-size "
                         "reference for hardware byte counters)")
    return ap.parse_args()


def source_hash(files) -> str:
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def make_workload(seed=0, K=20):
    from paper_2503_12886_amd import synth
    from paper_2503_12886_amd.trainer import StepConfig, mlp_pack
    cfg = StepConfig(N=50_000, K=K, B=16, width=512, height=512)
    bases = synth.make_scene(cfg.N, cfg.K, seed=seed)
    mlp = mlp_pack(synth.make_mlp(K=cfg.K, seed=5))
    theta = synth.make_tracking(cfg.B, seed=2)
    cams = synth.make_cameras(cfg.B, cfg.width, cfg.height, seed=1, yaw_deg=10.0)
    targets = np.stack(synth.make_targets(cams, seed=3))
    return cfg, bases, mlp, theta, cams, targets


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py runs on one GPU; --gpus must be 1 "
                                   "(no multi-GPU path is implemented)"}))
        sys.exit(2)
    import torch
    from paper_2503_12886_amd import gbr, synth
    from paper_2503_12886_amd.trainer import Trainer

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    cfg, bases, mlp, theta, cams, targets = make_workload()
    cfg.tile, cfg.chunk = args.tile, args.chunk
    tr = Trainer(cfg, bases, mlp)
    tr.set_batch(theta, targets, cams)
    tr.render_targets()                          # ground-truth avatar's frames
    tr.load_bases(synth.perturb_scene(bases))    # fit from a perturbed start

    # warm-up (sizes the tile-entry buffers), then the dominant kernel from a
    # per-kernel breakdown of one eager step
    for _ in range(3):
        tr.step()
    breakdown = eager_breakdown(tr)
    dominant = max(("composite_fwd", "composite_bwd", "tile_sort", "binning", "gather_bwd", "adam", "blend",
                    "blend_bwd", "preprocess"), key=lambda k: breakdown.get(k, 0.0))
    dom_id = gbr.KERNEL_NAMES.index(dominant)

    # timed region: graph-captured batched steps, one status read per step.
    # The dominant kernel is bracketed on its launch stream by the library's
    # wall-clock stamp kernels, which a graph replays with every step; their
    # device accumulator is cleared when the timed region starts.
    gbr.gbr_timing(tr.ctx, dom_id, True)
    if not args.no_graph:
        tr.capture()
    steps = 5 if args.quick else args.steps
    warm = 2 if args.quick else args.warmup
    if args.no_graph:
        for _ in range(warm):
            tr.step()
    else:
        tr.run_steps(warm)
    torch.cuda.synchronize()
    gbr.gbr_timing_accum(tr.ctx, dom_id, reset=True)
    first_step = tr.steps_launched
    t0 = time.perf_counter()
    if args.no_graph:
        for _ in range(steps):
            st = tr.step()
    else:
        st = tr.run_steps(steps)              # each replay enqueued before the previous step's status read
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dom_total, dom_n = gbr.gbr_timing_accum(tr.ctx, dom_id)
    gbr.gbr_timing(tr.ctx, dom_id, False)
    launched = tr.steps_launched - first_step    # more than steps only if a replay overflowed and ran again
    if dom_n != launched or launched != steps:
        print(f"note: {launched} replays for {steps} steps, {dom_n} bracketed {dominant} launches",
              file=sys.stderr, flush=True)
    ms_step = (t1 - t0) * 1e3 / steps
    value = cfg.B * steps / (t1 - t0)
    dom_avg = dom_total / max(dom_n, 1)
    # contributing pairs of the last timed step (the fit changes the scene, so
    # the pre-region count would not match the timed launches)
    n_contrib = gbr.gbr_inspect(tr.ctx, "n_contrib", cfg.B * cfg.width * cfg.height).astype(np.int64)
    X = int(n_contrib.sum())
    entries = int(st.entries)
    # per-kernel breakdown of one eager step where the timed region ended
    if tr.graph is not None:
        gbr.gbr_graph_destroy(tr.graph)
        tr.graph = None
    breakdown = eager_breakdown(tr)

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "img/s", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "reduced Gaussian blendshape avatar training step: N=50000 Gaussians, K=20, "
                               "B=16 frames 512x512, weight MLP 56-256-256-20, L1 loss, Adam; batched, "
                               "graph-captured, one host sync per step (the status read), each replay "
                               "enqueued before the previous step's status read",
                   "N": cfg.N, "K": cfg.K, "B": cfg.B, "resolution": [cfg.width, cfg.height],
                   "tile": cfg.tile, "chunk": cfg.chunk, "graph": not args.no_graph},
        "entries_per_step": entries, "contributing_pairs_per_step": X,
        "kernels_ms": breakdown,
    }

    # roofline of the dominant kernel
    if dominant in ("composite_fwd", "composite_bwd"):
        per = FWD_FLOP_PER_PAIR if dominant == "composite_fwd" else BWD_FLOP_PER_PAIR
        achieved = X * per / (dom_avg * 1e-3) / 1e12
        roof = {"bound": "alu", "kernel": dominant, "achieved": round(achieved, 3), "peak": FP32_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4),
                "work_per_launch": f"{X} contributing pairs x {per} FLOP", "avg_ms": round(dom_avg, 4),
                "timed_launches": [first_step, launched]}
    else:
        per_entry = {"tile_sort": 8 + 8 + 4 + 4, "binning": 8 + 4}.get(dominant, 0)
        achieved = entries * per_entry / (dom_avg * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": dominant, "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "work_per_launch": f"{entries} entries x {per_entry} B", "avg_ms": round(dom_avg, 4),
                "timed_launches": [first_step, launched]}
    prof = os.path.join(ROOT, "profiles", f"{dominant}_{WORKLOAD_TAG}.traffic.json")
    roof["traffic"] = None
    if os.path.exists(prof):
        meta = json.load(open(prof))
        if meta.get("sources") and meta.get("source_hash") == source_hash(meta["sources"]):
            roof["traffic"] = round(meta["bytes_per_launch"])
    out["roofline"] = roof

    # per-frame scheme on the same GPU
    if not args.quick and not args.timed_only:
        nf = args.per_frame_frames
        tr.per_frame_steps(range(cfg.B))          # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done = 0
        while done < nf:
            k = min(cfg.B, nf - done)
            tr.per_frame_steps(range(k))
            done += k
        torch.cuda.synchronize()
        pf = nf / (time.perf_counter() - t0)
        out["per_frame"] = {"value": round(pf, 2), "unit": "img/s", "frames": nf,
                            "ms_per_frame": round(1e3 / pf, 4), "batched_over_per_frame": round(value / pf, 3)}
        # naive batch-parallel scheme (frames rasterised one by one, a host sync each; one update per batch)
        tr.naive_batch_steps(1)                   # warm-up
        torch.cuda.synchronize()
        ns = args.naive_steps
        t0 = time.perf_counter()
        tr.naive_batch_steps(ns)
        torch.cuda.synchronize()
        nb = cfg.B * ns / (time.perf_counter() - t0)
        out["naive_batch"] = {"value": round(nb, 2), "unit": "img/s", "steps": ns, "frames": cfg.B * ns,
                              "batched_over_naive": round(value / nb, 3)}

    tr.close()

    if args.copy_calib_mib > 0:
        n = args.copy_calib_mib * (1 << 20) // 4
        src = torch.rand(n, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if not args.quick and not args.timed_only:
        out["tangent"] = tangent_leg(args)
    if args.k_sweep:
        out["k_sweep"] = k_sweep_leg([int(k) for k in args.k_sweep.split(",") if k], args)

    if not args.quick and not args.timed_only and not args.no_serve:
        out["serve"] = serve_leg(args.serve_seconds)
    if not args.quick and not args.timed_only and not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(out), flush=True)


SERVE_NS = (20_000, 40_000, 60_000, 80_000, 100_000, 100_000, 50_000, 30_000)


def eager_breakdown(tr) -> dict:
    """Kernel times (ms) of one eager training step, from HIP events around
    each launch on the trainer's stream."""
    from paper_2503_12886_amd import gbr
    for k in range(len(gbr.KERNEL_NAMES)):
        gbr.gbr_timing(tr.ctx, k, True)
    tr.step()
    out = {}
    for k, name in enumerate(gbr.KERNEL_NAMES):
        try:
            out[name] = round(gbr.gbr_timing_read(tr.ctx, k), 4)
        except gbr.GbrError:
            pass
        gbr.gbr_timing(tr.ctx, k, False)
    return out


def serve_leg(seconds: float) -> dict:
    """Animation serving: 8 resident avatars (N above, K=20), Poisson requests at
    2000/s with a tracking vector and a 512x512 camera each, batches formed every
    <= 2 ms, admission by a 2 GiB in-flight memory budget, 3 overlapping slots."""
    from paper_2503_12886_amd import synth
    from paper_2503_12886_amd.serve import AvatarSpec, Batcher, GpuExecutor, Request, Server
    from paper_2503_12886_amd.trainer import mlp_pack
    rate = 2000.0
    bases = [synth.make_scene(n, 20, seed=100 + i) for i, n in enumerate(SERVE_NS)]
    mlps = [mlp_pack(synth.make_mlp(K=20, seed=200 + i)) for i in range(len(SERVE_NS))]
    ex = GpuExecutor(bases, mlps, n_slots=3, max_batch=16, width=512, height=512)
    n = int(rate * seconds)
    t, av, th, yaw = synth.make_request_stream(n, rate, len(SERVE_NS), seed=4)
    cams = synth.make_cameras(n, 512, 512, seed=5)
    warm = [Request(rid=-1 - i, avatar=i, theta=th[0], cam=cams[0], t_arrival=0.0) for i in range(len(SERVE_NS))]
    b = Batcher([AvatarSpec(N=x, K=20) for x in SERVE_NS], budget_bytes=2 << 30, max_batch=16, window_s=0.002)
    Server(b, ex).run(warm)                                  # warm-up (code objects, first launches)
    reqs = [Request(rid=i, avatar=int(av[i]), theta=th[i], cam=cams[i], t_arrival=float(t[i])) for i in range(n)]
    b = Batcher([AvatarSpec(N=x, K=20) for x in SERVE_NS], budget_bytes=2 << 30, max_batch=16, window_s=0.002)
    stats = Server(b, ex).run(reqs)
    ex.close()
    stats.update({"offered_req_per_s": rate, "avatars": list(SERVE_NS), "resolution": [512, 512],
                  "window_ms": 2.0, "budget_bytes": 2 << 30, "slots": 3,
                  "latency": "arrival to render complete on the GPU"})
    return {k: (round(v, 4) if isinstance(v, float) else v) for k, v in stats.items()}


def tangent_leg(args) -> dict:
    """The same batched step with the Gaussians in tangent space (Eq. 4): bound
    to a synthetic head mesh deformed per frame, transformed before the render
    and the gradient carried back; graph-captured ms per step."""
    import torch
    from paper_2503_12886_amd import synth
    from paper_2503_12886_amd.trainer import Trainer, mlp_pack
    cfg, _, mlp, theta, cams, targets = make_workload()
    cfg.tile, cfg.chunk = args.tile, args.chunk
    verts, faces, uv = synth.make_head_mesh()
    vb = synth.deform_mesh(verts, cfg.B, seed=21)
    tri, bary = synth.bind_gaussians(faces, verts, cfg.N, seed=22)
    bases = synth.make_tangent_scene(cfg.N, cfg.K, seed=0)
    tr = Trainer(cfg, bases, mlp)
    tr.bind_mesh(faces, uv, tri, bary, verts.shape[0])
    tr.set_batch(theta, targets, cams, verts=vb)
    tr.render_targets()
    tr.load_bases(synth.perturb_scene(bases, pos_std=5e-4))
    for _ in range(3):
        tr.step()
    tr.capture()
    tr.run_steps(5)
    torch.cuda.synchronize()
    n = 30
    t0 = time.perf_counter()
    tr.run_steps(n)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / n
    # the transform's own cost: frames, forward transform and adjoint, alone
    from paper_2503_12886_amd import gbr
    with torch.cuda.stream(tr.stream):
        for _ in range(3):
            tr._to_deformed()
            gbr.gbr_tangent_backward(tr.ctx, tr.draw_d, tr.tri, tr.frames, tr.draw_t)
        tr.stream.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            tr._to_deformed()
            gbr.gbr_tangent_backward(tr.ctx, tr.draw_d, tr.tri, tr.frames, tr.draw_t)
        tr.stream.synchronize()
        dtx = (time.perf_counter() - t0) / n
    tr.close()
    v = cfg.B / dt
    return {"value": round(v, 2), "unit": "img/s", "ms_per_step": round(dt * 1e3, 4), "steps": n,
            "triangles": int(faces.shape[0]), "transform_ms": round(dtx * 1e3, 4),
            "note": "a surface-bound scene of its own, so the step time is not comparable to the main line; "
                    "transform_ms is the tangent frames, transform and adjoint per step"}


def k_sweep_leg(ks, args) -> dict:
    """Graph-captured ms per batched step at each blendshape count K (the
    paper reports training time linear in K); same N, B, resolution."""
    import torch
    from paper_2503_12886_amd import synth
    from paper_2503_12886_amd.trainer import Trainer
    res = {}
    for k in ks:
        cfg, bases, mlp, theta, cams, targets = make_workload(K=k)
        cfg.tile, cfg.chunk = args.tile, args.chunk
        tr = Trainer(cfg, bases, mlp)
        tr.set_batch(theta, targets, cams)
        tr.render_targets()
        tr.load_bases(synth.perturb_scene(bases))
        for _ in range(3):
            tr.step()
        tr.capture()
        tr.run_steps(5)
        torch.cuda.synchronize()
        n = 30
        t0 = time.perf_counter()
        tr.run_steps(n)
        torch.cuda.synchronize()
        res[str(k)] = round((time.perf_counter() - t0) * 1e3 / n, 4)
        tr.close()
    return {"unit": "ms per step", "steps": 30, "ms": res}


def cpu_baseline(budget_s: float) -> dict:
    """The float64 oracle on this host, one thread, on a bounded sample of the
    same workload: whole frames of the batch (blend, render, L1 loss
    gradient, render adjoint, blend adjoint) until the budget is used, plus
    one Adam update of every parameter amortised over the 16-frame batch."""
    from oracle import blendshape as bs
    from oracle import raster
    cfg, bases, mlp, theta, cams, targets = make_workload()
    from paper_2503_12886_amd import synth
    p = synth.make_mlp(K=cfg.K, seed=5)
    t0 = time.perf_counter()
    psi, cache = bs.mlp_forward(p, theta)
    frames = 0
    dpsi = np.zeros_like(psi)
    while True:
        b = frames % cfg.B
        raw = bs.blend(bases, psi[b:b + 1])[0].astype(np.float32)
        img, _, _, _ = raster.render(raw, cams[b])
        _, G = bs.loss_l1([img], [targets[b]])
        draw, _ = raster.render_grad(raw, cams[b], G[0])
        _, dps = bs.blend_adjoint(draw[None], bases, psi[b:b + 1])
        dpsi[b] = dps[0]
        frames += 1
        if time.perf_counter() - t0 > budget_s:
            break
    t_frames = time.perf_counter() - t0
    t1 = time.perf_counter()
    bs.mlp_backward(p, cache, dpsi)
    flat = bases.astype(np.float64).ravel()
    bs.adam_step(flat, flat * 1e-3, np.zeros_like(flat), np.zeros_like(flat), 1, 1e-3)
    t_adam = time.perf_counter() - t1
    per_img = t_frames / frames + t_adam / cfg.B
    return {"value": round(1.0 / per_img, 5), "unit": "img/s", "cores": 1, "kind": "oracle",
            "sample": f"{frames} frames, cycling over the 16-frame batch (N=50000, K=20, 512x512): float64 blend + "
                      f"render + L1 gradient + "
                      f"render adjoint + blend adjoint, {t_frames:.1f} s; plus one MLP backward and Adam update of "
                      f"all {flat.size} base parameters ({t_adam:.1f} s) amortised over 16 frames",
            "cpu": cpu_model()}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip() + f" ({os.cpu_count()} logical cores visible)"
    except OSError:
        pass
    return "unknown"


if __name__ == "__main__":
    main()
