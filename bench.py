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
same step with the Gaussians in a mesh's tangent space, and the
graph-captured step time at other blendshape counts (--k-sweep, K = 5, 10,
20, 40 by default).

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
    ap.add_argument("--k-sweep", type=str, default="5,10,20,40",
                    help="comma-separated blendshape counts: graph-captured ms per step at each K "
                         "('' skips it; so do --quick and --timed-only)")
    ap.add_argument("--tile", type=int, default=16)
    ap.add_argument("--chunk", type=int, default=64)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=8.0)
    ap.add_argument("--quick", action="store_true", help="few steps, no per-frame/CPU legs (for profilers)")
    ap.add_argument("--timed-only", action="store_true",
                    help="the timed region at full length, no other legs (for a profiler's per-kernel averages)")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-uneven", action="store_true")
    ap.add_argument("--uneven-steps", type=int, default=20)
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
    # contributing pairs where the timed region starts (the fit changes the
    # scene from step to step; counted again where it ends)
    X_first = count_pairs(tr)
    gbr.gbr_timing_accum(tr.ctx, dom_id, reset=True)
    first_step = tr.steps_launched
    record = []
    t0 = time.perf_counter()
    if args.no_graph:
        for _ in range(steps):
            st = tr.step()
            record.append((time.perf_counter(), int(st.entries)))
    else:
        st = tr.run_steps(steps, record=record)   # each replay enqueued before the previous step's status read
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
    # contributing pairs of the last timed step; the roofline uses the mean of
    # the counts where the region starts and ends
    X_last = count_pairs(tr)
    X = (X_first + X_last) // 2
    entries = int(st.entries)
    hits, visible = hit_entries(tr), visible_splats(tr)
    # per-step times: the intervals between consecutive steps' status arrivals
    ts = np.array([t0] + [r[0] for r in record])
    dts = np.diff(ts) * 1e3
    step_stats = {"ms_p10": round(float(np.percentile(dts, 10)), 4),
                  "ms_p50": round(float(np.percentile(dts, 50)), 4),
                  "ms_p90": round(float(np.percentile(dts, 90)), 4),
                  "entries_first": record[0][1] if record else entries,
                  "entries_last": record[-1][1] if record else entries,
                  "contributing_pairs_first": X_first, "contributing_pairs_last": X_last,
                  "note": "interval between consecutive status arrivals (replays are pipelined two deep); "
                          "entries from each step's status, pairs counted where the region starts and ends"}
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
        "entries_per_step": entries, "contributing_pairs_per_step": X, "step_time": step_stats,
        "kernels_ms": breakdown,
        "kernel_roofline": kernel_roofline(breakdown, cfg, X, entries, hits, visible, ms_step),
    }

    # roofline of the dominant kernel
    if dominant in ("composite_fwd", "composite_bwd"):
        per = FWD_FLOP_PER_PAIR if dominant == "composite_fwd" else BWD_FLOP_PER_PAIR
        achieved = X * per / (dom_avg * 1e-3) / 1e12
        roof = {"bound": "alu", "kernel": dominant, "achieved": round(achieved, 3), "peak": FP32_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4),
                "work_per_launch": f"{X} contributing pairs x {per} FLOP (mean of the counts at the timed "
                                   f"region's start, {X_first}, and end, {X_last})",
                "avg_ms": round(dom_avg, 4), "timed_launches": [first_step, launched]}
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
    if not args.quick and not args.timed_only and not args.no_uneven:
        out["uneven"] = uneven_leg(args.uneven_steps)
    if args.k_sweep and not args.quick and not args.timed_only:
        out["k_sweep"] = k_sweep_leg([int(k) for k in args.k_sweep.split(",") if k], args)

    if not args.quick and not args.timed_only and not args.no_serve:
        out["serve"] = serve_leg(args.serve_seconds)
    if not args.quick and not args.timed_only and not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(out), flush=True)


SERVE_NS = (20_000, 40_000, 60_000, 80_000, 100_000, 100_000, 50_000, 30_000)


def count_pairs(tr) -> int:
    """Contributing (pixel, Gaussian) pairs of the context's last pass."""
    from paper_2503_12886_amd import gbr
    npx = sum(c.width * c.height for c in tr.cams)
    return int(gbr.gbr_inspect(tr.ctx, "n_contrib", npx).astype(np.int64).sum())


def hit_entries(tr) -> int:
    """Tile entries of the last pass that some pixel took (the partials the
    backward writes and the gather reads): consumed entries with a nonzero
    contribution byte."""
    from paper_2503_12886_amd import gbr
    t = tr.ctx.tile
    n_tiles = sum(((c.width + t - 1) // t) * ((c.height + t - 1) // t) for c in tr.cams)
    ts = gbr.gbr_inspect(tr.ctx, "tile_start", n_tiles + 1).astype(np.int64)
    last = gbr.gbr_inspect(tr.ctx, "tile_last", n_tiles).astype(np.int64)
    cm = gbr.gbr_inspect(tr.ctx, "cmask", int(ts[-1])) != 0
    pos = np.arange(int(ts[-1])) - np.repeat(ts[:-1], np.diff(ts))
    return int((cm & (pos < np.repeat(last, np.diff(ts)))).sum())


def visible_splats(tr) -> int:
    from paper_2503_12886_amd import gbr
    r = gbr.gbr_inspect(tr.ctx, "rects", tr.cfg.B * tr.cfg.N)
    return int((r[:, 2] >= r[:, 0]).sum())


def kernel_roofline(ms: dict, cfg, X: int, P: int, P_hit: int, visible: int, step_ms: float) -> dict:
    """Each kernel group's algorithmic work against its own bound (times from
    the eager breakdown step), and the step's fraction: the sum over groups of
    work / peak, over the measured step time.  Algorithmic bytes count the 14
    live features of a Gaussian (56 B), not the 16 stored."""
    B, N, K = cfg.B, cfg.N, cfg.K
    G = 56
    npx = B * cfg.width * cfg.height
    n_tiles = B * ((cfg.width + cfg.tile - 1) // cfg.tile) * ((cfg.height + cfg.tile - 1) // cfg.tile)
    mlp_flop = 2 * B * (cfg.d_in * cfg.hidden + cfg.hidden * cfg.hidden + cfg.hidden * K)
    n_mlp = cfg.d_in * cfg.hidden + cfg.hidden + cfg.hidden * cfg.hidden + cfg.hidden + K * cfg.hidden + K
    work = {   # group: (bound, amount, what)
        "blend": ("hbm", (K + 1) * N * G + B * N * G, "bases read, blended Gaussians written"),
        "preprocess": ("hbm", B * N * (G + 48), "blended Gaussians read, 48-B splat records written"),
        "depth_order": ("hbm", visible * 24, "24 B per visible splat (key read, rank written, order written)"),
        "binning": ("hbm", P * 4 + B * N * 8, "each tile entry emitted once (4 B), per-splat count and offset"),
        "tile_scan": ("hbm", n_tiles * 8, "per-tile count read, start written"),
        "tile_sort": ("hbm", n_tiles * 8, "per-tile work read, schedule written"),
        "composite_fwd": ("alu", X * FWD_FLOP_PER_PAIR, f"contributing pairs x {FWD_FLOP_PER_PAIR} FLOP"),
        "loss": ("hbm", npx * 36, "image and target read, image gradient written (3 channels)"),
        "composite_bwd": ("alu", X * BWD_FLOP_PER_PAIR, f"contributing pairs x {BWD_FLOP_PER_PAIR} FLOP"),
        "gather_bwd": ("hbm", P_hit * 36 + B * N * 2 * G, "9-float partial per hit entry, blended Gaussians "
                                                           "read, their gradient written"),
        "blend_bwd": ("hbm", (B + K) * N * G, "draw and delta bases read (dweights)"),
        "adam": ("hbm", B * N * G + (K + 1) * N * G * 6 + n_mlp * 4 * 7,
                 "draw read; bases, m, v read and written; the MLP's parameters, gradient, m, v"),
        "mlp": ("alu", 3 * mlp_flop, "forward, activation gradients and parameter gradients"),
    }
    out, total_s = {}, 0.0
    for k, (bound, amount, what) in work.items():
        t = ms.get(k)
        if not t:
            continue
        if bound == "hbm":
            ideal = amount / (HBM_PEAK_GBS * 1e9)
            out[k] = {"bound": "hbm", "bytes": int(amount), "achieved_GBs": round(amount / (t * 1e-3) / 1e9, 1),
                      "frac": round(ideal / (t * 1e-3), 4), "work": what}
        else:
            ideal = amount / (FP32_VECTOR_PEAK_TFLOPS * 1e12)
            out[k] = {"bound": "alu", "flop": int(amount),
                      "achieved_TFLOPs": round(amount / (t * 1e-3) / 1e12, 3),
                      "frac": round(ideal / (t * 1e-3), 4), "work": what}
        total_s += ideal
    out["step"] = {"frac": round(total_s / (step_ms * 1e-3), 4), "ideal_ms": round(total_s * 1e3, 4),
                   "step_ms": round(step_ms, 4),
                   "note": "sum over kernel groups of work / peak of its bound, over the timed step; peaks "
                           "8 TB/s and 157.3 TFLOP/s"}
    out["counts"] = {"contributing_pairs": X, "entries": P, "hit_entries": P_hit, "visible_splats": visible}
    return out


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
    <= 2 ms, 3 overlapping slots, a 2 GiB device-memory budget: the slots'
    contexts are sized to hold a third of it each (the library's accounting),
    and a request joins a batch only while it fits its slot and the footprint
    of the work in flight fits the budget."""
    from paper_2503_12886_amd import synth
    from paper_2503_12886_amd.serve import (AvatarSpec, Batcher, GpuExecutor, Request, Server, frame_footprint,
                                            slot_spec_for_budget)
    from paper_2503_12886_amd.trainer import mlp_pack
    rate, budget, n_slots, max_batch = 2000.0, 2 << 30, 3, 8
    spec = slot_spec_for_budget(budget, n_slots, SERVE_NS, 512, 512, max_batch)
    bases = [synth.make_scene(n, 20, seed=100 + i) for i, n in enumerate(SERVE_NS)]
    mlps = [mlp_pack(synth.make_mlp(K=20, seed=200 + i)) for i in range(len(SERVE_NS))]
    ex = GpuExecutor(bases, mlps, n_slots=n_slots, max_batch=max_batch, width=512, height=512, slot=spec)
    n = int(rate * seconds)
    t, av, th, yaw = synth.make_request_stream(n, rate, len(SERVE_NS), seed=4)
    cams = synth.make_cameras(n, 512, 512, seed=5)
    avatars = [AvatarSpec(N=x, K=20) for x in SERVE_NS]
    warm = [Request(rid=-1 - i, avatar=i, theta=th[0], cam=cams[0], t_arrival=0.0) for i in range(len(SERVE_NS))]
    b = Batcher(avatars, budget_bytes=budget, max_batch=max_batch, window_s=0.002, slot=spec)
    Server(b, ex).run(warm)                                  # warm-up (code objects, first launches)
    reqs = [Request(rid=i, avatar=int(av[i]), theta=th[i], cam=cams[i], t_arrival=float(t[i])) for i in range(n)]
    b = Batcher(avatars, budget_bytes=budget, max_batch=max_batch, window_s=0.002, slot=spec)
    stats = Server(b, ex).run(reqs)
    held = ex.memory()
    ov = ex.overflows
    ex.close()
    stats.update({"offered_req_per_s": rate, "avatars": list(SERVE_NS), "resolution": [512, 512],
                  "window_ms": 2.0, "budget_bytes": budget, "slots": n_slots, "max_batch": max_batch,
                  "slot_capacity_splats": spec.max_splats, "slot_planned_bytes": spec.bytes,
                  "slots_held_bytes": held, "entry_overflows": ov,
                  "frame_footprint_bytes": {str(x): frame_footprint(x, 512, 512, max(SERVE_NS))
                                            for x in sorted(set(SERVE_NS))},
                  "latency": "arrival to render complete on the GPU",
                  "admission": "a frame's footprint is the library's planned workspace for it (per-splat, "
                               "per-pixel, per-tile, tile bitmap rows at the largest avatar's length, 32 tile "
                               "entries per Gaussian); deferred counts the times the head of the queue waited for "
                               "budget or slot capacity"})
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
    # what stays outside the pass: the per-(frame, triangle) frames (the
    # transform and its adjoint run inside the projection and its adjoint)
    from paper_2503_12886_amd import gbr
    with torch.cuda.stream(tr.stream):
        for _ in range(3):
            gbr.gbr_tangent_frames(tr.ctx, tr.verts, tr.faces, tr.face_uv, tr.frames)
        tr.stream.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            gbr.gbr_tangent_frames(tr.ctx, tr.verts, tr.faces, tr.face_uv, tr.frames)
        tr.stream.synchronize()
        dtx = (time.perf_counter() - t0) / n
    tr.close()
    v = cfg.B / dt
    return {"value": round(v, 2), "unit": "img/s", "ms_per_step": round(dt * 1e3, 4), "steps": n,
            "triangles": int(faces.shape[0]), "frames_ms": round(dtx * 1e3, 4),
            "note": "a surface-bound scene of its own, so the step time is not comparable to the main line; the "
                    "transform and its adjoint run inside the projection and its adjoint; what "
                    "stays apart, frames_ms, is the per-(frame, triangle) frames kernel (a launch per step, host-timed)"}


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


UNEVEN_RES = [(256, 256), (384, 384), (512, 512)]


def uneven_leg(n_steps: int) -> dict:
    """The uneven batch: N = 100,000, K = 20, B = 64 frames of 256/384/512 px
    squares drawn uniformly, camera distance U[0.4, 0.7], random U[0,1]
    targets.  The autotuner times one render + backward per (tile, chunk);
    then a graph-captured step at its pick -- blend, one render of all 64
    frames, L1 loss, render adjoint, dweights, and the bases' Adam step with
    dbases formed inside it -- is replayed with one status read each."""
    import torch
    from paper_2503_12886_amd import gbr, synth
    from paper_2503_12886_amd.trainer import ADAM_BETAS, ADAM_EPS, bases_lr_table
    B, N, K = 64, 100_000, 20
    bases_np = synth.make_scene(N, K, seed=21)
    w_np = synth.make_weights(B, K, seed=22)
    cams = synth.make_cameras(B, seed=23, resolutions=UNEVEN_RES, dist=(0.4, 0.7))
    npx = sum(c.width * c.height for c in cams)
    targets = torch.from_numpy(np.concatenate([t.ravel() for t in synth.make_targets(cams, seed=24)])).cuda()
    ctx = gbr.Context(tile=16, chunk=64, max_frames=B, max_splats=B * N, max_pixels=npx, max_entries=8 * B * N)
    bases = torch.from_numpy(bases_np).cuda()
    m, v = torch.zeros_like(bases), torch.zeros_like(bases)
    w = torch.from_numpy(w_np).cuda()
    dw = torch.empty_like(w)
    raw = torch.empty(B, N, 16, device="cuda")
    draw = torch.empty_like(raw)
    images = torch.empty(3 * npx, device="cuda")
    dimages = torch.empty_like(images)
    offs = [b * N for b in range(B + 1)]
    lr = bases_lr_table()
    gbr.gbr_blend(ctx, bases, w, raw)
    gbr.gbr_render(ctx, raw, offs, cams, images)
    st = gbr.gbr_query_status(ctx)
    if st.overflow:
        gbr.gbr_reserve(ctx, st.entries + st.entries // 4 + 4096)
    tile, chunk, times = gbr.gbr_autotune(ctx, raw, offs, cams, torch.empty_like(images), dimages, draw)
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()           # capture needs a stream of its own (not the null stream)
    torch.cuda.set_stream(stream)

    def enqueue():
        gbr.gbr_blend(ctx, bases, w, raw)
        gbr.gbr_render(ctx, raw, offs, cams, images)
        gbr.gbr_loss(ctx, images, targets, 1, dimages)
        gbr.gbr_render_backward(ctx, dimages, draw)
        gbr.gbr_blend_backward(ctx, draw, bases, w, None, dw)
        gbr.gbr_blend_adam_step(ctx, 0, draw, w, bases, m, v, lr, ADAM_BETAS[0], ADAM_BETAS[1], ADAM_EPS)

    for _ in range(3):                     # eager warm-up at the pick (sizes the entry buffers)
        enqueue()
        st = gbr.gbr_query_status(ctx)
        if st.overflow:
            gbr.gbr_reserve(ctx, st.entries + st.entries // 4 + 4096)
    torch.cuda.synchronize()
    gbr.gbr_graph_begin(ctx, stream)
    try:
        enqueue()
    finally:
        graph = gbr.gbr_graph_end(ctx, stream)
    for _ in range(3):
        gbr.gbr_graph_launch(graph, stream)
        gbr.gbr_query_status(ctx)
    dts, overflowed = [], 0
    t0 = time.perf_counter()
    for _ in range(n_steps):
        ta = time.perf_counter()
        gbr.gbr_graph_launch(graph, stream)
        st = gbr.gbr_query_status(ctx)
        overflowed += int(st.overflow)
        dts.append((time.perf_counter() - ta) * 1e3)
    dt = time.perf_counter() - t0
    torch.cuda.synchronize()
    torch.cuda.set_stream(torch.cuda.default_stream())
    gbr.gbr_graph_destroy(graph)
    ctx.close()
    combos = [f"{t}/{c}" for t in (8, 16, 32) for c in (64, 128, 256)]
    return {"value": round(B * n_steps / dt, 2), "unit": "img/s", "steps": n_steps,
            "ms_per_step": round(dt * 1e3 / n_steps, 4), "ms_p10": round(float(np.percentile(dts, 10)), 4),
            "ms_p90": round(float(np.percentile(dts, 90)), 4), "overflowed_steps": overflowed,
            "entries_per_step": int(st.entries), "pixels": int(npx),
            "autotune": {"tile": tile, "chunk": chunk,
                         "render_backward_ms": {k: round(x, 4) for k, x in zip(combos, times)}},
            "workload": "N=100000, K=20, B=64 frames of 256/384/512 px squares, camera distance U[0.4,0.7]; "
                        "graph-captured step (blend, render, L1 loss, render adjoint, dweights, bases' Adam) "
                        "at the autotuner's tile/chunk, one status read per step (not pipelined)"}


def _oracle_frame(job):
    """One frame of the training step through the float64 oracle."""
    from oracle import blendshape as bs
    from oracle import raster
    bases, psi_b, cam, target, kind = job
    raw = bs.blend(bases, psi_b)[0].astype(np.float32)
    img, _, _, _ = raster.render(raw, cam)
    _, G = (bs.loss_l1 if kind == 1 else bs.loss_l2)([img], [target])
    draw, _ = raster.render_grad(raw, cam, G[0])
    _, dps = bs.blend_adjoint(draw[None], bases, psi_b)
    return dps[0]


def cpu_baseline(budget_s: float) -> dict:
    """The float64 oracle on this host's cores, on bounded samples of the
    workloads: whole frames (blend, render, loss gradient, render adjoint,
    blend adjoint) plus one MLP backward and Adam update of every parameter
    amortised over the batch.  Frames are independent, so the multi-core
    figure renders them in threads (the oracle's C functions release the
    interpreter lock), one per core."""
    from concurrent.futures import ThreadPoolExecutor

    from oracle import blendshape as bs
    from paper_2503_12886_amd import synth
    cfg, bases, mlp, theta, cams, targets = make_workload()
    p = synth.make_mlp(K=cfg.K, seed=5)
    psi, cache = bs.mlp_forward(p, theta)
    jobs = [(bases, psi[b:b + 1], cams[b], targets[b], 1) for b in range(cfg.B)]
    t1 = time.perf_counter()
    bs.mlp_backward(p, cache, np.zeros_like(psi))
    flat = bases.astype(np.float64).ravel()
    bs.adam_step(flat, flat * 1e-3, np.zeros_like(flat), np.zeros_like(flat), 1, 1e-3)
    t_adam = time.perf_counter() - t1
    # one core, the training batch's frames in turn
    t0 = time.perf_counter()
    frames = 0
    while frames < 1 or time.perf_counter() - t0 < budget_s * 0.5:
        _oracle_frame(jobs[frames % cfg.B])
        frames += 1
    t1c = (time.perf_counter() - t0) / frames + t_adam / cfg.B
    # every core: the whole batch once, a frame per thread
    ncores = max(1, min(16, len(os.sched_getaffinity(0))))
    t0 = time.perf_counter()
    with ThreadPoolExecutor(ncores) as ex:
        list(ex.map(_oracle_frame, jobs))
    tmc = (time.perf_counter() - t0 + t_adam) / cfg.B
    # the tiny workload in full: N = 2000, K = 8, one 128 x 128 frame, L2
    tb = synth.make_scene(2000, 8, seed=0)
    tw = synth.make_weights(1, 8, seed=2)
    tcam = synth.fixed_camera(128, 128, 150.0, 0.5, bg=(0.2, 0.3, 0.4))
    tt = synth.make_targets([tcam])[0]
    t0 = time.perf_counter()
    n1 = 0
    while n1 < 3 or time.perf_counter() - t0 < budget_s * 0.15:
        _oracle_frame((tb, tw, tcam, tt, 2))
        f = tb.astype(np.float64).ravel()
        bs.adam_step(f, f * 1e-3, np.zeros_like(f), np.zeros_like(f), 1, 1e-3)
        n1 += 1
    tiny = (time.perf_counter() - t0) / n1
    with ThreadPoolExecutor(ncores) as ex:
        t0 = time.perf_counter()
        list(ex.map(_oracle_frame, [(tb, tw, tcam, tt, 2)] * (4 * ncores)))
        tiny_mc = (time.perf_counter() - t0) / (4 * ncores)
    return {"value": round(1.0 / tmc, 5), "unit": "img/s", "cores": ncores, "kind": "oracle",
            "sample": f"the 16 frames of the training batch (N=50000, K=20, 512x512) once, one frame per thread on "
                      f"{ncores} threads: float64 blend + render + L1 gradient + render adjoint + blend adjoint, "
                      f"plus one MLP backward and Adam update of all {flat.size} base parameters "
                      f"({t_adam:.2f} s) amortised over 16 frames",
            "single_core": {"value": round(1.0 / t1c, 5), "unit": "img/s", "frames": frames},
            "tiny_workload": {"single_core_img_s": round(1.0 / tiny, 3), "multi_core_img_s": round(1.0 / tiny_mc, 3),
                              "frames": n1, "workload": "N=2000, K=8, one 128x128 frame, L2 loss, Adam on all "
                                                        "parameters (single core), frames only (multi-core)"},
            "cpu": cpu_model()}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip() + (f" ({os.cpu_count()} logical cores visible, "
                                                        f"{len(os.sched_getaffinity(0))} usable)")
    except OSError:
        pass
    return "unknown"


if __name__ == "__main__":
    main()
