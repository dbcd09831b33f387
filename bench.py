#!/usr/bin/env python3
"""Benchmark: gamma navigation steps/s on one MI355X (FP64 transport).

One "step" of the benchmark is one transport_batch over the whole workload
(1e6 photons in the Pb/Si sampling calorimeter), i.e. one pass of the hot
path: locate, voxel ComputeStep/ComputeSafety, box distances, physics and
tallies.  The metric counts navigation steps (transport-loop iterations of
single tracks) per second.  Primaries are resident in HBM before timing
starts; geometry upload is excluded, as the paper times only the parallel
phase (Alg. 2, phase 5).

Prints one JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic FP64 work per counted unit (add/mul/compare = 1, fma = 2,
# div and sqrt = 1 each), for box-only geometries such as the calorimeter.
# See the table of per-unit costs in the design notes.
FLOPS = {
    "step": 10,          # s_phys = n_lambda / mu, compare, advance (6), depth update (2)
    "frame": 3,          # touchable frame for an axis-aligned placement (3 sub)
    "dist_out": 12,      # box exit: 3 x (sub, |.|, div) + 3 min
    "dist_in": 33,       # translation (3) + box slab entry (30)
    "safety": 8,         # box signed distance: 3 x (|.|, sub) + 2 max
    "inside": 11,        # translation (3) + box classification (8)
    "node": 10,          # voxel index or exit-plane distance
    "mu": 12,            # log-interpolation of three tables
    "compton": 150,      # Butcher-Messel trial(s), rotation, renormalisation
    "pe": 4,
    "pair": 40,
}

PEAK_FP64_TFLOPS = 78.6  # MI355X vector FP64 (256 CUs x 2.4 GHz x 128 flop/clk)


def algorithmic_flops(c):
    geo = c["steps"] - c["shortcuts"]
    return (FLOPS["step"] * c["steps"] + (FLOPS["frame"] + FLOPS["safety"]) * geo
            + FLOPS["dist_out"] * c["dist_out"] + FLOPS["dist_in"] * c["dist_in"]
            + FLOPS["inside"] * c["inside"] + FLOPS["node"] * c["voxel_nodes"]
            + FLOPS["mu"] * (c["tracks"] + c["compton"])
            + FLOPS["compton"] * c["compton"] + FLOPS["pe"] * c["pe"] + FLOPS["pair"] * c["pair"])


def _oracle_slice(args):
    """Oracle transport of primaries [lo, hi) of the calorimeter workload (worker);
    `voxels` selects the oracle's cell-grid search instead of brute force."""
    n_sample, lo, hi, voxels = args
    import oracle
    import workloads as W
    geoms, prim, _ = W.calorimeter(n=n_sample, seed=0)
    og = oracle.Geometry(geoms[0])
    og.set_voxels(voxels)
    sub = prim.subset(np.arange(lo, hi))
    t0 = time.perf_counter()
    r = og.transport(sub, seed=0, n_events=prim.n_events)
    return r["counters"]["steps"], time.perf_counter() - t0


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n_sample, workers):
    """Oracle steps/s on host cores: one thread over the sample, then `workers`
    processes over equal slices of it (each a plain single-threaded oracle);
    both with brute-force navigation and with the oracle's voxel mode."""
    out = {}
    for voxels in (False, True):
        tag = "voxel_" if voxels else ""
        steps1, dt1 = _oracle_slice((n_sample, 0, n_sample, voxels))
        out[tag + "single"] = (steps1 / dt1, dt1, steps1)
        if workers > 1:
            import multiprocessing as mp
            cuts = np.linspace(0, n_sample, workers + 1).astype(int)
            t0 = time.perf_counter()
            with mp.get_context("fork").Pool(workers) as pool:
                res = pool.map(_oracle_slice, [(n_sample, int(a), int(b), voxels)
                                               for a, b in zip(cuts[:-1], cuts[1:])])
            dt = time.perf_counter() - t0
            steps = sum(r[0] for r in res)
            out[tag + "all"] = (steps / dt, dt, steps)
    return out


def kernel_source_hash():
    """Hash of the transport kernel sources (ties stored counter readings to a build)."""
    import hashlib
    h = hashlib.sha256()
    for f in ("gnav_transport.hip", "gnav_physics.h", "gnav_device.h", "gnav_internal.h"):
        with open(os.path.join(ROOT, "paper_1209_5235_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(kernel):
    """HBM bytes per launch of the headline kernel from the committed counter
    summary, or None when it was taken for another kernel or other sources."""
    path = os.path.join(ROOT, "profiles", "k_transport_calorimeter_1e6_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("kernel_source_hash") != kernel_source_hash() or t.get("kernel") != kernel:
        return None
    return t.get("bytes_per_launch")


def time_batches(ctx, gid, prim_d, tally, stream, reps, **kw):
    """Median kernel time (ms, HIP events on the launch stream) of `reps` batches
    after one warm-up, and the counters of an extra counting batch."""
    import torch
    tally.reset(stream)
    ctx.transport_batch(gid, prim_d, tally, stream=stream, **kw)
    ms = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        tally.reset(stream)
        a.record(stream)
        ctx.transport_batch(gid, prim_d, tally, stream=stream, **kw)
        b.record(stream)
        torch.cuda.synchronize()
        ms.append(a.elapsed_time(b))
    res = tally.read(stream)
    tally.reset(stream)
    ctx.transport_batch(gid, prim_d, tally, stream=stream, count_work=True, **kw)
    work = tally.read(stream)["counters"]
    return float(np.median(ms)), res, work


def oracle_rates(desc, prim, n_sample):
    """Oracle steps/s (one thread) on the first n_sample primaries, brute force and
    voxel mode; the same deterministic subset for both."""
    import oracle
    sub = prim.subset(np.arange(min(n_sample, prim.n)))
    out = {}
    for voxels in (False, True):
        og = oracle.Geometry(desc)
        og.set_voxels(voxels)
        t0 = time.perf_counter()
        r = og.transport(sub, seed=0, n_events=prim.n_events)
        dt = time.perf_counter() - t0
        out["voxel" if voxels else "brute_force"] = r["counters"]["steps"] / dt
    out["sample"] = f"first {sub.n} primaries, one thread"
    return out


def _progress(what):
    print(f"done: {what}", file=sys.stderr, flush=True)


def barrel_variants(ctx, gnav, n, reps, train_photons, oracle_sample=0):
    """Barrel workload: FP64 plain walk against the bound and learned candidate
    orders (identical results) and the two FP32-distance forms."""
    import torch
    import workloads as W
    from paper_1209_5235_amd import learned
    geoms, prim, _ = W.barrel(n=n, seed=0)
    gid, _ = ctx.upload_geometry(geoms[0])
    stream = torch.cuda.current_stream()
    prim_d = gnav.primaries_to_device(prim, "cuda")
    tally = ctx.tally_create(prim.n_events)
    out = {"workload": f"barrel: 64 tubs layers x 128 segments, 2x16 cons rings, 32 orbs; {n:.0e} "
                       "photons from the axis, log-uniform 0.05-20 MeV, seed 0"}
    base_ms, base, base_w = time_batches(ctx, gid, prim_d, tally, stream, reps)
    steps = base["counters"]["steps"]

    def entry(ms, res, work):
        e = {"ms": ms, "steps_per_s": res["counters"]["steps"] / ms * 1e3, "speedup": base_ms / ms,
             "dist_in_fp64": work["dist_in"], "dist_in_fp32": work["dist_in_f32"]}
        same = all(res["counters"][k] == base["counters"][k]
                   for k in ("steps", "pe", "compton", "pair", "crossings", "escaped", "tracks"))
        d = np.abs(res["edep_event"] - base["edep_event"]) / np.maximum(base["edep_event"], 1e-300)
        e["same_counters"] = bool(same)
        e["max_rel_event_deposit_diff"] = float(d[base["edep_event"] > 0].max())
        return e

    out["fp64"] = {"ms": base_ms, "steps_per_s": steps / base_ms * 1e3, "steps": steps,
                   "dist_in_fp64": base_w["dist_in"]}
    if oracle_sample > 0:
        out["fp64"]["oracle_steps_per_s"] = oracle_rates(geoms[0], prim, oracle_sample)
    _progress("barrel fp64")
    out["fp64_bound_order"] = entry(*time_batches(ctx, gid, prim_d, tally, stream, reps, order=1))
    _progress("barrel bound order")
    out["fp32_screened"] = entry(*time_batches(ctx, gid, prim_d, tally, stream, reps, precision=1))
    _progress("barrel fp32 screened")
    pure = entry(*time_batches(ctx, gid, prim_d, tally, stream, reps, precision=2))
    # pure FP32: deposit histogram chi-square per degree of freedom against FP64
    tally.reset(stream)
    ctx.transport_batch(gid, prim_d, tally, stream=stream, precision=2)
    pr = tally.read(stream)
    bins = np.logspace(-3, np.log10(25.0), 41)
    ha = np.histogram(base["edep_event"], bins)[0].astype(float)
    hb = np.histogram(pr["edep_event"], bins)[0].astype(float)
    m = (ha + hb) > 0
    pure["chi2_per_ndf_event_deposits"] = float(np.sum((ha[m] - hb[m]) ** 2 / (ha[m] + hb[m])) /
                                               max(int(m.sum()) - 1, 1))
    pure["pushes"] = pr["counters"]["pushes"]
    pure["stuck"] = pr["counters"]["stuck"]
    out["fp32_pure"] = pure
    _progress("barrel fp32 pure")
    # per-query FP32 error against FP64 (the FP64 query path equals the oracle per query)
    rng = np.random.Generator(np.random.Philox(key=77))
    q = 100_000
    pts = np.column_stack([rng.uniform(-1500, 1500, q), rng.uniform(-1500, 1500, q),
                           rng.uniform(-2900, 2900, q)])
    dirs = W.primaries.isotropic(rng, q)
    pt, dt = torch.from_numpy(pts).cuda(), torch.from_numpy(dirs).cuda()
    s64, l64, _ = ctx.compute_step(gid, pt, dt, with_next=False)
    s32, l32, _ = ctx.compute_step(gid, pt, dt, with_next=False, precision=2)
    s64, l64, s32, l32 = (x.cpu().numpy() for x in (s64, l64, s32, l32))
    fin = np.isfinite(s64) & np.isfinite(s32)
    err = np.abs(s32[fin] - s64[fin])
    out["fp32_pure"]["per_query"] = {
        "queries": q, "limiter_agreement": float(np.mean(l32 == l64)),
        "abs_err_median_mm": float(np.median(err)), "abs_err_p99_mm": float(np.quantile(err, 0.99)),
        "rel_err_p99": float(np.quantile(err / np.maximum(s64[fin], 1.0), 0.99))}
    # learned order: record crossings (other seeds), train on the GPU, time
    if train_photons > 0:
        t0 = time.perf_counter()
        _, tprim, _ = W.barrel(n=train_photons, seed=1)
        rec = learned.record_crossings(ctx, gid, gnav.primaries_to_device(tprim, "cuda"),
                                       tprim.n_events, capacity=8_000_000, seed=1)
        x, cls, label = learned.records_to_tensors(rec)
        t1 = time.perf_counter()
        net, losses = learned.train(ctx, ctx.ordering_classes(gid), x, cls, label, epochs=2, batch=4096)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        ctx.set_mlp(gid, net)
        e = entry(*time_batches(ctx, gid, prim_d, tally, stream, reps, order=2))
        e["training"] = {"crossings": int(x.shape[0]), "epochs": 2, "batch": 4096,
                         "record_s": t1 - t0, "train_s": t2 - t1,
                         "accuracy_top1": learned.accuracy(net, x[:200_000], cls[:200_000],
                                                           label[:200_000])}
        out["fp64_learned_order"] = e
        _progress("barrel learned order")
        ctx.set_mlp(gid, None)
        net.free()
        # the same comparison with bounding-box voxel node lists (as Geant4's smart
        # voxels), where start nodes hold many more candidates
        gid_b, _ = ctx.upload_geometry(geoms[0], voxel_lists=1)
        tally_b = ctx.tally_create(prim.n_events)
        ms_p, res_p, w_p = time_batches(ctx, gid_b, prim_d, tally_b, stream, reps)
        rec = learned.record_crossings(ctx, gid_b, gnav.primaries_to_device(tprim, "cuda"),
                                       tprim.n_events, capacity=8_000_000, seed=1)
        x, cls, label = learned.records_to_tensors(rec)
        net, _ = learned.train(ctx, ctx.ordering_classes(gid_b), x, cls, label, epochs=2, batch=4096)
        ctx.set_mlp(gid_b, net)
        ms_l, res_l, w_l = time_batches(ctx, gid_b, prim_d, tally_b, stream, reps, order=2)
        ms_bo, res_bo, w_bo = time_batches(ctx, gid_b, prim_d, tally_b, stream, reps, order=1)
        ms_s, res_s, w_s = time_batches(ctx, gid_b, prim_d, tally_b, stream, reps, precision=1)
        ms_f, res_f, _ = time_batches(ctx, gid_b, prim_d, tally_b, stream, reps, precision=2)
        keys = ("steps", "pe", "compton", "pair", "crossings", "escaped", "tracks")
        same = all(res_l["counters"][k] == res_p["counters"][k] for k in keys)
        out["bbox_voxel_lists"] = {
            "fp64_ms": ms_p, "fp64_steps_per_s": res_p["counters"]["steps"] / ms_p * 1e3,
            "dist_in_fp64": w_p["dist_in"], "learned_ms": ms_l, "learned_speedup": ms_p / ms_l,
            "learned_dist_in_fp64": w_l["dist_in"], "learned_same_counters": bool(same),
            "bound_order_ms": ms_bo, "bound_order_speedup": ms_p / ms_bo,
            "fp32_screened_ms": ms_s, "fp32_screened_speedup": ms_p / ms_s,
            "fp32_screened_dist_in_fp64": w_s["dist_in"], "fp32_screened_dist_in_fp32": w_s["dist_in_f32"],
            "fp32_screened_same_counters": all(res_s["counters"][k] == res_p["counters"][k] for k in keys),
            "fp32_pure_ms": ms_f, "fp32_pure_speedup": ms_p / ms_f,
            "training_crossings": int(x.shape[0])}
        ctx.set_mlp(gid_b, None)
        net.free()
        tally_b.free()
    tally.free()
    return out


# The paper's Table 1 (Spheres, N = 1e5, free path only), milliseconds, as context.
PAPER_TABLE1_MS = {"regular": {"gtx470": 33, "cpu_1_thread": 442, "cpu_12_threads": 54},
                   "random": {"gtx470": 114, "cpu_1_thread": 458, "cpu_12_threads": 56}}


def paper_free_path(ctx, gnav, reps, oracle_sample):
    """Alg. 1 free path alone on the paper's Spheres geometry with its Random and
    Regular particle sets (mu = rho x 0.06146 cm2/g, Eq. 9), N = 1e5."""
    import torch
    import workloads as W
    desc = W.geometry.spheres()
    gid, _ = ctx.upload_geometry(desc)
    stream = torch.cuda.current_stream()
    out = {"workload": "Spheres: 8000 Al orbs r = 100 mm on a 20^3 grid in a 5 m vacuum cube, "
                       "particles from the centre, mu = rho x 0.06146 cm2/g, N = 1e5, FP64"}
    for name, (pos, dirs, life) in (("random", W.primaries.paper_random(100_000, seed=0)),
                                    ("regular", W.primaries.paper_regular())):
        p, d, y = (torch.from_numpy(a).cuda() for a in (pos, dirs, life))
        ctx.free_path(gid, p, d, y, mu_mass=0.06146, stream=stream)
        ms = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            t, nb = ctx.free_path(gid, p, d, y, mu_mass=0.06146, stream=stream)
            b.record(stream)
            torch.cuda.synchronize()
            ms.append(a.elapsed_time(b))
        m = float(np.median(ms))
        e = {"gpu_ms": m, "particles_per_s": len(life) / m * 1e3,
             "boundaries_per_particle": float(nb.double().mean().cpu()),
             "paper_ms_context": PAPER_TABLE1_MS[name]}
        if oracle_sample > 0:
            import oracle
            og = oracle.Geometry(desc)
            og.set_paper_mode(True, 0.06146)
            t0 = time.perf_counter()
            for i in range(oracle_sample):
                og.free_path(pos[i], dirs[i], 1.0, float(life[i]))
            dt = time.perf_counter() - t0
            e["oracle_particles_per_s"] = oracle_sample / dt
            e["oracle_sample"] = f"first {oracle_sample} particles, one thread, brute-force navigation"
        out[name] = e
    return out


def tiny_config(ctx, gnav, reps, with_oracle):
    """The small configuration: eight boxes in a vacuum world, 1e4 photons of
    1 MeV from the origin (the parity case the oracle runs in seconds)."""
    import torch
    import workloads as W
    geoms, prim, _ = W.tiny(n=10_000, seed=0)
    gid, _ = ctx.upload_geometry(geoms[0])
    prim_d = gnav.primaries_to_device(prim, "cuda")
    tally = ctx.tally_create(prim.n_events)
    ms, res, _ = time_batches(ctx, gid, prim_d, tally, torch.cuda.current_stream(), reps)
    tally.free()
    steps = res["counters"]["steps"]
    out = {"workload": "tiny: 8 water/Pb boxes in a vacuum world, 1e4 photons of 1 MeV from the origin",
           "ms": ms, "steps": steps, "steps_per_s": steps / ms * 1e3}
    if with_oracle:
        out["oracle_steps_per_s"] = oracle_rates(geoms[0], prim, prim.n)
    return out


def batched_config(ctx, gnav, reps):
    """Uneven events over eight resident geometries in one launch: autotuned
    launch settings, then the tuned launch captured in a HIP graph."""
    import torch
    import workloads as W
    t0 = time.perf_counter()
    geoms, prim, event_geom = W.batched()
    gids = [ctx.upload_geometry(g)[0] for g in geoms]
    prim_d = gnav.primaries_to_device(prim, "cuda")
    eg = torch.from_numpy(np.asarray(event_geom, np.int32) + gids[0]).cuda()
    tally = ctx.tally_create(prim.n_events)
    stream = torch.cuda.current_stream()
    setup_s = time.perf_counter() - t0
    kw = dict(event_geom=eg)
    best = ctx.autotune(gids[0], prim_d, tally, trials=2, stream=stream, **kw)
    ms_e, res, _ = time_batches(ctx, gid=gids[0], prim_d=prim_d, tally=tally, stream=stream, reps=reps,
                                tuned=True, **kw)
    g = ctx.graph_create(gids[0], prim_d, tally, stream=stream, tuned=True, **kw)
    ms_g = []
    for _ in range(reps + 1):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        tally.reset(stream)
        a.record(stream)
        ctx.graph_launch(g, stream)
        b.record(stream)
        torch.cuda.synchronize()
        ms_g.append(a.elapsed_time(b))
    gr = tally.read(stream)
    ctx.graph_free(g)
    tally.free()
    steps = res["counters"]["steps"]
    same = gr["counters"] == res["counters"]
    return {"workload": f"batched: {prim.n_events} events, {prim.n} photons (lognormal sizes, median "
                        "2000, 10-50000) over 8 resident geometries (tiny, calorimeter, barrel, 5 barrel "
                        "variants), log-uniform 0.05-20 MeV",
            "photons": int(prim.n), "steps": steps, "tuned": best,
            "ms_eager_tuned": ms_e, "ms_graph_tuned": float(np.median(ms_g[1:])),
            "steps_per_s": steps / float(np.median(ms_g[1:])) * 1e3,
            "graph_same_counters": bool(same), "setup_s": setup_s}


def headline(args, ctx, gnav, cpu, workers):
    """The calorimeter throughput line with its roofline and CPU baseline."""
    import torch
    import workloads as W
    dev = torch.device("cuda:0")
    geoms, prim, _ = W.calorimeter(n=args.n, seed=0)
    gid, nt = ctx.upload_geometry(geoms[0])
    prim_d = gnav.primaries_to_device(prim, dev)
    tally = ctx.tally_create(prim.n_events)
    stream = torch.cuda.current_stream()
    kw = dict(seed=0, block=args.block, grid=args.grid)

    for _ in range(args.warmup):
        tally.reset(stream)
        ctx.transport_batch(gid, prim_d, tally, stream=stream, **kw)
    torch.cuda.synchronize()
    # counters of one batch (identical every batch: counter-keyed random numbers);
    # the work counters (candidate evaluations etc.) come from a counting launch
    tally.reset(stream)
    ctx.transport_batch(gid, prim_d, tally, stream=stream, count_work=True, **kw)
    c = tally.read(stream)["counters"]
    steps_per_batch = c["steps"]

    # timed region: K batches; per-launch durations from events on the launch stream
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        tally.reset(stream)
        starts[i].record(stream)
        ctx.transport_batch(gid, prim_d, tally, stream=stream, **kw)
        ends[i].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    print(f"timed region done: {args.steps} batches in {wall:.3f} s", file=sys.stderr, flush=True)
    kern_ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    avg_kern_s = float(np.mean(kern_ms)) / 1e3
    ms_per_step = wall * 1e3 / args.steps
    value = steps_per_batch * args.steps / wall

    flops = algorithmic_flops(c)
    achieved_tf = flops / avg_kern_s / 1e12
    # 64-slot blocks on a geometry of unrotated boxes run the axis-aligned box build
    block = args.block or 64
    d0 = geoms[0]
    axis_boxes = (block == 64 and bool(np.all(np.asarray(d0.solid_type) == 0)) and
                  bool(np.all(np.asarray(d0.pv_rot).reshape(-1, 9) == np.eye(3).ravel())))
    kernel = f"gnav::pool{block}{'_axis_boxes' if axis_boxes else ''}::k_transport<false, false, 0, 0>"
    traffic = stored_traffic(kernel)
    out = {
        "metric": "gamma navigation steps/s on 1 GPU",
        "value": value,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "sampling calorimeter: 50 Pb 5 mm / Si 10 mm layers x 20x20 cells "
                        "(3-level nesting, voxels), 1e6 photons along +z, log-uniform "
                        "0.1-10 MeV, Gaussian beam sigma 10 mm, FP64, Philox seed 0",
            "photons_per_batch": prim.n,
            "nav_steps_per_batch": steps_per_batch,
            "block": args.block or 64,
            "grid": args.grid or "default",
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved_tf,
            "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved_tf / PEAK_FP64_TFLOPS,
            "traffic": traffic,
            "kernel": kernel,
            "kernel_ms": avg_kern_s * 1e3,
            "flops_per_launch": flops,
            "kernel_source_hash": kernel_source_hash(),
        },
        "counters": c,
    }
    if cpu is not None:
        rate, dt, nsteps = cpu["single"]
        out["cpu_baseline"] = {
            "value": rate, "unit": "steps/s", "cores": 1, "kind": "oracle",
            "cpu": f"{cpu_model()}, {os.cpu_count()} logical CPUs visible",
            "sample": f"first {args.cpu_sample} primaries of the same calorimeter workload "
                      f"({nsteps} steps in {dt:.1f} s, one thread, brute-force navigation)",
        }
        if "all" in cpu:
            rate, dt, nsteps = cpu["all"]
            out["cpu_baseline_all_cores"] = {
                "value": rate, "unit": "steps/s", "cores": workers, "kind": "oracle",
                "sample": f"the same {args.cpu_sample} primaries in {workers} single-threaded "
                          f"oracle processes ({nsteps} steps in {dt:.1f} s wall)"}
        # the oracle's own cell-grid search: a faster CPU method, same answers
        rate, dt, nsteps = cpu["voxel_single"]
        out["cpu_baseline_voxel"] = {
            "value": rate, "unit": "steps/s", "cores": 1, "kind": "oracle, voxel mode",
            "sample": f"the same {args.cpu_sample} primaries, one thread, cell-grid navigation "
                      f"({nsteps} steps in {dt:.1f} s)"}
        if "voxel_all" in cpu:
            rate, dt, nsteps = cpu["voxel_all"]
            out["cpu_baseline_voxel_all_cores"] = {
                "value": rate, "unit": "steps/s", "cores": workers, "kind": "oracle, voxel mode",
                "sample": f"the same {args.cpu_sample} primaries in {workers} single-threaded "
                          f"processes, cell-grid navigation ({nsteps} steps in {dt:.1f} s wall)"}
    tally.free()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1_000_000, help="photons per batch")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--grid", type=int, default=0)
    ap.add_argument("--cpu-sample", type=int, default=1_000_000,
                    help="primaries of the same workload for the oracle timing (0: skip)")
    ap.add_argument("--cpu-workers", type=int, default=0,
                    help="oracle processes for the all-cores figure (0: min(16, cpus))")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--barrel-n", type=int, default=10_000_000,
                    help="photons of the barrel variant comparison (0: skip)")
    ap.add_argument("--train-photons", type=int, default=1_000_000,
                    help="photons whose crossings train the learned order (0: skip)")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-events config")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one 256 MiB device-to-device copy (reference for HBM counters)")
    ap.add_argument("--sections", default="headline,tiny,barrel,paper,batched",
                    help="comma-separated parts to run (profiling runs pick one); without "
                         "'headline' the line carries only the parts that ran")
    args = ap.parse_args()
    sections = set(args.sections.split(","))
    unknown = sections - {"headline", "tiny", "barrel", "paper", "batched"}
    if unknown:
        ap.error(f"unknown sections {sorted(unknown)}")

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the library drives one GPU; --gpus must be 1 (events are independent: "
              "a multi-GPU run would split the event range and sum the tallies)",
              file=sys.stderr)
        sys.exit(2)

    # the CPU baseline runs first, in processes forked before any GPU use
    cpu, workers = None, 0
    if "headline" in sections and not args.no_cpu and args.cpu_sample > 0:
        workers = args.cpu_workers or min(16, os.cpu_count() or 1)
        cpu = cpu_baseline(args.cpu_sample, workers)
        print(f"cpu baseline done: {cpu}", file=sys.stderr, flush=True)

    import torch
    from paper_1209_5235_amd import gnav

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    ctx = gnav.Context(0)
    if args.calibrate_copy:
        src = torch.ones(32 << 20, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    out = headline(args, ctx, gnav, cpu, workers) if "headline" in sections else {}
    if "tiny" in sections:
        out["tiny"] = tiny_config(ctx, gnav, 5, not args.no_cpu)
        _progress("tiny config")
    if "barrel" in sections and args.barrel_n > 0:
        out["variants"] = barrel_variants(ctx, gnav, args.barrel_n, 3, args.train_photons,
                                          0 if args.no_cpu else 20_000)
        print("barrel variants done", file=sys.stderr, flush=True)
    if "paper" in sections:
        out["paper_free_path"] = paper_free_path(ctx, gnav, 5, 0 if args.no_cpu else 3000)
        print("paper free-path config done", file=sys.stderr, flush=True)
    if "batched" in sections and not args.no_batched:
        out["batched"] = batched_config(ctx, gnav, 3)
        print("batched config done", file=sys.stderr, flush=True)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
