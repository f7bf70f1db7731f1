#!/usr/bin/env python
"""Throughput of one time-split Boltzmann step (stream + collide) on one MI355X.

Workload (default): the 64x64-cell driven cavity with a 20^3 velocity grid on
[-5, 5], Kn = 0.05, lid velocity 0.1, 20000 Monte Carlo pairs per cell per
step, CFL 0.5, second-order streaming, FP32 h with FP64 moment/correction sums.
The state starts at rest (h = 0) and evolves through the warm-up steps, so the
timed steps act on a developing cavity flow; all data stay resident in HBM.

Sample sharing: the headline run draws one set of N_t pairs per step that
every cell evaluates with its own h (sample group G = 0, the sharing of the
paper's Sec. 3); the variant with an independent Philox stream per cell
(G = 1) is timed in the same process and reported beside it.

One step = boltz_stream (wall densities + streaming kernels) followed by
boltz_collide in place (pair table + collision kernel): exactly what
boltz_step enqueues, with HIP events recorded between the two calls on the
launch stream to time each kernel group.

Prints one JSON line: node-updates/s (value), pairs/s, the HBM roofline of the
dominant kernel group, and the FP64 CPU oracle's throughput on a bounded
sample of the same workload (a baseline only).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "phase-space node-updates/s (stream+collide), collision pairs/s, % HBM peak"
HBM_PEAK_GBS = 8000.0
# Algorithmic HBM bytes per phase-space node and kernel group: one FP32 read
# and one FP32 write of h.  A whole step (stream + collide) moves 16 B/node.
BYTES_PER_NODE_KERNEL = 8
# LDS operations of one pair in one cell in the collision kernel: gathers of
# h_a and h_b and four 64-bit integer atomic adds (Eq. monteCarloInt).
LDS_READS_PER_PAIR, LDS_ATOMICS_PER_PAIR = 2, 4
N_CU, CLOCK_HZ = 256, 2.4e9
# HBM traffic of the collision launch group measured with rocprofv3 counters
# (FETCH_SIZE and WRITE_SIZE in KiB per dispatch, summed over the group's
# kernels), each scaled by what the counter reads for a device copy of the
# 131 MB state (bench.py --calibrate); valid only for the kernel sources whose
# SHA-256 is recorded (profiles/collide_counters_cavity64.md).
TRAFFIC = {"sha256": "7ed1a883756f02f6916d0e3229c0949d38f19b98a378371c3bb8888b550d7563",
           "fetch_kib": 66425.6 + 113.0, "write_kib": 128000.0 + 468.8,
           "fetch_scale": 128000.0 / 64018.4, "write_scale": 1.0}
KERNEL_SOURCES = ("adjoint.hpp", "boltz.hip", "collide.hpp", "device_math.hpp", "kernels.hpp")


def kernel_sources_sha256() -> str:
    import hashlib

    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1005_5405_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    t = TRAFFIC
    if not t["sha256"] or t["sha256"] != kernel_sources_sha256():
        return None
    return 1024.0 * (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"])


def _json_line(d):
    print(json.dumps(d), flush=True)


def cpu_baseline(preset, seconds_budget: float):
    """FP64 oracle on the host cores: full steps of the same workload."""
    import numpy as np

    import oracle

    threads = min(os.cpu_count() or 1, int(os.environ.get("OMP_NUM_THREADS", "16") or 16))
    oracle.set_threads(threads)
    used = oracle.get_threads()
    kw = preset.problem()
    o = oracle.Oracle(**kw)
    walls = oracle.Walls(lid_u=preset.lid(0.0))
    h = np.zeros(o.shape)
    steps, t0 = 0, time.perf_counter()
    while True:
        h = o.step(h, walls, steps)
        steps += 1
        if time.perf_counter() - t0 >= seconds_budget or steps >= 200:
            break
    dt = time.perf_counter() - t0
    ncells, nv = o.nx * o.ny, o.nv
    return {"value": ncells * nv * steps / dt, "unit": "node-updates/s", "cores": used, "kind": "oracle",
            "sample": "%d full step(s) of the same %dx%d-cell, %d-node, %d-pair, G=%d workload from rest, "
                      "FP64, OpenMP over cells, %.1f s" % (steps, o.nx, o.ny, nv, kw["n_pairs"],
                                                           kw["sample_group"], dt),
            "pairs_per_s": ncells * kw["n_pairs"] * steps / dt}


def run(pkg, torch, preset, steps: int, warmup: int):
    """Warm up, then time `steps` whole steps (boltz_step, the entry point of
    the hot path: streaming, then collision, with the step's shared pair
    records drawn in the last face launch).  A second pass of `steps`
    steps over the same workload calls the two halves (boltz_stream,
    boltz_collide) separately with HIP events on the launch stream between
    them: the kernel-group durations (events between launches add ~10 us
    per step, so the throughput comes from the first pass)."""
    kw = preset.problem()
    g = pkg.Boltz(**kw)
    stream = torch.cuda.current_stream()
    a, b = g.empty(0.0), g.empty()
    walls = pkg.Walls(lid_u=preset.lid(0.0))
    n = 0
    for _ in range(warmup):
        walls.lid_u = preset.lid(n * g.dt)
        g.step(a, b, walls, n)
        a, b = b, a
        n += 1
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        walls.lid_u = preset.lid(n * g.dt)
        g.step(a, b, walls, n)
        a, b = b, a
        n += 1
    torch.cuda.synchronize()
    wall_s = time.perf_counter() - t0
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    for k in range(steps):
        walls.lid_u = preset.lid(n * g.dt)
        ev[k][0].record(stream)
        g.stream(a, b, walls)
        ev[k][1].record(stream)
        g.collide(b, b, n)
        ev[k][2].record(stream)
        a, b = b, a
        n += 1
    torch.cuda.synchronize()
    status = g.read_status()
    if status:
        print("[bench] device status %d (numerical failure)" % status, file=sys.stderr, flush=True)
        sys.exit(3)
    t_stream = sum(e[0].elapsed_time(e[1]) for e in ev) / steps * 1e-3
    t_collide = sum(e[1].elapsed_time(e[2]) for e in ev) / steps * 1e-3
    nodes = g.ncells * g.nv
    return dict(g=g, kw=kw, wall_s=wall_s, t_stream=t_stream, t_collide=t_collide, nodes=nodes,
                value=nodes * steps / wall_s, pairs_per_s=g.ncells * g.n_pairs * steps / wall_s,
                ms_per_step=wall_s / steps * 1e3)


def run_adjoint(pkg, torch, preset, steps: int, warmup: int, window: int, every: int):
    """Reverse mode on the same workload with the bottom-wall profile
    T_w(x_i)/T0 = 1 + 0.05 sin(2 pi x_i): boltz_step_adjoint per step (forward
    streaming recomputed, collision adjoint, stream adjoint), its kernel groups
    timed through the separate calls it is made of, and one gradient of the
    time-averaged lid shear over `window` steps from rest with checkpoints
    every `every` steps (forward, segment recomputation, reverse sweep)."""
    import numpy as np

    from paper_1005_5405_amd.window import lid_shear_window

    kw = preset.problem()
    g = pkg.Boltz(**dict(kw, flags=pkg.WITH_ADJOINT))
    stream = torch.cuda.current_stream()
    x = (np.arange(g.nx) + 0.5) / g.nx
    prof = 1.0 + 0.05 * np.sin(2 * np.pi * x)
    walls = pkg.Walls(lid_u=preset.lid(0.0), tau_bottom_x=prof)
    a, b = g.empty(0.0), g.empty()
    for n in range(warmup):
        g.step(a, b, walls, n)
        a, b = b, a
    lam = g.empty_adjoint(0.0)
    lam2 = g.empty_adjoint(0.0)
    grad = torch.zeros(g.grad_size(), dtype=torch.float64, device="cuda")
    mom = torch.empty(g.ncells * 11, dtype=torch.float64, device="cuda")
    g.lid_shear_adjoint(a, walls, 1.0, lam, grad)
    # whole adjoint steps
    for n in range(2):
        g.step_adjoint(a, lam, lam, grad, walls, warmup + n)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for n in range(steps):
        g.step_adjoint(a, lam, lam, grad, walls, warmup + n)
    e1.record(stream)
    torch.cuda.synchronize()
    t_step = e0.elapsed_time(e1) * 1e-3 / steps
    # kernel groups of one adjoint step, through the calls it is made of
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
    for k in range(steps):
        ev[k][0].record(stream)
        g.stream(a, b, walls)
        ev[k][1].record(stream)
        g.collide_adjoint(b, lam, lam, warmup + k)
        ev[k][2].record(stream)
        g.stream_adjoint(a, lam, lam2, grad, walls)
        ev[k][3].record(stream)
        lam, lam2 = lam2, lam
    torch.cuda.synchronize()
    t_fw = sum(e[0].elapsed_time(e[1]) for e in ev) / steps * 1e-3
    t_ca = sum(e[1].elapsed_time(e[2]) for e in ev) / steps * 1e-3
    t_sa = sum(e[2].elapsed_time(e[3]) for e in ev) / steps * 1e-3
    status = g.read_status()
    finite = bool(torch.isfinite(lam).all().item())
    del a, b, lam, lam2, mom
    # windowed gradient
    theta = torch.tensor(np.concatenate([[preset.lid(0.0), 1.0, 1.0, 1.0], prof]), dtype=torch.float64,
                         requires_grad=True)
    h0 = torch.zeros(g.shape, dtype=torch.float32, device="cuda", requires_grad=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J = lid_shear_window(g, h0, theta, window, step0=0, every=every)
    J.backward()
    torch.cuda.synchronize()
    t_win = time.perf_counter() - t0
    # same-seed central differences of the forward map, h = 1e-3
    fd = {}
    for k, name in ((0, "lid_u"), (3, "tau_top"), (4 + g.nx // 4, "tau_bottom_%d" % (g.nx // 4))):
        vals = []
        for sgn in (1.0, -1.0):
            th = theta.detach().clone()
            th[k] += sgn * 1e-3
            with torch.no_grad():
                vals.append(lid_shear_window(g, h0.detach(), th, window, step0=0, every=every).item())
        fd[name] = {"adjoint": float(theta.grad[k]), "fd": (vals[0] - vals[1]) / 2e-3}
    nodes = g.ncells * g.nv
    return {"workload": preset.name + " with bottom profile 1 + 0.05 sin(2 pi x)", "steps": steps,
            "ms_per_adjoint_step": t_step * 1e3, "value": nodes / t_step, "unit": "node-updates/s",
            "status": status, "finite": finite,
            "kernels": {
                "forward_stream_ms": t_fw * 1e3,
                "collide_adjoint": {"kernel": "collide_adj_kernel + sample_kernel", "avg_ms": t_ca * 1e3,
                                    "bound": "lds", "hbm_bytes_per_node": 20,
                                    "hbm_frac": 20 * nodes / t_ca / 1e9 / HBM_PEAK_GBS},
                "stream_adjoint": {"kernel": "wall_kernel x2 + wall_adj_kernel x2 + sweep_adj_kernel x2 + "
                                             "grad_reduce_kernel", "avg_ms": t_sa * 1e3, "bound": "hbm",
                                   "hbm_bytes_per_node": 32,
                                   "hbm_frac": 32 * nodes / t_sa / 1e9 / HBM_PEAK_GBS}},
            "window": {"steps": window, "checkpoint_every": every, "seconds": t_win, "J": J.item(),
                       "gradient_vs_central_differences": fd}}


def batch_problems(count: int, seed: int = 0):
    """Cavities of the batching workload drawn with numpy's default_rng(seed):
    N x N cells with N uniform in 32..128, 16^3, 20^3 or 24^3 velocities on
    [-5, 5], Kn log-uniform in [0.01, 1], lid velocity uniform in [0.05, 0.3]
    (eps = lid velocity), 5000..30000 pairs per cell; shared samples (G = 0),
    mixture share 1/4, order 2, CFL 0.5, one Philox stream per cavity."""
    import numpy as np

    rng = np.random.default_rng(seed)
    probs, lids = [], []
    for i in range(count):
        n = int(rng.integers(32, 129))
        nv = int(rng.choice([16, 20, 24]))
        kn = float(10.0 ** rng.uniform(-2.0, 0.0))
        lid = float(rng.uniform(0.05, 0.3))
        nt = int(rng.integers(5000, 30001))
        probs.append(dict(nx=n, ny=n, nv=nv, vmax=5.0, delta=1.0 / kn, eps=lid, n_pairs=nt, cfl=0.5, order=2,
                          bc=0, sample_group=0, seed=1, cavity_id=i, mix16=4))
        lids.append(lid)
    return probs, lids


def run_batch(pkg, torch, count: int, steps: int, warmup: int):
    """The batching workload: `count` cavities advanced by boltz_batch_step
    (one launch per phase), first eagerly, then as replays of a captured
    two-step HIP graph."""
    import numpy as np

    probs, lids = batch_problems(count)
    t0 = time.perf_counter()
    b = pkg.Batch(probs)
    t_create = time.perf_counter() - t0
    walls = [pkg.Walls(lid_u=u) for u in lids]
    stream = torch.cuda.current_stream()
    h_a, h_b = b.empty(0.0), b.empty(0.0)
    tune_ms = b.tune(h_a, h_b, walls, steps=2)
    h_a.zero_()
    b.set_step(0)
    for _ in range(warmup):
        b.step(h_a, h_b, walls)
        h_a, h_b = h_b, h_a
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        b.step(h_a, h_b, walls)
        h_a, h_b = h_b, h_a
    e1.record(stream)
    torch.cuda.synchronize()
    wall_eager = time.perf_counter() - t0
    ms_eager = e0.elapsed_time(e1) / steps
    # captured graph of two steps (a -> b -> a)
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            b.step(h_a, h_b, walls)
            b.step(h_b, h_a, walls)
    stream.wait_stream(side)
    reps = max(1, steps // 2)
    g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(reps):
        g.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    wall_graph = time.perf_counter() - t0
    ms_graph = e0.elapsed_time(e1) / (2 * reps)
    status = [p.read_status() for p in b.problems]
    finite = bool(torch.isfinite(h_a).all().item())
    classes = {}
    for p in probs:
        classes[str(p["nv"]) + "^3"] = classes.get(str(p["nv"]) + "^3", 0) + 1
    out = {"workload": "%d cavities, N in 32..128, 16^3/20^3/24^3 velocities, Kn log-uniform [0.01, 1], lid "
                       "U[0.05, 0.3], 5000..30000 pairs/cell, G = 0 (numpy default_rng(0))" % count,
           "cavities": count, "velocity_grids": classes, "nodes": b.nodes, "pair_cells": b.pair_cells,
           "state_bytes": 4 * b.nodes, "create_s": t_create, "collide_block": b.collide_block,
           "tune_ms_per_step": {str(k): v for k, v in tune_ms.items()},
           "eager": {"steps": steps, "ms_per_step": ms_eager, "value": b.nodes / (ms_eager * 1e-3),
                     "pairs_per_s": b.pair_cells / (ms_eager * 1e-3), "wall_s": wall_eager},
           "graph": {"steps": 2 * reps, "ms_per_step": ms_graph, "value": b.nodes / (ms_graph * 1e-3),
                     "pairs_per_s": b.pair_cells / (ms_graph * 1e-3), "wall_s": wall_graph},
           "unit": "node-updates/s", "hbm_frac_step": 16 * b.nodes / (ms_graph * 1e-3) / 1e9 / HBM_PEAK_GBS,
           "status_nonzero": int(np.count_nonzero(status)), "finite": finite}
    del g, h_a, h_b, b
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", default="cavity64")
    ap.add_argument("--sample-group", type=int, default=0, help="cells sharing a pair stream (0 = all)")
    ap.add_argument("--order", type=int, default=None)
    ap.add_argument("--variant", choices=["auto", "skip"], default="auto",
                    help="also time the per-cell sample streams (G = 1)")
    ap.add_argument("--adjoint", choices=["auto", "skip"], default="auto",
                    help="also time the reverse mode (step adjoint, windowed lid-shear gradient)")
    ap.add_argument("--window", type=int, default=200, help="steps of the windowed gradient")
    ap.add_argument("--batch", choices=["auto", "skip"], default="auto",
                    help="also time the batching workload (many uneven cavities per step)")
    ap.add_argument("--batch-count", type=int, default=64)
    ap.add_argument("--cpu-baseline", choices=["auto", "skip"], default="auto")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--calibrate", action="store_true",
                    help="first copy the state once on the device (scale of the traffic counters)")
    ap.add_argument("--print-sha", action="store_true", help="print the kernel-source SHA-256 and exit")
    args = ap.parse_args()
    if args.print_sha:
        print(kernel_sources_sha256())
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(requested --gpus %d, WORLD_SIZE %d)" % (args.gpus, world), file=sys.stderr, flush=True)
        sys.exit(2)

    import torch

    import paper_1005_5405_amd as pkg

    over = {"sample_group": args.sample_group}
    if args.order is not None:
        over["order"] = args.order
    preset = pkg.PRESETS[args.config].with_(**over)
    print("[bench] %s: G=%d, warm-up %d + %d timed steps" % (args.config, args.sample_group, args.warmup,
                                                           args.steps), flush=True)
    if args.calibrate:
        n0 = preset.nx * preset.ny * preset.nv ** 3
        src = torch.zeros(n0, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print("[bench] calibration copy: %d bytes" % (4 * n0), flush=True)
    r = run(pkg, torch, preset, args.steps, args.warmup)
    g, kw, nodes = r["g"], r["kw"], r["nodes"]
    K = args.steps
    hbm_step = 2 * BYTES_PER_NODE_KERNEL * nodes / (r["wall_s"] / K) / 1e9
    # dominant kernel group: the collision (pair table + collision kernel)
    t_c = r["t_collide"]
    coll_gbs = BYTES_PER_NODE_KERNEL * nodes / t_c / 1e9
    pair_cells = g.ncells * g.n_pairs
    atom_rate = LDS_ATOMICS_PER_PAIR * pair_cells / t_c / (N_CU * CLOCK_HZ)
    roof = {"kernel": "collide_kernel + sample_kernel" if kw["sample_group"] != 1 else "collide_kernel",
            "bound": "hbm", "achieved": coll_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": coll_gbs / HBM_PEAK_GBS, "traffic": measured_traffic(), "avg_ms": t_c * 1e3,
            "algorithmic_bytes_per_launch": BYTES_PER_NODE_KERNEL * nodes,
            "lds_atomic_lane_ops_per_clk_per_cu": atom_rate,
            "note": "8 B/node (FP32 h read + write) per launch over the HIP-event average of the collision "
                    "launch group; the pair loop is bound by LDS integer atomics (4 per pair and cell), "
                    "whose measured gfx950 rate for random addresses is ~4.4 lane-ops/clk/CU (64-bit)"}
    stream_gbs = BYTES_PER_NODE_KERNEL * nodes / r["t_stream"] / 1e9
    stream_k = {"kernel": "wallconst_kernel (when the walls change) + wall_kernel x2 + stream4_kernel", "bound": "hbm",
                "avg_ms": r["t_stream"] * 1e3, "achieved": stream_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": stream_gbs / HBM_PEAK_GBS}
    line = {"metric": METRIC, "value": r["value"], "unit": "node-updates/s", "n_gpus": 1, "steps": K,
            "warmup": args.warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": preset.name, "cells": [g.nx, g.ny], "velocity_grid": list(g.nv3),
                       "pairs_per_cell": g.n_pairs, "sample_group": kw["sample_group"], "order": g.order,
                       "kn": preset.kn, "lid_u": preset.lid_u, "cfl": preset.cfl, "mix16": kw["mix16"],
                       "parallelism": "single GPU"},
            "pairs_per_s": r["pairs_per_s"], "hbm_frac_step": hbm_step / HBM_PEAK_GBS,
            "event_ms_per_step": (r["t_stream"] + r["t_collide"]) * 1e3,
            "kernel_timing": "second pass of the same steps: boltz_stream and boltz_collide called separately "
                             "with HIP events between them on the launch stream",
            "roofline": roof, "kernels": {"stream": stream_k}}
    if args.variant == "auto" and kw["sample_group"] != 1:
        print("[bench] variant: per-cell sample streams (G=1)", flush=True)
        v = run(pkg, torch, preset.with_(sample_group=1), max(10, K // 4), max(3, args.warmup // 4))
        line["variants"] = {"per_cell_samples_G1": {
            "value": v["value"], "ms_per_step": v["ms_per_step"], "pairs_per_s": v["pairs_per_s"],
            "collide_ms": v["t_collide"] * 1e3, "stream_ms": v["t_stream"] * 1e3,
            "steps": max(10, K // 4)}}
    if args.adjoint == "auto":
        print("[bench] variant: reverse mode (%d-step window)" % args.window, flush=True)
        line.setdefault("variants", {})["adjoint"] = run_adjoint(
            pkg, torch, preset, max(10, K // 4), max(3, args.warmup // 4), args.window, 20)
    if args.batch == "auto":
        print("[bench] variant: batch of %d cavities" % args.batch_count, flush=True)
        line.setdefault("variants", {})["batch"] = run_batch(pkg, torch, args.batch_count, max(4, K // 10),
                                                             max(1, args.warmup // 10))
    if args.cpu_baseline == "auto":
        print("[bench] CPU oracle baseline ...", flush=True)
        line["cpu_baseline"] = cpu_baseline(preset, args.cpu_seconds)
    _json_line(line)


if __name__ == "__main__":
    main()
