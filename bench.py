#!/usr/bin/env python
"""Throughput of one time-split Boltzmann step (stream + collide) on one MI355X.

Workload (default): the largest single-GPU configuration, the 200x200-cell
driven cavity with a 24^3 velocity grid on [-5, 5], Kn = 0.01, lid velocity
0.05 sin(0.5 t), 50000 Monte Carlo pairs per cell per step, CFL 0.5,
second-order streaming, FP32 h (2.2 GB per state) with FP64 moment and
correction sums.  The state starts at rest (h = 0) and evolves through the
warm-up steps, so the timed steps act on a developing cavity flow; all data
stay resident in HBM.

Sample sharing: the headline run draws one set of N_t pairs per step that
every cell evaluates with its own h (sample group G = 0, the sharing of the
paper's Sec. 3).  Beside it: the 64x64 cavity (20^3, 20000 pairs) with shared
samples, with an independent Philox stream per cell (G = 1) and with
first-order streaming; the full-length runs (200x200 for 2000 steps with the
lid shear every 10 steps, 64x64 for 1000 steps); the reverse mode; the batch.

One step = boltz_step (wall densities with the step's pair records drawn in
the last face launch, streaming, collision in place).  A second pass over the
same workload calls boltz_stream and boltz_collide with HIP events recorded
between them on the launch stream, to time each kernel group.

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
# Random-address LDS rates on the MI355X, lane-operations per clock and CU,
# measured by a standalone probe with every CU busy: ds_read_b32 (512 threads
# per workgroup) and ds_add_u64 (1024 threads per workgroup).  They bound the
# collision's pair loop: the time its LDS operations take at these rates.
LDS_READ_RATE, LDS_ADD64_RATE = 9.4, 4.43
# The paper's stream+collide rate on its own workload (GTX 260), derived from its printed streaming and
# collision flop rates and its flop counts per node and per cell-step; context only.
PAPER_NODE_UPDATES_PER_S = 1.0e9
# HBM traffic of the collision launch group measured with rocprofv3 counters
# (FETCH_SIZE and WRITE_SIZE in KiB per dispatch, summed over the group's
# kernels), each scaled by what the counter reads for a device copy of the
# state (bench.py --calibrate), per workload (cells, velocity grid, G); valid
# only for the kernel sources whose SHA-256 is recorded (the collide_counters
# summaries under profiles/).
TRAFFIC = {
    # sample_kernel + collide_kernel<1024, true, ACC_PART>
    "200x200_24_G0": {"sha256": "57597daa49de834632e57087beab4a53a322094cd1cfaa93aee33ff37e69ee7d", "fetch_kib": 143.0 + 1085867.5, "fetch_scale": 1.99993,
                      "write_kib": 1171.88 + 2164097.5, "write_scale": 1.0},
    # sample_kernel + collide_kernel<1024, true, ACC_FIXED>
    "64x64_20_G0": {"sha256": "57597daa49de834632e57087beab4a53a322094cd1cfaa93aee33ff37e69ee7d", "fetch_kib": 143.0 + 66042.5, "fetch_scale": 1.99943,
                    "write_kib": 468.75 + 128000.0, "write_scale": 1.0},
}
# VALU instructions (wave64) per dispatch of the per-cell-sample (G = 1)
# collision kernel of the 64x64 cavity, rocprofv3 --pmc SQ_INSTS_VALU; valid
# for the recorded kernel-source SHA-256.
VALU_G1 = {"sha256": "57597daa49de834632e57087beab4a53a322094cd1cfaa93aee33ff37e69ee7d", "valu_insts_per_dispatch": 4.98797e8}
KERNEL_SOURCES = ("adjoint.hpp", "boltz.hip", "collide.hpp", "device_math.hpp", "kernels.hpp", "sequential.hpp")


def kernel_sources_sha256() -> str:
    import hashlib

    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1005_5405_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _workload_key(kw) -> str:
    nv = kw["nv"] if isinstance(kw["nv"], int) else kw["nv"][0]
    return "%dx%d_%d_G%d%s" % (kw["nx"], kw["ny"], nv, kw["sample_group"], "_seq" if kw.get("flags", 0) & 8 else "")


def measured_traffic(kw):
    t = TRAFFIC.get(_workload_key(kw))
    if not t or t["sha256"] != kernel_sources_sha256():
        return None
    return 1024.0 * (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"])


def alu_roofline(v):
    """Vector-instruction issue roofline of the G = 1 collision: every lane
    draws its own pairs (Philox, FP64 geometry, weights), so the kernel is
    bound by VALU issue, not HBM.  Peak: one wave64 VALU instruction per clock
    per CU (four 16-lane SIMDs, four cycles each), 256 CUs at 2.4 GHz =
    3.93e13 lane-instructions/s (the FP32/FP64 vector FMA peaks of 157.3 and
    78.6 TFLOP/s count the same 64 lanes per clock and CU)."""
    peak = N_CU * CLOCK_HZ * 64
    insts = VALU_G1["valu_insts_per_dispatch"]
    ok = insts is not None and VALU_G1["sha256"] == kernel_sources_sha256()
    achieved = insts * 64 / v["t_collide"] if ok else None
    return {"bound": "alu", "unit": "lane-instructions/s", "peak": peak, "achieved": achieved,
            "frac": achieved / peak if ok else None,
            "valu_insts_per_dispatch": insts if ok else None,
            "note": "SQ_INSTS_VALU x 64 lanes over the HIP-event average of the launch"}


def _json_line(d):
    print(json.dumps(d), flush=True)


def _oracle_steps(oracle, preset, ny, threads, seconds_budget, max_steps=50):
    """Full steps of the FP64 oracle on an nx x ny slab of the preset's cavity
    from rest; returns (steps, seconds, threads used, problem)."""
    import numpy as np

    oracle.set_threads(threads)
    kw = preset.problem(ny=ny)
    o = oracle.Oracle(**kw)
    h = np.zeros(o.shape)
    steps, t0 = 0, time.perf_counter()
    while True:
        walls = oracle.Walls(lid_u=preset.lid(steps * o.dt))
        h = o.step(h, walls, steps)
        steps += 1
        if time.perf_counter() - t0 >= seconds_budget or steps >= max_steps:
            break
    return steps, time.perf_counter() - t0, oracle.get_threads(), o, kw


def cpu_baseline(preset, seconds_budget: float):
    """FP64 oracle on the host cores, full steps (walls, streaming, collision
    with its correction) of a slab of the same cavity: the preset's nx, its
    velocity grid, pair count, Knudsen number and time step (dt is set by
    the x spacing, which the slab keeps), fewer rows.  The cost per node and
    per cell does not depend on the row count.  Threads: OMP_NUM_THREADS
    (the host share of one GPU), and one thread (the paper's speed-up
    definition, Sec. 5.2)."""
    import oracle

    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
    # rows so that one multi-threaded step is about a second of work (the
    # oracle draws and scatters ~1e7 pairs per second and thread)
    rows = max(2, min(preset.ny, int(round(threads * 1e7 / (preset.nx * preset.n_pairs)))))
    steps, dt, used, o, kw = _oracle_steps(oracle, preset, rows, threads, seconds_budget)
    nodes = o.nx * o.ny * o.nv
    out = {"value": nodes * steps / dt, "unit": "node-updates/s", "cores": used, "kind": "oracle",
           "nproc": os.cpu_count(),
           "sample": "%d full step(s) from rest of a %dx%d-cell slab of the %s workload (same velocity grid, "
                     "%d pairs/cell, G=%d, dt), FP64, OpenMP over cells on %d threads, %.1f s"
                     % (steps, o.nx, o.ny, preset.name, kw["n_pairs"], kw["sample_group"], used, dt),
           "pairs_per_s": o.nx * o.ny * kw["n_pairs"] * steps / dt}
    s1, d1, u1, o1, _ = _oracle_steps(oracle, preset, 2, 1, max(2.0, seconds_budget / 3), max_steps=20)
    n1 = o1.nx * o1.ny * o1.nv
    out["single_thread"] = {"value": n1 * s1 / d1, "unit": "node-updates/s", "cores": u1,
                            "sample": "%d full step(s) of a %dx%d-cell slab, one thread, %.1f s"
                                      % (s1, o1.nx, o1.ny, d1),
                            "pairs_per_s": o1.nx * o1.ny * kw["n_pairs"] * s1 / d1}
    oracle.set_threads(threads)
    return out


def run_full_length(pkg, torch, preset, sample_group: int):
    """The preset's whole run from rest (its step count, the oscillating lid
    evaluated at the start of every step), with the lid shear D sampled every
    `moments_every` steps (every 10th step at least) on the device; returns the
    D(t) trace, the status word and the wall time."""
    kw = preset.problem(sample_group=sample_group)
    g = pkg.Boltz(**kw)
    every = preset.moments_every or 10
    nsamp = preset.steps // every
    a, b = g.empty(0.0), g.empty()
    mom = torch.empty(g.ncells * 11, dtype=torch.float64, device="cuda")
    D = torch.zeros(nsamp, dtype=torch.float64, device="cuda")
    walls = pkg.Walls(lid_u=preset.lid(0.0))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    k = 0
    for n in range(preset.steps):
        walls.lid_u = preset.lid(n * g.dt)
        g.step(a, b, walls, n)
        a, b = b, a
        if (n + 1) % every == 0 and k < nsamp:
            walls.lid_u = preset.lid((n + 1) * g.dt)
            g.moments(a, mom, walls, D[k:k + 1])
            k += 1
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    status = g.read_status()
    finite = bool(torch.isfinite(a).all().item())
    Dh = D.cpu().numpy()
    t = [(i + 1) * every * g.dt for i in range(nsamp)]
    lid = [preset.lid(x) for x in t]
    del a, b, mom
    torch.cuda.empty_cache()
    return {"workload": preset.name, "sample_group": sample_group, "steps": preset.steps,
            "moments_every": every, "wall_s": wall, "ms_per_step": wall / preset.steps * 1e3,
            "value": g.ncells * g.nv * preset.steps / wall, "status": status, "finite": finite,
            "D_trace": {"t": [round(x, 6) for x in t[:: max(1, nsamp // 50)]],
                        "D": [float("%.6g" % x) for x in Dh[:: max(1, nsamp // 50)]],
                        "lid_u": [float("%.6g" % x) for x in lid[:: max(1, nsamp // 50)]],
                        "samples": nsamp, "stride_shown": max(1, nsamp // 50),
                        "min": float(Dh.min()), "max": float(Dh.max()), "last": float(Dh[-1]),
                        "mean_last_quarter": float(Dh[3 * nsamp // 4:].mean())}}


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
           "state_bytes": 4 * b.nodes, "create_s": t_create,
           "tuned": {"ms_per_step_before": tune_ms["before"], "ms_per_step_after": tune_ms["after"],
                     "stream_tile": list(b.stream_tile),
                     "classes": [{"velocity_grid": list(c["nv"]), "problems": c["problems"], "cells": c["cells"],
                                  "collide_block": c["collide_block"], "pairs_per_lane": c["pairs_per_lane"],
                                  "workgroups": c["grid"], "cells_per_workgroup": c["cells_per_group"],
                                  "collide_ms": c["ms"]} for c in b.classes()],
                     "not_tuned": "the sample group G (part of each problem: it decides which samples a cell "
                                  "uses)"},
           "eager": {"steps": steps, "ms_per_step": ms_eager, "value": b.nodes / (ms_eager * 1e-3),
                     "pairs_per_s": b.pair_cells / (ms_eager * 1e-3), "wall_s": wall_eager},
           "graph": {"steps": 2 * reps, "ms_per_step": ms_graph, "value": b.nodes / (ms_graph * 1e-3),
                     "pairs_per_s": b.pair_cells / (ms_graph * 1e-3), "wall_s": wall_graph},
           "unit": "node-updates/s", "hbm_frac_step": 16 * b.nodes / (ms_graph * 1e-3) / 1e9 / HBM_PEAK_GBS,
           "status_nonzero": int(np.count_nonzero(status)), "finite": finite}
    del g, h_a, h_b, b
    torch.cuda.empty_cache()
    return out


def _roofline(r, kw, g):
    """HBM roofline of the collision launch group (sample + collision
    kernels), 8 B/node per launch over its HIP-event average."""
    nodes, t_c = r["nodes"], r["t_collide"]
    coll_gbs = BYTES_PER_NODE_KERNEL * nodes / t_c / 1e9
    pair_cells = g.ncells * g.n_pairs
    seq = bool(kw.get("flags", 0) & 8)
    kernel = ("sample_kernel + seq_level_kernel + seq_collide_kernel" if seq
              else "collide_kernel + sample_kernel" if kw["sample_group"] != 1 else "collide_kernel")
    note = ("8 B/node (FP32 h read + write) per launch over the HIP-event average of the collision launch group; "
            "its in-place pair loop (4 LDS reads and 4 LDS writes per record, one level of the shared records "
            "at a time, latency-bound at one wavefront per cell), not HBM, sets its time" if seq else
            "8 B/node (FP32 h read + write) per launch over the HIP-event average of the collision "
            "launch group; its pair loop (2 LDS gathers + 4 LDS integer atomic adds per pair and "
            "cell), not HBM, sets its time")
    return {"kernel": kernel,
            "bound": "hbm", "achieved": coll_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": coll_gbs / HBM_PEAK_GBS, "traffic": measured_traffic(kw), "avg_ms": t_c * 1e3,
            "algorithmic_bytes_per_launch": BYTES_PER_NODE_KERNEL * nodes,
            "pair_cells_per_s_in_kernel": pair_cells / t_c,
            "lds_atomic_lane_ops_per_clk_per_cu": (None if seq else
                                                   LDS_ATOMICS_PER_PAIR * pair_cells / t_c / (N_CU * CLOCK_HZ)),
            # per-cell streams (G = 1) draw their pairs in the kernel: vector
            # issue, not the LDS, bounds that pair loop (the ALU roofline)
            "lds_pair_loop": None if (seq or kw["sample_group"] == 1) else _lds_pair_bound(pair_cells, t_c),
            "note": note}


def _lds_pair_bound(pair_cells, t_c):
    """Time the collision's pair loop needs at the probe's random-address LDS
    rates (2 gathers + 4 64-bit adds per pair and cell), against the launch
    group's measured average (which also holds the node phases, the tile
    traffic and the sampler)."""
    clk_per_pair = LDS_READS_PER_PAIR / LDS_READ_RATE + LDS_ATOMICS_PER_PAIR / LDS_ADD64_RATE
    bound = pair_cells * clk_per_pair / (N_CU * CLOCK_HZ)
    return {"bound_ms": bound * 1e3, "frac": bound / t_c, "clk_per_pair_per_cu": clk_per_pair,
            "rates_lane_ops_per_clk_per_cu": {"ds_read_b32": LDS_READ_RATE, "ds_add_u64": LDS_ADD64_RATE},
            "note": "LDS-op time of the pair loop at the rates of a standalone random-address probe, "
                    "divided by the HIP-event average of the whole collision launch group"}


def _stream_kernels(r):
    stream_gbs = BYTES_PER_NODE_KERNEL * r["nodes"] / r["t_stream"] / 1e9
    kw = r["kw"]
    stretched = kw.get("rx", 0.0) not in (0.0, 1.0) or kw.get("ry", 0.0) not in (0.0, 1.0)
    name = ("wall_kernel (+ wallconst_kernel when the walls change) + stream_kernel<1> (each cell's Courant numbers)"
            if stretched else "wall_kernel x2 (+ wallconst_kernel when the walls change) + stream4_kernel")
    return {"kernel": name, "bound": "hbm",
            "avg_ms": r["t_stream"] * 1e3, "achieved": stream_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": stream_gbs / HBM_PEAK_GBS}


def _summary(r, kw, g, steps):
    return {"value": r["value"], "unit": "node-updates/s", "ms_per_step": r["ms_per_step"],
            "pairs_per_s": r["pairs_per_s"], "pairs_per_s_meaning": "pair-cell evaluations (cells x N_t per step)",
            "hbm_frac_step": 2 * BYTES_PER_NODE_KERNEL * r["nodes"] / (r["ms_per_step"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "collide": _roofline(r, kw, g), "stream": _stream_kernels(r), "steps": steps,
            "config": {"cells": [g.nx, g.ny], "velocity_grid": list(g.nv3), "pairs_per_cell": g.n_pairs,
                       "sample_group": kw["sample_group"], "order": g.order, "mix16": kw["mix16"]}}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", default="cavity200")
    ap.add_argument("--sample-group", type=int, default=0, help="cells sharing a pair stream (0 = all)")
    ap.add_argument("--order", type=int, default=None)
    ap.add_argument("--sequential", action="store_true",
                    help="the in-place sequential collision of Alg. 3 instead of the Jacobi form")
    ap.add_argument("--variant", choices=["auto", "skip"], default="auto",
                    help="also time the 64x64 cavity (shared samples, per-cell samples G = 1, order 1)")
    ap.add_argument("--full", choices=["auto", "skip"], default="auto",
                    help="also run the full-length 200x200 (2000 steps, D(t)) and 64x64 (1000 steps) runs")
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
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(requested --gpus %d, WORLD_SIZE %d)" % (args.gpus, world), file=sys.stderr, flush=True)
        sys.exit(2)

    import torch

    import paper_1005_5405_amd as pkg

    over = {"sample_group": args.sample_group}
    if args.order is not None:
        over["order"] = args.order
    if args.sequential:
        over["sequential"] = True
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
        del src, dst
    r = run(pkg, torch, preset, args.steps, args.warmup)
    g, kw, nodes = r["g"], r["kw"], r["nodes"]
    K = args.steps
    hbm_step = 2 * BYTES_PER_NODE_KERNEL * nodes / (r["wall_s"] / K) / 1e9
    line = {"metric": METRIC, "value": r["value"], "unit": "node-updates/s", "n_gpus": 1, "steps": K,
            "warmup": args.warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": preset.name, "cells": [g.nx, g.ny], "velocity_grid": list(g.nv3),
                       "velocity_box": [-preset.vmax, preset.vmax], "pairs_per_cell": g.n_pairs,
                       "sample_group": kw["sample_group"], "order": g.order, "kn": preset.kn,
                       "lid_u": ("%g sin(%g t)" % (preset.lid_u, preset.lid_omega)) if preset.lid_omega > 0
                       else preset.lid_u, "cfl": preset.cfl, "mix16": kw["mix16"], "parallelism": "single GPU",
                       "sequential_update": bool(args.sequential)},
            "pairs_per_s": r["pairs_per_s"],
            "pairs_per_s_meaning": "pair-cell evaluations (cells x N_t per step); with G = 0 every cell "
                                   "evaluates the same N_t drawn pairs",
            "hbm_frac_step": hbm_step / HBM_PEAK_GBS,
            "event_ms_per_step": (r["t_stream"] + r["t_collide"]) * 1e3,
            "kernel_timing": "second pass of the same steps: boltz_stream and boltz_collide called separately "
                             "with HIP events between them on the launch stream",
            "roofline": _roofline(r, kw, g), "kernels": {"stream": _stream_kernels(r)}}
    del r, g
    torch.cuda.empty_cache()
    variants = line.setdefault("variants", {})
    if args.variant == "auto":
        c64 = pkg.PRESETS["cavity64"]
        ks, ws = max(20, K // 2), max(5, args.warmup // 2)
        for name, pre in (("cavity64_G0", c64.with_(sample_group=0)), ("cavity64_G1", c64.with_(sample_group=1)),
                          ("cavity64_G0_order1", c64.with_(sample_group=0, order=1))):
            print("[bench] variant: %s" % name, flush=True)
            v = run(pkg, torch, pre, ks, ws)
            variants[name] = _summary(v, v["kw"], v["g"], ks)
            if name == "cavity64_G1":
                variants[name]["collide"]["alu_roofline"] = alu_roofline(v)
            del v
            torch.cuda.empty_cache()
        # the paper's own discretisation and workload (Sec. 5.1): 160 x 160 cells, 20^3 velocities stretched
        # 0.945 on [-3, 3], delta 1, 6144 pairs from the continuous Maxwellian shared by all cells
        pre = pkg.PRESETS["paper160"].with_(sample_group=0)
        print("[bench] variant: paper160_G0", flush=True)
        v = run(pkg, torch, pre, ks, ws)
        summ = _summary(v, v["kw"], v["g"], ks)
        summ["config"].update({"velocity_box": [-pre.vmax, pre.vmax], "rv": pre.rv, "continuous_pairs": True,
                               "kn": pre.kn, "lid_u": pre.lid_u})
        summ["paper_context"] = {
            "node_updates_per_s": PAPER_NODE_UPDATES_PER_S, "ratio": v["value"] / PAPER_NODE_UPDATES_PER_S,
            "source": "Sec. 5 figures for this workload: streaming ~30 GFLOP/s at 11 flop/node and collision "
                      "~140 GFLOP/s at 713 728 flop per cell-step combined, on a GeForce GTX 260 (192 cores, "
                      "111.9 GB/s, FP32 storage); context, not a target"}
        variants["paper160_G0"] = summ
        del v
        torch.cuda.empty_cache()
        # the in-place sequential collision of Alg. 3 on the same two workloads
        # and the paper-literal configuration: also first-order streaming on
        # spatial cells stretched 0.996 / 0.998 (Sec. 5.1)
        for name, pre in (("cavity64_G0_sequential", c64.with_(sample_group=0, sequential=True)),
                          ("paper160_G0_sequential", pkg.PRESETS["paper160"].with_(sample_group=0, sequential=True)),
                          ("paper160_literal", pkg.PRESETS["paper160_literal"])):
            print("[bench] variant: %s" % name, flush=True)
            v = run(pkg, torch, pre, ks, ws)
            variants[name] = _summary(v, v["kw"], v["g"], ks)
            variants[name]["config"].update({"sequential_update": True, "rx": pre.rx, "ry": pre.ry, "rv": pre.rv,
                                             "continuous_pairs": pre.continuous})
            if name == "paper160_literal":
                variants[name]["paper_context"] = {"node_updates_per_s": PAPER_NODE_UPDATES_PER_S,
                                                   "ratio": v["value"] / PAPER_NODE_UPDATES_PER_S}
            del v
            torch.cuda.empty_cache()
    if args.full == "auto":
        full = variants.setdefault("full_length", {})
        for key in ("cavity200", "cavity64"):
            pre = pkg.PRESETS[key]
            print("[bench] full-length run: %s, %d steps" % (key, pre.steps), flush=True)
            full[key] = run_full_length(pkg, torch, pre, 0)
    if args.adjoint == "auto":
        print("[bench] variant: reverse mode (%d-step window)" % args.window, flush=True)
        pre = pkg.PRESETS["cavity64"].with_(sample_group=0)
        variants["adjoint"] = run_adjoint(pkg, torch, pre, max(10, K // 4), max(3, args.warmup // 4), args.window,
                                          20)
    if args.batch == "auto":
        print("[bench] variant: batch of %d cavities" % args.batch_count, flush=True)
        variants["batch"] = run_batch(pkg, torch, args.batch_count, max(4, K // 10), max(1, args.warmup // 10))
    if args.cpu_baseline == "auto":
        print("[bench] CPU oracle baseline ...", flush=True)
        line["cpu_baseline"] = cpu_baseline(preset, args.cpu_seconds)
    _json_line(line)


if __name__ == "__main__":
    main()
