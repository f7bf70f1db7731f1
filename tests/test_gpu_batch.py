"""GPU tests of batches (boltz_batch_*): many problems advanced together with
one launch per phase.

Bars.  A batched step runs the same device code per problem as boltz_step on
that problem alone; with the same collision block size every problem whose
collision uses the 64-bit fixed-point accumulators (sums independent of the
order of the lanes) is reproduced bit for bit, the others (FP32
compare-and-swap accumulation, order-dependent rounding) to 1e-6 relative.
Graph replays of the batched step reproduce the eager steps to the same
bars (bit for bit for the fixed-point problems).  One
problem of the batch is also checked against the FP64 oracle (relative 1e-5
per step).
"""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_mod():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


@pytest.fixture(scope="module")
def lib():
    import paper_1005_5405_amd as pkg

    pkg.load_library()
    return pkg


# uneven problems: sizes, velocity grids (one without the fixed-point
# collide layout), shared and per-cell samples, a periodic one
PROBLEMS = [
    dict(nx=12, ny=9, nv=(8, 8, 8), vmax=3.5, delta=10.0, eps=0.1, n_pairs=1500, sample_group=0, mix16=4),
    dict(nx=5, ny=7, nv=(12, 12, 12), vmax=4.5, delta=3.0, eps=0.2, n_pairs=3000, sample_group=1, mix16=4),
    dict(nx=17, ny=4, nv=(6, 10, 8), vmax=(3.0, 4.0, 3.5), delta=1.0, eps=0.05, n_pairs=700, sample_group=3),
    dict(nx=6, ny=6, nv=(8, 8, 4), vmax=3.0, delta=20.0, eps=0.1, n_pairs=0, sample_group=0),
    dict(nx=9, ny=8, nv=(8, 8, 8), vmax=3.5, delta=5.0, eps=0.1, n_pairs=1000, sample_group=0, bc=1),
    dict(nx=3, ny=2, nv=(24, 24, 24), vmax=5.0, delta=20.0, eps=0.1, n_pairs=20000, sample_group=0, mix16=4),
    # pairs from the continuous Maxwellian (Box-Muller), binned to cells
    dict(nx=7, ny=5, nv=(8, 8, 8), vmax=3.0, delta=5.0, eps=0.1, n_pairs=2000, sample_group=0, flags=4),
]


def _walls(lib, i, nx):
    return lib.Walls(lid_u=0.05 + 0.03 * i, tau_left=1.0 + 0.01 * i, tau_right=1.0, tau_bottom=1.02,
                     tau_top=0.99, tau_bottom_x=(1.0 + 0.03 * np.cos(np.arange(nx))) if i == 2 else None)


def _fill(torch_mod, batch, seed):
    from paper_1005_5405_amd import inputs

    h = batch.empty(0.0)
    for i, p in enumerate(batch.problems):
        batch.view(h, i).copy_(torch_mod.from_numpy(
            inputs.random_field(p.shape, seed=seed + i, scale=0.2).astype(np.float32)).cuda())
    return h


def _singles(lib, block):
    old = os.environ.get("BOLTZ_COLLIDE_BLOCK")
    os.environ["BOLTZ_COLLIDE_BLOCK"] = str(block)
    try:
        return [lib.Boltz(**p) for p in PROBLEMS]
    finally:
        if old is None:
            del os.environ["BOLTZ_COLLIDE_BLOCK"]
        else:
            os.environ["BOLTZ_COLLIDE_BLOCK"] = old


def _fixed_layout(p):
    nv = int(np.prod(p["nv"]))
    return 16 * nv + 50000 <= 160 * 1024


def test_batch_matches_single_problems(lib, torch_mod):
    _say("batch vs single problems")
    batch = lib.Batch(PROBLEMS)
    batch.set_block(512)
    singles = _singles(lib, 512)
    walls = [_walls(lib, i, p["nx"]) for i, p in enumerate(PROBLEMS)]
    a = _fill(torch_mod, batch, 11)
    b = batch.empty()
    ref = [batch.view(a, i).clone() for i in range(batch.count)]
    batch.set_step(7)
    for k in range(3):
        batch.step(a, b, walls)
        a, b = b, a
        for i, s in enumerate(singles):
            out = s.empty()
            s.step(ref[i], out, walls[i] if PROBLEMS[i].get("bc", 0) == 0 else None, 7 + k)
            ref[i] = out
    torch_mod.cuda.synchronize()
    for i in range(batch.count):
        got = batch.view(a, i)
        if _fixed_layout(PROBLEMS[i]):
            assert torch_mod.equal(got, ref[i]), i
        else:
            d = (got - ref[i]).abs().max().item()
            assert d <= 1e-6 * ref[i].abs().max().item(), (i, d)
    for s in singles:
        assert s.read_status() == 0
    # another collision block size changes only the order of the FP64 moment sums
    for blk in (256, 1024):
        try:
            batch.set_block(blk)
        except lib.BoltzError:
            continue
        c = _fill(torch_mod, batch, 11)
        d = batch.empty()
        batch.set_step(7)
        batch.step(c, d, walls)
        batch.set_block(512)
        e = _fill(torch_mod, batch, 11)
        f = batch.empty()
        batch.set_step(7)
        batch.step(e, f, walls)
        torch_mod.cuda.synchronize()
        assert (d - f).abs().max().item() <= 1e-6 * f.abs().max().item(), blk


def test_batch_class_settings_and_stream_tiles(lib, torch_mod):
    """Records per lane, workgroup spread and the stream tile shape change no
    arithmetic: every setting reproduces the default one bit for bit (the
    compare-and-swap layout to 1e-6); all classes at one block size."""
    _say("batch class settings")
    batch = lib.Batch(PROBLEMS)
    walls = [_walls(lib, i, p["nx"]) for i, p in enumerate(PROBLEMS)]

    def run():
        a = _fill(torch_mod, batch, 51)
        b = batch.empty()
        batch.set_step(9)
        for k in range(2):
            batch.step(a, b, walls)
            a, b = b, a
        torch_mod.cuda.synchronize()
        return a

    batch.set_block(512)
    batch.set_stream_tile(16, 8)
    ref = run()
    cls = batch.classes()
    for tile, pu, spread in (((32, 4), 4, 0), ((16, 8), 2, 1), ((32, 4), 2, 2), ((16, 8), 4, 2)):
        batch.set_stream_tile(*tile)
        for k, c in enumerate(cls):
            # the partial-tile layout (24^3 here) runs 1024 threads and at most two workgroups per CU
            part = c["collide_block"] == 1024
            batch.set_class(k, c["collide_block"], pu, min(spread, 1) if part else spread)
        assert batch.stream_tile == tile
        got = run()
        for i in range(batch.count):
            g, r = batch.view(got, i), batch.view(ref, i)
            if _fixed_layout(PROBLEMS[i]):
                assert torch_mod.equal(g, r), (tile, pu, spread, i)
            else:
                assert (g - r).abs().max().item() <= 1e-6 * r.abs().max().item(), (tile, pu, spread, i)


def test_batch_problem_matches_oracle(lib, oracle_mod, torch_mod):
    _say("batch problem vs oracle")
    batch = lib.Batch(PROBLEMS)
    walls = [_walls(lib, i, p["nx"]) for i, p in enumerate(PROBLEMS)]
    a = _fill(torch_mod, batch, 21)
    b = batch.empty()
    batch.set_step(4)
    batch.step(a, b, walls)
    torch_mod.cuda.synchronize()
    for i in (0, 2, 4, 6):
        p = PROBLEMS[i]
        o = oracle_mod.Oracle(**p)
        w = walls[i]
        wo = oracle_mod.Walls(lid_u=w.lid_u, tau_left=w.tau_left, tau_right=w.tau_right, tau_bottom=w.tau_bottom,
                              tau_top=w.tau_top, tau_bottom_x=w.tau_bottom_x) if p.get("bc", 0) == 0 else None
        h = batch.view(a, i).cpu().numpy().astype(np.float64)
        ref = o.step(h, wo, 4)
        got = batch.view(b, i).cpu().numpy().astype(np.float64)
        assert np.abs(got - ref).max() <= 1e-5 * np.abs(ref).max(), i


def test_batch_graph_replays_match_eager_steps(lib, torch_mod):
    _say("batch graph replay")
    batch = lib.Batch(PROBLEMS)
    walls = [_walls(lib, i, p["nx"]) for i, p in enumerate(PROBLEMS)]
    # eager reference: 6 steps from step 3
    a = _fill(torch_mod, batch, 31)
    b = batch.empty()
    batch.set_step(3)
    eager = []
    for k in range(6):
        batch.step(a, b, walls)
        a, b = b, a
        eager.append(a.clone())
    torch_mod.cuda.synchronize()
    # graph of two steps (a -> b -> a), replayed three times
    ga = _fill(torch_mod, batch, 31)
    gb = batch.empty()
    batch.set_step(0)
    batch.step(ga, gb, walls)  # builds the wall tables outside the capture
    torch_mod.cuda.synchronize()
    ga.copy_(_fill(torch_mod, batch, 31))
    side = torch_mod.cuda.Stream()
    side.wait_stream(torch_mod.cuda.current_stream())
    g = torch_mod.cuda.CUDAGraph()
    with torch_mod.cuda.stream(side):
        with torch_mod.cuda.graph(g, stream=side):
            batch.step(ga, gb, walls)
            batch.step(gb, ga, walls)
    torch_mod.cuda.current_stream().wait_stream(side)
    batch.set_step(3)
    for r in range(3):
        g.replay()
        torch_mod.cuda.synchronize()
        for i in range(batch.count):
            got, ref = batch.view(ga, i), batch.view(eager[2 * r + 1], i)
            if _fixed_layout(PROBLEMS[i]):
                assert torch_mod.equal(got, ref), (r, i)
            else:
                assert (got - ref).abs().max().item() <= 1e-6 * ref.abs().max().item(), (r, i)
        # eager work between replays
        tmp = ga.clone()
        torch_mod.cuda.synchronize()
        assert torch_mod.equal(tmp, ga)


def test_batch_tune_and_validation(lib, oracle_mod, torch_mod):
    _say("batch tune")
    batch = lib.Batch(PROBLEMS)
    walls = [_walls(lib, i, p["nx"]) for i, p in enumerate(PROBLEMS)]
    a = _fill(torch_mod, batch, 41)
    b = batch.empty()
    ms = batch.tune(a, b, walls, steps=2)
    assert ms["before"] > 0 and ms["after"] > 0
    # the tuned settings: one class per velocity grid, each within its options
    cls = batch.classes()
    grids = {tuple(p["nv"]) for p in PROBLEMS}
    assert len(cls) == len(grids) == batch.nclasses and {c["nv"] for c in cls} == grids
    assert sum(c["cells"] for c in cls) == sum(p["nx"] * p["ny"] for p in PROBLEMS)
    for c in cls:
        assert c["collide_block"] in (256, 512, 1024) and c["pairs_per_lane"] in (2, 4) and 0 <= c["spread"] <= 2
        assert c["grid"] >= 1 and c["cells_per_group"] == -(-c["cells"] // c["grid"]) and c["ms"] > 0
    assert batch.stream_tile in ((16, 8), (32, 4))
    # a tuned step against the oracle
    a = _fill(torch_mod, batch, 43)
    batch.set_step(5)
    batch.step(a, b, walls)
    torch_mod.cuda.synchronize()
    o = oracle_mod.Oracle(**PROBLEMS[0])
    w = walls[0]
    wo = oracle_mod.Walls(lid_u=w.lid_u, tau_left=w.tau_left, tau_right=w.tau_right, tau_bottom=w.tau_bottom,
                          tau_top=w.tau_top)
    ref = o.step(batch.view(a, 0).cpu().numpy().astype(np.float64), wo, 5)
    got = batch.view(b, 0).cpu().numpy().astype(np.float64)
    assert np.abs(got - ref).max() <= 1e-5 * np.abs(ref).max()
    part = [k for k, c in enumerate(cls) if c["nv"] == (24, 24, 24)]
    assert part and cls[part[0]]["collide_block"] == 1024 and cls[part[0]]["spread"] <= 1
    with pytest.raises(lib.BoltzError):
        batch.set_class(part[0], 512)
    with pytest.raises(lib.BoltzError):
        batch.set_class(part[0], 1024, spread=2)
    with pytest.raises(lib.BoltzError):
        batch.set_class(0, 512, pairs_per_lane=3)
    with pytest.raises(lib.BoltzError):
        batch.set_class(99, 512)
    with pytest.raises(lib.BoltzError):
        batch.set_stream_tile(8, 8)
    with pytest.raises(lib.BoltzError):
        batch.set_block(128)
    with pytest.raises(lib.BoltzError):
        batch.step(a, a, walls)
    with pytest.raises(ValueError):
        batch.step(a, b, walls[:-1])
    # problem contexts of the batch work on their slices
    p0 = batch.problems[0]
    mom = torch_mod.zeros(p0.ncells * 11, dtype=torch_mod.float64, device="cuda")
    D = torch_mod.zeros(1, dtype=torch_mod.float64, device="cuda")
    p0.moments(batch.view(a, 0).contiguous(), mom, walls[0], D)
    torch_mod.cuda.synchronize()
    assert np.isfinite(D.item())
