"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Bars: node indices and Philox words bit-exact; h
within a relative 1e-5 per step and 1e-4 after 100 steps, measured as
max|h_gpu - h_ref| / max|h_ref|; the same bar on the Maxwellian-weighted
error max_j w_j |dh_j| / max_j w_j |h_ref,j|, which is not dominated by the
rarely visited tail nodes.  Moments are FP64 sums of the same FP32 data on
both sides.
"""
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


def _pair(lib, oracle_mod, **kw):
    return lib.Boltz(**kw), oracle_mod.Oracle(**kw)


def _dev(torch_mod, a):
    return torch_mod.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _errs(o, got, ref):
    d = np.abs(got - ref)
    rel = d.max() / max(np.abs(ref).max(), 1e-300)
    w = o.node_weights()
    wrel = (d * w).max() / max((np.abs(ref) * w).max(), 1e-300)
    return rel, wrel


WALLS = dict(lid_u=0.1, tau_left=1.05, tau_right=0.97, tau_bottom=1.02, tau_top=1.0)


def test_thresholds_bitwise(lib, oracle_mod, torch_mod):
    for nv, a in [((12, 12, 12), 4.5), ((20, 20, 20), 5.0), ((24, 24, 24), 5.0), ((7, 5, 9), (3.0, 2.5, 3.5))]:
        _say("thresholds", nv, a)
        g, o = _pair(lib, oracle_mod, nx=2, ny=2, nv=nv, vmax=a, delta=1.0, eps=0.1, n_pairs=10)
        for k in range(3):
            np.testing.assert_array_equal(g.axis_thresholds(k), o.thresholds[k])
        assert g.dt == o.dt and g.K == o.K and g.W == o.W and g.qfac == o.qfac
        assert np.all(o.thresholds[0] <= 4096)


PAIR_GRIDS = [((12, 12, 12), 4.5), ((20, 20, 20), 5.0), ((24, 24, 24), 5.0), ((7, 5, 9), (3.0, 2.5, 3.5)),
              ((6, 6, 6), 3.0)]


# the Maxwellian law alone (mix16 = 0) only on grids where it reaches every
# node (the others are refused by both sides before any device call)
@pytest.mark.parametrize("grid,G,mix16", [(g, G, m) for g in PAIR_GRIDS for G, m in [(1, 4), (0, 4), (5, 16)]] +
                         [(((6, 6, 6), 3.0), 1, 0), (((7, 5, 7), (3.0, 2.5, 3.0)), 1, 0)])
def test_pairs_bit_exact(lib, oracle_mod, torch_mod, grid, G, mix16):
    nv, a = grid
    g, o = _pair(lib, oracle_mod, nx=7, ny=6, nv=nv, vmax=a, delta=3.0, eps=0.1, n_pairs=50000,
                 sample_group=G, seed=0x1234567890ABCDEF, cavity_id=3, mix16=mix16)
    for cell, step, m0, count in [(0, 0, 0, 40000), (41, 123456789, 7, 20000), (17, 5, 2**31 - 5000, 5000)]:
        _say("pairs", nv, "G", G, "mix16", mix16, "cell", cell, "step", step, "m0", m0)
        gi, gq, gw = g.debug_pairs(cell, step, m0, count, words=True)
        oi, oq, ow = o.debug_pairs(cell, step, m0, count, words=True)
        np.testing.assert_array_equal(gw, ow)
        np.testing.assert_array_equal(gi, oi)
        # the kernel forms the importance weight in FP32 (weights of extreme
        # tail pairs fall into the FP32 subnormal range: absolute floor)
        np.testing.assert_allclose(gq, oq, rtol=2e-6, atol=1e-12 * oq.max())


STREAM_CASES = [
    dict(order=2, bc=0, nx=16, ny=16, nv=(12, 12, 12), vmax=4.5),
    dict(order=1, bc=0, nx=16, ny=16, nv=(12, 12, 12), vmax=4.5),
    dict(order=2, bc=0, nx=13, ny=11, nv=(8, 6, 5), vmax=(3.5, 3.0, 2.5)),   # ragged tiles, nv % 32 != 0
    dict(order=1, bc=0, nx=9, ny=3, nv=(5, 7, 3), vmax=(3.0, 3.5, 2.0)),     # odd grids, v = 0 nodes
    dict(order=2, bc=1, nx=10, ny=9, nv=(6, 6, 6), vmax=3.0),
    dict(order=1, bc=1, nx=5, ny=12, nv=(6, 4, 4), vmax=3.0),
    dict(order=2, bc=0, nx=2, ny=2, nv=(4, 4, 4), vmax=2.5),                 # smallest cavity
    dict(order=2, bc=0, nx=13, ny=11, nv=(6, 4, 8), vmax=(3.0, 2.5, 3.5)),   # vector kernel, ragged tiles
    dict(order=2, bc=1, nx=10, ny=9, nv=(4, 6, 4), vmax=3.0),                # vector kernel, periodic
    dict(order=1, bc=0, nx=17, ny=9, nv=(5, 3, 4), vmax=(3.0, 2.0, 2.5)),    # vector kernel, v_x = 0 nodes
]


@pytest.mark.parametrize("case", range(len(STREAM_CASES)))
def test_stream_parity(lib, oracle_mod, torch_mod, case):
    from paper_1005_5405_amd import inputs

    kw = dict(STREAM_CASES[case], delta=5.0, eps=0.1, n_pairs=100)
    _say("stream", kw)
    g, o = _pair(lib, oracle_mod, **kw)
    h = inputs.random_field(o.shape, seed=10 + case, scale=0.5).astype(np.float32).astype(np.float64)
    walls_o = oracle_mod.Walls(**WALLS) if kw["bc"] == 0 else None
    walls_g = lib.Walls(**WALLS) if kw["bc"] == 0 else None
    ref = o.stream(h, walls_o)
    hin, hout = _dev(torch_mod, h), g.empty()
    g.stream(hin, hout, walls_g)
    torch_mod.cuda.synchronize()
    rel, wrel = _errs(o, _host(hout), ref)
    assert rel <= 1e-5 and wrel <= 1e-5, (rel, wrel)
    # a uniform state and h = 0 with walls at rest are reproduced exactly
    for c in (0.0, 0.25):
        hu = np.full(o.shape, c)
        g.stream(_dev(torch_mod, hu), hout, lib.Walls() if kw["bc"] == 0 else None)
        torch_mod.cuda.synchronize()
        assert np.abs(_host(hout) - c).max() <= (0.0 if c == 0.0 else 2e-6)


COLLIDE_CASES = [
    dict(nx=5, ny=4, nv=(12, 12, 12), vmax=4.5, delta=10.0, eps=0.1, n_pairs=2000),
    dict(nx=3, ny=3, nv=(20, 20, 20), vmax=5.0, delta=20.0, eps=0.1, n_pairs=20000, mix16=4),
    dict(nx=2, ny=2, nv=(24, 24, 24), vmax=5.0, delta=100.0, eps=0.05, n_pairs=50000, mix16=4),
    dict(nx=3, ny=2, nv=(5, 7, 3), vmax=(3.0, 3.5, 2.0), delta=2.0, eps=0.3, n_pairs=3000),  # nv % 4 != 0
    dict(nx=2, ny=2, nv=(26, 26, 26), vmax=5.0, delta=1.0, eps=0.1, n_pairs=5000, mix16=16),  # largest LDS tile
    # 22 of 25 x-slabs of h in LDS, the others gathered from global memory; nv_z % 4 != 0
    dict(nx=3, ny=2, nv=(25, 24, 23), vmax=5.0, delta=50.0, eps=0.05, n_pairs=30000, mix16=4),
    dict(nx=4, ny=4, nv=(12, 12, 12), vmax=4.5, delta=10.0, eps=0.1, n_pairs=2000, sample_group=0),
    dict(nx=5, ny=3, nv=(20, 20, 20), vmax=5.0, delta=20.0, eps=0.1, n_pairs=20000, sample_group=4, mix16=4),
    dict(nx=4, ny=4, nv=(12, 12, 12), vmax=4.5, delta=10.0, eps=0.1, n_pairs=0),
    # shared records: whole 1024-record blocks only (every record dealt to lanes), and fewer
    # records than one block (none dealt)
    dict(nx=3, ny=3, nv=(12, 12, 12), vmax=4.5, delta=10.0, eps=0.1, n_pairs=2048, sample_group=0, mix16=4),
    dict(nx=3, ny=3, nv=(20, 20, 20), vmax=5.0, delta=20.0, eps=0.1, n_pairs=700, sample_group=0),
    # two passes over the pairs, half of the nodes each (grids too large for one pass)
    dict(nx=3, ny=2, nv=(24, 24, 24), vmax=5.0, delta=20.0, eps=0.1, n_pairs=20000, sample_group=0, mix16=4),
    dict(nx=2, ny=2, nv=(25, 25, 23), vmax=5.0, delta=10.0, eps=0.1, n_pairs=20000, sample_group=0, mix16=4),
]


@pytest.mark.parametrize("case", range(len(COLLIDE_CASES)))
@pytest.mark.parametrize("correction", [True, False])
def test_collide_parity(lib, oracle_mod, torch_mod, case, correction):
    from paper_1005_5405_amd import inputs

    kw = dict(COLLIDE_CASES[case], bc=1)
    _say("collide", kw, "correction", correction)
    g, o = _pair(lib, oracle_mod, **kw)
    V = o.node_velocities()
    h = np.stack([inputs.velocity_polynomial(V, seed=100 + c) for c in range(o.nx * o.ny)]).reshape(o.shape)
    h = (h + inputs.random_field(o.shape, seed=7, scale=0.05)).astype(np.float32).astype(np.float64)
    ref = o.collide(h, 42, correction=correction)
    hs, hout = _dev(torch_mod, h), g.empty()
    defect = torch_mod.zeros(o.nx * o.ny * 5, dtype=torch_mod.float64, device="cuda")
    g.collide(hs, hout, 42, correction=correction, defect=defect)
    torch_mod.cuda.synchronize()
    got = _host(hout)
    rel, wrel = _errs(o, got, ref)
    assert rel <= 1e-5 and wrel <= 1e-5, (rel, wrel)
    if kw["n_pairs"] == 0:
        np.testing.assert_array_equal(got, h)
    # in-place call gives the same result
    g.collide(hs, hs, 42, correction=correction)
    torch_mod.cuda.synchronize()
    assert np.abs(_host(hs) - got).max() <= 1e-6 * np.abs(got).max()
    # the device-reported defect is that of the stored FP32 values
    w = o.node_weights()
    psi = np.stack([np.ones(len(w)), V[:, 0], V[:, 1], V[:, 2], (V**2).sum(1)], 1)
    d_host = o.eps * np.einsum("j,jk,ycj->yck", w, psi, got - h).reshape(-1, 5)
    d_dev = defect.cpu().numpy().reshape(-1, 5)
    scale = o.eps * np.einsum("j,jk,ycj->yck", w, np.abs(psi), np.abs(got) + np.abs(h)).reshape(-1, 5)
    assert np.all(np.abs(d_dev - d_host) <= 1e-12 * scale)
    if correction:
        # conservation up to FP32 storage of h
        assert np.all(np.abs(d_dev) <= 1e-6 * scale)
    assert g.read_status() == 0


@pytest.mark.parametrize("layout", ["part", "hybrid"])
def test_collide_layouts_24cubed(lib, oracle_mod, torch_mod, layout, monkeypatch):
    """The one-pass layouts of grids too large for 64-bit accumulators next
    to the full tile (24^3): the partial-tile layout (chosen by default) and
    the hybrid one (FP32 accumulators on the outer slabs), each against the
    oracle, with shared samples over several cells per workgroup (320 cells,
    more than workgroups) and with per-cell samples."""
    from paper_1005_5405_amd import inputs

    if layout == "hybrid":
        monkeypatch.setenv("BOLTZ_COLLIDE_LAYOUT", "hybrid")
    for G in (0, 1):
        kw = dict(nx=16, ny=20, nv=24, vmax=5.0, delta=100.0, eps=0.05, n_pairs=20000, mix16=4, bc=1,
                  sample_group=G)
        _say("layout", layout, kw)
        g, o = _pair(lib, oracle_mod, **kw)
        assert g.collide_layout == layout and g.collide_block == 1024
        assert 24 * 24 * 12 <= g.collide_lds_nodes < 24**3
        h = inputs.random_field(o.shape, seed=31 + G, scale=0.3).astype(np.float32).astype(np.float64)
        ref = o.collide(h, 5)
        hs, hout = _dev(torch_mod, h), g.empty()
        g.collide(hs, hout, 5)
        torch_mod.cuda.synchronize()
        rel, wrel = _errs(o, _host(hout), ref)
        assert rel <= 1e-5 and wrel <= 1e-5, (rel, wrel)
        assert g.read_status() == 0


def test_equilibrium_is_bitwise_fixed_point(lib, oracle_mod, torch_mod):
    _say("equilibrium")
    g = lib.Boltz(nx=16, ny=16, nv=12, vmax=4.5, delta=10.0, eps=0.1, n_pairs=2000)
    h0, h1 = g.empty(0.0), g.empty(1.0)
    for n in range(3):
        g.step(h0, h1, lib.Walls(), n)
        h0, h1 = h1, h0
    torch_mod.cuda.synchronize()
    assert torch_mod.count_nonzero(h0).item() == 0


def test_non_spd_correction_is_reported(lib, oracle_mod, torch_mod):
    _say("non-spd")
    g = lib.Boltz(nx=2, ny=2, nv=6, vmax=3.0, delta=1.0, eps=0.1, n_pairs=100, bc=1)
    h = g.empty(-50.0)  # F = 1 + eps h = -4 < 0: the correction matrix is negative definite
    out = g.empty()
    g.read_status(clear=True)
    g.collide(h, out, 0)
    assert g.read_status(clear=True) & 1
    ref = g.empty()
    g.collide(h, ref, 0, correction=False)
    torch_mod.cuda.synchronize()
    # the failed correction leaves the raw update (LDS atomics add in any order)
    assert torch_mod.allclose(out, ref, rtol=1e-6, atol=0)
    assert g.read_status() == 0


# moments: rows read four nodes at a time (nv_z % 4 == 0) or one by one,
# fewer or more velocity rows than the 512 threads of a workgroup
@pytest.mark.parametrize("order,nv,vmax", [(2, 12, 4.5), (1, 12, 4.5), (2, (7, 5, 9), (3.0, 2.5, 3.5)),
                                           (2, (24, 24, 8), (5.0, 5.0, 3.0))])
def test_moments_and_lid_shear_parity(lib, oracle_mod, torch_mod, order, nv, vmax):
    from paper_1005_5405_amd import inputs

    _say("moments", order, nv)
    g, o = _pair(lib, oracle_mod, nx=12, ny=10, nv=nv, vmax=vmax, delta=10.0, eps=0.1, n_pairs=100, order=order)
    h = inputs.random_field(o.shape, seed=3, scale=0.5).astype(np.float32).astype(np.float64)
    mom_ref, D_ref = o.moments(h, oracle_mod.Walls(**WALLS), lid_shear=True)
    mom = torch_mod.zeros(o.nx * o.ny * 11, dtype=torch_mod.float64, device="cuda")
    D = torch_mod.zeros(1, dtype=torch_mod.float64, device="cuda")
    g.moments(_dev(torch_mod, h), mom, lib.Walls(**WALLS), D)
    got = mom.cpu().numpy().reshape(mom_ref.shape)
    scale = np.abs(mom_ref).reshape(-1, 11).max(0)
    assert np.all(np.abs(got - mom_ref).reshape(-1, 11) <= 1e-10 * scale)
    assert abs(D.item() - D_ref) <= 1e-10 * max(abs(D_ref), 1e-3)


def test_cavity_step_parity_1_and_100_steps(lib, oracle_mod, torch_mod):
    from paper_1005_5405_amd import CAVITY_16, inputs

    pre = CAVITY_16
    kw = pre.problem()
    g, o = _pair(lib, oracle_mod, **kw)
    walls_o, walls_g = oracle_mod.Walls(lid_u=pre.lid_u), lib.Walls(lid_u=pre.lid_u)
    # one step from a random state
    _say("step 1", kw)
    h = inputs.random_field(o.shape, seed=5, scale=0.3).astype(np.float32).astype(np.float64)
    ref = o.step(h, walls_o, 7)
    hin, hout = _dev(torch_mod, h), g.empty()
    g.step(hin, hout, walls_g, 7)
    torch_mod.cuda.synchronize()
    rel, wrel = _errs(o, _host(hout), ref)
    assert rel <= 1e-5 and wrel <= 1e-5, (rel, wrel)
    # 100 steps of the driven cavity from rest, run independently on both sides
    _say("step 100", kw)
    href = np.zeros(o.shape)
    a, b = g.empty(0.0), g.empty()
    for n in range(100):
        href = o.step(href, walls_o, n)
        g.step(a, b, walls_g, n)
        a, b = b, a
    torch_mod.cuda.synchronize()
    rel, wrel = _errs(o, _host(a), href)
    assert rel <= 1e-4 and wrel <= 1e-4, (rel, wrel)
    mom_ref, D_ref = o.moments(href, walls_o, lid_shear=True)
    mom = torch_mod.zeros(o.nx * o.ny * 11, dtype=torch_mod.float64, device="cuda")
    D = torch_mod.zeros(1, dtype=torch_mod.float64, device="cuda")
    g.moments(a, mom, walls_g, D)
    got = mom.cpu().numpy().reshape(mom_ref.shape)
    scale = np.abs(mom_ref).reshape(-1, 11).max(0)
    assert np.all(np.abs(got - mom_ref).reshape(-1, 11) <= 1e-4 * scale)
    assert abs(D.item() - D_ref) <= 1e-4 * abs(D_ref)
    assert g.read_status() == 0


@pytest.mark.parametrize("which", ["cavity64", "cavity200"])
def test_full_size_sampled_parity(lib, oracle_mod, torch_mod, which):
    """Full-size grids with the presets' per-cell sample streams (G = 1):
    streaming checked on every node for the 64x64 cavity, collision on sampled
    cells that the oracle computes one by one (both sizes)."""
    from paper_1005_5405_amd import PRESETS, inputs

    pre = PRESETS[which]
    kw = pre.problem()
    _say("full size", which)
    g, o = _pair(lib, oracle_mod, **kw)
    walls_o, walls_g = oracle_mod.Walls(lid_u=0.1), lib.Walls(lid_u=0.1)
    rng = np.random.default_rng(1)
    # input: smooth in space times a velocity polynomial, built on the device
    h32 = inputs.random_field((o.ny, o.nx, 1), seed=2, scale=0.3).astype(np.float32)
    prof = inputs.velocity_polynomial(o.node_velocities(), seed=3, scale=0.1).astype(np.float32)
    hin = (torch_mod.from_numpy(h32).cuda() * torch_mod.from_numpy(prof).cuda().view(1, 1, -1)).contiguous()
    hs = g.empty()
    g.stream(hin, hs, walls_g)
    hout = g.empty()
    g.collide(hs, hout, 9)
    torch_mod.cuda.synchronize()
    if which == "cavity64":
        ref_s = o.stream(hin.cpu().numpy().astype(np.float64), walls_o)
        rel, wrel = _errs(o, _host(hs), ref_s)
        assert rel <= 1e-5 and wrel <= 1e-5, (rel, wrel)
        del ref_s
    cells = np.unique(np.concatenate([[0, o.nx - 1, (o.ny - 1) * o.nx, o.nx * o.ny - 1],
                                      rng.integers(0, o.nx * o.ny, 6)]))
    idx = torch_mod.from_numpy(cells).cuda()
    hs_c = hs.view(-1, o.nv)[idx].cpu().numpy().astype(np.float64)
    got_c = hout.view(-1, o.nv)[idx].cpu().numpy().astype(np.float64)
    ref_c = o.collide_cells(hs_c, 9, cells)
    w = o.node_weights()
    for k in range(len(cells)):
        d = np.abs(got_c[k] - ref_c[k])
        assert d.max() <= 1e-5 * np.abs(ref_c[k]).max(), (which, cells[k])
        assert (d * w).max() <= 1e-5 * (np.abs(ref_c[k]) * w).max(), (which, cells[k])
    assert g.read_status() == 0


@pytest.mark.parametrize("which", ["cavity64", "cavity200"])
def test_headline_step_parity_full_size(lib, oracle_mod, torch_mod, which):
    """The launch configuration the benchmark times, at full size: boltz_step
    with one shared set of N_t pair records per step (G = 0), drawn in the
    last face launch and dealt to lanes, then the persistent collision with
    many cells per workgroup (each after the first staged while the previous
    one is corrected).  Sampled cells, chosen across several workgroups'
    cell lists, against the oracle's collision of the same post-stream values
    (the GPU streaming itself is checked on every node of the 64x64 cavity by
    test_full_size_sampled_parity).  boltz_collide without a defect buffer
    (the staged path) on the same post-stream state gives the same cells."""
    from paper_1005_5405_amd import PRESETS, inputs

    pre = PRESETS[which]
    kw = pre.problem(sample_group=0)
    _say("headline step", which, kw)
    g, o = _pair(lib, oracle_mod, **kw)
    step = 9
    lid = pre.lid(step * g.dt) if pre.lid_omega > 0 else pre.lid_u
    lid = lid if abs(lid) > 1e-3 else 0.05
    walls_o, walls_g = oracle_mod.Walls(lid_u=lid, tau_bottom=1.02), lib.Walls(lid_u=lid, tau_bottom=1.02)
    h32 = inputs.random_field((o.ny, o.nx, 1), seed=4, scale=0.3).astype(np.float32)
    prof = inputs.velocity_polynomial(o.node_velocities(), seed=5, scale=0.1).astype(np.float32)
    hin = (torch_mod.from_numpy(h32).cuda() * torch_mod.from_numpy(prof).cuda().view(1, 1, -1)).contiguous()
    del h32
    hout = g.empty()
    g.step(hin, hout, walls_g, step)
    hs = g.empty()
    g.stream(hin, hs, walls_g)
    del hin
    h2 = g.empty()
    g.collide(hs, h2, step)
    torch_mod.cuda.synchronize()
    assert g.read_status() == 0
    ncell = o.nx * o.ny
    rng = np.random.default_rng(11)
    # first cells of workgroups, cells staged after them, the corners
    cells = np.unique(np.concatenate([[0, 1, 255, 256, 257, 511, 512, 1023, 1024, o.nx - 1,
                                       (o.ny - 1) * o.nx, ncell - 2, ncell - 1],
                                      rng.integers(0, ncell, 7)]))
    cells = cells[cells < ncell]
    idx = torch_mod.from_numpy(cells).cuda()
    hs_c = hs.view(-1, o.nv)[idx].cpu().numpy().astype(np.float64)
    got_c = hout.view(-1, o.nv)[idx].cpu().numpy().astype(np.float64)
    got2_c = h2.view(-1, o.nv)[idx].cpu().numpy().astype(np.float64)
    ref_c = o.collide_cells(hs_c, step, cells)
    w = o.node_weights()
    for k in range(len(cells)):
        for got in (got_c[k], got2_c[k]):
            d = np.abs(got - ref_c[k])
            assert d.max() <= 1e-5 * np.abs(ref_c[k]).max(), (which, cells[k])
            assert (d * w).max() <= 1e-5 * (np.abs(ref_c[k]) * w).max(), (which, cells[k])
    # the whole state: the step and the separately called halves agree (the
    # same records; fixed-point sums do not depend on their order)
    assert torch_mod.allclose(hout, h2, rtol=1e-6, atol=1e-6 * hout.abs().max().item())


# Shared-sample steps through boltz_step: the pair records are drawn in the
# last face launch and every full block of 1024 records is stored dealt to
# lanes (a permutation, so the collision equals the oracle's); N_t = 2348 has
# two full blocks and a partial one.  Order 2 draws them with the y faces,
# order 1 with its single face launch; grids with v = 0 nodes included.
@pytest.mark.parametrize("case", [
    dict(order=2, nx=10, ny=9, nv=(12, 12, 12), vmax=4.5),
    dict(order=1, nx=7, ny=11, nv=(8, 8, 8), vmax=3.5),
    dict(order=2, nx=9, ny=6, nv=(7, 5, 8), vmax=(3.0, 2.5, 3.5)),
])
def test_shared_sample_step_parity(lib, oracle_mod, torch_mod, case):
    from paper_1005_5405_amd import inputs

    kw = dict(case, delta=10.0, eps=0.1, n_pairs=2348, sample_group=0, mix16=4)
    _say("shared-sample step", kw)
    g, o = _pair(lib, oracle_mod, **kw)
    h = inputs.random_field(o.shape, seed=17, scale=0.3).astype(np.float32).astype(np.float64)
    walls_o, walls_g = oracle_mod.Walls(**WALLS), lib.Walls(**WALLS)
    for step in (3, 4):
        ref = o.step(h, walls_o, step)
        hout = g.empty()
        g.step(_dev(torch_mod, h), hout, walls_g, step)
        torch_mod.cuda.synchronize()
        rel, wrel = _errs(o, _host(hout), ref)
        assert rel <= 1e-5 and wrel <= 1e-5, (step, rel, wrel)
        # the two halves called separately (records drawn by sample_kernel) agree
        hs, h2 = g.empty(), g.empty()
        g.stream(_dev(torch_mod, h), hs, walls_g)
        g.collide(hs, h2, step)
        torch_mod.cuda.synchronize()
        assert torch_mod.equal(h2, hout), step
    assert g.read_status() == 0


# Stretched velocity cells (Sec. 5.1, the paper's own discretisation: 20^3 on
# [-3, 3] in the ratio 0.945; 18^3 in 0.970): node tables, samples (the
# post-collision cells found by a binary search over the edges on the GPU, by
# counting edges in the oracle), collision and whole steps.
@pytest.mark.parametrize("nv,rv,G", [(20, 0.945, 1), (20, 0.945, 0), (18, 0.97, 0), ((20, 18, 20), 0.945, 1)])
def test_stretched_grid_parity(lib, oracle_mod, torch_mod, nv, rv, G):
    from paper_1005_5405_amd import inputs

    kw = dict(nx=7, ny=6, nv=nv, vmax=3.0, delta=1.0, eps=0.05, n_pairs=6144, sample_group=G, rv=rv)
    _say("stretched", kw)
    g, o = _pair(lib, oracle_mod, **kw)
    for k in range(3):
        np.testing.assert_array_equal(g.axis_thresholds(k), o.thresholds[k])
    assert g.dt == o.dt and g.K == o.K and g.W == o.W and g.qfac == o.qfac
    for cell, step in [(0, 0), (37, 12345)]:
        gi, gq, gw = g.debug_pairs(cell, step, 0, 6144, words=True)
        oi, oq, ow = o.debug_pairs(cell, step, 0, 6144, words=True)
        np.testing.assert_array_equal(gw, ow)
        np.testing.assert_array_equal(gi, oi)
        np.testing.assert_allclose(gq, oq, rtol=2e-6, atol=1e-12 * oq.max())
    h = inputs.random_field(o.shape, seed=21, scale=0.3).astype(np.float32).astype(np.float64)
    walls_o, walls_g = oracle_mod.Walls(**WALLS), lib.Walls(**WALLS)
    # stream, collide, step against the oracle
    ref_s = o.stream(h, walls_o)
    hs = g.empty()
    g.stream(_dev(torch_mod, h), hs, walls_g)
    ref_c = o.collide(_host(hs), 3)
    hc = g.empty()
    g.collide(hs, hc, 3)
    ref = o.step(h, walls_o, 3)
    hout = g.empty()
    g.step(_dev(torch_mod, h), hout, walls_g, 3)
    torch_mod.cuda.synchronize()
    for got, r in ((_host(hs), ref_s), (_host(hc), ref_c), (_host(hout), ref)):
        rel, wrel = _errs(o, got, r)
        assert rel <= 1e-5 and wrel <= 1e-5, (rel, wrel)
    # 20 steps from rest of the driven cavity with the paper's lid velocity
    href = np.zeros(o.shape)
    a, b = g.empty(0.0), g.empty()
    wo, wg = oracle_mod.Walls(lid_u=0.01), lib.Walls(lid_u=0.01)
    for n in range(20):
        href = o.step(href, wo, n)
        g.step(a, b, wg, n)
        a, b = b, a
    torch_mod.cuda.synchronize()
    rel, wrel = _errs(o, _host(a), href)
    assert rel <= 1e-4 and wrel <= 1e-4, (rel, wrel)
    assert g.read_status() == 0


# Continuous pairs (problem flag CONTINUOUS_PAIRS, the sampling kernel of
# Sec. 4 as printed: v, v1 from the Maxwellian by Box-Muller, binned to their
# cells): the same pairs bit for bit (cells of all four velocities, -1 for a
# velocity outside the box, the first Philox block), weights to FP32, and
# collision and step parity.
CONT_GRIDS = [dict(nv=12, vmax=4.5), dict(nv=(7, 5, 9), vmax=(3.0, 2.5, 3.5)), dict(nv=20, vmax=3.0, rv=0.945),
              dict(nv=(20, 18, 20), vmax=3.0, rv=0.97)]


@pytest.mark.parametrize("grid", range(len(CONT_GRIDS)))
def test_continuous_pairs_bit_exact(lib, oracle_mod, torch_mod, grid):
    kw = dict(nx=5, ny=4, delta=1.0, eps=0.05, n_pairs=6144, sample_group=0, flags=lib.CONTINUOUS_PAIRS,
              **CONT_GRIDS[grid])
    _say("continuous pairs", kw)
    g, o = _pair(lib, oracle_mod, **kw)
    for cell, step, m0, count in [(0, 0, 0, 6144), (3, 777, 100000, 20000)]:
        gi, gq, gw = g.debug_pairs(cell, step, m0, count, words=True)
        oi, oq, ow = o.debug_pairs(cell, step, m0, count, words=True)
        np.testing.assert_array_equal(gw, ow)
        np.testing.assert_array_equal(gi, oi)
        np.testing.assert_allclose(gq, oq, rtol=2e-6, atol=1e-12 * oq.max())
        assert 0.3 < (oi[:, 2] >= 0).mean() <= 1.0


@pytest.mark.parametrize("G", [0, 1])
def test_continuous_collide_and_step_parity(lib, oracle_mod, torch_mod, G):
    from paper_1005_5405_amd import inputs

    kw = dict(nx=6, ny=5, nv=20, vmax=3.0, rv=0.945, delta=1.0, eps=0.05, n_pairs=6144, sample_group=G,
              flags=lib.CONTINUOUS_PAIRS)
    _say("continuous collide", kw)
    g, o = _pair(lib, oracle_mod, **kw)
    h = inputs.random_field(o.shape, seed=61 + G, scale=0.3).astype(np.float32).astype(np.float64)
    ref = o.collide(h, 11)
    hs, hout = _dev(torch_mod, h), g.empty()
    g.collide(hs, hout, 11)
    torch_mod.cuda.synchronize()
    rel, wrel = _errs(o, _host(hout), ref)
    assert rel <= 1e-5 and wrel <= 1e-5, (rel, wrel)
    # 20 steps of the driven cavity from rest
    href = np.zeros(o.shape)
    a, b = g.empty(0.0), g.empty()
    wo, wg = oracle_mod.Walls(lid_u=0.01), lib.Walls(lid_u=0.01)
    for n in range(20):
        href = o.step(href, wo, n)
        g.step(a, b, wg, n)
        a, b = b, a
    torch_mod.cuda.synchronize()
    rel, wrel = _errs(o, _host(a), href)
    assert rel <= 1e-4 and wrel <= 1e-4, (rel, wrel)
    assert g.read_status() == 0
