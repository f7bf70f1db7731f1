"""GPU parity of the in-place sequential collision (Alg. 3,
BOLTZ_SEQUENTIAL_UPDATE) against the oracle's sequential loop, through the
C ABI.

The GPU keeps each cell's h in FP32 while the samples update it one after
another (the oracle in FP64); a level schedule of the shared records lets a
wavefront apply the records that share no node together, in an order that
gives every node its updates in sample order.  Both schedules (steps of one
level across groups of 1024 records, or levels within groups of 64 kept in
registers; the library picks one per problem, BOLTZ_SEQ_SCHEDULE forces it)
are tested.  Bars as for the Jacobi
collision: max|dh| / max|h_ref| and its Maxwellian-weighted form within
1e-5.  Results are bit-identical from call to call and between the
context's and the static scratch's records.
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


def _errs(o, got, ref):
    d = np.abs(got - ref)
    w = o.node_weights()
    return d.max() / max(np.abs(ref).max(), 1e-300), (d * w).max() / max((np.abs(ref) * w).max(), 1e-300)


def _state(o, seed, scale=0.05):
    from paper_1005_5405_amd import inputs

    V = o.node_velocities()
    h = np.stack([inputs.velocity_polynomial(V, seed=seed + c) for c in range(o.nx * o.ny)]).reshape(o.shape)
    return (h + inputs.random_field(o.shape, seed=seed, scale=scale)).astype(np.float32).astype(np.float64)


SEQ = 8
# time steps of the workloads with these grids (nu dt <= 0.1): the in-place
# loop, unlike the Jacobi form, compounds the increments within a step and
# is unstable at the nu dt of a few tenths the small periodic grids would
# get from their CFL number
CASES = [
    dict(nx=5, ny=4, nv=(12, 12, 12), vmax=4.5, delta=10.0, eps=0.1, n_pairs=2000, sample_group=0, dt=7.576e-3),
    # the 64x64 workload's grid, pairs and time step on 9 cells
    dict(nx=3, ny=3, nv=(20, 20, 20), vmax=5.0, delta=20.0, eps=0.1, n_pairs=20000, sample_group=0, mix16=4,
         dt=1.6447e-3),
    # 24^3 (two cells per CU), the 200x200 workload's step
    dict(nx=2, ny=2, nv=(24, 24, 24), vmax=5.0, delta=100.0, eps=0.05, n_pairs=50000, sample_group=0, mix16=4,
         dt=5.217e-4),
    # nv % 4 != 0 (scalar node phases), a ragged last group of records
    dict(nx=3, ny=2, nv=(5, 7, 3), vmax=(3.0, 3.5, 2.0), delta=2.0, eps=0.3, n_pairs=3001, sample_group=0,
         dt=0.02),
    # groups of four cells with their own records
    dict(nx=5, ny=3, nv=(20, 20, 20), vmax=5.0, delta=20.0, eps=0.1, n_pairs=20000, sample_group=4, mix16=4,
         dt=1.6447e-3),
    # fewer records than one group, and none
    dict(nx=4, ny=4, nv=(12, 12, 12), vmax=4.5, delta=10.0, eps=0.1, n_pairs=37, sample_group=0, dt=7.576e-3),
    dict(nx=4, ny=4, nv=(12, 12, 12), vmax=4.5, delta=10.0, eps=0.1, n_pairs=0, sample_group=0, dt=7.576e-3),
    # the paper's discretisation: 20^3 stretched 0.945 on [-3, 3], continuous pairs
    dict(nx=3, ny=2, nv=(20, 20, 20), vmax=3.0, delta=1.0, eps=0.01, n_pairs=6144, sample_group=0, rv=0.945,
         flags=4, dt=0.02),
    # many more cells than resident workgroups
    dict(nx=48, ny=40, nv=(12, 12, 12), vmax=4.5, delta=10.0, eps=0.1, n_pairs=2000, sample_group=0),
]


@pytest.fixture(params=["steps", "groups"])
def schedule(request, monkeypatch):
    monkeypatch.setenv("BOLTZ_SEQ_SCHEDULE", request.param)
    return request.param


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("correction", [True, False])
def test_sequential_collide_parity(lib, oracle_mod, torch_mod, case, correction, schedule):
    kw = dict(CASES[case], bc=1)
    kw["flags"] = kw.get("flags", 0) | SEQ
    _say("sequential collide", kw, "correction", correction, "schedule", schedule)
    g, o = lib.Boltz(**kw), oracle_mod.Oracle(**kw)
    assert g.collide_layout == "sequential"
    h = _state(o, 300 + case)
    ref = o.collide(h, 42, correction=correction)
    hs = torch_mod.from_numpy(h.astype(np.float32)).cuda()
    hout = g.empty()
    defect = torch_mod.zeros(o.nx * o.ny * 5, dtype=torch_mod.float64, device="cuda")
    g.collide(hs, hout, 42, correction=correction, defect=defect)
    torch_mod.cuda.synchronize()
    got = hout.cpu().numpy().astype(np.float64)
    rel, wrel = _errs(o, got, ref)
    _say("rel %.3g wrel %.3g" % (rel, wrel))
    assert rel <= 1e-5 and wrel <= 1e-5, (rel, wrel)
    if kw["n_pairs"] == 0:
        np.testing.assert_array_equal(got, h)
    # the same call again, and in place: bit-identical
    again = g.empty()
    g.collide(hs, again, 42, correction=correction)
    g.collide(hs, hs, 42, correction=correction)
    torch_mod.cuda.synchronize()
    assert torch_mod.equal(again, hout) and torch_mod.equal(hs, hout)
    # defect of the stored FP32 values
    V = o.node_velocities()
    w = o.node_weights()
    psi = np.stack([np.ones(len(w)), V[:, 0], V[:, 1], V[:, 2], (V**2).sum(1)], 1)
    d_host = o.eps * np.einsum("j,jk,ycj->yck", w, psi, got - h).reshape(-1, 5)
    d_dev = defect.cpu().numpy().reshape(-1, 5)
    scale = o.eps * np.einsum("j,jk,ycj->yck", w, np.abs(psi), np.abs(got) + np.abs(h)).reshape(-1, 5)
    assert np.all(np.abs(d_dev - d_host) <= 1e-12 * scale)
    if correction:
        assert np.all(np.abs(d_dev) <= 1e-6 * scale)
    else:
        # mass is conserved by every sample (FP32 rounding of the running h aside)
        assert np.all(np.abs(d_dev[:, 0]) <= 1e-5 * scale[:, 0])
    assert g.read_status() == 0


def test_sequential_differs_from_jacobi(lib, oracle_mod, torch_mod):
    """The two update forms differ by more than the parity bar at a large
    time step, so the parity above tells them apart."""
    kw = dict(nx=2, ny=2, nv=(12, 12, 12), vmax=4.5, delta=10.0, eps=0.1, n_pairs=2000, sample_group=0, bc=1,
              dt=0.02)
    o = oracle_mod.Oracle(**kw)
    oq = oracle_mod.Oracle(**dict(kw, flags=SEQ))
    g = lib.Boltz(**dict(kw, flags=SEQ))
    h = _state(o, 11)
    jac = o.collide(h, 3, correction=False)
    seq = oq.collide(h, 3, correction=False)
    hs, out = torch_mod.from_numpy(h.astype(np.float32)).cuda(), g.empty()
    g.collide(hs, out, 3, correction=False)
    torch_mod.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    rel_seq, wrel_seq = _errs(o, got, seq)
    rel_jac, wrel_jac = _errs(o, got, jac)
    assert rel_seq <= 1e-5 and wrel_seq <= 1e-5, (rel_seq, wrel_seq)
    assert wrel_jac > 100 * wrel_seq and wrel_jac > 1e-4, (wrel_jac, wrel_seq)


def test_sequential_step_parity(lib, oracle_mod, torch_mod, schedule):
    """boltz_step (walls, streaming, the records drawn in the face launch in
    sample order, levels, collision) against the oracle's step, 3 steps of
    the 16x16 cavity with a moving lid."""
    kw = dict(nx=16, ny=16, nv=12, vmax=4.5, delta=10.0, eps=0.1, n_pairs=2000, sample_group=0, flags=SEQ)
    _say("sequential step", kw)
    g, o = lib.Boltz(**kw), oracle_mod.Oracle(**kw)
    walls = lib.Walls(lid_u=0.1)
    owalls = oracle_mod.Walls(lid_u=0.1)
    h = np.zeros(o.shape)
    a, b = g.empty(0.0), g.empty()
    for s in range(3):
        g.step(a, b, walls, s)
        h = o.step(h, owalls, s)
        a, b = b, a
        torch_mod.cuda.synchronize()
        rel, wrel = _errs(o, a.cpu().numpy().astype(np.float64), h)
        _say("step", s, "rel %.3g wrel %.3g" % (rel, wrel))
        assert rel <= 1e-5 and wrel <= 1e-5, (s, rel, wrel)
    assert g.read_status() == 0


def test_sequential_full_size_sampled_cells(lib, oracle_mod, torch_mod, schedule):
    """The 64x64 cavity (20^3, 20000 shared pairs) at full size in the launch
    the benchmark's sequential variant times (boltz_step): sampled cells of
    the GPU's collision against the oracle's collision of the same cells,
    from the GPU's own post-stream state."""
    kw = dict(nx=64, ny=64, nv=20, vmax=5.0, delta=20.0, eps=0.1, n_pairs=20000, sample_group=0, mix16=4,
              flags=SEQ)
    _say("sequential full size", kw)
    g, o = lib.Boltz(**kw), oracle_mod.Oracle(**kw)
    walls = lib.Walls(lid_u=0.1)
    a, b = g.empty(0.0), g.empty()
    for s in range(4):
        g.step(a, b, walls, s)
        a, b = b, a
    # one more step split in its two halves
    hs = g.empty()
    g.stream(a, hs, walls)
    out = g.empty()
    g.collide(hs, out, 4)
    torch_mod.cuda.synchronize()
    assert g.read_status() == 0
    cells = np.random.default_rng(5).choice(64 * 64, 24, replace=False)
    cells = np.concatenate([[0, 63, 64 * 64 - 1], cells])
    hs_h = hs.cpu().numpy().reshape(64 * 64, -1).astype(np.float64)
    ref = o.collide_cells(hs_h[cells], 4, cells)
    got = out.cpu().numpy().reshape(64 * 64, -1)[cells].astype(np.float64)
    d = np.abs(got - ref)
    w = o.node_weights()
    assert d.max() <= 1e-5 * np.abs(ref).max()
    assert (d * w).max() <= 1e-5 * (np.abs(ref) * w).max()


def test_sequential_noalloc_equals_context_records(lib, torch_mod, schedule):
    kw = dict(nx=10, ny=8, nv=(20, 20, 20), vmax=5.0, delta=20.0, eps=0.1, n_pairs=20000, sample_group=0, mix16=4,
              bc=1, flags=SEQ)
    g = lib.Boltz(**kw)
    from paper_1005_5405_amd import inputs

    h = torch_mod.from_numpy(inputs.random_field((8, 10, 8000), seed=3, scale=0.2).astype(np.float32)).cuda()
    a, b = g.empty(), g.empty()
    g.collide(h, a, 9)
    g.collide_noalloc(h, b, 9)
    torch_mod.cuda.synchronize()
    assert torch_mod.equal(a, b)
    assert g.read_status() == 0
