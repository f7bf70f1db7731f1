"""boltz_collide_noalloc (shared-sample records in the library's static device
scratch, no allocation) against boltz_collide through the C ABI (GPU).

Two calls in a row on one GPU, the second with a smaller problem (fewer cells,
fewer pairs, another velocity grid): the static array keeps the first call's
records, the second overwrites part of it.  Each call must equal
boltz_collide of the same problem, whose records live in its context: the
same records and kernels, and fixed-point sums that do not depend on the
order of the lanes (the FP32 array of rare far-tail terms aside), so the
results agree to 1e-6 of the state's largest value, and both match the
oracle at the tolerance of the parity tests.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


CALLS = [
    # shared samples over all cells, 20^3, several cells per workgroup
    dict(nx=24, ny=20, nv=(20, 20, 20), vmax=5.0, delta=20.0, eps=0.1, n_pairs=20000, sample_group=0, bc=1),
    # smaller: groups of 3 cells, 12^3, a partial record block
    dict(nx=5, ny=4, nv=(12, 12, 12), vmax=4.5, delta=10.0, eps=0.1, n_pairs=2500, sample_group=3, bc=1),
]


def test_noalloc_collide_matches_context_records_two_calls():
    import torch

    import oracle
    import paper_1005_5405_amd as pkg
    from paper_1005_5405_amd import inputs

    for i, kw in enumerate(CALLS):
        _say("noalloc call", i, kw)
        g, o = pkg.Boltz(**kw), oracle.Oracle(**kw)
        V = o.node_velocities()
        h = np.stack([inputs.velocity_polynomial(V, seed=200 + c) for c in range(o.nx * o.ny)]).reshape(o.shape)
        h = (h + inputs.random_field(o.shape, seed=9 + i, scale=0.05)).astype(np.float32)
        hs = torch.from_numpy(h).cuda()
        ref_ctx, out = g.empty(), g.empty()
        g.collide(hs, ref_ctx, 17 + i)
        g.collide_noalloc(hs, out, 17 + i)
        torch.cuda.synchronize()
        assert g.read_status() == 0
        scale = ref_ctx.abs().max().item()
        assert (out - ref_ctx).abs().max().item() <= 1e-6 * scale
        ref = o.collide(h.astype(np.float64), 17 + i)
        got = out.cpu().numpy().astype(np.float64)
        w = o.node_weights()
        d = np.abs(got - ref)
        assert d.max() <= 1e-5 * np.abs(ref).max()
        assert (d * w).max() <= 1e-5 * (np.abs(ref) * w).max()
        del g


def test_noalloc_rejects_records_beyond_the_scratch():
    import torch

    import paper_1005_5405_amd as pkg

    # 64 groups x 20000 pairs x 24 B = 30.7 MB > 16 MiB
    gg = pkg.Boltz(nx=16, ny=8, nv=8, vmax=3.5, delta=1.0, eps=0.1, n_pairs=20000, sample_group=2, bc=1)
    h = gg.empty(0.0)
    with pytest.raises(pkg.BoltzError, match="scratch"):
        gg.collide_noalloc(h, h, 0)
    # per-cell samples use no scratch at all
    g = pkg.Boltz(nx=8, ny=8, nv=8, vmax=3.5, delta=1.0, eps=0.1, n_pairs=20000, sample_group=1, bc=1)
    hh = g.empty(0.0)
    g.collide_noalloc(hh, hh, 0)
    torch.cuda.synchronize()
    assert torch.count_nonzero(hh).item() == 0
