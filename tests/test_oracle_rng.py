"""Pins of the oracle's random-number and sampling layer (CPU only).

* Philox4x32-10: published known-answer vectors (tests/golden) and the
  round structure checked against numpy's independent Philox4x64-10.
* Direction map: cos/sin(2 pi u) against numpy's libm (degree-13/12
  polynomials: 5e-13).
* Node law on 12-bit fields: thresholds against the closed-form Maxwellian
  weights, exact left-closed intervals, sampled frequencies against the
  realised law (chi-square), mixture marginals and the w/p weight.
* Collision kinematics: momentum and energy of every sampled pair.
"""
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _kat():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                w = [int(x, 16) for x in line.split()]
                rows.append((w[:4], w[4:6], w[6:10]))
    return rows


def test_philox_known_answers(oracle_mod):
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, expect in rows:
        assert oracle_mod.philox4x32_10(ctr, key).tolist() == expect


def _philox_generic(ctr, key, mult, weyl, bits, rounds=10):
    """Philox-4xW round structure written for any word width W."""
    mask = (1 << bits) - 1
    c, k = list(ctr), list(key)
    for r in range(rounds):
        if r:
            k = [(k[0] + weyl[0]) & mask, (k[1] + weyl[1]) & mask]
        p0, p1 = mult[0] * c[0], mult[1] * c[2]
        c = [(p1 >> bits) ^ c[1] ^ k[0], p1 & mask, (p0 >> bits) ^ c[3] ^ k[1], p0 & mask]
    return c


def test_philox_round_structure_matches_numpy_4x64(oracle_mod):
    # numpy.random.Philox is Philox4x64-10; it increments the counter before
    # producing a block, so its first four words are block(counter=1).
    M64 = (0xD2E7470EE14C6C93, 0xCA5A826395121157)
    W64 = (0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B)
    rng = np.random.default_rng(5)
    for _ in range(4):
        key = [int(x) for x in rng.integers(0, 2**63, size=2, dtype=np.int64)]
        ctr0 = int(rng.integers(0, 2**62))
        bg = np.random.Philox(counter=ctr0, key=np.array(key, dtype=np.uint64))
        got = [int(x) for x in bg.random_raw(4)]
        assert got == _philox_generic([ctr0 + 1, 0, 0, 0], key, M64, W64, 64)
    # the 32-bit instance of the same structure agrees with the oracle
    M32, W32 = (0xD2511F53, 0xCD9E8D57), (0x9E3779B9, 0xBB67AE85)
    for _ in range(200):
        ctr = [int(x) for x in rng.integers(0, 2**32, size=4, dtype=np.uint64)]
        key = [int(x) for x in rng.integers(0, 2**32, size=2, dtype=np.uint64)]
        assert oracle_mod.philox4x32_10(ctr, key).tolist() == _philox_generic(ctr, key, M32, W32, 32)


def test_cos_sin_2pi_against_libm(oracle_mod):
    rng = np.random.default_rng(1)
    us = np.concatenate([(rng.integers(0, 2**16, 4000) + 0.5) * 2.0**-16,
                         (np.arange(64) + 0.5) / 64.0, [0.5 * 2.0**-16, 1 - 0.5 * 2.0**-16]])
    for u in us:
        c, s = oracle_mod.cos_sin_2pi(u)
        assert abs(c - np.cos(2 * np.pi * u)) <= 5e-13
        assert abs(s - np.sin(2 * np.pi * u)) <= 5e-13
        assert abs(c * c + s * s - 1.0) <= 1e-12


def _grid(n, a):
    dv = 2 * a / n
    v = (np.arange(n) + 0.5 - n / 2) * dv
    om = dv * np.exp(-v * v) / np.sqrt(np.pi)
    return v, om


@pytest.mark.parametrize("n,a", [(6, 3.0), (12, 4.5), (20, 5.0), (24, 5.0), (7, 3.0)])
def test_thresholds_realise_maxwellian_law(oracle_mod, n, a):
    o = oracle_mod.Oracle(2, 2, n, a, 1.0, 0.1, 10, bc=oracle_mod.BC_PERIODIC)
    v, om = _grid(n, a)
    np.testing.assert_allclose(o.v[0], v, rtol=0, atol=1e-14)
    assert np.all(o.v[0] == -o.v[0][::-1])  # exact antisymmetry of the nodes
    T = np.concatenate([[0], o.thresholds[0].astype(np.float64), [2.0**12]])
    assert np.all(np.diff(T) >= 0) and T[-2] <= 2.0**12
    p_hat = np.diff(T) / 2.0**12
    np.testing.assert_allclose(p_hat, om / om.sum(), rtol=0, atol=2.0**-12 + 1e-16)
    # W = (sum omega)^3, the discrete mass of Phi0 on the grid
    assert abs(o.W - om.sum() ** 3) <= 1e-15


def test_inverse_cdf_intervals_are_left_closed(oracle_mod):
    # node i is drawn for a 12-bit field f in [T_i, T_{i+1}): the special
    # values f = T_i and f = T_i - 1 fall on either side of each boundary
    o = oracle_mod.Oracle(2, 2, (20, 12, 7), (5.0, 4.5, 3.0), 1.0, 0.1, 10, bc=oracle_mod.BC_PERIODIC)
    F = 2**12
    for k in range(3):
        T = [int(t) for t in o.thresholds[k]]
        for i, t in enumerate(T, start=1):
            if t < F and (i == len(T) or T[i] > t):
                assert o.axis_draw(k, t) == i
            if 0 < t <= F and T[i - 2 if i >= 2 else 0] < t:
                assert o.axis_draw(k, t - 1) == i - 1
        assert o.axis_draw(k, 0) == sum(1 for t in T if t == 0)
        assert o.axis_draw(k, F - 1) == sum(1 for t in T if t < F)
        assert o.axis_draw(k, F) == -1


def test_sampled_nodes_follow_law(oracle_mod):
    n, a = 8, 3.0
    o = oracle_mod.Oracle(2, 2, n, a, 1.0, 0.1, 1, bc=oracle_mod.BC_PERIODIC, mix16=0)
    N = 200000
    idx, _ = o.debug_pairs(0, 3, 0, N)
    T = np.concatenate([[0], o.thresholds[0].astype(np.float64), [2.0**12]])
    p = np.diff(T) / 2.0**12
    comps = []
    for col in (0, 1):
        j = idx[:, col]
        comps += [j // (n * n), (j // n) % n, j % n]
    chi2_max = 0.0
    for c in comps:
        cnt = np.bincount(c, minlength=n)
        e = N * p
        m = e > 5
        chi2 = ((cnt[m] - e[m]) ** 2 / e[m]).sum()
        chi2_max = max(chi2_max, chi2 / m.sum())
        assert cnt[~m].sum() <= 50
    # reduced chi-square of six independent component histograms
    assert chi2_max < 3.0
    # a and b independent: joint x-component table
    ja, jb = idx[:, 0] // (n * n), idx[:, 1] // (n * n)
    tab = np.zeros((n, n))
    np.add.at(tab, (ja, jb), 1)
    e = N * np.outer(p, p)
    m = e > 5
    assert ((tab[m] - e[m]) ** 2 / e[m]).sum() / m.sum() < 2.0


def _laws(o, k):
    n = o.nv3[k]
    T = np.concatenate([[0], o.thresholds[k].astype(np.float64), [2.0**12]])
    pm = np.diff(T) / 2.0**12
    edges = np.array([-(-(i << 12) // n) for i in range(n + 1)], dtype=np.float64)
    pu = np.diff(edges) / 2.0**12
    return pm, pu


# mix16 = 0 only on a grid where the Maxwellian law reaches every node
@pytest.mark.parametrize("a,mix16", [(3.0, 0), (4.0, 4), (4.0, 8), (4.0, 16)])
def test_mixture_law_marginals(oracle_mod, a, mix16):
    n = 10
    o = oracle_mod.Oracle(2, 2, n, a, 1.0, 0.1, 1, bc=oracle_mod.BC_PERIODIC, mix16=mix16)
    N = 200000
    idx, _, wd = o.debug_pairs(1, 9, 0, N, words=True)
    beta = mix16 / 16.0
    # the component choices are the low byte of the first word
    assert abs(((wd[:, 0] >> 4) & 15 < mix16).mean() - beta) < 4 * np.sqrt(beta * (1 - beta) / N) + 1e-12
    assert abs(((wd[:, 0] & 15) < mix16).mean() - beta) < 4 * np.sqrt(beta * (1 - beta) / N) + 1e-12
    for col in (0, 1):
        j = idx[:, col]
        for k, c in enumerate([j // (n * n), (j // n) % n, j % n]):
            pm, pu = _laws(o, k)
            e = N * ((1 - beta) * pm + beta * pu)
            cnt = np.bincount(c, minlength=n)
            m = e > 5
            assert ((cnt[m] - e[m]) ** 2 / e[m]).sum() / m.sum() < 3.0


def _total_collision_weight(n, a, M):
    """sum over ordered node pairs (a, b) of w_a w_b times the direction
    average of |v_r . k| over the kept directions (both post-collision cells
    inside the box), by a midpoint rule in (u6, u7); written independently of
    the oracle.  On a uniform grid the post-collision cell of v_a + d is
    a + floor(d / dv + 1/2) per axis, so for an offset r = b - a and a
    direction k the kept first nodes form a box, one interval per axis, and
    the sum of w_a w_b over it is a product of per-axis interval sums."""
    dv = 2 * a / n
    v = (np.arange(n) + 0.5 - n / 2) * dv
    om = dv * np.exp(-v * v) / np.sqrt(np.pi)
    u = (np.arange(M) + 0.5) / M
    u6, u7 = np.meshgrid(u, u, indexing="ij")
    kz = (2 * u6 - 1).ravel()
    s = np.sqrt(1 - kz * kz)
    kk = np.stack([s * np.cos(2 * np.pi * u7.ravel()), s * np.sin(2 * np.pi * u7.ravel()), kz], 1)
    # prefix[r][i] = sum_{A < i} om_A om_{A + r} over A with A, A + r on the grid
    prefix = {}
    for r in range(-(n - 1), n):
        t = np.array([om[A] * om[A + r] if 0 <= A + r < n else 0.0 for A in range(n)])
        prefix[r] = np.concatenate([[0.0], np.cumsum(t)])
    total = 0.0
    for r in np.stack(np.meshgrid(*[np.arange(-(n - 1), n)] * 3, indexing="ij"), -1).reshape(-1, 3):
        alpha = dv * (kk @ r)
        d = alpha[:, None] * kk / dv
        oa, ob = np.floor(d + 0.5).astype(np.int64), np.floor(-d + 0.5).astype(np.int64)
        prod = np.abs(alpha)
        for i in range(3):
            lo = np.maximum.reduce([np.zeros_like(oa[:, i]), -oa[:, i], -r[i] - ob[:, i],
                                    np.full_like(oa[:, i], -r[i])])
            hi = np.minimum.reduce([np.full_like(oa[:, i], n - 1), n - 1 - oa[:, i], n - 1 - r[i] - ob[:, i],
                                    np.full_like(oa[:, i], n - 1 - r[i])])
            ok = lo <= hi
            P = prefix[int(r[i])]
            prod = prod * np.where(ok, P[np.clip(hi, 0, n - 1) + 1] - P[np.clip(lo, 0, n - 1)], 0.0)
        total += float(prod.mean())
    return total


# Unbiasedness of the importance weights of Eq. coll8Dim: whatever law the
# nodes are drawn from, the mean weight q N_t / (dt K) of a sample is the
# discrete collision integral of g = 1, i.e. the enumerated total above.  A
# law that can never draw some node (the 12-bit Maxwellian law alone on a
# wide grid) would miss that node's share and fail this; it is refused.
@pytest.mark.parametrize("a,mix16", [(3.0, 0), (3.0, 4), (4.0, 4), (4.0, 16)])
def test_mean_weight_equals_enumerated_collision_integral(oracle_mod, a, mix16):
    n, N = 6, 400000
    o = oracle_mod.Oracle(1, 1, n, a, 2.0, 0.1, N, bc=oracle_mod.BC_PERIODIC, mix16=mix16)
    _, q = o.debug_pairs(0, 5, 0, N)
    x = q * N / (o.dt * o.K)
    se = x.std(ddof=1) / np.sqrt(N)
    T = _total_collision_weight(n, a, 128)
    # the quadrature has converged well below the Monte Carlo error
    assert abs(_total_collision_weight(n, a, 64) - T) < 0.25 * se
    assert abs(x.mean() - T) < 4.5 * se, (x.mean(), T, se)


def test_maxwellian_law_alone_is_refused_where_it_misses_nodes(oracle_mod):
    # 8 cells on [-4, 4]: the 12-bit Maxwellian law leaves the two outer nodes
    # of each axis at probability zero
    with pytest.raises(ValueError, match="mix16 = 0"):
        oracle_mod.Oracle(1, 1, 8, 4.0, 1.0, 0.1, 100, bc=oracle_mod.BC_PERIODIC, mix16=0)
    T = oracle_mod.Oracle(1, 1, 8, 4.0, 1.0, 0.1, 100, bc=oracle_mod.BC_PERIODIC, mix16=4).thresholds[0]
    assert np.any(np.diff(np.concatenate([[0], T.astype(np.int64), [4096]])) == 0)


def test_pair_kinematics_conserve_momentum_energy(oracle_mod):
    o = oracle_mod.Oracle(3, 2, (12, 10, 8), (4.5, 4.0, 3.5), 1.0, 0.1, 100, bc=oracle_mod.BC_PERIODIC)
    idx, q, vel = o.debug_pairs(4, 7, 1000, 20000, velocities=True)
    va, vb, vs, v1s = vel[:, 0], vel[:, 1], vel[:, 2], vel[:, 3]
    scale = (va**2).sum(1) + (vb**2).sum(1) + 1e-300
    mom = np.abs((vs + v1s) - (va + vb)).max(1)
    ene = np.abs(((vs**2).sum(1) + (v1s**2).sum(1)) - scale)
    assert mom.max() <= 2e-15 * np.sqrt(scale).max()
    # |k|^2 = 1 to the 4e-13 truncation of the direction polynomials
    assert (ene / scale).max() <= 5e-12
    # the pre-collision velocities are the nodes a, b
    nodes = o.node_velocities()
    np.testing.assert_array_equal(va, nodes[idx[:, 0]])
    np.testing.assert_array_equal(vb, nodes[idx[:, 1]])
    # kept pairs: a*, b* are the velocity cells that contain v*, v1*
    kept = idx[:, 2] >= 0
    assert 0.5 < kept.mean() <= 1.0
    lo = np.array([-4.5, -4.0, -3.5])
    dv = 2 * (-lo) / np.array([12, 10, 8])
    for col, vv in ((2, vs), (3, v1s)):
        cells = np.floor((vv[kept] - lo) / dv).astype(int)
        j = (cells[:, 0] * 10 + cells[:, 1]) * 8 + cells[:, 2]
        # a floor computed with a different rounding may flip on a face: allow none here
        assert np.array_equal(j, idx[kept, col])
    # discarded pairs really leave the box
    out = ~kept
    if out.any():
        outside = (np.abs(vs[out]) > -lo).any(1) | (np.abs(v1s[out]) > -lo).any(1)
        assert outside.all()
    # the weight: K = (5/16) sqrt(2 pi) 1.016034 delta; q = 0 for discarded pairs
    K = (5.0 / 16.0) * np.sqrt(2 * np.pi) * 1.016034 * 1.0
    np.testing.assert_allclose(o.K, K, rtol=1e-15)
    assert np.all(q[~kept] == 0) and np.all(q[kept] >= 0)
