"""Pins of the oracle's continuous pair sampler (problem flag CONTINUOUS: the
sampling kernel of Sec. 4 as printed, v and v1 drawn from the Maxwellian by
the Box-Muller method and binned to their velocity cells), CPU only.

* -ln u of the sampler against numpy's log.
* The drawn velocities: every component normal with variance 1/2 (the
  Maxwellian Phi0 in these units; Kolmogorov-Smirnov), uncorrelated.
* Kinematics of every pair: momentum and energy of the continuous velocities,
  cells of all four velocities by an independent binning, weight
  q = dt K |v_r . k| / N_t, discards only for velocities outside the box.
* Collision integral, node by node: for constant h = c the mean loss at node j
  is g dt K (g = 2 c + eps c^2) times the integral of Phi0(v) nu(|v|) over
  cell j, nu the mean
  relative speed against a Maxwellian partner (a closed form), and the mean
  gain equals the mean loss (the collision operator annihilates Phi0).
"""
import math

import numpy as np
import pytest
from scipy import special, stats


def test_neg_ln_against_numpy(oracle_mod):
    rng = np.random.default_rng(3)
    w = np.concatenate([rng.integers(0, 2**32, 20000), [0, 1, 2**31 - 1, 2**31, 2**32 - 2, 2**32 - 1]])
    u = (w.astype(np.float64) + 1.0) * 2.0**-32
    got = np.array([oracle_mod.neg_ln(x) for x in u])
    ref = -np.log(u)
    assert got[-1] == 0.0  # u = 1
    err = np.abs(got - ref) / np.maximum(ref, 1e-300)
    assert np.all(np.abs(got - ref) <= 2e-16 * np.maximum(1.0, ref) + 4e-16 * ref), err.max()
    # near the sqrt(2) fold of the mantissa
    for x in (0.7071067811865475, 0.7071067811865476, 0.5, 0.25 * 1.4142135623730951):
        assert abs(oracle_mod.neg_ln(x) + math.log(x)) <= 1e-15


def _pairs(oracle_mod, n=12, a=4.0, count=100000, steps=(0,), **kw):
    o = oracle_mod.Oracle(1, 1, n, a, 1.0, 0.0 + kw.pop("eps", 0.1), count, bc=oracle_mod.BC_PERIODIC,
                          flags=oracle_mod.CONTINUOUS, **kw)
    out = [o.debug_pairs(0, s, 0, count, velocities=True) for s in steps]
    idx = np.concatenate([x[0] for x in out])
    q = np.concatenate([x[1] for x in out])
    vel = np.concatenate([x[2] for x in out])
    return o, idx, q, vel


def test_box_muller_velocities_are_maxwellian(oracle_mod):
    o, idx, q, vel = _pairs(oracle_mod, count=100000, steps=(0, 1))
    v = np.concatenate([vel[:, 0], vel[:, 1]])  # (2N, 3)
    N = len(v)
    for k in range(3):
        x = v[:, k]
        assert abs(x.mean()) < 5 * math.sqrt(0.5 / N)
        assert abs(x.var() - 0.5) < 5 * math.sqrt(2 * 0.25 / N)
        assert stats.kstest(x, "norm", args=(0.0, math.sqrt(0.5))).pvalue > 1e-3
    c = np.corrcoef(v.T)
    assert np.all(np.abs(c - np.eye(3)) < 5 / math.sqrt(N))
    # v and v1 of one pair are independent
    assert abs(np.corrcoef(vel[:, 0, 0], vel[:, 1, 0])[0, 1]) < 5 / math.sqrt(len(vel))


def _cells(o, x):
    """Cell index per component by binning on the uniform grid; -1 outside."""
    a = o.edges[0][-1]
    n = o.nv3[0]
    t = np.floor((x + a) * (n / (2 * a)))
    return np.where((t >= 0) & (t < n), t, -1).astype(np.int64)


def test_continuous_pair_kinematics_cells_and_weight(oracle_mod):
    o, idx, q, vel = _pairs(oracle_mod, n=10, a=2.5, count=60000)
    va, vb, vs, vbs = vel[:, 0], vel[:, 1], vel[:, 2], vel[:, 3]
    np.testing.assert_allclose(va + vb, vs + vbs, rtol=0, atol=2e-14)
    # energy to the truncation of the direction polynomials (|k|^2 = 1 to ~1e-12)
    e0 = (va**2).sum(1) + (vb**2).sum(1)
    np.testing.assert_allclose((vs**2).sum(1) + (vbs**2).sum(1), e0, rtol=1e-11, atol=1e-12)
    n = o.nv3[0]
    node = lambda c: np.where(np.all(c >= 0, 1), (c[:, 0] * n + c[:, 1]) * n + c[:, 2], -1)
    ca, cb, cs, cbs = (np.stack([_cells(o, v[:, k]) for k in range(3)], 1) for v in (va, vb, vs, vbs))
    inside = np.all(ca >= 0, 1) & np.all(cb >= 0, 1) & np.all(cs >= 0, 1) & np.all(cbs >= 0, 1)
    kept = idx[:, 2] >= 0
    assert np.array_equal(kept, inside)
    assert 0.5 < kept.mean() < 0.999  # the box [-2.5, 2.5] loses some tails
    assert np.array_equal(idx[:, 0], node(ca)) and np.array_equal(idx[:, 1], node(cb))
    assert np.array_equal(idx[kept, 2], node(cs)[kept]) and np.array_equal(idx[kept, 3], node(cbs)[kept])
    # q = dt K |alpha| / N_t with alpha the relative velocity along k: v* - v = alpha k
    alpha = np.linalg.norm(vs - va, axis=1)
    np.testing.assert_allclose(q[kept], o.qfac * alpha[kept], rtol=1e-11)  # |k| = 1 to ~1e-12
    assert np.all(q[~kept] == 0.0)


def _nu(s):
    """Mean |v1 - v| for v1 ~ Phi0 (components N(0, 1/2)) at |v| = s."""
    s = np.maximum(s, 1e-12)
    return np.exp(-s * s) / math.sqrt(math.pi) + (s + 0.5 / s) * special.erf(s)


def test_continuous_collision_integral_node_by_node(oracle_mod):
    """Loss and gain means per node against the closed form, h = c constant."""
    n, a, c = 6, 4.0, 0.7
    nb, count = 40, 50000
    eps = 0.1
    gc = 2.0 * c + eps * c * c  # g = h_a + h_b + eps h_a h_b for h = c
    o = oracle_mod.Oracle(1, 1, n, a, 1.0, eps, count, bc=oracle_mod.BC_PERIODIC, flags=oracle_mod.CONTINUOUS)
    nv = n**3
    L = np.zeros((nb, nv))
    G = np.zeros((nb, nv))
    for st in range(nb):
        idx, q = o.debug_pairs(0, st, 0, count)
        kept = idx[:, 2] >= 0
        w = q[kept] * gc
        L[st] = np.bincount(idx[kept, 0], w, nv) + np.bincount(idx[kept, 1], w, nv)
        G[st] = np.bincount(idx[kept, 2], w, nv) + np.bincount(idx[kept, 3], w, nv)
    # closed form: E[loss_j] = g dt K int_{cell j} Phi0(v) nu(|v|) dv (the k average of |v_r . k| is
    # |v_r| / 2, and v and v1 both sample cell j), by Gauss-Legendre in every cell
    x, wq = np.polynomial.legendre.leggauss(12)
    h = 2 * a / n
    E = np.zeros(nv)
    for i in range(n):
        xi = -a + h * (i + 0.5 * (x + 1))
        for j in range(n):
            yj = -a + h * (j + 0.5 * (x + 1))
            for k in range(n):
                zk = -a + h * (k + 0.5 * (x + 1))
                X, Y, Z = np.meshgrid(xi, yj, zk, indexing="ij")
                W = wq[:, None, None] * wq[None, :, None] * wq[None, None, :] * (h / 2) ** 3
                s = np.sqrt(X * X + Y * Y + Z * Z)
                E[(i * n + j) * n + k] = (W * np.exp(-s * s) * _nu(s)).sum() / math.pi**1.5
    E *= gc * o.dt * o.K
    mL, mG = L.mean(0), G.mean(0)
    seL, seG = L.std(0, ddof=1) / math.sqrt(nb), G.std(0, ddof=1) / math.sqrt(nb)
    big = E > 1e-3 * E.max()
    zl = np.abs(mL - E)[big] / seL[big]
    zg = np.abs(mG - E)[big] / seG[big]
    assert zl.max() < 5.0, zl.max()
    assert zg.max() < 5.0, zg.max()
    # a mistake in the weight normalisation (a factor 2) would move every node by many standard errors
    assert np.median(np.abs(mL - 2 * E)[big] / seL[big]) > 20
