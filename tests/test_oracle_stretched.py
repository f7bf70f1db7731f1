"""Pins of the oracle on stretched velocity grids (Sec. 5.1: cell lengths in
a progression ratio r_v, the smallest at the origin), CPU only.

* Node placement: widths in the ratio r_v on each half axis, adding up to the
  half width, mirror-symmetric, nodes at the cell centres, weights
  omega = width exp(-v^2) / sqrt(pi).
* The node law realises the Maxwellian weights of the stretched cells.
* Post-collision cells are the cells that contain v*, v1* (an independent
  search over the edges).
* The Monte Carlo collision mean matches a direct enumeration over every
  ordered node pair and a direction quadrature, node by node.
"""
import numpy as np
import pytest


@pytest.mark.parametrize("n,a,r", [(20, 3.0, 0.945), (18, 3.0, 0.97), (6, 3.0, 0.8)])
def test_stretched_nodes_and_weights(oracle_mod, n, a, r):
    o = oracle_mod.Oracle(2, 2, n, a, 1.0, 0.1, 10, bc=oracle_mod.BC_PERIODIC, rv=r)
    m = n // 2
    w0 = a / sum(r ** -i for i in range(m))
    widths = w0 * r ** -np.abs(np.arange(n) - m + 0.5 - np.sign(np.arange(n) - m + 0.5) * 0.5)
    e = o.edges[0]
    assert e[0] == -a and e[-1] == a and e[m] == 0.0
    assert np.all(e[m - np.arange(m + 1)] == -e[m + np.arange(m + 1)])
    np.testing.assert_allclose(np.diff(e), widths, rtol=1e-12)
    # ratio of neighbouring cells towards the origin
    np.testing.assert_allclose(np.diff(e)[m + 1:] * r, np.diff(e)[m:-1], rtol=1e-12)
    np.testing.assert_array_equal(o.v[0], 0.5 * (e[:-1] + e[1:]))
    np.testing.assert_allclose(o.omega[0], np.diff(e) * np.exp(-o.v[0] ** 2) / np.sqrt(np.pi), rtol=1e-14)
    # the node law on 12-bit fields realises omega / sum(omega)
    T = np.concatenate([[0], o.thresholds[0].astype(np.float64), [2.0**12]])
    np.testing.assert_allclose(np.diff(T) / 2.0**12, o.omega[0] / o.omega[0].sum(), rtol=0, atol=2.0**-12)
    # and the discrete mass approaches 1 as the box widens
    assert abs(o.W - o.omega[0].sum() ** 3) < 1e-15


def test_stretched_grid_validation(oracle_mod):
    for kw in (dict(rv=1.2), dict(rv=-0.5), dict(rv=0.9, nv=(7, 8, 8))):
        args = dict(nx=2, ny=2, nv=8, vmax=3.0, delta=1.0, eps=0.1, n_pairs=10, bc=oracle_mod.BC_PERIODIC)
        args.update(kw)
        with pytest.raises(ValueError):
            oracle_mod.Oracle(**args)


def _cells(edges, x):
    """Cell of x per axis by search over the edges; -1 outside [e_0, e_n)."""
    i = np.searchsorted(edges, x, side="right") - 1
    return np.where((x >= edges[0]) & (x < edges[-1]), i, -1)


def test_stretched_post_collision_cells(oracle_mod):
    o = oracle_mod.Oracle(3, 2, (20, 18, 20), (3.0, 3.0, 2.5), 1.0, 0.1, 100, bc=oracle_mod.BC_PERIODIC,
                          rv=0.945)
    idx, q, vel = o.debug_pairs(4, 7, 0, 50000, velocities=True)
    n = o.nv3
    kept = idx[:, 2] >= 0
    assert 0.5 < kept.mean() < 1.0
    for col, v in ((2, vel[:, 2]), (3, vel[:, 3])):
        c = np.stack([_cells(o.edges[k], v[:, k]) for k in range(3)], 1)
        inside = np.all(c >= 0, 1)
        j = (c[:, 0] * n[1] + c[:, 1]) * n[2] + c[:, 2]
        assert np.array_equal(j[kept], idx[kept, col])
        # a discarded pair has a post-collision velocity outside the box
    out_a = ~np.all(np.stack([_cells(o.edges[k], vel[:, 2, k]) for k in range(3)], 1) >= 0, 1)
    out_b = ~np.all(np.stack([_cells(o.edges[k], vel[:, 3, k]) for k in range(3)], 1) >= 0, 1)
    assert np.array_equal(~kept, out_a | out_b)
    # the pre-collision velocities are nodes
    V = o.node_velocities()
    np.testing.assert_array_equal(vel[:, 0], V[idx[:, 0]])


def _enumerate_direct(o, h, eps, M):
    """E[Delta N_j] (gain, loss) over the discrete collision operator: every
    ordered node pair (a, b) with weight w_a w_b, a midpoint rule in
    (u6, u7) for the direction k = (s cos 2 pi u7, s sin 2 pi u7, 2 u6 - 1),
    post-collision cells by search; written independently of the oracle."""
    V = o.node_velocities()
    w = o.node_weights()
    n = o.nv3
    u = (np.arange(M) + 0.5) / M
    u6, u7 = np.meshgrid(u, u, indexing="ij")
    kz = (2 * u6 - 1).ravel()
    s = np.sqrt(1 - kz * kz)
    kk = np.stack([s * np.cos(2 * np.pi * u7.ravel()), s * np.sin(2 * np.pi * u7.ravel()), kz], 1)
    G = np.zeros(len(w))
    L = np.zeros(len(w))
    for a in range(len(w)):
        alpha = (V - V[a]) @ kk.T  # (b, dir)
        vs = V[a][None, None, :] + alpha[..., None] * kk[None, :, :]
        v1s = V[:, None, :] - alpha[..., None] * kk[None, :, :]
        ca = np.stack([_cells(o.edges[k], vs[..., k]) for k in range(3)], -1)
        cb = np.stack([_cells(o.edges[k], v1s[..., k]) for k in range(3)], -1)
        kept = np.all(ca >= 0, -1) & np.all(cb >= 0, -1)
        g = h[a] + h + eps * h[a] * h
        wt = (w[a] * w * g)[:, None] * np.abs(alpha) * kept / (M * M)
        ja = (ca[..., 0] * n[1] + ca[..., 1]) * n[2] + ca[..., 2]
        jb = (cb[..., 0] * n[1] + cb[..., 1]) * n[2] + cb[..., 2]
        np.add.at(G, ja[kept], wt[kept])
        np.add.at(G, jb[kept], wt[kept])
        tot = wt.sum(1)
        L[a] += tot.sum()
        L += tot
    return o.dt * o.K * G, o.dt * o.K * L


def test_stretched_mc_mean_matches_enumeration_per_node(oracle_mod):
    n, a, r, eps, delta, nt, nb = 4, 2.5, 0.7, 0.5, 1.0, 20000, 200
    o = oracle_mod.Oracle(1, 1, n, a, delta, eps, nt, bc=oracle_mod.BC_PERIODIC, mix16=4, rv=r)
    V = o.node_velocities()
    w = o.node_weights()
    h = 0.8 * np.sin(0.7 * V[:, 0] + 0.3) * np.cos(0.5 * V[:, 1]) + 0.5 * np.cos(0.6 * V[:, 2] - 0.2)
    G = np.zeros((nb, n**3))
    L = np.zeros((nb, n**3))
    for st in range(nb):
        idx, q = o.debug_pairs(0, st, 0, nt)
        kept = idx[:, 2] >= 0
        ia, ib, isa, isb, qk = idx[kept, 0], idx[kept, 1], idx[kept, 2], idx[kept, 3], q[kept]
        c = qk * (h[ia] + h[ib] + eps * h[ia] * h[ib])
        G[st] = np.bincount(isa, c, n**3) + np.bincount(isb, c, n**3)
        L[st] = np.bincount(ia, c, n**3) + np.bincount(ib, c, n**3)
        if st == 0:
            _, dN, _ = o.collide(h.reshape(1, 1, -1), st, correction=False, want_dN=True)
            assert np.abs(dN.ravel() - (G[0] - L[0])).max() <= 1e-12 * (np.abs(G[0]) + np.abs(L[0])).max()
    Eg, El = _enumerate_direct(o, h, eps, 128)
    Eg2, El2 = _enumerate_direct(o, h, eps, 64)
    for S, E, E2 in ((L, El, El2), (G, Eg, Eg2)):
        mean, se = S.mean(0) / w, S.std(0, ddof=1) / np.sqrt(nb) / w
        # the direction quadrature (midpoint, discontinuous integrand) has
        # converged to about the Monte Carlo error; its change from 64 to
        # 128 points serves as its error estimate in the z-scores
        qe = np.abs(E - E2) / w
        assert np.max(qe / se) < 2.0
        se = np.sqrt(se**2 + qe**2)
        d = S - S.mean(0)
        skew = (d**3).mean(0) / np.maximum((d**2).mean(0), 1e-300) ** 1.5
        z = (mean - E / w) / se
        bound = 5.0 + 4.0 * np.abs(skew) / np.sqrt(nb)
        assert np.all(np.abs(z) < bound), np.max(np.abs(z) - bound)
        sym = np.abs(skew) < 2.0
        assert sym.mean() > 0.5 and 0.5 < float((z[sym] ** 2).mean()) < 1.7
