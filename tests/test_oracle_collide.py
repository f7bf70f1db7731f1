"""Pins of the oracle's collision step (CPU only).

* MC collision mean vs exhaustive enumeration on a 6^3 velocity grid
  (all ordered node pairs, deterministic direction quadrature).
* Exact conservation of mass, momentum and energy per collision step.
* h = 0 is a bitwise fixed point; a drifting Maxwellian stays within its
  Monte Carlo noise of the enumerated discrete bias.
* Collision scale: the initial decay rate of Pi_xy for h ~ v_x v_y equals the
  first Chapman-Enskog value p0/mu[1] = 1.016034 delta.
* Moments of a full Maxwellian; MC noise ~ N_t^-1/2.
"""
import numpy as np
import pytest

K_OVER_DELTA = (5.0 / 16.0) * np.sqrt(2 * np.pi) * 1.016034


def _axis(n, a):
    dv = 2 * a / n
    v = (np.arange(n) + 0.5 - n / 2) * dv
    om = dv * np.exp(-v * v) / np.sqrt(np.pi)
    return v, om, dv


def _enumerate_mean_dN(n, a, h, eps, dt, delta, M, parts=False):
    """E[Delta N_j] over the sampling law, written independently of the oracle.

    On a uniform grid the post-collision cell of v_a + d is a + floor(d/dv + 1/2)
    per axis, so the direction integral depends only on v_r = v_b - v_a.  The
    direction integral is a midpoint rule on (u6, u7) in (0,1)^2 with
    k = (s cos 2 pi u7, s sin 2 pi u7, 2 u6 - 1), i.e. uniform on the sphere.
    """
    v, om, dv = _axis(n, a)
    p = om / om.sum()
    W = om.sum() ** 3
    K = K_OVER_DELTA * delta
    grid = np.stack(np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij"), -1).reshape(-1, 3)
    pa = p[grid[:, 0]] * p[grid[:, 1]] * p[grid[:, 2]]
    u = (np.arange(M) + 0.5) / M
    u6, u7 = np.meshgrid(u, u, indexing="ij")
    kz = (2 * u6 - 1).ravel()
    s = np.sqrt(1 - kz * kz)
    kx, ky = s * np.cos(2 * np.pi * u7.ravel()), s * np.sin(2 * np.pi * u7.ravel())
    kk = np.stack([kx, ky, kz], 1)
    E = np.zeros(n**3)
    Eg = np.zeros(n**3)
    rng_off = np.arange(-(n - 1), n)
    for rx in rng_off:
        for ry in rng_off:
            for rz in rng_off:
                r = np.array([rx, ry, rz])
                alpha = dv * (kk @ r)
                d = alpha[:, None] * kk / dv
                oa = np.floor(d + 0.5).astype(np.int64)
                ob = np.floor(-d + 0.5).astype(np.int64)
                key = ((oa + 16) * np.array([1, 32, 1024])).sum(1) + 32768 * ((ob + 16) * np.array([1, 32, 1024])).sum(1)
                uk, inv = np.unique(key, return_inverse=True)
                wsum = np.bincount(inv, weights=np.abs(alpha)) / (M * M)
                first = np.zeros(len(uk), dtype=np.int64)
                first[inv[::-1]] = np.arange(len(inv))[::-1]
                OA, OB = oa[first], ob[first]
                A = grid[np.all((grid + r >= 0) & (grid + r < n), 1)]
                if len(A) == 0:
                    continue
                B = A + r
                ia = (A[:, 0] * n + A[:, 1]) * n + A[:, 2]
                ib = (B[:, 0] * n + B[:, 1]) * n + B[:, 2]
                g = h[ia] + h[ib] + eps * h[ia] * h[ib]
                wt = pa[ia] * pa[ib] * g  # (P,)
                As = A[None, :, :] + OA[:, None, :]
                Bs = B[None, :, :] + OB[:, None, :]
                kept = np.all((As >= 0) & (As < n), 2) & np.all((Bs >= 0) & (Bs < n), 2)
                contrib = wsum[:, None] * wt[None, :] * kept
                ias = (As[..., 0] * n + As[..., 1]) * n + As[..., 2]
                ibs = (Bs[..., 0] * n + Bs[..., 1]) * n + Bs[..., 2]
                np.add.at(E, ias[kept], contrib[kept])
                np.add.at(E, ibs[kept], contrib[kept])
                np.add.at(Eg, ias[kept], contrib[kept])
                np.add.at(Eg, ibs[kept], contrib[kept])
                np.add.at(E, np.broadcast_to(ia, kept.shape)[kept], -contrib[kept])
                np.add.at(E, np.broadcast_to(ib, kept.shape)[kept], -contrib[kept])
    if parts:
        # (gain, loss): the expected increments at a*, b* and (as positive
        # numbers) the expected decrements at a, b
        return dt * K * W * W * Eg, dt * K * W * W * (Eg - E)
    return dt * K * W * W * E


def _mc_dN(oracle_mod, n, a, h, eps, delta, nt, nsteps, mix16=4):
    o = oracle_mod.Oracle(1, 1, n, a, delta, eps, nt, bc=oracle_mod.BC_PERIODIC, mix16=mix16)
    samples = []
    for st in range(nsteps):
        _, dN, _ = o.collide(h.reshape(1, 1, -1), st, correction=False, want_dN=True)
        samples.append(dN.ravel())
    return o, np.array(samples)


def _h_test(n, a, kind, eps):
    v, _, _ = _axis(n, a)
    V = np.stack(np.meshgrid(v, v, v, indexing="ij"), -1).reshape(-1, 3)
    if kind == "nonequilibrium":
        return 0.6 * V[:, 0] * V[:, 1] - 0.4 * V[:, 2] + 0.3 * (V**2).sum(1) - 0.2 * V[:, 0] ** 3
    # drifting, heated Maxwellian: F = n/T^1.5 exp(-|v-u|^2/T) / exp(-|v|^2)
    u, T, rho = np.array([0.2, -0.1, 0.05]), 1.1, 1.05
    F = rho * T**-1.5 * np.exp((V**2).sum(1) - ((V - u) ** 2).sum(1) / T)
    return (F - 1) / eps


@pytest.mark.parametrize("kind,mix16", [("nonequilibrium", 0), ("maxwellian", 0), ("nonequilibrium", 4)])
def test_mc_mean_matches_enumeration_6cubed(oracle_mod, kind, mix16):
    # the mixture of the Maxwellian and uniform node laws (mix16 > 0) is an
    # importance-sampling estimate of the same integral: same expectation
    n, a, eps, delta = 6, 3.0, 0.5, 1.0
    h = _h_test(n, a, kind, eps)
    o, S = _mc_dN(oracle_mod, n, a, h, eps, delta, nt=20000, nsteps=100, mix16=mix16)
    mean = S.mean(0)
    se = S.std(0, ddof=1) / np.sqrt(S.shape[0])
    E = _enumerate_mean_dN(n, a, h, eps, o.dt, delta, M=256)
    E_half = _enumerate_mean_dN(n, a, h, eps, o.dt, delta, M=128)
    # Gaussian regime: nodes touched in (almost) every batch of N_t pairs
    live = (S != 0).mean(0) >= 0.9
    assert live.sum() > 0.6 * n**3
    # the quadrature has converged well below the Monte Carlo error
    assert np.max(np.abs(E - E_half)[live] / se[live]) < 0.5
    z = (mean - E)[live] / se[live]
    assert np.max(np.abs(z)) < 5.0, np.max(np.abs(z))
    chi2 = float((z**2).mean())
    assert 0.6 < chi2 < 1.6, chi2
    # rarely reached nodes carry a negligible share of the expected increment,
    # and their sampled total agrees with it within Poisson-size noise
    rare = ~live
    assert np.abs(E[rare]).sum() <= 0.05 * np.abs(E).sum()
    assert abs(mean[rare].sum() - E[rare].sum()) <= 5 * np.sqrt((se[rare] ** 2).sum()) + 1e-3 * np.abs(E).sum()
    if kind == "maxwellian":
        # the discrete bias of an equilibrium is small next to the response to
        # a comparable non-equilibrium perturbation
        h2 = _h_test(n, a, "nonequilibrium", eps)
        E2 = _enumerate_mean_dN(n, a, h2 * np.abs(h).max() / np.abs(h2).max(), eps, o.dt, delta, M=64)
        assert np.abs(E).sum() < 0.35 * np.abs(E2).sum()


def test_mc_mean_matches_enumeration_per_node_8cubed(oracle_mod):
    """Every node of an 8^3 grid on [-4, 4], whose 12-bit Maxwellian law gives
    the two outer nodes of each axis probability zero, with the mixture law
    (a quarter uniform) that reaches them all.  Gain and loss parts are
    compared separately, node by node, in units of h (E/w): the loss at a
    node comes from the draws of that node and is well sampled everywhere;
    the gain at the edge nodes comes mostly from rare, large events (bulk
    pairs landing there) whose batch sums are strongly skewed, so there the
    5-sigma bound is widened by the first Cornish-Fisher term of the sample
    mean's skewness (skew / sqrt(batches)).  The oracle's
    own scatter (collide's Delta N) is the gain minus the loss of its
    sampled pairs."""
    n, a, eps, delta, nt, nb = 8, 4.0, 0.5, 1.0, 20000, 1200
    v, _, _ = _axis(n, a)
    V = np.stack(np.meshgrid(v, v, v, indexing="ij"), -1).reshape(-1, 3)
    h = 0.8 * np.sin(0.7 * V[:, 0] + 0.3) * np.cos(0.5 * V[:, 1]) + 0.5 * np.cos(0.6 * V[:, 2] - 0.2) \
        + 0.3 * np.tanh(V[:, 0] * V[:, 1] / 4)
    with pytest.raises(ValueError, match="mix16 = 0"):
        oracle_mod.Oracle(1, 1, n, a, delta, eps, nt, bc=oracle_mod.BC_PERIODIC, mix16=0)
    o = oracle_mod.Oracle(1, 1, n, a, delta, eps, nt, bc=oracle_mod.BC_PERIODIC, mix16=4)
    w = o.node_weights()
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
            scale = (np.abs(G[0]) + np.abs(L[0])).max()
            assert np.abs(dN.ravel() - (G[0] - L[0])).max() <= 1e-12 * scale
    Eg, El = _enumerate_mean_dN(n, a, h, eps, o.dt, delta, M=256, parts=True)
    Eg2, El2 = _enumerate_mean_dN(n, a, h, eps, o.dt, delta, M=128, parts=True)
    for S, E, E2 in ((L, El, El2), (G, Eg, Eg2)):
        mean, se = S.mean(0), S.std(0, ddof=1) / np.sqrt(nb)
        # the quadrature has converged below the Monte Carlo error
        assert np.max(np.abs(E - E2) / se) < 1.0
    # loss: every node, in h units
    mean, se = L.mean(0) / w, L.std(0, ddof=1) / np.sqrt(nb) / w
    z = (mean - El / w) / se
    assert np.all(np.abs(El) > 0)
    assert np.max(np.abs(z)) < 5.0, np.max(np.abs(z))
    assert 0.6 < float((z**2).mean()) < 1.6
    # gain: every node, 5 sigma plus the Cornish-Fisher skewness term
    # (z^2 - 1) gamma / 6 of the sample mean (gamma = skew / sqrt(batches))
    mean, se = G.mean(0) / w, G.std(0, ddof=1) / np.sqrt(nb) / w
    d = G - G.mean(0)
    skew = (d**3).mean(0) / np.maximum((d**2).mean(0), 1e-300) ** 1.5
    z = (mean - Eg / w) / se
    bound = 5.0 + (25.0 - 1.0) / 6.0 * np.abs(skew) / np.sqrt(nb)
    assert np.all(np.abs(z) < bound), np.max(np.abs(z) - bound)
    sym = np.abs(skew) < 2.0
    assert np.max(np.abs(z[sym])) < 5.0 and 0.6 < float((z[sym] ** 2).mean()) < 1.6


def test_raw_increments_conserve_mass_per_pair(oracle_mod):
    o = oracle_mod.Oracle(4, 3, 8, 3.5, 2.0, 0.3, 3000, bc=oracle_mod.BC_PERIODIC)
    rng = np.random.default_rng(3)
    h = rng.standard_normal(o.shape)
    _, dN, _ = o.collide(h, 11, correction=False, want_dN=True)
    scale = np.abs(dN).sum(2)
    assert np.all(np.abs(dN.sum(2)) <= 1e-13 * scale)


@pytest.mark.parametrize("grid", [(12, 4.5), (8, 3.0)])
def test_correction_conserves_mass_momentum_energy(oracle_mod, grid):
    n, a = grid
    o = oracle_mod.Oracle(5, 4, n, a, 10.0, 0.1, 2000, bc=oracle_mod.BC_PERIODIC)
    rng = np.random.default_rng(7)
    h = 0.5 * rng.standard_normal(o.shape)
    out, dN, defect = o.collide(h, 3, correction=True, want_dN=True, want_defect=True)
    V = o.node_velocities()
    w = o.node_weights()
    psi = np.stack([np.ones(len(w)), V[:, 0], V[:, 1], V[:, 2], (V**2).sum(1)], 1)
    hc = h + dN / w
    scale = o.eps * np.einsum("j,jk,ycj->yck", w, np.abs(psi), np.abs(h) + np.abs(hc - h))
    assert np.all(np.abs(defect) <= 1e-12 * scale)
    # the same defect recomputed here from the returned state
    d2 = o.eps * np.einsum("j,jk,ycj->yck", w, psi, out - h)
    assert np.all(np.abs(d2) <= 1e-12 * scale)
    # before the correction momentum/energy are not conserved (the correction did work)
    d_raw = o.eps * np.einsum("j,jk,ycj->yck", w, psi, hc - h)
    assert np.abs(d_raw[..., 1:]).max() > 1e3 * np.abs(defect[..., 1:]).max()


def test_zero_is_bitwise_fixed_point(oracle_mod):
    o = oracle_mod.Oracle(6, 5, 12, 4.5, 10.0, 0.1, 2000, order=2)
    h = np.zeros(o.shape)
    assert np.all(o.collide(h, 0) == 0.0)
    rest = oracle_mod.Walls()
    assert np.all(o.stream(h, rest) == 0.0)
    assert np.all(o.step(h, rest, 5) == 0.0)
    o1 = oracle_mod.Oracle(6, 5, 12, 4.5, 10.0, 0.1, 2000, order=1)
    assert np.all(o1.step(h, rest, 5) == 0.0)


def test_collision_scale_is_first_chapman_enskog_viscosity(oracle_mod):
    # h ~ v_x v_y, eps -> 0: d Pi_xy/dt = -(p0/mu[1]) Pi_xy with
    # p0/mu[1] = 1.016034 delta (units L/V0, lambda0 = L/delta).
    n, a, delta = 16, 4.0, 1.0
    o = oracle_mod.Oracle(1, 1, n, a, delta, 1e-8, 100000, bc=oracle_mod.BC_PERIODIC)
    V = o.node_velocities()
    w = o.node_weights()
    h = V[:, 0] * V[:, 1]
    rates = []
    for st in range(8):
        _, dN, _ = o.collide(h.reshape(1, 1, -1), st, correction=False, want_dN=True)
        pxy0 = 2 * np.sum(w * h * V[:, 0] * V[:, 1])
        dpxy = 2 * np.sum(dN.ravel() * V[:, 0] * V[:, 1])
        rates.append(-dpxy / (pxy0 * o.dt))
    rate = np.mean(rates)
    assert abs(rate / (1.016034 * delta) - 1) < 0.03, rate


def test_moments_of_full_maxwellian(oracle_mod):
    eps = 0.2
    o = oracle_mod.Oracle(2, 2, 24, 5.0, 1.0, eps, 10, bc=oracle_mod.BC_PERIODIC)
    V = o.node_velocities()
    cases = [(0.3, [0.2, -0.4, 0.1], 0.25), (-0.5, [0.0, 0.3, -0.2], -0.4)]
    h = np.zeros(o.shape)
    for c, (rho, u, th) in enumerate(cases):
        u = np.array(u)
        n, T = 1 + eps * rho, 1 + eps * th
        F = n * T**-1.5 * np.exp((V**2).sum(1) - ((V - eps * u) ** 2).sum(1) / T)
        h[c // 2, c % 2] = (F - 1) / eps
    mom = o.moments(h)
    for c, (rho, u, th) in enumerate(cases):
        m = mom[c // 2, c % 2]
        assert abs(m[0] - rho) < 1e-9
        np.testing.assert_allclose(m[1:4], u, atol=1e-9)
        assert abs(m[4] - th) < 1e-9
        # isotropic stress: Pi = ((1+eps rho)(1+eps theta) - 1)/eps on the diagonal
        pd = ((1 + eps * rho) * (1 + eps * th) - 1) / eps
        np.testing.assert_allclose(m[[5, 8, 10]], pd, atol=1e-9)
        np.testing.assert_allclose(m[[6, 7, 9]], 0.0, atol=1e-9)


def test_mc_noise_scales_as_inverse_sqrt_nt(oracle_mod):
    n, a = 8, 3.5
    h = _h_test(n, a, "nonequilibrium", 0.2)
    sig = []
    for nt in (500, 2000, 8000):
        _, S = _mc_dN(oracle_mod, n, a, h, 0.2, 1.0, nt, 60)
        sig.append(np.sqrt((S.std(0) ** 2).sum()))
    r1, r2 = sig[0] / sig[1], sig[1] / sig[2]
    assert 1.7 < r1 < 2.3 and 1.7 < r2 < 2.3, (r1, r2)


def test_sample_groups_share_streams(oracle_mod):
    o1 = oracle_mod.Oracle(4, 4, 6, 3.0, 1.0, 0.1, 50, bc=oracle_mod.BC_PERIODIC, sample_group=4)
    i0, _ = o1.debug_pairs(0, 2, 0, 50)
    i3, _ = o1.debug_pairs(3, 2, 0, 50)
    i4, _ = o1.debug_pairs(4, 2, 0, 50)
    assert np.array_equal(i0, i3) and not np.array_equal(i0, i4)
    o0 = oracle_mod.Oracle(4, 4, 6, 3.0, 1.0, 0.1, 50, bc=oracle_mod.BC_PERIODIC, sample_group=0)
    assert np.array_equal(o0.debug_pairs(0, 2, 0, 50)[0], o0.debug_pairs(15, 2, 0, 50)[0])
    # different steps and seeds give different streams
    assert not np.array_equal(o0.debug_pairs(0, 2, 0, 50)[0], o0.debug_pairs(0, 3, 0, 50)[0])
