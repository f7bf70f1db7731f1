"""Pins of the oracle's in-place sequential collision (Alg. 3), CPU only.

In that form the samples update h one after another: sample m reads the
current h at its nodes a and b and changes h at a*, b*, a and b before
sample m + 1 is read.  The Jacobi form (Eq. collision_step) evaluates every
sample at the post-stream h.  The pins:

* With eps -> 0 the update is linear: sample m maps h to (I + T_m) h with
  T_m = q_m u_m (e_a + e_b)^T, u_m = e_a*/w_a* + e_b*/w_b* - e_a/w_a - e_b/w_b.
  The sequential result is the ordered matrix product applied to h^s,
  formed here as a product of matrices in a balanced tree.
* The difference from the Jacobi form is second order in the time step,
  sum over m of T_m (sum over m' < m of T_m') h^s at leading order; the
  ordering of the double sum is what a reversed or Jacobi loop gets wrong.
* One sample per cell: the sequential and Jacobi forms coincide.
* Every sample moves particles between nodes without creating any, so the
  weighted sum of h is unchanged without the correction, also where two of
  a sample's four nodes coincide (a literal load-all, store-all reading of
  Alg. 3 loses one of the two increments there: negative control below).
* With the correction the moments of the post-stream state are restored.
"""
import numpy as np
import pytest


def _oracle(oracle_mod, seq=True, **kw):
    args = dict(nx=1, ny=1, nv=4, vmax=2.5, delta=5.0, eps=1e-9, n_pairs=300, dt=0.05,
                bc=oracle_mod.BC_PERIODIC, sample_group=1, mix16=8)
    args.update(kw)
    if seq:
        args["flags"] = args.get("flags", 0) | oracle_mod.SEQUENTIAL
    return oracle_mod.Oracle(**args)


def _state(o, amp=0.6):
    V = o.node_velocities()
    h = amp * np.sin(0.7 * V[:, 0] + 0.3) * np.cos(0.5 * V[:, 1]) + 0.4 * np.cos(0.6 * V[:, 2] - 0.2)
    return h


def _maps(o, step, n):
    """The per-sample linear maps T_m of the kept samples, in sample order."""
    idx, q = o.debug_pairs(0, step, 0, n)
    w = o.node_weights()
    nv = len(w)
    T = []
    for (a, b, as_, bs), qm in zip(idx, q):
        if as_ < 0:
            continue
        u = np.zeros(nv)
        u[as_] += 1.0 / w[as_]
        u[bs] += 1.0 / w[bs]
        u[a] -= 1.0 / w[a]
        u[b] -= 1.0 / w[b]
        s = np.zeros(nv)
        s[a] += 1.0
        s[b] += 1.0
        T.append(qm * np.outer(u, s))
    return T


def _tree_product(mats):
    """M_{n-1} ... M_1 M_0 by pairwise products of neighbours."""
    while len(mats) > 1:
        nxt = [mats[i + 1] @ mats[i] for i in range(0, len(mats) - 1, 2)]
        if len(mats) % 2:
            nxt.append(mats[-1])
        mats = nxt
    return mats[0]


def test_linear_limit_is_the_ordered_product(oracle_mod):
    o = _oracle(oracle_mod)
    h = _state(o)
    got = o.collide(h.reshape(1, 1, -1), 3, correction=False).ravel()
    T = _maps(o, 3, 300)
    assert len(T) > 200
    eye = np.eye(len(h))
    ref = _tree_product([eye + t for t in T]) @ h
    scale = np.abs(ref).max()
    # eps h_a h_b terms are 1e-9 of the linear ones
    assert np.abs(got - ref).max() <= 1e-8 * scale
    # the order matters at this time step: the reversed product and the
    # Jacobi (sum) form are far away
    rev = _tree_product([eye + t for t in T[::-1]]) @ h
    jac = h + sum(T) @ h
    assert np.abs(rev - ref).max() > 1e-3 * scale
    assert np.abs(jac - ref).max() > 1e-3 * scale


def test_difference_from_jacobi_is_the_second_order_term(oracle_mod):
    dts = [2e-3, 1e-3]
    diffs = []
    for dt in dts:
        o = _oracle(oracle_mod, dt=dt)
        oj = _oracle(oracle_mod, seq=False, dt=dt)
        h = _state(o)
        seq = o.collide(h.reshape(1, 1, -1), 5, correction=False).ravel()
        jac = oj.collide(h.reshape(1, 1, -1), 5, correction=False).ravel()
        T = _maps(o, 5, 300)
        # leading term: sum_m T_m (sum_{m' < m} T_m') h
        pre = np.zeros_like(h)
        d2 = np.zeros_like(h)
        for t in T:
            d2 += t @ pre
            pre += t @ h
        D = seq - jac
        assert np.abs(D - d2).max() <= 0.05 * np.abs(d2).max()
        diffs.append(np.abs(D).max())
    # halving the time step quarters the difference
    assert 3.7 < diffs[0] / diffs[1] < 4.3


def test_one_sample_per_cell_equals_jacobi(oracle_mod):
    for corr in (False, True):
        kw = dict(nx=3, ny=2, nv=(6, 5, 6), vmax=3.0, eps=0.3, n_pairs=1, dt=0.01, delta=1.0)
        o = _oracle(oracle_mod, **kw)
        oj = _oracle(oracle_mod, seq=False, **kw)
        rng = np.random.default_rng(4)
        h = 0.5 * rng.standard_normal(o.shape)
        for step in range(4):
            a = o.collide(h, step, correction=corr)
            b = oj.collide(h, step, correction=corr)
            np.testing.assert_allclose(a, b, rtol=1e-14, atol=1e-14)


def test_mass_conserved_where_nodes_coincide(oracle_mod):
    # 3^3 nodes and 2000 samples: many samples have coinciding nodes
    o = _oracle(oracle_mod, nv=3, vmax=2.0, eps=0.5, n_pairs=2000, dt=0.02, mix16=16)
    h = _state(o, amp=0.9)
    w = o.node_weights()
    idx, q = o.debug_pairs(0, 1, 0, 2000)
    kept = idx[:, 2] >= 0
    coincide = kept & ((idx[:, 0] == idx[:, 2]) | (idx[:, 0] == idx[:, 3]) | (idx[:, 1] == idx[:, 2]) |
                       (idx[:, 1] == idx[:, 3]) | (idx[:, 2] == idx[:, 3]) | (idx[:, 0] == idx[:, 1]))
    assert coincide.sum() > 100
    out = o.collide(h.reshape(1, 1, -1), 1, correction=False).ravel()
    assert abs(np.dot(w, out - h)) <= 1e-13 * np.dot(w, np.abs(h))
    assert np.abs(out - h).max() > 1e-2
    # negative control: loading the four values first and storing the four
    # updated values afterwards drops an increment where nodes coincide
    lit = h.copy()
    eps = 0.5
    for (a, b, as_, bs), qm in zip(idx, q):
        if as_ < 0:
            continue
        ha, hb, hsa, hsb = lit[a], lit[b], lit[as_], lit[bs]
        qg = qm * ((ha + hb) + eps * ha * hb)
        ha -= qg / w[a]
        hb -= qg / w[b]
        hsa += qg / w[as_]
        hsb += qg / w[bs]
        lit[a], lit[b], lit[as_], lit[bs] = ha, hb, hsa, hsb
    assert abs(np.dot(w, lit - h)) > 1e-6 * np.dot(w, np.abs(h))


def test_correction_restores_the_moments(oracle_mod):
    o = _oracle(oracle_mod, nx=2, ny=2, nv=(8, 6, 8), vmax=3.0, eps=0.2, n_pairs=3000, dt=0.05,
                sample_group=0)
    rng = np.random.default_rng(9)
    h = 0.5 * rng.standard_normal(o.shape)
    out, dN, defect = o.collide(h, 2, want_dN=True, want_defect=True)
    w = o.node_weights()
    assert np.abs(defect).max() <= 1e-12 * o.eps * np.abs(h * w).sum(-1).max()
    # dN is the change of particles per node of the uncorrected update
    raw = o.collide(h, 2, correction=False)
    np.testing.assert_allclose(dN, (raw - h) * w, rtol=0, atol=1e-15 * np.abs(h * w).max())
    # and the correction did change something
    assert np.abs(out - raw).max() > 1e-6


def test_sequential_refuses_the_adjoint(oracle_mod):
    o = _oracle(oracle_mod)
    h = _state(o).reshape(1, 1, -1)
    with pytest.raises(RuntimeError):
        o.collide_adjoint(h, h, 0)
