"""Pins of the oracle on stretched spatial cells (Sec. 5.1: cell lengths in
progression ratios r_x, r_y, the smallest at the side walls and at the lid),
first-order streaming (Eq. streaming2D with the Courant numbers of each
cell), CPU only.

* Widths: they add up to the cavity side, mirror-symmetric in x, neighbours
  in the ratio r toward the walls / lid; r = 1 gives the uniform grid
  exactly.
* Mass: on a periodic grid the upwind finite-volume update keeps
  sum_ij dx_i dy_j h_ij for every velocity node (the fluxes telescope); a
  Courant number taken from the wrong cell breaks it.
* Geometry: for a state uniform in y the update is the cell average of the
  piecewise-constant profile shifted by v_x dt, computed here from interval
  overlaps on the stretched edges (likewise in y).
* Time step: the CFL number applies to the smallest cells.
* Lid shear: a state uniform in x gives the same D as on uniform x cells
  (the face weights add up to one).
"""
import numpy as np
import pytest


def _o(oracle_mod, **kw):
    args = dict(nx=10, ny=7, nv=(6, 4, 4), vmax=3.0, delta=1.0, eps=0.1, n_pairs=10, order=1,
                bc=oracle_mod.BC_PERIODIC, rx=0.9, ry=0.8)
    args.update(kw)
    return oracle_mod.Oracle(**args)


@pytest.mark.parametrize("n,r", [(10, 0.9), (11, 0.996), (7, 0.5), (2, 0.8)])
def test_widths(oracle_mod, n, r):
    o = _o(oracle_mod, nx=n, ny=n + 3, rx=r, ry=r)
    wx, wy = o.wx, o.wy
    assert abs(wx.sum() - 1.0) < 1e-15 and abs(wy.sum() - 1.0) < 1e-15
    np.testing.assert_allclose(wx, wx[::-1], rtol=1e-15)
    # x: smaller toward each side wall, ratio r between neighbours
    h = n // 2
    np.testing.assert_allclose(wx[:h - 1] / wx[1:h], r, rtol=1e-13)
    # y: smaller toward the lid (last row), ratio r between neighbours
    np.testing.assert_allclose(wy[1:] / wy[:-1], r, rtol=1e-13)
    u = _o(oracle_mod, nx=n, ny=n + 3, rx=1.0, ry=0.0)
    assert np.all(u.wx == 1.0 / n) and np.all(u.wy == 1.0 / (n + 3))


def test_uniform_limit_is_the_uniform_grid(oracle_mod):
    rng = np.random.default_rng(1)
    a = _o(oracle_mod, rx=1.0, ry=1.0, bc=oracle_mod.BC_CAVITY)
    b = _o(oracle_mod, rx=0.0, ry=0.0, bc=oracle_mod.BC_CAVITY)
    h = 0.3 * rng.standard_normal(a.shape)
    w = oracle_mod.Walls(lid_u=0.1, tau_left=1.05)
    assert a.dt == b.dt
    np.testing.assert_array_equal(a.stream(h, w), b.stream(h, w))


def test_mass_kept_on_a_periodic_stretched_grid(oracle_mod):
    o = _o(oracle_mod)
    rng = np.random.default_rng(2)
    h = rng.standard_normal(o.shape)
    area = np.outer(o.wy, o.wx)[:, :, None]
    m0 = (area * h).sum((0, 1))
    for _ in range(5):
        h = o.stream(h)
        np.testing.assert_allclose((area * h).sum((0, 1)), m0, rtol=0, atol=1e-13 * np.abs(m0).max())


def _shifted_average(edges, f, s):
    """Cell averages over [e_i, e_{i+1}) of the periodic piecewise-constant
    profile f (values on the cells of `edges`, period 1) shifted by s."""
    n = len(f)
    out = np.zeros(n)
    for i in range(n):
        lo, hi = edges[i] - s, edges[i + 1] - s
        tot = 0.0
        for p in (-1, 0, 1):
            for k in range(n):
                a, b = edges[k] + p, edges[k + 1] + p
                ov = min(hi, b) - max(lo, a)
                if ov > 0:
                    tot += ov * f[k]
        out[i] = tot / (edges[i + 1] - edges[i])
    return out


@pytest.mark.parametrize("axis", [0, 1])
def test_update_is_the_shifted_cell_average(oracle_mod, axis):
    o = _o(oracle_mod)
    rng = np.random.default_rng(3 + axis)
    V = o.node_velocities()
    prof = rng.standard_normal((o.nx if axis == 0 else o.ny, o.nv))
    if axis == 0:
        h = np.broadcast_to(prof[None, :, :], o.shape).copy()
        w = o.wx
    else:
        h = np.broadcast_to(prof[:, None, :], o.shape).copy()
        w = o.wy
    out = o.stream(h)
    edges = np.concatenate([[0.0], np.cumsum(w)])
    edges[-1] = 1.0
    for j in range(o.nv):
        s = V[j, axis] * o.dt
        ref = _shifted_average(edges, prof[:, j], s)
        got = out[0, :, j] if axis == 0 else out[:, 0, j]
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13)


def test_time_step_from_the_smallest_cells(oracle_mod):
    o = _o(oracle_mod, bc=oracle_mod.BC_CAVITY, cfl=0.5)
    vmx, vmy = abs(o.v[0][0]), abs(o.v[1][0])
    assert o.dt == pytest.approx(0.5 / max(vmx / o.wx.min(), vmy / o.wy.min()), rel=1e-15)
    # the unsplit first-order scheme is stable for Cx + Cy <= 1 in every cell
    assert vmx * o.dt / o.wx.min() + vmy * o.dt / o.wy.min() <= 1.0 + 1e-12
    for bad in (dict(order=2), dict(rx=1.5), dict(ry=-0.1)):
        with pytest.raises(ValueError):
            _o(oracle_mod, **bad)


def test_lid_shear_of_a_state_uniform_in_x(oracle_mod):
    kw = dict(bc=oracle_mod.BC_CAVITY, nv=(8, 8, 4), vmax=3.0)
    a = _o(oracle_mod, **kw)
    b = _o(oracle_mod, rx=1.0, **kw)
    rng = np.random.default_rng(5)
    prof = 0.2 * rng.standard_normal((a.ny, a.nv))
    h = np.broadcast_to(prof[:, None, :], a.shape).copy()
    w = oracle_mod.Walls(lid_u=0.2)
    _, Da = a.moments(h, w, lid_shear=True)
    _, Db = b.moments(h, w, lid_shear=True)
    assert Da == pytest.approx(Db, rel=1e-13, abs=1e-15)
    assert abs(Da) > 1e-3


def test_adjoint_refused_on_stretched_cells(oracle_mod):
    o = _o(oracle_mod, bc=oracle_mod.BC_CAVITY)
    h = np.zeros(o.shape)
    with pytest.raises(RuntimeError):
        o.stream_adjoint(h, h, oracle_mod.Walls(lid_u=0.1))
