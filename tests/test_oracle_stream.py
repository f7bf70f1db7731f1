"""Pins of the oracle's streaming step and diffuse walls (CPU only).

* A uniform state is unchanged (periodic, and cavity with walls at rest).
* Exact grid shifts: Beam-Warming at Courant numbers 1 and 2, the
  first-order scheme at Courant number 1.
* Total mass sum_cells sum_j w_j F_j is conserved through diffuse walls.
* Observed convergence orders 1 and 2 against the exact translation.
* Walls at rest facing h = 0: n_w = 1 and the re-emitted h_w = 0 exactly.
* Host-side validation errors.
"""
import numpy as np
import pytest


def _smooth(o, kx=1, ky=1, phase=0.3):
    x = (np.arange(o.nx) + 0.5) / o.nx
    y = (np.arange(o.ny) + 0.5) / o.ny
    X, Y = np.meshgrid(x, y)  # (ny, nx)
    base = np.sin(2 * np.pi * (kx * X + phase)) * np.cos(2 * np.pi * ky * Y)
    return base


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("bc", [0, 1])
def test_uniform_state_is_preserved(oracle_mod, order, bc):
    o = oracle_mod.Oracle(7, 5, (8, 6, 4), (3.5, 3.0, 2.5), 1.0, 0.1, 10, order=order, bc=bc)
    for c in (0.0, 0.37, -1.25):
        h = np.full(o.shape, c)
        out = o.stream(h, oracle_mod.Walls() if bc == 0 else None)
        assert np.abs(out - c).max() <= 1e-13 * max(1.0, abs(c))


@pytest.mark.parametrize("C", [1.0, 2.0])
def test_beam_warming_exact_shift(oracle_mod, C):
    # node with v_x = vsel: choose dt so that its Courant number is exactly C
    nx, ny = 12, 12
    o0 = oracle_mod.Oracle(nx, ny, (4, 4, 1), (2.0, 2.0, 1.0), 1.0, 0.1, 1, bc=1)
    vsel = o0.v[0][3]  # +1.5
    dt = C * o0.dx / vsel
    o = oracle_mod.Oracle(nx, ny, (4, 4, 1), (2.0, 2.0, 1.0), 1.0, 0.1, 1, bc=1, order=2, dt=dt,
                          flags=oracle_mod.ALLOW_UNSTABLE)
    rng = np.random.default_rng(0)
    h = rng.standard_normal(o.shape)
    out = o.stream(h)
    V = o.node_velocities()
    for j in range(o.nv):
        vx, vy = V[j, 0], V[j, 1]
        cx, cy = abs(vx) * dt / o.dx, abs(vy) * dt / o.dy
        if abs(cx - C) < 1e-14 and abs(cy - C) < 1e-14:
            sx, sy = int(round(C * np.sign(vx))), int(round(C * np.sign(vy)))
            expect = np.roll(np.roll(h[:, :, j], sx, axis=1), sy, axis=0)
            assert np.abs(out[:, :, j] - expect).max() <= 1e-14
            break
    else:
        raise AssertionError("no node with Courant number %g on both axes" % C)


def test_first_order_exact_shift(oracle_mod):
    # odd y grid: nodes with v_y = 0; dt makes C_x = 1 for the chosen v_x
    nx, ny = 9, 6
    o0 = oracle_mod.Oracle(nx, ny, (4, 3, 1), (2.0, 1.5, 1.0), 1.0, 0.1, 1, bc=1, order=1)
    vsel = o0.v[0][0]  # -1.5
    dt = o0.dx / abs(vsel)
    o = oracle_mod.Oracle(nx, ny, (4, 3, 1), (2.0, 1.5, 1.0), 1.0, 0.1, 1, bc=1, order=1, dt=dt,
                          flags=oracle_mod.ALLOW_UNSTABLE)
    rng = np.random.default_rng(1)
    h = rng.standard_normal(o.shape)
    out = o.stream(h)
    j = (0 * 3 + 1) * 1 + 0  # jx = 0 (v_x = -1.5), jy = 1 (v_y = 0)
    assert o.node_velocities()[j, 1] == 0.0
    expect = np.roll(h[:, :, j], -1, axis=1)
    assert np.abs(out[:, :, j] - expect).max() <= 1e-15


@pytest.mark.parametrize("order", [1, 2])
def test_total_mass_conserved_through_diffuse_walls(oracle_mod, order):
    eps = 0.2
    o = oracle_mod.Oracle(9, 7, (8, 8, 6), (3.5, 3.5, 3.0), 1.0, eps, 10, order=order)
    rng = np.random.default_rng(11)
    h = rng.standard_normal(o.shape)
    w = o.node_weights()
    walls = oracle_mod.Walls(lid_u=0.3, tau_left=1.1, tau_right=0.9, tau_bottom=1.05, tau_top=0.95)
    mass0 = np.einsum("j,yxj->", w, 1 + eps * h)
    for _ in range(5):
        h = o.stream(h, walls)
        mass = np.einsum("j,yxj->", w, 1 + eps * h)
        assert abs(mass - mass0) <= 1e-12 * mass0


@pytest.mark.parametrize("order", [1, 2])
def test_observed_convergence_order(oracle_mod, order):
    errs = []
    Ns = (16, 32, 64)
    T = 0.25
    for N in Ns:
        probe = oracle_mod.Oracle(N, N, (2, 2, 1), (1.0, 1.0, 1.0), 1.0, 0.1, 1, bc=1, order=order)
        nsteps = int(np.ceil(T / probe.dt))
        o = oracle_mod.Oracle(N, N, (2, 2, 1), (1.0, 1.0, 1.0), 1.0, 0.1, 1, bc=1, order=order,
                              dt=T / nsteps)
        h = np.repeat(_smooth(o)[:, :, None], o.nv, axis=2)
        for _ in range(nsteps):
            h = o.stream(h)
        x = (np.arange(N) + 0.5) / N
        X, Y = np.meshgrid(x, x)
        err = 0.0
        for j, (vx, vy, _) in enumerate(o.node_velocities()):
            exact = np.sin(2 * np.pi * (X - vx * T + 0.3)) * np.cos(2 * np.pi * (Y - vy * T))
            err = max(err, np.abs(h[:, :, j] - exact).max())
        errs.append(err)
    slopes = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(slopes > order - 0.25) and np.all(slopes < order + 0.35), slopes


@pytest.mark.parametrize("order", [1, 2])
def test_walls_at_rest_facing_equilibrium(oracle_mod, order):
    o = oracle_mod.Oracle(6, 5, 12, 4.5, 10.0, 0.1, 10, order=order)
    h = np.zeros(o.shape)
    nw = o.wall_density(h, oracle_mod.Walls())
    assert np.all(nw == 1.0)
    assert np.all(o.stream(h, oracle_mod.Walls()) == 0.0)
    # a heated left wall needs a smaller density to balance the same flux;
    # the other faces are untouched, except (order 2) the y-wall faces of
    # columns 0 and 1, which see the x-swept state next to the left wall
    nw2 = o.wall_density(h, oracle_mod.Walls(tau_left=1.2))
    ny, nx = o.ny, o.nx
    assert np.all(nw2[:ny] < 1.0) and np.all(nw2[ny:2 * ny] == 1.0)
    far = slice(2, nx) if order == 2 else slice(0, nx)
    assert np.all(nw2[2 * ny:2 * ny + nx][far] == 1.0) and np.all(nw2[2 * ny + nx:][far] == 1.0)


def test_moving_lid_drags_gas(oracle_mod):
    o = oracle_mod.Oracle(8, 8, 12, 4.5, 10.0, 0.1, 2000, order=2)
    h = np.zeros(o.shape)
    walls = oracle_mod.Walls(lid_u=0.1)
    for n in range(10):
        h = o.step(h, walls, n)
    mom, D = o.moments(h, walls, lid_shear=True)
    ux = mom[..., 1]
    assert ux[-1].mean() > 0 and ux[-1].mean() > 5 * abs(ux[0].mean())
    assert 0.1 < D < 1.0
    # x-momentum grows, total mass stays
    w = o.node_weights()
    assert abs(np.einsum("j,yxj->", w, h)) < 1e-10 * np.einsum("j,yxj->", w, np.abs(h))


def test_validation_errors(oracle_mod):
    with pytest.raises(ValueError):
        oracle_mod.Oracle(8, 8, 12, 4.5, 1.0, 0.1, 10, dt=1.0)  # Courant limit
    with pytest.raises(ValueError):
        oracle_mod.Oracle(1, 8, 12, 4.5, 1.0, 0.1, 10)  # cavity needs two cells per axis
    with pytest.raises(ValueError):
        oracle_mod.Oracle(8, 8, 12, 4.5, 1.0, -0.1, 10)  # eps > 0
    with pytest.raises(ValueError):
        oracle_mod.Oracle(8, 8, 12, 4.5, 1.0, 0.1, 2**31)  # pair counter range
    with pytest.raises(ValueError):
        oracle_mod.Oracle(8, 8, 12, 4.5, 1.0, 0.1, 10, order=3)
