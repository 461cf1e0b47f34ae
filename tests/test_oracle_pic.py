"""Pins of the oracle's PIC-loop pieces (the Yee field solve and the grid
charge and current), against what the mathematics fixes:

- the Yee scheme propagates a plane wave exactly with its discrete dispersion
  relation sin(w dt/2)/dt = sin(k d/2)/d, along every axis and polarisation;
- without current the scheme keeps div E and div B unchanged;
- Esirkepov's current satisfies the discrete continuity equation
  rho^{n+1} - rho^n + dt div J = 0 exactly, with rho from the separately
  coded cloud-in-cell charge; its total is q w v;
- with that current the loop keeps div E - rho unchanged (Gauss's law)."""
import math

import numpy as np
import pytest

from oracle import pic


def _grid(dim):
    if dim == 2:
        return (24, 20, 1), (0.35, 0.3, 1.0)
    return (12, 10, 8), (0.35, 0.3, 0.4)


# (axis of propagation, E component, B component, sign of B/E)
WAVES = [(0, 1, 2, +1), (0, 2, 1, -1), (1, 2, 0, +1), (1, 0, 2, -1), (2, 0, 1, +1), (2, 1, 0, -1)]


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("wave", WAVES)
def test_plane_wave_follows_discrete_dispersion(dim, wave):
    ax, ec, bc, sgn = wave
    n, dx = _grid(dim)
    if dim == 2 and ax == 2:
        pytest.skip("no propagation along z in 2D")
    dt = 0.4 * min(dx[:dim])
    m = 3                                        # wavelengths across the box
    L = n[ax] * dx[ax]
    k = 2 * math.pi * m / L
    w = 2.0 / dt * math.asin(dt / dx[ax] * math.sin(k * dx[ax] / 2))
    shape = (n[2], n[1], n[0])
    # coordinates of each component's points along the propagation axis
    e_off = [0.5 if q == ec else 0.0 for q in range(3)]     # E_q is staggered along q
    b_off = [0.0 if q == bc else 0.5 for q in range(3)]     # B_q along the two others
    idx = np.indices(shape)[2 - ax].astype(np.float64)
    xe = (idx + e_off[ax]) * dx[ax]
    xb = (idx + b_off[ax]) * dx[ax]
    E = [np.zeros(shape) for _ in range(3)]
    B = [np.zeros(shape) for _ in range(3)]
    E[ec] = np.cos(k * xe)
    # B at t = dt/2 is the exact discrete wave; B^0 = B^{1/2} + (dt/2) curl E^0
    B[bc] = sgn * np.cos(k * xb - w * dt / 2)
    c = pic.curl_E(E, dx)
    for q in range(3):
        B[q] += 0.5 * dt * c[q]
    steps = 200
    for _ in range(steps):
        pic.fdtd_step(E, B, None, dt, dx)
    ref = np.cos(k * xe - w * steps * dt)
    assert np.max(np.abs(E[ec] - ref)) < 1e-10
    for q in range(3):
        if q != ec:
            assert np.max(np.abs(E[q])) < 1e-12
    # and B a half step later is the discrete wave too
    c = pic.curl_E(E, dx)
    bh = B[bc] - 0.5 * dt * c[bc]
    assert np.max(np.abs(bh - sgn * np.cos(k * xb - w * (steps + 0.5) * dt))) < 1e-10


@pytest.mark.parametrize("dim", [2, 3])
def test_divergences_kept_without_current(dim):
    n, dx = _grid(dim)
    rng = np.random.default_rng(1)
    shape = (n[2], n[1], n[0])
    E = [rng.normal(size=shape) for _ in range(3)]
    B = [rng.normal(size=shape) for _ in range(3)]
    d0, b0 = pic.div_E(E, dx), pic.div_B(B, dx)
    for _ in range(10):
        pic.fdtd_step(E, B, None, 0.1, dx)
    assert np.max(np.abs(pic.div_E(E, dx) - d0)) < 1e-11
    assert np.max(np.abs(pic.div_B(B, dx) - b0)) < 1e-11


def _moves(dim, n, dx, count, rng, frac=0.95):
    box = np.array([n[a] * dx[a] for a in range(dim)])
    p0 = rng.uniform(0, 1, (count, dim)) * box
    d = rng.uniform(-frac, frac, (count, dim)) * np.array(dx[:dim])
    p1 = np.mod(p0 + d, box)        # some moves cross the periodic boundary
    return p0, p1, d


@pytest.mark.parametrize("dim", [2, 3])
def test_current_satisfies_discrete_continuity(dim):
    n, dx = _grid(dim)
    rng = np.random.default_rng(2)
    p0, p1, d = _moves(dim, n, dx, 500, rng)
    w = rng.uniform(0.5, 2.0, 500)
    vz = rng.normal(size=500)
    q, dt = -1.0, 0.13
    r0 = pic.deposit_rho(p0, w, q, dim, n, dx)
    r1 = pic.deposit_rho(p1, w, q, dim, n, dx)
    J = pic.deposit_current(p0, p1, vz, w, q, dt, dim, n, dx)
    resid = r1 - r0 + dt * pic.div_E(J, dx)      # div of J on its E points
    assert np.max(np.abs(resid)) < 1e-12 * np.max(np.abs(r0))
    # total current = q w v on each axis
    dV = dx[0] * dx[1] * (dx[2] if dim == 3 else 1.0)
    for a in range(dim):
        assert J[a].sum() * dV == pytest.approx(q * np.sum(w * d[:, a]) / dt, rel=1e-12)
    if dim == 2:
        assert J[2].sum() * dV == pytest.approx(q * np.sum(w * vz), rel=1e-12)


def test_current_of_a_resting_particle():
    n, dx = _grid(3)
    J = pic.deposit_current([[1.0, 1.1, 0.9]], [[1.0, 1.1, 0.9]], None, [1.0], -1.0, 0.1, 3, n, dx)
    assert all(np.max(np.abs(j)) == 0.0 for j in J)
    n, dx = _grid(2)
    J = pic.deposit_current([[1.0, 1.1]], [[1.0, 1.1]], [0.7], [2.0], -1.0, 0.1, 2, n, dx)
    rho = pic.deposit_rho([[1.0, 1.1]], [2.0], -1.0, 2, n, dx)
    assert np.max(np.abs(J[0])) == 0.0 and np.max(np.abs(J[1])) == 0.0
    np.testing.assert_allclose(J[2], 0.7 * rho, rtol=1e-14, atol=1e-300)


@pytest.mark.parametrize("dim", [2, 3])
def test_loop_keeps_gauss_law(dim):
    n, dx = _grid(dim)
    rng = np.random.default_rng(3)
    shape = (n[2], n[1], n[0])
    count = 300
    box = np.array([n[a] * dx[a] for a in range(dim)])
    pos = rng.uniform(0, 1, (count, dim)) * box
    vel = rng.uniform(-0.9, 0.9, (count, dim)) * np.array(dx[:dim])
    w = np.ones(count)
    vz = rng.normal(size=count)
    E = [rng.normal(size=shape) for _ in range(3)]
    B = [rng.normal(size=shape) for _ in range(3)]
    dt = 0.1
    g0 = pic.div_E(E, dx) - pic.deposit_rho(pos, w, -1.0, dim, n, dx)
    for _ in range(6):
        new = np.mod(pos + vel, box)
        J = pic.deposit_current(pos, new, vz, w, -1.0, dt, dim, n, dx)
        pic.fdtd_step(E, B, J, dt, dx)
        pos = new
    g1 = pic.div_E(E, dx) - pic.deposit_rho(pos, w, -1.0, dim, n, dx)
    assert np.max(np.abs(g1 - g0)) < 1e-10


def test_photon_advance_moves_at_c():
    rng = np.random.default_rng(4)
    d = rng.normal(size=(50, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    p = rng.uniform(0, 1, (50, 3))
    out = pic.photon_advance(p, d, 0.25, (None, None, None))
    assert np.allclose(np.linalg.norm(out - p, axis=1), 0.25, rtol=1e-14)
    out = pic.photon_advance(p, d, 3.0, (2.0, 2.0, 2.0))
    assert ((out >= 0) & (out < 2.0)).all()
