"""Pins of the oracle's per-node building blocks against the moment identities
that the paper's equilibria and source terms are built to satisfy (Sec. 3,
Eq. (24)-(36)), the enthalpy definition Eq. (8), the stencils of Eq. (38) on
polynomials, and the geometry of the wetting condition Eq. (39)-(41).

None of these re-types an oracle formula: each checks a *property* (a
moment, an exactness, a geometric angle) that a dropped term, a wrong sign,
a wrong index or a transposed operand would break.
"""
import math

import numpy as np
import pytest

CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=float)
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=float)
CS2 = 1.0 / 3.0
RNG = np.random.default_rng(1234)
TOL = 1e-14


def moments(q):
    m0 = q.sum()
    m1 = np.array([(CX * q).sum(), (CY * q).sum()])
    m2 = np.array([[(CX * CX * q).sum(), (CX * CY * q).sum()], [(CY * CX * q).sum(), (CY * CY * q).sum()]])
    return m0, m1, m2


def rnd(scale=1.0):
    return float(RNG.uniform(-scale, scale))


@pytest.mark.parametrize("trial", range(20))
def test_geq_moments(oracle_mod, trial):
    phi, ux, uy = RNG.uniform(-0.1, 1.1), rnd(0.05), rnd(0.05)
    m0, m1, _ = moments(oracle_mod.node_geq(phi, ux, uy))
    assert abs(m0 - phi) < TOL
    assert np.allclose(m1, [phi * ux, phi * uy], atol=TOL, rtol=0)


@pytest.mark.parametrize("trial", range(20))
def test_gsrc_moments(oracle_mod, trial):
    phi, a, b, lx, ly, md = RNG.uniform(0, 1), rnd(1e-3), rnd(1e-3), rnd(0.2), rnd(0.2), rnd(1e-2)
    m0, m1, _ = moments(oracle_mod.node_gsrc(phi, a, b, lx, ly, md))
    # zeroth moment phi*div(u), first moment d_t(phi u) + cs^2 lambda n
    assert abs(m0 - phi * md) < TOL
    assert np.allclose(m1, [a + CS2 * lx, b + CS2 * ly], atol=TOL, rtol=0)


@pytest.mark.parametrize("trial", range(20))
def test_feq_moments(oracle_mod, trial):
    p, rho, ux, uy = rnd(1e-2), RNG.uniform(1e-3, 1.2), rnd(0.05), rnd(0.05)
    m0, m1, m2 = moments(oracle_mod.node_feq(p, rho, ux, uy))
    u = np.array([ux, uy])
    assert abs(m0) < TOL
    assert np.allclose(m1, rho * u, atol=TOL, rtol=0)
    assert np.allclose(m2, p * np.eye(2) + rho * np.outer(u, u), atol=TOL, rtol=0)


@pytest.mark.parametrize("trial", range(20))
def test_fforce_moments(oracle_mod, trial):
    S = rnd(1e-3)
    F = np.array([rnd(1e-3), rnd(1e-3)])
    rf = np.array([rnd(1e-3), rnd(1e-3)])
    u = np.array([rnd(0.05), rnd(0.05)])
    Ft = np.array([rnd(1e-3), rnd(1e-3)])
    q = oracle_mod.node_fforce(S, F[0], F[1], rf[0], rf[1], u[0], u[1], Ft[0], Ft[1])
    m0, m1, m2 = moments(q)
    assert abs(m0 - S) < TOL
    assert np.allclose(m1, F + rf, atol=TOL, rtol=0)
    assert np.allclose(m2, CS2 * S * np.eye(2) + np.outer(u, Ft) + np.outer(Ft, u), atol=TOL, rtol=0)


@pytest.mark.parametrize("trial", range(20))
def test_heq_moments(oracle_mod, trial):
    H, T, cp, cpr = RNG.uniform(-5, 15), RNG.uniform(-1, 2), RNG.uniform(0.3, 2), RNG.uniform(0.3, 2)
    u = np.array([rnd(0.05), rnd(0.05)])
    m0, m1, m2 = moments(oracle_mod.node_heq(H, T, cp, cpr, u[0], u[1]))
    assert abs(m0 - H) < 1e-13
    assert np.allclose(m1, cp * T * u, atol=1e-14, rtol=0)
    assert np.allclose(m2, cpr * T * CS2 * np.eye(2) + cp * T * np.outer(u, u), atol=1e-14, rtol=0)


@pytest.mark.parametrize("trial", range(20))
def test_pressure_inverts_equilibrium(oracle_mod, trial):
    p, rho, ux, uy = rnd(1e-2), RNG.uniform(1e-3, 1.2), rnd(0.05), rnd(0.05)
    f = oracle_mod.node_feq(p, rho, ux, uy)
    tau = RNG.uniform(0.6, 3.5)
    assert abs(oracle_mod.node_pressure(f, 0.0, 0.0, tau, rho, ux, uy) - p) < 1e-15
    # the source and F_0 terms enter linearly with weights dt/2 and tau
    S, F0 = rnd(1e-3), rnd(1e-3)
    got = oracle_mod.node_pressure(f, S, F0, tau, rho, ux, uy)
    assert abs(got - p - 0.6 * (0.5 * S + tau * F0)) < 1e-15


def test_enthalpy_rule_reproduces_definition(oracle_mod):
    """Eq. (8): H = cp T + L f_l must hold for every H; f_l in [0,1];
    T and f_l continuous and non-decreasing in H."""
    cp, Tm, L = 1.3, 0.7, 4.0
    Hs, Hl = cp * Tm, cp * Tm + L
    Hs_grid = np.concatenate([np.linspace(-5, 15, 2001), [Hs, Hl, Hs - 1e-12, Hl + 1e-12]])
    prev = None
    for H in np.sort(Hs_grid):
        fl, T = oracle_mod.node_enthalpy(H, cp, Tm, L)
        assert 0.0 <= fl <= 1.0
        assert abs(cp * T + L * fl - H) < 1e-12
        if prev is not None:
            assert fl >= prev[0] - 1e-15 and T >= prev[1] - 1e-15
            assert abs(fl - prev[0]) < 0.01 and abs(T - prev[1]) < 0.02  # continuity on a fine grid
        prev = (fl, T)
    assert oracle_mod.node_enthalpy(Hs, cp, Tm, L) == (0.0, Tm)
    assert oracle_mod.node_enthalpy(Hl, cp, Tm, L) == (1.0, Tm)
    assert oracle_mod.node_enthalpy(0.5 * (Hs + Hl), cp, Tm, L) == (0.5, Tm)


def _poly_ext(nx, ny, fn):
    y = np.arange(-1, ny + 1, dtype=float)[:, None]
    x = np.arange(nx, dtype=float)[None, :]
    return fn(x + 0 * y, y + 0 * x)


@pytest.mark.parametrize("fn,gx,gy,lap", [
    (lambda x, y: 0.3 * x - 0.7 * y + 2.0, lambda x, y: 0.3 + 0 * x, lambda x, y: -0.7 + 0 * x, lambda x, y: 0 * x),
    (lambda x, y: x * x, lambda x, y: 2 * x, lambda x, y: 0 * x, lambda x, y: 2 + 0 * x),
    (lambda x, y: y * y, lambda x, y: 0 * x, lambda x, y: 2 * y, lambda x, y: 2 + 0 * x),
    (lambda x, y: x * y, lambda x, y: y, lambda x, y: x, lambda x, y: 0 * x),
])
def test_stencils_exact_on_quadratics(oracle_mod, fn, gx, gy, lap):
    nx, ny = 12, 7
    ext = _poly_ext(nx, ny, fn)
    Gx, Gy, Lp = oracle_mod.stencil(ext)
    y = np.arange(ny, dtype=float)[:, None] + 0 * np.arange(nx)[None, :]
    x = np.arange(nx, dtype=float)[None, :] + 0 * y
    sl = (slice(None), slice(1, nx - 1))  # away from the periodic seam
    assert np.allclose(Gx[sl], gx(x, y)[sl], atol=1e-12, rtol=0)
    assert np.allclose(Gy[sl], gy(x, y)[sl], atol=1e-12, rtol=0)
    assert np.allclose(Lp[sl], lap(x, y)[sl], atol=1e-12, rtol=0)


def test_stencil_periodic_and_weights(oracle_mod):
    """A single spike: the Laplacian stencil sums to zero (conservative) and
    carries the D2Q9 weights 2*w_i/cs^2 on the 8 neighbours."""
    nx, ny = 9, 5
    ext = np.zeros((ny + 2, nx))
    ext[3, 0] = 1.0  # node (x=0, y=2), its neighbours wrap around x
    _, _, Lp = oracle_mod.stencil(ext)
    assert abs(Lp.sum()) < 1e-13
    assert abs(Lp[2, 0] + 6 * (4 / 9 + 4 / 36)) < 1e-13
    assert abs(Lp[2, nx - 1] - 6 / 9) < 1e-13 and abs(Lp[3, nx - 1] - 6 / 36) < 1e-13


@pytest.mark.parametrize("theta", [30.0, 60.0, 90.0, 120.0, 150.0])
def test_wetting_ghost_geometry(oracle_mod, theta):
    """For a linear phi whose level lines meet the wall at angle theta the
    ghost value is the exact linear extrapolation (Eq. (39) satisfied)."""
    nx = 16
    a = 0.07
    t = math.tan(math.radians(90.0 - theta))
    b = -t * abs(a)  # d phi / dy such that n_w . grad(phi) = -tan(pi/2 - theta)|d phi/dx|
    x = np.arange(nx, dtype=float)
    row0 = 0.4 + a * x
    row1 = row0 + b
    g = oracle_mod.wetting_ghost(theta, row0, row1)
    inner = slice(2, nx - 2)
    assert np.allclose(g[inner], (row0 - b)[inner], atol=1e-14, rtol=0)
    # angle, measured through the liquid (phi increases with x), between the
    # wall and the upward direction of the level lines (-b, a)
    ang = math.degrees(math.atan2(a, -b))
    assert abs(ang - theta) < 1e-9


def test_wetting_sign(oracle_mod):
    """theta < 90 raises the ghost above the wall row where phi varies
    along the wall (liquid drawn onto the wall); theta = 90 copies it."""
    x = np.arange(10, dtype=float)
    r0 = 0.5 + 0.5 * np.tanh((x - 5) / 2)
    r1 = 0.5 + 0.5 * np.tanh((x - 4.5) / 2)
    assert np.array_equal(oracle_mod.wetting_ghost(90.0, r0, r1), r0)
    assert np.all(oracle_mod.wetting_ghost(60.0, r0, r1) >= r0)
    assert np.all(oracle_mod.wetting_ghost(120.0, r0, r1) <= r0)
