"""Pins of the oracle terms that the uniform-property pins do not reach
(no GPU): the Boussinesq body force and the surface-tension solid mask of
the bubble setting (Sec. 4.3), the fluid-solid force of Sec. 3.3, and the
mixing of heat capacity and conductivity between unequal phases (Eq. (1))
with the enthalpy rule (Eq. (8)-(9)).

Each is a closed form the paper's equations fix, chosen so that a plausible
mistake in the term fails it by far more than the discretisation error:
- a channel flow whose driving force is the Boussinesq term plus gravity
  (a flipped sign, a dropped term or a missing rho_0 changes the amplitude
  by 3x or more);
- the first step from rest of a frozen layer with an order-parameter
  interface, where the post-collision momentum of every node is a closed
  form of the force, the solid fraction and the mask (exact to rounding);
- the two-phase Neumann front with C_p,s/C_p,l = 0.5 and k_s/k_l = 3.8
  (the property ratios of Sec. 4.2.1) and a superheated liquid, against
  the similarity solution of the enthalpy formulation (swapped
  conductivities or heat capacities, or breakpoints of Eq. (9) that ignore
  the mixture heat capacity, move the front by 10-50 %);
- the one-step pressure response to a prescribed lagged mass source under
  uniform flow, which fixes the c_s^2 grad S term of F~ (Eq. (33), (36);
  exact to rounding: a dropped term, a flipped sign or a missing c_s^2
  misses it by 100 % or more).
"""
import math

import numpy as np
import pytest
from scipy.optimize import brentq

from paper_2403_16122_amd import workloads as W

CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=float)
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=float)

# (tau_f - 1/2)^2 = 3/16: the half-way bounce-back wall of BGK carries no slip
EXACT_WALL_TAU = 0.5 + math.sqrt(3.0) / 4.0
EXACT_WALL_NU = (EXACT_WALL_TAU - 0.5) / 3.0


def test_boussinesq_force_drives_the_channel_at_its_closed_form_amplitude(oracle_mod):
    """One liquid phase at a uniform temperature T above T_m (the wall held
    at the same T, so nothing freezes or conducts), g along the walls: the
    body force of Sec. 4.3 is (rho - rho_0 beta (T - T_ref)) g, and the
    steady flow is the parabola u = G (y + 1/2)(ny - 1/2 - y) / (2 mu).
    Here rho_0 beta (T - T_ref) = 0.75, so the amplitude is a quarter of the
    plain gravity-driven one; with the sign flipped it would be 1.75x, with
    the term dropped 1x, without rho_0 0.4x (measured error 2.7e-6 of the
    peak)."""
    nx, ny, g = 4, 32, 1e-5
    T0, Tref, beta, rho0 = 2.0, 0.5, 0.4, 1.25
    p = W.default_params(nx, ny, T_bottom=T0, rho_s=1.0, mu_l=EXACT_WALL_NU, gx=g,
                         bq_beta=beta, bq_rho0=rho0, bq_Tref=Tref)
    s = oracle_mod.OracleSolver(p, np.ones(nx * ny), np.full(nx * ny, T0), threads=1)
    s.step(10000)
    f = s.fields(["ux", "uy", "T", "rho"])
    assert np.abs(f["T"] - T0).max() < 1e-5 and np.abs(f["rho"] - 1.0).max() < 1e-6
    y = np.arange(ny)
    G = (1.0 - rho0 * beta * (T0 - Tref)) * g
    exact = G / (2.0 * EXACT_WALL_NU) * (y + 0.5) * (ny - 0.5 - y)
    assert np.ptp(f["ux"], axis=1).max() < 1e-14
    assert np.abs(f["ux"][:, 0] - exact).max() < 1e-4 * exact.max(), np.abs(f["ux"][:, 0] - exact).max()
    assert np.abs(f["uy"]).max() < 1e-5 * exact.max()  # measured 3.6e-6 (a weak residual circulation)


@pytest.mark.parametrize("chi", [0, 1])
def test_first_step_momentum_of_a_frozen_layer_with_an_interface(oracle_mod, chi):
    """A frozen liquid layer under gas (T = -20 everywhere: f_s^H = 1, so
    the solid fraction f_s = clamp(phi) runs from 1 to 0 across the
    interface), started at rest (f = f^eq(p = 0, u = 0) = 0).  After one
    step the streamed populations carry no momentum, so rho u* = F/2, the
    fluid-solid force is rho f = -f_s F/2 and the post-collision momentum
    rho u* + F/2 + rho f (Eq. (30)-(35), u_s = 0) is (1 - f_s/2) F at every
    node, with F = (1 - chi f_s) mu_phi grad(phi) + rho g: the surface
    tension kept only outside the solid when chi = 1 (Sec. 4.3) and
    everywhere when chi = 0 (Eq. (11)).  mu_phi of Eq. (12) is built here
    from the oracle's stencil (pinned on polynomials) with the theta = 90
    ghost rows (the adjacent row's value).  Exact to rounding; dropping the
    mask, or the fluid-solid force, moves it by O(f_s)."""
    nx, ny, g = 4, 24, -2e-5
    p = W.default_params(nx, ny, rho_s=0.9, st_solid_mask=chi, sigma=0.01, gy=g)
    phi0 = W.flat_layer(nx, ny, 12.0, p["W"])
    s = oracle_mod.OracleSolver(p, phi0, np.full(nx * ny, -20.0), threads=1)
    f0 = s.fields(["phi", "fs", "rho"])
    assert f0["fs"].max() > 0.9999 and f0["fs"].min() < 1e-4
    assert np.array_equal(f0["fs"], np.clip(f0["phi"], 0.0, 1.0))  # f_s^H = 1
    s.step(1)
    fp = s.pops("f")
    mx, my = np.tensordot(CX, fp, axes=1), np.tensordot(CY, fp, axes=1)
    phi, fs, rho = f0["phi"], f0["fs"], f0["rho"]
    ext = np.vstack([phi[:1], phi, phi[-1:]])
    _, gy, lap = oracle_mod.stencil(ext)
    beta, kappa = 12.0 * p["sigma"] / p["W"], 1.5 * p["sigma"] * p["W"]
    mu = 4.0 * beta * phi * (phi - 1.0) * (phi - 0.5) - kappa * lap
    Fy = (1.0 - chi * fs) * mu * gy + rho * g
    scale = np.abs(mu * gy).max()
    assert scale > 1e-5
    assert np.abs(my - (1.0 - 0.5 * fs) * Fy).max() < 1e-12 * scale
    assert np.abs(mx).max() == 0.0
    # the surface-tension part alone: chi = 1 removes the fraction f_s of it
    st = my - (1.0 - 0.5 * fs) * rho * g
    expect = (1.0 - 0.5 * fs) * (1.0 - chi * fs) * mu * gy
    assert np.abs(st - expect).max() < 1e-12 * scale


def two_phase_neumann(Cs, Cl, ks, kl, L, Tw, Tm, T0):
    """Similarity solution of solidification from a wall at T_w into liquid
    at T_0 > T_m for the enthalpy formulation H = C_p T + L f_l with phase
    heat capacities (Eq. (8), (1)): in each phase C dT/dt = k d2T/dz2, and
    the front at s = 2 lam sqrt(alpha_s t) releases the jump of H at T_m,
    L_eff = L + (C_l - C_s) T_m.  Returns (lam, alpha_s)."""
    a_s, a_l = ks / Cs, kl / Cl
    Leff = L + (Cl - Cs) * Tm
    nu = math.sqrt(a_s / a_l)

    def balance(lam):  # L_eff ds/dt = k_s dT_s/dz - k_l dT_l/dz at the front
        return (lam * math.sqrt(math.pi) * Leff - Cs * (Tm - Tw) * math.exp(-lam * lam) / math.erf(lam)
                + kl * (T0 - Tm) * math.exp(-lam * lam * nu * nu) / (math.erfc(lam * nu) * math.sqrt(a_l * a_s)))

    return brentq(balance, 1e-6, 5.0), a_s


def test_two_phase_front_with_unequal_heat_capacity_and_conductivity(oracle_mod):
    """Column of liquid at T_0 = 1.3 (T_m = 1) on a wall at 0, with
    C_p,s = 0.5, C_p,l = 1, k_s = 3.8 k_l (the ratios of Sec. 4.2.1),
    rho_s = rho_l (no flow).  The solid thickness sum_y f_s follows
    2 lam sqrt(alpha_s t) up to a constant offset of the half-spacing wall
    and the one-cell mushy zone (measured -0.57 lu at every time: -3.5 %,
    -1.8 %, -1.3 % at t = 1000, 4000, 8000).  Swapping k_s and k_l in
    Eq. (1) puts the front at -53 %, swapping the heat capacities at +23 %,
    and enthalpy breakpoints without the mixture heat capacity (a jump of L
    instead of L_eff) at +10 %."""
    nx, ny = 4, 160
    Cs, Cl, kl = 0.5, 1.0, 0.1
    ks, L, Tw, Tm, T0 = 3.8 * kl, 2.0, 0.0, 1.0, 1.3
    lam, a_s = two_phase_neumann(Cs, Cl, ks, kl, L, Tw, Tm, T0)
    p = W.default_params(nx, ny, rho_s=1.0, latent=L, cp_s=Cs, cp_l=Cl, cp_g=Cl, cp_ref=Cl,
                         k_s=ks, k_l=kl, k_g=kl, T_bottom=Tw)
    s = oracle_mod.OracleSolver(p, np.ones(nx * ny), np.full(nx * ny, T0), threads=1)
    offs = []
    for t in (1000, 4000, 8000):
        s.step(t - s.step_count)
        front = s.fields(["fs"])["fs"][:, 1].sum()
        exact = 2.0 * lam * math.sqrt(a_s * t)
        offs.append(front - exact)
        assert abs(front - exact) < 0.04 * exact, (t, front, exact)
    # the offset is a fixed fraction of a lattice spacing, not a rate error
    assert max(offs) - min(offs) < 0.05 and all(-1.0 < o < 0.0 for o in offs), offs


def test_lagged_mass_source_gradient_enters_the_pressure_through_the_forcing(oracle_mod):
    """The c_s^2 grad S term of F~ (Eq. (33), with S the lagged mass source
    of Eq. (38)) reaches the pressure of Eq. (36) through the forcing's rest
    component F_0 = w_0 (S - u.F~ / c_s^2).  One liquid phase above T_m
    (nothing freezes, rho uniform: the current S = rho mdot + u.grad rho is
    0), moving uniformly with u0 along x, started from f = f^eq(0, rho, u0)
    with a prescribed lagged S(x) = A sin(2 pi x / nx): after one step the
    pressure differs from the same step with S = 0 by
        dp = c_s^2 / (1 - w_0) tau_f (-w_0 u0 dS/dx) = -(4/15) tau_f u0 dS/dx,
    dS/dx being the isotropic stencil of S, (S(x+1) - S(x-1)) / 2 for a
    field constant in y.  Exact to rounding; without the term dp = 0, with
    its sign flipped -1x, with grad S not scaled by c_s^2 3x.  The lagged
    state is written through the oracle's checkpoint (four int64 header
    words, then g, f, h as nine planes each, then (phi u)_x, (phi u)_y,
    f_s^H, p and S of the previous step)."""
    nx, ny, u0, A = 16, 8, 0.02, 1e-3
    p = W.default_params(nx, ny, T_bottom=2.0, rho_s=1.0)
    n = nx * ny
    base = oracle_mod.OracleSolver(p, np.ones(n), np.full(n, 2.0), threads=1)
    rho = base.fields(["rho"])["rho"]
    assert np.ptp(rho) == 0.0
    feq = np.asarray(oracle_mod.node_feq(0.0, float(rho.flat[0]), u0, 0.0))
    blob0 = bytearray(base.save())
    off = 32 + 9 * n * 8  # the f planes follow the nine g planes

    def run(S_prev):
        o = oracle_mod.OracleSolver(p, np.ones(n), np.full(n, 2.0), threads=1)
        blob = bytearray(blob0)
        blob[off:off + 9 * n * 8] = np.repeat(feq, n).tobytes()
        hist = 32 + 27 * n * 8  # (phi u)_x, (phi u)_y, f_s^H, p, S
        blob[hist:hist + 8 * n] = np.full(n, u0).tobytes()
        blob[hist + 8 * n:hist + 16 * n] = np.zeros(n).tobytes()
        blob[hist + 32 * n:hist + 40 * n] = np.ascontiguousarray(S_prev, dtype=np.float64).reshape(-1).tobytes()
        o.load(bytes(blob))
        o.step(1)
        after = o.save()
        pr = np.frombuffer(after, dtype=np.float64, count=n, offset=hist + 24 * n)
        ux = np.frombuffer(after, dtype=np.float64, count=n, offset=hist)  # phi u with phi = 1
        return pr.reshape(ny, nx), ux.reshape(ny, nx)

    x = np.arange(nx)
    S = np.tile(A * np.sin(2.0 * np.pi * x / nx), (ny, 1))
    (p1, ux), (p0, ux0) = run(S), run(np.zeros_like(S))
    assert np.array_equal(ux, ux0)  # the lagged S moves the pressure only
    dp = p1 - p0
    dSdx = 0.5 * (np.roll(S, -1, axis=1) - np.roll(S, 1, axis=1))
    tau_f = 3.0 * p["mu_l"] / p["rho_l"] + 0.5
    # u is the step's velocity: u0 away from the walls, less in the wall rows,
    # where half-way bounce-back has already acted
    assert np.abs(ux[2:-2] - u0).max() < 1e-15
    expect = -(4.0 / 15.0) * tau_f * ux * dSdx
    scale = np.abs(expect).max()
    assert scale > 1e-6
    assert np.abs(dp - expect).max() < 1e-12 * scale, np.abs(dp - expect).max() / scale
