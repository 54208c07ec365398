"""Seeded synthetic inputs and workload parameter sets.

This module is shared by the HIP path's tests/bench and by the FP64 oracle's
tests.  It holds *no* arithmetic of the lattice Boltzmann method: only the
initial order-parameter profiles (the tanh droplet/layer/bubble shapes the
paper initialises its cases with, Eq. (43) and Eq. (45) of Sec. 4), the
initial temperature noise, and dictionaries of lattice-unit parameters.
Every physical-to-lattice choice that the paper leaves open is stated here
once so that both solvers receive identical inputs.

Lattice conventions: node (x, y) has index k = y*nx + x; x is periodic; the
bottom wall sits half a spacing below row 0 (y = -1/2) and the top wall half
a spacing above row ny-1.
"""
from __future__ import annotations

import math
from typing import Dict, List, Optional, Tuple

import numpy as np

# --------------------------------------------------------------------------
# Counter-based noise: splitmix64 (Steele, Lea & Flood, OOPSLA 2014).
# --------------------------------------------------------------------------
_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(x: np.ndarray) -> np.ndarray:
    """splitmix64 finaliser applied element-wise to uint64 counters."""
    z = np.asarray(x, dtype=np.uint64).copy()
    with np.errstate(over="ignore"):
        z = z + _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, n: int) -> np.ndarray:
    """U_k in [0,1): top 53 bits of splitmix64(seed XOR k*golden) / 2^53."""
    k = np.arange(n, dtype=np.uint64)
    with np.errstate(over="ignore"):
        ctr = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) ^ (k * _GOLDEN)
    bits = splitmix64(ctr) >> np.uint64(11)
    return bits.astype(np.float64) / float(1 << 53)


def temperature_noise(nx: int, ny: int, T_mean: float, amp: float, seed: Optional[int]) -> np.ndarray:
    """T0(k) = T_mean + amp*(2U_k - 1); seed None gives a noise-free field."""
    n = nx * ny
    if seed is None or amp == 0.0:
        return np.full(n, T_mean, dtype=np.float64)
    return T_mean + amp * (2.0 * uniform01(seed, n) - 1.0)


# --------------------------------------------------------------------------
# Initial order-parameter shapes (tanh profile across the interface, width W)
# --------------------------------------------------------------------------
def _tanh_profile(signed_dist_inside: np.ndarray, W: float) -> np.ndarray:
    return 0.5 + 0.5 * np.tanh(2.0 * signed_dist_inside / W)


def cap_radius(R: float, theta_deg: float) -> float:
    """Radius of a circular cap with contact angle theta whose area equals
    the semicircle pi R^2 / 2 (area of a cap = Rc^2 (t - sin t cos t))."""
    t = math.radians(theta_deg)
    area_unit = t - math.sin(t) * math.cos(t)
    return R * math.sqrt((0.5 * math.pi) / area_unit)


def sessile_droplet(nx: int, ny: int, R: float, theta_deg: float, W: float,
                    x0: Optional[float] = None) -> np.ndarray:
    """Circular-cap droplet sitting on the bottom wall (y = -1/2).

    The cap has contact angle theta and the area of a semicircle of radius R.
    Its centre is at (x0, -1/2 - Rc cos theta).  Distances are measured with
    the periodic x image nearest to the centre.
    """
    if x0 is None:
        x0 = nx / 2.0
    Rc = cap_radius(R, theta_deg)
    yc = -0.5 - Rc * math.cos(math.radians(theta_deg))
    x = np.arange(nx, dtype=np.float64)
    y = np.arange(ny, dtype=np.float64)
    dx = x[None, :] - x0
    dx = dx - nx * np.round(dx / nx)
    dy = y[:, None] - yc
    r = np.sqrt(dx * dx + dy * dy)
    return _tanh_profile(Rc - r, W).reshape(-1)


def free_droplet(nx: int, ny: int, R: float, W: float, xc: Optional[float] = None,
                 yc: Optional[float] = None) -> np.ndarray:
    """Free circular droplet (liquid inside) of radius R."""
    xc = nx / 2.0 if xc is None else xc
    yc = (ny - 1) / 2.0 if yc is None else yc
    x = np.arange(nx, dtype=np.float64)
    y = np.arange(ny, dtype=np.float64)
    dx = x[None, :] - xc
    dx = dx - nx * np.round(dx / nx)
    r = np.sqrt(dx * dx + (y[:, None] - yc) ** 2)
    return _tanh_profile(R - r, W).reshape(-1)


def flat_layer(nx: int, ny: int, H0: float, W: float) -> np.ndarray:
    """Liquid layer of thickness H0 above the bottom wall (Eq. (43) form);
    node y sits at height y + 1/2 above the wall."""
    y = np.arange(ny, dtype=np.float64) + 0.5
    col = _tanh_profile(H0 - y, W)
    return np.repeat(col[:, None], nx, axis=1).reshape(-1)


def place_bubbles(seed: int, n_bubbles: int, droplet_center: Tuple[float, float], Rc: float,
                  W: float, r_range=(3.0, 10.0), max_tries: int = 100000) -> List[Tuple[float, float, float]]:
    """Seeded rejection sampling of non-overlapping bubbles inside a droplet.

    Clearance of at least 2W from each other, from the droplet surface and
    from the wall plane y = -1/2.  Returns (x, y, r) tuples.
    """
    rng = np.random.default_rng(seed)
    xc, yc = droplet_center
    out: List[Tuple[float, float, float]] = []
    tries = 0
    while len(out) < n_bubbles and tries < max_tries:
        tries += 1
        r = rng.uniform(*r_range)
        bx = rng.uniform(xc - Rc, xc + Rc)
        by = rng.uniform(-0.5, yc + Rc)
        if math.hypot(bx - xc, by - yc) + r + 2 * W > Rc:
            continue
        if by - r - 2 * W < -0.5:
            continue
        if any(math.hypot(bx - ox, by - oy) < r + orr + 2 * W for ox, oy, orr in out):
            continue
        out.append((bx, by, r))
    return out


def droplet_with_bubbles(nx: int, ny: int, R: float, theta_deg: float, W: float,
                         bubbles: List[Tuple[float, float, float]]) -> np.ndarray:
    """Sessile droplet with gas bubbles carved out (product of tanh profiles)."""
    phi = sessile_droplet(nx, ny, R, theta_deg, W).reshape(ny, nx)
    x = np.arange(nx, dtype=np.float64)
    y = np.arange(ny, dtype=np.float64)
    for bx, by, br in bubbles:
        r = np.sqrt((x[None, :] - bx) ** 2 + (y[:, None] - by) ** 2)
        phi = phi * _tanh_profile(r - br, W)
    return phi.reshape(-1)


# --------------------------------------------------------------------------
# Lattice-unit parameter sets
# --------------------------------------------------------------------------
PARAM_KEYS = [
    "nx", "ny", "W", "M", "sigma",
    "rho_l", "rho_g", "rho_s", "mu_l", "mu_g", "mu_s",
    "cp_l", "cp_g", "cp_s", "cp_ref", "k_l", "k_g", "k_s",
    "latent", "T_melt", "T_bottom", "theta_bottom_deg", "theta_top_deg",
    "gx", "gy", "bq_beta", "bq_rho0", "bq_Tref",
    "st_solid_mask", "storage",
]


def default_params(nx: int, ny: int, **over) -> Dict[str, float]:
    """Defaults in lattice units (rho_l = 1, T_bottom = 0, T_melt = 1).

    W = 4, M = 0.1 (tau_g = 0.8); rho_g = 1e-3; rho_s = gamma; nu_l = 0.1;
    mu_g = 1e-3; sigma = 5e-3; uniform C_p = 1 and k = 0.1 (Pr = 1);
    latent heat L = C_p (T_m - T_w) / Ste with Ste = 0.1.
    """
    p = dict(
        nx=nx, ny=ny, W=4.0, M=0.1, sigma=0.005,
        rho_l=1.0, rho_g=1e-3, rho_s=0.9,
        mu_l=0.1, mu_g=1e-3, mu_s=0.1,
        cp_l=1.0, cp_g=1.0, cp_s=1.0, cp_ref=1.0,
        k_l=0.1, k_g=0.1, k_s=0.1,
        latent=10.0, T_melt=1.0, T_bottom=0.0,
        theta_bottom_deg=90.0, theta_top_deg=90.0,
        gx=0.0, gy=0.0, bq_beta=0.0, bq_rho0=1.0, bq_Tref=0.0,
        st_solid_mask=0, storage=0,
    )
    for k, v in over.items():
        if k not in p:
            raise KeyError(k)
        p[k] = v
    return p


def stefan_latent(stefan: float, cp: float = 1.0, T_melt: float = 1.0, T_bottom: float = 0.0) -> float:
    """L from the Stefan number definition Ste = c_p (T_m - T_w) / L (Sec. 3, Eq. (42))."""
    return cp * (T_melt - T_bottom) / stefan


def workload(name: str, seed: int = 0):
    """Return (params, phi0, T0, meta) for a named workload.

    sessile128  : 128x64, R=20 semicircle, theta 90, gamma 0.9, Ste 0.1, 2000 steps
    sessile512  : 512x256, R=80, theta 90, gamma 0.9, Ste 0.1, Bond 0.1 (planar)
    bubbles1024 : 1024x512, R=160, 1-8 bubbles r~U(3,10), theta~U(60,120)
    probe4096   : 4096x2048, the 512x256 physics scaled to R=640 (out-of-cache size)
    hou400      : 400x200 droplet with C_p,s/C_p,l = 0.5, k_s/k_l = 3.8, Pr 7.25, Ste 0.02
    """
    if name == "sessile128":
        nx, ny, R, th = 128, 64, 20.0, 90.0
        p = default_params(nx, ny, rho_s=0.9, latent=stefan_latent(0.1))
        phi0 = sessile_droplet(nx, ny, R, th, p["W"])
        T0 = temperature_noise(nx, ny, p["T_melt"], 1e-3, seed)
        return p, phi0, T0, dict(R=R, theta=th, steps=2000)
    if name in ("sessile512", "probe4096"):
        if name == "sessile512":
            nx, ny, R = 512, 256, 80.0
        else:
            nx, ny, R = 4096, 2048, 640.0
        th = 90.0
        sigma = 0.005
        bond = 0.1
        g = bond * sigma / (1.0 * R * R)  # Bo = rho_l g R^2 / sigma
        p = default_params(nx, ny, rho_s=0.9, latent=stefan_latent(0.1), gy=-g)
        phi0 = sessile_droplet(nx, ny, R, th, p["W"])
        T0 = temperature_noise(nx, ny, p["T_melt"], 1e-3, seed)
        return p, phi0, T0, dict(R=R, theta=th, bond=bond)
    if name == "bubbles1024":
        nx, ny, R = 1024, 512, 160.0
        rng = np.random.default_rng(seed)
        th = float(rng.uniform(60.0, 120.0))
        nb = int(rng.integers(1, 9))
        p = default_params(nx, ny, rho_s=0.9, latent=stefan_latent(0.1),
                           theta_bottom_deg=th, st_solid_mask=1)
        Rc = cap_radius(R, th)
        yc = -0.5 - Rc * math.cos(math.radians(th))
        bubbles = place_bubbles(seed + 1, nb, (nx / 2.0, yc), Rc, p["W"])
        phi0 = droplet_with_bubbles(nx, ny, R, th, p["W"], bubbles)
        T0 = temperature_noise(nx, ny, p["T_melt"], 1e-3, seed)
        return p, phi0, T0, dict(R=R, theta=th, bubbles=bubbles)
    if name == "hou400":
        # the sessile-droplet setup of Sec. 4.2.1 (Hou et al.'s water droplet):
        # 400x200, R = 40, W = 5, Pr = 7.25, Ste = 0.02, k_s/k_l = 3.8,
        # C_p,s/C_p,l = 0.5, gamma = 0.9, theta = 86.4 deg (synthetic: no images)
        nx, ny, R, th = 400, 200, 40.0, 86.4
        mu_l, cp_l = 0.1, 1.0
        k_l = mu_l * cp_l / 7.25
        p = default_params(nx, ny, W=5.0, rho_s=0.9, mu_l=mu_l, cp_l=cp_l, cp_g=cp_l, cp_s=0.5 * cp_l,
                           cp_ref=cp_l, k_l=k_l, k_g=k_l, k_s=3.8 * k_l, latent=stefan_latent(0.02),
                           theta_bottom_deg=th)
        phi0 = sessile_droplet(nx, ny, R, th, p["W"])
        T0 = temperature_noise(nx, ny, p["T_melt"], 1e-3, seed)
        return p, phi0, T0, dict(R=R, theta=th)
    raise KeyError(name)


def sweep_droplets(n: int, seed: int = 0, R_range=(16.0, 64.0), theta_range=(60.0, 150.0),
                   ste_range=(0.05, 0.3), gamma_range=(0.85, 1.1), max_bubbles: int = 8, storage: int = 0):
    """Droplets of a parametric sweep (the study of Sec. 4.2.2 widened):
    radius R, contact angle theta, Stefan number and density ratio
    gamma = rho_s/rho_l drawn uniformly, 0..max_bubbles gas bubbles placed
    inside, grid round(4R) x round(3R), liquid at T_m (+1e-3 noise) on a wall
    at T = 0.  Returns a list of dicts with params, phi0, T0 and the draws."""
    out = []
    for i in range(n):
        rng = np.random.default_rng([seed, i])
        R = float(rng.uniform(*R_range))
        th = float(rng.uniform(*theta_range))
        ste = float(rng.uniform(*ste_range))
        gamma = float(rng.uniform(*gamma_range))
        nb = int(rng.integers(0, max_bubbles + 1))
        nx, ny = int(round(4 * R)), int(round(3 * R))
        p = default_params(nx, ny, rho_s=gamma, latent=stefan_latent(ste), theta_bottom_deg=th, storage=storage)
        Rc = cap_radius(R, th)
        yc = -0.5 - Rc * math.cos(math.radians(th))
        bubbles = place_bubbles(int(rng.integers(1 << 31)), nb, (nx / 2.0, yc), Rc, p["W"], max_tries=2000)
        phi0 = droplet_with_bubbles(nx, ny, R, th, p["W"], bubbles)
        T0 = temperature_noise(nx, ny, p["T_melt"], 1e-3, int(rng.integers(1 << 31)))
        out.append(dict(params=p, phi0=phi0, T0=T0, R=R, theta=th, ste=ste, gamma=gamma, bubbles=bubbles))
    return out
