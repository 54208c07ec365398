"""Droplet shape and freezing time (test infrastructure only: the checker of
the batched sweep).

The paper reports the freezing time as a Fourier number (Eq. (42)), the
final height and aspect ratio H/R of frozen droplets (Sec. 4.2.1) and the
tip or plateau they form (Sec. 4.2.2), without saying how these are read
off a phi field.  The definitions used here (and by the GPU library):

* height: over every column, the highest place where phi crosses 1/2
  (linear interpolation between the two nodes), plus 1/2 for the wall at
  y = -1/2;
* base radius: half the distance between the outermost phi = 1/2 crossings
  of row 0;
* tip angle: angle between the least-squares lines x(y) fitted to the
  outermost left and right crossings of the rows whose height y + 1/2 lies
  in [0.75 H, 0.95 H] (undefined with fewer than two such rows);
* freezing time: the first time the liquid volume sum clamp(phi) f_l falls
  to `frac` of its initial value, linearly interpolated between samples.

Plain loops: these run on small fields only.
"""
from __future__ import annotations

import math
from typing import Dict, Optional, Sequence, Tuple

import numpy as np


def row_crossings(row: np.ndarray) -> Optional[Tuple[float, float]]:
    """Outermost phi = 1/2 crossings (x_left, x_right) of one row."""
    idx = [x for x in range(len(row)) if row[x] >= 0.5]
    if not idx:
        return None
    a, b = idx[0], idx[-1]
    n = len(row)
    xl = 0.0 if a == 0 else (a - 1) + (0.5 - row[a - 1]) / (row[a] - row[a - 1])
    xr = float(n - 1) if b == n - 1 else b + (row[b] - 0.5) / (row[b] - row[b + 1])
    return float(xl), float(xr)


def top_crossing(col: np.ndarray) -> Optional[float]:
    """Highest phi = 1/2 crossing of one column (y index, interpolated)."""
    ny = len(col)
    for y in range(ny - 1, -1, -1):
        if col[y] >= 0.5:
            if y == ny - 1:
                return float(y)
            return y + (col[y] - 0.5) / (col[y] - col[y + 1])
    return None


def shape_metrics(phi: np.ndarray) -> Dict[str, float]:
    """Height, base radius and tip angle of the phi = 1/2 contour of a
    (ny, nx) field whose row 0 sits half a spacing above the wall."""
    phi = np.asarray(phi, dtype=np.float64)
    ny, nx = phi.shape
    tops = [t for t in (top_crossing(phi[:, x]) for x in range(nx)) if t is not None]
    if not tops:
        return dict(height=math.nan, base_radius=math.nan, tip_angle_deg=math.nan, npts=0)
    H = max(tops) + 0.5
    base = row_crossings(phi[0])
    left, right = [], []
    for y in range(ny):
        h = y + 0.5
        if h < 0.75 * H or h > 0.95 * H:
            continue
        c = row_crossings(phi[y])
        if c is None:
            continue
        left.append((y, c[0]))
        right.append((y, c[1]))
    angle = math.nan
    if len(left) >= 2:
        bl = np.polyfit([p[0] for p in left], [p[1] for p in left], 1)[0]
        br = np.polyfit([p[0] for p in right], [p[1] for p in right], 1)[0]
        angle = math.degrees(math.atan(bl) - math.atan(br))
    return dict(height=H, base_radius=math.nan if base is None else 0.5 * (base[1] - base[0]),
                tip_angle_deg=angle, npts=len(left))


def freeze_time(steps: Sequence[float], liquid: Sequence[float], frac: float = 0.01) -> float:
    """First time the sampled liquid volume reaches frac * liquid[0]
    (linear interpolation between samples); NaN if it never does."""
    thr = frac * liquid[0]
    for j in range(1, len(steps)):
        if liquid[j] <= thr:
            d = liquid[j - 1] - liquid[j]
            w = (liquid[j - 1] - thr) / d if d > 0 else 1.0
            w = min(max(w, 0.0), 1.0)
            return steps[j - 1] + w * (steps[j] - steps[j - 1])
    return math.nan


def fourier_number(t: float, k_l: float, rho_l: float, cp_l: float, R: float) -> float:
    """Eq. (42): Fo = k_l t / (rho_l cp_l R^2)."""
    return k_l * t / (rho_l * cp_l * R * R)
