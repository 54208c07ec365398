"""Pins of the shape and freezing-time checker (oracle/shape.py) against
closed forms: a spherical cap, a wedge with a known apex angle, and liquid
series with known crossings."""
import math

import numpy as np
import pytest

from oracle import shape as S


def tanh_field(d, W=4.0):
    return 0.5 * (1.0 + np.tanh(2.0 * d / W))


def cap(nx, ny, Rc, theta_deg, xc):
    """phi of a circular cap meeting the wall y = -1/2 at angle theta."""
    yc = -0.5 - Rc * math.cos(math.radians(theta_deg))
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    return tanh_field(Rc - np.hypot(x - xc, y - yc)), yc


@pytest.mark.parametrize("theta", [60.0, 90.0, 120.0])
def test_cap_height_and_base(theta):
    Rc, xc = 30.0, 64.0
    phi, yc = cap(128, 96, Rc, theta, xc)
    m = S.shape_metrics(phi)
    assert m["height"] == pytest.approx(Rc * (1.0 - math.cos(math.radians(theta))), abs=2e-3)
    # chord of the circle on row 0 (y = 0)
    assert m["base_radius"] == pytest.approx(math.sqrt(Rc * Rc - yc * yc), abs=2e-2)


@pytest.mark.parametrize("apex", [60.0, 90.0, 120.0])
def test_wedge_tip_angle(apex):
    """Signed distance to an isosceles triangle standing on the wall: the
    fitted flanks give its apex angle."""
    nx, ny, xa, ya = 160, 120, 80.0, 70.0
    half = math.radians(apex / 2.0)
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    # inside: below both flanks; distance to the flanks (or to the apex above it)
    n1 = np.array([math.cos(half), math.sin(half)])    # outward normal of the right flank
    n2 = np.array([-math.cos(half), math.sin(half)])   # of the left flank
    d1 = (x - xa) * n1[0] + (y - ya) * n1[1]
    d2 = (x - xa) * n2[0] + (y - ya) * n2[1]
    outside = np.maximum(d1, d2)
    # above the apex cone the nearest point is the apex itself
    above = (d1 > 0) & (d2 > 0)
    dist = np.where(above, np.hypot(x - xa, y - ya), outside)
    phi = tanh_field(-dist)
    m = S.shape_metrics(phi)
    assert m["height"] == pytest.approx(ya + 0.5, abs=1e-9)
    assert m["npts"] >= 2
    assert m["tip_angle_deg"] == pytest.approx(apex, abs=0.05)


def test_mirror_symmetry_and_empty_field():
    phi, _ = cap(101, 60, 20.0, 100.0, 47.3)
    a, b = S.shape_metrics(phi), S.shape_metrics(phi[:, ::-1])
    for k in ("height", "base_radius", "tip_angle_deg"):
        assert a[k] == pytest.approx(b[k], rel=1e-12)
    e = S.shape_metrics(np.zeros((10, 12)))
    assert math.isnan(e["height"]) and e["npts"] == 0


def test_freeze_time_interpolates_the_threshold_crossing():
    steps = np.arange(0, 1001, 100.0)
    liquid = 5.0 * (1.0 - steps / 800.0).clip(0.0)   # reaches 1 % of 5 at t = 792
    assert S.freeze_time(steps, liquid) == pytest.approx(792.0, abs=1e-9)
    assert S.freeze_time(steps, liquid, frac=0.5) == pytest.approx(400.0, abs=1e-9)
    assert math.isnan(S.freeze_time(steps, np.full(steps.shape, 5.0)))
    # a jump below the threshold within one interval lands inside it
    assert 100.0 <= S.freeze_time([0, 100, 200], [2.0, 2.0, 0.0]) <= 200.0


def test_fourier_number():
    assert S.fourier_number(1000.0, 0.1, 1.0, 1.0, 10.0) == pytest.approx(1.0)
