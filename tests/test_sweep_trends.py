"""The paper's qualitative results of the parametric study (Sec. 4.2.2) in
the sweep data the batched GPU solver wrote (paper_2403_16122_amd/data,
16384 droplets from four generator seeds, FP16 storage; each droplet's
initial cap is regenerated here from its seed).  These are physics checks
of the solver's output, not parity: the freezing time grows with the
droplet volume and the contact angle, the volume change on freezing is
vertical (the contact line stays, the height changes by about
rho_l/rho_s), and gamma < 1 ends in a conical tip while gamma > 1 ends
flatter."""
import os

import numpy as np
import pytest

from paper_2403_16122_amd import workloads as W

DATA = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2403_16122_amd", "data")


@pytest.fixture(scope="module")
def sweep():
    from paper_2403_16122_amd.surrogate import load_training

    d = load_training(DATA)
    keep = d["frozen"] & np.isfinite(d["t_star"])
    d = {k: v[keep] for k, v in d.items()}
    rc = np.array([W.cap_radius(r, t) for r, t in zip(d["R"], d["theta"])])
    th = np.radians(d["theta"])
    d["base0"] = rc * np.sin(th)          # contact line of the initial cap
    d["height0"] = rc * (1.0 - np.cos(th))
    return d


def test_freezing_time_grows_with_volume_and_contact_angle(sweep):
    X = np.stack([np.ones_like(sweep["R"]), np.log(sweep["R"]), sweep["theta"], sweep["ste"], sweep["gamma"],
                  sweep["nbubbles"]], axis=1)
    c = np.linalg.lstsq(X, np.log(sweep["t_freeze"]), rcond=None)[0]
    print(f"log t_freeze: d/dlog R {c[1]:.3f}, d/dtheta {c[2]:.5f} per degree")
    assert 1.5 < c[1] < 2.5   # diffusive: t_freeze ~ R^2 at fixed Ste
    assert c[2] > 0.0          # larger contact angle, longer freezing (Sec. 4.2.2)


def test_volume_change_is_vertical(sweep):
    base = sweep["base_R"] * sweep["R"] / sweep["base0"]
    height = sweep["height_R"] * sweep["R"] / sweep["height0"]
    g = sweep["gamma"]
    print(f"base final/initial median {np.median(base):.3f}")
    assert abs(np.median(base) - 1.0) < 0.02
    assert np.all(np.quantile(base, [0.1, 0.9]) > [0.95, 0.95]) and np.quantile(base, 0.9) < 1.05
    for lo, hi in ((0.85, 0.95), (1.05, 1.1)):
        m = (g >= lo) & (g < hi)
        h, expect = np.median(height[m]), 1.0 / np.median(g[m])
        print(f"gamma in [{lo}, {hi}): height final/initial {h:.3f}, rho_l/rho_s {expect:.3f}")
        assert abs(h - expect) < 0.03 * expect


def test_expansion_makes_a_tip_and_shrinkage_a_flatter_top(sweep):
    g, tip = sweep["gamma"], sweep["tip_angle"]
    sharp, flat = np.nanmedian(tip[g < 0.95]), np.nanmedian(tip[g > 1.05])
    print(f"median tip angle: gamma < 0.95 {sharp:.1f} deg, gamma > 1.05 {flat:.1f} deg")
    assert sharp + 5.0 < flat
