"""Whole runs against the FP64 oracle (GPU, FP32 storage, the autotuned
launch): the quantities the paper reports over a freezing run -- freezing
time, frozen shape, solid volume and the centre freezing height H_c of
Sec. 4.2.1 -- rather than pointwise fields, which the method's sensitivity
(a 1e-7 perturbation grows to O(1e-2) in phi within 1000 steps at 512x256)
does not let two implementations share over long runs.

- The 128x64 droplet (the parity workload) run until 1 % of its liquid is
  left: t_freeze (sampled every 200 steps, the batch's definition), the
  height, base radius and tip angle of the frozen drop (shape checker on each
  side's phi), and the conserved and condensed volumes.
- The 512x256 droplet over its first 20000 steps: solid and liquid volume,
  sum phi, sum H and H_c every 5000 steps.
- The 128x64 droplet with seeds 0, 1 and 2 over its 2000 steps: the same
  integrals and the temperature field.
"""
import math

import numpy as np
import pytest

from oracle import shape as SH
from paper_2403_16122_amd import workloads as W
from sensitivity import perturbed_every_step

pytestmark = pytest.mark.gpu


def _lbm():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_16122_amd import lbm

    return lbm


def run_to_frozen(s, every=200, max_steps=80000):
    steps, liq = [0], [s.diag()["sum_liquid"]]
    while steps[-1] < max_steps:
        s.step(every)
        steps.append(steps[-1] + every)
        liq.append(s.diag()["sum_liquid"])
        if liq[-1] <= 0.01 * liq[0]:
            break
    return SH.freeze_time(steps, liq), steps[-1]


def test_sessile128_run_to_frozen_against_oracle(oracle_mod):
    lbm = _lbm()
    p, phi0, T0, _ = W.workload("sessile128", seed=0)
    g = lbm.Solver(p, phi0, T0)
    tile, xcd = g.autotune(reps=5)
    o = oracle_mod.OracleSolver(p, phi0, T0)
    tg, ng = run_to_frozen(g)
    to, no = run_to_frozen(o)
    print(f"sessile128 ({tile}/{xcd}): t_freeze GPU {tg:.1f} oracle {to:.1f} (rel {abs(tg - to) / to:.2e})", flush=True)
    sg, so = SH.shape_metrics(g.fields(["phi"])["phi"]), SH.shape_metrics(o.fields(["phi"])["phi"])
    dg, do = g.diag(), o.diag()
    print(f"  shape GPU {sg} oracle {so}", flush=True)
    rel = {k: abs(dg[k] - do[k]) / abs(do[k]) for k in ("sum_phi", "sum_phic", "sum_H")}
    print(f"  integrals rel {rel}", flush=True)
    assert math.isfinite(tg) and math.isfinite(to)
    assert abs(tg - to) <= 2e-3 * to
    for k in ("height", "base_radius"):
        assert abs(sg[k] - so[k]) <= 0.25, k
    assert abs(sg["tip_angle_deg"] - so["tip_angle_deg"]) <= 3.0
    assert rel["sum_phi"] <= 1e-5 and rel["sum_phic"] <= 1e-4 and rel["sum_H"] <= 1e-6


def test_sessile512_first_20000_steps_integrals_against_oracle(oracle_mod):
    lbm = _lbm()
    p, phi0, T0, _ = W.workload("sessile512", seed=0)
    g = lbm.Solver(p, phi0, T0)
    tile, xcd = g.autotune(reps=5)
    o = oracle_mod.OracleSolver(p, phi0, T0)
    worst = {}
    for n in range(5000, 20001, 5000):
        g.step(5000)
        o.step(5000)
        dg, do = g.diag(), o.diag()
        assert dg["rc"] == 0
        rel = {k: abs(dg[k] - do[k]) / abs(do[k]) for k in ("sum_phi", "sum_H", "sum_solid", "sum_liquid")}
        rel["h_c"] = abs(dg["h_c"] - do["h_c"])
        print(f"sessile512 ({tile}/{xcd}) step {n}: {rel} solid {do['sum_solid']:.1f} h_c {do['h_c']:.2f}",
              flush=True)
        for k, v in rel.items():
            worst[k] = max(worst.get(k, 0.0), v)
    # measured on MI355X over the four samples: sum phi 1.4e-5, sum H 1.1e-8,
    # solid 2.9e-4, liquid 9.5e-5 (relative), H_c 0.36 lu (of 19.5 at step
    # 20000); the bounds: 0.005 % of the phase volume, 0.2 % of the solid and
    # liquid volumes, half a lattice spacing of H_c (a column sum of f_s)
    assert worst["sum_phi"] <= 5e-5 and worst["sum_H"] <= 1e-6
    assert worst["sum_solid"] <= 2e-3 and worst["sum_liquid"] <= 2e-3
    assert worst["h_c"] <= 0.5


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_sessile128_seeds_integrals_after_2000_steps(oracle_mod, seed):
    """Seeds 1 and 2 of the parity workload, whose pointwise phi the method
    amplifies beyond the stated bound within a few hundred steps, over the
    workload's full 2000 steps: the integral quantities stay with the
    oracle's (volumes, enthalpy, centre freezing height) within twice the
    method's own sensitivity, floored at fixed bounds.  The sensitivity is
    measured as in the pointwise test: the oracle against itself with phi0
    perturbed by 1e-7 (three draws) and with phi moved by 1e-8 after every
    step (three draws).  For seed 2 it is bimodal: one of those six draws
    (the first) resolves one dip event the other way and moves the solid
    volume by 3.2e-5 and sum phi by 6.1e-7 (the mass source follows the
    solid), the others by 1e-6 to 7e-6 and 3e-8 to 6e-8."""
    lbm = _lbm()
    p, phi0, T0, _ = W.workload("sessile128", seed=seed)
    g = lbm.Solver(p, phi0, T0)
    tile, xcd = g.autotune(reps=5)
    o = oracle_mod.OracleSolver(p, phi0, T0)
    g.step(2000)
    o.step(2000)
    dg, do = g.diag(), o.diag()
    keys = ("sum_phi", "sum_phic", "sum_H", "sum_solid", "sum_liquid")

    def dev(d):
        r = {k: abs(d[k] - do[k]) / abs(do[k]) for k in keys}
        r["h_c"] = abs(d["h_c"] - do["h_c"])
        return r

    rel = dev(dg)
    fg, fo = g.fields(["T"]), o.fields(["T"])
    dT = float(np.abs(fg["T"] - fo["T"]).max())
    others = []
    for draw in range(3):
        z = np.random.default_rng(900 + draw).standard_normal(phi0.size)
        o2 = oracle_mod.OracleSolver(p, phi0 + 1e-7 * z, T0)
        o2.step(2000)
        others.append(o2)
    for draw in range(3):
        others.append(perturbed_every_step(oracle_mod, p, phi0, T0, 2000, 1e-8, 300 + draw))
    env = dict(sum_phi=1e-7, sum_phic=1e-7, sum_H=1e-7, sum_solid=2e-5, sum_liquid=2e-5, h_c=0.01)
    for o2 in others:
        for k, v in dev(o2.diag()).items():
            env[k] = max(env[k], 2.0 * v)
    print(f"sessile128 seed {seed} ({tile}/{xcd}) after 2000 steps: {rel} max|dT| {dT:.2e}; bounds {env}", flush=True)
    for k in env:
        assert rel[k] <= env[k], (k, rel[k], env[k])
    assert dT <= 1e-5
