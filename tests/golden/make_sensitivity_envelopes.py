"""Writes sensitivity_envelopes.json: how far the FP64 oracle moves from
itself on the 512x256 sessile droplet over 1000 steps, under perturbations of
the size FP32 rounding makes (test infrastructure; calls the oracle only).

    python tests/golden/make_sensitivity_envelopes.py      # ~15 min on 8 cores

Draws: phi0 perturbed by 1e-7 * N(0, 1) (seeds 5120-5123), and phi moved by
1e-8 * N(0, 1) at every node after every step (seeds 7000-7003).  Per draw:
max |dT|, relative L2 of u and of phi, max |dphi|, and the relative change of
the solid and liquid volumes, sum phi and sum H; the file keeps every draw
and the maximum over them.
"""
import json
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, os.path.dirname(HERE))

import oracle  # noqa: E402
from paper_2403_16122_amd import workloads as W  # noqa: E402
from sensitivity import perturbed_every_step  # noqa: E402

FIELDS = ("phi", "T", "ux", "uy")
VOLS = ("sum_solid", "sum_liquid", "sum_phi", "sum_H")


def rel_l2(a, b):
    return math.sqrt(float(np.sum((a - b) ** 2))) / max(math.sqrt(float(np.sum(b * b))), 1e-300)


def deviation(o2, fo, do):
    f2, d2 = o2.fields(FIELDS), o2.diag()
    r = dict(T=float(np.abs(f2["T"] - fo["T"]).max()),
             u=rel_l2(np.stack([f2["ux"], f2["uy"]]), np.stack([fo["ux"], fo["uy"]])),
             lphi=rel_l2(f2["phi"], fo["phi"]), phi=float(np.abs(f2["phi"] - fo["phi"]).max()))
    for k in VOLS:
        r[k] = abs(d2[k] - do[k]) / max(1.0, abs(do[k]))
    return r


def main():
    oracle.build_oracle(force=False)
    p, phi0, T0, _ = W.workload("sessile512", seed=0)
    steps = 1000
    o = oracle.OracleSolver(p, phi0, T0)
    o.step(steps)
    fo, do = o.fields(FIELDS), o.diag()
    draws = []
    for seed in range(5120, 5124):
        z = np.random.default_rng(seed).standard_normal(phi0.size)
        o2 = oracle.OracleSolver(p, phi0 + 1e-7 * z, T0)
        o2.step(steps)
        draws.append(dict(kind="initial 1e-7", seed=seed, **deviation(o2, fo, do)))
        print(draws[-1], flush=True)
    for seed in range(7000, 7004):
        o2 = perturbed_every_step(oracle, p, phi0, T0, steps, 1e-8, seed)
        draws.append(dict(kind="every step 1e-8", seed=seed, **deviation(o2, fo, do)))
        print(draws[-1], flush=True)
    keys = [k for k in draws[0] if k not in ("kind", "seed")]
    out = {"sessile512_1000": {"steps": steps, "draws": draws,
                               "max": {k: max(d[k] for d in draws) for k in keys}}}
    with open(os.path.join(HERE, "sensitivity_envelopes.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
