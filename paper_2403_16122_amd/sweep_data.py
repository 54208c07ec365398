"""Training data of the surrogate: droplets of the parametric sweep run to
freezing with the batched solver (FP16 storage), one record per droplet.

    python -m paper_2403_16122_amd.sweep_data --n 4096 --seed 1 --out train.npz

Inputs per droplet: R, theta (deg), Ste, gamma = rho_s/rho_l, bubble count.
Outputs: status, t_freeze (steps), t* (Fourier number, Eq. (42)), height/R,
base radius/R and tip angle (deg; NaN where undefined).
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

INPUTS = ("R", "theta", "ste", "gamma", "nbubbles")
OUTPUTS = ("t_star", "height_R", "tip_angle")


def run(n: int, seed: int, slots: int = 256, chunk: int = 512, every: int = 200, max_steps: int = 3_000_000):
    import torch

    from paper_2403_16122_amd import lbm, workloads as W

    recs = []
    for start in range(0, n, chunk):
        m = min(chunk, n - start)
        drops = W.sweep_droplets(start + m, seed=seed, storage=lbm.STORAGE["fp16"])[start:]
        b = lbm.Batch([d["params"] for d in drops], [d["phi0"] for d in drops], [d["T0"] for d in drops],
                      radii=[d["R"] for d in drops], slots=min(slots, m))
        b.configure(sample_every=every, max_steps=max_steps)
        b.autotune(reps=3)
        t0 = time.perf_counter()
        while True:
            b.step(100000, until_frozen=True)
            res = b.results()
            done = sum(r["status"] not in ("running", "queued") for r in res)
            print(f"droplets {start}..{start + m}: {done}/{m} finished after {time.perf_counter() - t0:.1f} s",
                  flush=True)
            if done == m:
                break
        for d, r in zip(drops, res):
            recs.append((d["R"], d["theta"], d["ste"], d["gamma"], len(d["bubbles"]), r["status"] == "frozen",
                         r["t_freeze"], r["t_star"], r["height"] / d["R"], r["base_radius"] / d["R"],
                         r["tip_angle_deg"]))
        del b
        torch.cuda.empty_cache()
    a = np.array(recs, dtype=np.float64)
    return dict(R=a[:, 0], theta=a[:, 1], ste=a[:, 2], gamma=a[:, 3], nbubbles=a[:, 4], frozen=a[:, 5] > 0,
                t_freeze=a[:, 6], t_star=a[:, 7], height_R=a[:, 8], base_R=a[:, 9], tip_angle=a[:, 10],
                seed=np.int64(seed))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--out", required=True)
    args = ap.parse_args()
    data = run(args.n, args.seed)
    np.savez(args.out, **data)
    print(f"wrote {args.out}: {args.n} droplets, {int(data['frozen'].sum())} frozen", flush=True)


if __name__ == "__main__":
    main()
