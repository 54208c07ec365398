"""Throughput of the fused coupled-lattice step on one MI355X.

A step is one time step of all three D2Q9 lattices (phase field, flow,
enthalpy) over the whole grid; the default workload is the 512x256 sessile
droplet (R = 80, theta = 90, rho_s/rho_l = 0.9, Ste = 0.1, Bond = 0.1, FP32
populations).  Inputs are resident in HBM before the timed region.

Prints one JSON line with MLUPS, the roofline of the step kernel (HBM
bound, algorithmic 256 B per node update), the FP64 oracle timed on the host
cores, and the same step kernel on a 4096x2048 grid whose 2.3 GB working
set does not fit the 256 MB Infinity Cache.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# algorithmic bytes per node update: 27 populations and 5 FP32 history
# values, each read and written once
BYTES_PER_NODE = {"fp32": 27 * 8 + 40, "fp16": 27 * 4 + 40, "bf16": 27 * 4 + 40}
# Unfused two-kernel step: the macro pass reads g, h (18 populations) and
# f_s^H and writes phi, rho, f_s^H; the collide pass reads all populations,
# the history fields and those three planes, and writes what the fused step
# writes: the fused figure + 18 population reads + 4 B + 3 x 4 B written and
# read back.
UNFUSED_BYTES_PER_NODE = {st: BYTES_PER_NODE[st] + 18 * (4 if st == "fp32" else 2) + 4 + 24
                          for st in ("fp32", "fp16", "bf16")}
HBM_PEAK_GBS = 8000.0
METRIC = "MLUPS (φ+flow+T lattices), % HBM peak; batched sweep droplets/s vs plain"


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("lbm_kernels.hip", "lbm_internal.h"):
        with open(os.path.join(ROOT, "paper_2403_16122_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, storage: str, tile: str, xcd: int):
    """HBM bytes per launch from rocprofv3 FETCH_SIZE/WRITE_SIZE runs stored
    under profiles/, valid only for the kernel source and the launch shape
    (tile, workgroup order) they were taken on."""
    tag = workload if storage == "fp32" else f"{workload}_{storage}"
    path = os.path.join(ROOT, "profiles", f"traffic_{tag}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_hash") != kernel_source_hash():
        return None
    rec = rec.get("launches", {}).get(f"{tile}/{int(xcd)}")
    return rec["bytes_per_launch"] if rec else None


def time_steps(solver, steps: int, warmup: int):
    import torch

    solver.step(warmup)
    torch.cuda.synchronize()
    stream = solver.stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    solver.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / 1e3, wall


def pick_launch(solver, args):
    """Launch shape: the library's autotuner (timed outside the measured
    region, state untouched) or a fixed choice."""
    if args.tile == "auto":
        return solver.autotune(reps=20 if solver.N < 1 << 20 else 3)
    mode = args.xcd if args.xcd is not None else (0 if args.no_xcd else 1)
    solver.set_launch(args.tile, mode)
    return args.tile, mode


def plain_until_frozen(lbm, d, every: int, max_steps: int):
    """One droplet alone on the plain single-grid solver (FP32 storage):
    step in intervals, read the liquid volume, stop at 1 % of the initial."""
    import torch

    s = lbm.Solver(dict(d["params"], storage=lbm.STORAGE["fp32"]), d["phi0"], d["T0"])
    s.autotune(reps=5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps, liq = [0], [s.diag()["sum_liquid"]]
    while steps[-1] < max_steps:
        s.step(every)
        steps.append(steps[-1] + every)
        liq.append(s.diag()["sum_liquid"])
        if liq[-1] <= 0.01 * liq[0]:
            break
    secs = time.perf_counter() - t0
    thr = 0.01 * liq[0]
    a, c = liq[-2], liq[-1]
    tf = steps[-2] + every * min(max((a - thr) / (a - c), 0.0), 1.0) if c <= thr and a > c else float("nan")
    return tf, steps[-1], secs


def sweep_bench(lbm, W, n: int, n_plain: int, time_limit: float):
    """The batched sweep: n droplets (R ~ U(16,64), theta ~ U(60,150),
    Ste ~ U(0.05,0.3), gamma ~ U(0.85,1.1), 0-8 bubbles, grid 4R x 3R, FP16
    storage) all run until frozen as one queue, against the plain FP32 solver
    one droplet at a time on a random subsample of the same droplets."""
    import numpy as np
    import torch

    every, max_steps = 200, 2_000_000
    drops = W.sweep_droplets(n, seed=0, storage=lbm.STORAGE["fp16"])
    b = lbm.Batch([d["params"] for d in drops], [d["phi0"] for d in drops], [d["T0"] for d in drops],
                  radii=[d["R"] for d in drops], slots=n)
    b.configure(sample_every=every, max_steps=max_steps)
    tile, grp = b.autotune(reps=5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while True:
        b.step(50000, until_frozen=True)
        res = b.results()
        done = sum(r["status"] != "running" and r["status"] != "queued" for r in res)
        print(f"sweep: {done}/{n} droplets finished after {time.perf_counter() - t0:.1f} s", file=sys.stderr,
              flush=True)
        if done == n or time.perf_counter() - t0 > time_limit:
            break
    secs = time.perf_counter() - t0
    node_steps = sum(d["params"]["nx"] * d["params"]["ny"] * r["steps"] for d, r in zip(drops, res))
    frozen = [r for r in res if r["status"] == "frozen"]
    out = {
        "workload": f"{n} droplets, R~U(16,64), theta~U(60,150), Ste~U(0.05,0.3), gamma~U(0.85,1.1), 0-8 bubbles, "
                    "grid round(4R) x round(3R), FP16 storage, each run until 1 % of its liquid is left",
        "droplets": n, "frozen": len(frozen), "seconds": round(secs, 2), "droplets_per_s": round(len(frozen) / secs, 3),
        "node_steps": int(node_steps), "MLUPS": round(node_steps / secs / 1e6, 1), "tile": tile, "xcd_group": grp,
        "t_freeze_steps": [round(float(q), 1) for q in np.nanpercentile([r["t_freeze"] for r in res], [0, 50, 100])],
    }
    if n_plain > 0:
        pick = np.random.default_rng(1).choice(n, min(n_plain, n), replace=False)
        ptime, pwork, errs = 0.0, 0, []
        for i in pick:
            tf, st, sec = plain_until_frozen(lbm, drops[i], every, max_steps)
            ptime += sec
            pwork += drops[i]["params"]["nx"] * drops[i]["params"]["ny"] * st
            errs.append(abs(res[i]["t_freeze"] - tf) / tf)
            print(f"plain: droplet {i} t_freeze {tf:.1f} (batched {res[i]['t_freeze']:.1f}) in {sec:.2f} s",
                  file=sys.stderr, flush=True)
        plain_dps = len(pick) / ptime
        out["plain_fp32"] = {
            "droplets_per_s": round(plain_dps, 3), "MLUPS": round(pwork / ptime / 1e6, 1),
            "sample": f"{len(pick)} random droplets of the same sweep, one at a time, FP32 storage, "
                      f"{ptime:.1f} s",
        }
        out["speedup_droplets_per_s"] = round(out["droplets_per_s"] / plain_dps, 2)
        out["t_freeze_rel_err_max"] = float(f"{max(errs):.2e}")
    return out


def surrogate_bench(sweep):
    """The learned surrogate: trained on the stored sweeps (sweep_train*.npz),
    scored on the 512 held-out droplets against the solver's values."""
    from paper_2403_16122_amd import surrogate as S

    data = os.path.join(ROOT, "paper_2403_16122_amd", "data")
    tr, te = S.load_training(data), S.load(os.path.join(data, "sweep_test.npz"))
    sur = S.Surrogate(ensemble=8, seed=0, fallback_rel=0.05)
    sur.fit(tr)
    ev = S.evaluate(sur, te)
    out = {"ensemble": 8, "train_droplets": int(len(tr["R"])), "train_seconds": round(sur.train_seconds, 2)}
    out.update({k: (round(v, 5) if v == v else None) if isinstance(v, float) else v for k, v in ev.items()})
    out["droplets_per_s"] = round(ev["n"] / ev["inference_seconds"], 1)
    out["fallback_rel"] = sur.fallback_rel
    # the same network with the 2 % fallback threshold
    sur.fallback_rel = 0.02
    ev2 = S.evaluate(sur, te)
    out["at_2pct"] = {k: (round(ev2[k], 5) if ev2[k] == ev2[k] else None)  # NaN (nothing accepted) -> null
                      for k in ("fallback_fraction", "with_fallback_t_star_rel_err_median",
                                "with_fallback_t_star_rel_err_p90", "accepted_t_star_rel_err_max")}
    if sweep and sweep.get("droplets_per_s"):
        out["speedup_vs_batched_solver"] = round(out["droplets_per_s"] / sweep["droplets_per_s"], 1)
    return out


def host_io(lbm, params, phi0, T0, N, steps, step_secs):
    """The boundary takes the initial fields from host memory and returns
    fields to host memory: time lbm_init from host arrays (workspace, copy
    in, population set-up) and one read-back of all ten fields, and the rate
    of a job that does both around the timed steps."""
    import torch

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s = lbm.Solver(params, phi0, T0)
    s.sync()
    t_init = time.perf_counter() - t0
    s.step(1)
    s.sync()
    t0 = time.perf_counter()
    s.fields(tuple(lbm.FIELD_BITS))
    t_fields = time.perf_counter() - t0
    del s
    torch.cuda.empty_cache()
    job = t_init + step_secs + t_fields
    return {"init_s": round(t_init, 4), "fields_all_s": round(t_fields, 4),
            "host_bytes": int(N * 8 * (2 + len(lbm.FIELD_BITS))),
            "job_MLUPS": round(N * steps / job / 1e6, 1),
            "note": "init from host arrays + the timed steps + one read-back of every field, wall clock"}


def to_frozen(lbm, params, phi0, T0, tile, xcd):
    """The bench's droplet from its initial state until 1 % of its liquid is
    left (diagnostics every 5000 steps): wall time, steps, and the frozen
    shape."""
    import torch

    solver = lbm.Solver(params, phi0, T0)
    solver.set_launch(tile, xcd)
    d0 = solver.diag()
    h0 = lbm.shape_of(phi0.reshape(params["ny"], params["nx"]))["height"]
    start = solver.step_count
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while solver.step_count - start < 1_000_000:
        solver.step(5000)
        d = solver.diag()
        if d["sum_liquid"] <= 0.01 * d0["sum_liquid"]:
            break
    secs = time.perf_counter() - t0
    shape = lbm.shape_of(solver.fields(("phi",))["phi"])
    note(f"droplet frozen after {solver.step_count} steps in {secs:.1f} s")
    return {"steps": int(solver.step_count), "seconds": round(secs, 2),
            "frozen": bool(d["sum_liquid"] <= 0.01 * d0["sum_liquid"]),
            "area_ratio": round(d["sum_phic"] / d0["sum_phic"], 4),
            "rho_l_over_rho_s": round(params["rho_l"] / params["rho_s"], 4),
            "height_ratio": round(shape["height"] / h0, 4), "base_radius": round(shape["base_radius"], 2),
            "aspect_ratio": round(shape["height"] / shape["base_radius"], 4),
            "tip_angle_deg": round(shape["tip_angle_deg"], 1),
            "note": "from the initial state, launch as timed above; diagnostics every 5000 steps inside the wall time"}


def oracle_rate(oracle, params, phi0, T0, budget_s: float, threads: int):
    """MLUPS of the FP64 oracle over `budget_s` seconds of steps from the
    initial state, and the number of steps taken."""
    o = oracle.OracleSolver(params, phi0, T0, threads=threads)
    n = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        o.step(5)
        n += 5
    dt = time.perf_counter() - t0
    return params["nx"] * params["ny"] * n / dt / 1e6, n, dt


def cpu_baseline(params, phi0, T0, budget_s: float):
    import oracle

    cores = oracle.oracle.default_threads()
    v, n, dt = oracle_rate(oracle, params, phi0, T0, budget_s, cores)
    v1, n1, dt1 = oracle_rate(oracle, params, phi0, T0, budget_s / 3, 1)
    return dict(value=round(v, 3), unit="MLUPS", cores=cores, kind="oracle",
                sample=f"{n} steps of the same workload from its initial state ({dt:.1f} s, FP64, OpenMP rows)",
                single_thread={"value": round(v1, 3), "unit": "MLUPS", "cores": 1,
                               "sample": f"{n1} steps from the initial state ({dt1:.1f} s, FP64, one thread)"})


def note(msg: str):
    """Progress line on stderr (the JSON result is the only stdout line)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--workload", default="sessile512")
    ap.add_argument("--tile", default="auto", help="auto (library autotuner) or a name of lbm.TILE_VARIANTS")
    ap.add_argument("--no-xcd", action="store_true", help="round-robin workgroup dispatch (xcd mode 0)")
    ap.add_argument("--xcd", type=int, default=None, help="workgroup-to-XCD mapping mode 0/1/2 (fixed tiles only)")
    ap.add_argument("--storage", default="fp32", choices=("fp32", "fp16", "bf16"),
                    help="population storage format (compute is FP32 in every case)")
    ap.add_argument("--no-storage-variants", dest="storage_variants", action="store_false",
                    help="skip the FP16/BF16 storage runs on the 4096x2048 probe")
    ap.add_argument("--probe-steps", type=int, default=100, help="steps on the 4096x2048 grid (0: skip)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="oracle timing budget (0: skip)")
    ap.add_argument("--sweep-droplets", type=int, default=256, help="droplets in the batched sweep (0: skip)")
    ap.add_argument("--sweep-plain", type=int, default=16, help="droplets of the sweep re-run one at a time in FP32")
    ap.add_argument("--sweep-time-limit", type=float, default=240.0)
    ap.add_argument("--no-to-frozen", dest="to_frozen", action="store_false",
                    help="skip running the 512x256 droplet to full solidification")
    ap.add_argument("--no-surrogate", dest="surrogate", action="store_false",
                    help="skip training and scoring the surrogate network")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="run one plain device copy of this many MiB first (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); "
              "sharding a grid into y-slabs, or a sweep by droplets, across GPUs is not built", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2403_16122_amd import lbm, workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.calib_copy_mb > 0:
        n = args.calib_copy_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    params, phi0, T0, meta = W.workload(args.workload, seed=0)
    params["storage"] = lbm.STORAGE[args.storage]
    bpn = BYTES_PER_NODE[args.storage]
    N = params["nx"] * params["ny"]
    solver = lbm.Solver(params, phi0, T0)
    tile, xcd = pick_launch(solver, args)
    torch.cuda.synchronize()
    secs, wall = time_steps(solver, args.steps, args.warmup)
    d = solver.diag()
    if d["rc"] != 0:
        print(f"bench.py: non-finite state after the timed steps ({d})", file=sys.stderr)
        sys.exit(3)
    mlups = N * args.steps / secs / 1e6
    # a two-step launch processes 2 N node-steps; achieved counts the
    # algorithmic bytes of those node-steps over the launch's duration
    spl = 2 if tile in lbm.TWO_STEP_VARIANTS else 1
    launch_s = secs * spl / args.steps
    achieved = bpn * N * spl / launch_s / 1e9
    traffic = measured_traffic(args.workload, args.storage, tile, xcd)
    out = {
        "metric": METRIC,
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(secs / args.steps * 1e3, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: {params['nx']}x{params['ny']} sessile droplet R={meta['R']:g} lu, "
                        f"theta {meta['theta']:g}, rho_s/rho_l {params['rho_s']:g}, Ste 0.1, Bond 0.1, "
                        f"W=4, M=0.1, rho_l/rho_g=1000, {args.storage.upper()} populations (planar 2-D)",
            "nx": params["nx"], "ny": params["ny"], "tile": tile, "xcd_remap": xcd, "storage": args.storage,
            "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": (("k_step2w" if tile.endswith("w") else "k_step2")
                       + " (two fused collide + pull-stream steps per launch)" if spl == 2
                       else "k_step (fused collide + pull-stream)"),
            "steps_per_launch": spl,
            "bytes_per_launch": bpn * N * spl,
            "note": ("working set fits the 256 MB Infinity Cache at this size; see hbm_probe"
                     + ("; bytes_per_launch counts 256 B per node-step for the launch's 2 N node-steps, while "
                        "the launch itself reads and writes the state once" if spl == 2 else "")),
        },
        "wall_s": round(wall, 3),
    }
    del solver
    out["host_io"] = host_io(lbm, params, phi0, T0, N, args.steps, secs)
    if args.to_frozen and args.workload == "sessile512" and args.storage == "fp32":
        out["to_frozen"] = to_frozen(lbm, params, phi0, T0, tile, xcd)
    torch.cuda.empty_cache()
    note(f"{args.workload}: {out['value']} MLUPS ({tile}, order {xcd})")
    if args.probe_steps > 0:
        pp, pphi, pT, _ = W.workload("probe4096", seed=0)
        pp["storage"] = params["storage"]
        Np = pp["nx"] * pp["ny"]
        ps = lbm.Solver(pp, pphi, pT)
        ptile, pxcd = pick_launch(ps, args)
        psecs, _ = time_steps(ps, args.probe_steps, 10)
        pl = psecs / args.probe_steps
        pspl = 2 if ptile in lbm.TWO_STEP_VARIANTS else 1  # node-steps per launch
        pach = bpn * Np / pl / 1e9
        out["hbm_probe"] = {
            "workload": "probe4096: 4096x2048 sessile droplet R=640 (same physics), 2.3 GB working set",
            "steps": args.probe_steps, "MLUPS": round(Np * args.probe_steps / psecs / 1e6, 1),
            "tile": ptile, "xcd_remap": pxcd, "steps_per_launch": pspl,
            "achieved": round(pach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(pach / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic("probe4096", args.storage, ptile, pxcd),
        }
        # practical bandwidth beside the nominal peak: a 2 GiB device copy
        # (read + write) and the step's measured traffic per second
        cn = (2 << 30) // 4
        ca = torch.ones(cn, dtype=torch.float32, device="cuda")
        cb = torch.empty_like(ca)
        cb.copy_(ca)
        c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        c0.record()
        for _ in range(10):
            cb.copy_(ca)
        c1.record()
        torch.cuda.synchronize()
        out["hbm_probe"]["plain_copy_GBps"] = round(2 * cn * 4 * 10 / (c0.elapsed_time(c1) / 1e3) / 1e9, 1)
        if out["hbm_probe"]["traffic"]:
            out["hbm_probe"]["traffic_GBps"] = round(out["hbm_probe"]["traffic"] / (pl * pspl) / 1e9, 1)
        del ca, cb
        torch.cuda.empty_cache()
        # the unfused two-kernel step on the same grid: what fusion saves
        ps.set_launch("unfused64x8", pxcd)
        usecs, _ = time_steps(ps, args.probe_steps, 10)
        ubpn = UNFUSED_BYTES_PER_NODE[args.storage]
        out["hbm_probe"]["unfused"] = {
            "launch": f"unfused64x8, order {pxcd}", "MLUPS": round(Np * args.probe_steps / usecs / 1e6, 1),
            "bytes_per_node": ubpn, "achieved": round(ubpn * Np / (usecs / args.probe_steps) / 1e9, 1),
            "fused_speedup": round(usecs / psecs, 3),
        }
        del ps
        torch.cuda.empty_cache()
        note(f"probe4096: {out['hbm_probe']['MLUPS']} MLUPS ({ptile}, order {pxcd})")
        # the same probe with 16-bit population storage (FP32 compute)
        if args.storage == "fp32" and args.storage_variants:
            out["storage_variants"] = {}
            for st in ("fp16", "bf16"):
                pp["storage"] = lbm.STORAGE[st]
                vs = lbm.Solver(pp, pphi, pT)
                vtile, vxcd = pick_launch(vs, args)
                vsecs, _ = time_steps(vs, args.probe_steps, 10)
                vl = vsecs / args.probe_steps
                vach = BYTES_PER_NODE[st] * Np / vl / 1e9
                out["storage_variants"][st] = {
                    "workload": "probe4096", "MLUPS": round(Np * args.probe_steps / vsecs / 1e6, 1),
                    "tile": vtile, "xcd_remap": vxcd, "bytes_per_node": BYTES_PER_NODE[st],
                    "achieved": round(vach, 1), "unit": "GB/s", "frac": round(vach / HBM_PEAK_GBS, 4),
                    "traffic": measured_traffic("probe4096", st, vtile, vxcd),
                }
                del vs
                torch.cuda.empty_cache()
                note(f"probe4096 {st}: {out['storage_variants'][st]['MLUPS']} MLUPS ({vtile}, order {vxcd})")
    if args.sweep_droplets > 0:
        out["sweep"] = sweep_bench(lbm, W, args.sweep_droplets, args.sweep_plain, args.sweep_time_limit)
        torch.cuda.empty_cache()
    if args.surrogate:
        out["surrogate"] = surrogate_bench(out.get("sweep"))
        note("surrogate done")
    if args.cpu_seconds > 0:
        out["cpu_baseline"] = cpu_baseline(params, phi0, T0, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
