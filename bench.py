"""Throughput of the fused coupled-lattice step on one MI355X.

A step is one time step of all three D2Q9 lattices (phase field, flow,
enthalpy) over the whole grid.  The headline workload is the largest
single-GPU configuration: the 1024x512 droplet (R = 160) with gas bubbles,
contact angle and bubble count from the seed, chi = 1, rho_s/rho_l = 0.9,
Ste = 0.1, FP32 populations; the same droplet is also timed with FP16 and
BF16 population storage.  Inputs are resident in HBM before the timed
region.

Prints one JSON line with MLUPS, the roofline of the dominant step kernel
on a 4096x2048 grid whose 2.3 GB state does not fit the 256 MB Infinity
Cache (algorithmic 256 B per node update; the HBM traffic rocprofv3
measured for that launch beside it), the 512x256 droplet and its run to
full solidification, the batched sweep, the surrogate network, and the
FP64 oracle timed on the host cores.
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


def run_sweep(lbm, W, n: int, storage: str, time_limit: float, chunk: int = 50000, persistent=None):
    """The batched sweep in one storage format: every droplet run until 1 %
    of its liquid is left; returns (results, seconds, node_steps, launch).
    persistent: None (each interval a replayed graph of per-step launches)
    or the grid barrier of one persistent launch per interval."""
    import torch

    every, max_steps = 200, 2_000_000
    drops = W.sweep_droplets(n, seed=0, storage=lbm.STORAGE[storage])
    b = lbm.Batch([d["params"] for d in drops], [d["phi0"] for d in drops], [d["T0"] for d in drops],
                  radii=[d["R"] for d in drops], slots=n)
    b.configure(sample_every=every, max_steps=max_steps, persistent=persistent)
    tile, grp = b.autotune(reps=5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while True:
        b.step(chunk, until_frozen=True)
        res = b.results()
        done = sum(r["status"] != "running" and r["status"] != "queued" for r in res)
        print(f"sweep {storage}{' persistent ' + persistent if persistent else ''}: {done}/{n} droplets finished "
              f"after {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
        if done == n or time.perf_counter() - t0 > time_limit:
            break
    secs = time.perf_counter() - t0
    node_steps = sum(d["params"]["nx"] * d["params"]["ny"] * r["steps"] for d, r in zip(drops, res))
    del b
    torch.cuda.empty_cache()
    return drops, res, secs, node_steps, (tile, grp)


def sweep_bench(lbm, W, n: int, n_plain: int, time_limit: float, reference: bool = True, chunk: int = 50000,
                persistent: bool = True):
    """The batched sweep: n droplets (R ~ U(16,64), theta ~ U(60,150),
    Ste ~ U(0.05,0.3), gamma ~ U(0.85,1.1), 0-8 bubbles, grid 4R x 3R, FP16
    storage) all run until frozen as one queue; the same queue in FP32
    storage (bitwise the plain FP32 solver's results) for the freezing-time
    error of every droplet; and the plain FP32 solver one droplet at a time
    on a random subsample, for its rate."""
    import numpy as np

    every, max_steps = 200, 2_000_000
    drops, res, secs, node_steps, (tile, grp) = run_sweep(lbm, W, n, "fp16", time_limit, chunk)
    frozen = [r for r in res if r["status"] == "frozen"]
    out = {
        "workload": f"{n} droplets, R~U(16,64), theta~U(60,150), Ste~U(0.05,0.3), gamma~U(0.85,1.1), 0-8 bubbles, "
                    "grid round(4R) x round(3R), FP16 storage, each run until 1 % of its liquid is left",
        "droplets": n, "frozen": len(frozen), "seconds": round(secs, 2), "droplets_per_s": round(len(frozen) / secs, 3),
        "node_steps": int(node_steps), "MLUPS": round(node_steps / secs / 1e6, 1), "tile": tile, "xcd_group": grp,
        "t_freeze_steps": [round(float(q), 1) for q in np.nanpercentile([r["t_freeze"] for r in res], [0, 50, 100])],
    }
    if persistent:
        # the same queue with every 200-step interval in one persistent launch
        try:
            _, resp, secsp, nsp, (tilep, grpp) = run_sweep(lbm, W, n, "fp16", time_limit, chunk,
                                                           persistent="per_xcd")
            same = all(a["steps"] == c["steps"] and (a["t_freeze"] == c["t_freeze"] or
                                                     (np.isnan(a["t_freeze"]) and np.isnan(c["t_freeze"])))
                       for a, c in zip(res, resp))
            out["persistent_intervals"] = {
                "barrier": "per_xcd", "seconds": round(secsp, 2),
                "droplets_per_s": round(sum(r["status"] == "frozen" for r in resp) / secsp, 3),
                "MLUPS": round(nsp / secsp / 1e6, 1), "tile": tilep, "xcd_group": grpp, "same_results": same,
                "note": "each 200-step interval as one cooperative launch with a grid barrier between steps, "
                        "against the replayed graph of per-step launches above"}
        except lbm.LbmError as e:
            out["persistent_intervals"] = {"error": str(e)}
    if not reference:
        return out
    _, res32, secs32, ns32, (tile32, grp32) = run_sweep(lbm, W, n, "fp32", time_limit)
    tf16 = np.array([r["t_freeze"] for r in res])
    tf32 = np.array([r["t_freeze"] for r in res32])
    ok = np.isfinite(tf16) & np.isfinite(tf32)
    err = np.abs(tf16[ok] - tf32[ok]) / tf32[ok]
    out["batched_fp32"] = {"seconds": round(secs32, 2), "droplets_per_s": round(int(ok.sum()) / secs32, 3),
                           "MLUPS": round(ns32 / secs32 / 1e6, 1), "tile": tile32, "xcd_group": grp32}
    out["t_freeze_rel_err_vs_fp32"] = {
        "droplets": int(ok.sum()), "median": float(f"{np.median(err):.2e}"), "p95": float(f"{np.quantile(err, 0.95):.2e}"),
        "max": float(f"{err.max():.2e}"), "above_1pct": int((err > 0.01).sum()),
        "note": "every droplet of the sweep, FP16-storage batch against the FP32-storage batch (which equals the plain "
                "FP32 solver bit for bit)"}
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
        out["t_freeze_rel_err_max_plain_sample"] = float(f"{max(errs):.2e}")
    return out


def surrogate_bench(sweep):
    """The learned surrogate: trained on the stored sweeps (sweep_train*.npz),
    scored on the 512 held-out droplets against the solver's values, with
    the solver as fallback where the error model predicts more than 2 %."""
    from paper_2403_16122_amd import surrogate as S

    data = os.path.join(ROOT, "paper_2403_16122_amd", "data")
    tr, te = S.load_training(data), S.load(os.path.join(data, "sweep_test.npz"))
    sur = S.Surrogate(ensemble=8, seed=0, fallback_rel=0.02)
    sur.fit(tr)
    ev = S.evaluate(sur, te)
    out = {"ensemble": 8, "train_droplets": int(len(tr["R"])), "train_seconds": round(sur.train_seconds, 2),
           "fallback_rel": sur.fallback_rel}
    out.update({k: (round(v, 5) if v == v else None) if isinstance(v, float) else v for k, v in ev.items()})
    out["droplets_per_s"] = round(ev["n"] / ev["inference_seconds"], 1)
    # the same networks with a 5 % threshold
    sur.fallback_rel = 0.05
    ev5 = S.evaluate(sur, te)
    out["at_5pct"] = {k: (round(ev5[k], 5) if ev5[k] == ev5[k] else None)  # NaN (nothing accepted) -> null
                      for k in ("acceptance", "accepted_t_star_rel_err_max", "accepted_t_star_rel_err_p95",
                                "with_fallback_t_star_rel_err_median", "with_fallback_t_star_rel_err_p90")}
    if sweep and sweep.get("droplets_per_s"):
        out["speedup_vs_batched_solver"] = round(out["droplets_per_s"] / sweep["droplets_per_s"], 1)
        # droplets per second of the merged predictor: the network for the
        # accepted share, the batched solver for the rest
        acc = ev["acceptance"]
        out["merged_droplets_per_s"] = round(1.0 / ((1.0 - acc) / sweep["droplets_per_s"] + acc / out["droplets_per_s"]),
                                             3)
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
    """The 512x256 droplet from its initial state until 1 % of its liquid is
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


def oracle_rate(oracle, params, phi0, T0, threads: int, budget_s: float = 0.0, steps: int = 0):
    """MLUPS of the FP64 oracle from the initial state: `steps` steps, or
    as many as fit in `budget_s` seconds (in chunks of 5)."""
    o = oracle.OracleSolver(params, phi0, T0, threads=threads)
    n = 0
    t0 = time.perf_counter()
    if steps > 0:
        o.step(steps)
        n = steps
    else:
        while time.perf_counter() - t0 < budget_s:
            o.step(5)
            n += 5
    dt = time.perf_counter() - t0
    del o
    return params["nx"] * params["ny"] * n / dt / 1e6, n, dt


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(W, params, phi0, T0, workload: str, budget_s: float, gpu_rates: dict):
    """The FP64 oracle on the host: the headline workload for ~budget_s
    seconds on every host thread this process may use and for a third of it
    on one thread, then the 128x64 case (all 2000 steps) and slices of the
    512x256 and 4096x2048 cases, each with GPU MLUPS of the same workload
    beside it.  The oracle is rebuilt from its source with -O3 -march=native
    for this host (same bits as the in-tree build: FP64, no FMA
    contraction)."""
    import tempfile

    import oracle

    build = "gcc -O3 -march=native -fopenmp (built on this host)"
    try:
        oracle.oracle.use_library(oracle.oracle.build_native(tempfile.mkdtemp(prefix="lbm_oracle_")))
    except Exception as e:  # a host without gcc: time the in-tree -O3 build instead
        build = f"in-tree gcc -O3 build (native build failed: {e})"
    cores = oracle.oracle.host_threads()
    v, n, dt = oracle_rate(oracle, params, phi0, T0, cores, budget_s=budget_s)
    v1, n1, dt1 = oracle_rate(oracle, params, phi0, T0, 1, budget_s=budget_s / 3)
    out = dict(value=round(v, 3), unit="MLUPS", cores=cores, kind="oracle",
               sample=f"{n} steps of {workload} from its initial state ({dt:.1f} s, FP64, OpenMP over rows)",
               nproc=os.cpu_count(), affinity=len(os.sched_getaffinity(0)),
               omp_num_threads=os.environ.get("OMP_NUM_THREADS"), cpu_model=cpu_model(), build=build,
               single_thread={"value": round(v1, 3), "unit": "MLUPS", "cores": 1,
                              "sample": f"{n1} steps from the initial state ({dt1:.1f} s)"},
               gpu_MLUPS=gpu_rates.get(workload))
    slices = {}
    for name, steps, steps1 in (("sessile128", 2000, 2000), ("sessile512", 200, 40), ("probe4096", 10, 1)):
        pp, pphi, pT, _ = W.workload(name, seed=0)
        pp["storage"] = 0
        r, _, t = oracle_rate(oracle, pp, pphi, pT, cores, steps=steps)
        r1, _, t1 = oracle_rate(oracle, pp, pphi, pT, 1, steps=steps1)
        slices[name] = {"steps": steps, "MLUPS": round(r, 3), "seconds": round(t, 2),
                        "single_thread": {"steps": steps1, "MLUPS": round(r1, 3), "seconds": round(t1, 2)},
                        "gpu_MLUPS": gpu_rates.get(name)}
        note(f"oracle {name}: {r:.2f} MLUPS on {cores} threads, {r1:.2f} on one")
    out["slices"] = slices
    return out


def note(msg: str):
    """Progress line on stderr (the JSON result is the only stdout line)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def describe(name: str, params: dict, meta: dict, storage: str) -> str:
    if name == "bubbles1024":
        rb = [b[2] for b in meta["bubbles"]]
        return (f"bubbles1024: {params['nx']}x{params['ny']} droplet R={meta['R']:g} lu with {len(rb)} gas bubbles "
                f"(r {min(rb):.1f}-{max(rb):.1f} lu), contact angle {meta['theta']:.1f} deg, chi=1, "
                f"rho_s/rho_l {params['rho_s']:g}, Ste 0.1, W=4, M=0.1, rho_l/rho_g=1000, "
                f"{storage.upper()} populations (planar 2-D, seed 0)")
    if name in ("sessile512", "probe4096"):
        return (f"{name}: {params['nx']}x{params['ny']} sessile droplet R={meta['R']:g} lu, theta {meta['theta']:g}, "
                f"rho_s/rho_l {params['rho_s']:g}, Ste 0.1, Bond 0.1, W=4, M=0.1, rho_l/rho_g=1000, "
                f"{storage.upper()} populations (planar 2-D)")
    return f"{name}: {params['nx']}x{params['ny']}, {storage.upper()} populations"


def kernel_name(tile: str) -> str:
    import paper_2403_16122_amd.lbm as lbm

    if tile in lbm.TWO_STEP_VARIANTS:
        return ("k_step2w" if tile.endswith("w") else "k_step2") + " (two fused collide + pull-stream steps per launch)"
    return "k_step (fused collide + pull-stream)"


def timed_run(lbm, W, name: str, storage: str, steps: int, warmup: int, args):
    """One workload in one storage format: autotuned launch, `steps` timed
    steps after `warmup`; returns (record, seconds, tile, xcd)."""
    import torch

    params, phi0, T0, meta = W.workload(name, seed=0)
    params["storage"] = lbm.STORAGE[storage]
    N = params["nx"] * params["ny"]
    s = lbm.Solver(params, phi0, T0)
    tile, xcd = pick_launch(s, args)
    torch.cuda.synchronize()
    secs, wall = time_steps(s, steps, warmup)
    d = s.diag()
    if d["rc"] != 0:
        print(f"bench.py: non-finite state after the timed steps of {name} {storage} ({d})", file=sys.stderr)
        sys.exit(3)
    del s
    torch.cuda.empty_cache()
    spl = 2 if tile in lbm.TWO_STEP_VARIANTS else 1
    rec = {"workload": name, "storage": storage, "steps": steps, "MLUPS": round(N * steps / secs / 1e6, 1),
           "us_per_step": round(secs / steps * 1e6, 3), "tile": tile, "xcd_remap": xcd, "steps_per_launch": spl,
           "state_MB": round(lbm.workspace_bytes(params) / 2 ** 20, 1)}
    note(f"{name} {storage}: {rec['MLUPS']} MLUPS ({tile}, order {xcd})")
    return rec, secs, wall, (params, phi0, T0, meta)


def persistent_vs_per_step(lbm, W, name: str, steps: int, warmup: int, barriers=("flat", "per_xcd")):
    """`steps` FP32 steps of a workload as one launch per step and as one
    persistent cooperative launch (lbm_step_persistent) with each of its two
    grid barriers, all on 64x8 tiles in tile order 2 from the same state;
    HIP events on the solver's stream bracket each.  A persistent call also
    clears its barrier words and reads them back (a few microseconds per
    call)."""
    import torch

    params, phi0, T0, _ = W.workload(name, seed=0)
    N = params["nx"] * params["ny"]
    rec = {"workload": name, "steps": steps, "tile": "64x8", "xcd_remap": 2}
    for mode in ("per_step",) + tuple("persistent_" + b for b in barriers):
        s = lbm.Solver(params, phi0, T0)
        s.set_launch("64x8", 2)
        if mode == "per_step":
            run = s.step
        else:
            barrier = mode[len("persistent_"):]
            run = lambda n, s=s, barrier=barrier: s.step_persistent(n, barrier)  # noqa: E731
        run(warmup)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s.stream)
        wg = run(steps)
        e1.record(s.stream)
        torch.cuda.synchronize()
        secs = e0.elapsed_time(e1) / 1e3
        rec[mode] = {"us_per_step": round(secs / steps * 1e6, 3), "MLUPS": round(N * steps / secs / 1e6, 1)}
        if mode != "per_step":
            rec[mode]["workgroups"] = wg
            rec[mode]["over_per_step"] = round(rec[mode]["us_per_step"] / rec["per_step"]["us_per_step"], 3)
        del s
        torch.cuda.empty_cache()
    note(f"{name}: per-step launches {rec['per_step']['us_per_step']} us/step, persistent "
         + ", ".join(f"{rec['persistent_' + b]['us_per_step']} ({b} barrier)" for b in barriers) + " us/step")
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="bubbles1024")
    ap.add_argument("--tile", default="auto", help="auto (library autotuner) or a name of lbm.TILE_VARIANTS")
    ap.add_argument("--no-xcd", action="store_true", help="round-robin workgroup dispatch (xcd mode 0)")
    ap.add_argument("--xcd", type=int, default=None, help="workgroup-to-XCD mapping mode 0/1/2 (fixed tiles only)")
    ap.add_argument("--storage", default="fp32", choices=("fp32", "fp16", "bf16"),
                    help="population storage format of the headline (compute is FP32 in every case)")
    ap.add_argument("--no-storage-variants", dest="storage_variants", action="store_false",
                    help="skip the FP16/BF16 storage runs")
    ap.add_argument("--probe-steps", type=int, default=100, help="steps on the 4096x2048 grid (0: skip)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="oracle timing budget (0: skip)")
    ap.add_argument("--sweep-droplets", type=int, default=256, help="droplets in the batched sweep (0: skip)")
    ap.add_argument("--sweep-plain", type=int, default=16, help="droplets of the sweep re-run one at a time in FP32")
    ap.add_argument("--sweep-time-limit", type=float, default=240.0)
    ap.add_argument("--sweep-chunk", type=int, default=50000,
                    help="steps between the sweep's progress checks (time limit and finished count)")
    ap.add_argument("--no-sweep-reference", dest="sweep_reference", action="store_false",
                    help="skip the FP32-storage run of the sweep (and the plain re-runs)")
    ap.add_argument("--no-to-frozen", dest="to_frozen", action="store_false",
                    help="skip running the 512x256 droplet to full solidification")
    ap.add_argument("--no-surrogate", dest="surrogate", action="store_false",
                    help="skip training and scoring the surrogate network")
    ap.add_argument("--no-others", dest="others", action="store_false",
                    help="headline workload only (no 128x64 and 512x256 rates)")
    ap.add_argument("--no-persistent", dest="persistent", action="store_false",
                    help="skip the persistent-launch comparison")
    ap.add_argument("--no-sweep-persistent", dest="sweep_persistent", action="store_false",
                    help="skip the sweep with one persistent launch per interval")
    ap.add_argument("--persistent-barrier", default="both", choices=("both", "flat", "per_xcd"),
                    help="the grid barriers of the persistent-launch comparison")
    ap.add_argument("--persistent-workloads", default="",
                    help="comma-separated workloads of the persistent-launch comparison (default: the 128x64 and "
                         "512x256 droplets, the headline workload and, with --probe-steps, the 4096x2048 grid)")
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
    head, secs, wall, (params, phi0, T0, meta) = timed_run(lbm, W, args.workload, args.storage, args.steps,
                                                            args.warmup, args)
    N = params["nx"] * params["ny"]
    gpu_rates = {args.workload: head["MLUPS"]}
    out = {
        "metric": METRIC,
        "value": round(N * args.steps / secs / 1e6, 2),
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
            "workload": describe(args.workload, params, meta, args.storage),
            "nx": params["nx"], "ny": params["ny"], "tile": head["tile"], "xcd_remap": head["xcd_remap"],
            "storage": args.storage, "state_MB": head["state_MB"], "parallelism": "single GPU",
        },
        "wall_s": round(wall, 3),
    }
    # the headline droplet in every population storage format (compute FP32)
    formats = {args.storage: head}
    if args.storage_variants:
        for st in ("fp32", "fp16", "bf16"):
            if st not in formats:
                formats[st] = timed_run(lbm, W, args.workload, st, args.steps, args.warmup, args)[0]
    out["storage_formats"] = formats
    out["host_io"] = host_io(lbm, params, phi0, T0, N, args.steps, secs)
    torch.cuda.empty_cache()
    if args.others:
        # the 128x64 parity case and the 512x256 droplet (cache-resident sizes)
        for name in ("sessile128", "sessile512"):
            if name == args.workload:
                continue
            rec, _, _, (pp, pphi, pT, _m) = timed_run(lbm, W, name, "fp32", max(args.steps, 200), args.warmup, args)
            gpu_rates[name] = rec["MLUPS"]
            out.setdefault("other_workloads", {})[name] = rec
            if name == "sessile512" and args.to_frozen:
                out["to_frozen"] = to_frozen(lbm, pp, pphi, pT, rec["tile"], rec["xcd_remap"])
            torch.cuda.empty_cache()
    if args.persistent:
        # one persistent launch over all steps against one launch per step
        per = {}
        if args.persistent_workloads:
            names = args.persistent_workloads.split(",")
        else:
            names = [n for n in ("sessile128", "sessile512") if n != args.workload] + [args.workload]
            if args.probe_steps > 0 and args.workload != "probe4096":
                names.append("probe4096")
        runs = [(n, (args.probe_steps or 100) if n == "probe4096" else max(args.steps, 200)) for n in names]
        barriers = ("flat", "per_xcd") if args.persistent_barrier == "both" else (args.persistent_barrier,)
        for name, n in runs:
            try:
                per[name] = persistent_vs_per_step(lbm, W, name, n, 10, barriers)
            except lbm.LbmError as e:
                per[name] = {"error": str(e)}
        out["persistent_launch"] = per
    if args.probe_steps > 0:
        # the roofline: the dominant step kernel on a state beyond the Infinity Cache
        prec, psecs, _, (pp, pphi, pT, _m) = timed_run(lbm, W, "probe4096", "fp32", args.probe_steps, 10, args)
        gpu_rates["probe4096"] = prec["MLUPS"]
        Np = pp["nx"] * pp["ny"]
        ptile, pxcd, pspl = prec["tile"], prec["xcd_remap"], prec["steps_per_launch"]
        launch_s = psecs * pspl / args.probe_steps  # average duration of one launch (HIP events on its stream)
        alg = BYTES_PER_NODE["fp32"] * Np * pspl    # 256 B per node update x node updates per launch
        achieved = alg / launch_s / 1e9
        traffic = measured_traffic("probe4096", "fp32", ptile, pxcd)
        out["roofline"] = {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": kernel_name(ptile), "workload": describe("probe4096", pp, _m, "fp32"),
            "tile": ptile, "xcd_remap": pxcd, "steps_per_launch": pspl, "launch_us": round(launch_s * 1e6, 2),
            "bytes_per_launch": alg,
            "note": ("achieved counts the algorithmic 256 B per node update for every node update the launch "
                     "performs; measured on the 4096x2048 grid, whose 2.3 GB state exceeds the 256 MB Infinity "
                     "Cache (the headline grid's does not)"
                     + ("; a two-step launch reads and writes the state once, so this is an effective rate: "
                        "hbm_traffic gives what the launch moves" if pspl == 2 else "")),
        }
        if traffic:
            out["roofline"]["hbm_traffic"] = {
                "bytes_per_launch": traffic, "GBps": round(traffic / launch_s / 1e9, 1),
                "frac": round(traffic / launch_s / 1e9 / HBM_PEAK_GBS, 4),
                "note": "rocprofv3 FETCH_SIZE + WRITE_SIZE of this launch shape, calibrated on a plain copy"}
        # practical bandwidth beside the nominal peak: a 2 GiB device copy
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
        out["roofline"]["plain_copy_GBps"] = round(2 * cn * 4 * 10 / (c0.elapsed_time(c1) / 1e3) / 1e9, 1)
        del ca, cb
        torch.cuda.empty_cache()
        probe = {"fp32": prec}
        # the unfused two-kernel step on the same grid: what fusion saves
        ps = lbm.Solver(dict(pp, storage=0), pphi, pT)
        ps.set_launch("unfused64x8", pxcd)
        usecs, _ = time_steps(ps, args.probe_steps, 10)
        del ps
        torch.cuda.empty_cache()
        ubpn = UNFUSED_BYTES_PER_NODE["fp32"]
        probe["unfused_fp32"] = {
            "launch": f"unfused64x8, order {pxcd}", "MLUPS": round(Np * args.probe_steps / usecs / 1e6, 1),
            "bytes_per_node": ubpn, "achieved": round(ubpn * Np / (usecs / args.probe_steps) / 1e9, 1),
            "fused_speedup": round(usecs / psecs, 3)}
        if args.storage_variants:
            for st in ("fp16", "bf16"):
                vrec, vsecs, _, _ = timed_run(lbm, W, "probe4096", st, args.probe_steps, 10, args)
                vl = vsecs * vrec["steps_per_launch"] / args.probe_steps
                vach = BYTES_PER_NODE[st] * Np * vrec["steps_per_launch"] / vl / 1e9
                vtr = measured_traffic("probe4096", st, vrec["tile"], vrec["xcd_remap"])
                vrec.update({"bytes_per_node": BYTES_PER_NODE[st], "achieved": round(vach, 1), "unit": "GB/s",
                             "frac": round(vach / HBM_PEAK_GBS, 4), "traffic": vtr})
                if vtr:
                    vrec["traffic_GBps"] = round(vtr / vl / 1e9, 1)
                probe[st] = vrec
        out["probe4096"] = probe
    if args.sweep_droplets > 0:
        out["sweep"] = sweep_bench(lbm, W, args.sweep_droplets, args.sweep_plain, args.sweep_time_limit,
                                   args.sweep_reference, args.sweep_chunk, args.sweep_persistent)
        torch.cuda.empty_cache()
    if args.surrogate:
        out["surrogate"] = surrogate_bench(out.get("sweep"))
        note("surrogate done")
    if args.cpu_seconds > 0:
        out["cpu_baseline"] = cpu_baseline(W, params, phi0, T0, args.workload, args.cpu_seconds, gpu_rates)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
