"""Batched sweep on the GPU through the C ABI.

* One launch over many grids computes exactly what the single-grid solver
  computes for each (same tile shape and storage: bitwise equal fields),
  whatever the tile layout, and the captured graph replays equal the same
  steps launched one by one, and a whole interval in one persistent launch.
* Run until frozen, the queue (more droplets than slots, so slots are
  refilled) gives each droplet the freezing time, height, base radius and
  tip angle that the FP64 oracle and the shape checker give for it.
* The device shape measurement equals the checker on the same field.
"""
import math

import numpy as np
import pytest

from oracle import shape as SH
from paper_2403_16122_amd import workloads as W

pytestmark = pytest.mark.gpu


def _lbm():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_16122_amd import lbm

    return lbm


def small_sweep(n, seed, storage=0, R_range=(7.0, 12.0), ste_range=(0.2, 0.3)):
    return W.sweep_droplets(n, seed=seed, R_range=R_range, ste_range=ste_range, max_bubbles=1, storage=storage)


def make_batch(lbm, drops, slots=None):
    return lbm.Batch([d["params"] for d in drops], [d["phi0"] for d in drops], [d["T0"] for d in drops],
                     radii=[d["R"] for d in drops], slots=slots)


@pytest.mark.parametrize("storage,tile,xcd", [(0, "64x4", 1), (1, "64x8", 0), (2, "128x4", 1), (1, "64x8", 2),
                                          (0, "32x8", 2)])
def test_batch_equals_single_solver_bitwise(storage, tile, xcd):
    lbm = _lbm()
    drops = small_sweep(5, seed=3, storage=storage)
    print(f"batch of {len(drops)} storage={storage} tile={tile} xcd={xcd}", flush=True)
    b = make_batch(lbm, drops)
    b.configure(sample_every=50, use_graph=True)
    b.set_launch(tile, xcd)
    b.step(200)
    names = ("phi", "T", "ux", "uy", "p", "fl")
    for i, d in enumerate(drops):
        s = lbm.Solver(d["params"], d["phi0"], d["T0"])
        s.set_launch(tile, 1)
        s.step(200)
        fs, fb = s.fields(names), b.fields(i, names)
        for k in names:
            assert np.array_equal(fs[k], fb[k]), (i, k, np.abs(fs[k] - fb[k]).max())
    assert all(r["steps"] == 200 for r in b.results())


@pytest.mark.parametrize("storage,tile,xcd", [(0, "two32x8w", 1), (1, "two32x8w", 0), (1, "two32x16w", 1),
                                          (2, "two32x16w", 0)])
def test_two_step_batch_equals_single_steps_bitwise(storage, tile, xcd):
    """Two steps per launch in the batch (intervals of a multiple of 4
    steps) give every droplet exactly the single solver's single-step
    state, in every storage format; an interval that is not a multiple of 4
    is refused while such a launch is set."""
    lbm = _lbm()
    drops = small_sweep(5, seed=4, storage=storage)
    print(f"two-step batch of {len(drops)} storage={storage} tile={tile} xcd={xcd}", flush=True)
    b = make_batch(lbm, drops)
    b.configure(sample_every=52, use_graph=True)
    b.set_launch(tile, xcd)
    with pytest.raises(lbm.LbmError):
        b.configure(sample_every=50)
    b.step(208)
    names = ("phi", "T", "ux", "uy", "p", "fl")
    for i, d in enumerate(drops):
        s = lbm.Solver(d["params"], d["phi0"], d["T0"])
        s.set_launch("64x8", 1)
        s.step(208)
        fs, fb = s.fields(names), b.fields(i, names)
        for k in names:
            assert np.array_equal(fs[k], fb[k]), (i, k, np.abs(fs[k] - fb[k]).max())
    assert all(r["steps"] == 208 for r in b.results())


def test_graph_replays_equal_individual_launches():
    lbm = _lbm()
    drops = small_sweep(4, seed=5, storage=1)
    g = make_batch(lbm, drops)
    e = make_batch(lbm, drops)
    g.configure(sample_every=40, use_graph=True)
    e.configure(sample_every=40, use_graph=False)
    for rep in range(4):  # every replay, with eager work and synchronisation in between
        print(f"replay {rep}", flush=True)
        g.step(40)
        e.step(40)
        for i in range(len(drops)):
            a, c = g.fields(i, ("phi", "T", "ux")), e.fields(i, ("phi", "T", "ux"))
            for k in a:
                assert np.array_equal(a[k], c[k]), (rep, i, k)


def test_autotune_does_not_advance_the_state():
    lbm = _lbm()
    drops = small_sweep(6, seed=7, storage=1)
    a = make_batch(lbm, drops)
    c = make_batch(lbm, drops)
    a.step(100)
    c.step(100)
    tile, grp = a.autotune(reps=3)
    print(f"autotune picked {tile} xcd_group={grp}", flush=True)
    c.set_launch(tile, grp)
    a.step(100)
    c.step(100)
    for i in range(len(drops)):
        fa, fc = a.fields(i, ("phi", "T")), c.fields(i, ("phi", "T"))
        assert np.array_equal(fa["phi"], fc["phi"]) and np.array_equal(fa["T"], fc["T"])


def oracle_freeze(oracle_mod, d, every, max_steps):
    o = oracle_mod.OracleSolver(d["params"], d["phi0"], d["T0"])
    steps, liq = [0], [o.diag()["sum_liquid"]]
    while steps[-1] < max_steps:
        o.step(every)
        steps.append(steps[-1] + every)
        liq.append(o.diag()["sum_liquid"])
        if liq[-1] <= 0.01 * liq[0]:
            break
    return SH.freeze_time(steps, liq), steps[-1], o


@pytest.mark.parametrize("barrier", ["flat", "per_xcd"])
@pytest.mark.parametrize("storage", [0, 1])
def test_persistent_intervals_equal_graph_replays(storage, barrier):
    """Each sampling interval as one persistent cooperative launch (a grid
    barrier between its steps) gives every droplet bitwise the state of the
    replayed per-step launches, over a queue run until frozen with slots
    refilled (so the tile map changes between intervals)."""
    lbm = _lbm()
    drops = small_sweep(5, seed=17, storage=storage, R_range=(6.0, 9.0), ste_range=(0.25, 0.3))
    print(f"persistent intervals storage={storage} barrier={barrier}", flush=True)
    g = make_batch(lbm, drops, slots=3)
    p = make_batch(lbm, drops, slots=3)
    g.configure(sample_every=40, max_steps=20000)
    g.set_launch("64x8", 2)
    p.configure(sample_every=40, max_steps=20000, persistent=barrier)
    p.set_launch("64x8", 2)
    with pytest.raises(lbm.LbmError):
        p.set_launch("64x4", 2)  # persistent intervals run 64x8 tiles only
    for rep in range(3):
        print(f"interval {rep}", flush=True)
        g.step(40)
        p.step(40)
        for i in range(3):
            a, c = g.fields(i, ("phi", "T", "ux", "p")), p.fields(i, ("phi", "T", "ux", "p"))
            for k in a:
                assert np.array_equal(a[k], c[k]), (rep, i, k)
    g.step(200000, until_frozen=True)
    p.step(200000, until_frozen=True)
    rg, rp = g.results(), p.results()
    for a, c in zip(rg, rp):
        print(f"graph {a}\npersistent {c}", flush=True)
        assert a["status"] == c["status"] and a["steps"] == c["steps"]
        for k in ("t_freeze", "liquid", "height", "base_radius", "tip_angle_deg"):
            assert (a[k] == c[k]) or (math.isnan(a[k]) and math.isnan(c[k])), k


def test_a_persistent_interval_whose_barrier_wait_runs_out_is_reported():
    """The failure path of the persistent interval, forced from the host:
    40 droplets of R 40-64 give some 3000 tiles over 512 co-resident
    workgroups, which step unequal numbers of tiles between barriers, so
    the early ones wait longer than a bound of 1 us.  The wait runs out,
    every workgroup leaves, and lbm_batch_step reports the time-out; a fresh
    queue then runs persistent intervals bitwise equal to the graph."""
    lbm = _lbm()
    drops = small_sweep(40, seed=21, storage=1, R_range=(40.0, 64.0), ste_range=(0.05, 0.3))
    print("forced batch barrier time-out", flush=True)
    b = make_batch(lbm, drops)
    b.configure(sample_every=20, persistent="per_xcd", wait_limit_us=1)
    with pytest.raises(lbm.LbmError) as err:
        b.step(20)
    assert err.value.code == lbm.LBM_EDEVICE and "timed out" in str(err.value)
    del b
    g = make_batch(lbm, drops[:3])
    p = make_batch(lbm, drops[:3])
    g.configure(sample_every=20)
    g.set_launch("64x8", 2)
    p.configure(sample_every=20, persistent="flat")
    p.set_launch("64x8", 2)
    g.step(40)
    p.step(40)
    for i in range(3):
        a, c = g.fields(i, ("phi", "T", "ux")), p.fields(i, ("phi", "T", "ux"))
        for k in a:
            assert np.array_equal(a[k], c[k]), (i, k)


def test_queue_until_frozen_against_oracle(oracle_mod):
    lbm = _lbm()
    drops = small_sweep(3, seed=11, R_range=(6.0, 8.0), ste_range=(0.25, 0.3))
    every, limit = 20, 40000
    b = make_batch(lbm, drops, slots=2)
    b.configure(sample_every=every, max_steps=limit)
    b.step(10 * limit, until_frozen=True)
    res = b.results()
    for i, (d, r) in enumerate(zip(drops, res)):
        print(f"drop {i}: R={d['R']:.2f} theta={d['theta']:.1f} Ste={d['ste']:.3f} -> {r}", flush=True)
        assert r["status"] == "frozen", r
        tf, stop, o = oracle_freeze(oracle_mod, d, every, limit)
        print(f"  oracle t_freeze {tf:.1f} (stopped at {stop})", flush=True)
        assert r["t_freeze"] == pytest.approx(tf, rel=5e-3)
        assert abs(r["steps"] - stop) <= every
        p = d["params"]
        assert r["t_star"] == pytest.approx(SH.fourier_number(r["t_freeze"], p["k_l"], p["rho_l"], p["cp_l"], d["R"]))
        m = SH.shape_metrics(o.fields(("phi",))["phi"])
        print(f"  oracle shape {m}", flush=True)
        assert r["height"] == pytest.approx(m["height"], abs=0.05)
        assert r["base_radius"] == pytest.approx(m["base_radius"], abs=0.1)
        if m["npts"] >= 3:
            assert r["tip_angle_deg"] == pytest.approx(m["tip_angle_deg"], abs=3.0)


def test_step_limit_retires_unfrozen_droplets():
    lbm = _lbm()
    drops = small_sweep(3, seed=13)
    b = make_batch(lbm, drops, slots=2)
    b.configure(sample_every=20, max_steps=60)
    b.step(1000, until_frozen=True)
    for r in b.results():
        assert r["status"] == "limit" and r["steps"] == 60 and math.isnan(r["t_freeze"])


@pytest.mark.parametrize("kind", ["cap", "wedge", "sweep"])
def test_device_shape_equals_checker(kind):
    lbm = _lbm()
    if kind == "cap":
        y, x = np.mgrid[0:70, 0:100].astype(float)
        phi = 0.5 * (1 + np.tanh(0.5 * (25.0 - np.hypot(x - 50.3, y + 8.0))))
    elif kind == "wedge":
        y, x = np.mgrid[0:90, 0:120].astype(float)
        h = math.radians(40.0)
        d = np.maximum((x - 60) * math.cos(h) + (y - 60) * math.sin(h), -(x - 60) * math.cos(h) + (y - 60) * math.sin(h))
        phi = 0.5 * (1 + np.tanh(-0.5 * d))
    else:
        phi = small_sweep(1, seed=17, R_range=(20.0, 20.0), ste_range=(0.1, 0.1))[0]["phi0"].reshape(60, 80)
    phi32 = phi.astype(np.float32).astype(np.float64)  # the device measures FP32 fields
    g, c = lbm.shape_of(phi), SH.shape_metrics(phi32)
    print(kind, g, c, flush=True)
    for k in ("height", "base_radius", "tip_angle_deg"):
        assert g[k] == pytest.approx(c[k], rel=1e-7, abs=1e-9)
    assert g["npts"] == c["npts"]


def test_batch_streaming_stores_bitwise_equal_cached():
    lbm = _lbm()
    drops = small_sweep(4, seed=19, storage=1)
    fields = []
    for mode in ("cached", "streaming"):
        print(f"batch store mode {mode}", flush=True)
        b = make_batch(lbm, drops)
        b.configure(sample_every=40, use_graph=True)
        b.set_store_mode(mode)
        b.step(120)
        fields.append([b.fields(i, ("phi", "T", "ux", "p")) for i in range(len(drops))])
    for fa, fb in zip(*fields):
        for k in fa:
            assert np.array_equal(fa[k], fb[k]), k
