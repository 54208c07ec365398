"""One persistent launch over many steps (lbm_step_persistent) against one
launch per step (lbm_step), through the C ABI.

The persistent kernel runs the same per-node update of Sec. 3 on 64x8 tiles
and orders the steps with a grid-wide barrier, so its states must be
bitwise those of per-step launches: a difference would be a halo pulled
before its neighbour's stores were visible (a barrier that does not order
them across the XCDs' L2s), not rounding.  Both barriers are checked: the
flat one (every workgroup writes its XCD's L2 back) and the per-XCD one
(the last workgroup to arrive on an XCD writes it back for all).  The grids
are ragged in both directions, and one has more tiles than workgroups that
can be resident at once, so that each workgroup steps several tiles between
two barriers.
"""
import numpy as np
import pytest

from paper_2403_16122_amd import workloads as W

pytestmark = pytest.mark.gpu


def _lbm():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_16122_amd import lbm

    return lbm


def pair(lbm, p, phi0, T0, storage, xcd):
    out = []
    for _ in range(2):
        s = lbm.Solver(dict(p, storage=lbm.STORAGE[storage]), phi0, T0)
        s.set_launch("64x8", xcd)
        out.append(s)
    return out


def droplet(nx, ny, seed=3):
    p = W.default_params(nx, ny, rho_s=0.9, theta_bottom_deg=70.0)
    phi0 = W.sessile_droplet(nx, ny, 0.14 * nx, 70.0, 4.0, x0=0.503 * nx)
    T0 = W.temperature_noise(nx, ny, p["T_melt"], 1e-3, seed)
    return p, phi0, T0


BARRIERS = ["flat", "per_xcd"]


@pytest.mark.parametrize("barrier", BARRIERS)
@pytest.mark.parametrize("storage", ["fp32", "fp16", "bf16"])
@pytest.mark.parametrize("xcd", [0, 1, 2])
def test_persistent_steps_bitwise_equal_per_step_launches(storage, xcd, barrier):
    lbm = _lbm()
    p, phi0, T0 = droplet(100, 37)
    print(f"persistent storage={storage} xcd={xcd} barrier={barrier} grid=100x37", flush=True)
    a, b = pair(lbm, p, phi0, T0, storage, xcd)
    a.step(41)
    wg = b.step_persistent(17, barrier)  # odd and even counts, and calls that continue a run
    b.step_persistent(24, barrier)
    assert b.step_count == a.step_count == 41
    ntx, nty = 2, 5  # 64x8 tiles over 100x37, the last column and row ragged
    order = {0: ntx * nty, 1: 8 * -(-(ntx * nty) // 8), 2: 8 * -(-ntx // 8) * nty}
    assert wg == order[xcd]  # every workgroup of the tile order fits at once
    assert b.save() == a.save()


@pytest.mark.parametrize("barrier", BARRIERS)
@pytest.mark.parametrize("xcd", [0, 1, 2])
def test_persistent_on_a_grid_narrower_than_a_tile(xcd, barrier):
    """40 columns under 64-wide tiles: every tile is ragged, and tile order
    2 deals padding workgroups that take no tile."""
    lbm = _lbm()
    p, phi0, T0 = droplet(40, 230)
    print(f"persistent grid=40x230 xcd={xcd} barrier={barrier}", flush=True)
    a, b = pair(lbm, p, phi0, T0, "fp16", xcd)
    a.step(21)
    b.step_persistent(21, barrier)
    assert b.save() == a.save()


@pytest.mark.parametrize("barrier", BARRIERS)
@pytest.mark.parametrize("xcd", [0, 1, 2])
def test_persistent_grid_strides_over_more_tiles_than_resident_workgroups(xcd, barrier):
    lbm = _lbm()
    p, phi0, T0 = droplet(1100, 530)
    ntiles = ((1100 + 63) // 64) * ((530 + 7) // 8)
    print(f"persistent grid=1100x530 tiles={ntiles} xcd={xcd} barrier={barrier}", flush=True)
    a, b = pair(lbm, p, phi0, T0, "fp32", xcd)
    a.step(12)
    wg = b.step_persistent(12, barrier)
    print(f"workgroups={wg}", flush=True)
    assert wg % 8 == 0 and wg < ntiles
    assert b.save() == a.save()


def test_persistent_mixes_with_per_step_launches_and_counts_steps():
    lbm = _lbm()
    p, phi0, T0, _ = W.workload("sessile128", seed=1)
    a, b = pair(lbm, p, phi0, T0, "fp16", 2)
    a.step(30)
    b.step_persistent(0)  # no-op
    b.step_persistent(1, "per_xcd")  # a single step: no barrier
    b.step(10)
    b.step_persistent(7, "per_xcd")
    b.step_persistent(12)
    assert b.step_count == 30
    assert b.save() == a.save()
    for bad in ((-1, 0, 0), (lbm.PERSIST_MAX_STEPS + 1, 0, 0), (5, 2, 0), (5, -1, 0), (5, 0, -1)):
        with pytest.raises(lbm.LbmError):
            b._check(b.L.lbm_step_persistent(b._h, bad[0], bad[1], bad[2], None), "lbm_step_persistent")
    assert b.step_count == 30


@pytest.mark.parametrize("barrier", BARRIERS)
def test_a_barrier_wait_that_runs_out_is_reported_and_every_wave_leaves(barrier):
    """The failure path, forced from the host: on 1100x530 (1206 tiles over
    512 workgroups, so some step three tiles and the others two) the
    two-tile workgroups wait several microseconds for the rest at the first
    barrier, longer than a bound of 1 us.  The first wait to run out sets
    the flag, every workgroup stops waiting and leaves, and the call
    returns LBM_EDEVICE with the reason; the device then runs the same
    steps normally."""
    lbm = _lbm()
    p, phi0, T0 = droplet(1100, 530)
    print(f"forced barrier time-out barrier={barrier}", flush=True)
    a, b = pair(lbm, p, phi0, T0, "fp32", 2)
    with pytest.raises(lbm.LbmError) as err:
        b.step_persistent(4, barrier, wait_limit_us=1)
    assert err.value.code == lbm.LBM_EDEVICE and "timed out" in str(err.value)
    assert b.step_count == 0  # the failed call does not count its steps
    a.step(4)
    c = lbm.Solver(dict(p, storage=lbm.STORAGE["fp32"]), phi0, T0)
    c.set_launch("64x8", 2)
    c.step_persistent(4, barrier)
    assert c.save() == a.save()


@pytest.mark.parametrize("barrier", BARRIERS)
def test_persistent_run_against_the_oracle(oracle_mod, barrier):
    """The 128x64 sessile droplet after 1000 steps in one launch, held to the
    FP32 bounds of the per-step path: max|d phi|, max|d T| <= 1e-5 and a
    relative L2 of u <= 1e-4."""
    lbm = _lbm()
    p, phi0, T0, _ = W.workload("sessile128", seed=0)
    g = lbm.Solver(p, phi0, T0)
    g.set_launch("64x8", 2)
    g.step_persistent(1000, barrier)
    o = oracle_mod.OracleSolver(p, phi0, T0)
    o.step(1000)
    fg, fo = g.fields(("phi", "T", "ux", "uy")), o.fields(("phi", "T", "ux", "uy"))
    dphi = float(np.abs(fg["phi"] - fo["phi"]).max())
    dT = float(np.abs(fg["T"] - fo["T"]).max())
    ug, uo = np.stack([fg["ux"], fg["uy"]]), np.stack([fo["ux"], fo["uy"]])
    eu = float(np.linalg.norm(ug - uo) / np.linalg.norm(uo))
    print(f"persistent 1000 steps: max|dphi|={dphi:.3e} max|dT|={dT:.3e} relL2(u)={eu:.3e}", flush=True)
    assert dphi <= 1e-5 and dT <= 1e-5 and eu <= 1e-4
