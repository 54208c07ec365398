"""The learned surrogate against the solver on held-out sweep droplets.

Training data (paper_2403_16122_amd/data) are 4096 droplets of the sweep run
to freezing by the batched solver (seed 1); the 512 held-out droplets are
seed 2.  The surrogate must predict t*, height/R and tip angle of held-out
droplets to the accuracy below, orders of magnitude faster than the solver,
and the droplets it sends back to the solver must get exactly the solver's
values.
"""
import os

import numpy as np
import pytest

from paper_2403_16122_amd import workloads as W

pytestmark = pytest.mark.gpu

# The stored sweep records against a fresh run of the batched solver: the
# records are written by paper_2403_16122_amd/sweep_data.py with the kernels
# of this build, so they are equal bit for bit (a kernel change that moves the
# FP32 rounding moves t* of these droplets by ~1e-5 and calls for writing them
# again).
STORED_REL = 1e-12

DATA = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2403_16122_amd", "data")


def _mods():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_16122_amd import surrogate as S

    return S


@pytest.fixture(scope="module")
def fitted():
    S = _mods()
    tr = S.load_training(DATA)
    te = S.load(os.path.join(DATA, "sweep_test.npz"))
    sur = S.Surrogate(ensemble=8, seed=0, fallback_rel=0.02)
    sur.fit(tr)
    return S, sur, te


def test_held_out_accuracy_and_inference_time(fitted):
    S, sur, te = fitted
    ev = S.evaluate(sur, te)
    print({k: (round(v, 5) if isinstance(v, float) else v) for k, v in ev.items()}, flush=True)
    assert ev["t_star_rel_err_median"] <= 0.02
    assert ev["t_star_rel_err_p90"] <= 0.05
    assert ev["height_R_abs_err_median"] <= 0.01
    assert ev["tip_angle_abs_err_median"] <= 3.0
    assert ev["inference_seconds"] < 0.05  # all 512 droplets


def test_error_model_ranks_errors_and_holds_the_2pct_threshold(fitted):
    """The error model (trained on out-of-fold errors, scaled on the
    calibration tenth) ranks the actual t* errors -- on the calibration
    droplets it was scaled on and on the held-out droplets -- far better
    than the ensemble's spread, and at the 2 % threshold the droplets it
    accepts keep their errors within it at the 95th percentile, while it
    accepts enough of them to save solver time.  Measured on MI355X: rank
    correlation 0.43 (calibration) and 0.36 (held out) against 0.06 for the
    spread; 31 % accepted, accepted error median 0.42 %, 95th percentile
    1.71 %."""
    S, sur, te = fitted
    ev = S.evaluate(sur, te)
    print({k: (round(v, 5) if isinstance(v, float) else v) for k, v in ev.items()}, flush=True)
    assert ev["error_model_spearman_calibration"] > 0.3
    assert ev["error_model_spearman"] > 0.3
    assert ev["error_model_spearman"] > ev["spread_spearman"] + 0.15
    assert ev["acceptance"] >= 0.15
    assert ev["accepted_t_star_rel_err_p95"] <= 0.025
    assert ev["accepted_t_star_rel_err_median"] <= 0.01
    assert ev["with_fallback_t_star_rel_err_p90"] <= 0.01


def test_fallback_reproduces_the_solver_and_speed_gain(fitted):
    S, sur, te = fitted
    drops = W.sweep_droplets(512, seed=2, storage=1)
    x = np.array([[d["R"], d["theta"], d["ste"], d["gamma"], len(d["bubbles"])] for d in drops])
    assert np.allclose(x, S.features(te))  # the stored held-out droplets are these
    # bound the test's solver time: keep the shortest-running dozen droplets
    order = np.argsort(te["t_freeze"])[:12]
    sub = [drops[i] for i in order]
    sur_all = S.Surrogate(**{k: getattr(sur, k) for k in ("ensemble", "seed", "calib_frac", "coverage")},
                          fallback_rel=0.0)  # everything falls back
    for k in ("net", "err_net", "xm", "xs", "ym", "ys", "em", "es", "err_scale"):
        setattr(sur_all, k, getattr(sur, k))
    out, fb, t = S.predict_with_fallback(sur_all, sub)
    assert fb.all() and t["solver_droplets"] == len(sub)
    # the batched solver on its own gives the same values, bit for bit
    from paper_2403_16122_amd import lbm

    b = lbm.Batch([d["params"] for d in sub], [d["phi0"] for d in sub], [d["T0"] for d in sub],
                  radii=[d["R"] for d in sub], slots=5)
    b.configure(sample_every=200, max_steps=3_000_000)
    b.step(30_000_000, until_frozen=True)
    for j, (i, r) in enumerate(zip(order, b.results())):
        assert out["t_star"][j] == r["t_star"] and out["height_R"][j] == r["height"] / sub[j]["R"]
        # and the stored held-out records, written by the same batched solver
        assert out["t_star"][j] == pytest.approx(te["t_star"][i], rel=STORED_REL)
        assert out["height_R"][j] == pytest.approx(te["height_R"][i], rel=STORED_REL)
    import time

    import torch

    per_solver = t["solver_seconds"] / len(sub)
    sur.predict(x[order])  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sur.predict(x[order])
    torch.cuda.synchronize()
    per_net = (time.perf_counter() - t0) / len(sub)
    print(f"solver {per_solver:.3f} s/droplet (batched, the 12 shortest runs); network {per_net:.2e} s/droplet",
          flush=True)
    assert per_solver / per_net > 100.0
