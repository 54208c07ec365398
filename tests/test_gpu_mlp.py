"""Surrogate network kernels (BF16 matrix cores, FP32 accumulation) against
the FP64 reference (oracle/mlp.py), through the C ABI.

Two references:
* the same arithmetic with BF16 rounding at the points where the kernels
  feed the matrix cores: the GPU differs by FP32 summation order (~1e-7)
  and, rarely, by an activation whose FP32 value sits on a BF16 rounding
  boundary and rounds the other way, moving one of the 128 terms of an
  output by 2^-8 of itself; outputs agree within 5e-4 of their magnitude
  sum sum_k |W3_jk h2_k| + |b3_j|, losses and gradients to ~1e-4;
* plain FP64: the GPU differs by the BF16 roundings themselves.  Each
  rounding is within 2^-8 relative; about five of them lie on any path
  from inputs to a gradient, so the relative L2 error stays below 3e-2.
"""
import numpy as np
import pytest

from oracle import mlp as M

pytestmark = pytest.mark.gpu


def _lbm():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_16122_amd import lbm

    return lbm


def problem(n, E, seed):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(n, M.IN)).astype(np.float32)
    t = rng.normal(size=(n, M.OUT)).astype(np.float32)
    mask = (rng.uniform(size=(n, M.OUT)) > 0.2).astype(np.float32)
    P = []
    for e in range(E):
        p = M.unpack(M.init(100 * seed + e))
        for b in ("b1", "b2", "b3"):
            p[b] = rng.normal(scale=0.1, size=p[b].shape)
        P.append(M.pack(p))
    return x, t, mask, np.array(P, dtype=np.float32)


def relL2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("n", [1, 37, 200, 1000])
def test_forward_matches_reference(n):
    lbm = _lbm()
    x, _, _, P = problem(n, 2, seed=n)
    net = lbm.MLP(ensemble=2, max_batch=1024)
    net.set_params(P)
    y = net.forward(x).cpu().numpy()
    for e in range(2):
        p64 = P[e].astype(np.float64)
        yb, (_, _, _, _, h2) = M.forward(p64, x, bf=True)
        scale = np.abs(M.bf16(h2)) @ np.abs(M.bf16(M.unpack(p64)["W3"])).T + np.abs(M.unpack(p64)["b3"])
        err = np.abs(y[e] - yb)
        print(f"n={n} member {e}: max |y - y_bf16ref| / scale = {np.max(err / scale):.2e}, "
              f"relL2 vs FP64 {relL2(y[e], M.forward(p64, x)[0]):.2e}", flush=True)
        assert np.all(err <= 5e-4 * scale)
        assert relL2(y[e], M.forward(p64, x)[0]) <= 3e-2


@pytest.mark.parametrize("n", [37, 1000])
def test_gradient_matches_reference(n):
    lbm = _lbm()
    x, t, mask, P = problem(n, 2, seed=7 + n)
    w = np.array([1.0, 0.5, 2.0], dtype=np.float32)
    net = lbm.MLP(ensemble=2, max_batch=1024)
    net.set_params(P)
    loss, g = net.gradient(x, t, mask, w)
    for e in range(2):
        p64 = P[e].astype(np.float64)
        Lb, gb = M.loss_and_grad(p64, x, t, mask, w, bf=True)
        L64, g64 = M.loss_and_grad(p64, x, t, mask, w)
        blocks = {}
        o = 0
        for name, shape in M.SHAPES:
            k = int(np.prod(shape))
            blocks[name] = (relL2(g[e][o:o + k], gb[o:o + k]), relL2(g[e][o:o + k], g64[o:o + k]))
            o += k
        print(f"n={n} member {e}: loss {loss[e]:.6e} ref {Lb:.6e}; per-block relL2 (bf16 ref, fp64 ref) {blocks}",
              flush=True)
        assert loss[e] == pytest.approx(Lb, rel=1e-4)
        assert loss[e] == pytest.approx(L64, rel=3e-2)
        for name, (eb, e64) in blocks.items():
            assert eb <= 1e-3, (name, eb)
            assert e64 <= 3e-2, (name, e64)


def test_adam_step_matches_reference():
    lbm = _lbm()
    x, t, mask, P = problem(300, 2, seed=3)
    net = lbm.MLP(ensemble=2, max_batch=512)
    net.set_params(P)
    _, g = net.gradient(x, t, mask)
    net.train(x, t, mask, steps=1, lr=1e-3)
    P1 = net.get_params()
    for e in range(2):
        ref, _, _ = M.adam(P[e].astype(np.float64), g[e].astype(np.float64), np.zeros(M.NPARAM), np.zeros(M.NPARAM),
                           1, 1e-3)
        assert np.max(np.abs(P1[e] - ref)) <= 2e-6


def test_training_reduces_the_loss_and_members_differ():
    lbm = _lbm()
    rng = np.random.default_rng(11)
    n = 2048
    x = rng.uniform(-1, 1, size=(n, M.IN)).astype(np.float32)
    t = np.stack([np.sin(2 * x[:, 0]) + 0.5 * x[:, 1] * x[:, 2], np.cos(x[:, 3]) - x[:, 4] ** 2,
                  x[:, 0] * x[:, 4]], axis=1).astype(np.float32)
    mask = np.ones_like(t)
    net = lbm.MLP(ensemble=4, seed=5, max_batch=n)
    l0 = net.train(x, t, mask, steps=1, lr=3e-3)
    l1 = net.train(x, t, mask, steps=400, lr=3e-3)
    print(f"loss {l0} -> {l1}", flush=True)
    assert np.all(l1 < 0.1 * l0)
    y = net.forward(x).cpu().numpy()
    assert np.std(y, axis=0).mean() > 0.0  # independent initialisations
