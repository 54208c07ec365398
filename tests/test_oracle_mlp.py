"""Pins of the FP64 surrogate reference (oracle/mlp.py): its analytic
gradient against central finite differences of its own loss (an independent
route to the same numbers), closed forms for special weights, the GELU
against its definition, BF16 rounding against FP32 bit patterns, and Adam's
first step."""
import math

import numpy as np
import pytest

from oracle import mlp as M


def data(n=7, seed=0):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(n, M.IN))
    t = rng.normal(size=(n, M.OUT))
    mask = (rng.uniform(size=(n, M.OUT)) > 0.2).astype(float)
    return x, t, mask


def test_gradient_matches_finite_differences():
    flat = M.init(3) * 0.5 + 0.01 * np.random.default_rng(4).normal(size=M.NPARAM)
    x, t, mask = data()
    w = np.array([1.0, 0.5, 2.0])
    L, g = M.loss_and_grad(flat, x, t, mask, w)
    rng = np.random.default_rng(5)
    idx = np.concatenate([rng.choice(M.NPARAM, 40, replace=False), [M.NPARAM - 1, M.NPARAM - 4, 640, 767]])
    h = 1e-6
    for i in idx:
        e = np.zeros(M.NPARAM)
        e[i] = h
        fd = (M.loss(flat + e, x, t, mask, w) - M.loss(flat - e, x, t, mask, w)) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-9), i


def test_zero_hidden_weights_give_the_output_bias():
    p = M.unpack(M.init(1))
    p["W3"][:] = 0.0
    p["b3"][:] = [1.5, -2.0, 0.25]
    y, _ = M.forward(M.pack(p), np.random.default_rng(0).normal(size=(4, M.IN)))
    assert np.array_equal(y, np.tile([1.5, -2.0, 0.25], (4, 1)))


def test_gelu_against_its_definition():
    for z in (-3.0, -0.5, 0.0, 0.7, 2.5):
        Phi = 0.5 * (1 + math.erf(z / math.sqrt(2)))
        assert M.gelu(np.array(z)) == pytest.approx(z * Phi, abs=1e-15)
        d = (M.gelu(np.array(z + 1e-6)) - M.gelu(np.array(z - 1e-6))) / 2e-6
        assert M.gelu_prime(np.array(z)) == pytest.approx(d, rel=1e-7, abs=1e-9)


def test_bf16_rounding():
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: to even gives 1; 1 + 3*2^-8 rounds up
    assert M.bf16(np.array([1 + 2 ** -8]))[0] == 1.0
    assert M.bf16(np.array([1 + 3 * 2 ** -8]))[0] == 1 + 2 ** -6
    assert M.bf16(np.array([-1.0 - 2 ** -7]))[0] == -1.0 - 2 ** -7
    a = np.random.default_rng(0).normal(size=1000)
    assert np.all(np.abs(M.bf16(a) - a) <= np.abs(a) * 2 ** -8 * (1 + 1e-6))  # unit roundoff of an 8-bit significand


def test_masked_targets_do_not_contribute():
    flat = M.init(2)
    x, t, mask = data(5, 1)
    L1, g1 = M.loss_and_grad(flat, x, t, mask, [1, 1, 1])
    t2 = t.copy()
    t2[mask == 0] += 100.0
    L2, g2 = M.loss_and_grad(flat, x, t2, mask, [1, 1, 1])
    assert L1 == pytest.approx(L2, rel=1e-14) and np.allclose(g1, g2, rtol=1e-12, atol=0)


def test_adam_first_step_moves_each_parameter_by_lr():
    flat = np.zeros(5)
    g = np.array([1.0, -2.0, 0.5, 1e-3, -4.0])
    new, m, v = M.adam(flat, g, np.zeros(5), np.zeros(5), 1, 0.01, eps=0.0)
    assert np.allclose(new, -0.01 * np.sign(g), rtol=1e-12)
