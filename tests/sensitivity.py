"""The method's own sensitivity, measured on the oracle (test helper).

The phase-field step amplifies small perturbations where the order parameter
develops dips in frozen rows (the sharpening flux lambda*n has no direction
at an extremum), so long runs of two correct implementations that round
differently part there.  The tests bound the GPU against the oracle by how
far the oracle moves from itself under perturbations of the size FP32
rounding makes.
"""
import numpy as np

W9 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def perturbed_every_step(oracle_mod, p, phi0, T0, steps, eps, seed):
    """The oracle with phi at every node moved by eps * N(0, 1) after every
    step (added to the g populations as w_i * delta, the split of a change
    of phi over populations at rest): a model of an implementation that
    rounds in every step, as FP32 arithmetic does.  The saved state is four
    int64 header words followed by the nine g planes."""
    n = p["nx"] * p["ny"]
    rng = np.random.default_rng(seed)
    o = oracle_mod.OracleSolver(p, phi0, T0)
    for _ in range(steps):
        o.step(1)
        blob = bytearray(o.save())
        g = np.frombuffer(blob, dtype=np.float64, count=9 * n, offset=32).reshape(9, n)
        g = g + W9[:, None] * (eps * rng.standard_normal(n))[None, :]
        blob[32:32 + 9 * n * 8] = g.tobytes()
        o.load(bytes(blob))
    return o
