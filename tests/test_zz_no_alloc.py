"""The allocation-free forward pass of the surrogate network
(lbm_mlp_forward_noalloc) against the handle's forward pass
(lbm_mlp_forward) with the same parameters: bit-equal outputs on two calls
in a row, the second with fewer samples and members, and the limits of the
library's static buffer refused."""
import ctypes as C

import numpy as np
import pytest

from paper_2403_16122_amd import lbm

pytestmark = pytest.mark.gpu


def _params(E, P, seed):
    """Parameters of E members with non-trivial biases (He-like scale)."""
    rng = np.random.default_rng(seed)
    return (rng.standard_normal((E, P)) * 0.2).astype(np.float32)


def _inputs(n, seed):
    return np.random.default_rng(seed).uniform(-1.5, 1.5, (n, 5)).astype(np.float32)


def _check_against_handle(E, n, seed):
    import torch

    m = lbm.MLP(ensemble=E, seed=seed, max_batch=max(n, 64))
    prm = _params(E, m.P, seed)
    m.set_params(prm)
    x = torch.as_tensor(_inputs(n, seed + 100), device="cuda")
    y_ref = m.forward(x)
    y = torch.full((E, n, 3), float("nan"), dtype=torch.float32, device="cuda")
    d_prm = torch.as_tensor(prm, device="cuda")
    lbm.mlp_forward_noalloc(d_prm, x, y)
    torch.cuda.synchronize()
    print(f"noalloc forward: E={E} n={n} max|dy|={float((y - y_ref).abs().max()):.3e}", flush=True)
    assert torch.isfinite(y).all()
    assert torch.equal(y, y_ref), float((y - y_ref).abs().max())


def test_noalloc_forward_equals_handle_forward_on_two_calls():
    _check_against_handle(E=5, n=700, seed=3)   # several workgroups, a ragged tail
    _check_against_handle(E=2, n=37, seed=4)    # then a smaller call over the same buffer


def test_noalloc_forward_refuses_sizes_beyond_its_buffer():
    import torch

    L = lbm.load_library()
    P = int(L.lbm_mlp_param_count())
    E = lbm.MLP_NOALLOC_MAX_ENSEMBLE + 1
    prm = torch.zeros((E, P), dtype=torch.float32, device="cuda")
    x = torch.zeros((4, 5), dtype=torch.float32, device="cuda")
    y = torch.zeros((E, 4, 3), dtype=torch.float32, device="cuda")
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = L.lbm_mlp_forward_noalloc(C.c_void_p(prm.data_ptr()), E, C.c_void_p(x.data_ptr()), 4,
                                   C.c_void_p(y.data_ptr()), st)
    assert rc == lbm.LBM_EINVAL
    assert b"static buffer" in L.lbm_mlp_last_error()
    rc = L.lbm_mlp_forward_noalloc(C.c_void_p(prm.data_ptr()), 1, C.c_void_p(x.data_ptr()), 0,
                                   C.c_void_p(y.data_ptr()), st)
    assert rc == lbm.LBM_EINVAL
    assert L.lbm_mlp_forward_noalloc(None, 1, C.c_void_p(x.data_ptr()), 4, C.c_void_p(y.data_ptr()), st) \
        == lbm.LBM_EINVAL
    torch.cuda.synchronize()
