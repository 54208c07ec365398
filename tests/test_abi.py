"""CPU checks of the C ABI: the library loads, exports every function that
include/lbm.h declares, and validates parameters without touching a GPU."""
import os
import re

import pytest

from paper_2403_16122_amd import lbm, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "lbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(lbm_[a-z_]+)\s*\(", src, flags=re.M)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("lbm_init", "lbm_step", "lbm_fields", "lbm_diag", "lbm_save", "lbm_load", "lbm_destroy"):
        assert n in names
    assert sorted(lbm.EXPORTED) == names


def test_library_exports_every_declared_symbol():
    L = lbm.load_library()
    for n in declared_functions():
        assert hasattr(L, n), n


def test_workspace_size_and_validation():
    p = W.default_params(128, 64)
    n = lbm.workspace_bytes(p)
    plane = (128 * 64 + 63) // 64 * 64
    assert n >= (2 * 27 + 8 + 10) * plane * 4
    for over in (dict(nx=2), dict(M=-1.0), dict(mu_l=0.0), dict(theta_bottom_deg=180.0),
                 dict(latent=0.0), dict(storage=7), dict(k_g=float("inf"))):
        q = dict(p, **over)
        with pytest.raises(lbm.LbmError) as e:
            lbm.workspace_bytes(q)
        assert e.value.code == lbm.LBM_EINVAL


def test_workspace_shrinks_with_16bit_storage():
    p = W.default_params(128, 64)
    plane = (128 * 64 + 63) // 64 * 64
    n32 = lbm.workspace_bytes(p)
    for name in ("fp16", "bf16"):
        n16 = lbm.workspace_bytes(dict(p, storage=lbm.STORAGE[name]))
        assert n32 - n16 == 2 * 27 * plane * 2  # both population buffers halve


def test_strerror_names_every_code():
    L = lbm.load_library()
    for code in (0, -1, -2, -3, -4, -5):
        assert L.lbm_strerror(code).decode() != "unknown error"


def test_batch_workspace_validation():
    """The batch's sizing call validates every droplet on the host: an empty
    batch, slot counts outside 1..65535, mixed storage formats and one
    invalid droplet are refused; the workspace grows with the number of
    droplets resident at once (slots), not with the queue behind them."""
    small = [W.default_params(24 + 4 * i, 18 + 2 * i) for i in range(6)]
    with pytest.raises(lbm.LbmError) as e:
        lbm.batch_workspace_bytes([], 4)
    assert e.value.code == lbm.LBM_EINVAL
    for slots in (0, 65536):
        with pytest.raises(lbm.LbmError) as e:
            lbm.batch_workspace_bytes(small, slots)
        assert e.value.code == lbm.LBM_EINVAL
    for bad in (dict(storage=lbm.STORAGE["fp16"]), dict(nx=2), dict(M=0.0)):
        with pytest.raises(lbm.LbmError) as e:
            lbm.batch_workspace_bytes(small[:3] + [dict(small[3], **bad)] + small[4:], 6)
        assert e.value.code == lbm.LBM_EINVAL, bad
    full = lbm.batch_workspace_bytes(small, 6)
    two = lbm.batch_workspace_bytes(small, 2)
    assert 0 < two < full
    assert lbm.batch_workspace_bytes(small, 6) == lbm.batch_workspace_bytes(small, 600)  # slots capped at n
    one = lbm.batch_workspace_bytes(small[:1], 1)
    assert one < two


def test_batch_refuses_a_wide_temperature_span_before_any_device_call():
    """16-bit storage keeps T - T_m per node as an FP16 reference; a batch
    whose droplet exceeds that span is refused by lbm_batch_init itself,
    before it creates a stream or touches the workspace (both NULL here)."""
    import ctypes as C

    import numpy as np

    L = lbm.load_library()
    nx, ny = 16, 12
    p = dict(W.default_params(nx, ny), storage=lbm.STORAGE["fp16"])
    phi = np.zeros(nx * ny)
    T = np.full(nx * ny, p["T_melt"] + 5.0e4)
    params = (lbm.Params * 1)(lbm.make_params(p))
    pa = (C.POINTER(C.c_double) * 1)(lbm._dptr(phi))
    ta = (C.POINTER(C.c_double) * 1)(lbm._dptr(T))
    h = C.c_void_p()
    rc = L.lbm_batch_init(params, 1, pa, ta, None, 1, None, 0, None, C.byref(h))
    assert rc == lbm.LBM_EINVAL and not h.value
    assert "temperature span" in L.lbm_batch_last_error().decode()


def test_largest_grid_keeps_a_buffer_below_4_GiB():
    """Kernels address a buffer by a 32-bit byte offset: the 27 FP32
    population planes (108 B per node) must span less than 2^32 bytes, the
    16-bit ones (54 B per node) too, and so must the 10 output-field planes."""
    ny = 16
    nx_max = ((1 << 32) - 1) // 108 // 64 * 64 // ny  # 39,768,192 nodes
    ok = W.default_params(nx_max, ny)
    assert lbm.workspace_bytes(ok) > 0
    with pytest.raises(lbm.LbmError) as e:
        lbm.workspace_bytes(dict(ok, nx=nx_max + 4))  # one more 64-node plane block
    assert e.value.code == lbm.LBM_EINVAL
    half = dict(W.default_params(2 * nx_max, ny), storage=lbm.STORAGE["fp16"])
    assert lbm.workspace_bytes(half) > 0  # 16-bit populations take twice the nodes
    with pytest.raises(lbm.LbmError):
        lbm.workspace_bytes(dict(half, storage=lbm.STORAGE["fp32"]))
