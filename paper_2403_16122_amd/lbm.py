"""Thin ctypes binding of ``liblbm.so`` (include/lbm.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  PyTorch provides the device workspace and the stream.  There
is no CPU fallback: importing the binding without the built library, or
creating a solver without a GPU, raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Iterable, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

FIELD_BITS = {"phi": 0, "T": 1, "ux": 2, "uy": 3, "p": 4, "fs": 5, "fl": 6, "rho": 7, "H": 8, "mdot": 9}
TILE_VARIANTS = {"64x4": 0, "32x8": 1, "64x8": 2, "64x16": 3, "128x4": 4,
                 "unfused64x8": 5,  # two-kernel step, kept to measure the gain from fusion
                 "two64x8": 6, "two32x8": 7, "two32x16": 8,  # two steps per launch (FP32 storage)
                 "two32x16w": 9, "two32x8w": 10}  # the same with two and three lanes per tile node
XCD_MODES = (0, 1, 2)  # row-major tiles; one row-major band per XCD; one column band per XCD
TILE_NAMES = {v: k for k, v in TILE_VARIANTS.items()}
TWO_STEP_VARIANTS = ("two64x8", "two32x8", "two32x16", "two32x16w", "two32x8w")
TWO_STEP_ANY_STORAGE = ("two32x16w", "two32x8w")  # the others: FP32 storage only (lbm_set_launch refuses them)
STORAGE = {"fp32": 0, "fp16": 1, "bf16": 2}
STORE_MODES = {"auto": 0, "cached": 1, "streaming": 2}  # lbm_set_store_mode  # LBM_STORE_FP32 / _FP16_SHIFT / _BF16_SHIFT

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_ENONFINITE, LBM_ESTATE = 0, -1, -2, -3, -4, -5

EXPORTED = [
    "lbm_workspace_bytes", "lbm_init", "lbm_step", "lbm_step_persistent", "lbm_fields", "lbm_fields_device",
    "lbm_diag", "lbm_pops", "lbm_state_bytes", "lbm_save", "lbm_load", "lbm_step_count", "lbm_sync",
    "lbm_destroy", "lbm_strerror", "lbm_last_error", "lbm_set_launch", "lbm_set_store_mode", "lbm_autotune",
    "lbm_batch_workspace_bytes", "lbm_batch_init", "lbm_batch_configure", "lbm_batch_set_launch",
    "lbm_batch_autotune", "lbm_batch_set_store_mode", "lbm_batch_step", "lbm_batch_results", "lbm_batch_fields",
    "lbm_batch_last_error", "lbm_batch_destroy", "lbm_shape_of",
    "lbm_mlp_param_count", "lbm_mlp_create", "lbm_mlp_set_params", "lbm_mlp_get_params", "lbm_mlp_forward",
    "lbm_mlp_gradient", "lbm_mlp_train", "lbm_mlp_last_error", "lbm_mlp_destroy", "lbm_mlp_forward_noalloc",
]
PERSIST_MAX_STEPS = 1000000  # LBM_PERSIST_MAX_STEPS
PERSIST_BARRIERS = {"flat": 0, "per_xcd": 1}  # LBM_BARRIER_FLAT / LBM_BARRIER_PER_XCD
INTERVAL_PERSIST = {"flat": 2, "per_xcd": 3}  # LBM_INTERVAL_PERSIST_FLAT / _PER_XCD
DROP_STATUS = {0: "queued", 1: "running", 2: "frozen", 3: "limit", 4: "nonfinite"}


class LbmError(RuntimeError):
    def __init__(self, code: int, what: str, detail: str = ""):
        self.code = code
        super().__init__(f"{what} failed: {code} ({detail})")


class Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32),
        ("W", C.c_double), ("M", C.c_double), ("sigma", C.c_double),
        ("rho_l", C.c_double), ("rho_g", C.c_double), ("rho_s", C.c_double),
        ("mu_l", C.c_double), ("mu_g", C.c_double), ("mu_s", C.c_double),
        ("cp_l", C.c_double), ("cp_g", C.c_double), ("cp_s", C.c_double), ("cp_ref", C.c_double),
        ("k_l", C.c_double), ("k_g", C.c_double), ("k_s", C.c_double),
        ("latent", C.c_double), ("T_melt", C.c_double), ("T_bottom", C.c_double),
        ("theta_bottom_deg", C.c_double), ("theta_top_deg", C.c_double),
        ("gx", C.c_double), ("gy", C.c_double),
        ("bq_beta", C.c_double), ("bq_rho0", C.c_double), ("bq_Tref", C.c_double),
        ("st_solid_mask", C.c_int32), ("storage", C.c_int32),
    ]


class Diag(C.Structure):
    _fields_ = [
        ("step", C.c_int64), ("sum_phi", C.c_double), ("sum_phic", C.c_double),
        ("sum_solid", C.c_double), ("sum_liquid", C.c_double), ("sum_H", C.c_double),
        ("max_u", C.c_double), ("h_c", C.c_double), ("nonfinite", C.c_int32),
    ]


class DropResult(C.Structure):
    _fields_ = [
        ("status", C.c_int32), ("slot", C.c_int32), ("steps", C.c_int64), ("t_freeze", C.c_double),
        ("t_star", C.c_double), ("liquid0", C.c_double), ("liquid", C.c_double), ("height", C.c_double),
        ("base_radius", C.c_double), ("tip_angle_deg", C.c_double),
    ]


_lib = None


def load_library():
    """Load the in-tree gfx950 library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it first (python -m paper_2403_16122_amd.build)")
    L = C.CDLL(LIB_PATH)
    vp, dp = C.c_void_p, C.POINTER(C.c_double)
    L.lbm_workspace_bytes.argtypes = [C.POINTER(Params), C.POINTER(C.c_size_t)]
    L.lbm_init.argtypes = [C.POINTER(Params), dp, dp, vp, C.c_size_t, vp, C.POINTER(vp)]
    L.lbm_step.argtypes = [vp, C.c_int32]
    L.lbm_step_persistent.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_int32)]
    L.lbm_fields.argtypes = [vp, C.c_uint32, C.POINTER(dp)]
    L.lbm_fields_device.argtypes = [vp, C.c_uint32, C.POINTER(vp)]
    L.lbm_diag.argtypes = [vp, C.POINTER(Diag)]
    L.lbm_pops.argtypes = [vp, C.c_int32, dp]
    L.lbm_state_bytes.argtypes = [vp]
    L.lbm_state_bytes.restype = C.c_size_t
    L.lbm_save.argtypes = [vp, vp, C.c_size_t]
    L.lbm_load.argtypes = [vp, vp, C.c_size_t]
    L.lbm_step_count.argtypes = [vp]
    L.lbm_step_count.restype = C.c_int64
    L.lbm_sync.argtypes = [vp]
    L.lbm_destroy.argtypes = [vp]
    L.lbm_destroy.restype = None
    L.lbm_strerror.argtypes = [C.c_int]
    L.lbm_strerror.restype = C.c_char_p
    L.lbm_last_error.argtypes = []
    L.lbm_last_error.restype = C.c_char_p
    L.lbm_set_launch.argtypes = [vp, C.c_int32, C.c_int32]
    L.lbm_set_store_mode.argtypes = [vp, C.c_int32]
    L.lbm_autotune.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    L.lbm_batch_workspace_bytes.argtypes = [C.POINTER(Params), C.c_int32, C.c_int32, C.POINTER(C.c_size_t)]
    L.lbm_batch_init.argtypes = [C.POINTER(Params), C.c_int32, C.POINTER(dp), C.POINTER(dp), dp, C.c_int32, vp,
                                 C.c_size_t, vp, C.POINTER(vp)]
    L.lbm_batch_configure.argtypes = [vp, C.c_int32, C.c_int64, C.c_double, C.c_int32, C.c_int32]
    L.lbm_batch_set_launch.argtypes = [vp, C.c_int32, C.c_int32]
    L.lbm_batch_set_store_mode.argtypes = [vp, C.c_int32]
    L.lbm_batch_autotune.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    L.lbm_batch_step.argtypes = [vp, C.c_int64, C.c_int32]
    L.lbm_batch_results.argtypes = [vp, C.POINTER(DropResult)]
    L.lbm_batch_fields.argtypes = [vp, C.c_int32, C.c_uint32, C.POINTER(dp)]
    L.lbm_batch_last_error.argtypes = []
    L.lbm_batch_last_error.restype = C.c_char_p
    L.lbm_batch_destroy.argtypes = [vp]
    L.lbm_batch_destroy.restype = None
    L.lbm_shape_of.argtypes = [dp, C.c_int32, C.c_int32, dp]
    fp = C.POINTER(C.c_float)
    L.lbm_mlp_param_count.argtypes = []
    L.lbm_mlp_param_count.restype = C.c_size_t
    L.lbm_mlp_create.argtypes = [C.c_int32, C.c_uint64, C.c_int32, vp, C.POINTER(vp)]
    L.lbm_mlp_set_params.argtypes = [vp, fp, C.c_size_t]
    L.lbm_mlp_get_params.argtypes = [vp, fp, C.c_size_t]
    L.lbm_mlp_forward.argtypes = [vp, vp, C.c_int32, vp]
    L.lbm_mlp_forward_noalloc.argtypes = [vp, C.c_int32, vp, C.c_int32, vp, vp]
    L.lbm_mlp_gradient.argtypes = [vp, vp, vp, vp, C.c_int32, fp, fp, dp]
    L.lbm_mlp_train.argtypes = [vp, vp, vp, vp, C.c_int32, fp, C.c_float, C.c_int32, dp]
    L.lbm_mlp_last_error.argtypes = []
    L.lbm_mlp_last_error.restype = C.c_char_p
    L.lbm_mlp_destroy.argtypes = [vp]
    L.lbm_mlp_destroy.restype = None
    _lib = L
    return L


def make_params(p: Dict) -> Params:
    s = Params()
    for name, _t in Params._fields_:
        setattr(s, name, p[name])
    return s


def workspace_bytes(params: Dict) -> int:
    L = load_library()
    n = C.c_size_t()
    rc = L.lbm_workspace_bytes(C.byref(make_params(params)), C.byref(n))
    if rc != LBM_OK:
        raise LbmError(rc, "lbm_workspace_bytes", L.lbm_strerror(rc).decode())
    return int(n.value)


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Solver:
    """One simulation on one GPU.  ``step`` is asynchronous on the torch
    stream that was current at construction."""

    def __init__(self, params: Dict, phi0: np.ndarray, T0: np.ndarray, device: Optional[int] = None,
                 stream=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("the solver needs a ROCm GPU (no CPU fallback)")
        self.L = load_library()
        self.torch = torch
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.nx, self.ny = int(params["nx"]), int(params["ny"])
        self.N = self.nx * self.ny
        phi0 = np.ascontiguousarray(phi0, dtype=np.float64).reshape(-1)
        T0 = np.ascontiguousarray(T0, dtype=np.float64).reshape(-1)
        if phi0.size != self.N or T0.size != self.N:
            raise ValueError("phi0/T0 must have nx*ny entries")
        self._p = make_params(params)
        nbytes = workspace_bytes(params)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            h = C.c_void_p()
            rc = self.L.lbm_init(C.byref(self._p), _dptr(phi0), _dptr(T0), C.c_void_p(self.workspace.data_ptr()),
                                 nbytes, C.c_void_p(self.stream.cuda_stream), C.byref(h))
        self._check(rc, "lbm_init")
        self._h = h

    def _check(self, rc: int, what: str):
        if rc != LBM_OK:
            raise LbmError(rc, what, self.L.lbm_last_error().decode())

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self.L.lbm_destroy(h)
            self._h = None

    def set_launch(self, tile: str = "64x4", xcd_remap=1):
        """xcd_remap: workgroup -> tile order, 0 row-major, 1 one contiguous band
        of tiles per XCD, 2 one band of tile columns per XCD (lbm_set_launch)."""
        self._check(self.L.lbm_set_launch(self._h, TILE_VARIANTS[tile], int(xcd_remap)), "lbm_set_launch")

    def set_store_mode(self, mode: str = "auto"):
        """auto (streaming stores once the state exceeds the Infinity Cache),
        cached or streaming (lbm_set_store_mode)."""
        self._check(self.L.lbm_set_store_mode(self._h, STORE_MODES[mode]), "lbm_set_store_mode")

    def autotune(self, reps: int = 20):
        """Pick the fastest launch shape for this grid; returns (tile, xcd_remap)."""
        v, x = C.c_int32(), C.c_int32()
        self._check(self.L.lbm_autotune(self._h, int(reps), C.byref(v), C.byref(x)), "lbm_autotune")
        return TILE_NAMES[v.value], int(x.value)

    def step(self, n: int = 1):
        self._check(self.L.lbm_step(self._h, int(n)), "lbm_step")

    def step_persistent(self, n: int = 1, barrier: str = "flat", wait_limit_us: int = 0) -> int:
        """The same n steps in one persistent cooperative launch with a grid
        barrier between steps (lbm_step_persistent), barrier "flat" or
        "per_xcd", each barrier wait bounded by wait_limit_us (0: 2 s);
        synchronises and returns the number of workgroups."""
        wg = C.c_int32(0)
        self._check(self.L.lbm_step_persistent(self._h, int(n), PERSIST_BARRIERS[barrier], int(wait_limit_us),
                                               C.byref(wg)), "lbm_step_persistent")
        return int(wg.value)

    def sync(self):
        self._check(self.L.lbm_sync(self._h), "lbm_sync")

    @property
    def step_count(self) -> int:
        return int(self.L.lbm_step_count(self._h))

    def fields(self, names: Iterable[str] = ("phi", "T", "ux", "uy", "p")) -> Dict[str, np.ndarray]:
        names = list(names)
        mask = 0
        for n in names:
            mask |= 1 << FIELD_BITS[n]
        order = sorted(names, key=lambda n: FIELD_BITS[n])
        outs = [np.empty(self.N, dtype=np.float64) for _ in order]
        arr = (C.POINTER(C.c_double) * len(outs))(*[_dptr(o) for o in outs])
        self._check(self.L.lbm_fields(self._h, mask, arr), "lbm_fields")
        return {n: o.reshape(self.ny, self.nx) for n, o in zip(order, outs)}

    def fields_device(self, names: Iterable[str]) -> Dict[str, "object"]:
        torch = self.torch
        names = list(names)
        mask = 0
        for n in names:
            mask |= 1 << FIELD_BITS[n]
        order = sorted(names, key=lambda n: FIELD_BITS[n])
        outs = [torch.empty(self.N, dtype=torch.float32, device=self.device) for _ in order]
        arr = (C.c_void_p * len(outs))(*[o.data_ptr() for o in outs])
        self._check(self.L.lbm_fields_device(self._h, mask, arr), "lbm_fields_device")
        return {n: o.view(self.ny, self.nx) for n, o in zip(order, outs)}

    def diag(self) -> Dict[str, float]:
        d = Diag()
        rc = self.L.lbm_diag(self._h, C.byref(d))
        if rc not in (LBM_OK, LBM_ENONFINITE):
            self._check(rc, "lbm_diag")
        out = {name: getattr(d, name) for name, _ in Diag._fields_}
        out["rc"] = rc
        return out

    def pops(self, lattice: str) -> np.ndarray:
        out = np.empty(9 * self.N, dtype=np.float64)
        self._check(self.L.lbm_pops(self._h, {"g": 0, "f": 1, "h": 2}[lattice], _dptr(out)), "lbm_pops")
        return out.reshape(9, self.ny, self.nx)

    def save(self) -> bytes:
        n = self.L.lbm_state_bytes(self._h)
        buf = C.create_string_buffer(n)
        self._check(self.L.lbm_save(self._h, buf, n), "lbm_save")
        return buf.raw

    def load(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        self._check(self.L.lbm_load(self._h, buf, len(blob)), "lbm_load")


def shape_of(phi: np.ndarray) -> Dict[str, float]:
    """Height, base radius and tip angle of the phi = 1/2 contour of a
    (ny, nx) field, measured by the library's device kernel."""
    L = load_library()
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    ny, nx = phi.shape
    out = np.empty(4, dtype=np.float64)
    rc = L.lbm_shape_of(_dptr(phi), nx, ny, _dptr(out))
    if rc != LBM_OK:
        raise LbmError(rc, "lbm_shape_of", L.lbm_batch_last_error().decode())
    return dict(height=out[0], base_radius=out[1], tip_angle_deg=out[2], npts=int(out[3]))


def batch_workspace_bytes(params_list, slots: int) -> int:
    L = load_library()
    arr = (Params * len(params_list))(*[make_params(p) for p in params_list])
    n = C.c_size_t()
    rc = L.lbm_batch_workspace_bytes(arr, len(params_list), int(slots), C.byref(n))
    if rc != LBM_OK:
        raise LbmError(rc, "lbm_batch_workspace_bytes", L.lbm_strerror(rc).decode())
    return int(n.value)


class Batch:
    """A queue of droplets run together on one GPU (the batched sweep).

    ``params_list[i]``, ``phi0_list[i]``, ``T0_list[i]`` describe droplet i
    (its own grid); ``radii`` gives R for the Fourier number of t_freeze.
    Up to ``slots`` droplets are resident at a time."""

    def __init__(self, params_list, phi0_list, T0_list, radii=None, slots: Optional[int] = None, stream=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("the batch needs a ROCm GPU (no CPU fallback)")
        self.L = load_library()
        self.torch = torch
        n = len(params_list)
        if not (len(phi0_list) == len(T0_list) == n) or n < 1:
            raise ValueError("one phi0 and one T0 per parameter set")
        self.n = n
        self.slots = int(slots or n)
        self.shapes = [(int(p["ny"]), int(p["nx"])) for p in params_list]
        # the library reads droplet i's arrays when it enters a slot: keep them alive
        self._phi0 = [np.ascontiguousarray(a, dtype=np.float64).reshape(-1) for a in phi0_list]
        self._T0 = [np.ascontiguousarray(a, dtype=np.float64).reshape(-1) for a in T0_list]
        for i, (ny, nx) in enumerate(self.shapes):
            if self._phi0[i].size != nx * ny or self._T0[i].size != nx * ny:
                raise ValueError(f"droplet {i}: phi0/T0 must have nx*ny entries")
        self._params = (Params * n)(*[make_params(p) for p in params_list])
        self._radii = None if radii is None else np.ascontiguousarray(radii, dtype=np.float64)
        nbytes = batch_workspace_bytes(params_list, self.slots)
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        pa = (C.POINTER(C.c_double) * n)(*[_dptr(a) for a in self._phi0])
        ta = (C.POINTER(C.c_double) * n)(*[_dptr(a) for a in self._T0])
        h = C.c_void_p()
        rc = self.L.lbm_batch_init(self._params, n, pa, ta, None if self._radii is None else _dptr(self._radii),
                                   self.slots, C.c_void_p(self.workspace.data_ptr()), nbytes,
                                   C.c_void_p(self.stream.cuda_stream), C.byref(h))
        self._check(rc, "lbm_batch_init")
        self._h = h

    def _check(self, rc: int, what: str):
        if rc != LBM_OK:
            raise LbmError(rc, what, self.L.lbm_batch_last_error().decode())

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self.L.lbm_batch_destroy(h)
            self._h = None

    def configure(self, sample_every: int = 100, max_steps: int = 0, freeze_frac: float = 0.01,
                  use_graph: bool = True, persistent: Optional[str] = None, wait_limit_us: int = 0):
        """persistent None: one launch per step, replayed as a hipGraph unless
        use_graph is False; "flat" or "per_xcd": each sampling interval in one
        persistent cooperative launch with that grid barrier (64x8 tiles),
        each barrier wait bounded by wait_limit_us (0: 2 s)."""
        mode = INTERVAL_PERSIST[persistent] if persistent else int(bool(use_graph))
        self._check(self.L.lbm_batch_configure(self._h, int(sample_every), int(max_steps), float(freeze_frac), mode,
                                               int(wait_limit_us)), "lbm_batch_configure")

    def set_launch(self, tile: str = "64x4", xcd_group: int = 1):
        self._check(self.L.lbm_batch_set_launch(self._h, TILE_VARIANTS[tile], int(xcd_group)), "lbm_batch_set_launch")

    def set_store_mode(self, mode: str = "auto"):
        self._check(self.L.lbm_batch_set_store_mode(self._h, STORE_MODES[mode]), "lbm_batch_set_store_mode")

    def autotune(self, reps: int = 10):
        v, x = C.c_int32(), C.c_int32()
        self._check(self.L.lbm_batch_autotune(self._h, int(reps), C.byref(v), C.byref(x)), "lbm_batch_autotune")
        return TILE_NAMES[v.value], int(x.value)

    def step(self, nsteps: int, until_frozen: bool = False):
        self._check(self.L.lbm_batch_step(self._h, int(nsteps), int(bool(until_frozen))), "lbm_batch_step")

    def results(self):
        out = (DropResult * self.n)()
        self._check(self.L.lbm_batch_results(self._h, out), "lbm_batch_results")
        res = []
        for r in out:
            d = {name: getattr(r, name) for name, _ in DropResult._fields_}
            d["status"] = DROP_STATUS.get(d["status"], str(d["status"]))
            res.append(d)
        return res

    def fields(self, drop: int, names: Iterable[str] = ("phi", "T", "ux", "uy", "p")) -> Dict[str, np.ndarray]:
        names = list(names)
        mask = 0
        for nm in names:
            mask |= 1 << FIELD_BITS[nm]
        order = sorted(names, key=lambda nm: FIELD_BITS[nm])
        ny, nx = self.shapes[drop]
        outs = [np.empty(nx * ny, dtype=np.float64) for _ in order]
        arr = (C.POINTER(C.c_double) * len(outs))(*[_dptr(o) for o in outs])
        self._check(self.L.lbm_batch_fields(self._h, int(drop), mask, arr), "lbm_batch_fields")
        return {nm: o.reshape(ny, nx) for nm, o in zip(order, outs)}


class MLP:
    """Ensemble of surrogate networks on the GPU (matrix-core BF16 kernels).

    Inputs and targets are torch tensors on the device (float32, row-major):
    x [n][5], t and mask [n][3]; ``forward`` returns [ensemble][n][3]."""

    def __init__(self, ensemble: int = 8, seed: int = 0, max_batch: int = 8192, stream=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("the network needs a ROCm GPU (no CPU fallback)")
        self.L = load_library()
        self.torch = torch
        self.E = int(ensemble)
        self.max_batch = int(max_batch)
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.P = int(self.L.lbm_mlp_param_count())
        h = C.c_void_p()
        rc = self.L.lbm_mlp_create(self.E, int(seed), self.max_batch, C.c_void_p(self.stream.cuda_stream), C.byref(h))
        self._check(rc, "lbm_mlp_create")
        self._h = h

    def _check(self, rc: int, what: str):
        if rc != LBM_OK:
            raise LbmError(rc, what, self.L.lbm_mlp_last_error().decode())

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self.L.lbm_mlp_destroy(h)
            self._h = None

    @staticmethod
    def _fp(a: np.ndarray):
        return a.ctypes.data_as(C.POINTER(C.c_float))

    def get_params(self) -> np.ndarray:
        out = np.empty(self.E * self.P, dtype=np.float32)
        self._check(self.L.lbm_mlp_get_params(self._h, self._fp(out), out.size), "lbm_mlp_get_params")
        return out.reshape(self.E, self.P)

    def set_params(self, params: np.ndarray):
        a = np.ascontiguousarray(params, dtype=np.float32).reshape(-1)
        self._check(self.L.lbm_mlp_set_params(self._h, self._fp(a), a.size), "lbm_mlp_set_params")

    def _dev(self, a, cols):
        t = self.torch.as_tensor(a, dtype=self.torch.float32, device=self.device).contiguous()
        if t.dim() != 2 or t.shape[1] != cols:
            raise ValueError(f"expected [n][{cols}]")
        return t

    def forward(self, x):
        x = self._dev(x, 5)
        n = x.shape[0]
        y = self.torch.empty((self.E, n, 3), dtype=self.torch.float32, device=self.device)
        self._check(self.L.lbm_mlp_forward(self._h, C.c_void_p(x.data_ptr()), n, C.c_void_p(y.data_ptr())),
                    "lbm_mlp_forward")
        return y

    def _w3(self, w):
        w = np.ones(3, dtype=np.float32) if w is None else np.ascontiguousarray(w, dtype=np.float32)
        return w

    def gradient(self, x, t, mask, w=None):
        x, t, mask = self._dev(x, 5), self._dev(t, 3), self._dev(mask, 3)
        n = x.shape[0]
        g = np.empty(self.E * self.P, dtype=np.float32)
        loss = np.empty(self.E, dtype=np.float64)
        w3 = self._w3(w)
        self._check(self.L.lbm_mlp_gradient(self._h, C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()),
                                            C.c_void_p(mask.data_ptr()), n, self._fp(w3), self._fp(g), _dptr(loss)),
                    "lbm_mlp_gradient")
        return loss, g.reshape(self.E, self.P)

    def train(self, x, t, mask, steps: int, lr: float = 1e-3, w=None):
        x, t, mask = self._dev(x, 5), self._dev(t, 3), self._dev(mask, 3)
        n = x.shape[0]
        loss = np.empty(self.E, dtype=np.float64)
        w3 = self._w3(w)
        self._check(self.L.lbm_mlp_train(self._h, C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()),
                                         C.c_void_p(mask.data_ptr()), n, self._fp(w3), float(lr), int(steps),
                                         _dptr(loss)), "lbm_mlp_train")
        return loss


MLP_NOALLOC_MAX_ENSEMBLE = 16  # LBM_MLP_NOALLOC_MAX_ENSEMBLE


def mlp_forward_noalloc(params, x, y, stream=None):
    """lbm_mlp_forward_noalloc: the network's forward pass from device FP32
    parameters ``params`` [ensemble][param_count] for device inputs ``x``
    [n][5] into the caller's device output ``y`` [ensemble][n][3] (all
    contiguous float32 torch tensors on the current device).  The library
    allocates nothing; calls overlapping on one GPU race."""
    import torch

    L = load_library()
    P = int(L.lbm_mlp_param_count())
    for name, t in (("params", params), ("x", x), ("y", y)):
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous float32 device tensor")
    if params.dim() != 2 or params.shape[1] != P or x.dim() != 2 or x.shape[1] != 5:
        raise ValueError("expected params [ensemble][param_count] and x [n][5]")
    E, n = params.shape[0], x.shape[0]
    if tuple(y.shape) != (E, n, 3):
        raise ValueError(f"expected y of shape ({E}, {n}, 3)")
    st = stream if stream is not None else torch.cuda.current_stream(x.device)
    rc = L.lbm_mlp_forward_noalloc(C.c_void_p(params.data_ptr()), E, C.c_void_p(x.data_ptr()), n,
                                   C.c_void_p(y.data_ptr()), C.c_void_p(st.cuda_stream))
    if rc != LBM_OK:
        raise LbmError(rc, "lbm_mlp_forward_noalloc", L.lbm_mlp_last_error().decode())
    return y
