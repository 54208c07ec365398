"""ctypes wrapper of the FP64 oracle library (test infrastructure only)."""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Dict, Iterable, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liblbm_oracle.so")

FIELD_BITS = {"phi": 0, "T": 1, "ux": 2, "uy": 3, "p": 4, "fs": 5, "fl": 6, "rho": 7, "H": 8, "mdot": 9}


class _Params(C.Structure):
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


class _Diag(C.Structure):
    _fields_ = [
        ("step", C.c_int64), ("sum_phi", C.c_double), ("sum_phic", C.c_double),
        ("sum_solid", C.c_double), ("sum_liquid", C.c_double), ("sum_H", C.c_double),
        ("max_u", C.c_double), ("h_c", C.c_double), ("nonfinite", C.c_int32),
    ]


# FP64 throughout, no fast-math and no FMA contraction, so every build of the
# same source (any -O level, any -march) gives the same bits.
_CFLAGS = ["-fopenmp", "-fPIC", "-shared", "-ffp-contract=off", "-std=c11", "-D_DEFAULT_SOURCE", "-Wall", "-Wextra"]


def build_oracle(force: bool = True) -> str:
    """Compile the oracle in-tree with gcc -O3 (portable: the library travels
    with the tree to other hosts)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O3"] + _CFLAGS + ["-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def build_native(out_dir: str) -> str:
    """The same source built with gcc -O3 -march=native into out_dir, for
    timing the oracle on the host it runs on."""
    out = os.path.join(out_dir, "liblbm_oracle_native.so")
    subprocess.run(["gcc", "-O3", "-march=native"] + _CFLAGS + ["-o", out, _SRC, "-lm"], check=True)
    return out


def use_library(path: str) -> None:
    """Load the oracle from another build of the same source (before the
    first solver is made)."""
    global _LIB, _lib
    _LIB = path
    _lib = None


_lib = None


def host_threads() -> int:
    """Host threads this process may use: its CPU affinity, capped by
    OMP_NUM_THREADS when that is set."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    omp = os.environ.get("OMP_NUM_THREADS", "")
    if omp.isdigit() and int(omp) > 0:
        n = min(n, int(omp))
    return max(1, n)


def default_threads() -> int:
    """Rows are split over at most 16 host threads by default."""
    return max(1, min(16, host_threads()))


def lib_path() -> str:
    return _LIB


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build_oracle(force=False)
    L = C.CDLL(_LIB)
    dp = C.POINTER(C.c_double)
    L.oracle_init.argtypes = [C.POINTER(_Params), dp, dp, C.POINTER(C.c_void_p)]
    L.oracle_validate.argtypes = [C.POINTER(_Params)]
    L.oracle_step.argtypes = [C.c_void_p, C.c_int32]
    L.oracle_fields.argtypes = [C.c_void_p, C.c_uint32, C.POINTER(dp)]
    L.oracle_diag.argtypes = [C.c_void_p, C.POINTER(_Diag)]
    L.oracle_pops.argtypes = [C.c_void_p, C.c_int32, dp]
    L.oracle_state_bytes.argtypes = [C.c_void_p]
    L.oracle_state_bytes.restype = C.c_size_t
    L.oracle_save.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t]
    L.oracle_load.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t]
    L.oracle_step_count.argtypes = [C.c_void_p]
    L.oracle_step_count.restype = C.c_int64
    L.oracle_set_threads.argtypes = [C.c_int32]
    L.oracle_destroy.argtypes = [C.c_void_p]
    L.oracle_destroy.restype = None
    d = C.c_double
    L.oracle_geq.argtypes = [d, d, d, dp]
    L.oracle_gsrc.argtypes = [d, d, d, d, d, d, dp]
    L.oracle_feq.argtypes = [d, d, d, d, dp]
    L.oracle_fforce.argtypes = [d, d, d, d, d, d, d, d, d, dp]
    L.oracle_heq.argtypes = [d, d, d, d, d, d, dp]
    L.oracle_pressure.argtypes = [dp, d, d, d, d, d, d, dp]
    L.oracle_enthalpy.argtypes = [d, d, d, d, dp, dp]
    L.oracle_stencil.argtypes = [C.c_int32, C.c_int32, dp, dp, dp, dp]
    L.oracle_wetting_ghost.argtypes = [C.c_int32, d, dp, dp, dp]
    for fn in ("geq", "gsrc", "feq", "fforce", "heq", "pressure", "enthalpy", "stencil", "wetting_ghost"):
        getattr(L, "oracle_" + fn).restype = None
    _lib = L
    return L


def _dptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _params(p: Dict) -> _Params:
    s = _Params()
    for name, _t in _Params._fields_:
        setattr(s, name, p[name])
    return s


class OracleSolver:
    """FP64 reference solver.  ``fields`` and ``diag`` report the macroscopic
    state at the current time level (the macro part of the next step)."""

    def __init__(self, params: Dict, phi0: np.ndarray, T0: np.ndarray, threads: Optional[int] = None):
        self.L = load()
        # OpenMP's thread count is process-wide: set it on every construction
        self.L.oracle_set_threads(int(threads) if threads else default_threads())
        self.nx, self.ny = int(params["nx"]), int(params["ny"])
        self.N = self.nx * self.ny
        phi0 = np.ascontiguousarray(phi0, dtype=np.float64).reshape(-1)
        T0 = np.ascontiguousarray(T0, dtype=np.float64).reshape(-1)
        if phi0.size != self.N or T0.size != self.N:
            raise ValueError("phi0/T0 must have nx*ny entries")
        self._p = _params(params)
        h = C.c_void_p()
        rc = self.L.oracle_init(C.byref(self._p), _dptr(phi0), _dptr(T0), C.byref(h))
        if rc != 0:
            raise ValueError(f"oracle_init failed ({rc})")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self.L.oracle_destroy(h)
            self._h = None

    def step(self, n: int = 1):
        rc = self.L.oracle_step(self._h, int(n))
        if rc != 0:
            raise RuntimeError(f"oracle_step failed ({rc})")

    @property
    def step_count(self) -> int:
        return int(self.L.oracle_step_count(self._h))

    def fields(self, names: Iterable[str] = ("phi", "T", "ux", "uy", "p")) -> Dict[str, np.ndarray]:
        names = list(names)
        mask = 0
        for n in names:
            mask |= 1 << FIELD_BITS[n]
        order = sorted(names, key=lambda n: FIELD_BITS[n])
        outs = [np.empty(self.N, dtype=np.float64) for _ in order]
        arr = (C.POINTER(C.c_double) * len(outs))(*[_dptr(o) for o in outs])
        rc = self.L.oracle_fields(self._h, mask, arr)
        if rc != 0:
            raise RuntimeError(f"oracle_fields failed ({rc})")
        return {n: o.reshape(self.ny, self.nx) for n, o in zip(order, outs)}

    def diag(self) -> Dict[str, float]:
        d = _Diag()
        rc = self.L.oracle_diag(self._h, C.byref(d))
        out = {name: getattr(d, name) for name, _ in _Diag._fields_}
        out["rc"] = rc
        return out

    def pops(self, lattice: str) -> np.ndarray:
        idx = {"g": 0, "f": 1, "h": 2}[lattice]
        out = np.empty(9 * self.N, dtype=np.float64)
        rc = self.L.oracle_pops(self._h, idx, _dptr(out))
        if rc != 0:
            raise RuntimeError("oracle_pops failed")
        return out.reshape(9, self.ny, self.nx)

    def save(self) -> bytes:
        n = self.L.oracle_state_bytes(self._h)
        buf = C.create_string_buffer(n)
        rc = self.L.oracle_save(self._h, buf, n)
        if rc != 0:
            raise RuntimeError("oracle_save failed")
        return buf.raw

    def load(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        rc = self.L.oracle_load(self._h, buf, len(blob))
        if rc != 0:
            raise RuntimeError(f"oracle_load failed ({rc})")


def validate(params: Dict) -> int:
    L = load()
    p = _params(params)
    return int(L.oracle_validate(C.byref(p)))


# ---- per-node building blocks ----------------------------------------------
def _call9(fn, *args) -> np.ndarray:
    out = np.empty(9, dtype=np.float64)
    fn(*[float(a) for a in args], _dptr(out))
    return out


def node_geq(phi, ux, uy):
    return _call9(load().oracle_geq, phi, ux, uy)


def node_gsrc(phi, dphiux, dphiuy, lnx, lny, mdot):
    return _call9(load().oracle_gsrc, phi, dphiux, dphiuy, lnx, lny, mdot)


def node_feq(p, rho, ux, uy):
    return _call9(load().oracle_feq, p, rho, ux, uy)


def node_fforce(S, Fx, Fy, rfx, rfy, ux, uy, Ftx, Fty):
    return _call9(load().oracle_fforce, S, Fx, Fy, rfx, rfy, ux, uy, Ftx, Fty)


def node_heq(H, T, cp, cp_ref, ux, uy):
    return _call9(load().oracle_heq, H, T, cp, cp_ref, ux, uy)


def node_pressure(f9, S, F0, tau_f, rho, ux, uy) -> float:
    f9 = np.ascontiguousarray(f9, dtype=np.float64)
    out = np.empty(1, dtype=np.float64)
    load().oracle_pressure(_dptr(f9), float(S), float(F0), float(tau_f), float(rho), float(ux), float(uy), _dptr(out))
    return float(out[0])


def node_enthalpy(H, cp, T_melt, latent):
    fl = C.c_double()
    T = C.c_double()
    load().oracle_enthalpy(float(H), float(cp), float(T_melt), float(latent), C.byref(fl), C.byref(T))
    return fl.value, T.value


def stencil(ext: np.ndarray):
    """ext: (ny+2, nx) array including ghost rows; returns gx, gy, lap (ny, nx)."""
    ext = np.ascontiguousarray(ext, dtype=np.float64)
    nyp2, nx = ext.shape
    ny = nyp2 - 2
    gx = np.empty((ny, nx)); gy = np.empty((ny, nx)); lap = np.empty((ny, nx))
    load().oracle_stencil(nx, ny, _dptr(ext), _dptr(gx), _dptr(gy), _dptr(lap))
    return gx, gy, lap


def wetting_ghost(theta_deg: float, row0: np.ndarray, row1: np.ndarray) -> np.ndarray:
    row0 = np.ascontiguousarray(row0, dtype=np.float64)
    row1 = np.ascontiguousarray(row1, dtype=np.float64)
    out = np.empty_like(row0)
    load().oracle_wetting_ghost(row0.size, float(theta_deg), _dptr(row0), _dptr(row1), _dptr(out))
    return out
