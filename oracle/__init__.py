"""FP64 CPU oracle (test infrastructure only).

Python access to ``liblbm_oracle.so`` via ctypes.  Only tests, the smoke
check and the benchmark's CPU-baseline leg may import this package; the GPU
library never does.
"""
from .oracle import (  # noqa: F401
    FIELD_BITS,
    OracleSolver,
    build_oracle,
    lib_path,
    load,
    node_fforce,
    node_feq,
    node_geq,
    node_gsrc,
    node_heq,
    node_enthalpy,
    node_pressure,
    stencil,
    wetting_ghost,
)
