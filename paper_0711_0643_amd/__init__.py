"""Direct-summation N-body engine for AMD Instinct MI355X (gfx950).

Hermite fourth-order block-step integration with the pairwise force on the
GPU (Portegies Zwart et al., "A parallel gravitational N-body kernel",
Sect. 2.1).  The compute path is the HIP library ``libnbody.so`` behind a C
ABI (``include/nbody.h``); this package only marshals arguments to it, with
PyTorch providing device memory and streams.
"""
from .nbody import (  # noqa: F401
    FP64,
    MIXED,
    NBODY_E_DTMIN,
    NBODY_E_INDEX,
    NBODY_E_INVAL,
    NBODY_E_NONFINITE,
    NBODY_E_STATE,
    NBODY_OK,
    NBodyError,
    Params,
    Sim,
    lib,
    library_path,
    status_name,
)

__all__ = ["FP64", "MIXED", "NBodyError", "Params", "Sim", "lib", "library_path", "status_name"]
