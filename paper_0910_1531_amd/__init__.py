"""MI355X FFT/Picard solver for three-dimensional classical DFT of charged hard spheres.

The compute path is the HIP library libdftpicard.so (C ABI in include/dft.h); this
package only marshals arguments to it.  PyTorch provides device memory and streams.
The library is loaded on first use (Solver, bulk, workspace_size, load) and an
ImportError is raised then if it has not been built: there is no fallback path.
"""
from . import _abi
from ._abi import (DFT_FP32_MIXED, DFT_FP64, FLAG_ALLOW_NON_NEUTRAL, FLAG_CUTOFF_LAMBDA, DftError, MAX_SPECIES,
                   NALPHA, STATUS_NAMES)
from .solver import Solver, bulk, make_params, workspace_size

load = _abi.load

__all__ = ["Solver", "bulk", "make_params", "workspace_size", "DftError", "DFT_FP64", "DFT_FP32_MIXED",
           "FLAG_ALLOW_NON_NEUTRAL", "FLAG_CUTOFF_LAMBDA", "MAX_SPECIES", "NALPHA", "STATUS_NAMES", "load"]
