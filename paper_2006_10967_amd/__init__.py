"""MI355X-native FR-PCPF: Flux Reconstruction of the preconditioned, localized conservative
phase-field interface method (Al-Salami, Kamra & Hu, arXiv 2006.10967) on one gfx950 GPU.

The method runs in the HIP library ``libpcpf.so`` built from ``csrc/`` (C ABI in
``include/pcpf.h``); :class:`Solver` is its thin Python binding.
"""
from ._lib import PcpfError, load  # noqa: F401
from .solver import (BF16, FP32, FP64, MODE_PHYS, MODE_PRECOND, REDUCE_L1, REDUCE_MASS,  # noqa: F401
                     REDUCE_RMS, DenseMeshArgs, MeshArgs, Solver, line_operators,
                     make_params, triangle_operators)

__all__ = ["Solver", "MeshArgs", "DenseMeshArgs", "line_operators", "triangle_operators", "make_params", "PcpfError", "load",
           "FP64", "FP32", "BF16", "MODE_PHYS", "MODE_PRECOND", "REDUCE_MASS", "REDUCE_L1",
           "REDUCE_RMS"]
