"""MI355X-native hot path of the deterministic neural-network quantum-state method
(arXiv 2601.21310): Slater-Condon H_SS, batched neural backflow amplitudes, variational
energy and gradient, and Epstein-Nesbet PT2, as hand-written HIP kernels for gfx950
behind a C ABI (include/dnqs.h).  This package is the Python binding.
"""
from ._native import (FP32, MIXED, SPLIT_BF16, Connections, Context, DetNQSEnergy, DnqsError, Graph, LIB_PATH,
                      TorchAllocator,
                      dets_to_device, dets_to_host, lib)

__all__ = ["FP32", "MIXED", "SPLIT_BF16", "Connections", "Context", "TorchAllocator", "DetNQSEnergy", "DnqsError", "Graph", "LIB_PATH",
           "dets_to_device", "dets_to_host", "lib"]
