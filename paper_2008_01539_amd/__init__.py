"""Localized fully implicit Newton solver for fractured reservoirs on
MI355X (gfx950): HIP kernels behind the C ABI of include/fim.h, with a thin
ctypes binding.

    from paper_2008_01539_amd import FimModel, Options, LOCAL

Also: ``FimBatch`` (several models per batched call), ``serve`` (the
continuous-batching serving loop), ``trace`` (per-iteration JSONL log).
"""
from .fim import (DD, DD_ADD, DEVICE, FP64, FULL, HOST, LIB_PATH, LOCAL, MIXED, PC_FRACTURE,
                  PC_FRACTURE_COUPLED, PC_JACOBI, RESID, FimBatch, FimError, FimModel, IterStats, NotConverged, Options, StepStats,
                  estimate_bytes, exported_symbols)

__all__ = ["FimModel", "FimBatch", "Options", "FimError", "NotConverged", "IterStats",
           "StepStats", "FULL", "LOCAL", "DD", "DD_ADD", "RESID", "FP64", "MIXED", "HOST", "DEVICE",
           "PC_JACOBI", "PC_FRACTURE", "PC_FRACTURE_COUPLED",
           "LIB_PATH", "estimate_bytes", "exported_symbols"]
