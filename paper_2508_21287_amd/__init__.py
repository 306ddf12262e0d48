"""MI355X-native enumeration of pattern-graph embeddings as int32 table joins
(the Delta-Motif method, arXiv 2508.21287), with hand-written HIP kernels for
gfx950 behind the C ABI of ``libdmotif.so`` (``include/dmotif.h``).

The native library is loaded lazily on first use; a missing build raises an
error (there is no CPU fallback).  ``workloads`` holds the seeded input
generators and imports nothing else from this package.
"""
from ._binding import (DMError, Context, DataGraph, Result, Server, plan, lib, EXPORTS, LIB_PATH, summarize,
                       free_results,
                       MOTIF_M3, MOTIF_M4, MOTIF_M5, MOTIF_M6, MOTIF_C4, MOTIF_C6, MOTIF_C12, MOTIF_M4_1,
                       MOTIF_M6_2O, MOTIF_M18_O_6, MOTIF_M7, MOTIF_ALL,
                       MOTIF_AUTO, MOTIF_M2_ONLY, MOTIF_NAMES, OUT_TABLE, OUT_COUNT_HASH)

__all__ = ["DMError", "Context", "DataGraph", "Result", "Server", "plan", "lib", "EXPORTS", "LIB_PATH", "summarize",
           "free_results",
           "MOTIF_M3", "MOTIF_M4", "MOTIF_M5", "MOTIF_M6", "MOTIF_C4", "MOTIF_C6", "MOTIF_C12", "MOTIF_M4_1",
           "MOTIF_M6_2O", "MOTIF_M18_O_6", "MOTIF_M7", "MOTIF_ALL",
           "MOTIF_AUTO", "MOTIF_M2_ONLY", "MOTIF_NAMES", "OUT_TABLE", "OUT_COUNT_HASH"]
