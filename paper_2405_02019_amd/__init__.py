"""MI355X-native simulator of the Potjans-Diesmann cortical microcircuit.

The simulation runs in hand-written HIP kernels for gfx950 behind the C ABI of
include/snn.h (libsnn.so); this package is its Python binding.
"""
from .snn import (ENGINE_AUTO, ENGINE_BAND, ENGINE_LDS, ENGINE_PERSISTENT, ENGINE_STEPWISE, SYN_COMPRESSED5, SYN_DEV8, SYN_PLAIN8,
                  Instance, SnnError, Simulator, balanced_windows, lib, sample_network)

__all__ = ["Instance", "Simulator", "SnnError", "balanced_windows", "lib", "sample_network", "SYN_PLAIN8",
           "SYN_COMPRESSED5", "SYN_DEV8", "ENGINE_AUTO", "ENGINE_BAND", "ENGINE_STEPWISE", "ENGINE_PERSISTENT", "ENGINE_LDS"]
