"""MI355X-native state-vector quantum-circuit simulator core (gfx950).

The compute path is libsv.so (hand-written HIP kernels behind a C ABI,
include/sv.h); this package is its thin Python binding.  Importing the package
loads the library and fails if it has not been built.
"""
from .binding import (KIND, MODE, Batcher, Plan, Program, StateVector, SvError, gate_kernel, header_symbols, load_library,
                      make_gates, make_opts, util_copy, version)

load_library()

__all__ = ["KIND", "MODE", "Batcher", "Plan", "Program", "StateVector", "SvError", "gate_kernel", "header_symbols", "load_library", "make_gates",
           "make_opts", "util_copy", "version"]
