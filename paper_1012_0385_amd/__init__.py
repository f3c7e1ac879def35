"""MI355X (gfx950) engine for the ASEP / KPZ lattice gas.

The simulation runs in ``libasep.so`` (hand-written HIP kernels behind the C ABI
of ``include/asep.h``); this package holds its build script and the ctypes
binding.  Importing the package does not load the library; the first call does,
and fails loudly if the library has not been built.
"""
from . import binding
from .binding import AsepError
from .sim import (Server, Simulation, ensemble_w2, load_tuning, make_params, resolve,
                  run_batch, sample_times)

__all__ = ["binding", "AsepError", "Server", "Simulation", "ensemble_w2", "load_tuning",
           "make_params", "resolve", "run_batch", "sample_times"]
