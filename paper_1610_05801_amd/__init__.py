"""MI355X-native longitudinal macro-particle tracking (libltrk).

Tracks macro-particles' (z, delta) turn by turn through a single-harmonic RF
bucket with Euler-Cromer, leap-frog, fourth-order Ruth or RK4 schemes
(Oeftiger 2014, section 1.1.2), with per-turn bunch moments, an extended map
(double-harmonic RF, phase offsets, slip factor to second order in delta)
with optional per-turn RF programmes and momentum ramps, a 6-D map with the
transverse linear one-turn map and chromaticity, a longitudinal wake kick, an FP32 +
Kahan-compensated state, batched tracking of uneven bunches and a
continuous-batching serving engine. All computation runs in the HIP library
libltrk.so built for gfx950; this package is its ctypes binding.
"""
from ._binding import *  # noqa: F401,F403
from ._binding import (EXPORTED, INTEGRATORS, DTYPES, Engine, EngineBusy, LtrkError, Ring,
                       Rf2, RfTurn, Twiss, Wake, LIB_PATH)

__all__ = [name for name in EXPORTED] + ["Engine", "EngineBusy", "LtrkError", "Ring", "Rf2", "RfTurn", "Twiss", "Wake",
                                          "INTEGRATORS", "DTYPES", "LIB_PATH"]
