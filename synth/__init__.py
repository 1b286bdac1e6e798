"""Seeded synthetic inputs for the transmission forward model.

This package generates *inputs only*: wavenumber grids, cross-section /
CIA / Rayleigh tables shaped like the paper's opacity data, temperature
profiles, parameter draws, channel edges and observation noise.  It holds
none of the forward model's arithmetic (no altitude, chord, opacity
weighting, optical depth, depth or binning code), so that the CPU oracle and
the HIP path can both consume the same arrays without sharing code.

Every generator takes an explicit ``numpy.random.Generator`` or a seed and
is deterministic for a given seed.
"""

from .constants import CONST, MASSES_AMU, R_JUP, R_SUN, GM_JUP  # noqa: F401
from .workloads import (  # noqa: F401
    Tables,
    Batch,
    Channels,
    make_config,
    CONFIG_NAMES,
)
