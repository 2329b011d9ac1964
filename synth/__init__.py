"""Seeded synthetic inputs for the boxcar search.

This package only draws random numbers and lays them out as complex
spectra.  It holds none of the search's arithmetic: a tone's per-bin power
is computed by the caller (from whichever significance code it trusts) and
passed in through ``tone_power``.  Both the FP64 oracle's tests and the GPU
library's tests and benchmark draw their inputs from here.
"""

from .spectra import (  # noqa: F401
    WORKLOADS,
    Tone,
    Workload,
    batched_workload,
    draw_tones,
    inject_tones,
    make_spectrum,
    make_spectrum_device,
    red_ramp,
    rng_for,
    white_noise,
    workload,
)
