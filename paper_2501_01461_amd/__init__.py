"""MI355X (gfx950) Hogbom CLEAN and tiled CLEAN with feedback.

The compute runs in ``libclean.so`` (HIP kernels behind a C ABI, include/clean.h);
``_native`` is its thin ctypes binding and ``synth`` the seeded input generator.
"""
from ._native import (CleanError, autotune, autotune_interval, bandwidth_probe, batched, clean_beam,  # noqa: F401
                      hogbom, hogbom_noalloc, load, psf_to_f16, restore, tiled_feedback, version)
