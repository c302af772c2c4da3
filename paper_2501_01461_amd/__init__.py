"""MI355X (gfx950) Hogbom CLEAN and tiled CLEAN with feedback.

The compute runs in ``libclean.so`` (HIP kernels behind a C ABI, include/clean.h);
``_native`` is its thin ctypes binding and ``synth`` the seeded input generator.
"""
from ._native import (CleanError, autotune, autotune_interval, autotune_batched, autotune_plan, bandwidth_probe, batched,  # noqa: F401
                      clean_beam, hogbom, hogbom_noalloc, load, psf_to_f16, restore, set_workspace_limit,
                      tiled_feedback, version)
