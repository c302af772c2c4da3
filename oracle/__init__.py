"""CPU oracle for Hogbom CLEAN and tiled CLEAN with feedback (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: the correctness reference for the GPU library.  Only
the test suite, the smoke check and the benchmark's CPU-baseline leg may load
it; the product never does, and it shares no code with the product.

The arithmetic lives in ``oracle.c`` (plain C, explicit fma, no contraction);
this module only marshals numpy arrays.  ``build()`` compiles the C file with
gcc; ``load()`` builds it on first use if the shared object is missing.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_CFLAGS = ["-O3", "-mavx2", "-mfma", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-shared", "-fPIC"]

STOP_NAMES = {0: "maxiter", 1: "threshold", 2: "capacity", 4: "nonfinite"}
_lib = None


def build() -> str:
    """Compile liboracle.so with gcc (always recompiles)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", *_CFLAGS, "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = C.CDLL(_LIB)
    P = C.c_void_p
    i32, i64, f64 = C.c_int32, C.c_int64, C.c_double
    plain = [P, i32, i32, P, i32, i32, f64, f64, i64, P, P, P, i64, P, P, P]
    lib.oracle_hogbom_f32.argtypes = plain
    lib.oracle_hogbom_f64.argtypes = plain
    tiled = [P, i32, i32, P, i32, i32, i32, i32, i32, f64, f64, f64, i64, P, P, P, i64, P, P, P, P]
    lib.oracle_tiled_f32.argtypes = tiled
    lib.oracle_tiled_f64.argtypes = tiled
    fb = [P, i32, i32, i32, i32, P, i32, i32, P, P, P, i64]
    lib.oracle_feedback_f32.argtypes = fb
    lib.oracle_feedback_f64.argtypes = fb
    for f in (lib.oracle_hogbom_f32, lib.oracle_hogbom_f64, lib.oracle_tiled_f32, lib.oracle_tiled_f64,
              lib.oracle_feedback_f32, lib.oracle_feedback_f64):
        f.restype = C.c_int
    lib.oracle_peak_f32.argtypes = [P, i32, i32, i32, i32, i32]
    lib.oracle_peak_f32.restype = i64
    lib.oracle_peak_f64.argtypes = [P, i32, i32, i32, i32, i32]
    lib.oracle_peak_f64.restype = i64
    lib.oracle_main_lobe_area.argtypes = [P, i32, i32]
    lib.oracle_main_lobe_area.restype = i64
    lib.oracle_restore_f64.argtypes = [P, P, i32, i32, f64, P]
    lib.oracle_restore_f64.restype = C.c_int
    _lib = lib
    return lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _inputs(dirty, psf):
    dirty = np.ascontiguousarray(dirty, dtype=np.float32)
    psf = np.ascontiguousarray(psf, dtype=np.float32)
    if dirty.ndim != 2 or psf.ndim != 2:
        raise ValueError("dirty and psf must be 2-D")
    return dirty, psf


def hogbom(dirty, psf, gain=0.1, threshold=0.0, max_iter=1000, cap=None, precision="f32", model=True):
    """Plain Hogbom CLEAN.  Returns dict(residual, idx, flux, model, n_iter, stop)."""
    lib = load()
    dirty, psf = _inputs(dirty, psf)
    ny, nx = dirty.shape
    cap = max_iter if cap is None else cap
    ft = np.float32 if precision == "f32" else np.float64
    res = np.empty((ny, nx), ft)
    idx = np.zeros(max(cap, 1), np.int32)
    flux = np.zeros(max(cap, 1), ft)
    mod = np.empty((ny, nx), np.float64) if model else None
    n = C.c_int64(0)
    stop = C.c_int32(0)
    fn = lib.oracle_hogbom_f32 if precision == "f32" else lib.oracle_hogbom_f64
    st = fn(_ptr(dirty), ny, nx, _ptr(psf), psf.shape[0], psf.shape[1], float(gain), float(threshold),
            int(max_iter), _ptr(res), _ptr(idx), _ptr(flux), int(cap), _ptr(mod), C.byref(n), C.byref(stop))
    if st != 0:
        raise ValueError(f"oracle_hogbom returned {st}")
    k = n.value
    return dict(residual=res, idx=idx[:k].copy(), flux=flux[:k].copy(), model=mod, n_iter=k,
                stop=stop.value)


def tiled(dirty, psf, tiles=(2, 2), interval=100, gain=0.1, threshold=0.0, max_iter=1000, cap=None,
          precision="f32", model=True, level=0.0):
    """Tiled Hogbom CLEAN with feedback.  Returns dict(..., n_rounds).

    level: the flux trigger, a fraction of the largest tile peak at each
    round's start below which a tile ends its round (0: interval only)."""
    lib = load()
    dirty, psf = _inputs(dirty, psf)
    ny, nx = dirty.shape
    cap = max_iter if cap is None else cap
    ft = np.float32 if precision == "f32" else np.float64
    res = np.empty((ny, nx), ft)
    idx = np.zeros(max(cap, 1), np.int32)
    flux = np.zeros(max(cap, 1), ft)
    mod = np.empty((ny, nx), np.float64) if model else None
    n = C.c_int64(0)
    stop = C.c_int32(0)
    rounds = C.c_int32(0)
    fn = lib.oracle_tiled_f32 if precision == "f32" else lib.oracle_tiled_f64
    st = fn(_ptr(dirty), ny, nx, _ptr(psf), psf.shape[0], psf.shape[1], int(tiles[0]), int(tiles[1]),
            int(interval), float(level), float(gain), float(threshold), int(max_iter), _ptr(res), _ptr(idx), _ptr(flux),
            int(cap), _ptr(mod), C.byref(n), C.byref(stop), C.byref(rounds))
    if st != 0:
        raise ValueError(f"oracle_tiled returned {st}")
    k = n.value
    return dict(residual=res, idx=idx[:k].copy(), flux=flux[:k].copy(), model=mod, n_iter=k,
                stop=stop.value, n_rounds=rounds.value)


def peak(r, rect=None):
    """Flat index of the peak of a 2-D float32/float64 array (or of the
    rectangle (y0, y1, x0, x1) of it): the largest |r|, every NaN above +Inf
    and equal to each other, the lowest row-major index on ties."""
    lib = load()
    r = np.ascontiguousarray(r)
    if r.dtype not in (np.float32, np.float64) or r.ndim != 2:
        raise ValueError("r must be a 2-D float32 or float64 array")
    y0, y1, x0, x1 = rect if rect is not None else (0, r.shape[0], 0, r.shape[1])
    fn = lib.oracle_peak_f32 if r.dtype == np.float32 else lib.oracle_peak_f64
    k = int(fn(_ptr(r), r.shape[1], int(y0), int(y1), int(x0), int(x1)))
    if k < 0:
        raise ValueError("empty or out-of-range rectangle")
    return k


def feedback(residual, psf, tiles, comp_tile, comp_idx, comp_flux, precision="f32"):
    """One feedback step applied to a copy of ``residual``; returns the copy."""
    lib = load()
    ft = np.float32 if precision == "f32" else np.float64
    r = np.array(residual, dtype=ft, copy=True, order="C")
    psf = np.ascontiguousarray(psf, dtype=np.float32)
    ct = np.ascontiguousarray(comp_tile, dtype=np.int32)
    ci = np.ascontiguousarray(comp_idx, dtype=np.int32)
    cf = np.ascontiguousarray(comp_flux, dtype=ft)
    fn = lib.oracle_feedback_f32 if precision == "f32" else lib.oracle_feedback_f64
    st = fn(_ptr(r), r.shape[0], r.shape[1], int(tiles[0]), int(tiles[1]), _ptr(psf), psf.shape[0],
            psf.shape[1], _ptr(ct), _ptr(ci), _ptr(cf), len(ci))
    if st != 0:
        raise ValueError(f"oracle_feedback returned {st}")
    return r


def main_lobe_area(psf):
    """Pixels of the PSF's main lobe: the 4-connected region above one half
    that contains the centre (-1 if the centre is not above one half)."""
    psf = np.ascontiguousarray(psf, dtype=np.float32)
    return int(load().oracle_main_lobe_area(_ptr(psf), psf.shape[0], psf.shape[1]))


def beam_sigma(psf):
    """Clean-beam sigma (pixels): FWHM = 2 sqrt(A / pi), A the main-lobe area."""
    area = main_lobe_area(psf)
    if area <= 0:
        raise ValueError("PSF centre is not above one half")
    return 2.0 * np.sqrt(area / np.pi) / (2.0 * np.sqrt(2.0 * np.log(2.0)))


def restore(model, residual, sigma):
    """Restored image (float64): residual + model (*) exp(-|d|^2 / (2 sigma^2)),
    over the square window |d| <= ceil(5 sigma)."""
    model = np.ascontiguousarray(model, dtype=np.float64)
    residual = np.ascontiguousarray(residual, dtype=np.float32)
    out = np.empty(model.shape, np.float64)
    st = load().oracle_restore_f64(_ptr(model), _ptr(residual), model.shape[0], model.shape[1], float(sigma),
                                   _ptr(out))
    if st != 0:
        raise ValueError(f"oracle_restore_f64 returned {st}")
    return out
