"""ctypes binding of the gfx950 CLEAN library (libclean.so).

Argument marshalling only: torch CUDA tensors supply device memory and the
current stream; every step of the computation runs in the library's kernels.
There is no CPU fallback: if the library is missing or no GPU is present the
calls raise.
"""
from __future__ import annotations

import ctypes as C
import math
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libclean.so")

CLEAN_OK = 0
STATUS = {0: "CLEAN_OK", -1: "CLEAN_E_INVAL", -2: "CLEAN_E_NONFINITE", -3: "CLEAN_E_NOMEM",
          -4: "CLEAN_E_HIP", -5: "CLEAN_E_TIMEOUT", -6: "CLEAN_E_UNSUPPORTED"}
STOP_NAMES = {0: "maxiter", 1: "threshold", 2: "capacity", 3: "cancelled", 4: "nonfinite"}
PSF_F32, PSF_F16 = 0, 1
FLAG_CHECK_FINITE = 1
FLAG_STREAM_RESIDUAL = 2
FLAG_FFT_FEEDBACK = 4
FLAG_FFT_TWO_LEVEL = 8

# every symbol include/clean.h declares
EXPORTS = ("clean_hogbom", "clean_hogbom_noalloc", "clean_tiled_feedback", "clean_batched", "clean_autotune",
           "clean_autotune_interval", "clean_autotune_plan", "clean_autotune_batched",
           "clean_beam_fit", "clean_restore", "clean_workspace_size", "clean_set_workspace_limit", "clean_psf_to_f16",
           "clean_bandwidth_probe",
           "clean_strerror",
           "clean_last_error", "clean_version")


class Params(C.Structure):
    _fields_ = [("gain", C.c_double), ("threshold", C.c_double), ("max_iter", C.c_int64),
                ("psf_dtype", C.c_int32), ("flags", C.c_int32), ("wg_per_tile", C.c_int32),
                ("px_per_thread", C.c_int32), ("feedback_level", C.c_double), ("cancel", C.c_void_p)]


class Stats(C.Structure):
    _fields_ = [("n_iter", C.c_int64), ("stop_reason", C.c_int32), ("n_rounds", C.c_int32),
                ("final_peak", C.c_double), ("residual_rms", C.c_double), ("model_flux", C.c_double),
                ("device_ms", C.c_float), ("wg_per_tile", C.c_int32), ("px_per_thread", C.c_int32),
                ("workgroups", C.c_int32), ("phase_us", C.c_float * 3), ("streamed", C.c_int32),
                ("xcd_local_clusters", C.c_int32), ("exchange_levels", C.c_int32)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["phase_us"] = list(self.phase_us)
        return d


class Plan(C.Structure):
    _fields_ = [("tiles_y", C.c_int32), ("tiles_x", C.c_int32), ("interval", C.c_int32),
                ("wg_per_tile", C.c_int32), ("px_per_thread", C.c_int32), ("band_min", C.c_double),
                ("band_max", C.c_double), ("iters_per_s", C.c_double), ("from_cache", C.c_int32)]


class Problem(C.Structure):
    _fields_ = [("dirty", C.c_void_p), ("psf", C.c_void_p), ("residual", C.c_void_p),
                ("comp_idx", C.c_void_p), ("comp_flux", C.c_void_p), ("model", C.c_void_p),
                ("comp_cap", C.c_int64), ("max_iter", C.c_int64), ("threshold", C.c_double),
                ("ny", C.c_int32), ("nx", C.c_int32), ("psf_ny", C.c_int32), ("psf_nx", C.c_int32),
                ("tiles_y", C.c_int32), ("tiles_x", C.c_int32), ("interval", C.c_int32)]


class CleanError(RuntimeError):
    def __init__(self, status, detail):
        super().__init__(f"{STATUS.get(status, status)}: {detail}")
        self.status = status


_lib = None


def load():
    """Load libclean.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it first (python -m paper_2501_01461_amd.build)")
    lib = C.CDLL(LIB_PATH)
    P, i32, i64, sz = C.c_void_p, C.c_int, C.c_int64, C.c_size_t
    lib.clean_hogbom.argtypes = [P, i32, i32, P, i32, i32, C.POINTER(Params), P, P, P, i64, P, P, sz,
                                 C.POINTER(Stats), P]
    lib.clean_tiled_feedback.argtypes = [P, i32, i32, P, i32, i32, i32, i32, i32, C.POINTER(Params), P, P, P,
                                         i64, P, P, sz, C.POINTER(Stats), P]
    lib.clean_hogbom_noalloc.argtypes = [P, i32, i32, P, i32, i32, C.POINTER(Params), P, P, P, i64, P,
                                         C.POINTER(Stats), P]
    lib.clean_batched.argtypes = [C.POINTER(Problem), i32, C.POINTER(Params), C.POINTER(Stats), P]
    lib.clean_autotune_batched.argtypes = [C.POINTER(Problem), i32, C.POINTER(Params), i64, C.POINTER(i32),
                                           C.POINTER(C.c_float), P]
    lib.clean_autotune.argtypes = [P, i32, i32, P, i32, i32, i32, i32, i32, C.POINTER(Params), P, P, P, i64, i64,
                                   C.POINTER(Params), P]
    lib.clean_autotune.restype = C.c_int
    lib.clean_autotune_interval.argtypes = [P, i32, i32, P, i32, i32, i32, i32, P, i32, C.POINTER(Params), i64,
                                            C.c_double, P, P, P, i64, C.POINTER(C.c_int), P, P, P]
    lib.clean_autotune_interval.restype = C.c_int
    lib.clean_autotune_plan.argtypes = [P, i32, i32, P, i32, i32, P, i32, P, i32, C.POINTER(Params), i64, C.c_double,
                                        C.c_double, C.c_char_p, C.POINTER(Plan), P, P, P]
    lib.clean_autotune_plan.restype = C.c_int
    lib.clean_beam_fit.argtypes = [P, i32, i32, i32, C.POINTER(C.c_int64), C.POINTER(C.c_double), P]
    lib.clean_beam_fit.restype = C.c_int
    lib.clean_restore.argtypes = [P, P, i32, i32, C.c_double, P, P]
    lib.clean_restore.restype = C.c_int
    lib.clean_workspace_size.argtypes = [i32, i32, i32, i32, i32, C.POINTER(Params)]
    lib.clean_workspace_size.restype = sz
    lib.clean_psf_to_f16.argtypes = [P, P, i64, P]
    lib.clean_set_workspace_limit.argtypes = [sz]
    lib.clean_set_workspace_limit.restype = sz
    lib.clean_bandwidth_probe.argtypes = [P, sz, i32, i32, C.POINTER(C.c_double), P]
    lib.clean_bandwidth_probe.restype = C.c_int
    for f in (lib.clean_hogbom, lib.clean_hogbom_noalloc, lib.clean_tiled_feedback, lib.clean_batched,
              lib.clean_psf_to_f16):
        f.restype = C.c_int
    lib.clean_strerror.argtypes = [C.c_int]
    lib.clean_strerror.restype = C.c_char_p
    lib.clean_last_error.restype = C.c_char_p
    lib.clean_version.restype = C.c_char_p
    _lib = lib
    return lib


def _check(status):
    if status != CLEAN_OK:
        raise CleanError(status, load().clean_last_error().decode())


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU: the CLEAN library runs only on the device")
    return torch


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _params(gain, threshold, max_iter, psf, flags, wg_per_tile, px_per_thread):
    torch = _torch()
    if psf.dtype == torch.float16:
        dt = PSF_F16
    elif psf.dtype == torch.float32:
        dt = PSF_F32
    else:
        raise TypeError("psf must be float32 or float16")
    return Params(float(gain), float(threshold), int(max_iter), dt, int(flags), int(wg_per_tile),
                  int(px_per_thread))


def _cancel(flag):
    """The cancel flag: None, or a pinned host int32 tensor of one element
    (torch.zeros(1, dtype=torch.int32).pin_memory()) that another thread sets
    to a non-zero value to stop the run at its next checkpoint."""
    if flag is None:
        return None
    torch = _torch()
    if flag.dtype != torch.int32 or flag.is_cuda or not flag.is_pinned() or flag.numel() < 1:
        raise TypeError("cancel must be a pinned host int32 tensor")
    return flag.data_ptr()


def _prep(dirty, psf):
    torch = _torch()
    if dirty.dtype != torch.float32 or dirty.dim() != 2 or psf.dim() != 2:
        raise TypeError("dirty must be 2-D float32; psf 2-D float32/float16")
    if not (dirty.is_cuda and psf.is_cuda):
        raise TypeError("dirty and psf must be device tensors")
    return dirty.contiguous(), psf.contiguous()


def _outputs(dirty, cap, model):
    torch = _torch()
    ny, nx = dirty.shape
    dev = dirty.device
    res = torch.empty((ny, nx), dtype=torch.float32, device=dev)
    idx = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    flux = torch.empty(max(cap, 1), dtype=torch.float32, device=dev)
    mod = torch.empty((ny, nx), dtype=torch.float64, device=dev) if model else None
    return res, idx, flux, mod


def _flags(check_finite, stream):
    return (FLAG_CHECK_FINITE if check_finite else 0) | (FLAG_STREAM_RESIDUAL if stream else 0)


def hogbom(dirty, psf, gain=0.1, threshold=0.0, max_iter=1000, cap=None, model=True, check_finite=False,
           wg_per_tile=0, px_per_thread=0, stream=False, out=None, cancel=None):
    """Plain Hogbom CLEAN; returns dict(residual, idx, flux, model, stats)."""
    lib = load()
    dirty, psf = _prep(dirty, psf)
    cap = int(max_iter if cap is None else cap)
    res, idx, flux, mod = out if out is not None else _outputs(dirty, cap, model)
    p = _params(gain, threshold, max_iter, psf, _flags(check_finite, stream), wg_per_tile, px_per_thread)
    p.cancel = _cancel(cancel)
    st = Stats()
    ny, nx = dirty.shape
    _check(lib.clean_hogbom(_ptr(dirty), ny, nx, _ptr(psf), psf.shape[0], psf.shape[1], C.byref(p), _ptr(res),
                            _ptr(idx), _ptr(flux), cap, _ptr(mod), None, 0, C.byref(st), _stream()))
    n = st.n_iter
    return dict(residual=res, idx=idx[:n], flux=flux[:n], model=mod, stats=st.as_dict())


def hogbom_noalloc(dirty, psf, gain=0.1, threshold=0.0, max_iter=1000, cap=None, check_finite=False,
                   wg_per_tile=0, px_per_thread=0, stream=False, out=None, cancel=None):
    """clean_hogbom_noalloc: plain Hogbom CLEAN whose call allocates nothing
    (its workspace is the library's per-GPU device scratch array).  `out`
    (residual, idx, flux, model) lets a caller that cannot allocate pass its
    own buffers.  Returns dict(residual, idx, flux, model, stats)."""
    lib = load()
    dirty, psf = _prep(dirty, psf)
    cap = int(max_iter if cap is None else cap)
    res, idx, flux, mod = out if out is not None else _outputs(dirty, cap, True)
    p = _params(gain, threshold, max_iter, psf, _flags(check_finite, stream), wg_per_tile, px_per_thread)
    p.cancel = _cancel(cancel)
    st = Stats()
    ny, nx = dirty.shape
    _check(lib.clean_hogbom_noalloc(_ptr(dirty), ny, nx, _ptr(psf), psf.shape[0], psf.shape[1], C.byref(p),
                                    _ptr(res), _ptr(idx), _ptr(flux), cap, _ptr(mod), C.byref(st), _stream()))
    n = st.n_iter
    return dict(residual=res, idx=idx[:n], flux=flux[:n], model=mod, stats=st.as_dict())


def tiled_feedback(dirty, psf, tiles=(2, 2), interval=100, gain=0.1, threshold=0.0, max_iter=1000, cap=None,
                   model=True, check_finite=False, wg_per_tile=0, px_per_thread=0, stream=False, out=None,
                   level=0.0, fft=False, fft_two_level=False, cancel=None):
    """Tiled Hogbom CLEAN with feedback; returns dict(residual, idx, flux, model, stats).

    level: flux trigger, the fraction of the largest tile peak at a round's
    start below which a tile ends its round (0: interval only)."""
    lib = load()
    dirty, psf = _prep(dirty, psf)
    cap = int(max_iter if cap is None else cap)
    res, idx, flux, mod = out if out is not None else _outputs(dirty, cap, model)
    p = _params(gain, threshold, max_iter, psf, _flags(check_finite, stream), wg_per_tile, px_per_thread)
    p.feedback_level = float(level)
    p.cancel = _cancel(cancel)
    if fft:
        p.flags |= FLAG_FFT_FEEDBACK
    if fft_two_level:
        p.flags |= FLAG_FFT_FEEDBACK | FLAG_FFT_TWO_LEVEL
    st = Stats()
    ny, nx = dirty.shape
    _check(lib.clean_tiled_feedback(_ptr(dirty), ny, nx, _ptr(psf), psf.shape[0], psf.shape[1], int(tiles[0]),
                                    int(tiles[1]), int(interval), C.byref(p), _ptr(res), _ptr(idx), _ptr(flux), cap,
                                    _ptr(mod), None, 0, C.byref(st), _stream()))
    n = st.n_iter
    return dict(residual=res, idx=idx[:n], flux=flux[:n], model=mod, stats=st.as_dict())


def _batch(problems, model):
    """The host problem array of a batch and its outputs: four allocations
    shared by the whole batch, one view per problem."""
    torch = _torch()
    n = len(problems)
    arr = (Problem * max(n, 1))()
    keep, outs = [], []
    psf_dtype = None
    prep = [_prep(q["dirty"], q["psf"]) for q in problems]
    caps = [max(int(q.get("cap", q["max_iter"])), 1) for q in problems]
    # each view starts on a 256-byte boundary (64 elements) like a tensor of its own
    npix = [d.numel() for d, _ in prep]
    up = lambda v: (v + 63) // 64 * 64
    dev_ = prep[0][0].device if n else None
    if n:
        slab_r = torch.empty(sum(map(up, npix)), dtype=torch.float32, device=dev_)
        slab_i = torch.empty(sum(map(up, caps)), dtype=torch.int32, device=dev_)
        slab_f = torch.empty(sum(map(up, caps)), dtype=torch.float32, device=dev_)
        slab_m = torch.empty(sum(map(up, npix)), dtype=torch.float64, device=dev_) if model else None
    op = oc = 0
    for i, q in enumerate(problems):
        d, p = prep[i]
        if psf_dtype is None:
            psf_dtype = p.dtype
        elif p.dtype != psf_dtype:
            raise TypeError("all PSFs of a batch must share one dtype")
        cap = int(q.get("cap", q["max_iter"]))
        ny, nx = d.shape
        res = slab_r[op:op + npix[i]].view(ny, nx)
        mod = slab_m[op:op + npix[i]].view(ny, nx) if model else None
        idx, flux = slab_i[oc:oc + caps[i]], slab_f[oc:oc + caps[i]]
        op += up(npix[i])
        oc += up(caps[i])
        keep += [d, p]
        outs.append((res, idx, flux, mod))
        ty, tx = q.get("tiles", (1, 1))
        arr[i] = Problem(d.data_ptr(), p.data_ptr(), res.data_ptr(), idx.data_ptr(), flux.data_ptr(),
                         mod.data_ptr() if mod is not None else None, cap, int(q["max_iter"]),
                         float(q["threshold"]), ny, nx, p.shape[0], p.shape[1], int(ty), int(tx),
                         int(q.get("interval", 1)))
    dt = PSF_F16 if psf_dtype == torch.float16 else PSF_F32
    return arr, outs, keep, dt


def batched(problems, gain=0.1, model=True, check_finite=False, px_per_thread=0, cancel=None, level=0.0):
    """Independent Hogbom problems in one persistent launch.

    problems: list of dicts with device tensors "dirty" (float32 2-D) and "psf"
    (float32 or float16, all the same dtype), and "threshold", "max_iter",
    optional "cap", and for a tiled problem "tiles" (ty, tx) and "interval".
    level: the flux trigger of the tiled problems.  px_per_thread 0: the shape
    autotune_batched chose for this batch, else the library's rule.  Returns a
    list of dict(residual, idx, flux, model, stats).  The outputs are views
    into four allocations shared by the whole batch.
    """
    lib = load()
    n = len(problems)
    if n == 0:
        return []
    arr, outs, keep, dt = _batch(problems, model)
    prm = Params(float(gain), 0.0, 0, dt, FLAG_CHECK_FINITE if check_finite else 0, 0, int(px_per_thread),
                 float(level), _cancel(cancel))
    stats = (Stats * n)()
    _check(lib.clean_batched(arr, n, C.byref(prm), stats, _stream()))
    res = []
    for i in range(n):
        r, idx, flux, mod = outs[i]
        k = stats[i].n_iter
        res.append(dict(residual=r, idx=idx[:k], flux=flux[:k], model=mod, stats=stats[i].as_dict()))
    return res


def autotune_batched(problems, gain=0.1, trial_iter=2000, level=0.0):
    """The batch launch shape the library's tuner measures fastest: returns
    dict(px_per_thread, trial_ms) (one launch time per candidate 8, 16, 32, 64;
    -1 where it did not fit).  Later batched() calls on batches of the same
    signature with px_per_thread=0 use it."""
    lib = load()
    arr, outs, keep, dt = _batch(problems, False)
    prm = Params(float(gain), 0.0, 0, dt, 0, 0, 0, float(level), None)
    best = C.c_int32(0)
    ms = (C.c_float * 4)()
    _check(lib.clean_autotune_batched(arr, len(problems), C.byref(prm), int(trial_iter), C.byref(best), ms,
                                      _stream()))
    return dict(px_per_thread=best.value, trial_ms=[float(v) for v in ms])


def autotune(dirty, psf, tiles=(1, 1), interval=100, gain=0.1, threshold=0.0, max_iter=1000, trial_iter=2000,
             stream=False):
    """The launch shape the library's tuner measures fastest for this problem:
    returns dict(wg_per_tile, px_per_thread) to pass to hogbom/tiled_feedback."""
    lib = load()
    dirty, psf = _prep(dirty, psf)
    cap = int(min(max_iter, trial_iter))
    res, idx, flux, _ = _outputs(dirty, cap, False)
    p = _params(gain, threshold, max_iter, psf, _flags(False, stream), 0, 0)
    best = Params()
    ny, nx = dirty.shape
    _check(lib.clean_autotune(_ptr(dirty), ny, nx, _ptr(psf), psf.shape[0], psf.shape[1], int(tiles[0]),
                              int(tiles[1]), int(interval), C.byref(p), _ptr(res), _ptr(idx), _ptr(flux), cap,
                              int(trial_iter), C.byref(best), _stream()))
    return dict(wg_per_tile=best.wg_per_tile, px_per_thread=best.px_per_thread)


def autotune_interval(dirty, psf, tiles, candidates, gain=0.1, threshold=0.0, max_iter=1000, trial_iter=2000,
                      growth_limit=1.0, level=0.0, fft=False, stream=False):
    """The feedback interval the library's tuner picks among `candidates`:
    the fastest whose trial run keeps the residual finite and its peak within
    growth_limit x the dirty peak.  Returns dict(interval (0: none
    acceptable), rates, peak_ratios) with one rate and ratio per candidate."""
    lib = load()
    dirty, psf = _prep(dirty, psf)
    cap = int(min(max_iter, trial_iter))
    res, idx, flux, _ = _outputs(dirty, cap, False)
    flags = _flags(False, stream) | (FLAG_FFT_FEEDBACK if fft else 0)
    p = _params(gain, threshold, max_iter, psf, flags, 0, 0)
    p.feedback_level = float(level)
    cand = (C.c_int * len(candidates))(*[int(c) for c in candidates])
    rates = (C.c_double * len(candidates))()
    ratios = (C.c_double * len(candidates))()
    chosen = C.c_int(0)
    ny, nx = dirty.shape
    _check(lib.clean_autotune_interval(_ptr(dirty), ny, nx, _ptr(psf), psf.shape[0], psf.shape[1], int(tiles[0]),
                                       int(tiles[1]), C.cast(cand, C.c_void_p), len(candidates), C.byref(p),
                                       int(trial_iter), float(growth_limit), _ptr(res), _ptr(idx), _ptr(flux), cap,
                                       C.byref(chosen), C.cast(rates, C.c_void_p), C.cast(ratios, C.c_void_p),
                                       _stream()))
    return dict(interval=chosen.value, rates=list(rates), peak_ratios=list(ratios))


def autotune_plan(dirty, psf, grids, intervals, gain=0.1, threshold=0.0, max_iter=1000, trial_iter=None,
                  band=(-0.1, 0.1), cache_path=None, level=0.0, fft=False):
    """Tile grid and feedback interval under an accuracy budget: every
    (grid, interval) candidate gets a trial of min(trial_iter, max_iter)
    iterations beside plain CLEAN; acceptable when restored(tiled) -
    restored(plain) stays inside `band` (Jy) everywhere; the fastest
    acceptable one wins.  Returns dict(tiles, interval (0: none), wg_per_tile,
    px_per_thread, band, iters_per_s, from_cache, candidates) with every
    candidate's band and rate (not filled on a cache hit)."""
    lib = load()
    dirty, psf = _prep(dirty, psf)
    flags = FLAG_FFT_FEEDBACK if fft else 0
    p = _params(gain, threshold, max_iter, psf, flags, 0, 0)
    p.feedback_level = float(level)
    g = (C.c_int * (2 * len(grids)))(*[int(v) for gr in grids for v in gr])
    iv = (C.c_int * len(intervals))(*[int(v) for v in intervals])
    nc = len(grids) * len(intervals)
    bands = (C.c_double * (2 * nc))()
    rates = (C.c_double * nc)()
    plan = Plan()
    ny, nx = dirty.shape
    trial = int(max_iter if trial_iter is None else trial_iter)
    _check(lib.clean_autotune_plan(_ptr(dirty), ny, nx, _ptr(psf), psf.shape[0], psf.shape[1], C.cast(g, C.c_void_p),
                                   len(grids), C.cast(iv, C.c_void_p), len(intervals), C.byref(p), trial,
                                   float(band[0]), float(band[1]),
                                   cache_path.encode() if cache_path else None, C.byref(plan),
                                   C.cast(bands, C.c_void_p), C.cast(rates, C.c_void_p), _stream()))
    cands = []
    for gi, gr in enumerate(grids):
        for ii, ivl in enumerate(intervals):
            k = gi * len(intervals) + ii
            cands.append(dict(tiles=tuple(gr), interval=int(ivl), band=[bands[2 * k], bands[2 * k + 1]],
                              iters_per_s=rates[k]))
    return dict(tiles=(plan.tiles_y, plan.tiles_x), interval=plan.interval, wg_per_tile=plan.wg_per_tile,
                px_per_thread=plan.px_per_thread, band=[plan.band_min, plan.band_max],
                iters_per_s=plan.iters_per_s, from_cache=bool(plan.from_cache), candidates=cands)


def clean_beam(psf):
    """The clean beam of a device PSF: dict(area (main-lobe pixels), sigma, fwhm) in pixels."""
    torch = _torch()
    lib = load()
    psf = psf.contiguous()
    dt = PSF_F16 if psf.dtype == torch.float16 else PSF_F32
    if psf.dtype not in (torch.float16, torch.float32):
        raise TypeError("psf must be float32 or float16")
    area, sigma = C.c_int64(0), C.c_double(0.0)
    _check(lib.clean_beam_fit(_ptr(psf), psf.shape[0], psf.shape[1], dt, C.byref(area), C.byref(sigma), _stream()))
    return dict(area=area.value, sigma=sigma.value, fwhm=sigma.value * 2.0 * (2.0 * math.log(2.0)) ** 0.5)


def restore(model, residual, sigma):
    """Restored image (float64 device tensor): residual + model (*) peak-1
    Gaussian clean beam of standard deviation sigma (pixels)."""
    torch = _torch()
    lib = load()
    model = model.contiguous()
    residual = residual.contiguous()
    if model.dtype != torch.float64 or residual.dtype != torch.float32 or model.shape != residual.shape:
        raise TypeError("model must be float64 and residual float32, of one shape")
    out = torch.empty(model.shape, dtype=torch.float64, device=model.device)
    _check(lib.clean_restore(_ptr(model), _ptr(residual), model.shape[0], model.shape[1], float(sigma), _ptr(out),
                             _stream()))
    return out


def psf_to_f16(psf):
    """FP32 -> FP16 (round to nearest even) on the device."""
    torch = _torch()
    lib = load()
    psf = psf.contiguous()
    out = torch.empty(psf.shape, dtype=torch.float16, device=psf.device)
    _check(lib.clean_psf_to_f16(_ptr(psf), _ptr(out), psf.numel(), _stream()))
    return out


def set_workspace_limit(nbytes):
    """Caps the library's internal device workspace (0: no cap); returns the
    previous cap.  A call needing more fails with CLEAN_E_NOMEM."""
    return int(load().clean_set_workspace_limit(int(nbytes)))


def bandwidth_probe(buf, mode=0, reps=10):
    """GB/s that reading (mode 0) or copying half onto half (mode 1) of the
    device tensor `buf` achieves, `reps` passes (the roofline denominators)."""
    lib = load()
    _torch()
    g = C.c_double(0.0)
    _check(lib.clean_bandwidth_probe(_ptr(buf), buf.numel() * buf.element_size(), int(mode), int(reps), C.byref(g),
                                     _stream()))
    return g.value


def version():
    return load().clean_version().decode()
