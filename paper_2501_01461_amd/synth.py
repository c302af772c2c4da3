"""Seeded synthetic inputs for the Hogbom CLEAN minor loop.

This module only makes inputs: a Y-shaped interferometer's point spread function
(PSF), a point-source sky and the dirty image (sky convolved with the PSF, plus
noise).  It holds none of the CLEAN arithmetic and imports nothing else from
this package, so the CPU oracle tests, the GPU tests and the benchmark can all
draw identical inputs from it.

The paper simulates point sources seen through the VLA in configuration D, with
one very bright source (Section 1, "Introduction"; the abstract quotes sources up
to 2.1 Jy).  That dataset is not available, so these generators stand in for it:

* PSF: 27 antennas on three arms at 0/120/240 degrees, nine per arm at radii
  proportional to k**1.7 (k = 1..9), as a VLA-like Y.  Baselines are rotated
  by a seeded hour angle in U(-pi/3, pi/3) ("snapshot"), or by several angles
  spread over a short track.  The longest baseline is scaled to M/4 uv cells
  of an M x M grid; each sample adds weight 1 at its nearest cell and at the
  conjugate cell (natural weighting, no autocorrelations).  PSF = real part of
  the inverse FFT, fftshifted so the peak sits at (M/2, M/2), divided by that
  peak value.
* Sky: distinct integer pixel positions, uniform over the image; fluxes
  log-uniform in [lo, hi] Jy, plus optional extra bright sources.
* Dirty image: sky convolved with the PSF (linear, centred: the PSF centre
  lands on each source), computed by FFT in float64, plus i.i.d. Gaussian
  noise; stored as float32.
"""
from __future__ import annotations

import numpy as np

try:  # multi-threaded FFT when scipy is present
    import scipy.fft as _fft

    def _fft2(a):
        return _fft.fft2(a, workers=-1)

    def _ifft2(a):
        return _fft.ifft2(a, workers=-1)

    def _rfft2(a):
        return _fft.rfft2(a, workers=-1)

    def _irfft2(a, s):
        return _fft.irfft2(a, s=s, workers=-1)
except ImportError:  # pragma: no cover
    _fft2, _ifft2 = np.fft.fft2, np.fft.ifft2
    _rfft2 = np.fft.rfft2

    def _irfft2(a, s):
        return np.fft.irfft2(a, s=s)

SEED_ROOT = 1461

# Grids at least this large take their float64 FFTs on a torch device when the
# caller names one (the 32768^2 PSF of the 16384^2 workload needs ~60 GB and
# minutes on the host); smaller ones always use the host FFT above.
DEVICE_FFT_MIN = 16384


def _dev_irfft2_half(half: np.ndarray, M: int, device) -> np.ndarray:
    """irfft2 of a real, Hermitian-symmetric grid given by its first M/2+1 columns, on `device`."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(half)).to(device).to(torch.complex128)
    out = torch.fft.irfft2(t, s=(M, M))
    del t
    return out


def _dev_convolve(grid: np.ndarray, psf: np.ndarray, n_y: int, n_x: int, device) -> np.ndarray:
    import torch
    g = torch.fft.rfft2(torch.from_numpy(grid).to(device))
    k = torch.fft.rfft2(torch.fft.ifftshift(torch.from_numpy(psf).to(device).to(torch.float64)))
    g *= k
    del k
    out = torch.fft.irfft2(g, s=grid.shape)[:n_y, :n_x].cpu().numpy()
    del g
    torch.cuda.empty_cache()
    return out


def streams(config: int, problem: int = 0, n: int = 5):
    """Independent child generators for one (config, problem) pair.

    Order: hour angle, positions, fluxes, noise, extra.
    """
    ss = np.random.SeedSequence([SEED_ROOT, int(config), int(problem)])
    return [np.random.default_rng(s) for s in ss.spawn(n)]


def y_array_positions(n_per_arm: int = 9, exponent: float = 1.7) -> np.ndarray:
    """Antenna (x, y) positions of a Y array, arbitrary length unit."""
    pos = []
    for arm in range(3):
        ang = np.deg2rad(90.0 + 120.0 * arm)
        for k in range(1, n_per_arm + 1):
            r = float(k) ** exponent
            pos.append((r * np.cos(ang), r * np.sin(ang)))
    return np.asarray(pos, dtype=np.float64)


def y_array_psf(M: int, rng: np.random.Generator, n_samples: int = 1,
                track_rad: float = 0.0, uv_fill: float = 0.25, device=None) -> np.ndarray:
    """Y-array PSF on an M x M grid, peak exactly 1.0 at (M//2, M//2).

    n_samples == 1 is a snapshot at one seeded hour angle; n_samples > 1 spreads
    the samples evenly over track_rad radians starting at that angle.  With a
    torch `device` and M >= DEVICE_FFT_MIN the inverse FFT runs there (float64;
    the result agrees with the host FFT to rounding) and a float32 array is
    returned.
    """
    if M < 4 or M % 2:
        raise ValueError("PSF side must be even and >= 4")
    pos = y_array_positions()
    i, j = np.triu_indices(len(pos), k=1)
    base = pos[i] - pos[j]                              # (351, 2)
    scale = (uv_fill * M) / np.max(np.hypot(base[:, 0], base[:, 1]))
    theta0 = rng.uniform(-np.pi / 3.0, np.pi / 3.0)
    if n_samples == 1:
        thetas = [theta0]
    else:
        thetas = theta0 + np.linspace(0.0, track_rad, n_samples)
    grid = np.zeros((M, M), dtype=np.float64)
    for th in thetas:
        c, s = np.cos(th), np.sin(th)
        u = scale * (c * base[:, 0] - s * base[:, 1])
        v = scale * (s * base[:, 0] + c * base[:, 1])
        iu = np.floor(u + 0.5).astype(np.int64)
        iv = np.floor(v + 0.5).astype(np.int64)
        np.add.at(grid, (iv % M, iu % M), 1.0)
        np.add.at(grid, ((-iv) % M, (-iu) % M), 1.0)
    # the grid is real and symmetric under (u, v) -> (-u, -v), so its inverse
    # FFT is real: take it from the half spectrum
    if device is not None and M >= DEVICE_FFT_MIN:
        import torch
        img = _dev_irfft2_half(grid[:, :M // 2 + 1], M, device)
        del grid
        img = torch.fft.fftshift(img)
        img /= img[M // 2, M // 2].clone()
        out = img.to(torch.float32).cpu().numpy()
        del img
        torch.cuda.empty_cache()
        return out
    img = _irfft2(grid[:, :M // 2 + 1], s=(M, M))
    img = np.fft.fftshift(img)
    img /= img[M // 2, M // 2]
    return img


def random_psf(M_y: int, M_x: int, rng: np.random.Generator, spread: float = 0.6) -> np.ndarray:
    """Asymmetric test PSF: peak 1 at (M_y//2, M_x//2), every other |value| < 1.

    Used by tests so that a flipped or transposed PSF index cannot go unseen.
    """
    p = rng.uniform(-spread, spread, size=(M_y, M_x))
    p[M_y // 2, M_x // 2] = 1.0
    return p


def sky(n_y: int, n_x: int, n_src: int, lo: float, hi: float,
        rng_pos: np.random.Generator, rng_flux: np.random.Generator,
        extra=()) -> tuple[np.ndarray, np.ndarray]:
    """Point sources at distinct pixels: returns (flat indices, fluxes in Jy)."""
    n_tot = n_src + len(extra)
    idx = rng_pos.choice(n_y * n_x, size=n_tot, replace=False).astype(np.int64)
    flux = np.exp(rng_flux.uniform(np.log(lo), np.log(hi), size=n_src))
    flux = np.concatenate([flux, np.asarray(extra, dtype=np.float64)])
    return idx, flux


def convolve_sky(n_y: int, n_x: int, idx: np.ndarray, flux: np.ndarray, psf: np.ndarray,
                 device=None) -> np.ndarray:
    """dirty[q] = sum_p flux_p * psf[q - p + centre] in float64, via FFT
    (on a torch `device` for grids of DEVICE_FFT_MIN and up when one is named).

    The PSF must be at least twice the image on each axis, so no index wraps.
    """
    M_y, M_x = psf.shape
    if M_y < 2 * n_y or M_x < 2 * n_x:
        raise ValueError("PSF must be at least twice the image size")
    grid = np.zeros((M_y, M_x), dtype=np.float64)
    np.add.at(grid, (idx // n_x, idx % n_x), flux)
    if device is not None and min(M_y, M_x) >= DEVICE_FFT_MIN:
        return _dev_convolve(grid, psf, n_y, n_x, device)
    kern = np.fft.ifftshift(psf.astype(np.float64))     # centre moved to (0, 0)
    out = _irfft2(_rfft2(grid) * _rfft2(kern), s=(M_y, M_x))
    return out[:n_y, :n_x]


def dirty_image(n_y: int, n_x: int, psf: np.ndarray, idx, flux, sigma: float,
                rng_noise: np.random.Generator, device=None) -> np.ndarray:
    d = convolve_sky(n_y, n_x, idx, flux, psf, device)
    if sigma > 0:
        d = d + rng_noise.normal(0.0, sigma, size=d.shape)
    return d


# --------------------------------------------------------------------------
# The workloads.  Sizes, source counts, flux ranges and stopping rules follow
# the five benchmark configurations; "psf_track" selects a 10-minute snapshot
# (2.5 degrees of rotation, 6 samples) instead of a single instant.
# --------------------------------------------------------------------------

CONFIGS = {
    0: dict(name="plain-256", n=256, n_src=20, lo=0.01, hi=1.0, extra=(2.1,), sigma=1e-3,
            gain=0.1, threshold=5e-3, max_iter=1000, tiles=(1, 1), interval=None),
    1: dict(name="tiled2x2-1024", n=1024, n_src=200, lo=0.005, hi=2.1, extra=(), sigma=1e-3,
            gain=0.1, threshold=0.0, max_iter=20000, tiles=(2, 2), interval=100),
    2: dict(name="tiled8x8-4096", n=4096, n_src=2000, lo=0.001, hi=2.1, extra=(), sigma=1e-3,
            gain=0.1, threshold=0.0, max_iter=200000, tiles=(8, 8), interval=200),
    4: dict(name="tiled16x16-16384", n=16384, n_src=20000, lo=0.001, hi=2.1, extra=(2.1,) * 5,
            sigma=1e-3, gain=0.1, threshold=5e-3, max_iter=1000000, tiles=(16, 16), interval=None),
}

BATCH_SIDES = (128, 192, 256, 384, 512, 768, 1024)


def make_problem(n: int, n_src: int, lo: float, hi: float, extra, sigma: float,
                 config: int, problem: int = 0, psf_track: bool = False,
                 psf_factor: int = 2, device=None) -> tuple[np.ndarray, np.ndarray, dict]:
    """(dirty float32 [n, n], psf float32 [psf_factor*n]^2, info)."""
    r_ha, r_pos, r_flux, r_noise, _ = streams(config, problem)
    M = psf_factor * n
    if psf_track:
        psf = y_array_psf(M, r_ha, n_samples=6, track_rad=np.deg2rad(2.5), device=device)
    else:
        psf = y_array_psf(M, r_ha, device=device)
    psf32 = psf.astype(np.float32, copy=False)
    del psf
    idx, flux = sky(n, n, n_src, lo, hi, r_pos, r_flux, extra)
    # the dirty image is made with the float32-stored PSF, the one CLEAN sees
    if device is not None and M >= DEVICE_FFT_MIN:
        d = dirty_image(n, n, psf32, idx, flux, sigma, r_noise, device)
    else:
        d = dirty_image(n, n, psf32.astype(np.float64), idx, flux, sigma, r_noise)
    info = dict(src_idx=idx, src_flux=flux, brightest=float(flux.max()))
    return d.astype(np.float32), psf32, info


def make_config(k: int, psf_track: bool = False, device=None):
    """Inputs and parameters of one of the single-image workloads (0, 1, 2, 4).

    `device` (a torch device) only matters for workload 4, whose float64 FFTs
    then run there."""
    c = dict(CONFIGS[k])
    dirty, psf, info = make_problem(c["n"], c["n_src"], c["lo"], c["hi"], c["extra"], c["sigma"],
                                    config=k, psf_track=psf_track, device=device)
    c.update(dirty=dirty, psf=psf, info=info)
    return c


def make_batch(n_problems: int = 256, config: int = 3, sides=BATCH_SIDES,
               src_range=(5, 200), lo: float = 0.005, hi: float = 2.1,
               sigma: float = 1e-3):
    """The batched workload: uneven images, each with its own PSF at twice its side."""
    r_meta = streams(config, 1_000_000)[0]
    side = r_meta.choice(np.asarray(sides), size=n_problems)
    nsrc = r_meta.integers(src_range[0], src_range[1] + 1, size=n_problems)
    probs = []
    for i in range(n_problems):
        d, p, info = make_problem(int(side[i]), int(nsrc[i]), lo, hi, (), sigma, config=config, problem=i)
        probs.append(dict(dirty=d, psf=p, info=info, n=int(side[i]), threshold=5.0 * sigma))
    return probs
