"""CPU checks of the FFT-feedback error bound used by the GPU tests.

A float32 FFT convolution from a library (scipy.fft in single precision) must
stay within the normwise bound, and the bound must be far below the size of a
single component's contribution, or the GPU check could not tell a dropped or
misplaced component from rounding.
"""
import numpy as np
import pytest

from paper_2501_01461_amd import synth
from tests import fft_tol


@pytest.mark.parametrize("ny,nx,ncomp,seed", [(64, 64, 200, 1), (50, 62, 120, 2), (96, 80, 300, 3)])
def test_library_float32_fft_within_bound(ny, nx, ncomp, seed):
    r = np.random.default_rng([31, seed])
    psf = synth.random_psf(2 * ny, 2 * nx + 2, r, 0.2).astype(np.float32)
    idx = r.choice(ny * nx, ncomp, replace=False)
    flux = r.uniform(-0.2, 0.2, ncomp).astype(np.float32)
    c = fft_tol.component_image(ny, nx, idx, flux)
    z32 = fft_tol.library_fft_convolution(c, psf, single=True)
    # float64 direct sum as the exact value
    cy, cx = psf.shape[0] // 2, psf.shape[1] // 2
    z = np.zeros((ny, nx))
    ys, xs = np.arange(ny)[:, None], np.arange(nx)[None, :]
    for p, f in zip(idx, flux):
        py, px = divmod(int(p), nx)
        z += float(f) * psf[cy + ys - py, cx + xs - px].astype(np.float64)
    err = np.abs(z32 - z).max()
    assert err <= fft_tol.convolution_bound(c, psf)
    # the float64 library form agrees with the direct sum to rounding
    assert np.abs(fft_tol.library_fft_convolution(c, psf, single=False) - z).max() < 1e-10
    # the per-element tolerance admits a correct float32 FFT with margin ...
    tol = fft_tol.transform_term(c, psf)
    assert err <= tol / 4, (err, tol)
    # ... and lies far below one component's contribution at the PSF peak
    assert tol < 1e-3 * np.median(np.abs(flux)), (tol, np.median(np.abs(flux)))
    # the direct float32 sum in the oracle's order stays within the
    # probabilistic per-pixel bound used beside it
    z32d = np.zeros((ny, nx), np.float32)
    for p, f in zip(idx, flux):
        py, px = divmod(int(p), nx)
        z32d = (np.float32(f) * psf[cy + ys - py, cx + xs - px] + z32d).astype(np.float32)
    A = fft_tol.abs_convolution(c, psf)
    assert np.all(np.abs(z32d - z) <= (fft_tol.gamma_prob(ncomp) + fft_tol.U32) * A + 1e-30)


def test_tile_of_matches_floor_split():
    ny, nx, ty, tx = 50, 62, 3, 4
    idx = np.arange(ny * nx)
    t = fft_tol.tile_of(ny, nx, ty, tx, idx)
    for q in range(0, ny * nx, 7):
        y, x = divmod(q, nx)
        ti = max(i for i in range(ty) if (i * ny) // ty <= y)
        tj = max(j for j in range(tx) if (j * nx) // tx <= x)
        assert t[q] == ti * tx + tj
