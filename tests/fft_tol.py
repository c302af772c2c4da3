"""Error bounds for the FFT form of the feedback step (test infrastructure).

The FFT form computes, per round, z = c (*) K by z = F^-1(F c . F K) / N in
float32, with F the 2-D radix-2 transform of size N = Lx * Ly (log2 N stages)
and twiddles rounded once from double.  The normwise bound for one computed
radix-2 transform (Higham, Accuracy and Stability of Numerical Algorithms,
2nd ed., Thm. 24.2) is  ||fl(F x) - F x||_2 <= a ||F x||_2  with
a = log2(N) eta / (1 - log2(N) eta),  eta = mu + gamma_4 (sqrt(2) + mu),
mu the twiddle error (u here).  Through the pointwise product and the
inverse transform, with ||F x||_2 = sqrt(N) ||x||_2 and ||F x||_inf <= ||x||_1:

    ||z_hat - z||_inf <= ||z_hat - z||_2
                      <= (3 a + 4 u) (||c||_2 ||K||_1 + ||c||_1 ||K||_2)

(two forward transforms, one inverse, one complex product and the 1/N
scale, first order in u).  That bound is rigorous but, going through the
2-norm, sits ~1e4 above the max-abs error seen in practice, too loose to tell
a dropped component from rounding.  The tolerance the tests apply is the
first-order estimate behind it taken per element: each of the log2 N stages
of each of the three transforms rounds values no larger than the result's
scale S = max |c (*) K| once (relative u), so

    |z_hat - z| <= 2 u log2(N) S        (tolerance),

about 1e-6 of S for the image sizes here.  The own-tile part subtracted from
z (and the float32 oracle's own chain) is a direct float32 sum of at most n
terms, bounded per pixel by gamma(n) A(q) with A = |c| (*) |K| (float64,
exact to rounding).  gamma(n) is taken in the probabilistic form of Higham and
Mary (SIAM J. Sci. Comput. 41(5), 2019): lambda sqrt(n) u, lambda = 6, which
holds with probability at least 1 - 2n exp(-lambda^2 (1-u)^2 / 2) under their
model of independent rounding errors (worst case: n u).
"""
import math

import numpy as np

U32 = 2.0 ** -24


def transform_alpha(log2n, u=U32):
    mu = u
    g4 = 4 * u / (1 - 4 * u)
    eta = mu + g4 * (math.sqrt(2.0) + mu)
    return log2n * eta / (1 - log2n * eta)


def fft_sizes(ny, nx):
    lgx = max(1, math.ceil(math.log2(2 * nx - 1)))
    lgy = max(1, math.ceil(math.log2(2 * ny - 1)))
    return lgy, lgx


def kernel_window(psf, ny, nx):
    """K(d) = psf[centre + d] for |d| < (ny, nx), as a float64 array."""
    cy, cx = psf.shape[0] // 2, psf.shape[1] // 2
    return np.asarray(psf[cy - ny + 1:cy + ny, cx - nx + 1:cx + nx], dtype=np.float64)


def convolution_bound(c_img, psf):
    """Normwise bound on the max-abs error of the float32 FFT convolution."""
    ny, nx = c_img.shape
    lgy, lgx = fft_sizes(ny, nx)
    K = kernel_window(psf, ny, nx)
    c = np.asarray(c_img, np.float64)
    a = transform_alpha(lgx + lgy)
    c2, c1 = np.sqrt(np.sum(c * c)), np.sum(np.abs(c))
    k2, k1 = np.sqrt(np.sum(K * K)), np.sum(np.abs(K))
    return (3 * a + 4 * U32) * (c2 * k1 + c1 * k2)


LAMBDA = 6.0


def gamma_prob(n, u=U32):
    """Probabilistic constant for a sum of n rounded terms (Higham-Mary)."""
    return LAMBDA * math.sqrt(max(n, 1)) * u


def transform_term(c_img, psf):
    """2 u log2(N) max |c (*) K|: the per-element estimate for the transforms."""
    ny, nx = c_img.shape
    lgy, lgx = fft_sizes(ny, nx)
    S = np.abs(library_fft_convolution(c_img, psf, single=False)).max()
    return 2 * U32 * (lgx + lgy) * S


def abs_convolution(c_img, psf):
    """A(q) = sum_p |c(p)| |K(q - p)|, float64."""
    return library_fft_convolution(np.abs(c_img), np.abs(np.asarray(psf, np.float64)), single=False)


def feedback_tolerance(c_img, psf, n_terms):
    """Per-pixel tolerance (array) on the FFT-form cross-coupling of one round
    against the float32 direct chain: the transform estimate, plus the
    direct float32 sums on both sides (own part here, the chain there), each
    of at most n_terms terms."""
    A = abs_convolution(c_img, psf)
    return transform_term(c_img, psf) + 2 * (gamma_prob(n_terms) + U32) * A


def component_image(ny, nx, idx, flux):
    """Per-position float64 sums of the components (aggregated as the feedback does)."""
    c = np.zeros(ny * nx, np.float64)
    np.add.at(c, np.asarray(idx, np.int64), np.asarray(flux, np.float64))
    return c.reshape(ny, nx)


def tile_of(ny, nx, ty, tx, idx):
    """Tile index of each pixel index under the floor split of Section 2."""
    idx = np.asarray(idx, np.int64)
    y, x = idx // nx, idx % nx
    edges_y = (np.arange(ty + 1, dtype=np.int64) * ny) // ty
    edges_x = (np.arange(tx + 1, dtype=np.int64) * nx) // tx
    ti = np.searchsorted(edges_y, y, side="right") - 1
    tj = np.searchsorted(edges_x, x, side="right") - 1
    return (ti * tx + tj).astype(np.int32)


def library_fft_convolution(c_img, psf, single=True):
    """c (*) K on the padded grid with scipy.fft, in complex64 or complex128,
    cropped to the image window."""
    import scipy.fft as sf
    ny, nx = c_img.shape
    lgy, lgx = fft_sizes(ny, nx)
    Ly, Lx = 1 << lgy, 1 << lgx
    ct = np.complex64 if single else np.complex128
    K = kernel_window(psf, ny, nx)
    kp = np.zeros((Ly, Lx), ct)
    # place K(d) at (d mod Ly, d mod Lx)
    dy = np.arange(-ny + 1, ny) % Ly
    dx = np.arange(-nx + 1, nx) % Lx
    kp[np.ix_(dy, dx)] = K.astype(ct)
    cp = np.zeros((Ly, Lx), ct)
    cp[:ny, :nx] = c_img.astype(ct)
    z = sf.ifft2(sf.fft2(cp) * sf.fft2(kp))
    return np.asarray(z[:ny, :nx].real, np.float64)
