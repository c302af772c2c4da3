"""Pins of the oracle's non-finite path (CPU).

The paper's minor loop (Section 3: find the highest-intensity pixel, append
gain x value, subtract gain x value x PSF) never meets a non-finite value on
converging input, but the tiled form can diverge (the interval and the PSF's
sidelobes decide it), and then values overflow to infinity and NaN.  The
reading pinned here:

- the peak search orders |r| as magnitudes with every NaN above +Inf and all
  NaNs equal (lowest row-major index on ties, as for finite values);
- a non-finite peak ends the run with stop reason 4 ("non-finite") before
  anything is appended; plain CLEAN tests it right after n == max_iter, the
  tiled form tests every tile's peak at a round's start, and a non-finite
  local peak ends that tile's round (which still ends with its feedback).

Each pin is independent of the oracle's own code: a Python brute force of the
order, overflow cases whose every value follows by hand, and the stop rule's
defining property on runs that diverge.
"""
import math

import numpy as np
import pytest

import oracle

STOP_MAXITER, STOP_THRESHOLD, STOP_CAPACITY, STOP_NONFINITE = 0, 1, 2, 4
F32_MAX = float(np.finfo(np.float32).max)


def same_nan_aware(a, b):
    """Bitwise equal, except that NaN matches NaN whatever its sign or payload."""
    a, b = np.asarray(a), np.asarray(b)
    if a.shape != b.shape or a.dtype != b.dtype:
        return False
    na, nb = np.isnan(a), np.isnan(b)
    if not np.array_equal(na, nb):
        return False
    u = np.uint32 if a.dtype == np.float32 else np.uint64
    return np.array_equal(a[~na].view(u), b[~nb].view(u))


# ---------------------------------------------------------- peak order ----

def brute_peak(a, rect=None):
    """Lowest row-major index of the largest |a|, NaN above +Inf, NaNs equal
    (Python float comparisons, no bit patterns)."""
    y0, y1, x0, x1 = rect if rect is not None else (0, a.shape[0], 0, a.shape[1])
    best, bkey = None, None
    for y in range(y0, y1):
        for x in range(x0, x1):
            v = float(a[y, x])
            key = (1, 0.0) if math.isnan(v) else (0, abs(v))
            if bkey is None or key > bkey:
                best, bkey = y * a.shape[1] + x, key
    return best


def special_array(shape, seed, dtype):
    """Random values with NaNs of random sign and payload, +-Inf, +-0,
    subnormals and repeated magnitudes."""
    r = np.random.default_rng([91, seed])
    a = r.normal(0, 1, shape).astype(dtype)
    n = a.size
    flat = a.reshape(-1)
    kinds = r.integers(0, 9, n)
    ib = np.uint32 if dtype == np.float32 else np.uint64
    bits = flat.view(ib)
    exp_all = ib(0x7F800000) if dtype == np.float32 else ib(0x7FF0000000000000)
    mant = ib(0x007FFFFF) if dtype == np.float32 else ib(0x000FFFFFFFFFFFFF)
    sign = ib(0x80000000) if dtype == np.float32 else ib(0x8000000000000000)
    for i in range(n):
        k = kinds[i]
        if k == 0 and r.random() < 0.3:        # NaN, random payload and sign
            m = ib(int(r.integers(1, int(mant) + 1)))
            bits[i] = exp_all | m | (sign if r.random() < 0.5 else ib(0))
        elif k == 1 and r.random() < 0.3:      # +-Inf
            bits[i] = exp_all | (sign if r.random() < 0.5 else ib(0))
        elif k == 2:                          # +-0
            bits[i] = sign if r.random() < 0.5 else ib(0)
        elif k == 3:                          # subnormal
            bits[i] = ib(int(r.integers(1, int(mant) + 1))) | (sign if r.random() < 0.5 else ib(0))
        elif k == 4:                          # repeat an earlier magnitude, either sign
            j = int(r.integers(0, i + 1))
            bits[i] = (bits[j] & ~sign) | (sign if r.random() < 0.5 else ib(0))
    return a


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("seed", range(40))
def test_peak_order_brute_force(dtype, seed):
    a = special_array((5, 7), seed, dtype)
    assert oracle.peak(a) == brute_peak(a)
    rect = (1, 4, 2, 6)
    assert oracle.peak(a, rect) == brute_peak(a, rect)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_peak_order_special_cases(dtype):
    z = np.zeros((2, 4), dtype)
    z[0, 3] = np.inf
    z[1, 0] = -np.inf
    assert oracle.peak(z) == 3                 # +Inf and -Inf tie: lower index
    z[1, 2] = np.nan
    assert oracle.peak(z) == 6                 # NaN above every infinity
    z[0, 1] = -np.nan
    assert oracle.peak(z) == 1                 # NaNs tie whatever their sign
    n = np.zeros((1, 3), dtype)
    n[0, 0] = -0.0
    assert oracle.peak(n) == 0                 # +-0 tie


# ------------------------------------------------------------ plain stop --

@pytest.mark.parametrize("precision", ["f32", "f64"])
@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf])
def test_plain_nonfinite_input_stops_at_once(precision, bad):
    d = np.random.default_rng([92]).normal(0, 1, (6, 8)).astype(np.float32)
    d[4, 5] = bad
    psf = np.zeros((12, 16), np.float32)
    psf[6, 8] = 1.0
    o = oracle.hogbom(d, psf, 0.1, 0.0, 10, precision=precision)
    assert o["n_iter"] == 0 and o["stop"] == STOP_NONFINITE
    assert same_nan_aware(o["residual"], d.astype(o["residual"].dtype))
    # n == max_iter is tested first
    o = oracle.hogbom(d, psf, 0.1, 0.0, 0, precision=precision)
    assert o["stop"] == STOP_MAXITER


def chain_case(nx=16):
    """One row; the PSF is 1 at its centre and -a one pixel to the right, so
    with gain 1 each iteration zeroes the peak and multiplies the next pixel
    by a: after k iterations pixel k holds a^(k+1) (one rounding per product)."""
    a = 3.0e38
    d = np.zeros((1, nx), np.float32)
    d[0, 0] = a
    psf = np.zeros((2, 2 * nx), np.float32)
    psf[1, nx] = 1.0
    psf[1, nx + 1] = -a
    return d, psf, float(np.float32(a))


def test_plain_overflow_closed_form_f32():
    d, psf, a = chain_case()
    o = oracle.hogbom(d, psf, 1.0, 0.0, 50)
    # iteration 1: c = a; pixel 0 -> fma(-a, 1, a) = 0; pixel 1 -> fma(-a, -a, 0) = +Inf
    assert o["n_iter"] == 1 and o["stop"] == STOP_NONFINITE
    assert list(o["idx"]) == [0] and o["flux"][0] == np.float32(a)
    want = np.zeros((1, 16), np.float32)
    want[0, 1] = np.inf
    assert same_nan_aware(o["residual"], want)
    assert o["model"][0, 0] == a and np.count_nonzero(o["model"]) == 1


def test_plain_overflow_closed_form_f64():
    d, psf, a = chain_case()
    o = oracle.hogbom(d, psf, 1.0, 0.0, 50, precision="f64")
    # pixel k holds a^(k+1) until that overflows float64: a^9 > 1.8e308
    vals, v = [], a
    while math.isfinite(v):
        vals.append(v)
        v = v * a
    assert len(vals) == 8
    assert o["n_iter"] == 8 and o["stop"] == STOP_NONFINITE
    assert list(o["idx"]) == list(range(8))
    assert [float(x) for x in o["flux"]] == vals
    want = np.zeros((1, 16), np.float64)
    want[0, 8] = np.inf
    assert same_nan_aware(o["residual"], want)


@pytest.mark.parametrize("precision", ["f32", "f64"])
@pytest.mark.parametrize("seed", range(4))
def test_plain_stops_at_the_first_nonfinite_peak(precision, seed):
    """The defining property on runs that diverge: after n_iter iterations
    the residual holds a non-finite value, after n_iter - 1 it holds none,
    and stopping early at max_iter gives the same prefix."""
    r = np.random.default_rng([93, seed])
    ny, nx = 9, 12
    d = r.normal(0, 1, (ny, nx)).astype(np.float32)
    psf = r.uniform(-40.0, 40.0, (2 * ny, 2 * nx)).astype(np.float32)
    psf[ny, nx] = 1.0
    o = oracle.hogbom(d, psf, 1.0, 0.0, 10000, precision=precision)
    n = o["n_iter"]
    assert o["stop"] == STOP_NONFINITE and 1 <= n < 10000
    assert not np.all(np.isfinite(o["residual"]))
    assert np.all(np.isfinite(o["flux"]))
    p = oracle.hogbom(d, psf, 1.0, 0.0, n - 1, precision=precision)
    assert p["stop"] == STOP_MAXITER and np.all(np.isfinite(p["residual"]))
    assert np.array_equal(p["idx"], o["idx"][:n - 1])
    q = oracle.hogbom(d, psf, 1.0, 0.0, n, precision=precision)
    assert q["stop"] == STOP_MAXITER and same_nan_aware(q["residual"], o["residual"])


# ------------------------------------------------------------ tiled stop --

def test_tiled_overflow_in_feedback_closed_form():
    """Two 2 x 2 tiles.  Tile 0 removes a = 3e38 at (0, 0) in round 1 (tile 1
    is below the threshold); the feedback puts fma(a, -a, 0) = -Inf into the
    sum at (0, 2), so r(0, 2) = 0 - (-Inf) = +Inf, and round 2 stops."""
    a = float(np.float32(3.0e38))
    d = np.zeros((2, 4), np.float32)
    d[0, 0] = a
    psf = np.zeros((4, 8), np.float32)
    psf[2, 4] = 1.0
    psf[2, 6] = -a                  # offset (0, +2): from (0, 0) onto (0, 2)
    for level in (0.0, 0.5):
        o = oracle.tiled(d, psf, (1, 2), 1, 1.0, 1e-3, 10, level=level)
        assert o["n_iter"] == 1 and o["n_rounds"] == 1 and o["stop"] == STOP_NONFINITE
        assert list(o["idx"]) == [0] and o["flux"][0] == np.float32(a)
        want = np.zeros((2, 4), np.float32)
        want[0, 2] = np.inf
        assert same_nan_aware(o["residual"], want)


def test_tiled_local_overflow_ends_the_round():
    """Tile 0's first local iteration overflows inside the tile; its next
    local peak is +Inf, which ends its round (interval 5) like a peak below
    the threshold would.  Tile 1 removes its own source meanwhile; the round
    ends with both components fed back, and round 2 stops."""
    a = float(np.float32(3.0e38))
    d = np.zeros((2, 4), np.float32)
    d[0, 0] = a
    d[0, 3] = 1.0                   # its (0, +1) neighbour lies outside the image
    psf = np.zeros((4, 8), np.float32)
    psf[2, 4] = 1.0
    psf[2, 5] = -a                  # offset (0, +1): from (0, 0) onto (0, 1), same tile
    o = oracle.tiled(d, psf, (1, 2), 5, 1.0, 1e-3, 10)
    assert o["n_rounds"] == 1 and o["stop"] == STOP_NONFINITE
    assert list(o["idx"]) == [0, 3]
    assert o["flux"][0] == np.float32(a) and o["flux"][1] == np.float32(1.0)
    want = np.zeros((2, 4), np.float32)
    want[0, 1] = np.inf
    assert same_nan_aware(o["residual"], want)


@pytest.mark.parametrize("precision", ["f32", "f64"])
@pytest.mark.parametrize("level", [0.0, 0.5])
def test_tiled_nonfinite_input_stops_at_once(precision, level):
    d = np.random.default_rng([94]).normal(0, 1, (8, 8)).astype(np.float32)
    d[6, 1] = np.nan
    psf = np.zeros((16, 16), np.float32)
    psf[8, 8] = 1.0
    o = oracle.tiled(d, psf, (2, 2), 4, 0.1, 0.0, 40, precision=precision, level=level)
    assert o["n_iter"] == 0 and o["n_rounds"] == 0 and o["stop"] == STOP_NONFINITE


@pytest.mark.parametrize("precision", ["f32", "f64"])
@pytest.mark.parametrize("seed,level", [(0, 0.0), (1, 0.0), (2, 0.5), (3, 0.3)])
def test_tiled_stops_at_the_first_nonfinite_round(precision, seed, level):
    """Diverging tiled runs: at the stop the residual holds a non-finite
    value; run with max_iter = n_iter (the stop rule n == max_iter comes
    first) the same components come back with a MAXITER stop."""
    r = np.random.default_rng([95, seed])
    ny, nx = 16, 20
    d = r.normal(0, 1, (ny, nx)).astype(np.float32)
    psf = r.uniform(-30.0, 30.0, (2 * ny, 2 * nx)).astype(np.float32)
    psf[ny, nx] = 1.0
    o = oracle.tiled(d, psf, (2, 2), 6, 1.0, 0.0, 100000, precision=precision, level=level)
    n = o["n_iter"]
    assert o["stop"] == STOP_NONFINITE and 1 <= n < 100000
    assert not np.all(np.isfinite(o["residual"]))
    assert np.all(np.isfinite(o["flux"]))
    q = oracle.tiled(d, psf, (2, 2), 6, 1.0, 0.0, n, precision=precision, level=level)
    assert q["stop"] == STOP_MAXITER and q["n_rounds"] == o["n_rounds"]
    assert np.array_equal(q["idx"], o["idx"])
    assert same_nan_aware(q["residual"], o["residual"])
