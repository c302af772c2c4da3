"""GPU parity of the FFT form of the feedback step (CLEAN_FLAG_FFT_FEEDBACK).

The FFT form computes the same residual update as the direct form (Section 3:
each tile's components convolved with the full PSF, subtracted from the other
tiles, after each tile subtracted its own) as the round's starting residual
minus one convolution of all the round's components, so it rounds differently
and is held to a tolerance (tests/fft_tol.py) rather than to the oracle's bits:

* one round (max_iter = tiles x interval): the local minor loops do not see
  feedback, so components and model are bit-exact against the float32
  oracle, and the residual is within the per-round feedback tolerance;
* several rounds: the invariant residual = dirty - components (*) PSF holds
  to the accumulated tolerance, round 1 is bit-exact, and component positions
  follow the oracle's until a divergence that is a near-tie at the scale of
  the observed flux drift (both picks are then correct).
"""
import numpy as np
import pytest

import oracle
from paper_2501_01461_amd import synth
from tests import fft_tol
from tests.gpu_util import announce, bits, dev, host

pytestmark = pytest.mark.gpu

U = fft_tol.U32


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2501_01461_amd as P
    P.load()
    return P


def sparse_dirty(ny, nx, seed, density=0.03, noise=0.02):
    r = np.random.default_rng([13, seed])
    d = r.normal(0, noise, (ny, nx)) + (r.random((ny, nx)) < density) * r.uniform(-2, 2, (ny, nx))
    return d.astype(np.float32)


def asym_psf(My, Mx, seed, spread=0.2):
    return synth.random_psf(My, Mx, np.random.default_rng([14, seed]), spread).astype(np.float32)


def round_tolerance(ny, nx, tiles, idx, flux, psf, start=None):
    """Per-pixel tolerance on one round's residual update: FFT estimate for
    the round's component image, the direct float32 sums (the oracle's own
    local updates and cross chain), and, given the round-start residual, the
    local chain's rounding of values no larger than |start| + A."""
    c = fft_tol.component_image(ny, nx, idx, flux)
    tol = fft_tol.feedback_tolerance(c, psf, len(idx))
    if start is not None:
        A = fft_tol.abs_convolution(c, psf)
        tol = tol + fft_tol.gamma_prob(len(idx)) * (np.abs(start).astype(np.float64) + A)
    return tol


def check_one_round(out, ref, psf, tiles, dirty):
    st = out["stats"]
    assert st["n_rounds"] == ref["n_rounds"] == 1
    assert st["n_iter"] == ref["n_iter"] and st["stop_reason"] == ref["stop"]
    gi, gf = host(out["idx"]), host(out["flux"])
    assert np.array_equal(gi, ref["idx"])
    assert np.array_equal(bits(gf), bits(ref["flux"]))
    assert np.array_equal(bits(host(out["model"])), bits(ref["model"]))
    gr = host(out["residual"]).astype(np.float64)
    ny, nx = gr.shape
    tol = round_tolerance(ny, nx, tiles, gi, gf, psf, dirty) + 2 * U * np.abs(ref["residual"]).astype(np.float64)
    err = np.abs(gr - ref["residual"])
    print(f"one round: max |gpu - oracle| {err.max():.3e}, tolerance min {tol.min():.3e} max {tol.max():.3e}, "
          f"max err/tol {(err / tol).max():.3f}")
    assert np.all(err <= tol), (err.max(), np.unravel_index(np.argmax(err - tol), err.shape))
    assert err.max() > 0 or len(gi) <= 1   # the FFT form really ran (it does not round like the chain)


ONE_ROUND = [
    # ny, nx, tiles, interval, seed, stream, f16
    (64, 64, (2, 2), 50, 61, False, False),
    (96, 80, (3, 2), 30, 62, False, False),      # ragged tiles, width not a multiple of 4 per tile
    (50, 62, (2, 2), 40, 63, True, False),       # residual streamed through HBM
    (128, 96, (4, 3), 20, 64, False, True),      # FP16-stored PSF
    (33, 200, (1, 4), 25, 65, False, False),     # wide and short: Lx 512, Ly 128
]


@pytest.mark.parametrize("two", [False, True], ids=["one-level", "two-level"])
@pytest.mark.parametrize("case", ONE_ROUND, ids=[f"{c[0]}x{c[1]}-{c[2][0]}x{c[2][1]}-I{c[3]}" + ("-stream" if c[5] else "")
                                                  + ("-f16" if c[6] else "") for c in ONE_ROUND])
def test_fft_one_round_small(lib, case, two):
    import torch
    ny, nx, tiles, interval, seed, stream, f16 = case
    announce("fft one round", case, "two-level" if two else "one-level")
    dirty = sparse_dirty(ny, nx, seed)
    psf = asym_psf(2 * ny, 2 * nx + 2, seed)
    n = tiles[0] * tiles[1] * interval
    psf_ref = psf.astype(np.float16).astype(np.float32) if f16 else psf
    ref = oracle.tiled(dirty, psf_ref, tiles, interval, 0.1, 0.0, n)
    dpsf = dev(psf).to(torch.float16) if f16 else dev(psf)
    out = lib.tiled_feedback(dev(dirty), dpsf, tiles, interval, 0.1, 0.0, n, stream=stream, fft=True,
                             fft_two_level=two)
    check_one_round(out, ref, psf_ref, tiles, dirty)


# The wide tile (px_per_thread = 128) at small sizes: its kernel takes the
# radix-16 transform passes and the fused column sweeps, at odd and even
# transform lengths (radix-2 and radix-4 leftovers), with the x phases' row
# pairs grouped by XCD.
WIDE_ONE_ROUND = [
    # ny, nx, tiles, interval, seed, f16
    (64, 64, (2, 2), 50, 81, False),           # Lx = Ly = 128: radix-2, one radix-16, one radix-4 pass
    (96, 128, (3, 2), 30, 82, False),          # 256: two radix-16 passes
    (128, 128, (4, 4), 20, 83, True),          # FP16-stored PSF
    (250, 256, (2, 2), 40, 84, False),         # 512; ragged 125-row tiles
]


@pytest.mark.parametrize("two", [False, True], ids=["one-level", "two-level"])
@pytest.mark.parametrize("case", WIDE_ONE_ROUND, ids=[f"{c[0]}x{c[1]}-{c[2][0]}x{c[2][1]}-I{c[3]}"
                                                       + ("-f16" if c[5] else "") for c in WIDE_ONE_ROUND])
def test_fft_one_round_wide_tile(lib, case, two):
    import torch
    ny, nx, tiles, interval, seed, f16 = case
    announce("fft one round wide tile", case, "two-level" if two else "one-level")
    dirty = sparse_dirty(ny, nx, seed)
    psf = asym_psf(2 * ny, 2 * nx + 2, seed)
    n = tiles[0] * tiles[1] * interval
    psf_ref = psf.astype(np.float16).astype(np.float32) if f16 else psf
    ref = oracle.tiled(dirty, psf_ref, tiles, interval, 0.1, 0.0, n)
    dpsf = dev(psf).to(torch.float16) if f16 else dev(psf)
    out = lib.tiled_feedback(dev(dirty), dpsf, tiles, interval, 0.1, 0.0, n, fft=True, fft_two_level=two,
                             px_per_thread=128)
    assert out["stats"]["px_per_thread"] == 128 and out["stats"]["streamed"] == 0
    check_one_round(out, ref, psf_ref, tiles, dirty)


@pytest.mark.parametrize("case", [(64, 64, (2, 2), 20, 85, 1000, 0.0), (96, 128, (3, 2), 25, 86, 1200, 0.5)],
                         ids=["64x64-2x2-I20", "96x128-3x2-I25-f0.5"])
def test_fft_many_rounds_wide_tile(lib, case):
    ny, nx, tiles, interval, seed, n, level = case
    announce("fft many rounds wide tile", case)
    dirty = sparse_dirty(ny, nx, seed)
    psf = asym_psf(2 * ny, 2 * nx + 2, seed)
    ref = oracle.tiled(dirty, psf, tiles, interval, 0.1, 0.0, n, level=level)
    out = lib.tiled_feedback(dev(dirty), dev(psf), tiles, interval, 0.1, 0.0, n, level=level, fft=True,
                             px_per_thread=128)
    assert out["stats"]["px_per_thread"] == 128
    check_many_rounds(out, ref, dirty, psf, tiles, interval)


@pytest.mark.parametrize("two", [False, True], ids=["one-level", "two-level"])
def test_fft_one_round_config1(lib, two):
    """1024^2 image, 2048^2 snapshot PSF, 2x2 tiles, interval 100: one round (400 components)."""
    announce("fft one round config1", "two-level" if two else "one-level")
    c = synth.make_config(1)
    n = 4 * c["interval"]
    ref = oracle.tiled(c["dirty"], c["psf"], c["tiles"], c["interval"], 0.1, 0.0, n)
    out = lib.tiled_feedback(dev(c["dirty"]), dev(c["psf"]), c["tiles"], c["interval"], 0.1, 0.0, n, fft=True,
                             fft_two_level=two)
    check_one_round(out, ref, c["psf"], c["tiles"], c["dirty"])


@pytest.fixture(scope="module")
def config2():
    return synth.make_config(2)


@pytest.mark.parametrize("f16", [False, True], ids=["f32", "f16"])
def test_fft_one_round_config2(lib, config2, f16):
    """4096^2 image, 8192^2 PSF, 8x8 tiles, interval 10: one round (640
    components), transforms of length 8192, residual streamed."""
    import torch
    announce("fft one round config2", f16)
    c = config2
    psf_ref = c["psf"].astype(np.float16).astype(np.float32) if f16 else c["psf"]
    ref = oracle.tiled(c["dirty"], psf_ref, (8, 8), 10, 0.1, 0.0, 640)
    dpsf = dev(c["psf"]).to(torch.float16) if f16 else dev(c["psf"])
    out = lib.tiled_feedback(dev(c["dirty"]), dpsf, (8, 8), 10, 0.1, 0.0, 640, fft=True)
    check_one_round(out, ref, psf_ref, (8, 8), c["dirty"])


# ------------------------------------------------------------ many rounds --

def invariant_error(dirty, psf, idx, flux, residual):
    """|residual - (dirty - components (*) PSF)|, float64."""
    ny, nx = dirty.shape
    c = fft_tol.component_image(ny, nx, idx, flux)
    z = fft_tol.library_fft_convolution(c, psf, single=False)
    return np.abs(residual.astype(np.float64) - (dirty.astype(np.float64) - z))


def invariant_tolerance(dirty, psf, tiles, idx, flux, residual, rounds, interval):
    """Accumulated tolerance: every local update rounds once (relative u of a
    residual value), every round adds one feedback tolerance."""
    ny, nx = dirty.shape
    T = tiles[0] * tiles[1]
    rscale = 2 * max(float(np.abs(dirty).max()), float(np.abs(residual).max()))
    per_round = np.zeros((ny, nx))
    k = 0
    while k < len(idx):
        m = min(len(idx), k + T * interval)
        per_round = np.maximum(per_round, round_tolerance(ny, nx, tiles, idx[k:m], flux[k:m], psf))
        k = m
    updates = len(idx) / T + rounds + 1
    return rounds * per_round + fft_tol.gamma_prob(updates) * rscale


def check_many_rounds(out, ref, dirty, psf, tiles, interval, gain=0.1):
    gi, gf = host(out["idx"]), host(out["flux"])
    gr = host(out["residual"])
    st = out["stats"]
    R = st["n_rounds"]
    # invariant, for the GPU run and (as a check of the tolerance) the oracle's
    tol = invariant_tolerance(dirty, psf, tiles, gi, gf, gr, R, interval)
    e_gpu = invariant_error(dirty, psf, gi, gf, gr)
    e_ref = invariant_error(dirty, psf, ref["idx"], ref["flux"], ref["residual"])
    print(f"{R} rounds: invariant error gpu {e_gpu.max():.3e} (max err/tol {(e_gpu / tol).max():.3f}), "
          f"oracle {e_ref.max():.3e} (max err/tol {(e_ref / tol).max():.3f}), tolerance max {tol.max():.3e}")
    assert np.all(e_ref <= tol)
    assert np.all(e_gpu <= tol)
    # round 1 bit-exact
    T = tiles[0] * tiles[1]
    n1 = min(T * interval, len(gi), len(ref["idx"]))
    assert np.array_equal(gi[:n1], ref["idx"][:n1])
    assert np.array_equal(bits(gf[:n1]), bits(ref["flux"][:n1]))
    # positions until a near-tie divergence
    n = min(len(gi), len(ref["idx"]))
    same = gi[:n] == ref["idx"][:n]
    k = n if same.all() else int(np.argmin(same))
    drift = np.abs(gf[:k].astype(np.float64) - ref["flux"][:k]).max() if k else 0.0
    print(f"positions agree for {k} of {n} components; max flux drift {drift:.3e}")
    if k < n:
        rounds_before = k // (T * interval)
        E = 16 * drift / gain + rounds_before * tol.max() / max(R, 1)
        gap = abs(abs(float(gf[k])) - abs(float(ref["flux"][k])))
        assert gap <= gain * E + 4 * U * abs(float(gf[k])), (k, gap, gain * E)
    else:
        assert len(gi) == len(ref["idx"]) and st["stop_reason"] == ref["stop"]


MANY = [
    # ny, nx, tiles, interval, seed, max_iter, level, stream
    (64, 64, (2, 2), 20, 71, 1000, 0.0, False),
    (96, 80, (3, 2), 25, 72, 1200, 0.5, False),
    (50, 62, (2, 2), 15, 73, 600, 0.0, True),
    (45, 64, (3, 2), 20, 74, 700, 0.0, False),    # odd height: the last row pair has one row
]


@pytest.mark.parametrize("two", [False, True], ids=["one-level", "two-level"])
@pytest.mark.parametrize("case", MANY, ids=[f"{c[0]}x{c[1]}-{c[2][0]}x{c[2][1]}-I{c[3]}-f{c[6]}"
                                             + ("-stream" if c[7] else "") for c in MANY])
def test_fft_many_rounds_small(lib, case, two):
    ny, nx, tiles, interval, seed, n, level, stream = case
    announce("fft many rounds", case, "two-level" if two else "one-level")
    dirty = sparse_dirty(ny, nx, seed)
    psf = asym_psf(2 * ny, 2 * nx + 2, seed)
    ref = oracle.tiled(dirty, psf, tiles, interval, 0.1, 0.0, n, level=level)
    out = lib.tiled_feedback(dev(dirty), dev(psf), tiles, interval, 0.1, 0.0, n, level=level, stream=stream, fft=True,
                             fft_two_level=two)
    check_many_rounds(out, ref, dirty, psf, tiles, interval)


def test_fft_many_rounds_config1_track(lib):
    """1024^2 / 2x2 / interval 100 with the 2.5-degree track PSF, full 20000
    iterations (50 rounds)."""
    announce("fft many rounds config1 track")
    c = synth.make_config(1, psf_track=True)
    ref = oracle.tiled(c["dirty"], c["psf"], c["tiles"], c["interval"], 0.1, 0.0, c["max_iter"])
    out = lib.tiled_feedback(dev(c["dirty"]), dev(c["psf"]), c["tiles"], c["interval"], 0.1, 0.0, c["max_iter"],
                             fft=True)
    check_many_rounds(out, ref, c["dirty"], c["psf"], c["tiles"], c["interval"])
