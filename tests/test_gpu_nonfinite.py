"""GPU parity on runs that go non-finite (diverging method, or NaN/Inf input
that was not screened out), against the oracle.

The reading (Section 3's peak search extended to non-finite values): |r| is
ordered as magnitudes with every NaN above +Inf and all NaNs equal; a
non-finite peak ends the run (stop reason 4) before anything is appended; in
the tiled form a non-finite local peak ends the tile's round, and a
non-finite tile peak at a round's start ends the run.  Every case compares
the iteration count, stop reason, round count, component positions and
float32 bits, and the residual and model bits with NaN matching NaN, across
the register tiles (4-wide and scalar groups), the streamed residual, the
wide tile and the batched kernel.
"""
import numpy as np
import pytest

import oracle
from tests.gpu_util import announce, assert_same_run, dev, host

pytestmark = pytest.mark.gpu
STOP_NONFINITE = 4


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2501_01461_amd as P
    P.load()
    return P


def peak_class(v):
    return "nan" if np.isnan(v) else ("inf" if np.isinf(v) else "finite")


def expected_final_peak(res, tiles=None):
    """Value of the largest |r| (NaN above Inf) over the image, or over the
    tile peaks (the largest, lowest tile id on ties)."""
    if tiles is None:
        return float(res.reshape(-1)[oracle.peak(res)])
    ny, nx = res.shape
    best = None
    for i in range(tiles[0]):
        for j in range(tiles[1]):
            rect = (i * ny // tiles[0], (i + 1) * ny // tiles[0], j * nx // tiles[1], (j + 1) * nx // tiles[1])
            v = float(res.reshape(-1)[oracle.peak(res, rect)])
            m = (1, 0.0) if np.isnan(v) else (0, abs(v))
            if best is None or m > best[0]:
                best = (m, v)
    return best[1]


def check_final_peak(gpu, ref, tiles=None):
    want = expected_final_peak(ref["residual"], tiles)
    got = gpu["stats"]["final_peak"]
    assert peak_class(got) == peak_class(want), (got, want)
    if not np.isnan(want):
        assert abs(got) == abs(want), (got, want)


def diverging_case(ny, nx, seed, extra=(0, 0), amp=40.0):
    """Random dirty image; random PSF (peak 1 at the centre) whose sidelobes
    reach `amp`: with gain 1 every iteration multiplies the residual's scale,
    so a run overflows to Inf within a few dozen iterations."""
    r = np.random.default_rng([96, seed])
    d = r.normal(0, 1, (ny, nx)).astype(np.float32)
    psf = r.uniform(-amp, amp, (2 * ny + extra[0], 2 * nx + extra[1])).astype(np.float32)
    psf[psf.shape[0] // 2, psf.shape[1] // 2] = 1.0
    return d, psf


# ------------------------------------------------------------------ plain --

PLAIN = [
    # ny, nx, psf extra, seed, wg_per_tile, px_per_thread, stream
    (40, 48, (0, 0), 1, 0, 0, False),
    (37, 50, (2, 6), 2, 0, 0, False),       # scalar groups
    (96, 128, (4, 0), 3, 3, 8, False),
    (64, 64, (0, 2), 4, 2, 32, False),
    (48, 64, (0, 0), 5, 2, 0, True),        # streamed residual
    (37, 50, (0, 4), 6, 3, 0, True),        # streamed, scalar groups
]


@pytest.mark.parametrize("case", PLAIN, ids=[f"{c[0]}x{c[1]}-wg{c[4]}-ppt{c[5]}{'-stream' if c[6] else ''}"
                                             for c in PLAIN])
def test_plain_diverging(lib, case):
    ny, nx, extra, seed, wg, ppt, stream = case
    announce("plain diverging", case)
    d, psf = diverging_case(ny, nx, seed, extra)
    ref = oracle.hogbom(d, psf, 1.0, 0.0, 5000)
    assert ref["stop"] == STOP_NONFINITE
    out = lib.hogbom(dev(d), dev(psf), 1.0, 0.0, 5000, wg_per_tile=wg, px_per_thread=ppt, stream=stream)
    assert_same_run(out, ref, nan_aware=True)
    check_final_peak(out, ref)


def test_plain_overflow_closed_form(lib):
    """Pixel 0 holds a = 3e38, the PSF is 1 at the centre and -a one pixel to
    the right: iteration 1 leaves +Inf at pixel 1, and the run stops."""
    announce("plain overflow closed form")
    a = np.float32(3.0e38)
    d = np.zeros((4, 16), np.float32)
    d[0, 0] = a
    psf = np.zeros((8, 32), np.float32)
    psf[4, 16] = 1.0
    psf[4, 17] = -a
    for stream in (False, True):
        out = lib.hogbom(dev(d), dev(psf), 1.0, 0.0, 50, stream=stream)
        st = out["stats"]
        assert st["n_iter"] == 1 and st["stop_reason"] == STOP_NONFINITE
        assert host(out["idx"]).tolist() == [0] and host(out["flux"])[0] == a
        res = host(out["residual"])
        assert np.isposinf(res[0, 1]) and np.count_nonzero(res) == 1
        assert np.isposinf(st["final_peak"])


@pytest.mark.parametrize("stream", [False, True])
@pytest.mark.parametrize("scalar", [False, True])
def test_plain_nan_from_psf(lib, stream, scalar):
    """A NaN in the PSF window turns one pixel NaN after the first iteration;
    the next peak search ranks it above every value (a planted +Inf
    elsewhere too would lose) and the run stops with n = 1."""
    announce("plain nan from psf", stream, scalar)
    ny, nx = (24, 30) if scalar else (24, 32)
    r = np.random.default_rng([97, int(stream), int(scalar)])
    d = r.normal(0, 0.1, (ny, nx)).astype(np.float32)
    d[10, 11] = 5.0
    psf = r.uniform(-0.3, 0.3, (2 * ny, 2 * nx)).astype(np.float32)
    cy, cx = ny, nx
    psf[cy, cx] = 1.0
    psf[cy + 3, cx - 2] = np.nan          # reaches pixel (13, 9) from the peak (10, 11)
    psf[cy - 4, cx + 5] = np.inf          # reaches pixel (6, 16)
    ref = oracle.hogbom(d, psf, 0.5, 0.0, 100)
    assert ref["n_iter"] == 1 and ref["stop"] == STOP_NONFINITE
    out = lib.hogbom(dev(d), dev(psf), 0.5, 0.0, 100, stream=stream)
    assert_same_run(out, ref, nan_aware=True)
    assert np.isnan(out["stats"]["final_peak"])


@pytest.mark.parametrize("bad", ["nan", "inf", "both"])
def test_nonfinite_input_without_check(lib, bad):
    announce("nonfinite input", bad)
    d = np.random.default_rng([98]).normal(0, 1, (32, 40)).astype(np.float32)
    if bad in ("inf", "both"):
        d[3, 7] = -np.inf
    if bad in ("nan", "both"):
        d[20, 30] = np.nan
    psf = np.random.default_rng([99]).uniform(-0.2, 0.2, (64, 80)).astype(np.float32)
    psf[32, 40] = 1.0
    ref = oracle.hogbom(d, psf, 0.1, 0.0, 50)
    out = lib.hogbom(dev(d), dev(psf), 0.1, 0.0, 50)
    assert_same_run(out, ref, nan_aware=True)
    assert out["stats"]["n_iter"] == 0 and out["stats"]["stop_reason"] == STOP_NONFINITE
    check_final_peak(out, ref)
    t = lib.tiled_feedback(dev(d), dev(psf), (2, 2), 10, 0.1, 0.0, 50, level=0.5)
    tr = oracle.tiled(d, psf, (2, 2), 10, 0.1, 0.0, 50, level=0.5)
    assert t["stats"]["n_rounds"] == tr["n_rounds"] == 0
    assert_same_run(t, tr, nan_aware=True)
    check_final_peak(t, tr, (2, 2))


# ------------------------------------------------------------------ tiled --

TILED = [
    # ny, nx, tiles, interval, seed, level, wg, ppt, stream
    (48, 64, (2, 2), 6, 11, 0.0, 0, 0, False),
    (50, 62, (2, 2), 9, 12, 0.0, 0, 0, False),      # odd tile widths: scalar groups
    (64, 128, (2, 4), 40, 13, 0.0, 2, 4, False),    # long interval, 2 workgroups per tile
    (48, 64, (2, 2), 6, 14, 0.5, 0, 0, False),      # flux trigger
    (48, 64, (2, 2), 8, 15, 0.0, 0, 0, True),       # streamed residual
    (50, 62, (3, 2), 7, 16, 0.3, 0, 0, True),       # streamed, scalar groups, flux trigger
    (64, 64, (2, 2), 10, 17, 0.0, 0, 128, False),   # wide tile
    (96, 128, (2, 2), 25, 18, 0.4, 0, 128, False),  # wide tile, flux trigger
]


@pytest.mark.parametrize("case", TILED, ids=[f"{c[0]}x{c[1]}-{c[2][0]}x{c[2][1]}-I{c[3]}-L{c[5]}-ppt{c[7]}"
                                             f"{'-stream' if c[8] else ''}" for c in TILED])
def test_tiled_diverging(lib, case):
    ny, nx, tiles, interval, seed, level, wg, ppt, stream = case
    announce("tiled diverging", case)
    d, psf = diverging_case(ny, nx, seed, amp=30.0)
    ref = oracle.tiled(d, psf, tiles, interval, 1.0, 0.0, 100000, level=level)
    assert ref["stop"] == STOP_NONFINITE
    out = lib.tiled_feedback(dev(d), dev(psf), tiles, interval, 1.0, 0.0, 100000, level=level, wg_per_tile=wg,
                             px_per_thread=ppt, stream=stream)
    st = out["stats"]
    assert st["streamed"] == int(stream)
    if ppt == 128:
        assert st["px_per_thread"] == 128
    assert st["n_rounds"] == ref["n_rounds"]
    assert_same_run(out, ref, nan_aware=True)
    check_final_peak(out, ref, tiles)


@pytest.mark.parametrize("form", ["register", "stream", "wide"])
def test_tiled_nan_from_psf_outside_the_tile(lib, form):
    """A NaN in the PSF at the offset that the register tiles' groups past a
    tile's end read (the window of image pixel (0, 0)): those groups hold NaN
    without it being in the tile, which must not count.  Tile 0's pixel (0, 0)
    gets the NaN at the first feedback, and the next round stops."""
    announce("tiled nan outside tile", form)
    ny, nx, tiles = 48, 64, (2, 2)
    r = np.random.default_rng([100])
    d = r.normal(0, 0.05, (ny, nx)).astype(np.float32)
    d[30, 40] = 4.0                       # tile 3's peak
    psf = r.uniform(-0.2, 0.2, (2 * ny, 2 * nx)).astype(np.float32)
    cy, cx = ny, nx
    psf[cy, cx] = 1.0
    psf[cy - 30, cx - 40] = np.nan        # offset -(30, 40): from (30, 40) onto (0, 0)
    kw = dict(stream=True) if form == "stream" else (dict(px_per_thread=128) if form == "wide" else {})
    ref = oracle.tiled(d, psf, tiles, 5, 0.5, 0.0, 400)
    assert ref["stop"] == STOP_NONFINITE and ref["n_rounds"] == 1
    out = lib.tiled_feedback(dev(d), dev(psf), tiles, 5, 0.5, 0.0, 400, **kw)
    assert out["stats"]["n_rounds"] == 1
    assert_same_run(out, ref, nan_aware=True)
    assert np.isnan(out["stats"]["final_peak"])


def test_tiled_overflow_in_feedback_closed_form(lib):
    """Two tiles; tile 0 removes a = 3e38 at (0, 0), the feedback puts
    fma(a, -a, 0) = -Inf into the sum at (0, 8), r = +Inf there, round 2 stops."""
    announce("tiled overflow in feedback")
    a = np.float32(3.0e38)
    d = np.zeros((8, 16), np.float32)
    d[0, 0] = a
    psf = np.zeros((16, 32), np.float32)
    psf[8, 16] = 1.0
    psf[8, 24] = -a
    ref = oracle.tiled(d, psf, (1, 2), 1, 1.0, 1e-3, 10)
    assert ref["n_iter"] == 1 and ref["stop"] == STOP_NONFINITE and ref["n_rounds"] == 1
    for kw in ({}, {"stream": True}, {"px_per_thread": 128}):
        out = lib.tiled_feedback(dev(d), dev(psf), (1, 2), 1, 1.0, 1e-3, 10, **kw)
        assert out["stats"]["n_rounds"] == 1
        assert_same_run(out, ref, nan_aware=True)
        assert np.isposinf(host(out["residual"])[0, 8])


# ---------------------------------------------------------------- batched --

def test_batched_mixed_diverging(lib):
    """Diverging and converging problems in one launch: each is identical to
    the oracle run on it alone."""
    announce("batched diverging")
    import torch
    probs, refs = [], []
    for i, (ny, nx) in enumerate([(40, 48), (64, 64), (32, 32), (56, 40), (48, 64), (24, 32)]):
        if i % 2 == 0:
            d, psf = diverging_case(ny, nx, 200 + i)
            gain, thr = 1.0, 0.0
        else:
            r = np.random.default_rng([101, i])
            d = r.normal(0, 0.05, (ny, nx)).astype(np.float32)
            d[ny // 3, nx // 2] = 2.0
            psf = r.uniform(-0.3, 0.3, (2 * ny, 2 * nx)).astype(np.float32)
            psf[ny, nx] = 1.0
            gain, thr = 1.0, 1e-2
        refs.append(oracle.hogbom(d, psf, gain, thr, 3000))
        probs.append(dict(dirty=dev(d), psf=dev(psf), threshold=thr, max_iter=3000))
    outs = lib.batched(probs, gain=1.0)
    torch.cuda.synchronize()
    assert any(r["stop"] == STOP_NONFINITE for r in refs)
    for o, r in zip(outs, refs):
        assert_same_run(o, r, nan_aware=True)
