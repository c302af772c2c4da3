"""The plan tuner (clean_autotune_plan) on the 1024^2 workload with the
10-minute-track PSF: every candidate's reported band equals the band of
direct tiled and plain runs restored by the library (computed here with
numpy), the choice follows the rule (the fastest candidate whose band lies in
the budget and whose run stayed finite), the plan cache returns the stored
plan without trials, and a budget no candidate meets gives interval 0."""
import numpy as np
import pytest

from paper_2501_01461_amd import synth
from tests.gpu_util import announce, dev

pytestmark = pytest.mark.gpu
GRIDS = [(2, 2), (4, 4)]
INTERVALS = [5, 10, 25, 100]
BAND = (-0.1, 0.1)


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2501_01461_amd as P
    P.load()
    return P


@pytest.fixture(scope="module")
def track(lib):
    c = synth.make_config(1, psf_track=True)
    return c, dev(c["dirty"]), dev(c["psf"])


def test_plan_bands_and_choice(lib, track, tmp_path):
    c, d, p = track
    n = c["max_iter"]
    announce("plan tuner", GRIDS, INTERVALS)
    cache = str(tmp_path / "plans.txt")
    plan = lib.autotune_plan(d, p, GRIDS, INTERVALS, c["gain"], 0.0, n, band=BAND, cache_path=cache)
    assert not plan["from_cache"]
    sigma = lib.clean_beam(p)["sigma"]
    mp = lib.hogbom(d, p, c["gain"], 0.0, n)
    rp = lib.restore(mp["model"], mp["residual"], sigma).cpu().numpy()
    best = None
    for cand in plan["candidates"]:
        mt = lib.tiled_feedback(d, p, cand["tiles"], cand["interval"], c["gain"], 0.0, n)
        rt = lib.restore(mt["model"], mt["residual"], sigma).cpu().numpy()
        diff = rt - rp
        lo, hi = float(diff.min()), float(diff.max())
        assert cand["band"] == [lo, hi], (cand, lo, hi)
        ok = np.isfinite([lo, hi]).all() and BAND[0] <= lo and hi <= BAND[1] and mt["stats"]["stop_reason"] != 4
        if ok and (best is None or cand["iters_per_s"] > best["iters_per_s"]):
            best = cand
    assert best is not None, "the track PSF reaches the band at short intervals"
    assert (plan["tiles"], plan["interval"]) == (best["tiles"], best["interval"])
    assert plan["band"] == best["band"] and plan["iters_per_s"] == best["iters_per_s"]
    announce(f"plan: {plan['tiles']} I={plan['interval']} band {plan['band']} {plan['iters_per_s']:.0f} it/s")
    # the cache returns the stored plan without trials
    again = lib.autotune_plan(d, p, GRIDS, INTERVALS, c["gain"], 0.0, n, band=BAND, cache_path=cache)
    assert again["from_cache"]
    for k in ("tiles", "interval", "wg_per_tile", "px_per_thread", "band", "iters_per_s"):
        assert again[k] == plan[k], k
    assert all(np.isnan(cd["band"]).all() for cd in again["candidates"])


def test_plan_none_acceptable(lib, track):
    c, d, p = track
    announce("plan tuner, impossible budget")
    plan = lib.autotune_plan(d, p, [(2, 2)], [50, 100], c["gain"], 0.0, 4000, band=(-1e-9, 1e-9))
    assert plan["interval"] == 0
    assert all(np.isfinite(cd["band"]).all() for cd in plan["candidates"])
