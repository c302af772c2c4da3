"""GPU parity of the batched form: every problem of one persistent launch is
bit-identical to the CPU oracle run on that problem alone."""
import numpy as np
import pytest

import oracle
from paper_2501_01461_amd import synth
from tests.gpu_util import announce, assert_same_run, bits, dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2501_01461_amd as P
    P.load()
    return P


def random_problem(seed, ny, nx, thr, n):
    r = np.random.default_rng([31, seed])
    d = r.normal(0, 0.02, (ny, nx)) + (r.random((ny, nx)) < 0.03) * r.uniform(-2, 2, (ny, nx))
    psf = synth.random_psf(2 * ny + 2 * (seed % 3), 2 * nx + 2 * (seed % 2), r, 0.3)
    return dict(dirty=d.astype(np.float32), psf=psf.astype(np.float32), threshold=thr, max_iter=n)


def to_dev(problems):
    return [dict(dirty=dev(p["dirty"]), psf=dev(p["psf"]), threshold=p["threshold"], max_iter=p["max_iter"],
                 **({"cap": p["cap"]} if "cap" in p else {})) for p in problems]


def test_batched_uneven_scalar_groups(lib):
    """Mixed sizes, some widths not a multiple of 4 (the whole batch uses 1-wide groups)."""
    sizes = [(20, 30), (64, 64), (33, 47), (100, 80), (8, 8), (150, 122), (64, 12), (90, 90)]
    probs = [random_problem(i, ny, nx, 0.05 * (i % 2), 60 + 25 * i) for i, (ny, nx) in enumerate(sizes)]
    probs[3]["cap"] = 20
    announce("batched scalar", sizes)
    outs = lib.batched(to_dev(probs), gain=0.1)
    for p, o in zip(probs, outs):
        ref = oracle.hogbom(p["dirty"], p["psf"], 0.1, p["threshold"], p["max_iter"], cap=p.get("cap"))
        assert_same_run(o, ref)


@pytest.mark.parametrize("ppt", [0, 8, 64])
def test_batched_y_array_problems(lib, ppt):
    """Own Y-array PSF per problem, threshold stops, several launch shapes."""
    sides = [64, 256, 128, 96, 192, 64, 320, 128, 256, 64, 160, 96]
    probs = []
    for i, s in enumerate(sides):
        d, p, _ = synth.make_problem(s, 5 + 3 * i, 0.01, 2.1, (), 1e-3, config=93, problem=i)
        probs.append(dict(dirty=d, psf=p, threshold=5e-3, max_iter=3000))
    announce("batched y-array", ppt)
    outs = lib.batched(to_dev(probs), gain=0.1, px_per_thread=ppt)
    for p, o in zip(probs, outs):
        ref = oracle.hogbom(p["dirty"], p["psf"], 0.1, p["threshold"], p["max_iter"])
        assert ref["stop"] == 1
        assert_same_run(o, ref)
    if ppt == 8:
        # 25-workgroup clusters in a grid of about 100: the device-wide queue
        assert all(o["stats"]["xcd_local_clusters"] == 0 for o in outs)


@pytest.mark.parametrize("f16", [False, True], ids=["f32", "f16"])
def test_batched_per_xcd_schedule(lib, f16):
    """8 images of 256^2 (8-workgroup clusters) and 8 of 128^2 (2 workgroups)
    at 16 px/thread: an 80-workgroup grid, 10 per XCD, so each XCD pulls whole
    problems and keeps their exchanges in its L2.  Bit for bit the oracle
    (on the float16-rounded PSFs when they are stored so)."""
    probs = []
    for i, s in enumerate([256] * 8 + [128] * 8):
        d, p, _ = synth.make_problem(s, 6 + i, 0.01, 2.1, (), 1e-3, config=96, problem=i)
        probs.append(dict(dirty=d, psf=p, threshold=5e-3, max_iter=1500))
    announce("batched per-XCD schedule", f16)
    dprobs = to_dev(probs)
    if f16:
        for q in dprobs:
            q["psf"] = lib.psf_to_f16(q["psf"])
    outs = lib.batched(dprobs, gain=0.1, px_per_thread=16)
    assert outs[0]["stats"]["workgroups"] == 80
    assert all(o["stats"]["xcd_local_clusters"] == 1 for o in outs)
    for p, o in zip(probs, outs):
        psf = p["psf"].astype(np.float16).astype(np.float32) if f16 else p["psf"]
        ref = oracle.hogbom(p["dirty"], psf, 0.1, p["threshold"], p["max_iter"])
        assert_same_run(o, ref)


def test_batched_equals_single_calls(lib):
    probs = [random_problem(40 + i, 48 + 16 * i, 64, 0.0, 150) for i in range(6)]
    announce("batched vs single")
    outs = lib.batched(to_dev(probs))
    for p, o in zip(probs, outs):
        s = lib.hogbom(dev(p["dirty"]), dev(p["psf"]), 0.1, 0.0, p["max_iter"])
        assert np.array_equal(host(o["idx"]), host(s["idx"]))
        assert np.array_equal(bits(host(o["flux"])), bits(host(s["flux"])))
        assert np.array_equal(bits(host(o["residual"])), bits(host(s["residual"])))


def test_batched_fp16_psfs(lib):
    sides = [64, 128, 96]
    probs, refs = [], []
    for i, s in enumerate(sides):
        d, p, _ = synth.make_problem(s, 10, 0.01, 2.1, (), 1e-3, config=94, problem=i)
        probs.append(dict(dirty=dev(d), psf=lib.psf_to_f16(dev(p)), threshold=5e-3, max_iter=2000))
        refs.append(oracle.hogbom(d, p.astype(np.float16).astype(np.float32), 0.1, 5e-3, 2000))
    announce("batched fp16")
    outs = lib.batched(probs)
    for o, ref in zip(outs, refs):
        assert_same_run(o, ref)


def test_batched_config3_all_problems(lib):
    """The 256-problem workload (sides 128..1024, own PSFs, threshold 5 sigma)
    in one launch.  Every problem is compared bit for bit with a clean_hogbom
    call on it alone (a seat-queue or per-XCD scheduling error in any problem
    shows), and a stratified quarter of them (64, the largest included) with
    the oracle directly."""
    announce("batched config3")
    probs = synth.make_batch(256)
    dprobs = [dict(dirty=dev(p["dirty"]), psf=dev(p["psf"]), threshold=p["threshold"], max_iter=100000)
              for p in probs]
    outs = lib.batched(dprobs)
    assert all(o["stats"]["stop_reason"] == 1 for o in outs)
    # 32-workgroup clusters at most, 256 workgroups: the per-XCD schedule
    assert all(o["stats"]["xcd_local_clusters"] == 1 for o in outs)
    for q, o in zip(dprobs, outs):
        s = lib.hogbom(q["dirty"], q["psf"], 0.1, q["threshold"], q["max_iter"])
        assert o["stats"]["n_iter"] == s["stats"]["n_iter"]
        assert np.array_equal(host(o["idx"]), host(s["idx"]))
        assert np.array_equal(bits(host(o["flux"])), bits(host(s["flux"])))
        assert np.array_equal(bits(host(o["residual"])), bits(host(s["residual"])))
        assert np.array_equal(bits(host(o["model"])), bits(host(s["model"])))
    order = sorted(range(len(probs)), key=lambda i: probs[i]["n"])
    sample = order[::4][:63] + [order[-1]]
    for i in sample:
        p = probs[i]
        ref = oracle.hogbom(p["dirty"], p["psf"], 0.1, p["threshold"], 100000)
        assert_same_run(outs[i], ref)


MIXED = [
    # side, sources, tiles, interval, threshold
    (128, 30, (2, 2), 20, 0.0),
    (96, 12, (1, 1), 1, 5e-3),
    (160, 40, (2, 3), 9, 0.0),
    (64, 8, (1, 1), 1, 0.0),
    (192, 50, (3, 2), 40, 5e-3),
    (120, 20, (2, 1), 60, 0.0),
    (256, 60, (4, 4), 7, 0.0),
    (80, 10, (1, 2), 15, 5e-3),
]


@pytest.mark.parametrize("level", [0.0, 0.5], ids=["interval", "flux-trigger"])
def test_batched_mixed_plain_and_tiled(lib, level):
    """Plain and tiled problems (grids 1 x 2 .. 4 x 4, intervals 7..60,
    thresholds) in one launch: each is bit for bit the oracle's plain or tiled
    run, with its own round count."""
    probs, refs = [], []
    for i, (n, ns, tiles, ivl, thr) in enumerate(MIXED):
        d, p, _ = synth.make_problem(n, ns, 0.01, 2.1, (), 1e-3, config=98, problem=i)
        max_iter = 1500
        if tiles == (1, 1):
            refs.append(oracle.hogbom(d, p, 0.1, thr, max_iter))
        else:
            refs.append(oracle.tiled(d, p, tiles, ivl, 0.1, thr, max_iter, level=level))
        probs.append(dict(dirty=dev(d), psf=dev(p), threshold=thr, max_iter=max_iter, tiles=tiles, interval=ivl))
    announce("batched mixed", level)
    outs = lib.batched(probs, gain=0.1, level=level)
    for (n, ns, tiles, ivl, thr), o, ref in zip(MIXED, outs, refs):
        if tiles != (1, 1):
            assert o["stats"]["n_rounds"] == ref["n_rounds"], (tiles, ivl)
        assert_same_run(o, ref)


def test_batched_tiled_equals_single_calls(lib):
    """Tiled problems of a batch run alone through clean_tiled_feedback give
    the same bits (FP16 PSFs, so the half-precision loads of the tiled
    batched path are covered too)."""
    probs = []
    for i, (n, ns, tiles, ivl, thr) in enumerate(MIXED):
        if tiles == (1, 1):
            continue
        d, p, _ = synth.make_problem(n, ns, 0.01, 2.1, (), 1e-3, config=99, problem=i)
        probs.append(dict(dirty=dev(d), psf=lib.psf_to_f16(dev(p)), threshold=thr, max_iter=1200, tiles=tiles,
                          interval=ivl))
    announce("batched tiled = single calls")
    outs = lib.batched(probs, gain=0.1)
    for q, o in zip(probs, outs):
        s = lib.tiled_feedback(q["dirty"], q["psf"], q["tiles"], q["interval"], 0.1, q["threshold"], q["max_iter"])
        assert o["stats"]["n_rounds"] == s["stats"]["n_rounds"]
        assert np.array_equal(host(o["idx"]), host(s["idx"]))
        assert np.array_equal(bits(host(o["flux"])), bits(host(s["flux"])))
        assert np.array_equal(bits(host(o["residual"])), bits(host(s["residual"])))
        assert np.array_equal(bits(host(o["model"])), bits(host(s["model"])))


def test_batched_tuned_shape(lib):
    """The batch tuner times the candidate shapes, batched() with
    px_per_thread=0 then runs the shape it chose, and the result is the
    oracle's bit for bit (as it is for every shape)."""
    probs, refs = [], []
    for i, (n, ns, tiles, ivl, thr) in enumerate(MIXED):
        d, p, _ = synth.make_problem(n, ns, 0.01, 2.1, (), 1e-3, config=97, problem=i)
        if tiles == (1, 1):
            refs.append(oracle.hogbom(d, p, 0.1, thr, 800))
        else:
            refs.append(oracle.tiled(d, p, tiles, ivl, 0.1, thr, 800))
        probs.append(dict(dirty=dev(d), psf=dev(p), threshold=thr, max_iter=800, tiles=tiles, interval=ivl))
    announce("batched tuned shape")
    t = lib.autotune_batched(probs, gain=0.1, trial_iter=200)
    assert t["px_per_thread"] in (8, 16, 32, 64)
    ms = t["trial_ms"]
    assert len(ms) == 4 and any(v > 0 for v in ms)
    assert ms[(8, 16, 32, 64).index(t["px_per_thread"])] == min(v for v in ms if v > 0)
    outs = lib.batched(probs, gain=0.1)
    for o, ref in zip(outs, refs):
        assert o["stats"]["px_per_thread"] == t["px_per_thread"]
        assert_same_run(o, ref)
    # an explicit shape still wins over the tuned one
    other = 16 if t["px_per_thread"] != 16 else 32
    outs = lib.batched(probs, gain=0.1, px_per_thread=other)
    for o, ref in zip(outs, refs):
        assert o["stats"]["px_per_thread"] == other
        assert_same_run(o, ref)


def test_batched_degenerate_problems(lib):
    """A batch of edge cases: no iterations asked, a 1 x 1 image, an image
    whose peak is already under the threshold, a zero image, capacity 0."""
    probs = [random_problem(40, 16, 20, 0.0, 0),                 # max_iter 0: the dirty image back
             random_problem(41, 1, 1, 0.0, 5),                   # 1 x 1 image, 2 x 2 PSF (+ extra)
             dict(random_problem(42, 24, 24, 0.0, 50)),
             dict(random_problem(43, 12, 16, 0.0, 30)),
             dict(random_problem(44, 20, 12, 0.0, 40), cap=0)]
    probs[2]["threshold"] = 10.0                                  # first peak below the threshold
    probs[3]["dirty"] = np.zeros((12, 16), np.float32)            # ties everywhere: index 0 each time
    announce("batched degenerate")
    outs = lib.batched(to_dev(probs), gain=0.1)
    for p, o in zip(probs, outs):
        ref = oracle.hogbom(p["dirty"], p["psf"], 0.1, p["threshold"], p["max_iter"], cap=p.get("cap"))
        assert_same_run(o, ref)
    assert outs[0]["stats"]["n_iter"] == 0 and outs[2]["stats"]["n_iter"] == 0
    assert outs[4]["stats"]["n_iter"] == 0 and outs[4]["stats"]["stop_reason"] == 2


def test_batched_degenerate_problems_per_xcd(lib):
    """The same edge cases under the per-XCD schedule: 16 one-workgroup
    problems (a 16-workgroup grid, 2 per XCD), including odd widths."""
    probs = [random_problem(50, 16, 20, 0.0, 0),
             random_problem(51, 1, 1, 0.0, 5),
             dict(random_problem(52, 24, 24, 0.0, 50)),
             dict(random_problem(53, 12, 16, 0.0, 30)),
             dict(random_problem(54, 20, 12, 0.0, 40), cap=0)]
    probs[2]["threshold"] = 10.0
    probs[3]["dirty"] = np.zeros((12, 16), np.float32)
    probs += [random_problem(60 + i, 20 + 3 * i, 17 + 5 * i, 0.0, 60 + 10 * i) for i in range(11)]
    announce("batched degenerate, per-XCD schedule")
    outs = lib.batched(to_dev(probs), gain=0.1)
    assert outs[0]["stats"]["workgroups"] == 16
    assert all(o["stats"]["wg_per_tile"] == 1 for o in outs)
    assert all(o["stats"]["xcd_local_clusters"] == 1 for o in outs)
    for p, o in zip(probs, outs):
        ref = oracle.hogbom(p["dirty"], p["psf"], 0.1, p["threshold"], p["max_iter"], cap=p.get("cap"))
        assert_same_run(o, ref)
    assert outs[4]["stats"]["n_iter"] == 0 and outs[4]["stats"]["stop_reason"] == 2
