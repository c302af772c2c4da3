"""Run control on the GPU: the caller's cancel flag (plain, tiled, batched)
and the internal-workspace limit (CLEAN_E_NOMEM).

A cancelled run stops at a checkpoint (plain: a multiple of 4096
iterations; tiled: a round's start) and its results are those of the same
call with max_iter = the iterations done, bit for bit."""
import threading

import numpy as np
import pytest

from paper_2501_01461_amd import synth
from tests.gpu_util import announce, bits, dev, host

pytestmark = pytest.mark.gpu
STOP_CANCELLED = 3


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2501_01461_amd as P
    P.load()
    return P


@pytest.fixture(scope="module")
def track():
    c = synth.make_config(1, psf_track=True)
    return c, dev(c["dirty"]), dev(c["psf"])


def flag():
    import torch
    return torch.zeros(1, dtype=torch.int32).pin_memory()


def same(a, b):
    assert a["stats"]["n_iter"] == b["stats"]["n_iter"]
    assert np.array_equal(host(a["idx"]), host(b["idx"]))
    assert np.array_equal(bits(host(a["flux"])), bits(host(b["flux"])))
    assert np.array_equal(bits(host(a["residual"])), bits(host(b["residual"])))
    assert np.array_equal(bits(host(a["model"])), bits(host(b["model"])))


def set_later(f, seconds):
    t = threading.Timer(seconds, lambda: f.__setitem__(0, 1))
    t.start()
    return t


def test_cancel_plain(lib, track):
    c, d, p = track
    f = flag()
    f[0] = 1
    announce("cancel plain, preset")
    r = lib.hogbom(d, p, 0.1, 0.0, 400000, cancel=f)
    assert r["stats"]["stop_reason"] == STOP_CANCELLED and r["stats"]["n_iter"] == 0
    f[0] = 0
    announce("cancel plain, after 0.3 s")
    t = set_later(f, 0.3)
    r = lib.hogbom(d, p, 0.1, 0.0, 400000, cancel=f)
    t.join()
    st = r["stats"]
    assert st["stop_reason"] == STOP_CANCELLED, st
    assert 0 < st["n_iter"] < 400000 and st["n_iter"] % 4096 == 0
    same(r, lib.hogbom(d, p, 0.1, 0.0, st["n_iter"]))


def test_cancel_tiled(lib, track):
    c, d, p = track
    f = flag()
    f[0] = 1
    announce("cancel tiled, preset")
    r = lib.tiled_feedback(d, p, (2, 2), 100, 0.1, 0.0, 2000000, cancel=f)
    assert r["stats"]["stop_reason"] == STOP_CANCELLED and r["stats"]["n_iter"] == 0
    assert r["stats"]["n_rounds"] == 0
    f[0] = 0
    announce("cancel tiled, after 0.3 s")
    t = set_later(f, 0.3)
    r = lib.tiled_feedback(d, p, (2, 2), 100, 0.1, 0.0, 2000000, cancel=f)
    t.join()
    st = r["stats"]
    assert st["stop_reason"] == STOP_CANCELLED, st
    assert 0 < st["n_iter"] < 2000000 and st["n_iter"] == 400 * st["n_rounds"]
    ref = lib.tiled_feedback(d, p, (2, 2), 100, 0.1, 0.0, st["n_iter"])
    assert ref["stats"]["n_rounds"] == st["n_rounds"]
    same(r, ref)


def test_cancel_batched(lib):
    probs = []
    for i, s in enumerate([256, 192, 128, 256, 96, 160]):
        d, p, _ = synth.make_problem(s, 10 + i, 0.01, 2.1, (), 1e-3, config=97, problem=i)
        probs.append(dict(dirty=dev(d), psf=dev(p), threshold=0.0, max_iter=300000))
    f = flag()
    f[0] = 1
    announce("cancel batched, preset")
    outs = lib.batched(probs, gain=0.1, cancel=f)
    assert all(o["stats"]["stop_reason"] == STOP_CANCELLED and o["stats"]["n_iter"] == 0 for o in outs)
    f[0] = 0
    announce("cancel batched, after 0.2 s")
    t = set_later(f, 0.2)
    outs = lib.batched(probs, gain=0.1, cancel=f)
    t.join()
    assert any(o["stats"]["stop_reason"] == STOP_CANCELLED for o in outs)
    for q, o in zip(probs, outs):
        n = o["stats"]["n_iter"]
        assert o["stats"]["stop_reason"] in (0, STOP_CANCELLED)
        if o["stats"]["stop_reason"] == STOP_CANCELLED:
            assert n % 4096 == 0
        same(o, lib.hogbom(q["dirty"], q["psf"], 0.1, 0.0, n))


def test_workspace_limit_nomem(lib, track):
    c, d, p = track
    announce("workspace limit")
    old = lib.set_workspace_limit(1 << 20)
    try:
        with pytest.raises(lib.CleanError) as e:
            lib.tiled_feedback(d, p, (2, 2), 100, 0.1, 0.0, 1000)      # feedback buffer alone is 4 MiB
        assert e.value.status == -3
        small = synth.make_config(0)
        r = lib.hogbom(dev(small["dirty"]), dev(small["psf"]), 0.1, 5e-3, 1000)
        assert r["stats"]["n_iter"] > 0
        out = lib.hogbom_noalloc(dev(small["dirty"]), dev(small["psf"]), 0.1, 5e-3, 1000)   # allocates nothing
        assert out["stats"]["n_iter"] == r["stats"]["n_iter"]
    finally:
        lib.set_workspace_limit(old)
    r = lib.tiled_feedback(d, p, (2, 2), 100, 0.1, 0.0, 1000)
    assert r["stats"]["n_iter"] == 1000
