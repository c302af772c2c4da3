"""Resume on the GPU: a run continued from the residual it returned equals the
longer run, bit for bit: plain CLEAN at any iteration, tiled CLEAN with the
interval trigger at a round boundary (each side also equals the oracle)."""
import numpy as np
import pytest

import oracle
from paper_2501_01461_amd import synth
from tests.gpu_util import announce, bits, dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2501_01461_amd as P
    P.load()
    return P


def same_sequence(full, a, b):
    assert np.array_equal(host(full["idx"]), np.concatenate([host(a["idx"]), host(b["idx"])]))
    assert np.array_equal(bits(host(full["flux"])), bits(np.concatenate([host(a["flux"]), host(b["flux"])])))
    assert np.array_equal(bits(host(full["residual"])), bits(host(b["residual"])))


@pytest.mark.parametrize("shape", [dict(), dict(stream=True), dict(px_per_thread=4)],
                         ids=["register", "streamed", "4-px"])
def test_plain_resume(lib, shape):
    c = synth.make_config(0)
    d, p = dev(c["dirty"]), dev(c["psf"])
    announce("plain resume", shape)
    full = lib.hogbom(d, p, 0.1, 0.0, 700, **shape)
    a = lib.hogbom(d, p, 0.1, 0.0, 250, **shape)
    b = lib.hogbom(a["residual"].clone(), p, 0.1, 0.0, 450, **shape)
    same_sequence(full, a, b)
    ref = oracle.hogbom(c["dirty"], c["psf"], 0.1, 0.0, 700)
    assert np.array_equal(host(full["idx"]), ref["idx"])
    assert np.array_equal(bits(host(full["residual"])), bits(ref["residual"]))


@pytest.mark.parametrize("case", [((2, 2), 25, {}), ((3, 2), 20, {}), ((2, 2), 25, dict(px_per_thread=128))],
                         ids=["2x2", "3x2", "wide"])
def test_tiled_resume_at_round_boundary(lib, case):
    tiles, ivl, shape = case
    c = synth.make_config(0)
    d, p = dev(c["dirty"]), dev(c["psf"])
    T = tiles[0] * tiles[1]
    announce("tiled resume", case)
    full = lib.tiled_feedback(d, p, tiles, ivl, 0.1, 0.0, 7 * T * ivl, **shape)
    a = lib.tiled_feedback(d, p, tiles, ivl, 0.1, 0.0, 3 * T * ivl, **shape)
    b = lib.tiled_feedback(a["residual"].clone(), p, tiles, ivl, 0.1, 0.0, 4 * T * ivl, **shape)
    assert (a["stats"]["n_rounds"], b["stats"]["n_rounds"], full["stats"]["n_rounds"]) == (3, 4, 7)
    same_sequence(full, a, b)
    ref = oracle.tiled(c["dirty"], c["psf"], tiles, ivl, 0.1, 0.0, 7 * T * ivl)
    assert np.array_equal(host(full["idx"]), ref["idx"])
    assert np.array_equal(bits(host(full["residual"])), bits(ref["residual"]))
