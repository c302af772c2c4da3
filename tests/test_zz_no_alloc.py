"""The allocation-free entry point clean_hogbom_noalloc against clean_hogbom.

Called through the C ABI (ctypes binding): on two calls in a row, the second
with a smaller image (its scratch array keeps the first call's contents, so
stale control words or exchange slots would show), the components, residual,
model, iteration count and stop reason must equal clean_hogbom's bit for bit;
so must a streamed-residual call and a forced launch shape.  A launch whose
workspace does not fit the scratch array is refused with CLEAN_E_UNSUPPORTED
before anything runs.
"""
import numpy as np
import pytest

from paper_2501_01461_amd import synth
from tests.gpu_util import announce, assert_same_run, dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2501_01461_amd as P
    P.load()
    return P


def as_ref(out):
    """clean_hogbom's result in the oracle's dict layout, for assert_same_run."""
    return dict(n_iter=out["stats"]["n_iter"], stop=out["stats"]["stop_reason"], idx=host(out["idx"]),
                flux=host(out["flux"]), residual=host(out["residual"]), model=host(out["model"]))


def case(ny, nx, seed):
    r = np.random.default_rng([120, seed])
    d = (r.normal(0, 0.02, (ny, nx)) + (r.random((ny, nx)) < 0.02) * r.uniform(-2, 2, (ny, nx))).astype(np.float32)
    psf = synth.random_psf(2 * ny, 2 * nx + 2, np.random.default_rng([121, seed]), 0.3).astype(np.float32)
    return d, psf


@pytest.mark.parametrize("kw", [{}, {"stream": True}, {"wg_per_tile": 12, "px_per_thread": 8}],
                         ids=["register", "streamed", "shape"])
def test_noalloc_equals_hogbom_twice(lib, kw):
    for (ny, nx, seed, n, thr) in [(192, 256, 1, 700, 0.0), (60, 84, 2, 300, 0.02)]:
        announce("noalloc", kw, ny, nx)
        d, psf = case(ny, nx, seed)
        ref = lib.hogbom(dev(d), dev(psf), 0.1, thr, n, **kw)
        out = lib.hogbom_noalloc(dev(d), dev(psf), 0.1, thr, n, **kw)
        assert out["stats"]["n_iter"] > 0
        assert out["stats"]["wg_per_tile"] == ref["stats"]["wg_per_tile"]
        assert out["stats"]["streamed"] == ref["stats"]["streamed"]
        assert_same_run(out, as_ref(ref))
        assert out["stats"]["final_peak"] == ref["stats"]["final_peak"]
        assert out["stats"]["residual_rms"] == ref["stats"]["residual_rms"]
        assert out["stats"]["model_flux"] == ref["stats"]["model_flux"]


def test_noalloc_refuses_a_launch_larger_than_its_scratch(lib):
    """A forced cluster of 2048 workgroups needs about 90 KB of workspace,
    more than the 64 KiB array: refused before anything is launched."""
    announce("noalloc too large")
    d = dev(np.zeros((2048, 2048), np.float32))
    psf = dev(np.zeros((4096, 4096), np.float32))
    with pytest.raises(lib.CleanError) as e:
        lib.hogbom_noalloc(d, psf, 0.1, 0.0, 3, wg_per_tile=2048, px_per_thread=4)
    assert e.value.status == -6 and "allocation-free" in str(e.value)
