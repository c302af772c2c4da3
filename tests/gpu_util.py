"""Helpers shared by the GPU tests: device tensors in, numpy out, exact compares."""
import sys

import numpy as np


def announce(*parts):
    """Name the case before it touches the GPU (flushed, so a fault still shows it)."""
    print("CASE", *parts, file=sys.stderr, flush=True)


def dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    return t.detach().cpu().numpy()


def bits(a):
    a = np.ascontiguousarray(a)
    return a.view(np.uint32 if a.dtype == np.float32 else np.uint64)


def same_bits(a, b, nan_aware=False):
    """Bitwise equal; with nan_aware, NaN matches NaN whatever its sign or
    payload (both sides create NaNs by invalid operations, whose sign the
    IEEE standard leaves open)."""
    a, b = np.ascontiguousarray(a), np.ascontiguousarray(b)
    if a.shape != b.shape or a.dtype != b.dtype:
        return False
    if not nan_aware:
        return np.array_equal(bits(a), bits(b))
    na, nb = np.isnan(a), np.isnan(b)
    return np.array_equal(na, nb) and np.array_equal(bits(a)[~na], bits(b)[~nb])


def assert_same_run(gpu, ref, check_model=True, nan_aware=False):
    """Bit-for-bit: iteration count, stop reason, components, residual, model
    (nan_aware: NaN positions must agree, their bit patterns need not)."""
    st = gpu["stats"]
    assert st["n_iter"] == ref["n_iter"], (st["n_iter"], ref["n_iter"])
    assert st["stop_reason"] == ref["stop"], (st["stop_reason"], ref["stop"])
    gi, gf = host(gpu["idx"]), host(gpu["flux"])
    if not np.array_equal(gi, ref["idx"]):
        k = int(np.argmax(gi != ref["idx"]))
        raise AssertionError(f"component {k}: index {gi[k]} vs oracle {ref['idx'][k]}")
    if not np.array_equal(bits(gf), bits(ref["flux"])):
        k = int(np.argmax(bits(gf) != bits(ref["flux"])))
        raise AssertionError(f"component {k}: flux {gf[k]!r} vs oracle {ref['flux'][k]!r}")
    gr = host(gpu["residual"])
    if not same_bits(gr, ref["residual"], nan_aware):
        d = np.abs(gr.astype(np.float64) - ref["residual"])
        raise AssertionError(f"residual differs at {np.count_nonzero(bits(gr) != bits(ref['residual']))} px, "
                             f"max |diff| {d.max()}")
    if check_model and gpu["model"] is not None:
        gm = host(gpu["model"])
        assert same_bits(gm, ref["model"], nan_aware), "model image differs"
