"""Edge cases of the C ABI on the GPU: an empty batch, zero steps, stepping
past the end of a string, ragged durations in one batch, a string of two
samples, reads outside the output, out-of-order calls."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2311_18505_amd import binding, workloads as W

pytestmark = pytest.mark.gpu


def _gpu():
    if not binding.device_available():
        pytest.skip("no GPU")
    print("[gpu] device ready", flush=True)


def _code(fn):
    with pytest.raises(binding.SbError) as ex:
        fn()
    return ex.value.code


@pytest.mark.parametrize("precision", ["fp64", "fp32c", "fp64_plain"])
def test_edge_cases(precision):
    _gpu()
    b = binding.StringBatch(4, precision)
    try:
        # nothing set or excited: stepping is out of order, reading too
        assert _code(lambda: b.step(10)) == binding.SB_ESTATE
        p0, e0 = W.single_nonlinear(seconds=0.01)
        assert _code(lambda: b.excite(0, [e0])) == binding.SB_ESTATE
        # ragged durations, one string of two samples (the initial
        # conditions only), and an unexcited slot in between
        items = [(dict(p0, n_samples=480), e0), (dict(p0, n_samples=2), e0),
                 (dict(p0, n_samples=97), W.pluck(0.3, 1e-3))]
        b.set_params(0, [p for p, _ in items])
        b.excite(0, [e for _, e in items])
        b.step(0)                                   # no-op
        b.step(100)
        b.step(10000)                               # clamps at each string's end
        b.step(5)                                   # all done: nothing to step
        refs = oracle.run_many(items)
        for i, ((p, _), r) in enumerate(zip(items, refs)):
            inf = b.info(i)
            y = b.read_output(i)
            err = float(np.linalg.norm(np.asarray(y, np.float64) - r["y_u"]) / max(np.linalg.norm(r["y_u"]), 1e-300))
            print("[gpu] %s slot %d: %d samples, done %d, rel-L2 %.3e" % (precision, i, p["n_samples"],
                                                                          inf["samples_done"], err), flush=True)
            assert inf["samples_done"] == p["n_samples"] and inf["flags"] == 0
            assert err <= (1e-10 if precision != "fp32c" else 1e-3)
        # reads outside the output, and of the slot never excited
        assert _code(lambda: b.read_output(0, 470, 20)) == binding.SB_EINVAL
        assert _code(lambda: b.read_output(3, 0, 1)) == binding.SB_ESTATE
        assert _code(lambda: b.read_output(7, 0, 1)) == binding.SB_EINVAL
        # a negative step count
        assert _code(lambda: b.step(-1)) == binding.SB_EINVAL
    finally:
        b.close()
