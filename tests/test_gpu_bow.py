"""GPU parity of the bow (eq. 5) through the C ABI against the FP64 oracle.

The bow adds, in every sweep of the coupled solve, the exact solution of the
step's stick/slip problem (a rank-one correction along g = T_u0^{-1} J_p(x_B));
at convergence the step solves the same equations as the oracle's direct
method, so FP64 agrees to rounding.  Cases: the single bowed string (fixed
and moving bow), a seeded batch of bowed nonlinear strings mixed with plucks
and hammers, a low string in the largest size class, FP32 compensated, and
the plain path's refusal.
"""
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


def rel_l2(y, ref):
    return float(np.linalg.norm(np.asarray(y, np.float64) - ref) / np.linalg.norm(ref))


def _run(items, precision):
    print("[gpu] bow %s: %d strings, up to %d samples" % (precision, len(items), max(p["n_samples"] for p, _ in items)),
          flush=True)
    b = binding.StringBatch(len(items), precision)
    b.set_params(0, [p for p, _ in items])
    b.excite(0, [e for _, e in items])
    b.step(max(p["n_samples"] for p, _ in items))
    outs = [b.read_output(i) for i in range(len(items))]
    infos = [b.info(i) for i in range(len(items))]
    b.close()
    return outs, infos


def _items():
    p, e = W.single_bowed(seconds=0.25)
    items = [(p, e), (p, dict(e, x_end=0.2))]
    items += W.bowed_batch(40, seconds=0.1)
    items += W.random_batch(8, seconds=0.1)
    # a low bowed string (largest size class), moving bow
    low = W.string(20.7, 1e-5, 1.2, 0.5, 1e-4, 2400)
    items.append((low, W.bow(0.1, 0.1, 60.0, x_end=0.13)))
    return items


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32c", 1e-3)])
def test_bowed_strings_match_oracle(precision, tol):
    _gpu()
    items = _items()
    refs = oracle.run_many(items)
    outs, infos = _run(items, precision)
    errs = [rel_l2(y, r["y_u"]) for y, r in zip(outs, refs)]
    worst = int(np.argmax(errs))
    print("[gpu] bow %s: median rel-L2 %.3e, worst %.3e (string %d, N=(%d,%d), class %d, max sweeps %d)"
          % (precision, np.median(errs), errs[worst], worst, infos[worst]["N_t"], infos[worst]["N_l"],
             infos[worst]["size_class"], infos[worst]["max_sweeps"]), flush=True)
    assert infos[-1]["size_class"] == 5
    assert all(inf["flags"] == 0 and inf["samples_done"] == p["n_samples"] for (p, _), inf in zip(items, infos))
    assert max(errs) <= tol


def test_plain_path_refuses_a_bow():
    _gpu()
    p, e = W.single_bowed(seconds=0.01)
    b = binding.StringBatch(1, "fp64_plain")
    b.set_params(0, [p])
    with pytest.raises(binding.SbError):
        b.excite(0, [e])
    b.close()
