"""Several excitations per note on the GPU against the oracle's schedule.

Strings start plucked, hammered or bowed; after some steps a new hammer or
bow is set on the sounding string (string_batch_restrike), some twice; the
output must match the oracle run with the same schedule (orc_run_schedule):
FP64 <= 1e-10, FP32 compensated <= 1e-3.
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


def _cases(seconds=0.05):
    ns = int(round(seconds * 48000))
    lin, _ = W.single_linear(seconds=seconds)
    nl = W.string(98.0, 2e-4, 2.5, 0.8, 3e-4, ns)
    hi = W.string(330.0, 1e-3, 1.8, 1.2, 2e-4, ns)
    low = W.string(20.7, 1e-5, 1.2, 0.5, 1e-4, ns)   # largest size class
    ham, bow = W.hammer(0.13, 2.5), W.bow(0.11, 0.1, 80.0, x_end=0.14)
    # (params, initial excitation, [(step, new excitation), ...])
    return [
        (lin, W.pluck(0.2, 1e-3), [(ns // 3, ham)]),
        (nl, W.hammer(0.12, 3.0), [(ns // 4, W.hammer(0.2, 2.0)), (ns // 2, bow)]),
        (nl, bow, [(ns // 3, W.hammer(0.17, 1.5))]),
        (hi, W.pluck(0.15, 5e-4), [(ns // 5, W.bow(0.09, 0.15, 150.0)), (ns // 2, W.bow(0.2, 0.05, 60.0))]),
        (low, W.hammer(0.1, 2.0), [(ns // 2, W.hammer(0.25, 2.0))]),
    ]


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32c", 1e-3)])
def test_restrike_matches_oracle_schedule(precision, tol):
    _gpu()
    cases = _cases()
    refs = [oracle.run(p, e, schedule=sch)["y_u"] for p, e, sch in cases]
    b = binding.StringBatch(len(cases), precision)
    b.set_params(0, [p for p, _, _ in cases])
    b.excite(0, [e for _, e, _ in cases])
    ns = cases[0][0]["n_samples"]
    events = sorted({n for _, _, sch in cases for n, _ in sch})
    done = 2
    for n in events:
        # step so that the next step computed is n (samples_done = n + 1)
        b.step(n + 1 - done)
        done = n + 1
        for i, (_, _, sch) in enumerate(cases):
            for m, x in sch:
                if m == n:
                    b.restrike(i, [x])
    b.step(ns - done)
    outs = [b.read_output(i) for i in range(len(cases))]
    infos = [b.info(i) for i in range(len(cases))]
    with pytest.raises(binding.SbError):
        b.rewind(0, 1)            # a re-excited slot cannot rewind to its excitation
    b.close()
    errs = [rel_l2(y, r) for y, r in zip(outs, refs)]
    print("[gpu] restrike %s: rel-L2 %s, classes %s" % (precision, np.array2string(np.array(errs), precision=2),
                                                         [inf["size_class"] for inf in infos]), flush=True)
    assert all(inf["flags"] == 0 and inf["samples_done"] == ns for inf in infos)
    assert max(errs) <= tol
