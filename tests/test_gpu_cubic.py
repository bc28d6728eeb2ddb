"""The hammer's cubic interpolant (Sec. 3.3 with p = 3) on the GPU through the
C ABI: mixed batches of cubic and linear hammers (some clamped, one struck
in the first interval where a mirrored ghost node enters) against the
oracle -- FP64 rel-L2 <= 1e-10, FP32 compensated <= 1e-3; a re-excitation by a
cubic hammer mid-note; the plain path's refusal."""
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


def _items(seconds):
    items = []
    for i, (p, e) in enumerate(W.random_batch(24, seconds=seconds, seed=W.SEED + 41)):
        if e["type"] == 2:
            e = dict(e, interp_order=3 if i % 4 else 1)
        items.append((dict(p, boundary=1 if i % 5 == 0 else 0), e))
    q = W.string(300.0, 1e-3, 3.0, 1.0, 3e-4, int(seconds * 48000))
    items.append((q, dict(W.hammer(0.02, 3.0), interp_order=3)))
    items.append((dict(q, boundary=1), dict(W.hammer(0.02, 3.0), interp_order=3)))
    return items


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32c", 1e-3)])
def test_cubic_hammer_batch(precision, tol):
    _gpu()
    items = _items(0.05)
    n_cubic = sum(1 for _, e in items if e.get("interp_order") == 3)
    refs = oracle.run_many(items)
    print("[gpu] %s: %d strings, %d cubic hammers" % (precision, len(items), n_cubic), flush=True)
    b = binding.StringBatch(len(items), precision)
    try:
        b.set_params(0, [p for p, _ in items])
        b.excite(0, [e for _, e in items])
        b.step(max(p["n_samples"] for p, _ in items))
        outs = [b.read_output(i) for i in range(len(items))]
        infos = [b.info(i) for i in range(len(items))]
    finally:
        b.close()
    errs = [rel_l2(y, r["y_u"]) for y, r in zip(outs, refs)]
    worst = int(np.argmax(errs))
    print("[gpu] %s cubic batch: worst rel-L2 %.3e (string %d)" % (precision, errs[worst], worst), flush=True)
    assert n_cubic >= 10
    assert all(inf["flags"] == 0 for inf in infos)
    assert max(errs) <= tol


def test_cubic_hammer_restrike_fp64():
    _gpu()
    p = W.string(300.0, 1e-3, 3.0, 1.0, 3e-4, 4800)
    e0 = W.pluck(0.2, 1e-3)
    ham = dict(W.hammer(0.13, 3.0), interp_order=3)
    step = 959          # the step that computes sample 960
    ref = oracle.run(p, e0, schedule=[(step, ham)])["y_u"]
    b = binding.StringBatch(1, "fp64")
    try:
        b.set_params(0, [p])
        b.excite(0, [e0])
        b.step(step + 1 - 2)
        b.restrike_list([0], [ham])
        b.step(p["n_samples"])
        y = b.read_output(0)
    finally:
        b.close()
    err = rel_l2(y, ref)
    print("[gpu] cubic hammer re-excitation fp64: rel-L2 %.3e" % err, flush=True)
    assert err <= 1e-10


def test_cubic_hammer_refused_on_the_plain_path():
    _gpu()
    p, _ = W.single_nonlinear(seconds=0.01)
    b = binding.StringBatch(1, "fp64_plain")
    try:
        b.set_params(0, [p])
        with pytest.raises(binding.SbError) as ex:
            b.excite(0, [dict(W.hammer(0.12, 2.0), interp_order=3)])
        assert ex.value.code == binding.SB_EINVAL
    finally:
        b.close()
