"""GPU serving: continuous batching through the C ABI.

Requests arrive while others are being stepped and join the next chunk
launch; each request's audio must be the same as when it is synthesised
alone (every string's arithmetic is independent of its neighbours in a
wavefront and of the chunking), and every request must finish.
"""
from __future__ import annotations

import numpy as np
import pytest

from paper_2311_18505_amd import binding, serving, workloads as W

pytestmark = pytest.mark.gpu


def _gpu():
    if not binding.device_available():
        pytest.skip("no GPU")
    print("[gpu] device ready", flush=True)


def _alone(req):
    b = binding.StringBatch(1, "fp32c")
    b.set_params(0, [req.params])
    b.excite(0, [req.excitation])
    b.step(req.params["n_samples"])
    y = b.read_output(0)
    b.close()
    return y


def test_serving_alone_equals_mix():
    _gpu()
    arrivals, items = W.serving_requests(rate_hz=600.0, seconds=0.5)
    # short requests keep the test quick: 0.05 .. 0.3 s
    rng = np.random.default_rng(7)
    for p, _ in items:
        p["n_samples"] = int(rng.integers(2400, 14400))
    reqs = serving.requests_from(arrivals, items)
    keep = [r.rid for r in reqs[::max(1, len(reqs) // 6)]][:6]
    print("[gpu] serving %d requests, keeping %s" % (len(reqs), keep), flush=True)
    srv = serving.Server(capacity=256)
    stats, outs = srv.run(reqs, keep=keep)
    srv.close()
    summ = stats.summary()
    print("[gpu] served:", summ, flush=True)
    assert summ["requests_done"] == len(reqs) and summ["refused"] == 0
    assert summ["max_active"] > 1      # requests overlapped on the device
    for rid in keep:
        y_mix = outs[rid]
        y_one = _alone(reqs[rid])
        assert y_mix.shape == y_one.shape
        diff = float(np.max(np.abs(y_mix.astype(np.float64) - y_one)))
        print("[gpu] request %d: %d samples, max |mix - alone| = %.3e" % (rid, len(y_one), diff), flush=True)
        assert np.all(np.isfinite(y_one))
        assert diff == 0.0


def test_gather_output_matches_read_output():
    _gpu()
    items = W.random_batch(10, seconds=0.02)
    b = binding.StringBatch(10, "fp32c")
    b.set_params(0, [p for p, _ in items])
    b.excite(0, [e for _, e in items])
    b.step(960)
    slots = [3, 0, 7, 9]
    offs = [0, 100, 500, 959]
    rows = b.gather_output(slots, offs, 64)
    for i, (s, o) in enumerate(zip(slots, offs)):
        n = min(64, items[s][0]["n_samples"] - o)
        ref = b.read_output(s, o, n)
        assert np.array_equal(rows[i, :n], ref)
    b.close()
