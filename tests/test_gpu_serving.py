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


def test_serving_alone_equals_mix_and_the_oracle():
    _gpu()
    import oracle
    arrivals, items = W.serving_requests(rate_hz=600.0, seconds=0.5)
    # short requests keep the test quick: 0.05 .. 0.3 s
    rng = np.random.default_rng(7)
    for p, _ in items:
        p["n_samples"] = int(rng.integers(2400, 14400))
    # one request on a transverse grid one point finer than the stability
    # bound (lossless linear pluck): it diverges, the energy monitor flags it
    # and it must fail alone
    bad_p, bad_e = W.single_linear(seconds=0.25)
    bad_p = dict(bad_p, sigma0_t=0.0, sigma1_t=0.0)
    bad_p["grid_t"] = binding.plan_grid(bad_p)[0] + 1
    items.insert(len(items) // 3, (bad_p, bad_e))
    arrivals = np.sort(np.append(arrivals, arrivals[len(arrivals) // 3]))
    reqs = serving.requests_from(arrivals, items)
    bad_rid = len(items) // 3
    keep = [r.rid for r in reqs[::max(1, len(reqs) // 8)]][:8] + [bad_rid]
    print("[gpu] serving %d requests, keeping %s, diverging request %d" % (len(reqs), keep, bad_rid), flush=True)
    srv = serving.Server(capacity=256)
    stats, outs = srv.run(reqs, keep=keep)
    srv.close()
    summ = stats.summary()
    print("[gpu] served:", summ, flush=True)
    assert stats.failed == [bad_rid]
    assert bad_rid not in outs
    assert summ["requests_done"] == len(reqs) - 1 and summ["refused"] == 0
    assert summ["max_active"] > 1      # requests overlapped on the device
    kept = [rid for rid in keep if rid != bad_rid]
    refs = oracle.run_many([(reqs[rid].params, reqs[rid].excitation) for rid in kept])
    for rid, ref in zip(kept, refs):
        y_mix = outs[rid]
        y_one = _alone(reqs[rid])
        assert y_mix.shape == y_one.shape == ref["y_u"].shape
        diff = float(np.max(np.abs(y_mix.astype(np.float64) - y_one)))
        err = float(np.linalg.norm(y_mix.astype(np.float64) - ref["y_u"]) / np.linalg.norm(ref["y_u"]))
        print("[gpu] request %d: %d samples, max |mix - alone| = %.3e, rel-L2 vs oracle %.3e"
              % (rid, len(y_one), diff, err), flush=True)
        assert np.all(np.isfinite(y_one))
        assert diff == 0.0
        assert err <= 1e-3


def test_flagged_slot_reads_as_unstable_and_zero_past_its_end():
    """A slot stopped by the energy monitor: gather and read return
    SB_EUNSTABLE with the samples it produced and zeros after them, never the
    stale contents of reused device memory; the other slots read normally."""
    _gpu()
    p, e = W.single_linear(seconds=0.25)
    p = dict(p, sigma0_t=0.0, sigma1_t=0.0)
    nt, _ = binding.plan_grid(p)
    b = binding.StringBatch(2, "fp64")
    b.set_params(0, [p, dict(p, grid_t=nt + 1)])
    b.excite(0, [e, e])
    b.step(p["n_samples"])
    rows, done, flags = b.gather_output([0, 1], [0, 0], p["n_samples"], status=True)
    print("[gpu] flagged slot: done %s flags %s" % (list(done), list(flags)), flush=True)
    assert flags[0] == 0 and done[0] == p["n_samples"]
    assert flags[1] & 1 and 2 < done[1] < p["n_samples"]
    # (the samples before the check that flagged it may already have blown up)
    assert np.all(rows[1, done[1]:] == 0.0)
    with pytest.raises(binding.SbError) as ei:
        b.gather_output([1], [0], 16)
    assert ei.value.code == binding.SB_EUNSTABLE
    with pytest.raises(binding.SbError) as ei:
        b.read_output(1)
    assert ei.value.code == binding.SB_EUNSTABLE
    assert np.array_equal(b.read_output(0), rows[0])
    b.close()


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
