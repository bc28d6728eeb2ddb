"""GPU physics and full-size parity through the C ABI.

* the FP64 energy monitor computed on the GPU equals the oracle's discrete
  energy H^{n+1/2} at its check steps;
* a grid one point finer than the stability bound is flagged by the monitor
  and stops (the bound is sharp);
* stepping in chunks equals stepping at once, bit for bit;
* FP32 compensated output keeps the partial frequencies of the FP64 oracle
  within 0.1 cent and rel-L2 within 1e-3 over 1 s;
* full sizes: the single nonlinear string (2 s, FP64, rel-L2 <= 1e-10), the
  64-string subset of the uniform batch (2 s, FP32 compensated, <= 1e-3),
  theta = 1 and the largest size class.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2311_18505_amd import binding, workloads as W
from tests.spectral import cents, fit_partials

pytestmark = pytest.mark.gpu


def _gpu():
    if not binding.device_available():
        pytest.skip("no GPU")
    print("[gpu] device ready", flush=True)


def rel_l2(y, ref):
    return float(np.linalg.norm(np.asarray(y, np.float64) - ref) / np.linalg.norm(ref))


def _run(items, precision, chunk=None, monitor=None):
    print("[gpu] %s: %d strings, up to %d samples" % (precision, len(items), max(p["n_samples"] for p, _ in items)),
          flush=True)
    b = binding.StringBatch(len(items), precision)
    b.set_params(0, [p for p, _ in items])
    b.excite(0, [e for _, e in items])
    if monitor is not None:
        b.set_monitor(*monitor)
    n = max(p["n_samples"] for p, _ in items)
    if chunk is None:
        b.step(n)
    else:
        for _ in range(0, n, chunk):
            b.step(chunk)
    outs = []
    for i in range(len(items)):
        try:
            outs.append(b.read_output(i))
        except binding.SbError as err:     # a flagged slot reads as unstable
            assert err.code == binding.SB_EUNSTABLE
            outs.append(None)
    infos = [b.info(i) for i in range(len(items))]
    energies = [b.read_energy(i) for i in range(len(items))]
    b.close()
    return outs, infos, energies


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32c", 1e-4)])
def test_energy_monitor_matches_oracle(precision, tol):
    _gpu()
    # a lossy nonlinear pluck (no hammer, constant f0): the monitor checks growth
    p = W.string(300.0, 1e-3, 3.0, 1.0, 3e-4, 4802)
    e = W.pluck(0.14, 0.02)
    ref = oracle.run(p, e, want=("y_u", "energy"))
    (y,), (inf,), ((H, step),) = _run([(p, e)], precision)
    print("[gpu] H^{n+1/2} at n=%d: gpu %.15e oracle %.15e" % (step, H, ref["energy"][step]), flush=True)
    assert step == 4799 and inf["flags"] == 0
    assert abs(H - ref["energy"][step]) <= tol * abs(ref["energy"][step])


def test_one_point_finer_grid_is_flagged():
    _gpu()
    p, e = W.single_linear(seconds=0.25)
    p = dict(p, sigma0_t=0.0, sigma1_t=0.0)
    nt, _ = binding.plan_grid(p)
    good = dict(p)
    bad = dict(p, grid_t=nt + 1)
    outs, infos, _ = _run([(good, e), (bad, e)], "fp64")
    print("[gpu] stable: flags %d done %d; one point finer: flags %d done %d"
          % (infos[0]["flags"], infos[0]["samples_done"], infos[1]["flags"], infos[1]["samples_done"]), flush=True)
    assert infos[0]["flags"] == 0 and infos[0]["samples_done"] == p["n_samples"]
    assert infos[1]["flags"] & 1
    assert infos[1]["samples_done"] < p["n_samples"]
    # reading the flagged slot returns SB_EUNSTABLE; the stable one reads normally
    assert outs[0] is not None and outs[1] is None


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_chunked_equals_one_shot(precision):
    _gpu()
    items = W.random_batch(48, seconds=0.06, modulation=True)
    whole, _, _ = _run(items, precision)
    chunked, _, _ = _run(items, precision, chunk=480)
    odd, _, _ = _run(items, precision, chunk=333)
    for a, b, c in zip(whole, chunked, odd):
        assert np.array_equal(a, b) and np.array_equal(a, c)


@pytest.mark.parametrize("which", ["linear", "nonlinear"])
def test_fp32c_partials_within_a_tenth_of_a_cent(which):
    _gpu()
    if which == "linear":
        p, e = W.single_linear(seconds=1.0)
        modes = np.array([1, 2, 3, 4, 6, 7])
    else:
        p, e = W.single_nonlinear(seconds=1.0)
        modes = np.array([1, 2, 3, 4, 5])
    ref = oracle.run(p, e, want=("y_u",))["y_u"]
    (y,), (inf,), _ = _run([(p, e)], "fp32c")
    err = rel_l2(y, ref)
    guesses = modes * p["f0"] * np.sqrt(1 + p["B"] * modes ** 2)
    f_ref, _, _ = fit_partials(ref[2400:], p["fs"], guesses)
    f_gpu, _, _ = fit_partials(np.asarray(y, np.float64)[2400:], p["fs"], guesses)
    dc = cents(f_gpu, f_ref)
    print("[gpu] %s fp32c: rel-L2 %.3e, partial offsets (cents) %s" % (which, err, np.round(dc, 5)), flush=True)
    assert err <= 1e-3
    assert np.max(np.abs(dc)) <= 0.1


def test_fp64_nonlinear_full_two_seconds():
    _gpu()
    p, e = W.single_nonlinear(seconds=2.0)
    ref = oracle.run(p, e, want=("y_u",))["y_u"]
    (y,), (inf,), _ = _run([(p, e)], "fp64")
    err = rel_l2(y, ref)
    print("[gpu] nonlinear 2 s fp64: rel-L2 %.3e, max sweeps %d" % (err, inf["max_sweeps"]), flush=True)
    assert inf["samples_done"] == p["n_samples"]
    assert err <= 1e-10


def test_uniform_batch_subset_fp32c():
    """The 64-string subset of the 4096-string uniform batch, full 2 s."""
    _gpu()
    items = W.uniform_batch_4096()[:64]
    print("[cpu] oracle on 64 strings x 2 s", flush=True)
    refs = oracle.run_many(items)
    outs, infos, _ = _run(items, "fp32c")
    errs = [rel_l2(y, r["y_u"]) for y, r in zip(outs, refs)]
    worst = int(np.argmax(errs))
    print("[gpu] subset fp32c: median rel-L2 %.3e, worst %.3e (string %d, N=(%d,%d))"
          % (np.median(errs), errs[worst], worst, infos[worst]["N_t"], infos[worst]["N_l"]), flush=True)
    assert all(inf["samples_done"] == p["n_samples"] and inf["flags"] == 0 for (p, _), inf in zip(items, infos))
    assert max(errs) <= 1e-3


def test_theta_one_and_largest_class_fp64():
    _gpu()
    lin = W.single_linear(seconds=0.5, theta=1.0)
    big = (W.string(20.7, 1e-5, 3.0, 1.0, 1e-4, 2400), W.hammer(0.15, 2.0))
    wide = (W.string(35.6, 1e-5, 1.3, 1.0, 1e-4, 2400), W.pluck(0.2, 1e-3))
    items = [lin, big, wide]
    refs = oracle.run_many(items)
    outs, infos, _ = _run(items, "fp64")
    for (p, _), y, r, inf in zip(items, outs, refs, infos):
        err = rel_l2(y, r["y_u"])
        print("[gpu] N=(%d,%d) class %d: rel-L2 %.3e" % (inf["N_t"], inf["N_l"], inf["size_class"], err), flush=True)
        assert err <= 1e-10
    assert infos[1]["size_class"] == 6 and infos[2]["size_class"] == 6


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32c", 1e-3)])
def test_maximum_grid_sizes(precision, tol):
    """The largest grids the batched paths accept (1024 intervals, the top of
    size class 7): N_l = 1024 (hammered, nonlinear) and N_t = 1024 (plucked,
    linear), beside a small string in the same batch; one interval more is
    refused with SB_EBUDGET."""
    _gpu()
    long_l = (W.string(20.0, 1e-6, 1.1713, 0.5, 1e-4, 2400), W.hammer(0.12, 2.0))
    long_t = (W.string(14.88, 1e-8, 1.0, 0.5, 1e-4, 2400), W.pluck(0.2, 1e-3))
    small = W.random_batch(1, seconds=0.05)[0]
    items = [long_l, long_t, small]
    refs = oracle.run_many(items)
    outs, infos, _ = _run(items, precision)
    assert (infos[0]["N_l"], infos[1]["N_t"]) == (1024, 1024)
    for y, r, inf in zip(outs, refs, infos):
        err = rel_l2(y, r["y_u"])
        print("[gpu] %s N=(%d,%d) class %d: rel-L2 %.3e" % (precision, inf["N_t"], inf["N_l"], inf["size_class"], err),
              flush=True)
        assert inf["flags"] == 0 and err <= tol
    b = binding.StringBatch(1, precision)
    try:
        with pytest.raises(binding.SbError) as ex:
            b.set_params(0, [W.string(14.87, 1e-8, 1.0, 0.5, 1e-4, 2400)])
        assert ex.value.code == binding.SB_EBUDGET
    finally:
        b.close()
