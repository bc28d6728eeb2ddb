"""Clamped string ends (Sec. 4.1, eq. (10)) on the GPU through the C ABI.

* mixed batches (every third string simply supported, the rest clamped, so
  waves hold both; clamped strings in all seven size classes) against the FP64
  oracle: FP64 rel-L2 <= 1e-10, FP32
  compensated <= 1e-3;
* the plain FP64 comparator with clamped ends, <= 1e-10;
* the FP64 energy monitor equals the oracle's clamped energy;
* FP32 compensated partials of a clamped string within 0.1 cent of the
  oracle's, and raised over the simply supported string's by the amount the
  oracle shows.
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


def _run(items, precision):
    print("[gpu] %s: %d strings (%d clamped), up to %d samples" % (
        precision, len(items), sum(p.get("boundary", 0) for p, _ in items),
        max(p["n_samples"] for p, _ in items)), flush=True)
    b = binding.StringBatch(len(items), precision)
    b.set_params(0, [p for p, _ in items])
    b.excite(0, [e for _, e in items])
    b.step(max(p["n_samples"] for p, _ in items))
    outs = [b.read_output(i) for i in range(len(items))]
    infos = [b.info(i) for i in range(len(items))]
    energies = [b.read_energy(i) for i in range(len(items))]
    b.close()
    print("[gpu] batch done", flush=True)
    return outs, infos, energies


def _mixed(n, seconds, seed):
    items = W.random_batch(n, seconds=seconds, seed=seed)
    items = [(dict(p, boundary=0 if i % 3 == 2 else 1), e) for i, (p, e) in enumerate(items)]
    # low clamped strings in the two largest size classes, hammered and plucked
    low = W.string(20.7, 1e-5, 1.2, 0.5, 1e-4, int(seconds * 48000))
    mid = W.string(40.0, 1e-5, 1.1, 0.5, 1e-4, int(seconds * 48000))
    return items + [(dict(low, boundary=1), W.hammer(0.12, 2.0)), (dict(mid, boundary=1), W.pluck(0.2, 1e-3))]


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32c", 1e-3)])
def test_clamped_mixed_batch(precision, tol):
    _gpu()
    items = _mixed(24, 0.05, seed=17)
    refs = [r["y_u"] for r in oracle.run_many(items)]
    outs, infos, _ = _run(items, precision)
    errs = [rel_l2(y, r) for y, r in zip(outs, refs)]
    print("[gpu] %s clamped batch: worst rel-L2 %.3e" % (precision, max(errs)), flush=True)
    assert all(i["flags"] == 0 for i in infos)
    assert set(i["size_class"] for (p, _), i in zip(items, infos) if p["boundary"] == 1) == set(range(8))
    assert max(errs) <= tol


@pytest.mark.parametrize("which", ["linear", "nonlinear"])
def test_clamped_plain_fp64(which):
    _gpu()
    p, e = W.single_linear(seconds=0.25) if which == "linear" else W.single_nonlinear(seconds=0.25)
    p = dict(p, boundary=1)
    ref = oracle.run(p, e)["y_u"]
    (y,), (inf,), _ = _run([(p, e)], "fp64_plain")
    err = rel_l2(y, ref)
    print("[gpu] plain fp64 clamped %s: rel-L2 %.3e" % (which, err), flush=True)
    assert inf["samples_done"] == p["n_samples"]
    assert err <= 1e-10


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32c", 1e-4)])
def test_clamped_energy_monitor_matches_oracle(precision, tol):
    _gpu()
    p = dict(W.string(300.0, 1e-3, 3.0, 1.0, 3e-4, 4802), boundary=1)
    e = W.pluck(0.14, 0.02)
    ref = oracle.run(p, e, want=("y_u", "energy"))
    (y,), (inf,), ((H, step),) = _run([(p, e)], precision)
    print("[gpu] clamped H^{n+1/2} at n=%d: gpu %.15e oracle %.15e" % (step, H, ref["energy"][step]), flush=True)
    assert step == 4799 and inf["flags"] == 0
    assert abs(H - ref["energy"][step]) <= tol * abs(ref["energy"][step])


def test_clamped_fp32c_partials():
    _gpu()
    p, e = W.single_linear(seconds=1.0)
    p = dict(p, sigma0_t=0.0, sigma1_t=0.0)
    modes = np.array([1, 2, 3, 4])
    guesses = modes * p["f0"] * np.sqrt(1 + p["B"] * modes ** 2)
    refs = oracle.run_many([(dict(p, boundary=1), e), (p, e)])
    outs, _, _ = _run([(dict(p, boundary=1), e), (p, e)], "fp32c")
    f = [fit_partials(np.asarray(y, np.float64), p["fs"], guesses, decay_guess=0.0, max_samples=24000)[0]
         for y in (outs[0], outs[1], refs[0]["y_u"], refs[1]["y_u"])]
    dc = cents(f[0], f[2])
    raise_gpu, raise_ref = cents(f[0], f[1]), cents(f[2], f[3])
    print("[gpu] clamped partial offsets %s; raise gpu %s oracle %s (cents)"
          % (np.round(dc, 5), np.round(raise_gpu, 3), np.round(raise_ref, 3)), flush=True)
    assert np.max(np.abs(dc)) <= 0.1
    assert np.all(raise_ref > 3.0)
    assert np.max(np.abs(raise_gpu - raise_ref)) <= 0.1
