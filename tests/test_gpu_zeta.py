"""The second readout channel, zeta at x_out (Sec. 3.4 shows u and zeta
outputs), on the GPU through the C ABI.

* mixed batches (two strings in three with the channel; hammers, plucks, a
  bow and a clamped string among them) against the oracle's zeta readout:
  FP64 rel-L2 <= 1e-10, FP32 compensated <= 1e-3, u unchanged to the same
  bounds;
* a nonlinear plucked string over 1 s in FP32 compensated: zeta within 1e-3
  and its strongest spectral peaks (the longitudinal modes and the phantom
  partials the transverse motion drives) at the oracle's frequencies within
  0.1 cent;
* the plain FP64 path refuses the channel, and a slot set without it
  refuses the read.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2311_18505_amd import analysis, binding, workloads as W

pytestmark = pytest.mark.gpu


def _gpu():
    if not binding.device_available():
        pytest.skip("no GPU")
    print("[gpu] device ready", flush=True)


def rel_l2(y, ref):
    return float(np.linalg.norm(np.asarray(y, np.float64) - ref) / np.linalg.norm(ref))


def _items(seconds):
    items = W.random_batch(24, seconds=seconds, seed=W.SEED + 23)
    items = [(dict(p, readout_zeta=0 if i % 3 == 2 else 1), e) for i, (p, e) in enumerate(items)]
    bowed = W.bowed_batch(1, seconds=seconds)[0]
    items.append((dict(bowed[0], readout_zeta=1), bowed[1]))
    items.append((dict(W.single_nonlinear(seconds=seconds)[0], readout_zeta=1, boundary=1), W.single_nonlinear()[1]))
    return items


def _run(items, precision):
    print("[gpu] %s: %d strings (%d with the zeta channel)"
          % (precision, len(items), sum(p["readout_zeta"] for p, _ in items)), flush=True)
    b = binding.StringBatch(len(items), precision)
    try:
        b.set_params(0, [p for p, _ in items])
        b.excite(0, [e for _, e in items])
        b.step(max(p["n_samples"] for p, _ in items))
        u = [b.read_output(i) for i in range(len(items))]
        z = [b.read_output_zeta(i) if p["readout_zeta"] else None for i, (p, _) in enumerate(items)]
        infos = [b.info(i) for i in range(len(items))]
        refused = None
        off = [i for i, (p, _) in enumerate(items) if not p["readout_zeta"]]
        if off:
            try:
                b.read_output_zeta(off[0])
            except binding.SbError as ex:
                refused = ex.code
    finally:
        b.close()
    print("[gpu] batch done", flush=True)
    return u, z, infos, refused


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32c", 1e-3)])
def test_zeta_channel_mixed_batch(precision, tol):
    _gpu()
    items = _items(0.05)
    refs = oracle.run_many(items, want=("y_u", "y_z"))
    u, z, infos, refused = _run(items, precision)
    eu = [rel_l2(y, r["y_u"]) for y, r in zip(u, refs)]
    ez = [rel_l2(y, r["y_z"]) for y, r, (p, _) in zip(z, refs, items) if p["readout_zeta"] and np.any(r["y_z"])]
    print("[gpu] %s: worst u rel-L2 %.3e, worst zeta rel-L2 %.3e over %d channels"
          % (precision, max(eu), max(ez), len(ez)), flush=True)
    assert all(i["flags"] == 0 for i in infos)
    assert refused == binding.SB_ESTATE
    assert len(ez) >= 16
    assert max(eu) <= tol and max(ez) <= tol


def test_zeta_channel_one_second_spectrum():
    _gpu()
    p = dict(W.string(110.0, 1e-4, 3.0, 0.5, 1e-4, 48000), readout_zeta=1)
    e = W.pluck(0.2, 3e-3)
    ref = oracle.run(p, e, want=("y_z",))["y_z"]
    (u,), (z,), _, _ = _run([(p, e)], "fp32c")
    err = rel_l2(z, ref)
    f_ref, l_ref = analysis.find_peaks(ref, p["fs"], floor_db=-60.0)
    f_gpu, l_gpu = analysis.find_peaks(np.asarray(z, np.float64), p["fs"], floor_db=-60.0)
    top = np.argsort(l_ref)[::-1][:6]
    offs = [1200 * np.log2(f_gpu[np.argmin(np.abs(f_gpu - f_ref[i]))] / f_ref[i]) for i in top]
    print("[gpu] zeta 1 s fp32c: rel-L2 %.3e; strongest peaks %s Hz, offsets (cents) %s"
          % (err, np.round(f_ref[top], 2), np.round(offs, 4)), flush=True)
    assert err <= 1e-3
    assert np.max(np.abs(offs)) <= 0.1


def test_zeta_channel_refused_on_the_plain_path():
    _gpu()
    p, _ = W.single_nonlinear(seconds=0.01)
    b = binding.StringBatch(1, "fp64_plain")
    try:
        with pytest.raises(binding.SbError) as ex:
            b.set_params(0, [dict(p, readout_zeta=1)])
        assert ex.value.code == binding.SB_EINVAL
    finally:
        b.close()
