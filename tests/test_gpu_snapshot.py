"""Checkpoint and resume of slots through the C ABI (string_batch_snapshot /
string_batch_restore): step(a) + snapshot + step(c) + restore + step(b)
equals step(a + b) bit for bit, output, progress and energy monitor, on every
batched path and on the plain FP64 path, with host and device buffers; and the
refusals (another slot's snapshot, a wrong size, a damaged header, a slot
re-excited since the snapshot)."""
from __future__ import annotations

import ctypes as C

import numpy as np
import pytest

from paper_2311_18505_amd import binding, hiptime, workloads as W

pytestmark = pytest.mark.gpu


def _gpu():
    if not binding.device_available():
        pytest.skip("no GPU")
    print("[gpu] device ready", flush=True)


def _items():
    """Plucks and hammers over several size classes, f0 modulation, a bowed
    string, clamped ends, the zeta channel and the cubic grid interpolant."""
    items = list(W.random_batch(10, seconds=0.05, modulation=True, seed=W.SEED + 91))
    p, e = W.single_bowed(seconds=0.05)
    items.append((p, e))
    q, f = items[2]
    items.append((dict(q, boundary=1, readout_zeta=1, alpha=max(q["alpha"], 1.5)), f))
    items.append((dict(items[3][0], grid_interp=3, alpha=max(items[3][0]["alpha"], 1.5)), items[3][1]))
    items.append((W.string(40.0, 1e-5, 1.1, 0.5, 1e-4, 2400), W.hammer(0.12, 2.0)))    # class 6
    return items


def _batch(items, precision):
    b = binding.StringBatch(len(items), precision)
    b.set_params(0, [p for p, _ in items])
    b.excite(0, [e for _, e in items])
    return b


def _final(b, items):
    outs = [b.read_output(i) for i in range(len(items))]
    zs = [b.read_output_zeta(i) if p.get("readout_zeta") else None for i, (p, _) in enumerate(items)]
    infos = [b.info(i) for i in range(len(items))]
    energies = [b.read_energy(i) for i in range(len(items))]
    return outs, zs, infos, energies


def _same(x, y):
    ox, zx, ix, ex = x
    oy, zy, iy, ey = y
    for k in range(len(ox)):
        assert np.array_equal(ox[k], oy[k]), "output of slot %d differs" % k
        assert (zx[k] is None) == (zy[k] is None)
        if zx[k] is not None:
            assert np.array_equal(zx[k], zy[k]), "zeta output of slot %d differs" % k
        for f in ("samples_done", "flags", "max_sweeps", "total_sweeps"):
            assert ix[k][f] == iy[k][f], "%s of slot %d differs" % (f, k)
        assert ex[k] == ey[k], "energy of slot %d differs" % k


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_snapshot_restore_resumes_bitwise(precision):
    _gpu()
    items = _items()
    n = max(p["n_samples"] for p, _ in items)
    a, c = 700, 900
    print("[gpu] snapshot %s: %d strings, %d samples, snapshot after %d" % (precision, len(items), n, a), flush=True)
    b = _batch(items, precision)
    try:
        b.step(n)
        ref = _final(b, items)
    finally:
        b.close()
    assert all(inf["flags"] == 0 for inf in ref[2])
    assert {inf["size_class"] for inf in ref[2]} >= {0, 1, 2, 3, 6}

    h = hiptime.hip()
    b = _batch(items, precision)
    dev = {}
    try:
        b.step(a)
        snaps = {}
        for i in range(len(items)):
            nb = b.snapshot_bytes(i)
            if i % 2:                                # device buffers for odd slots
                ptr = C.c_void_p()
                assert h.hipMalloc(C.byref(ptr), nb) == 0
                dev[i] = (ptr, nb)
                b.snapshot_device(i, ptr.value, nb)
            else:
                snaps[i] = b.snapshot(i)
        b.step(c)                                   # a continuation that is thrown away
        for i in range(len(items)):
            if i % 2:
                b.restore_device(i, dev[i][0].value, dev[i][1])
            else:
                b.restore(i, snaps[i])
        assert all(b.info(i)["samples_done"] == min(a + 2, items[i][0]["n_samples"]) for i in range(len(items)))
        b.step(n - a)
        _same(_final(b, items), ref)
        # a finished slot restored again resumes the same way
        b.restore(0, snaps[0])
        b.step(n - a)
        assert np.array_equal(b.read_output(0), ref[0][0])
    finally:
        for ptr, _ in dev.values():
            h.hipFree(ptr)
        b.close()


def test_snapshot_restore_plain_fp64():
    _gpu()
    p, e = W.single_nonlinear(seconds=0.02)
    items = [(p, e)]
    b = _batch(items, "fp64_plain")
    try:
        b.step(p["n_samples"])
        ref = _final(b, items)
    finally:
        b.close()
    b = _batch(items, "fp64_plain")
    try:
        b.step(301)
        s = b.snapshot(0)
        b.step(200)
        b.restore(0, s)
        b.step(p["n_samples"])
        _same(_final(b, items), ref)
    finally:
        b.close()


def test_snapshot_refusals():
    _gpu()
    items = W.random_batch(3, seconds=0.02, seed=W.SEED + 92)
    items[1] = (dict(items[1][0]), W.hammer(0.13, 1.5))
    b = binding.StringBatch(4, "fp32c")
    try:
        b.set_params(0, [p for p, _ in items])
        with pytest.raises(binding.SbError) as ei:
            b.snapshot_bytes(0)                     # not excited yet
        assert ei.value.code == binding.SB_ESTATE
        b.excite(0, [e for _, e in items])
        b.step(200)
        s0, s1 = b.snapshot(0), b.snapshot(1)
        for bad, code in ((s1, binding.SB_EINVAL),          # another slot's snapshot
                          (s0[:-4], binding.SB_EINVAL),     # wrong size
                          (np.concatenate([s0, np.zeros(8, np.uint8)]), binding.SB_EINVAL)):
            with pytest.raises(binding.SbError) as ei:
                b.restore(0, bad)
            assert ei.value.code == code
        damaged = s0.copy()
        damaged[0] ^= 0xFF
        with pytest.raises(binding.SbError) as ei:
            b.restore(0, damaged)
        assert ei.value.code == binding.SB_EINVAL
        with pytest.raises(binding.SbError) as ei:
            b.snapshot(3)                          # never set
        assert ei.value.code == binding.SB_ESTATE
        # re-excited since the snapshot: refused; a fresh snapshot restores
        b.restrike(1, [W.hammer(0.13, 1.0)])
        with pytest.raises(binding.SbError) as ei:
            b.restore(1, s1)
        assert ei.value.code == binding.SB_ESTATE
        s1b = b.snapshot(1)
        b.step(100)
        b.restore(1, s1b)
        assert b.info(1)["samples_done"] == 202
        b.restore(0, s0)                           # the untouched slot still restores
    finally:
        b.close()
