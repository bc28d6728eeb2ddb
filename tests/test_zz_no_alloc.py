"""The allocation-free gather (string_batch_gather_output_noalloc) through the
C ABI: its rows, progress and flags equal string_batch_gather_output's on two
calls in a row, the second smaller, and it refuses more rows than its fixed
scratch holds."""
from __future__ import annotations

import ctypes as C

import numpy as np
import pytest

from paper_2311_18505_amd import binding, hiptime, workloads as W

pytestmark = pytest.mark.gpu


def _noalloc(b, slots, offs, count):
    """Rows gathered by the allocation-free entry point into a device buffer
    (allocated here by the test, outside the call), copied back."""
    h = hiptime.hip()
    sl = np.ascontiguousarray(slots, dtype=np.int32)
    of = np.ascontiguousarray(offs, dtype=np.int64)
    rows = np.zeros((len(sl), count), dtype=b.dtype)
    done = np.zeros(len(sl), dtype=np.int64)
    flags = np.zeros(len(sl), dtype=np.int32)
    dptr = C.c_void_p()
    assert h.hipMalloc(C.byref(dptr), max(1, rows.nbytes)) == 0
    try:
        st = b.lib.string_batch_gather_output_noalloc(
            b.h, len(sl), sl.ctypes.data_as(C.POINTER(C.c_int32)), of.ctypes.data_as(C.POINTER(C.c_int64)), count,
            dptr, done.ctypes.data_as(C.POINTER(C.c_int64)), flags.ctypes.data_as(C.POINTER(C.c_int32)))
        assert h.hipMemcpy(rows.ctypes.data_as(C.c_void_p), dptr, rows.nbytes, 2) == 0   # device to host
    finally:
        h.hipFree(dptr)
    return st, rows, done, flags


@pytest.mark.parametrize("precision", ["fp32c", "fp64"])
def test_noalloc_gather_equals_gather(precision):
    if not binding.device_available():
        pytest.skip("no GPU")
    items = W.random_batch(12, seconds=0.03, seed=W.SEED + 77)
    b = binding.StringBatch(12, precision)
    b.set_params(0, [p for p, _ in items])
    b.excite(0, [e for _, e in items])
    b.step(700)
    calls = [([4, 0, 11, 7, 2, 9, 3], [0, 100, 250, 699, 5, 640, 1400], 96),
             ([6, 1], [33, 0], 40)]
    for k, (slots, offs, count) in enumerate(calls):
        print("[gpu] noalloc %s call %d: %d rows x %d" % (precision, k, len(slots), count), flush=True)
        ref, rdone, rflags = b.gather_output(slots, offs, count, status=True)
        st, rows, done, flags = _noalloc(b, slots, offs, count)
        assert st == binding.SB_OK
        assert np.array_equal(rows, ref)
        assert np.array_equal(done, rdone) and np.array_equal(flags, rflags)
        assert np.all(done == 702) and np.all(flags == 0)
    # more rows than the fixed scratch holds are refused before any work
    n = binding.SB_NOALLOC_MAX_ROWS + 1
    z32, z64 = np.zeros(n, dtype=np.int32), np.zeros(n, dtype=np.int64)
    st = b.lib.string_batch_gather_output_noalloc(b.h, n, z32.ctypes.data_as(C.POINTER(C.c_int32)),
                                                  z64.ctypes.data_as(C.POINTER(C.c_int64)), 8, None, None, None)
    assert st == binding.SB_EINVAL
    assert "maximum" in b.lib.string_batch_last_error(b.h).decode()
    b.close()
