"""Python binding of libstringfdtd (ctypes; argument marshalling only).

The functions mirror the C ABI of include/stringfdtd.h one to one; every step
of the synthesis runs in the HIP library.  ``StringBatch`` wraps a handle for
convenience.  There is no CPU fallback: without the built library (or without
a GPU) the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# STRINGFDTD_LIB names another build of the library (the LDS-poisoning debug
# build, libstringfdtd_poison.so, in its test)
LIB_PATH = os.environ.get("STRINGFDTD_LIB") or os.path.join(HERE, "libstringfdtd.so")

SB_OK, SB_EINVAL, SB_ENOMEM, SB_EBUDGET, SB_EUNSTABLE, SB_ESTATE, SB_EDEVICE = 0, -1, -2, -3, -4, -5, -6
SB_FP64, SB_FP32C, SB_FP64_PLAIN = 0, 1, 2
PRECISIONS = {"fp64": SB_FP64, "fp32c": SB_FP32C, "fp64_plain": SB_FP64_PLAIN}
# rows of the allocation-free gather's fixed scratch
SB_NOALLOC_MAX_ROWS = 16384
# concurrent launch units of a batched step: classes 0..4 merged, class 5,
# classes 6 and 7 one after the other
NUM_LAUNCHES = 3
LAUNCH_CLASSES = ((0, 1, 2, 3, 4), (5,), (6, 7))
STATUS_NAMES = {0: "SB_OK", -1: "SB_EINVAL", -2: "SB_ENOMEM", -3: "SB_EBUDGET", -4: "SB_EUNSTABLE",
                -5: "SB_ESTATE", -6: "SB_EDEVICE"}


class SbStringParams(C.Structure):
    _fields_ = [
        ("fs", C.c_double), ("f0", C.c_double), ("B", C.c_double), ("alpha", C.c_double),
        ("theta", C.c_double), ("sigma0_t", C.c_double), ("sigma1_t", C.c_double),
        ("sigma0_l", C.c_double), ("sigma1_l", C.c_double), ("x_out", C.c_double),
        ("n_samples", C.c_int64), ("mod_type", C.c_int32), ("grid_t", C.c_int32),
        ("mod_depth_cents", C.c_double), ("mod_rate_hz", C.c_double), ("glide_semitones", C.c_double),
        ("grid_l", C.c_int32), ("boundary", C.c_int32),
        ("readout_zeta", C.c_int32), ("grid_interp", C.c_int32),
    ]


class SbExcitation(C.Structure):
    _fields_ = [
        ("type", C.c_int32), ("interp_order", C.c_int32), ("x", C.c_double), ("c0", C.c_double),
        ("v_H", C.c_double), ("M_H", C.c_double), ("K_H", C.c_double), ("alpha_H", C.c_double),
        ("rhoA", C.c_double), ("x_end", C.c_double), ("v_B", C.c_double), ("F_B", C.c_double),
        ("attack", C.c_double), ("fric_a", C.c_double), ("fric_eps", C.c_double),
    ]


class SbStringInfo(C.Structure):
    _fields_ = [
        ("N_t", C.c_int32), ("N_l", C.c_int32), ("n_samples", C.c_int64), ("samples_done", C.c_int64),
        ("flags", C.c_int32), ("max_sweeps", C.c_int32), ("total_sweeps", C.c_int64),
        ("size_class", C.c_int32), ("lanes", C.c_int32), ("slots_t", C.c_int32), ("slots_l", C.c_int32),
    ]


_lib = None

# (name, restype, argtypes) of every entry point of include/stringfdtd.h
_P = C.c_void_p
SIGNATURES = [
    ("string_batch_create", C.c_int, [C.c_int, C.c_int, _P, C.POINTER(_P)]),
    ("string_batch_set_params", C.c_int, [_P, C.c_int, C.c_int, C.POINTER(SbStringParams)]),
    ("string_batch_excite", C.c_int, [_P, C.c_int, C.c_int, C.POINTER(SbExcitation)]),
    ("string_batch_step", C.c_int, [_P, C.c_int64]),
    ("string_batch_step_range", C.c_int, [_P, C.c_int, C.c_int, C.c_int64]),
    ("string_batch_rewind", C.c_int, [_P, C.c_int, C.c_int]),
    ("string_batch_snapshot_bytes", C.c_int, [_P, C.c_int, C.POINTER(C.c_int64)]),
    ("string_batch_snapshot", C.c_int, [_P, C.c_int, _P, C.c_int64, C.c_int]),
    ("string_batch_restore", C.c_int, [_P, C.c_int, _P, C.c_int64, C.c_int]),
    ("string_batch_read_output", C.c_int, [_P, C.c_int, C.c_int64, C.c_int64, _P, C.c_int]),
    ("string_batch_read_output_zeta", C.c_int, [_P, C.c_int, C.c_int64, C.c_int64, _P, C.c_int]),
    ("string_batch_output_ptr", C.c_int, [_P, C.c_int, C.POINTER(_P)]),
    ("string_batch_gather_output", C.c_int, [_P, C.c_int, C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.c_int64,
                                             _P, C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_int32)]),
    ("string_batch_gather_output_noalloc", C.c_int, [_P, C.c_int, C.POINTER(C.c_int32), C.POINTER(C.c_int64),
                                                     C.c_int64, _P, C.POINTER(C.c_int64), C.POINTER(C.c_int32)]),
    ("string_batch_graph_capture", C.c_int, [_P, C.c_int64, C.c_int]),
    ("string_batch_graph_launch", C.c_int, [_P]),
    ("string_batch_autotune", C.c_int, [_P, C.c_int64, C.POINTER(C.c_int32)]),
    ("string_batch_launch_times", C.c_int, [_P, C.POINTER(C.c_float), C.POINTER(C.c_int32)]),
    ("string_batch_restrike", C.c_int, [_P, C.c_int, C.c_int, C.c_void_p]),
    ("string_batch_restrike_list", C.c_int, [_P, C.c_int, C.POINTER(C.c_int32), C.c_void_p]),
    ("string_batch_set_blocks_per_cu", C.c_int, [_P, C.POINTER(C.c_int32)]),
    ("string_batch_read_energy", C.c_int, [_P, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    ("string_batch_info", C.c_int, [_P, C.c_int, C.POINTER(SbStringInfo)]),
    ("string_batch_set_monitor", C.c_int, [_P, C.c_int, C.c_double]),
    ("string_batch_set_solver", C.c_int, [_P, C.c_double, C.c_int]),
    ("string_plan_grid", C.c_int, [C.POINTER(SbStringParams), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    ("string_batch_destroy", C.c_int, [_P]),
    ("string_batch_last_error", C.c_char_p, [_P]),
]


class SbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (STATUS_NAMES.get(code, "?"), code, msg))
        self.code = code


def _foreign_hip_runtimes():
    """HIP runtime files mapped in this process that are not /opt/rocm's."""
    try:
        with open("/proc/self/maps") as fh:
            paths = {line.split()[-1] for line in fh if "libamdhip64" in line}
    except OSError:
        return []
    return sorted(p for p in paths if not os.path.realpath(p).startswith("/opt/rocm"))


def load():
    """Load the built library; raise if it has not been built.

    The library is compiled and linked for the ROCm release under /opt/rocm.
    A process that has already loaded another release's HIP runtime (PyTorch
    wheels bundle their own) would run the library on that runtime instead,
    so loading is refused there: use the library from a process that does not
    import torch.
    """
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libstringfdtd.so is not built (run __graft_entry__.build())")
        foreign = _foreign_hip_runtimes()
        if foreign:
            raise RuntimeError("a HIP runtime from another ROCm release is loaded in this process (%s); "
                               "libstringfdtd must run on /opt/rocm's runtime: do not import torch in "
                               "processes that use it" % ", ".join(foreign))
        lib = C.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def params_struct(p: dict) -> SbStringParams:
    s = SbStringParams()
    for f, _ in SbStringParams._fields_:
        if f in p:
            setattr(s, f, p[f])
    return s


def excitation_struct(e: dict) -> SbExcitation:
    s = SbExcitation()
    for f, _ in SbExcitation._fields_:
        if f in e:
            setattr(s, f, e[f])
    if e.get("type") == 3 and "x_end" not in e:
        s.x_end = s.x          # a bow that stays in place
    return s


def plan_grid(p: dict):
    """(N_t, N_l) planned by the library (host only)."""
    nt, nl = C.c_int32(), C.c_int32()
    st = load().string_plan_grid(C.byref(params_struct(p)), C.byref(nt), C.byref(nl))
    if st != SB_OK:
        raise SbError(st, "string_plan_grid")
    return nt.value, nl.value


def device_available() -> bool:
    """True if the library can create a batch on a HIP device."""
    lib = load()
    h = C.c_void_p()
    st = lib.string_batch_create(1, SB_FP64, None, C.byref(h))
    if st == SB_OK:
        lib.string_batch_destroy(h)
        return True
    return False


class StringBatch:
    """A batch handle of `capacity` string slots."""

    def __init__(self, capacity: int, precision: str = "fp32c", stream=None):
        self.lib = load()
        self.precision = PRECISIONS[precision]
        self.dtype = np.float32 if self.precision == SB_FP32C else np.float64
        h = C.c_void_p()
        st = self.lib.string_batch_create(capacity, self.precision, C.c_void_p(stream or 0), C.byref(h))
        if st != SB_OK:
            raise SbError(st, self.lib.string_batch_last_error(None).decode())
        self.h = h
        self.capacity = capacity
        self.n_samples = {}

    def _check(self, st, what):
        if st != SB_OK:
            raise SbError(st, "%s: %s" % (what, self.lib.string_batch_last_error(self.h).decode()))
        return st

    def set_params(self, first: int, params: list):
        arr = (SbStringParams * len(params))(*[params_struct(p) for p in params])
        self._check(self.lib.string_batch_set_params(self.h, first, len(params), arr), "set_params")
        for i, p in enumerate(params):
            self.n_samples[first + i] = int(p["n_samples"])

    def excite(self, first: int, excs: list):
        arr = (SbExcitation * len(excs))(*[excitation_struct(e) for e in excs])
        self._check(self.lib.string_batch_excite(self.h, first, len(excs), arr), "excite")

    def step(self, n_steps: int, first: int | None = None, count: int | None = None):
        if first is None:
            return self._check(self.lib.string_batch_step(self.h, n_steps), "step")
        return self._check(self.lib.string_batch_step_range(self.h, first, count, n_steps), "step_range")

    def rewind(self, first: int = 0, count: int | None = None):
        count = self.capacity - first if count is None else count
        self._check(self.lib.string_batch_rewind(self.h, first, count), "rewind")

    def snapshot_bytes(self, idx: int) -> int:
        n = C.c_int64()
        self._check(self.lib.string_batch_snapshot_bytes(self.h, idx, C.byref(n)), "snapshot_bytes")
        return n.value

    def snapshot(self, idx: int) -> np.ndarray:
        """Slot idx's stepping state as a byte array (host)."""
        buf = np.zeros(self.snapshot_bytes(idx), dtype=np.uint8)
        self._check(self.lib.string_batch_snapshot(self.h, idx, buf.ctypes.data_as(C.c_void_p), buf.nbytes, 0),
                    "snapshot")
        return buf

    def restore(self, idx: int, snap) -> None:
        """Puts back a snapshot of slot idx taken by snapshot()."""
        buf = np.ascontiguousarray(snap, dtype=np.uint8)
        self._check(self.lib.string_batch_restore(self.h, idx, buf.ctypes.data_as(C.c_void_p), buf.nbytes, 0),
                    "restore")

    def snapshot_device(self, idx: int, dst_ptr: int, nbytes: int) -> None:
        self._check(self.lib.string_batch_snapshot(self.h, idx, C.c_void_p(dst_ptr), nbytes, 1), "snapshot")

    def restore_device(self, idx: int, src_ptr: int, nbytes: int) -> None:
        self._check(self.lib.string_batch_restore(self.h, idx, C.c_void_p(src_ptr), nbytes, 1), "restore")

    def read_output(self, idx: int, offset: int = 0, count: int | None = None) -> np.ndarray:
        if count is None:
            count = self.n_samples[idx] - offset
        out = np.empty(count, dtype=self.dtype)
        self._check(self.lib.string_batch_read_output(self.h, idx, offset, count,
                                                      out.ctypes.data_as(C.c_void_p), 0), "read_output")
        return out

    def read_output_zeta(self, idx: int, offset: int = 0, count: int | None = None) -> np.ndarray:
        """The zeta channel of a slot set with readout_zeta = 1."""
        if count is None:
            count = self.n_samples[idx] - offset
        out = np.empty(count, dtype=self.dtype)
        self._check(self.lib.string_batch_read_output_zeta(self.h, idx, offset, count,
                                                           out.ctypes.data_as(C.c_void_p), 0), "read_output_zeta")
        return out

    def restrike(self, first: int, excs):
        """A new hammer or bow on sounding slots first.. (before their next step)."""
        arr = (SbExcitation * len(excs))(*[excitation_struct(e) for e in excs])
        self._check(self.lib.string_batch_restrike(self.h, first, len(excs), C.cast(arr, C.c_void_p)), "restrike")

    def restrike_list(self, slots, excs):
        """A new hammer or bow on each of the listed sounding slots."""
        sl = np.ascontiguousarray(slots, dtype=np.int32)
        arr = (SbExcitation * len(excs))(*[excitation_struct(e) for e in excs])
        self._check(self.lib.string_batch_restrike_list(self.h, len(sl), sl.ctypes.data_as(C.POINTER(C.c_int32)),
                                                        C.cast(arr, C.c_void_p)), "restrike_list")

    def graph_capture(self, steps_per_launch: int, n_launches: int):
        self._check(self.lib.string_batch_graph_capture(self.h, steps_per_launch, n_launches), "graph_capture")

    def graph_launch(self):
        self._check(self.lib.string_batch_graph_launch(self.h), "graph_launch")

    def launch_times(self):
        """(ms, strings) per launch of the last batched step (NUM_LAUNCHES each)."""
        ms, n = (C.c_float * NUM_LAUNCHES)(), (C.c_int32 * NUM_LAUNCHES)()
        self._check(self.lib.string_batch_launch_times(self.h, ms, n), "launch_times")
        return list(ms), list(n)

    def set_blocks_per_cu(self, blocks):
        arr = (C.c_int32 * NUM_LAUNCHES)(*blocks)
        self._check(self.lib.string_batch_set_blocks_per_cu(self.h, arr), "set_blocks_per_cu")

    def autotune(self, probe_steps: int = 480) -> list:
        chosen = (C.c_int32 * NUM_LAUNCHES)()
        self._check(self.lib.string_batch_autotune(self.h, probe_steps, chosen), "autotune")
        return list(chosen)

    def gather_output(self, slots, offsets, count: int, status: bool = False):
        """Rows of `count` samples: row i holds samples offsets[i].. of slots[i]
        (zero where the slot has not produced them).  With status=True returns
        (rows, samples_done, flags) and does not raise for flagged slots;
        otherwise a flagged slot raises SbError(SB_EUNSTABLE)."""
        sl = np.ascontiguousarray(slots, dtype=np.int32)
        of = np.ascontiguousarray(offsets, dtype=np.int64)
        out = np.empty((len(sl), count), dtype=self.dtype)
        done = np.zeros(len(sl), dtype=np.int64)
        flags = np.zeros(len(sl), dtype=np.int32)
        st = self.lib.string_batch_gather_output(
            self.h, len(sl), sl.ctypes.data_as(C.POINTER(C.c_int32)), of.ctypes.data_as(C.POINTER(C.c_int64)),
            count, out.ctypes.data_as(C.c_void_p), 0, done.ctypes.data_as(C.POINTER(C.c_int64)),
            flags.ctypes.data_as(C.POINTER(C.c_int32)))
        if status and st == SB_EUNSTABLE:
            return out, done, flags
        self._check(st, "gather_output")
        return (out, done, flags) if status else out

    def read_output_device(self, idx: int, dst_ptr: int, offset: int, count: int):
        self._check(self.lib.string_batch_read_output(self.h, idx, offset, count, C.c_void_p(dst_ptr), 1),
                    "read_output")

    def output_ptr(self, idx: int) -> int:
        p = C.c_void_p()
        self._check(self.lib.string_batch_output_ptr(self.h, idx, C.byref(p)), "output_ptr")
        return p.value

    def info(self, idx: int) -> dict:
        inf = SbStringInfo()
        self._check(self.lib.string_batch_info(self.h, idx, C.byref(inf)), "info")
        return {f: getattr(inf, f) for f, _ in SbStringInfo._fields_}

    def read_energy(self, idx: int):
        H, n = C.c_double(), C.c_int64()
        self._check(self.lib.string_batch_read_energy(self.h, idx, C.byref(H), C.byref(n)), "read_energy")
        return H.value, n.value

    def set_monitor(self, period: int, growth_tol: float):
        self._check(self.lib.string_batch_set_monitor(self.h, period, growth_tol), "set_monitor")

    def set_solver(self, tol: float, max_sweeps: int):
        self._check(self.lib.string_batch_set_solver(self.h, tol, max_sweeps), "set_solver")

    def close(self):
        if getattr(self, "h", None):
            self.lib.string_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
