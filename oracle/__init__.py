"""FP64 CPU oracle for the string scheme of arXiv 2311.18505 (test infrastructure).

Only the tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It wraps ``oracle.c``, a literal
implementation of the matrix recursion of eq. (7)-(9) with the excitations of
Sec. 3.3, compiled with FMA contraction disabled.  It shares nothing with the
GPU library.

Parameter dictionaries use the same keys as the GPU binding (they come from
the seeded workload generator); this module maps them onto its own C structs.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


class OrcString(C.Structure):
    _fields_ = [
        ("fs", C.c_double), ("f0", C.c_double), ("B", C.c_double), ("alpha", C.c_double),
        ("theta", C.c_double), ("sigma0_t", C.c_double), ("sigma1_t", C.c_double),
        ("sigma0_l", C.c_double), ("sigma1_l", C.c_double), ("x_out", C.c_double),
        ("n_samples", C.c_int64), ("mod_type", C.c_int32), ("grid_t", C.c_int32),
        ("mod_depth_cents", C.c_double), ("mod_rate_hz", C.c_double),
        ("glide_semitones", C.c_double), ("grid_l", C.c_int32), ("boundary", C.c_int32),
        ("grid_interp", C.c_int32),
    ]


class OrcExcitation(C.Structure):
    _fields_ = [
        ("type", C.c_int32), ("interp_order", C.c_int32), ("x", C.c_double), ("c0", C.c_double),
        ("v_H", C.c_double), ("M_H", C.c_double), ("K_H", C.c_double),
        ("alpha_H", C.c_double), ("rhoA", C.c_double),
        ("x_end", C.c_double), ("v_B", C.c_double), ("F_B", C.c_double), ("attack", C.c_double),
        ("fric_a", C.c_double), ("fric_eps", C.c_double),
    ]


class OrcGrid(C.Structure):
    _fields_ = [
        ("N_t", C.c_int32), ("N_l", C.c_int32), ("h_t", C.c_double), ("h_l", C.c_double),
        ("k", C.c_double), ("gamma0", C.c_double), ("gamma_max", C.c_double),
        ("kappa", C.c_double), ("theta", C.c_double),
    ]


_DP = C.POINTER(C.c_double)


class OrcOutputs(C.Structure):
    _fields_ = [
        ("y_u", _DP), ("y_z", _DP), ("energy", _DP), ("traj_u", _DP), ("traj_z", _DP),
        ("u_H", _DP), ("flops", C.c_double), ("steps_done", C.c_int64),
        ("bow_phi", _DP), ("bow_vrel", _DP), ("flops_nofill", C.c_double),
    ]


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so (plain gcc, FP64, no FMA contraction)."""
    with _lock:
        if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            tmp = _LIB_PATH + ".tmp%d" % os.getpid()
            subprocess.check_call([
                "gcc", "-O2", "-std=c99", "-D_GNU_SOURCE", "-ffp-contract=off", "-fno-fast-math",
                "-fPIC", "-shared", "-o", tmp, _SRC, "-lm",
            ])
            os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        build()
        lib = C.CDLL(_LIB_PATH)
        lib.orc_grid_plan.argtypes = [C.POINTER(OrcString), C.POINTER(OrcGrid)]
        lib.orc_grid_plan.restype = C.c_int
        lib.orc_run.argtypes = [C.POINTER(OrcString), C.POINTER(OrcExcitation), C.POINTER(OrcOutputs)]
        lib.orc_run.restype = C.c_int
        lib.orc_run_schedule.argtypes = [C.POINTER(OrcString), C.POINTER(OrcExcitation), C.c_int,
                                         C.POINTER(C.c_int64), C.POINTER(OrcExcitation), C.POINTER(OrcOutputs)]
        lib.orc_run_schedule.restype = C.c_int
        lib.orc_dump_system.argtypes = [C.POINTER(OrcString), C.POINTER(OrcExcitation), C.c_int64,
                                        _DP, _DP, C.c_double, C.c_double, _DP, _DP, _DP, _DP]
        lib.orc_dump_system.restype = C.c_int
        lib.orc_gamma_at.argtypes = [C.POINTER(OrcString), C.c_int64]
        lib.orc_gamma_at.restype = C.c_double
        lib.orc_apply_I_lt.argtypes = [C.c_int, C.c_int, C.c_int, _DP, _DP]
        lib.orc_apply_I_lt.restype = C.c_int
        lib.orc_bow_solve.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, _DP]
        lib.orc_bow_solve.restype = C.c_double
        _lib = lib
    return _lib


STRING_KEYS = ("fs", "f0", "B", "alpha", "theta", "sigma0_t", "sigma1_t", "sigma0_l", "sigma1_l",
               "x_out", "n_samples", "mod_type", "mod_depth_cents", "mod_rate_hz",
               "glide_semitones", "grid_t", "grid_l", "boundary", "grid_interp")
EXC_KEYS = ("type", "interp_order", "x", "c0", "v_H", "M_H", "K_H", "alpha_H", "rhoA", "x_end", "v_B", "F_B", "attack",
            "fric_a", "fric_eps")


def _string(p: dict) -> OrcString:
    s = OrcString()
    for key in STRING_KEYS:
        if key in p:
            setattr(s, key, p[key])
    return s


def _exc(e: dict | None) -> OrcExcitation:
    x = OrcExcitation()
    if e:
        for key in EXC_KEYS:
            if key in e:
                setattr(x, key, e[key])
    return x


class OracleError(RuntimeError):
    pass


def grid(p: dict) -> dict:
    g = OrcGrid()
    st = _load().orc_grid_plan(C.byref(_string(p)), C.byref(g))
    if st != 0:
        raise OracleError("orc_grid_plan failed with status %d" % st)
    return {f: getattr(g, f) for f, _ in OrcGrid._fields_}


def gamma_at(p: dict, n: int) -> float:
    return _load().orc_gamma_at(C.byref(_string(p)), n)


def bow_solve(b: float, c: float, a: float, eps: float) -> tuple:
    """(phi, v_rel) of the bow's scalar problem of one step (eq. 5)."""
    v = C.c_double()
    phi = _load().orc_bow_solve(b, c, a, eps, C.byref(v))
    return phi, v.value


def _ptr(a):
    return a.ctypes.data_as(_DP) if a is not None else None


def run(p: dict, e: dict | None, want=("y_u",), allow_fail: bool = False, schedule=None) -> dict:
    """Run one string for p['n_samples'] samples; return the requested arrays.

    want: any of "y_u", "y_z", "energy", "traj_u", "traj_z", "u_H", "bow_phi", "bow_vrel".
    schedule: optional [(step, excitation)] of hammers or bows applied to the
    sounding string before the step that computes w^{step+1}.
    """
    lib = _load()
    g = grid(p)
    ns = int(p["n_samples"])
    nt, nl = g["N_t"] - 1, max(g["N_l"] - 1, 0)
    res: dict = {"grid": g}
    arrs = {}
    for key in ("y_u", "y_z", "energy", "u_H", "bow_phi", "bow_vrel"):
        arrs[key] = np.zeros(ns) if key in want else None
    arrs["traj_u"] = np.zeros((ns, nt)) if "traj_u" in want else None
    arrs["traj_z"] = np.zeros((ns, max(nl, 0))) if "traj_z" in want else None
    out = OrcOutputs()
    for key in ("y_u", "y_z", "energy", "traj_u", "traj_z", "u_H", "bow_phi", "bow_vrel"):
        setattr(out, key, _ptr(arrs[key]))
    if schedule:
        steps = (C.c_int64 * len(schedule))(*[int(n) for n, _ in schedule])
        excs = (OrcExcitation * len(schedule))(*[_exc(x) for _, x in schedule])
        st = lib.orc_run_schedule(C.byref(_string(p)), C.byref(_exc(e)), len(schedule), steps, excs, C.byref(out))
    else:
        st = lib.orc_run(C.byref(_string(p)), C.byref(_exc(e)), C.byref(out))
    if st != 0 and not allow_fail:
        raise OracleError("orc_run failed with status %d" % st)
    for key in want:
        res[key] = arrs[key]
    res["status"] = st
    res["flops"] = out.flops
    res["flops_nofill"] = out.flops_nofill
    res["steps_done"] = out.steps_done
    return res


def apply_I_lt(Nt: int, Nl: int, order: int, p) -> np.ndarray:
    """I_(l)->(t) p of the scheme (order 1 or 3) on grids of Nt and Nl intervals."""
    p = np.ascontiguousarray(p, dtype=np.float64)
    out = np.zeros(Nt)
    st = _load().orc_apply_I_lt(Nt, Nl, order, _ptr(p), _ptr(out))
    if st != 0:
        raise OracleError("orc_apply_I_lt failed with status %d" % st)
    return out


def run_many(items, want=("y_u",), threads: int | None = None) -> list:
    """Run several (params, excitation) pairs, one string per host thread."""
    threads = threads or min(len(items), os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=max(threads, 1)) as ex:
        return list(ex.map(lambda pe: run(pe[0], pe[1], want), items))


def dump_system(p: dict, e: dict | None, n: int, w_n, w_nm1, uH_n=0.0, uH_nm1=0.0) -> dict:
    """Dense A (joint, with the hammer unknown if any), B, C and right-hand side at step n."""
    lib = _load()
    g = grid(p)
    nt, nl = g["N_t"] - 1, max(g["N_l"] - 1, 0)
    n_ = nt + nl
    na = n_ + (1 if e and e.get("type") == 2 else 0)
    A = np.zeros((na, na)); Bm = np.zeros((n_, n_)); Cm = np.zeros((n_, n_)); r = np.zeros(na)
    w_n = np.ascontiguousarray(w_n, dtype=np.float64)
    w_nm1 = np.ascontiguousarray(w_nm1, dtype=np.float64)
    st = lib.orc_dump_system(C.byref(_string(p)), C.byref(_exc(e)), n, _ptr(w_n), _ptr(w_nm1),
                             uH_n, uH_nm1, _ptr(A), _ptr(Bm), _ptr(Cm), _ptr(r))
    if st != 0:
        raise OracleError("orc_dump_system failed with status %d" % st)
    return {"A": A, "B": Bm, "C": Cm, "rhs": r, "grid": g}
