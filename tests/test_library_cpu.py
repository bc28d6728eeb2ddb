"""CPU tests of the C-ABI library: it loads, exports every declared entry
point, plans the same grids as the oracle, and validates arguments.  No
compute call runs without a GPU."""
from __future__ import annotations

import ctypes as C
import os
import re

import pytest

import oracle
from paper_2311_18505_amd import binding, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    inc = os.path.join(ROOT, "include")
    for f in sorted(os.listdir(inc)):
        if f.endswith(".h"):
            txt = open(os.path.join(inc, f)).read()
            names += re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(string_\w+)\s*\(", txt, re.M)
    return names


def test_library_exports_every_declared_symbol():
    lib = binding.load()
    names = _declared()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    # the binding wraps exactly the declared entry points
    assert sorted(n for n, _, _ in binding.SIGNATURES) == sorted(names)


def _grid_cases():
    cases = [W.single_linear(), W.single_nonlinear(), W.single_linear(theta=1.0)]
    cases += W.random_batch(200)
    cases += W.random_batch(100, durations=("uniform", 0.5, 4.0), modulation=True, seed=7)
    cases += [(dict(p, boundary=1), e) for p, e in W.random_batch(100, modulation=True, seed=9)]
    cases += [(dict(p, boundary=1), e) for p, e in (W.single_linear(), W.single_nonlinear())]
    return cases


def test_planned_grids_match_oracle():
    for p, _ in _grid_cases():
        g = oracle.grid(p)
        assert binding.plan_grid(p) == (g["N_t"], g["N_l"]), p


@pytest.mark.parametrize("bad", [
    dict(f0=-1.0), dict(f0=float("nan")), dict(alpha=0.5), dict(theta=0.4), dict(B=-1e-4),
    dict(x_out=1.0), dict(n_samples=1), dict(sigma0_t=-1.0), dict(fs=0.0), dict(mod_type=3),
    dict(boundary=2), dict(boundary=-1), dict(readout_zeta=2), dict(grid_interp=2), dict(grid_interp=3, grid_l=3),
])
def test_plan_grid_rejects_invalid(bad):
    p, _ = W.single_nonlinear()
    p = dict(p, **bad)
    with pytest.raises(binding.SbError) as ex:
        binding.plan_grid(p)
    assert ex.value.code == binding.SB_EINVAL


def test_create_without_gpu_fails_cleanly():
    lib = binding.load()
    if binding.device_available():
        pytest.skip("a GPU is present")
    h = C.c_void_p()
    st = lib.string_batch_create(4, binding.SB_FP32C, None, C.byref(h))
    assert st in (binding.SB_EDEVICE, binding.SB_ENOMEM)
    assert lib.string_batch_last_error(None)
    # invalid arguments are rejected before any device call
    assert lib.string_batch_create(0, binding.SB_FP32C, None, C.byref(h)) == binding.SB_EINVAL
    assert lib.string_batch_create(4, 7, None, C.byref(h)) == binding.SB_EINVAL
