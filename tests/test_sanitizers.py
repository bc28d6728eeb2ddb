"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

* The FP64 oracle: every entry point of oracle.h, on short strings that reach
  its branches (tests/sanitize/oracle_driver.c), built with
  -fsanitize=address,undefined and -fno-sanitize-recover=all; it must finish
  with no report, and its results must equal those of the uninstrumented
  liboracle on the same cases.
* The library's host planner (grid sizing, the layouts of FP32 batches,
  coefficient and excitation tables, the plain path's tables;
  tests/sanitize/planner_driver.cpp) over a seeded sweep of valid and
  invalid parameters, built the same way with hipcc (host code only: each
  -fsanitize goes to the host compiler).

The kernels and the HIP runtime calls are outside these builds (no GPU
sanitizer on the test machines); the GPU tests' bitwise determinism checks
(chunked = one shot, mix = alone, snapshot resume) stand in for them.
"""
from __future__ import annotations

import os
import re
import shutil
import subprocess

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _clean(res):
    assert res.returncode == 0, res.stdout[-2000:] + res.stderr[-4000:]
    for marker in ("runtime error", "AddressSanitizer", "LeakSanitizer"):
        assert marker not in res.stderr, res.stderr[-4000:]


def _string(f0, B, alpha, **kw):
    p = dict(fs=48000.0, f0=f0, B=B, alpha=alpha, sigma0_t=1.0, sigma1_t=3e-4, sigma0_l=1.0, sigma1_l=3e-4,
             x_out=0.3, n_samples=400)
    p.update(kw)
    return p


def _hammer(x, v, order):
    return dict(type=2, interp_order=order, x=x, v_H=v, M_H=4.9e-3, K_H=4.5e9, alpha_H=2.5, rhoA=6.3e-3)


def _bow(x, x_end, order):
    return dict(type=3, interp_order=order, x=x, x_end=x_end, v_B=0.1, F_B=100.0, attack=0.002, fric_a=100.0,
                fric_eps=0.2)


# the driver's cases, as the uninstrumented oracle runs them
CASES = {
    "pluck": (_string(110.0, 1e-4, 1.5), dict(type=1, x=0.27, c0=1e-3), None),
    "hammer_linear": (_string(220.0, 3e-4, 2.5), _hammer(0.12, 2.0, 1), None),
    "hammer_cubic_end": (_string(220.0, 3e-4, 2.5), _hammer(0.02, 2.0, 3), None),
    "bow_cubic": (_string(196.0, 1e-4, 1.0), _bow(0.12, 0.2, 3), None),
    "bow_linear_nonlinear": (_string(196.0, 1e-4, 2.0), _bow(0.015, 0.05, 1), None),
    "clamped_hammer": (_string(80.0, 2e-4, 2.0, boundary=1), _hammer(0.11, 3.0, 3), None),
    "cubic_grid": (_string(300.0, 1e-3, 3.0, grid_interp=3), dict(type=1, x=0.14, c0=0.02), None),
    "vibrato": (_string(150.0, 1e-4, 1.7, mod_type=1, mod_depth_cents=25.0, mod_rate_hz=6.0),
                dict(type=1, x=0.3, c0=1e-3), None),
    "glide": (_string(150.0, 1e-4, 1.7, mod_type=2, mod_depth_cents=25.0, mod_rate_hz=6.0, glide_semitones=-2.0),
              dict(type=1, x=0.3, c0=1e-3), None),
    "restrike": (_string(130.0, 1e-4, 1.6), _hammer(0.13, 1.5, 1),
                 [(120, _hammer(0.2, 1.0, 3)), (260, _bow(0.1, 0.15, 1))]),
}


def test_oracle_under_asan_ubsan(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_asan")
    cmd = ["gcc", "-O1", "-g", "-std=c99", "-D_GNU_SOURCE", "-ffp-contract=off", "-fno-fast-math",
           "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "oracle"), os.path.join(HERE, "sanitize", "oracle_driver.c"),
           os.path.join(ROOT, "oracle", "oracle.c"), "-lm", "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    res = subprocess.run([exe], capture_output=True, text=True, env=SAN_ENV, timeout=600)
    _clean(res)
    rows = {ln.split()[0]: ln.split()[1:] for ln in res.stdout.splitlines() if ln.strip()}
    assert set(CASES) < set(rows)
    for name, (p, e, sched) in CASES.items():
        st, steps, sy, se = int(rows[name][0]), int(rows[name][1]), float(rows[name][2]), float(rows[name][3])
        ref = oracle.run(p, e, want=("y_u", "energy"), schedule=sched)
        assert st == 0 and steps == p["n_samples"] - 2, name
        ry, re_ = float(np.sum(ref["y_u"])), float(np.sum(ref["energy"][:-1]))
        assert abs(sy - ry) <= 1e-12 * max(1.0, abs(ry)), (name, sy, ry)
        assert abs(se - re_) <= 1e-12 * max(1.0, abs(re_)), (name, se, re_)
    for name in ("invalid_alpha", "invalid_f0", "invalid_position"):
        assert int(rows[name][0]) == -1, name
    assert int(rows["dump_system"][0]) == 0 and int(rows["apply_I_lt"][0]) == 0
    # the slip root of the scalar bow problem satisfies its equation
    phi, v = float(rows["bow_solve"][2]), float(rows["bow_solve"][3])
    assert abs(v - (-0.3 - 0.05 * phi)) <= 1e-12


def test_planner_under_asan_ubsan(tmp_path):
    hipcc = "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "planner_asan")
    csrc = os.path.join(ROOT, "paper_2311_18505_amd", "csrc")
    cmd = [hipcc, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-ffp-contract=off",
           "-I", csrc, "-I", os.path.join(ROOT, "include"),
           os.path.join(HERE, "sanitize", "planner_driver.cpp"), os.path.join(csrc, "planner.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    res = subprocess.run([exe, "600"], capture_output=True, text=True, env=SAN_ENV, timeout=600)
    _clean(res)
    m = re.search(r"strings (\d+) ok (\d+) refused (\d+) budget (\d+) excitations ok (\d+) refused (\d+) "
                  r"plain ok (\d+) refused (\d+) narrow layouts (\d+)", res.stdout)
    assert m, res.stdout
    n, ok, refused, budget, exc_ok, exc_refused, plain_ok, plain_refused, narrow = (int(x) for x in m.groups())
    # (the driver checks every planned layout: each grid covered, the fewest
    # slots per lane among the class's width levels)
    assert narrow > 50
    # the sweep reaches valid and invalid strings, excitations and plain-path plans
    assert n == 600 and ok > 200 and refused > 200 and budget >= 1
    assert exc_ok > 300 and exc_refused > 10 and plain_ok > 100 and plain_refused > 10
