"""The LDS-poisoning debug build (libstringfdtd_poison.so, compiled with
SFD_POISON_LDS=1) as a race and stale-read detector: its step kernel fills
every group's LDS with NaN at the start of each task and the per-step arrays
at the end of each step, so a read of LDS that the task or step has not
written (a missing barrier, a wrong index into another group's region, an
array assumed to persist) turns the output NaN or trips the energy monitor.
The mixed batch of tests/lds_poison_run.py runs through it in a process of
its own and must finish unflagged, finite, and equal to the regular build's
output (rel-L2 <= 1e-12 in FP64, <= 1e-5 in FP32 compensated; the bowed
strings, chaotic in FP32, are held to finite and unflagged there)."""
from __future__ import annotations

import os
import subprocess
import sys

import numpy as np
import pytest

from paper_2311_18505_amd import binding
from tests import lds_poison_run as R

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
POISON_LIB = os.path.join(ROOT, "paper_2311_18505_amd", "libstringfdtd_poison.so")


def rel_l2(y, ref):
    ref = np.asarray(ref, np.float64)
    return float(np.linalg.norm(np.asarray(y, np.float64) - ref) / max(np.linalg.norm(ref), 1e-300))


def test_poisoned_lds_build_matches_regular_build(tmp_path):
    if not binding.device_available():
        pytest.skip("no GPU")
    assert os.path.exists(POISON_LIB), "libstringfdtd_poison.so is not built (run __graft_entry__.build())"
    out = str(tmp_path / "poison.npz")
    print("[gpu] poisoned build in a child process", flush=True)
    res = subprocess.run([sys.executable, "-u", "-m", "tests.lds_poison_run", out], cwd=ROOT,
                         env=dict(os.environ, STRINGFDTD_LIB=POISON_LIB), capture_output=True, text=True,
                         timeout=240)
    print(res.stdout[-2000:], flush=True)
    assert res.returncode == 0, res.stderr[-4000:]
    got = np.load(out)
    its = R.items()
    bow = [e.get("type") == 3 for _, e in its]   # SB_EXC_BOW
    for precision, tol in (("fp64", 1e-12), ("fp32c", 1e-5)):
        print("[gpu] regular build, %s" % precision, flush=True)
        outs, infos = R.run(precision)
        classes = {inf["size_class"] for inf in infos}
        assert classes == set(range(8)), classes
        assert np.array_equal(got[precision + "_class"], [inf["size_class"] for inf in infos])
        assert all(inf["flags"] == 0 for inf in infos)
        assert np.all(got[precision + "_flags"] == 0), got[precision + "_flags"]
        worst = 0.0
        for i, y in enumerate(outs):
            yp = got["%s_%d" % (precision, i)]
            assert np.all(np.isfinite(yp)), "slot %d reads NaN through the poisoned build" % i
            if bow[i] and precision == "fp32c":
                continue
            worst = max(worst, rel_l2(yp, y))
        print("[gpu] %s: poisoned vs regular build, worst rel-L2 %.3e" % (precision, worst), flush=True)
        assert worst <= tol
