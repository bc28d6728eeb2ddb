"""Builds libstringfdtd.so (HIP for gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libstringfdtd.so")
SOURCES = ["capi.cpp", "planner.cpp", "step_kernel.hip", "plain_kernel.hip", "static_scratch.hip"]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.sep not in c or os.path.exists(c)):
            return c
    raise RuntimeError("hipcc not found")


# the library, and its debug twin whose step kernel poisons dead LDS with NaN
VARIANTS = {"": [], "_poison": ["-DSFD_POISON_LDS=1"]}


def _command(variant: str, out: str) -> list:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    return [hipcc(), "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
            # packed FP32 arithmetic stays off on the test machines
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            # host-side planning reproduces FP64 grid sizes bit for bit
            "-Xarch_host", "-ffp-contract=off",
            "-I", os.path.join(os.path.dirname(HERE), "include")] + VARIANTS[variant] + ["-o", out] + srcs


def lib_path(variant: str = "") -> str:
    return os.path.join(HERE, "libstringfdtd%s.so" % variant)


def build(verbose: bool = False) -> str:
    """Compile every source for gfx950 into libstringfdtd.so and its LDS-poisoning
    debug twin libstringfdtd_poison.so, side by side (always rebuilds)."""
    procs = []
    for variant in VARIANTS:
        out = lib_path(variant)
        tmp = out + ".tmp%d" % os.getpid()
        cmd = _command(variant, tmp)
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((out, tmp, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
    failed = []
    for out, tmp, proc in procs:
        log, _ = proc.communicate()
        if proc.returncode != 0:
            sys.stderr.write(log)
            failed.append(os.path.basename(out))
        else:
            os.replace(tmp, out)
    if failed:
        raise RuntimeError("hipcc failed building %s" % ", ".join(failed))
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
