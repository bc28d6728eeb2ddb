"""Builds libstringfdtd.so (HIP for gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libstringfdtd.so")
# the stepping kernels' instantiation families compile as translation units of
# their own, in parallel
SOURCES = ["capi.cpp", "planner.cpp", "step_launch.hip", "step_f32_plain.hip", "step_f32_bow.hip",
           "step_f32_cubic.hip", "step_f64_plain.hip", "step_f64_bow.hip", "step_f64_cubic.hip",
           "plain_kernel.hip", "static_scratch.hip"]
# the slowest first, so that the pool ends together
_HEAVY = ("step_f32_plain.hip", "step_f32_bow.hip", "step_f32_cubic.hip", "step_f64_bow.hip", "step_f64_cubic.hip",
          "step_f64_plain.hip")


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.sep not in c or os.path.exists(c)):
            return c
    raise RuntimeError("hipcc not found")


# the library, and its debug twin whose step kernel poisons dead LDS with NaN
VARIANTS = {"": [], "_poison": ["-DSFD_POISON_LDS=1"]}

FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         # packed FP32 arithmetic stays off on the test machines
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # host-side planning reproduces FP64 grid sizes bit for bit
         "-Xarch_host", "-ffp-contract=off"]


def _compile_command(variant: str, src: str, obj: str) -> list:
    return [hipcc()] + FLAGS + ["-I", os.path.join(os.path.dirname(HERE), "include")] + VARIANTS[variant] + \
        ["-c", "-o", obj, os.path.join(CSRC, src)]


def _link_command(objs: list, out: str) -> list:
    return [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", out] + objs


def lib_path(variant: str = "") -> str:
    return os.path.join(HERE, "libstringfdtd%s.so" % variant)


def _run(cmd: list, verbose: bool):
    if verbose:
        print(" ".join(cmd), flush=True)
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    return p.returncode, p.stdout


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile every source for gfx950 into libstringfdtd.so and its LDS-poisoning
    debug twin libstringfdtd_poison.so (always rebuilds; the translation units
    compile in parallel)."""
    jobs = jobs or max(1, min(16, os.cpu_count() or 1))
    tmp = tempfile.mkdtemp(prefix="sfd_build_")
    try:
        order = sorted(SOURCES, key=lambda s: _HEAVY.index(s) if s in _HEAVY else len(_HEAVY))
        tasks = []
        for variant in VARIANTS:
            for src in order:
                obj = os.path.join(tmp, "%s%s.o" % (os.path.splitext(src)[0], variant))
                tasks.append((variant, src, obj))
        tasks.sort(key=lambda t: order.index(t[1]))
        with ThreadPoolExecutor(max_workers=jobs) as pool:
            results = list(pool.map(lambda t: _run(_compile_command(*t), verbose), tasks))
        failed = [t[1] + t[0] for t, (rc, _) in zip(tasks, results) if rc != 0]
        for t, (rc, log) in zip(tasks, results):
            if rc != 0:
                sys.stderr.write(log)
        if failed:
            raise RuntimeError("hipcc failed compiling %s" % ", ".join(failed))
        for variant in VARIANTS:
            out = lib_path(variant)
            part = out + ".tmp%d" % os.getpid()
            objs = [t[2] for t in tasks if t[0] == variant]
            rc, log = _run(_link_command(objs, part), verbose)
            if rc != 0:
                sys.stderr.write(log)
                raise RuntimeError("hipcc failed linking %s" % os.path.basename(out))
            os.replace(part, out)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
