"""One mixed batch stepped through the library build that STRINGFDTD_LIB
names (the LDS-poisoning debug build in test_gpu_lds_poison.py, which runs
this module in a process of its own and the regular build in its own
process): every size class, plucks and hammers (linear and cubic), f0
modulation, bowed and clamped strings, the zeta channel, the cubic grid
interpolant, with the energy monitor checking every 48 steps."""
from __future__ import annotations

import sys

import numpy as np

from paper_2311_18505_amd import binding, workloads as W

SECONDS = 0.03


def items():
    n = int(SECONDS * 48000)
    its = list(W.random_batch(40, seconds=SECONDS, modulation=True, seed=W.SEED + 93))
    p, e = W.single_bowed(seconds=SECONDS)
    its.append((p, e))
    its.append((p, dict(W.bow(0.015, 0.1, 100.0, x_end=0.05), interp_order=3)))
    q, f = its[3]
    its.append((dict(q, boundary=1, readout_zeta=1, alpha=max(q["alpha"], 1.5)), f))
    its.append((dict(its[5][0], grid_interp=3, alpha=max(its[5][0]["alpha"], 1.5)), its[5][1]))
    its.append((W.string(180.0, 3e-4, 2.5, 1.0, 2e-4, n), dict(W.hammer(0.03, 2.0), interp_order=3)))
    its.append((W.string(40.0, 1e-5, 1.1, 0.5, 1e-4, n), W.hammer(0.12, 2.0)))          # class 6
    its.append((W.string(20.0, 1e-6, 1.1713, 0.5, 1e-4, n), W.hammer(0.12, 2.0)))       # class 7
    its.append((dict(W.string(20.7, 1e-5, 3.0, 1.0, 1e-4, n), boundary=1), W.pluck(0.2, 1e-3)))
    return its


def run(precision):
    its = items()
    b = binding.StringBatch(len(its), precision)
    try:
        b.set_params(0, [p for p, _ in its])
        b.excite(0, [e for _, e in its])
        b.set_monitor(48, 1e-4 if precision == "fp32c" else 1e-9)
        b.step(max(p["n_samples"] for p, _ in its))
        outs = [b.read_output(i) for i in range(len(its))]
        infos = [b.info(i) for i in range(len(its))]
    finally:
        b.close()
    return outs, infos


def main(path):
    res = {}
    for precision in ("fp64", "fp32c"):
        print("[poison] %s: %d strings through %s" % (precision, len(items()), binding.LIB_PATH), flush=True)
        outs, infos = run(precision)
        for i, y in enumerate(outs):
            res["%s_%d" % (precision, i)] = y
        res[precision + "_flags"] = np.array([inf["flags"] for inf in infos])
        res[precision + "_class"] = np.array([inf["size_class"] for inf in infos])
    np.savez(path, **res)
    print("[poison] done", flush=True)


if __name__ == "__main__":
    main(sys.argv[1])
