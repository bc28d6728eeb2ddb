"""Full-size parity: the uneven batch of 16384 nonlinear strings (durations
U(0.5, 4) s, vibrato or glide, FP32 compensated) stepped as the benchmark
times it -- one step of the whole batch in its three concurrent launches,
blocks per CU from the autotuner -- and checked on sampled strings against
the FP64 oracle (rel-L2 <= 1e-3).  The sample takes, in every size class,
the longest string and two seeded others, plus six seeded strings of the
whole batch; all strings must finish unflagged."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2311_18505_amd import binding, workloads as W

pytestmark = pytest.mark.gpu


def _gpu():
    if not binding.device_available():
        pytest.skip("no GPU")
    print("[gpu] device ready", flush=True)


def rel_l2(y, ref):
    return float(np.linalg.norm(np.asarray(y, np.float64) - ref) / np.linalg.norm(ref))


def _sample(items, classes, rng):
    pick = []
    for c in sorted(set(classes)):
        members = [i for i, k in enumerate(classes) if k == c]
        longest = max(members, key=lambda i: items[i][0]["n_samples"])
        others = [i for i in members if i != longest]
        pick += [longest] + [int(i) for i in rng.choice(others, min(2, len(others)), replace=False)]
    rest = [i for i in range(len(items)) if i not in set(pick)]
    pick += [int(i) for i in rng.choice(rest, 6, replace=False)]
    return pick


def test_uneven16384_sampled_strings_fp32c():
    _gpu()
    items = W.uneven_batch_16384()
    n_max = max(p["n_samples"] for p, _ in items)
    b = binding.StringBatch(len(items), "fp32c")
    try:
        b.set_params(0, [p for p, _ in items])
        b.excite(0, [e for _, e in items])
        classes = [b.info(i)["size_class"] for i in range(len(items))]
        tuned = b.autotune(480)
        print("[gpu] %d strings, blocks/CU %s; stepping %d samples" % (len(items), tuned, n_max), flush=True)
        b.rewind()
        b.step(n_max)
        pick = _sample(items, classes, np.random.default_rng(W.SEED + 5))
        outs = [b.read_output(i) for i in pick]
        infos = [b.info(i) for i in range(len(items))]
        print("[gpu] step done; %d sampled strings read" % len(pick), flush=True)
    finally:
        b.close()
    assert all(inf["flags"] == 0 and inf["samples_done"] == inf["n_samples"] for inf in infos)
    print("[cpu] oracle on %d strings, up to %d samples" % (len(pick), max(items[i][0]["n_samples"] for i in pick)),
          flush=True)
    refs = oracle.run_many([items[i] for i in pick], threads=16)
    errs = [rel_l2(y, r["y_u"]) for y, r in zip(outs, refs)]
    for i, err in zip(pick, errs):
        print("[gpu] string %d class %d, %d samples: rel-L2 %.3e" % (i, classes[i], items[i][0]["n_samples"], err),
              flush=True)
    assert set(classes[i] for i in pick) == set(classes)
    assert max(errs) <= 1e-3
