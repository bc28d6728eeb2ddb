"""GPU batch scheduling: captured launches and the autotuner.

A captured graph of chunked launches must reproduce eager stepping exactly,
on every replay (with eager work and synchronisations between replays), and
the autotuner's choice must leave results unchanged and the batch rewound.
"""
from __future__ import annotations

import numpy as np
import pytest

from paper_2311_18505_amd import binding, hiptime, workloads as W

pytestmark = pytest.mark.gpu


def _gpu():
    if not binding.device_available():
        pytest.skip("no GPU")
    print("[gpu] device ready", flush=True)


def _batch(items, precision="fp32c"):
    b = binding.StringBatch(len(items), precision)
    b.set_params(0, [p for p, _ in items])
    b.excite(0, [e for _, e in items])
    return b


def test_graph_replays_match_eager():
    _gpu()
    items = W.random_batch(40, seconds=0.1, modulation=True)
    n = max(p["n_samples"] for p, _ in items)
    eager = _batch(items)
    for _ in range(0, n, 480):
        eager.step(480)
    ref = [eager.read_output(i) for i in range(len(items))]
    eager.close()
    print("[gpu] eager reference done", flush=True)

    g = _batch(items)
    g.graph_capture(480, 5)              # 2400 steps per replay
    for rep in range(3):
        g.rewind()
        for _ in range(0, n, 2400):
            g.graph_launch()
            hiptime.synchronize()
            _ = g.info(0)                    # eager work between replays
        outs = [g.read_output(i) for i in range(len(items))]
        bad = [i for i in range(len(items)) if not np.array_equal(outs[i], ref[i])]
        print("[gpu] replay pass %d: %d mismatching strings" % (rep, len(bad)), flush=True)
        assert not bad
    # a changed slot invalidates the graph
    g.excite(0, [items[0][1]])
    with pytest.raises(binding.SbError):
        g.graph_launch()
    g.close()


def test_autotune_keeps_results_and_rewinds():
    _gpu()
    items = W.random_batch(64, seconds=0.05)
    n = max(p["n_samples"] for p, _ in items)
    a = _batch(items)
    a.step(n)
    ref = [a.read_output(i) for i in range(len(items))]
    a.close()
    t = _batch(items)
    chosen = t.autotune(240)
    print("[gpu] autotune chose", chosen, flush=True)
    assert any(c > 0 for c in chosen)
    assert all(t.info(i)["samples_done"] == 2 for i in range(len(items)))
    t.step(n)
    for i in range(len(items)):
        assert np.array_equal(t.read_output(i), ref[i])
    t.close()
