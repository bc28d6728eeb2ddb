"""The dataset generator's note drawing (host only): deterministic, labelled,
events inside the notes at block boundaries."""
from __future__ import annotations

import json

from paper_2311_18505_amd import dataset


def test_draw_notes_is_seeded_and_serialisable():
    a = dataset.draw_notes(64, seconds=(0.2, 0.5), restrike_prob=1.0)
    b = dataset.draw_notes(64, seconds=(0.2, 0.5), restrike_prob=1.0)
    assert json.dumps([dataset.labels(x) for x in a]) == json.dumps([dataset.labels(x) for x in b])
    kinds = {x["excitation"]["type"] for x in a}
    assert kinds == {1, 2, 3}
    for x in a:
        ns = x["params"]["n_samples"]
        steps = [s for s, _ in x["events"]]
        assert steps == sorted(steps)
        for s, e in x["events"]:
            assert 2 <= s < ns - 1 and (s + 1) % dataset.BLOCK == 0
            assert e["type"] in (2, 3)
    assert sum(len(x["events"]) for x in a) >= 64
