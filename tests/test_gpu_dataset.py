"""The dataset generator on the GPU: notes with several excitations each
against the oracle's schedule."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2311_18505_amd import binding, dataset

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32c", 1e-3)])
def test_dataset_notes_match_oracle(precision, tol):
    if not binding.device_available():
        pytest.skip("no GPU")
    notes = dataset.draw_notes(24, seconds=(0.05, 0.1), restrike_prob=1.0)
    print("[gpu] dataset %s: %d notes, %d events" % (precision, len(notes), sum(len(x["events"]) for x in notes)),
          flush=True)
    audio = dataset.synthesize(notes, precision, capacity=16)
    refs = oracle.run_many([(x["params"], x["excitation"]) for x in notes])   # warm the oracle library
    errs = []
    for x, y in zip(notes, audio):
        ref = oracle.run(x["params"], x["excitation"], schedule=x["events"])["y_u"]
        errs.append(float(np.linalg.norm(np.asarray(y, np.float64) - ref) / np.linalg.norm(ref)))
    print("[gpu] dataset %s: worst rel-L2 %.3e" % (precision, max(errs)), flush=True)
    assert len(refs) == len(notes)
    assert max(errs) <= tol
