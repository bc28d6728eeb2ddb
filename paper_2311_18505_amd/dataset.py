"""Offline synthesis of labelled string notes (the paper's dataset use, Sec. 1).

Each note is one string with seed-drawn physical parameters (f0, B, alpha,
losses, vibrato or glide), an initial pluck, hammer or bow, and optionally
further hammers or bows during the note (string_batch_restrike).  Notes are
synthesised in batches of up to `capacity` slots on the GPU library; the
labels are the parameters themselves.

Re-excitation times are quantised to blocks of `block` samples (480 = 10 ms
at 48 kHz), so a batch steps from one block boundary to the next and sets the
new excitations of all its notes at once between launches.

Usage as a program (writes labels.json and, per batch, one .npy of
zero-padded rows of audio):

    python -m paper_2311_18505_amd.dataset --notes 4096 --seconds 1 --out DIR
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

from . import binding, workloads as W

BLOCK = 480


def draw_notes(n: int, seed: int = W.SEED + 21, seconds=(0.5, 2.0), restrike_prob: float = 0.5,
               block: int = BLOCK) -> list:
    """Notes: dicts with 'params', 'excitation' and 'events' [(step, excitation)].

    Strings as in workloads.random_batch with modulation; the first
    excitation is a pluck, hammer or bow (1/3 each); with probability
    restrike_prob a note gets one or two further hammers or bows at block
    boundaries inside its first 80 %."""
    rng = np.random.default_rng(seed)
    lo, hi = seconds
    base = W.random_batch(n, seed=seed, durations=("uniform", lo, hi), modulation=True)
    bows = W.bowed_batch(n, seed=seed + 1, seconds=1.0)
    notes = []
    for i in range(n):
        p, e = base[i]
        ns = p["n_samples"]
        kind = rng.integers(0, 3)
        if kind == 2:
            e = dict(bows[i][1], x_end=bows[i][1]["x"])
        events = []
        if rng.uniform() < restrike_prob:
            nb = max(1, int(0.8 * ns) // block)
            k = int(rng.integers(1, 3))
            for b in sorted(set(int(x) for x in rng.integers(1, max(2, nb), k))):
                step = b * block - 1     # the step that computes sample b * block
                if step < 2:
                    continue
                if rng.uniform() < 0.5:
                    x = W.hammer(rng.uniform(0.05, 0.3), rng.uniform(0.5, 4.0))
                else:
                    x = W.bow(rng.uniform(0.05, 0.3), rng.uniform(0.05, 0.2), float(np.exp(rng.uniform(np.log(20), np.log(200)))),
                              attack=rng.uniform(0.005, 0.05), fric_a=rng.uniform(20, 200), fric_eps=rng.uniform(0.1, 0.5))
                events.append((step, x))
        notes.append({"params": p, "excitation": e, "events": events})
    return notes


def synthesize(notes: list, precision: str = "fp32c", capacity: int = 4096, log=None) -> list:
    """Audio of every note (numpy arrays of the batch precision), in order;
    None for a note whose string the device flagged (energy monitor or
    solver), which the dataset leaves out."""
    out = [None] * len(notes)
    for first in range(0, len(notes), capacity):
        part = notes[first:first + capacity]
        b = binding.StringBatch(len(part), precision)
        try:
            b.set_params(0, [x["params"] for x in part])
            b.excite(0, [x["excitation"] for x in part])
            ns = max(x["params"]["n_samples"] for x in part)
            # events by step: the batch steps to each one and re-excites there
            by_step = {}
            for i, x in enumerate(part):
                for step, ex in x["events"]:
                    by_step.setdefault(step, []).append((i, ex))
            done = 2
            for step in sorted(by_step):
                b.step(step + 1 - done)
                done = step + 1
                live = [(i, ex) for i, ex in by_step[step] if done < part[i]["params"]["n_samples"]]
                if live:
                    b.restrike_list([i for i, _ in live], [ex for _, ex in live])
            b.step(ns - done)
            for i in range(len(part)):
                try:
                    out[first + i] = b.read_output(i)
                except binding.SbError as err:
                    if err.code != binding.SB_EUNSTABLE:
                        raise
                    out[first + i] = None
        finally:
            b.close()
        if log:
            log("batch %d-%d done" % (first, first + len(part)))
    return out


def labels(note: dict) -> dict:
    def clean(d):
        return {k: (float(v) if isinstance(v, (float, np.floating)) else int(v) if isinstance(v, (int, np.integer)) else v)
                for k, v in d.items()}
    return {"params": clean(note["params"]), "excitation": clean(note["excitation"]),
            "events": [[int(s), clean(x)] for s, x in note["events"]]}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--notes", type=int, default=4096)
    ap.add_argument("--seconds", type=float, nargs=2, default=(0.5, 2.0))
    ap.add_argument("--restrike-prob", type=float, default=0.5)
    ap.add_argument("--precision", default="fp32c", choices=["fp32c", "fp64"])
    ap.add_argument("--capacity", type=int, default=4096)
    ap.add_argument("--seed", type=int, default=W.SEED + 21)
    ap.add_argument("--out", required=True)
    args = ap.parse_args()
    os.makedirs(args.out, exist_ok=True)
    notes = draw_notes(args.notes, seed=args.seed, seconds=tuple(args.seconds), restrike_prob=args.restrike_prob)
    t = time.perf_counter()
    audio = synthesize(notes, args.precision, args.capacity, log=lambda m: print("[dataset] " + m, flush=True))
    dt = time.perf_counter() - t
    kept = [(x, a) for x, a in zip(notes, audio) if a is not None]
    for first in range(0, len(kept), args.capacity):
        part = [a for _, a in kept[first:first + args.capacity]]
        rows = np.zeros((len(part), max(len(a) for a in part)), dtype=part[0].dtype)
        for i, a in enumerate(part):
            rows[i, :len(a)] = a
        np.save(os.path.join(args.out, "audio_%06d.npy" % first), rows)   # zero-padded rows
    with open(os.path.join(args.out, "labels.json"), "w") as f:
        json.dump([dict(labels(x), samples=len(a)) for x, a in kept], f)
    if len(kept) < len(notes):
        print("[dataset] %d notes flagged by the device and left out" % (len(notes) - len(kept)), flush=True)
    secs = sum(x["params"]["n_samples"] for x in notes) / 48000.0
    print("[dataset] %d notes, %.0f audio-s in %.1f s (%.0f audio-s/s)" % (len(notes), secs, dt, secs / dt), flush=True)


if __name__ == "__main__":
    main()
