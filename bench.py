#!/usr/bin/env python3
"""Benchmark of batched FP32 string synthesis on one MI355X.

One bench step synthesises a whole batch of strings from their excitation to
their last sample through the C ABI: a rewind on the device, then one eager
string_batch_step over the longest duration (the size classes' launches
forked onto their own streams and joined), with every input already in
device memory.  The same step replayed from a captured HIP graph, and the
same batch stepped in 480-sample chunks, are timed beside it.  Prints one
JSON line: grid-point updates per second (the sum over strings of
(N_t - 1 + N_l - 1) per time step), audio seconds per second, the roofline
position of each launch's kernel (the one with the most updates reported as
`roofline`), the FP64 CPU oracle timed on a sample of the same workload and
the GPU output's error against it on that sample (rel-L2 and partial offsets
in cents), the uniform 4096-string batch, the bowed, clamped and dataset
batches (each with the same error on 16 of its strings, and the oracle's own
spread under a 1e-7 change of f0 for any string above 1e-3), the plain FP64
per-string method on the single nonlinear string, and a real-time serving
run with Poisson arrivals (p50/p99 latencies).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "grid-point updates/s & audio-s/s, batched FP32 vs plain FP64; p99 latency"
PEAK_FP32_VECTOR = 157.3e12   # MI355X FP32 vector FLOP/s (256 CU x 2.4 GHz x 256)

# HBM traffic of one launch of the dominant kernel (step_kernel_small, the
# uneven 16384-string batch, one full step), from two rocprofv3 --pmc runs
# (FETCH_SIZE, WRITE_SIZE) scaled by what the same counters read for a
# 512 MiB device copy (x2.000 and x1.000); profiles/hbm_traffic_uneven16384.md.
# Valid only for the kernel sources it was measured on (kernel_source_hash).
TRAFFIC = {"kernel": "step_kernel_small<float, true>", "source_sha256": "32212cc91f09c9de",
           "fetch_bytes": 0.7706e9, "write_bytes": 8.626e9}

# the kernels of the three launch units of a step (size classes 0..4 merged,
# 5, then 6 and 7 on one stream)
LAUNCH_KERNELS = ["step_kernel_small<float, true>", "step_kernel<64, 8, float, true>",
                  "step_kernel<64, 10 and 16, float, true>"]

WORKLOADS = {
    # 16384 nonlinear strings, durations U(0.5, 4) s, vibrato or glide, FP32
    "uneven16384": lambda W: W.uneven_batch_16384(),
    # 4096 nonlinear strings of 2 s
    "uniform4096": lambda W: W.uniform_batch_4096(),
}


def unknowns(info):
    return (info["N_t"] - 1) + max(info["N_l"] - 1, 0)


KERNEL_SOURCES = ("step_kernel.h", "bow.h", "interp.h", "sfd_types.h")

# the bow, clamped and dataset legs' accuracy samples: their first strings,
# the opening samples of each (compared with the oracle in the cpu_baseline leg)
SAMPLE_STRINGS = 16
SAMPLE_CUT = 9600


def kernel_source_hash() -> str:
    """sha256 prefix over the sources the stepping kernels are built from."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2311_18505_amd", "csrc")
    for name in KERNEL_SOURCES:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """TRAFFIC when the kernels are built from the sources it was measured on, else None."""
    if kernel_source_hash() != TRAFFIC["source_sha256"]:
        return None
    return TRAFFIC["fetch_bytes"] + TRAFFIC["write_bytes"]


def cpu_baseline(items, seconds_cap, threads):
    """The FP64 oracle on a bounded sample of the workload, one string per
    host thread.  Returns the baseline record, the oracle's arithmetic per
    grid-point update (its RHS matvecs and banded elimination, without and
    with partial pivoting's fill) and the sample's outputs."""
    import oracle
    sample = []
    for p, e in items[:threads * 4]:
        # the note cut to its first seconds_cap: a glide keeps the full
        # note's rate (its interval scales with the cut) and both grids stay
        # those planned for the full note, so the cut oracle run computes the
        # same samples as the first ones of the GPU's full-length run
        ns = min(p["n_samples"], int(seconds_cap * p["fs"]))
        g = oracle.grid(p)
        q = dict(p, n_samples=ns, grid_t=g["N_t"], grid_l=g["N_l"])
        if p.get("mod_type", 0) == 2:
            q["glide_semitones"] = p["glide_semitones"] * ns / p["n_samples"]
        sample.append((q, e))
    t0 = time.perf_counter()
    res = oracle.run_many(sample, threads=threads)
    dt = time.perf_counter() - t0
    upd = 0
    flops = flops_nf = 0.0
    for r in res:
        g = r["grid"]
        n = (g["N_t"] - 1) + max(g["N_l"] - 1, 0)
        upd += n * r["steps_done"]
        flops += r["flops"]
        flops_nf += r["flops_nofill"]
    rec = {"value": upd / dt, "unit": "grid-point updates/s", "cores": threads, "kind": "oracle",
           "sample": "first %d strings of the workload, each cut to its first %.2f s (%d updates; glides keep "
                     "their rate, grids those of the full note), FP64, one string per thread"
                     % (len(sample), seconds_cap, upd),
           "seconds": dt, "host_cpus": os.cpu_count(), "cpu_model": cpu_model()}
    return rec, flops_nf / upd, flops / upd, [r["y_u"] for r in res]


def accuracy(outs, refs, fs):
    """Error of each GPU output against the oracle's on the same samples:
    rel-L2, and the offset in cents of the GPU output's spectral peaks from
    the oracle's (the six strongest peaks within 40 dB of each reference,
    both located by the same estimator on the same window)."""
    from paper_2311_18505_amd import analysis
    rel, cts = [], []
    for y, ref in zip(outs, refs):
        y = np.asarray(y, dtype=np.float64)[:len(ref)]
        rel.append(float(np.linalg.norm(y - ref) / np.linalg.norm(ref)))
        fr, lr = analysis.find_peaks(ref, fs, floor_db=-40.0)
        fy, _ = analysis.find_peaks(y, fs, floor_db=-60.0)
        for f in fr[np.argsort(lr)[::-1][:6]]:
            if len(fy):
                c = 1200.0 * np.log2(fy / f)
                j = int(np.argmin(np.abs(c)))
                cts.append(abs(float(c[j])))
    return {"strings": len(refs), "rel_l2_max": max(rel), "rel_l2_median": float(np.median(rel)),
            "partial_offset_cents_max": max(cts) if cts else None,
            "partial_offset_cents_median": float(np.median(cts)) if cts else None,
            "partials_compared": len(cts)}


def cut_note(p, e, events, seconds_cap):
    """A note cut to its first seconds_cap for the oracle so that it computes
    the same samples as the first ones of the GPU's full-length run: both
    grids pinned to the full note's, a glide and a moving bow keep their
    rates (their spans scale with the cut), events past the cut dropped.
    None for a note whose re-excitation moves a bow (its travel time follows
    the note's length)."""
    import oracle
    ns_full = p["n_samples"]
    ns = min(ns_full, int(seconds_cap * p["fs"]))
    g = oracle.grid(p)
    q = dict(p, n_samples=ns, grid_t=g["N_t"], grid_l=g["N_l"])
    if p.get("mod_type", 0) == 2:
        q["glide_semitones"] = p["glide_semitones"] * ns / ns_full
    if e.get("type") == 3 and e.get("x_end", e["x"]) != e["x"]:
        e = dict(e, x_end=e["x"] + (e["x_end"] - e["x"]) * ns / ns_full)
    kept = [(st, x) for st, x in (events or []) if st + 1 < ns]
    if any(x.get("type") == 3 and x.get("x_end", x["x"]) != x["x"] for _, x in kept):
        return None
    return q, e, kept


def leg_accuracy(sample, seconds_cap, threads):
    """accuracy() of a leg's sampled GPU outputs [(params, excitation, events,
    output)] against the oracle on the same notes cut to seconds_cap."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    jobs, outs = [], []
    for p, e, ev, y in sample:
        c = cut_note(p, e, ev, seconds_cap)
        if c is not None:
            jobs.append(c)
            outs.append(y)
    run = lambda c: oracle.run(c[0], c[1], schedule=c[2] or None)["y_u"]
    with ThreadPoolExecutor(max_workers=max(1, threads)) as ex:
        refs = list(ex.map(run, jobs))
        rec = accuracy(outs, refs, 48000.0)
        # a string above 1e-3 next to the oracle's own spread under a 1e-7
        # relative change of f0 (either sign): bowed strings near a stick/slip
        # tie move by O(1) under such changes, which bounds what any
        # arithmetic can reproduce
        rel = [float(np.linalg.norm(np.asarray(y, np.float64)[:len(r)] - r) / np.linalg.norm(r))
               for y, r in zip(outs, refs)]
        above = [i for i, x in enumerate(rel) if x > 1e-3]
        nudged = [(dict(jobs[i][0], f0=jobs[i][0]["f0"] * (1 + d)), jobs[i][1], jobs[i][2])
                  for i in above for d in (1e-7, -1e-7)]
        spread_runs = list(ex.map(run, nudged))
    rec["above_1e-3"] = [{"rel_l2": rel[i], "oracle_spread_1e-7_f0": max(
        float(np.linalg.norm(q - refs[i]) / np.linalg.norm(refs[i])) for q in spread_runs[2 * k:2 * k + 2])}
        for k, i in enumerate(above)]
    rec["sample"] = "%d strings of the leg, each cut to its first %.2f s" % (len(jobs), seconds_cap)
    return rec


def cpu_model() -> str:
    """The host CPU's model name (Linux), or "unknown"."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def plain_leg(W, binding, hiptime, seconds):
    """The plain FP64 per-string method (eq. (7), one string per launch, banded
    LU) on the single nonlinear hammered string, timed with HIP events."""
    p, e = W.single_nonlinear(seconds=seconds)
    b = binding.StringBatch(1, "fp64_plain")
    b.set_params(0, [p])
    b.excite(0, [e])
    inf = b.info(0)
    hiptime.synchronize()
    ev0, ev1 = hiptime.Event(), hiptime.Event()
    ev0.record(0)
    b.step(p["n_samples"])
    ev1.record(0)
    ev1.synchronize()
    ms = ev0.elapsed_ms(ev1)
    done = b.info(0)
    b.close()
    upd = unknowns(inf) * (p["n_samples"] - 2)
    return {"value": upd / (ms / 1e3), "unit": "grid-point updates/s", "audio_s_per_s": seconds / (ms / 1e3),
            "ms": ms, "workload": "single nonlinear hammered string, %.1f s (N_t=%d, N_l=%d), FP64, "
                                  "one string per launch" % (seconds, inf["N_t"], inf["N_l"]),
            "finished": done["samples_done"] == p["n_samples"] and done["flags"] == 0}


def uniform_leg(W, binding, hiptime):
    """The uniform batch: 4096 nonlinear strings of 2 s, FP32 compensated,
    autotuned, one eager step of the whole batch after a warm-up (HIP
    events)."""
    items = W.uniform_batch_4096()
    b = binding.StringBatch(len(items), "fp32c")
    b.set_params(0, [p for p, _ in items])
    b.excite(0, [e for _, e in items])
    infos = [b.info(i) for i in range(len(items))]
    steps = max(p["n_samples"] for p, _ in items)
    tuned = b.autotune(480)
    b.step(steps)                       # warm-up
    b.rewind()
    hiptime.synchronize()
    ev0, ev1 = hiptime.Event(), hiptime.Event()
    ev0.record(0)
    b.step(steps)
    ev1.record(0)
    ev1.synchronize()
    ms = ev0.elapsed_ms(ev1)
    bad = sum(1 for i in range(len(items)) if b.info(i)["flags"] != 0 or b.info(i)["samples_done"] != infos[i]["n_samples"])
    b.close()
    upd = sum(unknowns(inf) * (inf["n_samples"] - 2) for inf in infos)
    return {"value": upd / (ms / 1e3), "unit": "grid-point updates/s", "audio_s_per_s": len(items) * 2.0 / (ms / 1e3),
            "ms": ms, "updates": upd, "blocks_per_cu": tuned, "strings_not_finished": bad,
            "workload": "4096 nonlinear strings of 2.0 s (seeded draws), FP32 compensated"}


def bow_leg(W, binding, hiptime, n, seconds):
    """Bowed strings (eq. 5) in FP32 compensated: a seeded batch of n bowed
    nonlinear strings, and the same strings plucked, one launch each (HIP
    events); the ratio is the cost of the stick/slip solve inside the sweeps."""
    items = W.bowed_batch(n, seconds=seconds)
    pluck = W.pluck(0.2, 1e-3)
    res = {}
    for name, excs in (("bowed", [e for _, e in items]), ("plucked", [pluck] * n)):
        b = binding.StringBatch(n, "fp32c")
        b.set_params(0, [p for p, _ in items])
        b.excite(0, excs)
        infos = [b.info(i) for i in range(n)]
        steps = max(p["n_samples"] for p, _ in items)
        b.step(480)                     # first launch of the kernels, not timed
        b.rewind()
        hiptime.synchronize()
        ev0, ev1 = hiptime.Event(), hiptime.Event()
        ev0.record(0)
        b.step(steps)
        ev1.record(0)
        ev1.synchronize()
        ms = ev0.elapsed_ms(ev1)
        bad = sum(1 for i in range(n) if b.info(i)["flags"] != 0 or b.info(i)["samples_done"] != infos[i]["n_samples"])
        sweeps = sum(b.info(i)["total_sweeps"] for i in range(n))
        if name == "bowed":
            sample = [(items[i][0], excs[i], [], b.read_output(i, 0, min(items[i][0]["n_samples"], SAMPLE_CUT)))
                      for i in range(min(n, SAMPLE_STRINGS))]
        b.close()
        upd = sum(unknowns(inf) * (inf["n_samples"] - 2) for inf in infos)
        res[name] = {"value": upd / (ms / 1e3), "ms": ms, "audio_s_per_s": n * seconds / (ms / 1e3),
                     "sweeps_per_step_mean": sweeps / max(1, sum(inf["n_samples"] - 2 for inf in infos)),
                     "strings_not_finished": bad}
    return {"value": res["bowed"]["value"], "unit": "grid-point updates/s",
            "audio_s_per_s": res["bowed"]["audio_s_per_s"], "ms": res["bowed"]["ms"],
            "sweeps_per_step_mean": res["bowed"]["sweeps_per_step_mean"],
            "strings_not_finished": res["bowed"]["strings_not_finished"],
            "plucked_same_strings": res["plucked"], "bowed_vs_plucked": res["bowed"]["value"] / res["plucked"]["value"],
            "workload": "%d bowed nonlinear strings of %.1f s (seeded draws), FP32 compensated" % (n, seconds)}, sample


def clamped_leg(W, binding, hiptime, n, seconds):
    """Clamped ends (Sec. 4.1) in FP32 compensated: a seeded batch of n
    nonlinear strings (plucks and hammers), clamped and simply supported, one
    launch each (HIP events).  Clamped strings run in the kernel instantiation
    that also carries the bow; the ratio is what that costs."""
    items = W.random_batch(n, seconds=seconds, seed=W.SEED + 31)
    res = {}
    for name, bnd in (("clamped", 1), ("simply_supported", 0)):
        b = binding.StringBatch(n, "fp32c")
        b.set_params(0, [dict(p, boundary=bnd) for p, _ in items])
        b.excite(0, [e for _, e in items])
        infos = [b.info(i) for i in range(n)]
        steps = max(p["n_samples"] for p, _ in items)
        b.step(480)                     # first launch of the kernels, not timed
        b.rewind()
        hiptime.synchronize()
        ev0, ev1 = hiptime.Event(), hiptime.Event()
        ev0.record(0)
        b.step(steps)
        ev1.record(0)
        ev1.synchronize()
        ms = ev0.elapsed_ms(ev1)
        bad = sum(1 for i in range(n) if b.info(i)["flags"] != 0 or b.info(i)["samples_done"] != infos[i]["n_samples"])
        if bnd == 1:
            sample = [(dict(items[i][0], boundary=1), items[i][1], [],
                       b.read_output(i, 0, min(items[i][0]["n_samples"], SAMPLE_CUT)))
                      for i in range(min(n, SAMPLE_STRINGS))]
        b.close()
        upd = sum(unknowns(inf) * (inf["n_samples"] - 2) for inf in infos)
        res[name] = {"value": upd / (ms / 1e3), "ms": ms, "audio_s_per_s": n * seconds / (ms / 1e3),
                     "strings_not_finished": bad}
    return {"value": res["clamped"]["value"], "unit": "grid-point updates/s",
            "audio_s_per_s": res["clamped"]["audio_s_per_s"], "ms": res["clamped"]["ms"],
            "strings_not_finished": res["clamped"]["strings_not_finished"],
            "simply_supported_same_strings": res["simply_supported"],
            "clamped_vs_simply_supported": res["clamped"]["value"] / res["simply_supported"]["value"],
            "workload": "%d nonlinear strings of %.1f s (seeded draws, plucks and hammers), FP32 compensated"
                        % (n, seconds)}, sample


def dataset_leg(hiptime, n, seconds):
    """The dataset generator: n labelled notes of U(seconds) s, a third each
    plucked, hammered and bowed, half of them given one or two more hammers
    or bows mid-note (FP32 compensated, one batch); wall time of the
    synthesis with the host work of its re-excitations."""
    from paper_2311_18505_amd import dataset
    notes = dataset.draw_notes(n, seconds=seconds, restrike_prob=0.5)
    dataset.synthesize(notes[:64], "fp32c", capacity=64)      # first launches of the kernels
    hiptime.synchronize()
    t0 = time.perf_counter()
    audio = dataset.synthesize(notes, "fp32c", capacity=n)
    hiptime.synchronize()
    wall = time.perf_counter() - t0
    secs = sum(x["params"]["n_samples"] for x in notes) / 48000.0
    sample = [(x["params"], x["excitation"], x["events"], a[:SAMPLE_CUT])
              for x, a in zip(notes[:SAMPLE_STRINGS], audio[:SAMPLE_STRINGS]) if a is not None]
    return {"value": secs / wall, "unit": "audio-s/s", "notes_per_s": n / wall, "wall_s": wall,
            "notes": n, "events": sum(len(x["events"]) for x in notes),
            "finite": bool(all(np.isfinite(a).all() for a in audio if a is not None)),
            "flagged_notes": sum(1 for a in audio if a is None),
            "workload": "%d notes of U(%.1f, %.1f) s, pluck/hammer/bow, half re-excited mid-note once or twice, "
                        "FP32 compensated" % (n, seconds[0], seconds[1])}, sample


def serving_leg(W, serving, rate, seconds, capacity):
    """Continuous-batching server under Poisson arrivals (one string per
    request, durations U(0.25, 3) s), in real time."""
    arrivals, items = W.serving_requests(rate_hz=rate, seconds=seconds)
    reqs = serving.requests_from(arrivals, items)
    srv = serving.Server(capacity=capacity)
    stats, _ = srv.run(reqs, log=lambda m: print("[bench] serving " + m, file=sys.stderr, flush=True))
    srv.close()
    rec = stats.summary()
    rec.update({"rate_hz": rate, "seconds": seconds, "requests": len(reqs),
                "offered_audio_s_per_s": sum(p["n_samples"] / p["fs"] for p, _ in items) / seconds,
                "chunk_samples": serving.CHUNK, "capacity": capacity})
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="uneven16384", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-seconds", type=float, default=0.25, help="duration cap of the oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--plain-seconds", type=float, default=2.0, help="duration of the plain FP64 comparator run")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-uniform", action="store_true", help="skip the uniform 4096-string batch leg")
    ap.add_argument("--no-chunked", action="store_true", help="skip timing the batch in 480-sample chunks")
    ap.add_argument("--bow-strings", type=int, default=4096, help="strings of the bowed-batch leg")
    ap.add_argument("--no-bow", action="store_true")
    ap.add_argument("--clamped-strings", type=int, default=4096, help="strings of the clamped-ends leg")
    ap.add_argument("--no-clamped", action="store_true")
    ap.add_argument("--dataset-notes", type=int, default=16384, help="notes of the dataset-generator leg")
    ap.add_argument("--no-dataset", action="store_true")
    ap.add_argument("--serving-seconds", type=float, default=60.0, help="arrival window of the serving run")
    ap.add_argument("--serving-rate", type=float, default=2000.0)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after the run, one device copy of this size (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the strings are independent and the library has no "
              "multi-GPU path (got --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    from paper_2311_18505_amd import binding, hiptime, workloads as W

    t_setup = time.perf_counter()
    items = WORKLOADS[args.workload](W)
    params = [p for p, _ in items]
    excs = [e for _, e in items]
    b = binding.StringBatch(len(items), "fp32c")
    b.set_params(0, params)
    b.excite(0, excs)
    infos = [b.info(i) for i in range(len(items))]
    n_max = max(p["n_samples"] for p in params)
    upd_of = [unknowns(inf) * (inf["n_samples"] - 2) for inf in infos]
    updates = sum(upd_of)
    audio_s = sum(p["n_samples"] / p["fs"] for p in params)
    print("[bench] %s: %d strings, %.3e grid-point updates per step, %.0f audio-s, setup %.1f s"
          % (args.workload, len(items), updates, audio_s, time.perf_counter() - t_setup), file=sys.stderr, flush=True)
    # persistent blocks per CU for each launch
    tuned = b.autotune(480)
    print("[bench] autotuned blocks/CU per launch %s" % tuned, file=sys.stderr, flush=True)

    for w in range(args.warmup):
        b.rewind()
        b.step(n_max)
        hiptime.synchronize()
        print("[bench] warmup %d done" % w, file=sys.stderr, flush=True)

    ev0, ev1 = hiptime.Event(), hiptime.Event()
    hiptime.synchronize()
    t0 = time.perf_counter()
    ev0.record(0)
    for k in range(args.steps):
        b.rewind()
        b.step(n_max)
    ev1.record(0)
    ev1.synchronize()
    hiptime.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_ms(ev1)
    launch_ms, launch_strings = b.launch_times()      # kernels of the last timed step
    print("[bench] %d steps: wall %.3f s, events %.3f ms; launch kernels (ms) %s"
          % (args.steps, wall, gpu_ms, ["%.1f" % m for m in launch_ms]), file=sys.stderr, flush=True)
    # the same step as one replay of a captured HIP graph (outside the timed region)
    b.rewind()
    b.graph_capture(n_max, 1)
    hiptime.synchronize()
    g0, g1 = hiptime.Event(), hiptime.Event()
    g0.record(0)
    b.graph_launch()
    g1.record(0)
    g1.synchronize()
    graph_ms = g0.elapsed_ms(g1)
    print("[bench] graph replay: %.3f ms" % graph_ms, file=sys.stderr, flush=True)
    # the oracle's sample: the first strings' first samples (read after the
    # replay, which recomputes the same outputs)
    n_cpu = min(len(items), 4 * min(16, os.cpu_count() or 1))
    cut = int(args.cpu_seconds * 48000)
    gpu_sample = [b.read_output(i, 0, min(params[i]["n_samples"], cut)) for i in range(n_cpu)]
    chunked_ms = None
    if not args.no_chunked:
        # the same batch stepped in 480-sample chunks (one step call each)
        b.rewind()
        hiptime.synchronize()
        c0, c1 = hiptime.Event(), hiptime.Event()
        c0.record(0)
        for _ in range(0, n_max, 480):
            b.step(480)
        c1.record(0)
        c1.synchronize()
        chunked_ms = c0.elapsed_ms(c1)
        print("[bench] 480-sample chunks: %.3f ms" % chunked_ms, file=sys.stderr, flush=True)

    # every string must have finished cleanly
    bad = 0
    sweeps = 0
    for i in range(len(items)):
        inf = b.info(i)
        sweeps += inf["total_sweeps"]
        if inf["flags"] != 0 or inf["samples_done"] != inf["n_samples"]:
            bad += 1
    b.close()
    if bad:
        print("[bench] %d strings did not finish cleanly" % bad, file=sys.stderr, flush=True)

    sec_per_step = wall / args.steps
    value = updates / sec_per_step
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "grid-point updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec_per_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "strings": len(items), "fs": 48000,
                   "updates_per_step": updates, "audio_seconds_per_step": audio_s,
                   "precision": "FP32 with compensated state updates, FP64 energy monitor",
                   "launch": "three concurrent persistent launch units per step (size classes 0-4 merged, 5, "
                             "then 6 and 7; forked onto their streams and joined), each grid of a string laid out "
                             "on the fewest of MM, 3MM/4 and MM/2 slots per lane it fits in, blocks/CU "
                             "autotuned; the same step replayed from a HIP graph is reported beside",
                   "blocks_per_cu": tuned},
        "audio_s_per_s": audio_s / sec_per_step,
        "sweeps_per_step_mean": sweeps / max(1, sum(inf["n_samples"] - 2 for inf in infos)),
        "strings_not_finished": bad,
        "gpu_ms_per_step": gpu_ms / args.steps,
        "graph_replay_ms": graph_ms,
        "chunked_480_ms": chunked_ms,
    }
    samples = {}   # leg -> [(params, excitation, events, GPU output)] for accuracy_vs_oracle
    if not args.no_plain:
        pl = plain_leg(W, binding, hiptime, args.plain_seconds)
        print("[bench] plain FP64: %.1f ms, %.3e updates/s" % (pl["ms"], pl["value"]), file=sys.stderr, flush=True)
        out["plain_fp64"] = pl
        out["batched_vs_plain"] = value / pl["value"]
    if not args.no_uniform and args.workload != "uniform4096":
        un = uniform_leg(W, binding, hiptime)
        print("[bench] uniform 4096: %.1f ms, %.3e updates/s" % (un["ms"], un["value"]), file=sys.stderr, flush=True)
        out["uniform4096_fp32c"] = un
    if not args.no_bow:
        bw, samples["bow_fp32c"] = bow_leg(W, binding, hiptime, args.bow_strings, 1.0)
        print("[bench] bow: %.1f ms, %.3e updates/s (%.2f x the same strings plucked)"
              % (bw["ms"], bw["value"], bw["bowed_vs_plucked"]), file=sys.stderr, flush=True)
        out["bow_fp32c"] = bw
    if not args.no_clamped:
        cl, samples["clamped_fp32c"] = clamped_leg(W, binding, hiptime, args.clamped_strings, 1.0)
        print("[bench] clamped: %.1f ms, %.3e updates/s (%.2f x the same strings simply supported)"
              % (cl["ms"], cl["value"], cl["clamped_vs_simply_supported"]), file=sys.stderr, flush=True)
        out["clamped_fp32c"] = cl
    if not args.no_dataset:
        ds, samples["dataset_fp32c"] = dataset_leg(hiptime, args.dataset_notes, (0.5, 2.0))
        print("[bench] dataset: %d notes (%d re-excitations) in %.2f s, %.0f audio-s/s"
              % (ds["notes"], ds["events"], ds["wall_s"], ds["value"]), file=sys.stderr, flush=True)
        out["dataset_fp32c"] = ds
    if not args.no_serving:
        from paper_2311_18505_amd import serving
        print("[bench] serving: %.0f requests/s for %.0f s" % (args.serving_rate, args.serving_seconds),
              file=sys.stderr, flush=True)
        sv = serving_leg(W, serving, args.serving_rate, args.serving_seconds, 16384)
        print("[bench] serving done: %s" % json.dumps(sv), file=sys.stderr, flush=True)
        out["serving"] = sv
        if "plain_fp64" in out:
            # one stream, FIFO, one request at a time: the plain method sustains
            # (its audio-s/s) / (mean request duration) requests per second
            mean_T = 0.5 * (0.25 + 3.0)
            out["serving"]["plain_fp64_max_rate_hz"] = out["plain_fp64"]["audio_s_per_s"] / mean_T
    if not args.no_cpu:
        threads = min(16, os.cpu_count() or 1)
        rec, flops_per_update, flops_fill, refs = cpu_baseline(items, args.cpu_seconds, threads)
        out["cpu_baseline"] = {k: v for k, v in rec.items() if k != "seconds"}
        out["accuracy_vs_oracle"] = dict(accuracy(gpu_sample, refs, 48000.0),
                                         sample=rec["sample"], precision="FP32 compensated vs FP64 oracle")
        print("[bench] accuracy vs oracle: %s" % json.dumps(out["accuracy_vs_oracle"]), file=sys.stderr, flush=True)
        # the bow, clamped and dataset legs: their first strings' opening
        # samples against the oracle
        for leg, smp in samples.items():
            out[leg]["accuracy_vs_oracle"] = dict(leg_accuracy(smp, SAMPLE_CUT / 48000.0, threads),
                                                  precision="FP32 compensated vs FP64 oracle")
            print("[bench] %s accuracy vs oracle: %s" % (leg, json.dumps(out[leg]["accuracy_vs_oracle"])),
                  file=sys.stderr, flush=True)
        # roofline of each launch's kernel: the oracle's arithmetic per
        # grid-point update (banded elimination without pivoting's fill) times
        # the updates of that launch's strings, over the kernel's own duration
        # (HIP events on its stream, last timed step)
        by_launch = []
        for u in range(binding.NUM_LAUNCHES):
            if launch_ms[u] <= 0:
                continue
            upd_u = sum(x for x, inf in zip(upd_of, infos) if inf["size_class"] in binding.LAUNCH_CLASSES[u])
            ach = flops_per_update * upd_u / (launch_ms[u] / 1e3)
            by_launch.append({"kernel": LAUNCH_KERNELS[u], "classes": list(binding.LAUNCH_CLASSES[u]),
                              "ms": launch_ms[u], "strings": launch_strings[u], "updates": upd_u,
                              "achieved_tflops": ach / 1e12, "frac": ach / PEAK_FP32_VECTOR})
        # the dominant kernel: the launch that carries the most updates
        dom = max(by_launch, key=lambda r: r["updates"])
        out["roofline"] = {"bound": "alu", "achieved": dom["achieved_tflops"], "peak": PEAK_FP32_VECTOR / 1e12,
                           "unit": "TFLOP/s", "frac": dom["frac"],
                           "traffic": measured_traffic() if dom["kernel"] == TRAFFIC["kernel"] else None,
                           "kernel": dom["kernel"], "kernel_ms_per_launch": dom["ms"],
                           "flops_per_update": flops_per_update,
                           "flops_per_update_with_pivoting_fill": flops_fill,
                           "whole_step_frac": flops_per_update * updates / (gpu_ms / args.steps / 1e3) / PEAK_FP32_VECTOR}
        out["roofline_by_launch"] = by_launch
    print(json.dumps(out), flush=True)
    if args.copy_probe_mib > 0:
        hiptime.copy_probe(args.copy_probe_mib << 20)
        print("[bench] copy probe: %d MiB device to device" % args.copy_probe_mib, file=sys.stderr, flush=True)


if __name__ == "__main__":
    main()
