"""GPU parity of the bow (eq. 5) through the C ABI against the FP64 oracle.

The bow adds, in every sweep of the coupled solve, the exact solution of the
step's stick/slip problem (a rank-one correction along g = T_u0^{-1} J_p(x_B));
at convergence the step solves the same equations as the oracle's direct
method, so FP64 agrees to rounding.  Cases: the single bowed string (fixed
and moving bow), a seeded batch of bowed nonlinear strings mixed with plucks
and hammers, a low string in the largest size class, FP32 compensated, and
the plain path's refusal.

Stick/slip motion amplifies rounding differences: over longer runs the
element-wise distance between two FP64 implementations grows at the rate the
problem itself sets.  The longer FP64 case therefore bounds the GPU's
distance to the oracle by the oracle's own spread under a 1e-13 relative
change of the bow force (or 1e-10, whichever is larger).  In FP32 a few
bowed strings are that sensitive within 0.05 s already; those are bounded
by 3x the oracle's spread under 1e-7 relative changes of their parameters.
"""
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


def agree_window(ref, others, tol):
    """Samples from the start over which every run in `others` stays within
    tol x max|ref| of ref, element by element."""
    scale = np.max(np.abs(ref))
    dev = np.max([np.abs(np.asarray(q, np.float64) - ref) for q in others], axis=0)
    bad = np.nonzero(dev > tol * scale)[0]
    return int(bad[0]) if len(bad) else len(ref)


def check_in_window(y, ref, others):
    """Element-wise parity over the window in which the nudged oracle runs
    still agree with the oracle within 1e-4: there the GPU output must lie
    within 1e-3 x max|ref| of it (an FP32 rounding of the parameters moves the
    oracle by less than 1e-4 there).  Returns the window length."""
    n = agree_window(ref, others, 1e-4)
    scale = np.max(np.abs(ref))
    d = float(np.max(np.abs(np.asarray(y[:n], np.float64) - ref[:n]))) / scale if n else 0.0
    assert d <= 1e-3, (n, d)
    return n


def _run(items, precision):
    print("[gpu] bow %s: %d strings, up to %d samples" % (precision, len(items), max(p["n_samples"] for p, _ in items)),
          flush=True)
    b = binding.StringBatch(len(items), precision)
    b.set_params(0, [p for p, _ in items])
    b.excite(0, [e for _, e in items])
    b.step(max(p["n_samples"] for p, _ in items))
    outs = [b.read_output(i) for i in range(len(items))]
    infos = [b.info(i) for i in range(len(items))]
    b.close()
    return outs, infos


def _items(seconds=0.05):
    p, e = W.single_bowed(seconds=0.25)
    items = [(p, e), (p, dict(e, x_end=0.2))]
    items += W.bowed_batch(40, seconds=seconds)
    items += W.random_batch(8, seconds=seconds)
    # a low bowed string (largest size class), moving bow
    low = W.string(20.7, 1e-5, 1.2, 0.5, 1e-4, 2400)
    items.append((low, W.bow(0.1, 0.1, 60.0, x_end=0.13)))
    return items


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32c", 1e-3)])
def test_bowed_strings_match_oracle(precision, tol):
    _gpu()
    items = _items()
    refs = oracle.run_many(items)
    outs, infos = _run(items, precision)
    errs = [rel_l2(y, r["y_u"]) for y, r in zip(outs, refs)]
    worst = int(np.argmax(errs))
    print("[gpu] bow %s: median rel-L2 %.3e, worst %.3e (string %d, N=(%d,%d), class %d, max sweeps %d)"
          % (precision, np.median(errs), errs[worst], worst, infos[worst]["N_t"], infos[worst]["N_l"],
             infos[worst]["size_class"], infos[worst]["max_sweeps"]), flush=True)
    assert infos[-1]["size_class"] == 7
    assert all(inf["flags"] == 0 and inf["samples_done"] == p["n_samples"] for (p, _), inf in zip(items, infos))
    if precision == "fp64":
        # stick/slip decisions make a few bowed strings sensitive at the
        # rounding level: two FP64 solutions of the step's slip root that
        # differ in the last bit move string 17's output by ~1e-10 within
        # 0.05 s.  Those are held to 10x the oracle's own spread under a
        # 1e-13 relative change of the bow force, the rest to 1e-10.
        above = [i for i in range(len(items)) if errs[i] > tol]
        for i in above:
            p, e = items[i]
            assert e.get("type") == 3, i
            spread = rel_l2(oracle.run(p, dict(e, F_B=e["F_B"] * (1 + 1e-13)))["y_u"], refs[i]["y_u"])
            print("[gpu] bow fp64 string %d: rel-L2 %.2e, oracle spread under 1e-13 F_B %.2e" % (i, errs[i], spread),
                  flush=True)
            assert errs[i] <= max(tol, 10 * spread)
        assert len(above) <= 2
        return
    # FP32: a few bowed strings are ill-conditioned already over 0.05 s (a
    # 1e-7 relative change of f0 or v_B moves the oracle's output by O(1));
    # bound each string by 3x the oracle's spread under such changes
    bowed = [i for i, (_, e) in enumerate(items) if e.get("type") == 3 and errs[i] > tol]
    nudged = []
    for i in bowed:
        p, e = items[i]
        for rel in (1e-7, -1e-7):
            nudged += [(dict(p, **{key: p[key] * (1 + rel)}), e) for key in ("f0", "B", "alpha")]
            nudged += [(p, dict(e, **{key: e[key] * (1 + rel)})) for key in ("x", "v_B", "F_B")]
    print("[cpu] oracle: %d nudged runs for %d strings above %.0e" % (len(nudged), len(bowed), tol), flush=True)
    spread_runs = oracle.run_many(nudged) if nudged else []
    ratio = {}
    for j, i in enumerate(bowed):
        runs = [q["y_u"] for q in spread_runs[12 * j:12 * j + 12]]
        spread = max(rel_l2(q, refs[i]["y_u"]) for q in runs)
        ratio[i] = errs[i] / max(tol, 3 * spread)
        win = check_in_window(outs[i], refs[i]["y_u"], runs)
        print("[gpu] bow fp32c string %d: rel-L2 %.2e, oracle spread %.2e, element-wise within 1e-3 over the "
              "first %d samples" % (i, errs[i], spread, win), flush=True)
        assert win >= 240
    assert all(errs[i] <= tol for i in range(len(items)) if i not in ratio)
    assert all(r <= 1.0 for r in ratio.values())


def test_bowed_fp64_within_the_problems_conditioning():
    _gpu()
    items = _items(seconds=0.1)
    refs = oracle.run_many(items)
    nudged = [(p, dict(e, F_B=e["F_B"] * (1 + 1e-13)) if e.get("type") == 3 else e) for p, e in items]
    refs2 = oracle.run_many(nudged)
    outs, infos = _run(items, "fp64")
    worst = 0.0
    for y, r, r2, inf in zip(outs, refs, refs2, infos):
        spread = rel_l2(r2["y_u"], r["y_u"])
        err = rel_l2(y, r["y_u"])
        worst = max(worst, err / max(1e-10, 10 * spread))
        assert inf["flags"] == 0
    print("[gpu] bow fp64 0.1 s: worst error / bound %.3f" % worst, flush=True)
    assert worst <= 1.0


def test_bowed_fp32c_long_run_within_conditioning():
    """Over 1 s some bowed strings (chattering slip at strong force) are
    ill-conditioned: a change of f0, B, alpha or the bow position by 1e-7
    relative -- the rounding of the FP32 coefficients -- moves the oracle's own
    output by up to O(1).  FP32 compensated must stay within 1e-3 or within 3x
    that spread of the oracle, whichever is larger."""
    _gpu()
    items = W.bowed_batch(4096, seconds=1.0)
    pick = [22, 103, 123, 129, 158, 162, 188, 263]
    items = [items[i] for i in pick]
    refs = oracle.run_many(items)
    nudged = []
    for p, e in items:
        for key in ("f0", "B", "alpha"):
            nudged.append((dict(p, **{key: p[key] * (1 + 1e-7)}), e))
        nudged.append((p, dict(e, x=e["x"] * (1 + 1e-7))))
    print("[cpu] oracle: %d nudged runs of 1 s" % len(nudged), flush=True)
    spread_runs = oracle.run_many(nudged)
    outs, infos = _run(items, "fp32c")
    worst = 0.0
    for j, ((p, _), y, r, inf) in enumerate(zip(items, outs, refs, infos)):
        runs = [q["y_u"] for q in spread_runs[4 * j:4 * j + 4]]
        spread = max(rel_l2(q, r["y_u"]) for q in runs)
        err = rel_l2(y, r["y_u"])
        win = check_in_window(y, r["y_u"], runs)
        print("[gpu] bow fp32c 1 s: f0 %.1f rel-L2 %.2e, oracle spread %.2e, element-wise within 1e-3 over the "
              "first %d samples" % (p["f0"], err, spread, win), flush=True)
        assert win >= 480
        assert inf["flags"] == 0
        worst = max(worst, err / max(1e-3, 3 * spread))
    assert worst <= 1.0


def test_plain_fp64_bow_matches_oracle():
    """The plain FP64 comparator carries the bow's unit force through its
    band elimination as a second right-hand side."""
    _gpu()
    p, e = W.single_bowed(seconds=0.05)
    items = [(p, e), (p, dict(e, x_end=0.2))] + W.bowed_batch(3, seconds=0.05)
    refs = oracle.run_many(items)
    for (pp, ee), r in zip(items, refs):
        b = binding.StringBatch(1, "fp64_plain")
        b.set_params(0, [pp])
        b.excite(0, [ee])
        b.step(pp["n_samples"])
        y, inf = b.read_output(0), b.info(0)
        b.close()
        err = rel_l2(y, r["y_u"])
        print("[gpu] plain bow: N=(%d,%d) rel-L2 %.3e" % (inf["N_t"], inf["N_l"], err), flush=True)
        assert inf["flags"] == 0 and inf["samples_done"] == pp["n_samples"]
        assert err <= 1e-10
