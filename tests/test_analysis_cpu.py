"""The spectral analyzer on signals with known content, and on the oracle's
strings: it must find f0 and B of an inharmonic tone and the phantom
partials of the nonlinear string, and none on the linear one."""
from __future__ import annotations

import numpy as np

import oracle
from paper_2311_18505_amd import analysis, workloads as W


def _tone(f0, B, fs, seconds, phantoms=()):
    t = np.arange(int(seconds * fs)) / fs
    y = np.zeros_like(t)
    for n in range(1, 13):
        fn = n * f0 * np.sqrt(1 + B * n * n)
        y += np.exp(-0.5 * n * t) * np.sin(2 * np.pi * fn * t + 0.3 * n) / n
    for (i, j), a in phantoms:
        fi, fj = (m * f0 * np.sqrt(1 + B * m * m) for m in (i, j))
        y += a * np.exp(-t) * np.sin(2 * np.pi * (fi + fj) * t)
    return y


def test_known_inharmonic_tone_and_phantoms():
    # B large enough that f_i + f_j sits well below f_{i+j} (by about
    # 1.5 f0 B i j (i+j)), so the phantoms are resolved from the partials
    fs, f0, B = 48000.0, 110.0, 5e-3
    y = _tone(f0, B, fs, 1.0, phantoms=[((2, 3), 3e-3), ((1, 5), 2e-3)])
    res = analysis.analyze(y, fs)
    assert abs(1200 * np.log2(res["f0"] / f0)) < 0.05
    assert abs(res["B"] / B - 1) < 0.02
    found = {ij for _, _, ij in res["phantoms"]}
    assert {(2, 3), (1, 5)} <= found
    plain = analysis.analyze(_tone(f0, B, fs, 1.0), fs)
    assert plain["phantoms"] == []


def test_nonlinear_string_shows_phantoms_and_linear_does_not():
    """Sec. 4's qualitative result: the coupled nonlinear string (alpha > 1)
    has partials at sums of transverse ones; the linear string has none."""
    fs = 48000.0
    p_nl = W.string(110.0, 2e-4, 3.0, 0.5, 1e-4, int(0.5 * fs))
    p_lin = dict(p_nl, alpha=1.0)
    e = W.pluck(0.13, 3e-3)
    y_nl = oracle.run(p_nl, e)["y_u"]
    y_lin = oracle.run(p_lin, e)["y_u"]
    a_nl = analysis.analyze(y_nl, fs)
    a_lin = analysis.analyze(y_lin, fs)
    assert abs(1200 * np.log2(a_lin["f0"] / 110.0)) < 5.0
    assert len(a_nl["phantoms"]) >= 1
    assert a_lin["phantoms"] == []


def test_command_line_reads_rows(tmp_path, capsys):
    import json
    fs = 48000.0
    rows = np.stack([_tone(110.0, 5e-3, fs, 1.0), _tone(220.0, 1e-3, fs, 1.0)])
    path = tmp_path / "audio.npy"
    np.save(path, rows)
    analysis.main([str(path), "--fs", "48000"])
    out = [json.loads(l) for l in capsys.readouterr().out.splitlines()]
    assert [o["row"] for o in out] == [0, 1]
    assert abs(1200 * np.log2(out[0]["f0"] / 110.0)) < 0.05
    assert abs(1200 * np.log2(out[1]["f0"] / 220.0)) < 0.05
