"""Writes paper_constants.json: values obtained by evaluating formulas printed
in the paper (arXiv 2311.18505), each with the passage it comes from.  Uses no
project code."""
import json
import math
import os

out = {}
# Sec. 3.2: theta = (1 + 4/pi^2)/2
out["theta"] = {"value": 0.5 * (1 + 4 / math.pi ** 2), "source": "Sec. 3.2, theta-scheme parameter"}


def h_t(gamma, kappa, k):
    # Sec. 3.2, printed transverse spacing
    return math.sqrt((gamma ** 2 * k ** 2 + math.sqrt(gamma ** 4 * k ** 4 + 16 * kappa ** 2 * k ** 2)) / 2)


cases = []
for fs, f0, B in [(48000.0, 110.0, 1e-4), (48000.0, 82.4, 2e-4), (44100.0, 300.0, 1e-3), (96000.0, 55.0, 3e-5)]:
    gamma = 2 * f0                                   # Sec. 4.1: f0 = gamma / 2
    kappa = gamma * math.sqrt(B) / math.pi           # Sec. 4.1: K = (pi kappa / gamma)^2
    cases.append({"fs": fs, "f0": f0, "B": B, "N_t": int(math.floor(1 / h_t(gamma, kappa, 1 / fs)))})
out["h_t_theta1"] = {"cases": cases, "source": "Sec. 3.2 spacing h^(t); N_t = floor(1/h^(t))"}
out["kappa_config1"] = {"value": 220.0 * math.sqrt(1e-4) / math.pi,
                        "source": "Sec. 4.1, K = (pi kappa/gamma)^2 with gamma = 2 f0, f0 = 110 Hz, K = 1e-4"}
out["fig2"] = {"f0": 300.0, "alpha": 3.0, "x_P": 0.14, "a": {"kappa": 6.08, "c0": 0.0078},
               "b": {"kappa": 9.63, "c0": 0.0085}, "source": "Sec. 4.2 and the caption of Fig. 2"}
out["phi2"] = {"formula": "gamma^2 k^2 (alpha^2 - 1) / 4", "source": "remark after eq. (9)"}
with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_constants.json"), "w") as fh:
    json.dump(out, fh, indent=1)
