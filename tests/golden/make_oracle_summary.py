"""Writes oracle_c1_summary.json: a text summary of the FP64 oracle on the
small plain workload (128^2 object, 169 frames of 32^2, noiseless, known
probe, beta 0.75, 10 RAAR iterations).  Calls only oracle/ and the seeded
input recipes; run from the repository root:
    python tests/golden/make_oracle_summary.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from sharp_data import gen  # noqa: E402


def summary():
    s = gen.config_scan(1)
    I = O.forward_intensity(s.obj, s.probe, s.positions).astype(np.float32).astype(np.float64)
    r = O.raar(I, s.positions, (s.n, s.n), s.m, 10, s.beta, psi0=s.psi0, w0=s.probe)
    D = O.illumination_density(s.probe, s.positions, (s.n, s.n))
    psi = r["psi"]
    probes = [(0, 0), (17, 93), (64, 64), (100, 5), (127, 127)]
    return {
        "_about": "FP64 oracle, plain workload 128^2 / 169 x 32^2, known probe, beta 0.75, 10 iterations, "
                  "intensities rounded to float32 first (as the GPU consumes them). Written by make_oracle_summary.py.",
        "eps_a": [float(x) for x in r["eps_a"]],
        "dweighted_norm_psi": float(np.linalg.norm(D * psi)),
        "psi_samples": {f"{y},{x}": [float(psi[y, x].real), float(psi[y, x].imag)] for y, x in probes},
    }


if __name__ == "__main__":
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_c1_summary.json")
    with open(out, "w") as f:
        json.dump(summary(), f, indent=1)
    print("wrote", out)
