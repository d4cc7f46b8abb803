"""Bare-mass tuning for the smooth-link solve workload, using the oracle only.

The workload asks for the mass at which the smallest singular value of the
mass-normalised operator D_m = D / (2 kappa), kappa = 1 / (2 (4 + m0)), on an
8^4 lattice of smooth links U = exp(0.3 i H) (H = sum_a h_a lambda_a / 2,
h_a ~ N(0, 1)), csw = 1, antiperiodic in time, is about 0.01.  sigma_min(m0)
has a single minimum near the critical mass; this script scans m0 (three
significant digits of sigma_min are enough to place the mass), then
minimises |sigma_min - 0.01| by golden-section search on the bracket around
the best scan point, and writes the result (and the attained value, which
may stay above 0.01 if the links are too smooth to produce such a small
singular value at this volume) to tests/golden/smooth_links_mass.json.

    python -m oracle.tune_mass [--seed S] [--out PATH]
"""

from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

from . import clover_packed, sigma_min

DIMS = (8, 8, 8, 8)
CSW = 1.0
TARGET = 0.01


def sig(U, m0):
    kappa = 1.0 / (2.0 * (4.0 + m0))
    A = clover_packed(U, DIMS, CSW, kappa)
    return float(sigma_min(U, A, kappa, DIMS, t_bc=-1.0, mass_form=True, inner_rtol=1e-8, tol=1e-3))


def main():
    import synth

    ap = argparse.ArgumentParser()
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--out", default=os.path.join(os.path.dirname(__file__), "..", "tests", "golden",
                                                  "smooth_links_mass.json"))
    a = ap.parse_args()
    U = synth.gauge_smooth(DIMS, a.seed)
    t0 = time.time()
    scan = {}
    for m0 in (0.0, -0.1, -0.2, -0.25, -0.3, -0.35, -0.4):
        scan[float(m0)] = sig(U, float(m0))
        print(f"m0 {m0:+.3f}  sigma_min {scan[float(m0)]:.5f}  ({time.time() - t0:.0f} s)", flush=True)
    f = lambda m: abs(sig(U, m) - TARGET)
    best = min(scan, key=lambda m: abs(scan[m] - TARGET))
    lo, hi = best - 0.05, best + 0.05
    gr = (np.sqrt(5) - 1) / 2
    c, d = hi - gr * (hi - lo), lo + gr * (hi - lo)
    fc, fd = f(c), f(d)
    for _ in range(8):
        if fc < fd:
            hi, d, fd = d, c, fc
            c = hi - gr * (hi - lo)
            fc = f(c)
        else:
            lo, c, fc = c, d, fd
            d = lo + gr * (hi - lo)
            fd = f(d)
        print(f"bracket [{lo:+.5f}, {hi:+.5f}]  ({time.time() - t0:.0f} s)", flush=True)
    m0 = 0.5 * (lo + hi)
    s = sig(U, m0)
    res = {
        "lattice": list(DIMS),
        "links": "smooth, U = exp(0.3 i H), seed %d" % a.seed,
        "csw": CSW,
        "t_bc": -1,
        "target_sigma_min": TARGET,
        "m0": m0,
        "kappa": 1.0 / (2.0 * (4.0 + m0)),
        "sigma_min": s,
        "scan": scan,
        "written_by": "python -m oracle.tune_mass (oracle only)",
    }
    with open(a.out, "w") as fh:
        json.dump(res, fh, indent=1)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
