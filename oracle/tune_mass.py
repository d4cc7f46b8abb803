"""Bare-mass tuning for the smooth-link solve workload, using the oracle only.

The workload asks for the mass at which the smallest singular value of the
mass-normalised operator D_m = D / (2 kappa), kappa = 1 / (2 (4 + m0)), on an
8^4 lattice of smooth links U = exp(0.3 i H) (H = sum_a h_a lambda_a / 2,
h_a ~ N(0, 1)), csw = 1, antiperiodic in time, is about 0.01.  sigma_min(m0)
has a single minimum near the critical mass; this script scans m0 on a
grid (three significant digits of sigma_min are enough to place the mass),
takes one parabolic-interpolation step through the three grid points around
the one closest to the target, and writes the better of the two (and the
attained value, which stays above 0.01 when the lowest momentum the volume
allows keeps the smallest singular value away from zero) to
tests/golden/smooth_links_mass.json.

    python -m oracle.tune_mass [--seed S] [--grid M0 M0 M0 ...] [--out PATH]
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
    ap.add_argument("--grid", type=float, nargs="+", default=[-0.2, -0.25, -0.3])
    a = ap.parse_args()
    U = synth.gauge_smooth(DIMS, a.seed)
    t0 = time.time()
    scan = {}
    for m0 in a.grid:
        scan[float(m0)] = sig(U, float(m0))
        print(f"m0 {m0:+.3f}  sigma_min {scan[float(m0)]:.5f}  ({time.time() - t0:.0f} s)", flush=True)
    f = lambda m: abs(scan[m] - TARGET)
    grid = sorted(scan)
    i = min(range(len(grid)), key=lambda k: f(grid[k]))
    m0, s = grid[i], scan[grid[i]]
    if 0 < i < len(grid) - 1:
        (x0, x1, x2), (y0, y1, y2) = grid[i - 1:i + 2], [f(g) for g in grid[i - 1:i + 2]]
        den = (x1 - x0) * (y1 - y2) - (x1 - x2) * (y1 - y0)
        if den != 0:
            xv = x1 - 0.5 * ((x1 - x0) ** 2 * (y1 - y2) - (x1 - x2) ** 2 * (y1 - y0)) / den
            if x0 < xv < x2:
                sv = sig(U, xv)
                print(f"m0 {xv:+.5f}  sigma_min {sv:.5f}  (vertex, {time.time() - t0:.0f} s)", flush=True)
                if abs(sv - TARGET) < f(m0):
                    m0, s = xv, sv
    res = {
        "lattice": list(DIMS),
        "links": "smooth, U = exp(0.3 i H), seed %d" % a.seed,
        "csw": CSW,
        "t_bc": -1,
        "target_sigma_min": TARGET,
        "m0": m0,
        "kappa": 1.0 / (2.0 * (4.0 + m0)),
        "sigma_min": s,
        "scan": {str(k): v for k, v in scan.items()},
        "written_by": "python -m oracle.tune_mass (oracle only)",
    }
    with open(a.out, "w") as fh:
        json.dump(res, fh, indent=1)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
