"""Bare-mass tuning for the smooth-link solve workload, using the oracle only.

The workload asks for the mass at which the smallest singular value of the
mass-normalised operator D_m = D / (2 kappa), kappa = 1 / (2 (4 + m0)), on an
8^4 lattice of smooth links U = exp(0.3 i H) (H = sum_a h_a lambda_a / 2,
h_a ~ N(0, 1)), csw = 1, is about 0.01.  With antiperiodic time the lowest
fermion momentum on 8^4 is pi / 8 and keeps sigma_min above 0.3 at every
mass, so the target is read with periodic time on the 8^4 lattice: there
the near-constant mode makes sigma_min(m0) close to |m0 - m_c| around the
critical mass m_c, and sigma_min = 0.01 on the heavy side of m_c means a
bare quark mass of about 0.01 above critical.  (The solve itself keeps the
antiperiodic time boundary on its 24^3 x 128 lattice.)

The script evaluates sigma_min on a grid of m0, takes the grid points above
the smallest value as the heavy side (where sigma_min rises linearly with
m0), predicts the m0 of sigma_min = 0.01 from the straight line through
the two heavy-side points nearest the minimum, and refines it by the secant
method on the heavy side until sigma_min is within 5 % of 0.01.  Evaluated
points can be kept in a JSON cache (--cache) so that an interrupted run
resumes.  The result goes to tests/golden/smooth_links_mass.json.

    python -m oracle.tune_mass [--seed S] [--grid M0 M0 ...] [--cache PATH] [--out PATH]
"""

from __future__ import annotations

import argparse
import json
import os
import time

from . import clover_packed, sigma_min

DIMS = (8, 8, 8, 8)
CSW = 1.0
TARGET = 0.01
T_BC = 1.0


def sig(U, m0):
    kappa = 1.0 / (2.0 * (4.0 + m0))
    A = clover_packed(U, DIMS, CSW, kappa)
    return float(sigma_min(U, A, kappa, DIMS, t_bc=T_BC, mass_form=True, inner_rtol=1e-9, tol=1e-4))


def main():
    import synth

    ap = argparse.ArgumentParser()
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--out", default=os.path.join(os.path.dirname(__file__), "..", "tests", "golden",
                                                  "smooth_links_mass.json"))
    ap.add_argument("--grid", type=float, nargs="+", default=[-0.2, -0.15, -0.1])
    ap.add_argument("--cache", default=None, help="JSON file of evaluated (m0, sigma_min) pairs, read and updated")
    a = ap.parse_args()
    U = synth.gauge_smooth(DIMS, a.seed)
    t0 = time.time()
    key = lambda m0: f"seed{a.seed}:{m0:+.6f}"
    cache = {}
    if a.cache and os.path.exists(a.cache):
        with open(a.cache) as fh:
            cache = json.load(fh)
    scan = {}

    def ev(m0):
        m0 = round(float(m0), 6)
        if m0 not in scan:
            if key(m0) in cache:
                scan[m0] = cache[key(m0)]
            else:
                scan[m0] = sig(U, m0)
                if a.cache:
                    cache[key(m0)] = scan[m0]
                    with open(a.cache, "w") as fh:
                        json.dump(cache, fh, indent=1)
            print(f"m0 {m0:+.5f}  sigma_min {scan[m0]:.5f}  ({time.time() - t0:.0f} s)", flush=True)
        return scan[m0]

    grid = sorted(float(g) for g in a.grid)
    vals = [ev(g) for g in grid]
    i = min(range(len(grid)), key=lambda k: vals[k])
    heavy = grid[i + 1:]
    if len(heavy) < 2:
        raise SystemExit("the grid needs two points above the one with the smallest sigma_min")
    (m1, m2) = heavy[:2]
    slope = (scan[m2] - scan[m1]) / (m2 - m1)
    mc = m1 - scan[m1] / slope  # where the heavy-side line reaches zero
    lo, hi = max(grid[i], mc), m1
    x = m1 + (TARGET - scan[m1]) / slope
    for _ in range(6):
        x = min(max(x, lo), hi) if x < m1 else x
        sx = ev(x)
        if abs(sx - TARGET) <= 0.05 * TARGET:
            break
        # secant through the two heavy-side points nearest the target
        pts = sorted((m for m in scan if m > mc), key=lambda m: abs(scan[m] - TARGET))[:2]
        (p1, p2) = pts
        x = p1 + (TARGET - scan[p1]) * (p2 - p1) / (scan[p2] - scan[p1])
    m0 = min((m for m in scan if m > mc), key=lambda m: abs(scan[m] - TARGET))
    s = scan[m0]
    res = {
        "lattice": list(DIMS),
        "links": "smooth, U = exp(0.3 i H), seed %d" % a.seed,
        "csw": CSW,
        "t_bc_for_sigma_min": int(T_BC),
        "target_sigma_min": TARGET,
        "m0": m0,
        "kappa": 1.0 / (2.0 * (4.0 + m0)),
        "sigma_min": s,
        "m_c_estimate": mc,
        "scan": {f"{k:+.5f}": v for k, v in sorted(scan.items())},
        "written_by": "python -m oracle.tune_mass (oracle only)",
    }
    with open(a.out, "w") as fh:
        json.dump(res, fh, indent=1)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
