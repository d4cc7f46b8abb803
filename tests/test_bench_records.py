"""The benchmark's stored HBM-traffic record matches what it describes.

`bench.py` reports `roofline.traffic` (the dominant fine kernel's counted
bytes per launch) only while the kernel's sources and its launch
configurations are the ones the counters were taken with.  These CPU checks
keep the record, the committed autotuner cache and the kernel sources in
step, so that a change to any of them shows here rather than as a missing
traffic figure.
"""

import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _cached_configs(dims):
    """{nrhs: [R, tile, variant]} of the committed cache for one lattice, in the
    form bench.py builds from mrhs_get_tuning."""
    out = {}
    with open(bench.TUNE_CACHE) as fh:
        for line in fh:
            f = line.split()
            if len(f) != 18 or tuple(int(v) for v in f[2:6]) != tuple(dims):
                continue
            n, R = int(f[6]), int(f[7])
            tile = [int(v) for v in f[8:12]]
            curve, occ, nt, chunks, cap = (int(v) for v in f[12:17])
            walk = curve == 2
            variant = ((0 if walk else curve) + 2 * (occ == 4) + 4 * nt
                       + 8 * {1: 0, 2: 1, 4: 2}[chunks] + 32 * cap + 128 * walk)
            out[str(n)] = [R, tile, variant]
    return out


def test_traffic_record_matches_sources():
    assert bench.FINE_TRAFFIC["sources"] == bench.fine_sources_digest()


def test_traffic_record_matches_cached_configurations():
    cached = _cached_configs(bench.DIMS)
    rec = bench.FINE_TRAFFIC["configs"]
    assert rec, "empty record"
    for n, cfg in rec.items():
        assert cached.get(n) == cfg, (n, cached.get(n), cfg)


def test_dominant_kernel_name_matches_the_walk_instance():
    # the record names the t-walk kernel with two RHS per thread and the
    # compiler's register budget, the instance every recorded Nrhs uses
    assert bench.FINE_TRAFFIC["kernel"] == "fine_walk_kernel<2, 0, false>"
    for cfg in bench.FINE_TRAFFIC["configs"].values():
        assert cfg[0] == 2 and cfg[2] & 128 and not cfg[2] & 2
