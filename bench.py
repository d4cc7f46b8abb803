#!/usr/bin/env python3
"""Benchmark of the MRHS Wilson-clover hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--nrhs 1,6,12,24,48,64]

Workload: the fine Wilson-clover operator D = A - kappa H on a 24^4 lattice,
antiperiodic in time, Haar-random SU(3) links (seeded), clover term built on
the GPU with csw = 1.0, kappa = 0.13, Gaussian sources seeded per RHS, FP32,
fields laid out [site][12][Nrhs].  One step applies D once for every Nrhs in
the sweep.  The timed region holds exactly K steps with inputs resident in
device memory; it is bracketed by device synchronisation.

Reported (one JSON line on stdout):
  value       aggregate GFLOP/s over the sweep (1920 flops per site per RHS)
  per_nrhs    per-Nrhs time, GFLOP/s, algorithmic GB/s and roofline fraction,
              back-to-back ("warm"); with --cold-reps also after a 1 GiB
              cache-evicting write ("cold")
  roofline    for the dominant kernel (the R=4 instantiation used for Nrhs >= 12):
              algorithmic bytes per launch / mean launch time from HIP events
  cpu_baseline  the FP64 CPU oracle on a bounded sample of the same workload
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

DIMS = (24, 24, 24, 24)
KAPPA, CSW = 0.13, 1.0
FLOPS_PER_SITE_RHS = 1920          # hop 1320 + clover 552 + combine 48
HBM_PEAK_GBS = 8000.0              # MI355X HBM3E, published
NRHS_DEFAULT = (1, 6, 12, 24, 48, 64)


def alg_bytes(V: int, nrhs: int) -> int:
    """Algorithmic HBM bytes of one FP32 apply: links 288 + clover 288 + in/out 2*96*N per site."""
    return V * (288 + 288 + 192 * nrhs)


def kernel_name(nrhs: int) -> str:
    if nrhs % 4 == 0 and nrhs >= 8:
        r = 4
    elif nrhs % 2 == 0:
        r = 2
    else:
        r = 1
    return f"fine_kernel<float, {r}, 0, true>"


def cpu_baseline(dims, nrhs_sample: int = 2):
    """The FP64 oracle's D apply on the full 24^4 lattice for a few RHS."""
    import oracle as O
    import synth

    try:
        from threadpoolctl import threadpool_info

        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = 1
    U = synth.gauge_haar(dims, 1)
    A = O.clover_packed_direct(U, dims, CSW, KAPPA)
    psi = synth.spinor_source(dims, nrhs_sample, 100)
    t0 = time.perf_counter()
    O.dwc(U, A, KAPPA, psi, dims)
    dt = time.perf_counter() - t0
    V = int(np.prod(dims))
    return {
        "value": FLOPS_PER_SITE_RHS * V * nrhs_sample / dt / 1e9,
        "unit": "GFLOP/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"one FP64 D apply, 24^4, Nrhs={nrhs_sample} ({dt:.1f} s; numpy einsum, single-threaded;"
        f" BLAS pool {threads} threads unused by this path)",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--nrhs", type=str, default=",".join(map(str, NRHS_DEFAULT)))
    ap.add_argument("--cold-reps", type=int, default=0,
                    help="also time each apply after a 1 GiB cache-evicting write (0 = skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run a 1 GiB device-to-device copy first (reference for HBM byte counters)")
    a = ap.parse_args()

    if a.gpus != 1:
        print(
            f"bench.py measures one GPU only; --gpus {a.gpus} is not supported "
            "(the multi-GPU domain decomposition is not part of this build)",
            file=sys.stderr,
        )
        sys.exit(2)

    import torch

    import paper_2211_13719_amd as mrhs
    import synth

    nrhs_list = [int(x) for x in a.nrhs.split(",") if x]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    V = int(np.prod(DIMS))

    if a.calib_copy:
        src_c = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst_c = torch.empty_like(src_c)
        for _ in range(3):
            dst_c.copy_(src_c)
        torch.cuda.synchronize()
        del src_c, dst_c

    t_setup = time.perf_counter()
    U = synth.gauge_haar(DIMS, 1)
    ctx = mrhs.Context(DIMS, t_bc=-1, stream=stream)
    ctx.set_gauge(U)
    ctx.build_clover(CSW, KAPPA)
    nmax = max(nrhs_list)
    src = synth.spinor_source(DIMS, nmax, 100, np.complex64)
    fields = {}
    for n in nrhs_list:
        x = torch.from_numpy(np.ascontiguousarray(src[:, :, :n])).to(dev)
        fields[n] = (x, torch.empty_like(x))
    del src
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t_setup
    print(f"[bench] setup {setup_s:.1f} s, sweep {nrhs_list}", file=sys.stderr, flush=True)

    def step(events=None):
        for n in nrhs_list:
            x, y = fields[n]
            if events is not None:
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                ctx.dwc(y, x)
                e1.record(stream)
                events.append((n, e0, e1))
            else:
                ctx.dwc(y, x)

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()

    # ---- timed region: exactly K steps --------------------------------------------
    events = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        step(events)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    print(f"[bench] timed {a.steps} steps in {wall:.3f} s", file=sys.stderr, flush=True)

    per = {}
    for n in nrhs_list:
        ts = [e0.elapsed_time(e1) for (m, e0, e1) in events if m == n]
        per[n] = {"warm_ms": float(np.median(ts)), "warm_mean_ms": float(np.mean(ts))}

    # ---- cold: evict the 256 MB last-level cache before every apply -------------------
    flush = torch.empty(1 << 28, dtype=torch.float32, device=dev) if a.cold_reps else None  # 1 GiB
    for n in (nrhs_list if a.cold_reps else []):
        x, y = fields[n]
        ts = []
        for _ in range(a.cold_reps):
            flush.fill_(1.0)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            ctx.dwc(y, x)
            e1.record(stream)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        per[n]["cold_ms"] = float(np.median(ts))
    del flush

    for n in nrhs_list:
        b = alg_bytes(V, n)
        f = FLOPS_PER_SITE_RHS * V * n
        for tag in ("warm", "cold") if a.cold_reps else ("warm",):
            ms = per[n][f"{tag}_ms"]
            per[n][f"{tag}_gflops"] = f / ms / 1e6
            per[n][f"{tag}_gbs"] = b / ms / 1e6
            per[n][f"{tag}_hbm_frac"] = b / ms / 1e6 / HBM_PEAK_GBS
        per[n]["kernel"] = kernel_name(n)
        per[n]["srhs_speedup"] = None

    if 1 in per:
        for n in nrhs_list:
            per[n]["srhs_speedup"] = n * per[1]["warm_ms"] / per[n]["warm_ms"]

    # dominant kernel: the instantiation with the largest share of the step
    share = {}
    for n in nrhs_list:
        share.setdefault(kernel_name(n), []).append(n)
    dom = max(share, key=lambda k: sum(per[n]["warm_mean_ms"] for n in share[k]))
    launches = [(m, e0.elapsed_time(e1)) for (m, e0, e1) in events if kernel_name(m) == dom]
    mean_bytes = float(np.mean([alg_bytes(V, m) for m, _ in launches]))
    mean_ms = float(np.mean([t for _, t in launches]))
    achieved = mean_bytes / mean_ms / 1e6

    total_flops = sum(FLOPS_PER_SITE_RHS * V * n for n in nrhs_list)
    ms_per_step = wall * 1e3 / a.steps
    value = total_flops / (ms_per_step * 1e-3) / 1e9

    result = {
        "metric": "MRHS Dslash GFLOP/s vs Nrhs (fine Wilson-clover D_wc, FP32)",
        "value": round(value, 1),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "fine MRHS Wilson-clover D_wc+clover, 24^4, FP32, Haar SU(3) links, csw=1.0, kappa=0.13, "
            "antiperiodic t, Gaussian sources; one step = one apply per Nrhs in the sweep",
            "lattice": list(DIMS),
            "nrhs": nrhs_list,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": dom,
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None,
            "mean_alg_bytes_per_launch": mean_bytes,
            "mean_launch_ms": mean_ms,
            "launches_per_step": len(share[dom]),
        },
        "per_nrhs": {str(n): {k: (round(v, 4) if isinstance(v, float) else v) for k, v in per[n].items()}
                     for n in nrhs_list},
        "cpu_baseline": None,
    }
    if not a.no_cpu_baseline:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(DIMS)
    print(json.dumps(result), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
