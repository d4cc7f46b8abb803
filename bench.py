#!/usr/bin/env python3
"""Benchmark of the MRHS Wilson-clover multigrid hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-solve] [--no-cpu-baseline]
                    [--tune-cache PATH | --retune] [--solve-nrhs 12,24,48,64] [--m0 M]

One step is one pass over every operator of the hot path, each on its
workload shape (inputs resident in device memory, all synthetic and seeded):

  fine D_wc      24^4, FP32, Haar SU(3) links, csw 1.0, kappa 0.13, antiperiodic t,
                 Gaussian sources; one apply for each Nrhs in 1, 6, 12, 24, 48, 64;
                 the FP64 operator (the outer solver's residuals) at Nrhs 1, 12, 48
  coarse D_c     Galerkin blocks of that operator (16 Gaussian vectors per step,
                 FP64 block-orthonormalised, 4^4 then 2^4 aggregates): 6^4 and 3^4
                 coarse lattices, Nb = 32, Nrhs in 12, 24, 48, 64; FP32 vector ALU
                 and BF16 / FP16 matrix cores
  intergrid      restrict, prolong (FP32 vector ALU and BF16 matrix cores), block-normalise
                 24^4 <-> 6^4 at Nrhs = 24, FP32 fields
  reductions     dot and norm of 24^4 fields at Nrhs = 24, FP64 sums

The timed region holds exactly K steps, bracketed by device synchronisation.
`value` is the FP32 fine D_wc rate (algorithmic GFLOP/s of its six applies
over their summed median times; `value_by_nrhs` per Nrhs); the whole step's
mixed-precision rate is `composite_step`.  `per_op` gives per-operator times,
GFLOP/s and algorithmic GB/s from HIP events on the stream the kernels run
on, warm (back to back) and cold (after a 1 GiB device copy that flushes the
caches); `roofline` is for the dominant kernel.  After the timed region (not part of `value`), `solve` times the
mixed-precision MG solve (FP64 FGMRES, FP32 fine level, BF16 coarse levels
and intergrid, graph-replayed V-cycle) on 24^3 x 128 smooth links at the bare
mass stored in tests/golden/smooth_links_mass.json, for batches of 12, 24, 48
and 64 RHS (FGMRES(5), or the longest restart whose fields fit in the free HBM),
and the same solver on one RHS with FP32 coarse levels, in seconds per RHS to
a true residual of 1e-10.  `cpu_baseline` times the FP64 CPU oracle on
the host's cores (a process pool over right-hand sides) on bounded samples
of the same workloads, before anything touches the GPU.

Fine-kernel launch configurations come from the autotuner's text cache
(paper_2211_13719_amd/tuning/fine.txt, tuned on an MI355X); lattices or Nrhs
missing there are tuned on the spot and appended, and --retune ignores it.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DIMS = (24, 24, 24, 24)
KAPPA, CSW = 0.13, 1.0
NRHS_FINE = (1, 6, 12, 24, 48, 64)
NRHS_F64 = (1, 12, 48)  # the FP64 operator of the outer solver's residuals, in the step beside the FP32 one
NRHS_COARSE = (12, 24, 48, 64)
N_INTER = 24
NB = 32
HBM_PEAK_GBS = 8000.0

FLOPS_DWC = 1920          # per site per RHS: hop 1320 + clover 552 + combine 48
SOLVE_DIMS = (24, 24, 24, 128)
# multigrid set-up and V-cycle of the solve workload (hyper-parameters, not from the paper)
# 15 set-up sweeps instead of 10: 21 instead of 23 outer steps at 12 RHS (0.98 vs 1.08 s), 0.32 vs 0.36 s on
# one RHS, for about 1 s more set-up; 20 sweeps or 50 MR steps per sweep gain nothing further
SOLVE_SETUP = dict(setup_iters=15, smooth_steps=30, adapt_iters=0)
# 24^3x128, 12 RHS, even-odd fine smoother: nu_post 4 with 128 coarsest steps 1.09 s (23 outer steps),
# nu_post 6 with 64 steps 1.31 s (24); on one RHS 4 / 128 is the fastest setting measured too (0.367 s)
SOLVE_VC = dict(nu_pre=0, nu_post=4, coarsest_iters=128)
# FGMRES restart length with the FP32 basis, 24^3x128 (seconds, 18 outer steps at every m): 12 RHS m = 4 / 5 / 6 /
# 8 / 10: 0.700 / 0.689 / 0.694 / 0.710 / 0.711; 48 RHS m = 4 / 5 / 6 / 7: 2.122 / 2.102 / 2.112 / 2.124
SOLVE_RESTART, SOLVE_MAXIT = 5, 1000
SOLVE_MRHS_FINE_EO = True  # 24^3x128, 12 / 24 RHS, nu_post 6: 24 instead of 28 outer steps, 10-13 % less time
# level-1 (6^3 x 32) smoothing on the coarse even-odd Schur complement: 24^3x128, 12 RHS, 18 instead of 21 outer
# steps, 0.90 vs 1.03 s
SOLVE_MRHS_COARSE_EO = True
# Schwarz (SAP) smoothing of the fine level, measured beside the even-odd smoother: cycles per smoothing pass and
# MR steps per 4^4 block solve
SOLVE_SAP_CYCLES, SOLVE_SAP_ITERS = 1, 4
# outer Krylov basis in FP32 between FP64 restarts (FP64 true residual and solution): half the outer solver's
# memory traffic; the FP64 basis is timed beside it on the first batch size
SOLVE_KRYLOV_F32 = True
TUNE_CACHE = os.path.join(HERE, "paper_2211_13719_amd", "tuning", "fine.txt")
FINE_SOURCES = ("fine.hip", "internal.h", "api.hip")

# HBM traffic of the dominant fine kernel per launch (bytes; rocprofv3
# FETCH_SIZE + WRITE_SIZE per dispatch, each scaled by what the counter reads
# for a 1 GiB device copy), recorded with a digest of the kernel's sources and
# the launch configurations it was counted under.  `roofline.traffic` carries
# it only while the kernel name, sources and configurations still match.
FINE_TRAFFIC = {
    "kernel": "fine_walk_kernel<2, 0, false>",
    "sources": "2bd0a9649f6a2c6c",
    "configs": {"6": [2, [4, 4, 4, 3], 224], "12": [2, [24, 8, 2, 3], 224], "24": [2, [24, 8, 2, 3], 132],
                "48": [2, [24, 4, 4, 3], 132], "64": [2, [6, 6, 6, 12], 132]},
    "bytes_per_launch": 5.250e9,
    "note": "2.0 x FETCH_SIZE + 1.0 x WRITE_SIZE per dispatch (copy-calibrated), mean over Nrhs 6, 12, 24, 48, 64; "
            "profiles/fine_kernel_hbm_counters_24x24x24x24.md",
}



def fine_sources_digest():
    h = hashlib.sha256()
    for f in FINE_SOURCES:
        with open(os.path.join(HERE, "paper_2211_13719_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def fine_bytes(V, n):
    return V * (288 + 288 + 192 * n)


def coarse_bytes(V, n, prec):
    blk = 9 * NB * NB * (4 if prec in ("bf16", "f16") else 8)
    return V * (blk + NB * n * 16)


def coarse_flops(V, n):
    return 8 * 9 * NB * NB * V * n


def fine_kernel_name(ctx, n):
    """Template instance of the FP32 fine kernel the tuned configuration of n uses."""
    R, _, variant, _ = ctx.get_tuning(n)
    R = R or (2 if n % 2 == 0 else 1)
    occ = 4 if variant & 2 else 0
    if variant & 128:  # the t-walk kernel
        return f"fine_walk_kernel<{R}, {occ}, false>"  # false: D itself, not the fused residual
    return f"fine_kernel<float, {R}, 0, true, true, {occ}, HIP_vector_type<float, 2u> >"


# Inputs of the oracle timing, set in the parent before the worker pool forks
# (the workers read them through copy-on-write memory, nothing is pickled).
_CPU = {}


def _cpu_task(task):
    """One worker's share of an oracle timing: the oracle on a slice of the
    right-hand sides, numpy on one thread.  Returns a checksum (the results
    stay in the worker)."""
    import oracle as O
    from threadpoolctl import threadpool_limits

    kind, k0, k1 = task
    c = _CPU
    with threadpool_limits(limits=1):
        if kind == "dwc":
            r = O.dwc(c["U"], c["A"], KAPPA, c["psi"][:, :, k0:k1], DIMS)
        elif kind == "coarse":
            r = O.coarse_apply(c["B"], c["e"][:, :, k0:k1], (6, 6, 6, 6))
        elif kind == "restrict":
            r = O.restrict(c["W"], c["psi"][:, :, k0:k1], DIMS, (4, 4, 4, 4))
        elif kind == "dot":
            r = O.dot(c["f"][:, :, k0:k1], c["g"][:, :, k0:k1])
        else:  # "solve": the oracle's own FP64 GMRES solve on 8^4
            r = O.solve_ref(c["U8"], c["A8"], KAPPA, c["b8"][:, :, k0:k1], (8, 8, 8, 8))
    return float(np.abs(r).sum())


def fabric_probe():
    """Read bandwidth of device buffers by size (mrhs_read_probe: 2048
    workgroups of 256 threads, grid-stride 16-byte reads, so that each XCD's
    workgroups cover an eighth of the buffer): 16 MiB fits the L2s (4 MiB per
    XCD), 64 and 128 MiB the 256 MiB Infinity Cache but not the L2s, 2 GiB
    neither.  Depth 1 (one load in flight per thread) against depth 8 tells a
    latency-bound rate from a bandwidth-bound one."""
    import torch

    import paper_2211_13719_amd as mrhs

    ctx = mrhs.Context((2, 2, 2, 2), t_bc=-1)
    out = {}
    for depth in (1, 4, 8):
        row = {}
        for mib in (16, 64, 128, 192, 512, 2048):
            x = torch.ones(mib << 18, dtype=torch.float32, device="cuda")
            sweeps = max(2, (8 << 30) // (mib << 20))
            ms = ctx.read_probe(x, sweeps, 2048, depth)
            row[f"{mib}MiB"] = round((mib << 20) * sweeps / ms / 1e6, 1)
            del x
        out[f"depth{depth}"] = row
    ctx.close()
    return {"read_GBps_by_depth_and_buffer_size": out, "method": "mrhs_read_probe, 2048 workgroups of 256 threads"}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline():
    """The FP64 oracle, as written (numpy, one thread per process), timed on the
    host's cores with a process pool over right-hand sides (they are
    independent), on a bounded sample of each workload:

      dwc       24^4 D_wc (Haar links, csw 1.0, kappa 0.13), 8 RHS per worker
      coarse    6^4 coarse stencil, Nb 32 (Gaussian + 4 I blocks: the cost does
                not depend on the values), 24 RHS per worker
      restrict  24^4 -> 6^4, 16 basis vectors (Gaussian: value-independent cost), 8 RHS per worker
      dot       24^4 fields, 24 RHS per worker
      solve     the oracle's FP64 GMRES solve on 8^4 Haar links, 1 RHS per worker

    Runs before anything touches the GPU, so the forked workers hold no GPU
    state.  `value` is the D_wc rate in the metric's unit."""
    import multiprocessing as mp

    import oracle as O
    import synth

    cores = max(1, min(len(os.sched_getaffinity(0)), 16))
    V = int(np.prod(DIMS))
    t_in = time.perf_counter()
    U = synth.gauge_haar(DIMS, 1)
    _CPU.update(U=U, A=O.clover_packed_direct(U, DIMS, CSW, KAPPA),
                psi=synth.spinor_source(DIMS, 8, 100),
                B=synth.gaussian_blocks(6**4, NB, 3),
                e=synth.coarse_source(6**4, NB, 24, 4),
                W=synth.gaussian_vectors(V, 16, 12, 300),
                f=synth.spinor_source(DIMS, 24, 5), g=synth.spinor_source(DIMS, 24, 6))
    d8 = (8, 8, 8, 8)
    U8 = synth.gauge_haar(d8, 1)
    _CPU.update(U8=U8, A8=O.clover_packed(U8, d8, CSW, KAPPA), b8=synth.spinor_source(d8, 1, 9000))
    t_in = time.perf_counter() - t_in
    # (kind, RHS per worker, flops per RHS or None, unit)
    plan = [("dwc", 8, FLOPS_DWC * V, "GFLOP/s"), ("coarse", 24, 8 * 9 * NB * NB * 6**4, "GFLOP/s"),
            ("restrict", 8, 8 * 6 * 2 * 16 * V, "GFLOP/s"), ("dot", 24, 8 * 12 * V, "GFLOP/s"),
            ("solve", 1, None, "s/RHS")]
    per_op = {}
    with mp.get_context("fork").Pool(cores) as pool:
        pool.map(_cpu_task, [("dot", 0, 1)] * cores)  # start the workers
        for kind, per, flops, unit in plan:
            # every worker applies the oracle to the same `per` right-hand sides
            # (the cost does not depend on the values; shared inputs keep the
            # host memory of the sample small)
            tasks = [(kind, 0, per)] * cores
            nrhs = per * cores
            t0 = time.perf_counter()
            pool.map(_cpu_task, tasks, chunksize=1)
            dt = time.perf_counter() - t0
            # rate of the whole pool: flops over wall time, or wall seconds per RHS solved
            val = flops * nrhs / dt / 1e9 if flops else dt / nrhs
            per_op[kind] = {"value": round(val, 4), "unit": unit, "nrhs": nrhs, "wall_s": round(dt, 3),
                            "workers": len(tasks)}
    _CPU.clear()
    return {
        "value": per_op["dwc"]["value"],
        "unit": "GFLOP/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"FP64 oracle D_wc on 24^4 (Haar links, csw 1.0, kappa 0.13), {per_op['dwc']['nrhs']} RHS, "
                  f"a pool of {cores} single-threaded numpy processes with 8 RHS each "
                  f"({per_op['dwc']['wall_s']:.1f} s wall); other ops in per_op",
        "nproc": os.cpu_count(),
        "cpu_model": cpu_model(),
        "input_generation_s": round(t_in, 1),
        "per_op": per_op,
    }


class Timer:
    def __init__(self, torch, stream):
        self.torch, self.stream, self.ev = torch, stream, []

    def __call__(self, key, fn):
        e0 = self.torch.cuda.Event(enable_timing=True)
        e1 = self.torch.cuda.Event(enable_timing=True)
        e0.record(self.stream)
        fn()
        e1.record(self.stream)
        self.ev.append((key, e0, e1))

    def times(self):
        out = {}
        for key, e0, e1 in self.ev:
            out.setdefault(key, []).append(e0.elapsed_time(e1))
        return out


def bench_evenodd(ctx, mg, torch, stream, fine, coarse, V, warmup, steps):
    """The checkerboarded pieces, outside the step: on the 24^4 lattice in FP32,
    M_eooe (hop between the parities), M_ooee and its inverse on one parity, per
    Nrhs, with the MRHS speedup N t(1) / t(N); on the 6^4 coarse level (Nb 32)
    the coarse M_eooe (eight hop directions into one parity) in FP32 and BF16
    and the inverse self blocks.  Bytes and flops per output site: M_eooe 576 +
    192 N bytes (all eight links of the site, in and out rows) and 1320 N
    flops; M_ooee 288 + 192 N bytes and 552 N flops; coarse M_eooe 8 Nb^2
    block entries (8 or 4 bytes) + 16 Nb N bytes and 64 Nb^2 N flops; inverse
    self blocks Nb^2 entries + 16 Nb N bytes and 8 Nb^2 N flops."""
    nh = V // 2
    ops = []
    vch = mg.volume[1] // 2
    for n in sorted(n for (lev, n) in coarse if lev == 1):
        e, o = coarse[(1, n)][0][:vch], coarse[(1, n)][1][:vch]
        for prec, bs in (("f32", 8), ("bf16", 4)):
            ops.append(((f"coarse_meooe_{prec}", n), 64 * NB * NB * vch * n, vch * (8 * NB * NB * bs + 16 * NB * n),
                        lambda e=e, o=o, p=prec: mg.coarse_hop_eo(1, o, e, 0, prec=p)))
        ops.append((("coarse_sinv_bf16", n), 8 * NB * NB * vch * n, vch * (NB * NB * 4 + 16 * NB * n),
                    lambda e=e, o=o: mg.coarse_self_eo(1, o, e, 1, inverse=True, prec="bf16")))
    for n in sorted(fine):
        x, y = fine[n][0][:nh], fine[n][1][:nh]
        ops.append((("meooe", n), 1320 * nh * n, nh * (576 + 192 * n), lambda x=x, y=y: ctx.hop_eo(y, x, 0)))
        ops.append((("mooee", n), 552 * nh * n, nh * (288 + 192 * n), lambda x=x, y=y: ctx.clover_eo(y, x, 1)))
        ops.append((("mooee_inv", n), 552 * nh * n, nh * (288 + 192 * n),
                    lambda x=x, y=y: ctx.clover_eo(y, x, 1, inverse=True)))
    for _ in range(max(warmup, 1)):
        for _, _, _, fn in ops:
            fn()
    torch.cuda.synchronize()
    timer = Timer(torch, stream)
    for _ in range(steps):
        for key, _, _, fn in ops:
            timer(key, fn)
    torch.cuda.synchronize()
    times = timer.times()
    out = {}
    for key, flops, nbytes, _ in ops:
        ms = float(np.median(times[key]))
        out[f"{key[0]}@{key[1]}"] = {
            "ms": round(ms, 5),
            "gflops": round(flops / ms / 1e6, 1),
            "alg_gbs": round(nbytes / ms / 1e6, 1),
            "hbm_frac": round(nbytes / ms / 1e6 / HBM_PEAK_GBS, 4),
        }
    for kind in ("meooe", "mooee", "mooee_inv"):  # the coarse ops start at Nrhs 12: no t(1)
        if (kind, 1) in times:
            t1 = float(np.median(times[(kind, 1)]))
            for n in sorted(fine):
                out[f"{kind}@{n}"]["mrhs_speedup"] = round(n * t1 / float(np.median(times[(kind, n)])), 3)
    return out


def solve_restart(elems, free_bytes, krylov_f32=SOLVE_KRYLOV_F32, reserve=4 << 30):
    """FGMRES restart length for a batch whose fine fields hold `elems` complex numbers
    (V x 12 x Nrhs): the largest m <= SOLVE_RESTART whose solver fields fit in the device
    memory left after the set-up, less a reserve.  Per complex element: m + 1 basis vectors
    (FP64, or FP32 with an FP32 work field beside them), m FP32 preconditioned directions,
    one FP64 work field, the caller's FP64 x and b, four FP32 V-cycle fields of the fine
    level and five half-lattice FP32 fields of the even-odd smoother (2.5 full ones)."""
    for m in range(SOLVE_RESTART, 1, -1):
        basis = 8 * (m + 1) + 8 if krylov_f32 else 16 * (m + 1)
        per = basis + 8 * m + 16 + 2 * 16 + 4 * 8 + 20
        if elems * per <= free_bytes - reserve:
            return m
    return 2


def run_solve(mrhs, torch, synth, nrhs_list, mass, cache):
    """MRHS mixed-precision solves (one per batch size) vs the same solver on one RHS
    with FP32 coarse levels and FP32 intergrid."""
    kappa = mass["kappa"]
    U = synth.gauge_smooth(SOLVE_DIMS, 5)
    ctx = mrhs.Context(SOLVE_DIMS, t_bc=-1)
    ctx.set_gauge(U)
    del U
    ctx.build_clover(CSW, kappa)
    ctx.tune(sorted({1, 16, *nrhs_list}), cache)
    eo_hop = {str(n): dict(zip(("walk", "rhs_per_thread", "tile", "us", "us_tiled"), ctx.get_eo_walk(n)))
              for n in sorted({1, *nrhs_list})}
    f64_op = {str(n): dict(zip(("walk", "tile", "variant", "us", "us_tiled"), ctx.get_f64_walk(n)))
              for n in sorted({1, *nrhs_list})}
    mg = mrhs.Multigrid(ctx, [(4, 4, 4, 4), (2, 2, 2, 2)], [16, 16])
    t0 = time.perf_counter()
    for l in range(2):
        mg.set_basis(l, synth.gaussian_vectors(mg.volume[l], 16, mg.ncomp[l], 600 + l))
    mg.setup(**SOLVE_SETUP, coarse_prec="bf16", **SOLVE_VC)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    print(f"[bench] solve setup {setup_s:.1f} s", file=sys.stderr, flush=True)
    mg.tune(sorted(set(nrhs_list)))  # coarse stencil kernels and BF16 launch shapes per batch size
    free0, total = torch.cuda.mem_get_info()
    print(f"[bench] device memory after set-up: {free0 / 2**30:.1f} GiB free of {total / 2**30:.1f} GiB",
          file=sys.stderr, flush=True)
    vc = dict(SOLVE_VC, fine_eo=SOLVE_MRHS_FINE_EO, coarse_eo=SOLVE_MRHS_COARSE_EO)
    kp = mrhs.F32 if SOLVE_KRYLOV_F32 else mrhs.F64
    kw = dict(tol=1e-10, max_iters=SOLVE_MAXIT, check=False, krylov_prec=kp)
    mrhs_res, phases = {}, None
    for n in nrhs_list:
        m = solve_restart(synth.volume(SOLVE_DIMS) * 12 * n, free0)
        try:
            b = torch.from_numpy(synth.spinor_source(SOLVE_DIMS, n, 4000)).cuda()
            x = torch.zeros_like(b)
            st = mg.solve(x, b, use_graph=True, coarse_prec="bf16", restart=m, **kw, **vc)
            if st["status"] not in (0, 7):  # 7: ran to max_iters, reported below as not converged
                mg._check(st["status"])
        except Exception as exc:  # e.g. out of memory at the largest batch: keep the other batches
            mrhs_res[str(n)] = {"restart": m, "error": f"{type(exc).__name__}: {exc}"}
            print(f"[bench] MRHS solve N={n} failed: {exc}", file=sys.stderr, flush=True)
            b = x = None
            torch.cuda.empty_cache()
            continue
        mrhs_res[str(n)] = {
            "s_per_rhs": round(st["seconds_total"] / n, 4),
            "seconds": round(st["seconds_total"], 3),
            "iters": st["iters"],
            "restart": m,
            "converged": int(sum(st["converged"])),
            "max_true_resid": max(st["rel_resid"]),
        }
        print(f"[bench] MRHS solve N={n}: {st['seconds_total']:.2f} s, {st['iters']} iterations, "
              f"FGMRES({m}), {sum(st['converged'])}/{n} converged", file=sys.stderr, flush=True)
        if phases is None:  # per-phase breakdown from a timed (graph-free) solve of the first batch
            x.zero_()
            stt = mg.solve(x, b, use_graph=False, timers=True, coarse_prec="bf16", restart=m, **kw, **vc)
            phases = {"nrhs": n, "total_s": round(stt["seconds_total"], 4),
                      **{k: round(v, 4) for k, v in stt["seconds_phase"].items()}}
            print(f"[bench] timed MRHS solve {stt['seconds_total']:.2f} s", file=sys.stderr, flush=True)
        del b, x
        torch.cuda.empty_cache()
    # the same MRHS solve (first batch size) with the other level-1 smoother
    # (full coarse stencil instead of the coarse Schur complement, or back)
    coarse_eo = None
    n0 = nrhs_list[0]
    try:
        b = torch.from_numpy(synth.spinor_source(SOLVE_DIMS, n0, 4000)).cuda()
        x = torch.zeros_like(b)
        m = solve_restart(synth.volume(SOLVE_DIMS) * 12 * n0, free0)
        alt = not SOLVE_MRHS_COARSE_EO
        st = mg.solve(x, b, use_graph=True, coarse_prec="bf16", restart=m, **kw, **dict(vc, coarse_eo=alt))
        if st["status"] not in (0, 7):
            mg._check(st["status"])
        coarse_eo = {"coarse_eo": int(alt), "nrhs": n0, "s_per_rhs": round(st["seconds_total"] / n0, 4),
                     "seconds": round(st["seconds_total"], 3), "iters": st["iters"],
                     "converged": int(sum(st["converged"])), "max_true_resid": max(st["rel_resid"])}
        print(f"[bench] MRHS solve N={n0} with coarse_eo={int(alt)}: {st['seconds_total']:.2f} s, "
              f"{st['iters']} iterations", file=sys.stderr, flush=True)
        del b, x
        torch.cuda.empty_cache()
    except Exception as exc:
        coarse_eo = {"error": f"{type(exc).__name__}: {exc}"}
        b = x = None
        torch.cuda.empty_cache()
    # the same MRHS solve (first batch size) with Schwarz (SAP) smoothing on the
    # fine level: one cycle of four MR steps per 4^4 block (Sec. 9 outlook)
    sap = None
    try:
        b = torch.from_numpy(synth.spinor_source(SOLVE_DIMS, n0, 4000)).cuda()
        x = torch.zeros_like(b)
        m = solve_restart(synth.volume(SOLVE_DIMS) * 12 * n0, free0)
        vs = dict(vc, fine_eo=False, fine_sap=True, sap_iters=SOLVE_SAP_ITERS, nu_post=SOLVE_SAP_CYCLES)
        st = mg.solve(x, b, use_graph=True, coarse_prec="bf16", restart=m, **kw, **vs)
        if st["status"] not in (0, 7):
            mg._check(st["status"])
        sap = {"nrhs": n0, "cycles": SOLVE_SAP_CYCLES, "mr_steps_per_block": SOLVE_SAP_ITERS,
               "s_per_rhs": round(st["seconds_total"] / n0, 4), "seconds": round(st["seconds_total"], 3),
               "iters": st["iters"], "converged": int(sum(st["converged"])), "max_true_resid": max(st["rel_resid"])}
        print(f"[bench] MRHS solve N={n0} with SAP smoothing: {st['seconds_total']:.2f} s, {st['iters']} iterations",
              file=sys.stderr, flush=True)
        del b, x
        torch.cuda.empty_cache()
    except Exception as exc:
        sap = {"error": f"{type(exc).__name__}: {exc}"}
        b = x = None
        torch.cuda.empty_cache()
    # the same MRHS solve (first batch size) with the other outer Krylov basis precision
    other_basis = None
    try:
        b = torch.from_numpy(synth.spinor_source(SOLVE_DIMS, n0, 4000)).cuda()
        x = torch.zeros_like(b)
        alt = not SOLVE_KRYLOV_F32
        m = solve_restart(synth.volume(SOLVE_DIMS) * 12 * n0, free0, alt)
        st = mg.solve(x, b, use_graph=True, coarse_prec="bf16", restart=m,
                      **dict(kw, krylov_prec=mrhs.F32 if alt else mrhs.F64), **vc)
        if st["status"] not in (0, 7):
            mg._check(st["status"])
        other_basis = {"krylov_basis": "fp32" if alt else "fp64", "nrhs": n0, "restart": m,
                       "s_per_rhs": round(st["seconds_total"] / n0, 4), "seconds": round(st["seconds_total"], 3),
                       "iters": st["iters"], "converged": int(sum(st["converged"])),
                       "max_true_resid": max(st["rel_resid"])}
        print(f"[bench] MRHS solve N={n0} with the {'FP32' if alt else 'FP64'} Krylov basis: "
              f"{st['seconds_total']:.2f} s, {st['iters']} iterations", file=sys.stderr, flush=True)
        del b, x
        torch.cuda.empty_cache()
    except Exception as exc:
        other_basis = {"error": f"{type(exc).__name__}: {exc}"}
        print(f"[bench] MRHS solve N={n0} with the other Krylov basis failed: {exc}", file=sys.stderr, flush=True)
        b = x = None
        torch.cuda.empty_cache()
    # the comparator is the faster of the two fine smoothers on one RHS, with
    # the FP32 coarse stencil kernel tuned for one RHS
    mg.tune([1])
    b1 = torch.from_numpy(synth.spinor_source(SOLVE_DIMS, 1, 4000)).cuda()
    srhs = {}
    for eo in (False, True):
        x1 = torch.zeros_like(b1)
        srhs[eo] = mg.solve(x1, b1, use_graph=True, coarse_prec="f32", restart=SOLVE_RESTART, **kw,
                            **dict(SOLVE_VC, fine_eo=eo))
        print(f"[bench] SRHS solve (fine_eo={int(eo)}) {srhs[eo]['seconds_total']:.2f} s, {srhs[eo]['iters']} "
              "iterations", file=sys.stderr, flush=True)
    srhs_eo = min(srhs, key=lambda e: srhs[e]["seconds_total"] if srhs[e]["converged"][0] else 1e30)
    s1 = srhs[srhs_eo]
    ok = [k for k, v in mrhs_res.items() if v.get("converged") == int(k)]
    best = min(ok, key=lambda k: mrhs_res[k]["s_per_rhs"]) if ok else None
    out = {
        "workload": "24^3x128, smooth links U = exp(0.3 i H), csw 1.0, antiperiodic t, "
                    f"m0 {mass['m0']:.4f} (kappa {kappa:.6f}), 3 levels 24^3x128 -> 6^3x32 -> 3^3x16, "
                    "16 basis vectors per step, Gaussian sources, true residual 1e-10",
        "setup_s": round(setup_s, 3),
        "mrhs": mrhs_res,
        "mrhs_s_per_rhs": mrhs_res[best]["s_per_rhs"] if best else None,
        "mrhs_best_nrhs": int(best) if best else None,
        "srhs_s_per_rhs": round(s1["seconds_total"], 4),
        "srhs_iters": s1["iters"],
        "srhs_true_resid": s1["rel_resid"][0],
        "srhs_converged": int(s1["converged"][0]),
        "srhs_fine_eo": int(srhs_eo),
        "srhs_coarse_f32_kernel": {str(l): mg.get_tuning(l, 1) for l in (1, 2)},
        "mrhs_coarse_bf16_shape": {str(l): {str(n): mg.get_lowp_tuning(l, n)["cfg"] for n in nrhs_list}
                                   for l in (1, 2)},
        "srhs_s_by_fine_eo": {str(int(e)): round(v["seconds_total"], 4) for e, v in srhs.items()},
        "speedup": round(s1["seconds_total"] / mrhs_res[best]["s_per_rhs"], 3) if best else None,
        "mrhs_phase_s": phases,
        "mrhs_other_level1_smoother": coarse_eo,
        "mrhs_sap_smoother": sap,
        "mrhs_other_krylov_basis": other_basis,
        "eo_hop_kernel": eo_hop,
        "fine_f64_kernel": f64_op,
        "config": f"FP64 FGMRES({SOLVE_RESTART}, shorter where the batch's fields would not fit in HBM) with the "
                  f"Krylov basis in {'FP32 between FP64 restarts' if SOLVE_KRYLOV_F32 else 'FP64'} (both MRHS and "
                  f"SRHS), set-up {SOLVE_SETUP}, V-cycle {SOLVE_VC}; MRHS: BF16 coarse "
                  f"levels and BF16 matrix-core restrict/prolong, fine_eo {int(SOLVE_MRHS_FINE_EO)} (fine smoothing "
                  f"on the even-odd Schur complement), coarse_eo {int(SOLVE_MRHS_COARSE_EO)} (level-1 smoothing on "
                  "the coarse Schur complement), graph replay; SRHS comparator: same solver, one RHS, FP32 "
                  "coarse levels and FP32 intergrid, the faster of the two fine smoothers",
        "mass_tuning": {k: mass.get(k) for k in ("sigma_min", "t_bc_for_sigma_min", "target_sigma_min")},
    }
    mg.close()
    ctx.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--solve-nrhs", default="12,24,48,64", help="comma-separated batch sizes of the MRHS solve")
    ap.add_argument("--m0", type=float, default=None,
                    help="bare mass of the solve workload (default: the tuned value in tests/golden)")
    ap.add_argument("--tune-cache", default=TUNE_CACHE, help="autotuner text cache (read, appended)")
    ap.add_argument("--retune", action="store_true", help="tune the fine kernel afresh, ignoring the cache")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run a 1 GiB device-to-device copy first (reference for HBM byte counters)")
    ap.add_argument("--fabric-probe", action="store_true",
                    help="only measure the read bandwidth of device buffers of 16 MiB .. 2 GiB (L2-, Infinity-Cache- "
                         "and HBM-resident) and print it as one JSON line")
    a = ap.parse_args()

    if a.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {a.gpus} is not supported (the lattice domain decomposition "
              "across GPUs is not part of this build)", file=sys.stderr)
        sys.exit(2)

    if a.fabric_probe:
        print(json.dumps(fabric_probe()), flush=True)
        return

    # the oracle's timing runs first: its worker processes fork from a process
    # that has not touched the GPU
    cpu = None
    if not a.no_cpu_baseline:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        cpu = cpu_baseline()
        print(f"[bench] cpu baseline {cpu['value']} GFLOP/s on {cpu['cores']} cores", file=sys.stderr, flush=True)

    import torch

    import paper_2211_13719_amd as mrhs
    import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    if a.calib_copy:
        src_c = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst_c = torch.empty_like(src_c)
        for _ in range(3):
            dst_c.copy_(src_c)
        torch.cuda.synchronize()
        del src_c, dst_c

    t_setup = time.perf_counter()
    V = int(np.prod(DIMS))
    U = synth.gauge_haar(DIMS, 1)
    ctx = mrhs.Context(DIMS, t_bc=-1, stream=stream)
    ctx.set_gauge(U)
    del U
    ctx.build_clover(CSW, KAPPA)
    cache = None if a.retune else a.tune_cache
    if cache:
        os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
    ctx.tune(list(NRHS_FINE), cache)
    tuning = {str(n): dict(zip(("rhs_per_thread", "tile", "variant", "tuned_us"), ctx.get_tuning(n))) for n in NRHS_FINE}
    eo_tuning = {str(n): dict(zip(("walk", "rhs_per_thread", "tile", "us", "us_tiled"), ctx.get_eo_walk(n)))
                 for n in NRHS_FINE}
    f64_tuning = {str(n): dict(zip(("walk", "tile", "variant", "us", "us_tiled"), ctx.get_f64_walk(n)))
                  for n in NRHS_F64}
    mg = mrhs.Multigrid(ctx, [(4, 4, 4, 4), (2, 2, 2, 2)], [16, 16])
    mg.set_basis(0, synth.gaussian_vectors(V, 16, 12, 300))
    mg.block_orthonormalise(0)
    mg.build_coarse(1)
    mg.set_basis(1, synth.gaussian_vectors(mg.volume[1], 16, 32, 400))
    mg.block_orthonormalise(1)
    mg.build_coarse(2)
    mg.tune(list(NRHS_COARSE))
    coarse_tuning = {str(l): {str(n): {"f32": mg.get_tuning(l, n), **mg.get_lowp_tuning(l, n)} for n in NRHS_COARSE}
                     for l in (1, 2)}
    src = synth.spinor_source(DIMS, max(NRHS_FINE), 100, np.complex64)
    fine = {}
    for n in NRHS_FINE:
        x = torch.from_numpy(np.ascontiguousarray(src[:, :, :n])).to(dev)
        fine[n] = (x, torch.empty_like(x))
    del src
    fine64 = {}
    for n in NRHS_F64:
        x = fine[n][0].to(torch.complex128)
        fine64[n] = (x, torch.empty_like(x))
    coarse = {}
    for lev in (1, 2):
        for n in NRHS_COARSE:
            e = torch.from_numpy(synth.coarse_source(mg.volume[lev], NB, n, 50 * lev, np.complex64)).to(dev)
            coarse[(lev, n)] = (e, torch.empty_like(e))
    fi, _ = fine[N_INTER]
    fb = fi.clone()
    y = torch.empty((mg.volume[1], NB, N_INTER), dtype=torch.complex64, device=dev)
    fo = torch.empty_like(fi)
    dres = torch.empty(N_INTER, dtype=torch.complex128, device=dev)
    nres = torch.empty(N_INTER, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t_setup
    print(f"[bench] setup {setup_s:.1f} s", file=sys.stderr, flush=True)

    # (key, flops, alg bytes, callable)
    ops = []
    for n in NRHS_FINE:
        x, yf = fine[n]
        ops.append((("dwc", n), FLOPS_DWC * V * n, fine_bytes(V, n), lambda x=x, yf=yf: ctx.dwc(yf, x)))
    for n in NRHS_F64:
        x, yf = fine64[n]
        ops.append((("dwc_f64", n), FLOPS_DWC * V * n, 2 * fine_bytes(V, n), lambda x=x, yf=yf: ctx.dwc(yf, x)))
    for lev in (1, 2):
        Vc = mg.volume[lev]
        for prec in ("f32", "bf16", "f16"):
            for n in NRHS_COARSE:
                e, o = coarse[(lev, n)]
                ops.append(((f"coarse_l{lev}_{prec}", n), coarse_flops(Vc, n), coarse_bytes(Vc, n, prec),
                            lambda lev=lev, o=o, e=e, p=prec: mg.coarse_apply(lev, o, e, p)))
    Vc1 = mg.volume[1]
    ig_flops = 8 * 6 * 2 * 16 * V * N_INTER
    ops.append((("restrict", N_INTER), ig_flops, V * (12 * 16 * 8 + 96 * N_INTER) + Vc1 * NB * N_INTER * 8,
                lambda: mg.restrict(0, y, fi)))
    ops.append((("prolong", N_INTER), ig_flops, V * (12 * 16 * 8 + 96 * N_INTER) + Vc1 * NB * N_INTER * 8,
                lambda: mg.prolong(0, fo, y)))
    ig_bytes_bf16 = V * (12 * 16 * 4 + 96 * N_INTER) + Vc1 * NB * N_INTER * 8
    ops.append((("restrict_bf16", N_INTER), ig_flops, ig_bytes_bf16, lambda: mg.restrict(0, y, fi, prec="bf16")))
    ops.append((("prolong_bf16", N_INTER), ig_flops, ig_bytes_bf16, lambda: mg.prolong(0, fo, y, prec="bf16")))
    ops.append((("block_normalise", N_INTER), 6 * V * 12 * N_INTER, 2 * V * 96 * N_INTER,
                lambda: mg.block_normalise(0, fb)))
    ops.append((("dot", N_INTER), 8 * V * 12 * N_INTER, 2 * V * 96 * N_INTER, lambda: ctx.dot(fi, fo, out=dres)))
    ops.append((("norm", N_INTER), 4 * V * 12 * N_INTER, V * 96 * N_INTER, lambda: ctx.norm2(fi, out=nres)))

    def step(timer=None):
        for key, _, _, fn in ops:
            if timer is None:
                fn()
            else:
                timer(key, fn)

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()

    timer = Timer(torch, stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        step(timer)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    print(f"[bench] timed {a.steps} steps in {wall:.3f} s", file=sys.stderr, flush=True)

    times = timer.times()
    per_op = {}
    for key, flops, nbytes, _ in ops:
        ms = float(np.median(times[key]))
        name = f"{key[0]}@{key[1]}"
        per_op[name] = {
            "ms": round(ms, 5),
            "gflops": round(flops / ms / 1e6, 1),
            "alg_gbs": round(nbytes / ms / 1e6, 1),
            "hbm_frac": round(nbytes / ms / 1e6 / HBM_PEAK_GBS, 4),
        }
    if ("dwc", 1) in times:
        t1 = float(np.median(times[("dwc", 1)]))
        for n in NRHS_FINE:
            per_op[f"dwc@{n}"]["mrhs_speedup"] = round(n * t1 / float(np.median(times[("dwc", n)])), 3)

    # cold-cache figures: each op once more per rep, after a 512 MiB -> 512 MiB
    # device copy on the same stream (1 GiB of traffic, four times the 256 MB
    # Infinity Cache and far beyond the L2s), timed alone by HIP events
    flush_a = torch.empty(1 << 27, dtype=torch.float32, device=dev)
    flush_b = torch.empty_like(flush_a)
    flush_a.fill_(1.0)
    cold = Timer(torch, stream)
    for _ in range(max(3, a.steps // 2)):
        for key, _, _, fn in ops:
            flush_b.copy_(flush_a)
            cold(key, fn)
    torch.cuda.synchronize()
    del flush_a, flush_b
    cold_times = cold.times()
    for key, flops, nbytes, _ in ops:
        ms = float(np.median(cold_times[key]))
        e = per_op[f"{key[0]}@{key[1]}"]
        e["ms_cold"] = round(ms, 5)
        e["hbm_frac_cold"] = round(nbytes / ms / 1e6 / HBM_PEAK_GBS, 4)

    # dominant kernel: the fine D_wc instantiation with the largest share of the step
    share = {}
    for n in NRHS_FINE:
        share.setdefault(fine_kernel_name(ctx, n), []).append(n)
    dom = max(share, key=lambda k: sum(np.mean(times[("dwc", n)]) for n in share[k]))
    launches = [(n, t) for n in share[dom] for t in times[("dwc", n)]]
    mean_bytes = float(np.mean([fine_bytes(V, n) for n, _ in launches]))
    mean_ms = float(np.mean([t for _, t in launches]))
    achieved = mean_bytes / mean_ms / 1e6
    traffic = None
    cfg_now = {str(n): [tuning[str(n)]["rhs_per_thread"], list(tuning[str(n)]["tile"]), tuning[str(n)]["variant"]]
               for n in share[dom]}
    if (FINE_TRAFFIC and FINE_TRAFFIC["kernel"] == dom and FINE_TRAFFIC["sources"] == fine_sources_digest()
            and FINE_TRAFFIC["configs"] == cfg_now):
        traffic = FINE_TRAFFIC["bytes_per_launch"]

    total_flops = sum(f for _, f, _, _ in ops)
    ms_per_step = wall * 1e3 / a.steps

    evenodd = bench_evenodd(ctx, mg, torch, stream, fine, coarse, V, a.warmup, a.steps)

    # headline: the FP32 fine D_wc on 24^4 over the Nrhs set (algorithmic
    # flops of the six applies over their summed median times), and per Nrhs
    dwc_keys = [("dwc", n) for n in NRHS_FINE]
    dwc_flops = sum(f for k, f, _, _ in ops if k in dwc_keys)
    dwc_ms = sum(float(np.median(times[k])) for k in dwc_keys)
    value = dwc_flops / dwc_ms / 1e6
    value_by_nrhs = {str(n): per_op[f"dwc@{n}"]["gflops"] for n in NRHS_FINE}
    # the whole step's composite rate, with the arithmetic each part runs in
    mix = {}
    for (name, n), flops, _, _ in ops:
        if name.endswith("_bf16"):
            prec = "bf16 operands, fp32 accumulation"
        elif name.endswith("_f16"):
            prec = "fp16 operands, fp32 accumulation"
        elif name in ("dot", "norm", "block_normalise"):
            prec = "fp32 inputs, fp64 sums"
        elif name == "dwc_f64":
            prec = "fp64"
        else:
            prec = "fp32"
        mix[prec] = mix.get(prec, 0.0) + flops / 1e9
    composite = {
        "gflops": round(total_flops / (ms_per_step * 1e-3) / 1e9, 1),
        "ms_per_step": round(ms_per_step, 4),
        "gflop_per_step_by_precision": {k: round(v, 2) for k, v in mix.items()},
        "note": "all ops of one step (fine D_wc in fp32 and fp64, coarse stencils in fp32/bf16/fp16, intergrid, "
                "reductions) over the step's wall time; a mixed-precision figure, not an fp32 rate",
    }

    result = {
        "metric": "MRHS Dslash/coarse-stencil GFLOP/s vs Nrhs; mixed-prec MG s/RHS to 1e-10",
        "value": round(value, 1),
        "unit": "GFLOP/s",
        "value_note": "FP32 fine Wilson-clover D_wc, 24^4, algorithmic flops of the applies at Nrhs "
                      "1, 6, 12, 24, 48, 64 over their summed median times (HIP events); per Nrhs in value_by_nrhs",
        "value_by_nrhs": value_by_nrhs,
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
            "workload": "MRHS Wilson-clover hot path, one pass: fine D_wc 24^4 FP32 Nrhs 1..64 and FP64 Nrhs "
                        "1, 12, 48 (Haar links, csw 1.0, kappa 0.13, antiperiodic t); Galerkin coarse stencil 6^4 "
                        "and 3^4, Nb 32, "
                        "Nrhs 12..64, FP32/BF16/FP16; restrict/prolong/block-normalise 24^4<->6^4 and dot/norm, "
                        "Nrhs 24",
            "lattice": list(DIMS),
            "nrhs_fine": list(NRHS_FINE),
            "nrhs_fine_f64": list(NRHS_F64),
            "nrhs_coarse": list(NRHS_COARSE),
        },
        "roofline": {
            "bound": "hbm",
            "kernel": dom,
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "traffic_note": FINE_TRAFFIC["note"] if traffic else "no counter record for this kernel build "
                            "and configuration",
            "alg_bytes_per_launch_mean": mean_bytes,
            "launch_ms_mean": round(mean_ms, 5),
            "launches_per_step": len(share[dom]),
        },
        "per_op": per_op,
        "composite_step": composite,
        "evenodd": evenodd,
        "fine_tuning": tuning,
        "eo_hop_tuning": eo_tuning,
        "fine_f64_tuning": f64_tuning,
        "coarse_f32_tuning": coarse_tuning,
        "fine_sources": fine_sources_digest(),
        "solve": None,
        "cpu_baseline": None,
    }
    mg.close()
    ctx.close()
    del fine, coarse
    torch.cuda.empty_cache()
    if not a.no_solve:
        mpath = os.path.join(HERE, "tests", "golden", "smooth_links_mass.json")
        if a.m0 is not None:
            mass = {"m0": a.m0, "kappa": 1.0 / (2.0 * (4.0 + a.m0)), "sigma_min": None}
        elif os.path.exists(mpath):
            with open(mpath) as fh:
                mass = json.load(fh)
        else:
            mass = {"m0": 0.0, "kappa": 0.125, "sigma_min": None}
        print("[bench] solve ...", file=sys.stderr, flush=True)
        try:
            result["solve"] = run_solve(mrhs, torch, synth, [int(v) for v in a.solve_nrhs.split(",")], mass,
                                        cache)
        except Exception as exc:  # report the failure in the JSON line instead of losing the kernel results
            result["solve"] = {"error": f"{type(exc).__name__}: {exc}"}
            print(f"[bench] solve failed: {exc}", file=sys.stderr, flush=True)
    result["cpu_baseline"] = cpu
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
