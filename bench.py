#!/usr/bin/env python3
"""Throughput of simultaneous local upscaling on one MI355X.

One step is one pass of the plain hot path over one batch of synthetic
samples, with the random variables xi already resident in HBM:

  1. coefficient samples a(x, xi) on the fine grid       (stomsfem_coef_bumps)
  2. local upscaling S_K(xi) for every (element, sample)  (stomsfem_upscale)
  3. coarse solve S U = b per sample, Monte Carlo mean   (stomsfem_coarse_solve)

Default workload: 32 x 32 coarse elements, H/h = 32 (1024 x 1024 fine Q1
grid), 4096 samples (4,194,304 element-sample pairs), FP64.  The metric is
upscaled (element x sample) pairs per second for the whole step.

Prints one JSON line with a roofline entry for the dominant kernel (the local
upscaling, timed with HIP events on the stream it runs on) and a CPU baseline
(the FP64 oracle on the host cores, on a bounded sample of the same workload).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_VALU_PEAK_TFLOPS = 78.6   # MI355X: 256 CUs x 2.4 GHz x 128 FP64 flop/clk
HBM_PEAK_GBS = 8000.0


def plain_flops_per_pair(m: int) -> float:
    """FP64 operations of the sliding-window LDL^T Schur-complement algorithm
    for one (element, sample) pair (an FMA counts 2): per pivot j with c
    active rows below it, the rank-1 window update c(c+1)/2 FMA, the column
    scaling c mul + 1 div, the 3-rhs forward step 3c FMA and the y y^T/d
    accumulation 9 ops; plus 20 ops per interior row for assembling the
    9-point stencil row and its Dirichlet lifts, and 12 per boundary element
    for g.K_BB g'."""
    n = m - 1
    NI = n * n
    f = 0.0
    for j in range(NI):
        c = min(m, NI - 1 - j)
        f += c * (c + 1) + c + 1 + 6 * c + 9
    f += 20 * NI + 12 * max(4 * (m - 1), 1)
    return f


def cpu_baseline(wl, budget_s: float = 15.0):
    import numpy as np

    import oracle
    from paper_1607_00693_amd import workloads as W

    threads = os.cpu_count() or 1
    nprobe = 2
    xi = W.uniform_xi(wl.nsamples, wl.nxi, wl.seed)

    def run(ns):
        t0 = time.perf_counter()
        a = oracle.coef_bumps(xi[:ns], wl.nfine, **wl.coef_params(), nthreads=threads)
        S, _, _ = oracle.upscale(a, wl.nc, wl.nc, wl.m, nthreads=threads)
        oracle.coarse_solve(S, wl.nc, wl.nc, nthreads=threads)
        return time.perf_counter() - t0

    t = run(nprobe)
    ns = int(max(nprobe, min(wl.nsamples, nprobe * budget_s / max(t, 1e-6))))
    t = run(ns)
    pairs = ns * wl.M
    return {
        "value": pairs / t,
        "unit": "pairs/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"first {ns} of {wl.nsamples} samples ({pairs} element-sample pairs): coefficient "
                  f"generation + upscaling + coarse solve, OpenMP over pairs, {t:.1f} s",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="mesh32", choices=["mesh32", "mesh8"])
    ap.add_argument("--nsamples", type=int, default=0, help="override the sample count (0 = workload default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1 "
                          "(sharding over samples is described in the design notes)"}))
        sys.exit(2)

    import dataclasses

    import torch

    from paper_1607_00693_amd import stomsfem
    from paper_1607_00693_amd import workloads as W

    wl = W.MESH32 if args.workload == "mesh32" else W.MESH8
    if args.nsamples:
        wl = dataclasses.replace(wl, nsamples=args.nsamples)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()

    xi = torch.from_numpy(W.uniform_xi(wl.nsamples, wl.nxi, wl.seed)).to(dev)
    a = torch.empty((wl.nsamples, wl.nfine, wl.nfine), dtype=torch.float64, device=dev)
    S = torch.empty((wl.nsamples, wl.M, 10), dtype=torch.float64, device=dev)
    nU = (wl.nc - 1) ** 2
    U = torch.empty((wl.nsamples, nU), dtype=torch.float64, device=dev)
    qm = torch.empty(nU, dtype=torch.float64, device=dev)
    qv = torch.empty(nU, dtype=torch.float64, device=dev)
    status = torch.empty((wl.nsamples, wl.M), dtype=torch.int32, device=dev)

    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]

    def step(record):
        if record:
            ev[0].record(stream)
        stomsfem.coef_bumps(xi, wl.nfine, **wl.coef_params(), out=a, stream=stream)
        if record:
            ev[1].record(stream)
        stomsfem.upscale(a, wl.nc, wl.nc, wl.m, S=S, status=status, stream=stream)
        if record:
            ev[2].record(stream)
        stomsfem.coarse_solve(S, wl.nc, wl.nc, U=U, qoi_mean=qm, qoi_var=qv, stream=stream)
        if record:
            ev[3].record(stream)

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    print(f"[bench] warmup done ({args.warmup} steps)", file=sys.stderr, flush=True)

    t_gen = t_up = t_co = 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(True)
        ev[3].synchronize()
        t_gen += ev[0].elapsed_time(ev[1])
        t_up += ev[1].elapsed_time(ev[2])
        t_co += ev[2].elapsed_time(ev[3])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    bad = int((status != 0).sum().item())
    ms = (t1 - t0) * 1000.0 / args.steps
    pairs = wl.nsamples * wl.M
    t_up /= args.steps
    t_gen /= args.steps
    t_co /= args.steps
    flops = plain_flops_per_pair(wl.m) * pairs
    achieved = flops / (t_up * 1e-3) / 1e12
    bytes_alg = pairs * (wl.m * wl.m * 8 + 10 * 8 + 4)
    print(f"[bench] {args.steps} steps: {ms:.2f} ms/step (gen {t_gen:.2f}, upscale {t_up:.2f}, coarse {t_co:.2f} ms),"
          f" non-OK pairs {bad}", file=sys.stderr, flush=True)

    out = {
        "metric": "upscaled (patch x sample)/s, plain FP64 path",
        "value": pairs / (ms * 1e-3),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{wl.name}: {wl.nc}x{wl.nc} coarse, H/h={wl.m}, {wl.nsamples} samples, "
                        f"{wl.nxi} bumps (xi~U[-1,1]), f=1, zero Dirichlet",
            "nc": wl.nc, "m": wl.m, "nsamples": wl.nsamples, "pairs": pairs,
        },
        "kernel_ms": {"coef_bumps": t_gen, "upscale": t_up, "coarse_solve_qoi": t_co},
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": FP64_VALU_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP64_VALU_PEAK_TFLOPS,
            "traffic": None,
            "kernel": "local upscaling (FP64 VALU)",
            "flops_per_pair": plain_flops_per_pair(wl.m),
            "hbm_frac_algorithmic": bytes_alg / (t_up * 1e-3) / 1e9 / HBM_PEAK_GBS,
        },
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
