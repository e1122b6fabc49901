#!/usr/bin/env python3
"""Benchmark of the collision-operator hot path on one MI355X.

One step = one evaluation of Q_h(f) with the FP64 conservation projection over
the whole batch (4096 cells, 2D 32x32 velocity grid on [-8, 8]^2, hard spheres,
M = 8 directions, radial rank 5), inputs resident in HBM. The mixed-precision
path (FX16) is the headline value; the plain FP32 path is timed on the same
workload for comparison. Prints ONE JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--cpu-seconds S]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    # name: (N, L, kernel, M, description)
    "hs2d_32": (32, 8.0, "hard_sphere", 8, "4096 cells, 2D 32x32 velocity grid on [-8,8]^2, hard spheres, "
                "M=8 directions x K_r=5 radial ranks (21 transforms), FP64 conservation projection"),
    "hs2d_64_noisy": (64, 10.0, "hard_sphere", 16, "20000 cells, 2D 64x64 velocity grid on [-10,10]^2, hard "
                      "spheres, M=16 x K_r=5 (41 transforms), mixtures + 1% noise, FP64 conservation projection"),
}
HBM_PEAK = 8.0e12          # B/s
FP16_MFMA_PEAK = 2.5e15    # dense FLOP/s
FP32_MFMA_PEAK = 157.3e12  # dense FLOP/s


def mfma_flops_per_cell(precision: str, transforms: int, N: int = 32) -> float:
    """MFMA floating-point operations one cell issues (2 per multiply-add).

    A complex 32-point DFT pass over a 32 x 32 tile is a real GEMM with
    M = 32, K = 64, N = 64 (2 * 32 * 64 * 64 flops); the real-input first
    forward pass has K = 32; the loss transform's second pass needs only the
    real half. FX16 issues 6 FP16 products per GEMM, FP32 one.
    """
    full = 2 * 32 * 64 * 64
    per_cell = full / 2 + full            # forward: real-input pass + complex pass
    per_cell += (transforms - 1) * 2 * full  # packed gain transforms, two passes each
    per_cell += 2 * full                  # loss transform (both passes computed)
    if N > 32:                            # tile-64: four 32-point sub-transforms per cell
        per_cell *= 4
    return per_cell * (6 if precision == "fx16" else 1)


def time_launches(fn, steps: int, warmup: int, stream):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        starts[i].record(stream)
        fn()
        ends[i].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = np.array([s.elapsed_time(e) for s, e in zip(starts, ends)]) / 1e3
    return wall, per


def cpu_baseline(f64: np.ndarray, target_s: float, N: int, L: float, kernel: str, M: int):
    """The FP64 oracle on a bounded prefix of the same cells (single-threaded FFTs)."""
    from oracle import spectral as sp
    s = sp.Setup(d=2, N=N, L=L, kernel=kernel, M=M)
    bank = sp.filter_bank(s)
    done, t_used, chunk = 0, 0.0, 16
    outs = []
    while t_used < target_s and done < len(f64):
        c = f64[done:done + chunk]
        t0 = time.perf_counter()
        q = sp.project_conservative(sp.q_fast(c, s, bank), 2, L)
        t_used += time.perf_counter() - t0
        outs.append(q)
        done += len(c)
    return done, t_used, np.concatenate(outs)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--workload", default="hs2d_32", choices=sorted(WORKLOADS))
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="after timing, copy a buffer of this many MiB once (a plain copy kernel of "
                         "known size, for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the operator is cell-local: N GPUs run N independent shards).", file=sys.stderr)
        return 2

    import torch
    import workloads as wl
    from paper_2103_14890_amd import qcoll

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    NN, LL, KERN, MM, DESC = WORKLOADS[args.workload]
    f64 = wl.config_inputs(args.workload)
    cells = f64.shape[0]
    f = torch.tensor(f64, dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()

    res = {}
    precs = ("fx16", "fp32") if NN <= 32 else ("fx16",)
    for prec in precs:
        plan = qcoll.Plan(2, NN, LL, KERN, MM, precision=prec, conserve=True)
        q = torch.empty((cells, NN, NN), dtype=torch.float64, device=dev)
        wall, per = time_launches(lambda: plan.eval(f, q), args.steps, args.warmup, stream)
        info = plan.info()
        res[prec] = dict(plan=plan, q=q, wall=wall, per=per, info=info)

    if args.calibrate_copy > 0:
        src = torch.ones(args.calibrate_copy << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # accuracy on a sample, against the oracle (also the CPU-baseline run)
    ncpu, t_cpu, q_ref = cpu_baseline(f64.astype(np.float32).astype(np.float64), args.cpu_seconds, NN, LL, KERN, MM)
    for prec in res:
        qg = res[prec]["q"][:ncpu].cpu().numpy()
        res[prec]["rel_err"] = float(np.linalg.norm(qg - q_ref) / np.linalg.norm(q_ref))
        qa = res[prec]["q"].cpu().numpy()
        res[prec]["mass"] = float((np.abs(qa.sum(axis=(1, 2))) / np.abs(qa).sum(axis=(1, 2))).max())

    mix = res["fx16"]
    T = float(np.mean(mix["per"]))
    value = cells / T
    flops = mfma_flops_per_cell("fx16", mix["info"]["transforms"], NN) * cells
    dense = mfma_flops_per_cell("fp32", mix["info"]["transforms"], NN) * cells
    fp32 = res.get("fp32")
    if fp32 is not None:
        T32 = float(np.mean(fp32["per"]))
        flops32 = mfma_flops_per_cell("fp32", fp32["info"]["transforms"], NN) * cells
    threads = 1   # the oracle's numpy FFTs run on one core
    out = {
        "metric": "cell Q(f,f) evals/s at N_v=32^2, mixed vs FP32 at rel.err<=1e-5; p99 latency",
        "value": value,
        "unit": "cell-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": T * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16x6+f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {DESC}",
                   "cells": cells, "N_v": f"{NN}x{NN}", "kernel": KERN, "M": MM,
                   "K_r": mix["info"]["K_r"]},
        "roofline": {"bound": "mfma", "achieved": flops / T / 1e12, "peak": FP16_MFMA_PEAK / 1e12,
                     "unit": "TFLOP/s", "frac": flops / T / FP16_MFMA_PEAK, "traffic": None},
        "cpu_baseline": {"value": ncpu / t_cpu, "unit": "cell-evals/s", "cores": threads, "kind": "oracle",
                         "sample": f"first {ncpu} cells of the same workload, FP64 numpy FFT oracle "
                                   f"+ projection, {t_cpu:.1f} s"},
        "rel_err_l2": mix["rel_err"],
        "mass_defect_max": mix["mass"],
        "dense_gemm_tflops": dense / T / 1e12,
        "fp32_path": None if fp32 is None else {
            "value": cells / T32, "ms_per_step": T32 * 1e3, "rel_err_l2": fp32["rel_err"],
            "roofline_frac": flops32 / T32 / FP32_MFMA_PEAK, "mass_defect_max": fp32["mass"]},
        "speedup_vs_fp32": None if fp32 is None else T32 / T,
        "launch_ms": {"p5": float(np.percentile(mix["per"], 5) * 1e3),
                      "p50": float(np.median(mix["per"]) * 1e3),
                      "p95": float(np.percentile(mix["per"], 95) * 1e3)},
        "p99_latency_ms": None,
    }
    print(json.dumps(out))
    for prec in res:
        res[prec]["plan"].close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
