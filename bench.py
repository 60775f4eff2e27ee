#!/usr/bin/env python3
"""Benchmark of the ST-HOSVD hot path on one MI355X.

Workload (N=1): a 200x200x200x16 float64 tensor (core 20x20x20x8 with spectra
decaying by 0.7 per index in every mode, orthonormal factors, relative noise
1e-5; seed 2), compressed with eps = 1e-4 in mode order 0,1,2,3, followed by the
Multi-TTM reconstruction of the 50x50x50x16 sub-tensor at (75,75,75,0).
One step = tucker_sthosvd + tucker_reconstruct + tucker_free, inputs resident
in HBM.  value = input bytes / time per step (GB/s).

Also reported: Gram TFLOP/s (sum_n J_n^2 K_n, the symmetric count, over the
main Gram kernels' time), the roofline of the dominant kernel (the mode-0 FP64
Gram, timed with HIP events on the call's stream during the timed steps), and
the FP64 CPU oracle timed on the host over the same step.
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

METRIC = "ST-HOSVD input GB/s + Gram TFLOP/s, mixed/batched vs FP64 GPU at rel err≤1.05ε"
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0


def gram_flops(dims, ranks, order):
    """sum over modes of J_n^2 * K_n with the sizes at the time mode n is processed."""
    cur = list(dims)
    tot = []
    for n in order:
        K = 1
        for k, v in enumerate(cur):
            if k != n:
                K *= v
        tot.append(cur[n] * cur[n] * K)
        cur[n] = ranks[n]
    return tot


def cpu_baseline(X, dims, eps, order, begin, end, nbytes):
    import oracle
    t0 = time.perf_counter()
    ref = oracle.sthosvd(X, dims, eps, order)
    oracle.reconstruct(ref, begin, end)
    dt = time.perf_counter() - t0
    return {"value": nbytes / dt / 1e9, "unit": "GB/s", "cores": len(os.sched_getaffinity(0)),
            "kind": "oracle", "seconds": dt, "ranks": ref.ranks,
            "sample": "one full step (ST-HOSVD eps=1e-4 + 50x50x50x16 reconstruction) of the same "
                      "200x200x200x16 float64 tensor, FP64 loops with OpenMP"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--eps", type=float, default=1e-4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(see DESIGN.md for how the method would shard); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1901_06043_amd as tk
    import synthetic

    X, dims = synthetic.decaying_200()
    order = [0, 1, 2, 3]
    begin, end = [75, 75, 75, 0], [125, 125, 125, 16]
    x = torch.from_numpy(X.reshape(dims[::-1])).to("cuda")
    nbytes = x.numel() * x.element_size()
    out = torch.empty([e - b for b, e in zip(begin, end)][::-1], dtype=torch.float64, device="cuda")

    def step():
        t = tk.sthosvd(x, args.eps, mode_order=order)
        t.reconstruct(begin, end, out=out)
        rec = (list(t.ranks), [(m.gram_ms, m.eig_ms, m.ttm_ms, m.gram_kernel_ms) for m in t.timings],
               t.norm2, list(t.discarded))
        t.free()
        return rec

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed / args.steps * 1e3
    ranks = recs[-1][0]
    assert all(r[0] == ranks for r in recs), "ranks changed between steps"

    # per-mode breakdown (median over steps)
    tim = np.array([r[1] for r in recs])  # steps x N x 4
    med = np.median(tim, axis=0)
    flops = gram_flops(dims, ranks, order)
    gram_kernel_ms = [float(med[n][3]) for n in order]
    gram_tflops = sum(flops) / (sum(gram_kernel_ms) * 1e-3) / 1e12
    # dominant kernel: the mode-0 Gram (FP64 MFMA): J^2 K symmetric flops per launch
    n0 = order[0]
    k0 = float(np.mean(tim[:, n0, 3]))
    ach = flops[0] / (k0 * 1e-3) / 1e12
    roofline = {"kernel": "gram_f64_kernel (mode %d, J=%d, K=%d)" % (n0, dims[n0], int(np.prod(dims)) // dims[n0]),
                "bound": "mfma", "achieved": round(ach, 3), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": round(ach / PEAK_FP64_TFLOPS, 4), "traffic": None,
                "avg_launch_ms": round(k0, 5), "algorithmic_flops_per_launch": flops[0]}

    # relative error of the last step from Corollary 1 (sum of discarded eigenvalues)
    relerr = float(np.sqrt(max(sum(recs[-1][3]), 0.0) / recs[-1][2]))
    line = {
        "metric": METRIC, "value": round(nbytes / (ms_per_step * 1e-3) / 1e9, 3), "unit": "GB/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "ST-HOSVD FP64 of a 200x200x200x16 float64 tensor (core 20x20x20x8, "
                               "0.7 spectral decay, noise 1e-5), eps=%g, order 0123, + 50x50x50x16 "
                               "subrange reconstruction" % args.eps,
                   "dims": dims, "eps": args.eps, "mode_order": order, "ranks": ranks,
                   "gram_precision": "fp64"},
        "gram_tflops": round(gram_tflops, 3),
        "relerr": relerr,
        "per_mode_ms": {str(n): {"gram": round(float(med[n][0]), 4), "gram_kernel": round(float(med[n][3]), 4),
                                 "eig": round(float(med[n][1]), 4), "ttm": round(float(med[n][2]), 4)}
                        for n in order},
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(X, dims, args.eps, order, begin, end, nbytes)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
