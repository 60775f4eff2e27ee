#!/usr/bin/env python3
"""Benchmark of the ST-HOSVD hot path on one MI355X.

Headline (N=1) workload: a 200x200x200x16 float64 tensor (core 20x20x20x8 with
spectra decaying by 0.7 per index in every mode, orthonormal factors, relative
noise 1e-5; seed 2), compressed with eps = 1e-4 in mode order 0,1,2,3 with the
FP64 path, followed by the Multi-TTM reconstruction of the 50x50x50x16
sub-tensor at (75,75,75,0).  One step = tucker_sthosvd + tucker_reconstruct +
tucker_free, inputs resident in HBM.  value = input bytes / time per step.

Also reported on the same JSON line:
* gram_tflops: sum_n J_n^2 K_n (the symmetric count) over the main Gram
  kernels' time;
* roofline: the dominant kernel (the mode-0 FP64 Gram), its average launch
  time from HIP events recorded inside the library on the call's stream
  during the timed steps, against the FP64 MFMA peak;
* cpu_baseline: the FP64 CPU oracle timed on the host over whole steps of the
  same workload;
* precision_form: the 256x256x256x11x50 float32 combustion-shaped tensor at
  eps 1e-2..1e-5 with FP64, FP32-MFMA, BF16x6 and BF16x3 Grams: time, input
  GB/s, Gram TFLOP/s, ranks against the FP64 GPU path, explicit relative error
  against 1.05 eps, largest principal-angle sine against the FP64 factors;
* large_share: the 672x672x33x626 float32 Fourier-field tensor in mode order
  3,2,0,1 at eps 1e-4 with every Gram form, plus full and subrange
  reconstruction;
* batched_form: 1024 independent float32 3-way tensors (sizes U{16..128},
  ranks U{2..I/4}, noise 1e-4) at eps 1e-3, one batched run replayed from a
  captured HIP graph against a loop of single-tensor calls, per Gram form.
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
FORMS = ["fp64", "fp32", "bf16x6", "bf16x3"]


def gram_flops(dims, ranks, order):
    """Per processed mode: J_n^2 * K_n with the sizes at the time mode n is processed."""
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


def profiled_traffic(name="gram_tri_kernel_200x200x200x16_traffic.md"):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary, or None if the kernel source changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    kv = {}
    for ln in open(path):
        if ":" in ln and not ln.startswith(("|", "#", " ")):
            k, v = ln.split(":", 1)
            kv[k.strip()] = v.strip()
    try:
        src = open(os.path.join(ROOT, kv["source_file"]), "rb").read()
        if hashlib.sha256(src).hexdigest() != kv["source_sha256"]:
            return None
        return int(kv["traffic_bytes_per_launch"])
    except (KeyError, OSError, ValueError):
        return None


def cpu_baseline(X, dims, eps, order, begin, end, nbytes, min_seconds=10.0):
    import oracle
    n, t0 = 0, time.perf_counter()
    while True:
        ref = oracle.sthosvd(X, dims, eps, order)
        oracle.reconstruct(ref, begin, end)
        n += 1
        dt = time.perf_counter() - t0
        if dt >= min_seconds:
            break
    per = dt / n
    return {"value": round(nbytes / per / 1e9, 4), "unit": "GB/s", "cores": len(os.sched_getaffinity(0)),
            "kind": "oracle", "seconds_per_step": round(per, 4), "steps": n, "ranks": ref.ranks,
            "sample": "%d full steps (ST-HOSVD eps=%g + 50x50x50x16 reconstruction) of the same "
                      "200x200x200x16 float64 tensor, FP64 loops with OpenMP, about %.0f s" % (n, eps, dt)}


def relerr_slabs(t, x, dims, torch, nslab=10):
    """||X - X^|| / ||X|| in FP64, reconstructing the last mode in slabs."""
    num = den = 0.0
    step = max(1, -(-dims[-1] // nslab))
    N = len(dims)
    for s0 in range(0, dims[-1], step):
        s1 = min(dims[-1], s0 + step)
        xh = t.reconstruct([0] * (N - 1) + [s0], list(dims[:-1]) + [s1], out_dtype=torch.float64)
        xs = x[s0:s1].to(torch.float64)
        num += float((xs - xh).pow(2).sum())
        den += float(xs.pow(2).sum())
        del xh, xs
    return (num / den) ** 0.5 if den > 0 else 0.0


def max_sin(tk, torch, ref_factors, t, ref_ranks):
    out = []
    for n, U in enumerate(ref_factors):
        if t.ranks[n] != ref_ranks[n]:
            out.append(None)
            continue
        s = torch.linalg.svdvals(U.t() @ t.factor(n))
        out.append(float(torch.sqrt(torch.clamp(1 - s.min() ** 2, min=0.0))))
    return out


def run_form(tk, torch, x, dims, eps, order, prec, reps):
    """Median wall time of `reps` compressions (after one warm-up), returning the last handle."""
    t = tk.sthosvd(x, eps, mode_order=order, prec=prec, dims=dims)
    t.free()
    torch.cuda.synchronize()
    ts = []
    for r in range(reps):
        t0 = time.perf_counter()
        t = tk.sthosvd(x, eps, mode_order=order, prec=prec, dims=dims)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
        if r + 1 < reps:
            t.free()
    ts.sort()
    return t, ts[len(ts) // 2] * 1e3


def compare_forms(tk, torch, x, dims, eps_list, order, reps, nbytes, extra=None):
    rows = []
    for eps in eps_list:
        ref = None
        for prec in FORMS:
            print(f"# {prec} eps={eps}", file=sys.stderr, flush=True)
            t, ms = run_form(tk, torch, x, dims, eps, order, prec, reps)
            fl = gram_flops(dims, t.ranks, order)
            gk = [t.timings[n].gram_kernel_ms for n in order]
            e = relerr_slabs(t, x, dims, torch)
            row = {"eps": eps, "gram": prec, "ms": round(ms, 3), "input_GBs": round(nbytes / ms / 1e6, 2),
                   "gram_tflops": round(sum(fl) / (sum(gk) * 1e-3) / 1e12, 2), "ranks": list(t.ranks),
                   "relerr": e, "within_1.05eps": bool(e <= 1.05 * eps), "gram_used": t.gram_precision,
                   "per_mode_ms": {str(n): [round(t.timings[n].gram_ms, 3), round(t.timings[n].eig_ms, 3),
                                            round(t.timings[n].ttm_ms, 3)] for n in order}}
            if prec == "fp64":
                ref = (list(t.ranks), [t.factor(n).clone() for n in range(len(dims))], ms)
                row["speedup_vs_fp64"] = 1.0
                row["ranks_match_fp64"] = True
            else:
                row["speedup_vs_fp64"] = round(ref[2] / ms, 3)
                row["ranks_match_fp64"] = list(t.ranks) == ref[0]
                row["max_sin_angle_vs_fp64"] = max_sin(tk, torch, ref[1], t, ref[0])
            if extra is not None:
                row.update(extra(t))
            rows.append(row)
            t.free()
    return rows


def precision_section(tk, torch, synthetic, reps):
    t0 = time.perf_counter()
    x, dims, _ = synthetic.combustion(device="cuda")
    torch.cuda.synchronize()
    gen = time.perf_counter() - t0
    nbytes = x.numel() * 4
    rows = compare_forms(tk, torch, x, dims, [1e-2, 1e-3, 1e-4, 1e-5], list(range(5)), reps, nbytes)
    del x
    torch.cuda.empty_cache()
    return {"workload": "256x256x256x11x50 float32 combustion-shaped tensor (64 advected Gaussian bumps per "
                        "variable, per-variable scale 10^U[-6,3], max-rescaled per variable; seed 3), "
                        "mode order 0,1,2,3,4", "dims": dims, "bytes": nbytes, "generate_s": round(gen, 2),
            "reps": reps, "results": rows}


def large_section(tk, torch, synthetic, reps):
    t0 = time.perf_counter()
    x, dims = synthetic.fourier_fields(device="cuda")
    torch.cuda.synchronize()
    gen = time.perf_counter() - t0
    nbytes = x.numel() * 4
    order = [3, 2, 0, 1]

    def recon(t):
        # full reconstruction (float32) and the 672x672x1x1 subrange at v=0, t=313
        out = torch.empty_like(x)
        torch.cuda.synchronize()
        a = time.perf_counter()
        t.reconstruct(out=out)
        torch.cuda.synchronize()
        full = time.perf_counter() - a
        del out
        a = time.perf_counter()
        t.reconstruct([0, 0, 0, 313], [672, 672, 1, 314], out_dtype=torch.float32)
        torch.cuda.synchronize()
        sub = time.perf_counter() - a
        return {"reconstruct_full_ms": round(full * 1e3, 3),
                "reconstruct_full_GBs_written": round(nbytes / full / 1e9, 2),
                "reconstruct_sub_ms": round(sub * 1e3, 3)}

    rows = compare_forms(tk, torch, x, dims, [1e-4], order, reps, nbytes, extra=recon)
    del x
    torch.cuda.empty_cache()
    return {"workload": "672x672x33x626 float32 Fourier-field tensor (512 modes per variable, |k|^-5/3 "
                        "energy spectrum, noise 1e-4; seed 5), mode order 3,2,0,1",
            "dims": dims, "bytes": nbytes, "generate_s": round(gen, 2), "reps": reps, "results": rows}


def batched_section(tk, torch, synthetic, reps):
    t0 = time.perf_counter()
    data = synthetic.small_batch(count=1024)
    gen = time.perf_counter() - t0
    xs = [torch.from_numpy(X.reshape(d[::-1])).to("cuda") for X, d in data]
    dims = [d for _, d in data]
    nbytes = sum(x.numel() * 4 for x in xs)
    eps = 1e-3
    rows = []
    for prec in ["fp64", "fp32", "bf16x6"]:
        print(f"# batched {prec}", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        b = tk.Batch(xs, eps, prec=prec, dims=dims)
        create_s = time.perf_counter() - t0
        b.run()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            b.run()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        eager_ms = sorted(ts)[len(ts) // 2] * 1e3
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            b.run()
        g.replay()
        torch.cuda.synchronize()
        ts = []
        for _ in range(max(reps, 5)):
            t0 = time.perf_counter()
            g.replay()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        graph_ms = sorted(ts)[len(ts) // 2] * 1e3
        ranks = b.ranks()
        # loop of single-tensor calls (same arithmetic)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        single_ranks = []
        for x, d in zip(xs, dims):
            t = tk.sthosvd(x, eps, prec=prec, dims=d)
            single_ranks.append(list(t.ranks))
            t.free()
        torch.cuda.synchronize()
        loop_ms = (time.perf_counter() - t0) * 1e3
        worst = 0.0
        for i in range(0, len(xs), 16):  # relative error on every 16th tensor
            t = b.item(i)
            xh = t.reconstruct(out_dtype=torch.float64)
            x64 = xs[i].to(torch.float64)
            e = float(torch.linalg.vector_norm((x64 - xh).reshape(-1)) / torch.linalg.vector_norm(x64.reshape(-1)))
            worst = max(worst, e)
            t.free()
        rows.append({"gram": prec, "graph_ms": round(graph_ms, 3), "eager_run_ms": round(eager_ms, 3),
                     "loop_of_single_calls_ms": round(loop_ms, 2), "speedup_vs_loop": round(loop_ms / graph_ms, 2),
                     "input_GBs": round(nbytes / graph_ms / 1e6, 2), "plan_create_s": round(create_s, 3),
                     "tiles_gram_chunks_ttm_tiles": list(b.tiles()),
                     "ranks_match_single_calls": sum(r == q for r, q in zip(ranks, single_ranks)),
                     "worst_relerr_sampled": worst, "within_1.05eps": bool(worst <= 1.05 * eps)})
        del g
        b.free()
    fp64_graph = rows[0]["graph_ms"]
    for r in rows:
        r["speedup_vs_fp64_graph"] = round(fp64_graph / r["graph_ms"], 3)
    del xs
    torch.cuda.empty_cache()
    return {"workload": "1024 float32 3-way tensors, sizes U{16..128}, Tucker ranks U{2..I/4}, noise 1e-4 "
                        "(seeds 4000+i), eps 1e-3, mode order 0,1,2", "count": 1024, "bytes": nbytes,
            "generate_s": round(gen, 2), "results": rows}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--eps", type=float, default=1e-4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sections", default="precision,large,batched",
                    help="extra sections after the headline line's own workload: precision,large,batched "
                         "(or none)")
    ap.add_argument("--form-reps", type=int, default=3, help="timed compressions per form in extra sections")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; run with --gpus 1",
              file=sys.stderr)
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

    tim = np.array([r[1] for r in recs])  # steps x N x 4
    med = np.median(tim, axis=0)
    flops = gram_flops(dims, ranks, order)
    gram_kernel_ms = [float(med[n][3]) for n in order]
    gram_tflops = sum(flops) / (sum(gram_kernel_ms) * 1e-3) / 1e12
    # dominant kernel: the mode-0 FP64 Gram (whole-triangle kernel), J^2 K flops per launch
    n0 = order[0]
    k0 = float(np.mean(tim[:, n0, 3]))
    ach = flops[0] / (k0 * 1e-3) / 1e12
    roofline = {"kernel": "gram_tri_kernel (FP64 Gram, mode %d, J=%d, K=%d)" % (n0, dims[n0], int(np.prod(dims)) // dims[n0]),
                "bound": "mfma", "achieved": round(ach, 3), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": round(ach / PEAK_FP64_TFLOPS, 4), "traffic": profiled_traffic(),
                "avg_launch_ms": round(k0, 5), "algorithmic_flops_per_launch": flops[0],
                "algorithmic_bytes_per_launch": nbytes}

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
    del x, out
    torch.cuda.empty_cache()
    sections = [s for s in args.sections.split(",") if s and s != "none"]
    if "precision" in sections:
        line["precision_form"] = precision_section(tk, torch, synthetic, args.form_reps)
    if "large" in sections:
        line["large_share"] = large_section(tk, torch, synthetic, max(1, args.form_reps - 1))
    if "batched" in sections:
        line["batched_form"] = batched_section(tk, torch, synthetic, args.form_reps)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(X, dims, args.eps, order, begin, end, nbytes)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
