#!/usr/bin/env python3
"""Benchmark of the ST-HOSVD hot path on one MI355X.

Headline workload (one GPU's share of a combustion-shaped grid): the
672x672x33x626 float32 Fourier-field tensor (2 space, 33 variables, 626 time
steps; 512 modes per variable with a |k|^-5/3 energy spectrum, relative noise
1e-4; seed 5, generated on the GPU), 37.3 GB resident in HBM.  One step is
the whole hot path on it:
  tucker_sthosvd (eps = 1e-4, mode order 3,2,0,1, FP64 Gram arithmetic:
  FP64 MFMA Grams and mode products, FP64 eigensolve and truncation)
  + full reconstruction into a preallocated float32 tensor
  + the 672x672x1x1 subrange reconstruction at variable 0, time step 313
  + tucker_free.
value = input bytes / time per step (GB/s).  `compress_ms` / `compress_GBs`
give the ST-HOSVD part alone (the metric's own definition).

Also on the same JSON line:
* gram_tflops: sum_n J_n^2 K_n (the symmetric count) over the main Gram
  kernels' time (HIP events recorded inside the library on the call's stream);
* roofline: the single longest kernel of the compression (by the library's
  per-launch HIP events over the timed steps), its algorithmic work per
  launch (Gram: J^2 K flops; mode product: 2 R J K flops) over its average
  launch time, against the FP64 MFMA peak; `traffic` from the committed
  rocprofv3 FETCH_SIZE/WRITE_SIZE summary of that kernel (null if its source
  changed since);
* cpu_baseline: the FP64 CPU oracle timed on the host on a down-scaled
  instance of the same generator (168x168x33x157, the same per-variable
  fields on a coarser grid), whole ST-HOSVD + reconstruction steps;
* large_forms: the headline tensor with the FP32, BF16x6 and BF16x3 Grams
  (and the AUTO selection when the library has it): median compression time
  of >= 3 runs, speed-up over the FP64 compression, ranks against FP64,
  relative error (explicit FP64 reconstruction) against 1.05 eps, largest
  principal-angle sine against the FP64 factors;
* decaying_200: the 200x200x200x16 float64 tensor (core 20x20x20x8, 0.7
  spectral decay, noise 1e-5) at eps 1e-4, ST-HOSVD + 50x50x50x16 subrange
  reconstruction, with its own roofline of the mode-0 Gram;
* precision_form: the 256x256x256x11x50 float32 combustion-shaped tensor at
  eps 1e-2..1e-5 with every Gram form;
* batched_form: 1024 independent float32 3-way tensors (sizes U{16..128},
  ranks U{2..I/4}, noise 1e-4) at eps 1e-3, one batched run replayed from a
  captured HIP graph against a loop of single-tensor calls, per Gram form;
  `hbm_floor_frac` = (input bytes read once at 8 TB/s) / replay time, the
  replay's fraction of its HBM floor.

`--sections none --no-cpu-baseline --steps 2 --warmup 1` is the short run
used under rocprofv3.
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
HBM_PEAK_BPS = 8.0e12  # MI355X HBM3E, bytes per second
PEAK_HBM_GBS = 8000.0
FORMS = ["fp64", "fp32", "bf16x6", "bf16x3"]
LARGE_DIMS = [672, 672, 33, 626]
LARGE_ORDER = [3, 2, 0, 1]
LARGE_SUB = ([0, 0, 0, 313], [672, 672, 1, 314])
CPU_SAMPLE_DIMS = [168, 168, 33, 157]


def log(msg):
    print("# " + msg, file=sys.stderr, flush=True)


def mode_work(dims, ranks, order):
    """Per processed mode n (in `order`): (n, J, K, R, L = product of the sizes before n, Gram
    flops J^2 K, TTM flops 2 R J K, Gram elements read, TTM elements read + written)."""
    cur = list(dims)
    out = []
    for n in order:
        K = 1
        for k, v in enumerate(cur):
            if k != n:
                K *= v
        J, R = cur[n], ranks[n]
        L = 1
        for v in cur[:n]:
            L *= v
        out.append({"mode": n, "J": J, "K": K, "R": R, "L": L, "gram_flops": J * J * K, "ttm_flops": 2 * R * J * K,
                    "gram_elems": J * K, "ttm_elems": (J + R) * K})
        cur[n] = R
    return out


def profiled_traffic(name):
    """HBM bytes per launch of a kernel from a committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary, or None if the kernel source changed since it was taken."""
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
        for f, h in zip(kv["source_file"].split(","), kv["source_sha256"].split(",")):
            src = open(os.path.join(ROOT, f.strip()), "rb").read()
            if hashlib.sha256(src).hexdigest() != h.strip():
                return None
        return int(kv["traffic_bytes_per_launch"])
    except (KeyError, OSError, ValueError):
        return None


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


def max_sin(torch, ref_factors, t, ref_ranks):
    out = []
    for n, U in enumerate(ref_factors):
        if t.ranks[n] != ref_ranks[n]:
            out.append(None)
            continue
        s = torch.linalg.svdvals(U.t() @ t.factor(n))
        out.append(float(torch.sqrt(torch.clamp(1 - s.min() ** 2, min=0.0))))
    return out


def run_form(tk, torch, x, dims, eps, order, prec, reps):
    """Median and minimum wall time of `reps` compressions (after one warm-up),
    returning the last handle."""
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
    return t, ts[len(ts) // 2] * 1e3, ts[0] * 1e3


def form_row(tk, torch, t, x, dims, eps, order, ms, ms_min, nbytes, ref):
    work = mode_work(dims, t.ranks, order)
    gk = [t.timings[w["mode"]].gram_kernel_ms for w in work]
    e = relerr_slabs(t, x, dims, torch)
    row = {"eps": eps, "gram": t.requested_precision, "ms": round(ms, 3), "ms_min": round(ms_min, 3),
           "input_GBs": round(nbytes / ms / 1e6, 2),
           "gram_tflops": round(sum(w["gram_flops"] for w in work) / (sum(gk) * 1e-3) / 1e12, 2),
           "ranks": list(t.ranks), "relerr": e, "within_1.05eps": bool(e <= 1.05 * eps),
           "gram_used": t.gram_precision,
           "per_mode_ms": {str(n): [round(t.timings[n].gram_ms, 3), round(t.timings[n].eig_ms, 3),
                                    round(t.timings[n].ttm_ms, 3)] for n in order}}
    if ref is None:
        row["speedup_vs_fp64"] = 1.0
        row["ranks_match_fp64"] = True
    else:
        row["speedup_vs_fp64"] = round(ref[2] / ms, 3)
        row["ranks_match_fp64"] = list(t.ranks) == ref[0]
        row["max_sin_angle_vs_fp64"] = max_sin(torch, ref[1], t, ref[0])
    return row


def compare_forms(tk, torch, x, dims, eps_list, order, reps, nbytes, forms=FORMS, fp64_ref=None):
    rows = []
    for eps in eps_list:
        ref = fp64_ref
        for prec in forms:
            log(f"{prec} eps={eps}")
            t, ms, ms_min = run_form(tk, torch, x, dims, eps, order, prec, reps)
            rows.append(form_row(tk, torch, t, x, dims, eps, order, ms, ms_min, nbytes,
                                 None if prec == "fp64" else ref))
            if prec == "fp64":
                ref = (list(t.ranks), [t.factor(n).clone() for n in range(len(dims))], ms)
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


def decaying_section(tk, torch, synthetic, steps, warmup, eps=1e-4):
    import numpy as np
    X, dims = synthetic.decaying_200()
    order = [0, 1, 2, 3]
    begin, end = [75, 75, 75, 0], [125, 125, 125, 16]
    x = torch.from_numpy(X.reshape(dims[::-1])).to("cuda")
    nbytes = x.numel() * x.element_size()
    out = torch.empty([e - b for b, e in zip(begin, end)][::-1], dtype=torch.float64, device="cuda")

    def step():
        t = tk.sthosvd(x, eps, mode_order=order)
        t.reconstruct(begin, end, out=out)
        rec = (list(t.ranks), [t.timings[n].gram_kernel_ms for n in range(4)])
        t.free()
        return rec

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs = [step() for _ in range(steps)]
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    ranks = recs[-1][0]
    work = mode_work(dims, ranks, order)
    k0 = float(np.mean([r[1][order[0]] for r in recs]))
    ach = work[0]["gram_flops"] / (k0 * 1e-3) / 1e12
    del x, out
    torch.cuda.empty_cache()
    return {"workload": "ST-HOSVD FP64 of a 200x200x200x16 float64 tensor (core 20x20x20x8, 0.7 spectral "
                        "decay, noise 1e-5; seed 2), eps=%g, order 0123, + 50x50x50x16 subrange "
                        "reconstruction at (75,75,75,0)" % eps,
            "steps": steps, "ms_per_step": round(ms, 4), "input_GBs": round(nbytes / ms / 1e6, 3), "ranks": ranks,
            "roofline": {"kernel": "gram_tri_kernel (FP64 Gram, mode 0, J=200, K=640000)", "bound": "mfma",
                         "achieved": round(ach, 3), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(ach / PEAK_FP64_TFLOPS, 4), "avg_launch_ms": round(k0, 5),
                         "traffic": profiled_traffic("gram_tri_kernel_200x200x200x16_traffic.md")}}


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
        log(f"batched {prec}")
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
                     "input_GBs": round(nbytes / graph_ms / 1e6, 2),
                     "hbm_floor_frac": round(nbytes / HBM_PEAK_BPS / (graph_ms / 1e3), 4),
                     "plan_create_s": round(create_s, 3),
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


def cpu_baseline(synthetic, eps, min_seconds=10.0):
    """The oracle on the down-scaled instance of the headline generator, whole
    ST-HOSVD + full reconstruction steps, for at least `min_seconds`."""
    import numpy as np

    import oracle
    X, dims = synthetic.fourier_fields(CPU_SAMPLE_DIMS)
    X = X.astype(np.float64)
    nbytes = X.size * 4  # the input as stored (float32)
    n, t0 = 0, time.perf_counter()
    while True:
        ref = oracle.sthosvd(X, dims, eps, LARGE_ORDER)
        oracle.reconstruct(ref)
        n += 1
        dt = time.perf_counter() - t0
        if dt >= min_seconds:
            break
    per = dt / n
    return {"value": round(nbytes / per / 1e9, 4), "unit": "GB/s", "cores": len(os.sched_getaffinity(0)),
            "kind": "oracle", "seconds_per_step": round(per, 3), "steps": n, "ranks": ref.ranks,
            "sample": "%d whole steps (ST-HOSVD eps=%g, order 3,2,0,1, + full reconstruction) of the "
                      "%s float32 Fourier-field tensor (the headline generator on a grid 1/4 the size in "
                      "space and time, %.2f GB), FP64 loops with OpenMP, %.1f s" %
                      (n, eps, "x".join(map(str, dims)), nbytes / 1e9, dt)}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--eps", type=float, default=1e-4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sections", default="forms,decaying,precision,batched",
                    help="extra sections after the headline: forms,decaying,precision,batched (or none)")
    ap.add_argument("--form-reps", type=int, default=3, help="timed compressions per form in extra sections")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (its sharding is a design, "
              "not code); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1901_06043_amd as tk
    import synthetic

    t0 = time.perf_counter()
    x, dims = synthetic.fourier_fields(LARGE_DIMS, device="cuda")
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    nbytes = x.numel() * x.element_size()
    order = LARGE_ORDER
    sub_b, sub_e = LARGE_SUB
    out = torch.empty_like(x)
    sub = torch.empty([e - b for b, e in zip(sub_b, sub_e)][::-1], dtype=torch.float32, device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]

    def step():
        ev[0].record()
        t = tk.sthosvd(x, args.eps, mode_order=order, prec="fp64")
        ev[1].record()
        t.reconstruct(out=out)
        ev[2].record()
        t.reconstruct(sub_b, sub_e, out=sub)
        ev[3].record()
        rec = {"ranks": list(t.ranks),
               "t": [(m.gram_ms, m.eig_ms, m.ttm_ms, m.gram_kernel_ms) for m in t.timings],
               "norm2": t.norm2, "disc": list(t.discarded)}
        t.free()
        torch.cuda.synchronize()
        rec["phase_ms"] = [ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2]), ev[2].elapsed_time(ev[3])]
        return rec

    log(f"headline: {dims} generated in {gen_s:.2f} s; {args.warmup} warm-up + {args.steps} timed steps")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed / args.steps * 1e3
    ranks = recs[-1]["ranks"]
    assert all(r["ranks"] == ranks for r in recs), "ranks changed between steps"

    tim = np.array([r["t"] for r in recs])  # steps x N x 4
    med = np.median(tim, axis=0)
    phase = np.median(np.array([r["phase_ms"] for r in recs]), axis=0)
    work = mode_work(dims, ranks, order)
    gram_kernel_ms = [float(med[w["mode"]][3]) for w in work]
    gram_tflops = sum(w["gram_flops"] for w in work) / (sum(gram_kernel_ms) * 1e-3) / 1e12
    # dominant kernel: the longest single launch among the Gram and mode-product kernels
    cands = []
    for w in work:
        n = w["mode"]
        cands.append(("gram", n, float(np.mean(tim[:, n, 3])), w["gram_flops"]))
        cands.append(("ttm", n, float(np.mean(tim[:, n, 2])), w["ttm_flops"]))
    kind, n_dom, k_ms, k_flops = max(cands, key=lambda c: c[2])
    wd = next(w for w in work if w["mode"] == n_dom)
    ach = k_flops / (k_ms * 1e-3) / 1e12
    es = 4 if n_dom == order[0] else 8  # the input (float32) feeds the first mode only
    if kind == "ttm":
        kname = "ttm_dma_kernel (FP64 mode product, mode %d, J=%d -> R=%d, K=%d)" % (n_dom, wd["J"], wd["R"], wd["K"])
        tfile = "ttm_dma_kernel_672x672x33x626_mode%d_traffic.md" % n_dom
        abytes = wd["J"] * wd["K"] * es + wd["R"] * wd["K"] * 8
    else:
        # the direct-load tile-pair kernel needs 16-byte aligned rows or columns
        L = wd["L"]
        dma = (wd["J"] * es % 16 == 0) if L == 1 else (L * es % 16 == 0 and (L >= 64 or L % (128 // es) == 0))
        kern = "gram_dma_kernel" if dma else "gram_mp_pair_kernel"
        kname = "%s (FP64 Gram, mode %d, J=%d, K=%d)" % (kern, n_dom, wd["J"], wd["K"])
        tfile = "%s_672x672x33x626_mode%d_traffic.md" % (kern, n_dom)
        abytes = wd["J"] * wd["K"] * es
    roofline = {"kernel": kname, "bound": "mfma", "achieved": round(ach, 3), "peak": PEAK_FP64_TFLOPS,
                "unit": "TFLOP/s", "frac": round(ach / PEAK_FP64_TFLOPS, 4), "traffic": profiled_traffic(tfile),
                "avg_launch_ms": round(k_ms, 4), "algorithmic_flops_per_launch": k_flops,
                "algorithmic_bytes_per_launch": abytes,
                "timing": "HIP events recorded by the library around this launch on the call's stream, "
                          "mean over the timed steps"}
    relerr = float(np.sqrt(max(sum(recs[-1]["disc"]), 0.0) / recs[-1]["norm2"]))
    line = {
        "metric": METRIC, "value": round(nbytes / (ms_per_step * 1e-3) / 1e9, 3), "unit": "GB/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "672x672x33x626 float32 Fourier-field tensor (512 modes per variable, |k|^-5/3 "
                               "spectrum, noise 1e-4; seed 5): ST-HOSVD eps=%g, mode order 3,2,0,1, FP64 Gram "
                               "arithmetic and FP64 eigensolve, + full float32 reconstruction + 672x672x1x1 "
                               "subrange reconstruction" % args.eps,
                   "dims": dims, "eps": args.eps, "mode_order": order, "ranks": ranks, "gram_precision": "fp64"},
        "compress_ms": round(float(phase[0]), 3),
        "compress_GBs": round(nbytes / (float(phase[0]) * 1e-3) / 1e9, 3),
        "reconstruct_full_ms": round(float(phase[1]), 3),
        "reconstruct_sub_ms": round(float(phase[2]), 3),
        "gram_tflops": round(gram_tflops, 3),
        "relerr_from_discarded": relerr,
        "per_mode_ms": {str(w["mode"]): {"gram": round(float(med[w["mode"]][0]), 3),
                                          "gram_kernel": round(float(med[w["mode"]][3]), 3),
                                          "eig": round(float(med[w["mode"]][1]), 3),
                                          "ttm": round(float(med[w["mode"]][2]), 3)} for w in work},
        "roofline": roofline,
    }
    del out, sub
    sections = [s for s in args.sections.split(",") if s and s != "none"]
    if "forms" in sections:
        log("large_forms: FP64 reference")
        t, ms, ms_min = run_form(tk, torch, x, dims, args.eps, order, "fp64", args.form_reps)
        rows = [form_row(tk, torch, t, x, dims, args.eps, order, ms, ms_min, nbytes, None)]
        ref = (list(t.ranks), [t.factor(n).clone() for n in range(len(dims))], ms)
        t.free()
        forms = [f for f in FORMS[1:]] + (["auto"] if "auto" in tk.PREC_CODES else [])
        rows += compare_forms(tk, torch, x, dims, [args.eps], order, args.form_reps, nbytes, forms=forms,
                              fp64_ref=ref)
        line["large_forms"] = {"workload": "the headline tensor, ST-HOSVD only", "reps": args.form_reps,
                               "results": rows}
    del x
    torch.cuda.empty_cache()
    if "decaying" in sections:
        log("decaying_200")
        line["decaying_200"] = decaying_section(tk, torch, synthetic, 20, 3)
    if "precision" in sections:
        line["precision_form"] = precision_section(tk, torch, synthetic, args.form_reps)
    if "batched" in sections:
        line["batched_form"] = batched_section(tk, torch, synthetic, args.form_reps)
    if not args.no_cpu_baseline:
        log("cpu_baseline")
        line["cpu_baseline"] = cpu_baseline(synthetic, args.eps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
