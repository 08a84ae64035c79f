"""Benchmark: throughput of whole DE generations on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--sections ...]

A step is one generation of the headline workload: shifted Rastrigin,
D = 1000, N = 2048, F = 0.5, CR = 0.9, NEC crossover, FP64 (index draws,
crossover mask, masked DE/rand/1 mutation, fitness, greedy selection and the
best-so-far update, with the population resident in HBM).  `value` is
pop*dim*gen/s = N * D * K / (time of K generations).

The same JSON line carries:
  roofline      the fused generation kernel's algorithmic bytes per launch
                over its event-timed average duration, against 8 TB/s;
  cpu_baseline  the CPU oracle on a bounded sample of the same workload;
  variants      bin / classic exp (three GPU mappings) / NEC x FP64 / FP32;
  rosenbrock    shifted Rosenbrock D = 10000, N = 8192, FP32 (HBM-sized);
  rotated       rotated ellipsoid D = 2048, N = 4096: product TFLOP/s per mode;
  batched       512 independent NEC runs of uneven shape in one launch;
  table1_masks  the crossover-only grid of Table 1 (masks written to HBM);
  fig456_nec_vs_pexp  the NEC / p-exp mask sweep of Figs 4-6;
  paper_runs    the three runs of Table 2 (Ackley, Griewank, Rosenbrock) end
                to end, with best value and generation reached.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"bf16": 2500.0, "fp32": 157.3, "fp64": 78.6}


def rho(xo: str, D: int, CR: float) -> float:
    """Expected fraction of crossed elements (mask density)."""
    if xo == "bin":
        return 1.0 / D + (1.0 - 1.0 / D) * CR
    if CR >= 1.0:
        return 1.0
    return (1.0 - CR ** D) / ((1.0 - CR) * D)


def alg_bytes(xo, N, D, CR, esz):
    """Algorithmic HBM bytes of one generation: read each parent row, read the
    three donor rows where the mask is set, write the trial into the other
    buffer: esz * N * D * (2 + 3 rho)."""
    return esz * N * D * (2.0 + 3.0 * rho(xo, D, CR))


def lower_bytes(xo, N, D, CR, esz, win):
    """Bytes the winners-only write-back needs: parent + masked donors +
    winner rows."""
    return esz * N * D * (1.0 + 3.0 * rho(xo, D, CR) + win)


def time_gens(gpu, K):
    import torch
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s)
    gpu.generation(K)
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def kernel_ms(gpu, K):
    """Average duration of the generation's main kernel (HIP events around each
    launch on the launch stream)."""
    import torch
    gpu.profile(True)
    gpu.generation(K)
    torch.cuda.synchronize()
    ms, n = gpu.profile_read()
    gpu.profile(False)
    return ms / max(n, 1)


def winners(gpu, K, run=0):
    """Average fraction of rows replaced per generation over K generations."""
    import numpy as np
    _, f0, _ = gpu.state(run)
    wins = 0
    for _ in range(K):
        _, fa, _ = gpu.state(run)
        gpu.generation(1)
        _, fb, _ = gpu.state(run)
        wins += int(np.count_nonzero(fb < fa))
    return wins / (K * len(f0))


def run_variant(cfg, K, W, prof_K, graph=False):
    """Times K generations (direct launches, or replayed 64-generation graphs
    when `graph`), then the main kernel's average duration with events."""
    import paper_2101_06599_amd as de
    gpu = de.DE([cfg])
    gpu.graph(graph)
    gpu.generation(W)
    ms = time_gens(gpu, K)
    kms = kernel_ms(gpu, prof_K)
    f, idx, g, _ = gpu.best(0)
    out = dict(ms_per_gen=ms / K, kernel_ms=kms,
               pop_dim_gen_s=cfg["N"] * cfg["D"] * K / (ms / 1e3), best=f, best_gen=g)
    return gpu, out


def traffic_from_profile(kernel_tag):
    """HBM bytes per launch measured with rocprofv3 counters, if the kernel
    source is unchanged since they were taken (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(kernel_tag)
    if not rec:
        return None
    if rec.get("source_sha") != source_sha():
        return None
    return rec.get("bytes_per_launch")


def source_sha():
    h = hashlib.sha256()
    for f in ("k_generation.hip", "de_device.h", "de_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_2101_06599_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def cpu_baseline(cfg, seconds=15.0):
    import oracle
    kw = {k: cfg[k] for k in ("N", "D", "F", "CR", "xo", "fn", "dtype", "lo", "hi", "olo", "ohi",
                              "seed")}
    # the oracle's per-individual loops use OpenMP with the process's default
    # thread count (OMP_NUM_THREADS, else the host's cores)
    threads = oracle.set_threads(0)
    r = oracle.Run(**kw)
    t0 = time.perf_counter()
    g = 0
    while True:
        r.generation(1)
        g += 1
        if time.perf_counter() - t0 > seconds:
            break
    dt = time.perf_counter() - t0
    return {"value": cfg["N"] * cfg["D"] * g / dt, "unit": "pop*dim*gen/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{g} generations of the same workload (N={cfg['N']}, D={cfg['D']}, "
                      f"{cfg['xo']}, {cfg['dtype']}) after initialisation, {threads} OpenMP "
                      f"threads, {dt:.1f} s"}


# Table 1 of the paper: total time (presumably seconds) of mask generation over
# Cr in {0.2, 0.4, 0.6, 0.8, 1.0} x 100 repeats, CuPy on a GTX 760:
# (D, Np) -> (CUDA-nec, CUDA-bin).
PAPER_TABLE1 = {(10, 100): (1.76, 6.99), (10, 1000): (1.18, 0.64), (10, 10000): (1.34, 0.94),
                (100, 100): (1.16, 0.66), (100, 1000): (1.23, 0.64), (100, 10000): (1.11, 1.36),
                (1000, 100): (0.66, 0.56), (1000, 1000): (1.07, 1.00), (1000, 10000): (4.31, 4.56),
                (10000, 100): (1.48, 0.97), (10000, 1000): (4.43, 3.91),
                (10000, 10000): (33.26, 39.14)}


def time_masks(torch, de, run, out, reps):
    """Seconds for masks of generations 1..reps of one run written to `out`:
    the ABI call is made directly with prepared arguments, so the loop adds
    little host time between the launches."""
    import ctypes as C
    h = de.DE([run])
    s = torch.cuda.current_stream()
    L, hh = de.lib(), h._h
    ptr, st = C.c_void_p(out.data_ptr()), C.c_void_p(s.cuda_stream)
    L.de_masks(hh, 0, 1, ptr, st)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s)
    for g in range(1, reps + 1):
        L.de_masks(hh, 0, g, ptr, st)
    e1.record(s)
    torch.cuda.synchronize()
    h.close()
    return e0.elapsed_time(e1) / 1e3


def table1(torch, de, reps=100):
    """The paper's crossover-only grid: masks of 100 generations per Cr, summed
    over the five Cr values, with the masks written to device memory."""
    res = {}
    for (D, N), (p_nec, p_bin) in PAPER_TABLE1.items():
        row = {}
        for xo, paper in (("nec", p_nec), ("bin", p_bin), ("exp", None)):
            total = 0.0
            out = torch.empty((N, D), dtype=torch.uint8, device="cuda:0")
            for CR in (0.2, 0.4, 0.6, 0.8, 1.0):
                total += time_masks(torch, de, dict(N=N, D=D, CR=CR, xo=xo, exp_impl="scan",
                                                    fn="sphere", dtype="fp32", seed=0), out, reps)
            del out
            row[xo] = {"total_s": total}
            if paper is not None:
                row[xo].update(paper_cuda_s=paper, speedup_vs_paper=paper / total)
        res[f"D{D}_N{N}"] = row
    return res


def fig456(torch, de, reps=100):
    """Figs 4-6 of the paper: crossover-mask time of NEC against the classic
    exponential crossover with one work-item per individual (p-exp), for
    N in {100, 1000, 5000} and D from 2 to 5000, 100 generations per point.
    The figures do not name Cr: each point sums Cr in {0.2, ..., 1.0} as
    Table 1 does.  The wavefront-scan mapping of the classic crossover is
    timed beside them."""
    res = {}
    for N in (100, 1000, 5000):
        for D in (2, 10, 50, 100, 500, 1000, 2000, 5000):
            row = {}
            for name, xo, impl in (("nec", "nec", "lane"), ("p_exp", "exp", "job"),
                                   ("exp_scan", "exp", "scan")):
                total = 0.0
                out = torch.empty((N, D), dtype=torch.uint8, device="cuda:0")
                for CR in (0.2, 0.4, 0.6, 0.8, 1.0):
                    total += time_masks(torch, de, dict(N=N, D=D, CR=CR, xo=xo, exp_impl=impl,
                                                        fn="sphere", dtype="fp32", seed=0),
                                        out, reps)
                row[name + "_s"] = total
                del out
            row["p_exp_over_nec"] = row["p_exp_s"] / row["nec_s"]
            res[f"N{N}_D{D}"] = row
    return res


# Tables 3-5 of the paper (Sec. 4, GTX 760, CuPy): the CUDA-DE rows,
# variant -> (best value, generation of the best, seconds for the whole run).
# "L" is the new exponential crossover (our "nec").
PAPER_TABLE345 = {
    "ackley": {"nec": (2.62e-05, 29991, 323.97), "bin": (2.28e-04, 29983, 321.45)},
    "griewank": {"nec": (1.73e-16, 19936, 149.03), "bin": (2.22e-16, 6041, 143.95)},
    "rosenbrock": {"nec": (1.16e-07, 9996, 58.92), "bin": (9.93e-10, 10000, 56.72)},
}


def paper_runs(torch, de, synth, seeds=(0, 1, 2, 3, 4)):
    """The three runs of Table 2 end to end (every generation, FP64) over
    several seeds: time per run and the best value and generation each seed
    reaches.  The paper's CUDA-DE figures sit beside them as context (other
    hardware, other random streams, one run each)."""
    res = {}
    for name, base in synth.TABLE2.items():
        for xo in ("nec", "bin"):
            times, vals, gens_best = [], [], []
            for seed in seeds:
                cfg = dict(base, xo=xo, seed=seed)
                gens = cfg.pop("gens")
                h = de.DE([cfg])
                s = torch.cuda.current_stream()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                torch.cuda.synchronize()
                e0.record(s)
                h.generation(gens)
                e1.record(s)
                torch.cuda.synchronize()
                times.append(e0.elapsed_time(e1) / 1e3)
                f, _, g, _ = h.best(0)
                vals.append(f)
                gens_best.append(g)
                h.close()
            pv, pg, pt = PAPER_TABLE345[name][xo]
            t = sum(times) / len(times)
            res[f"{name}_D{base['D']}_N{base['N']}_{xo}"] = {
                "generations": base["gens"], "seeds": list(seeds), "time_s_mean": t,
                "us_per_gen": t / base["gens"] * 1e6, "best_values": vals,
                "best_value_median": sorted(vals)[len(vals) // 2], "best_gens": gens_best,
                "paper_cuda": {"best_value": pv, "best_gen": pg, "time_s": pt},
                "speedup_vs_paper": pt / t}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--sections", default="all",
                    help="comma list of: head (headline only), variants, rosenbrock, rotated, "
                         "batched, table1, fig456, paper_runs, tuning, cpu, copy (default: all "
                         "but copy)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(there is no cross-GPU path)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2101_06599_amd as de
    from paper_2101_06599_amd import synth
    torch.cuda.set_device(0)
    de.lib()
    secs = set(args.sections.split(",")) if args.sections != "all" else {
        "variants", "rosenbrock", "rotated", "batched", "table1", "fig456", "paper_runs", "tuning",
        "cpu"}
    K, W = args.steps, args.warmup

    head = dict(synth.RASTRIGIN_D1000, xo="nec", dtype="fp64")
    gpu, h = run_variant(head, K, W, prof_K=min(K, 200))
    win = winners(gpu, 20)
    gpu.close()
    g_graph, h_graph = run_variant(head, K, W, prof_K=10, graph=True)
    g_graph.close()
    N, D, CR = head["N"], head["D"], head["CR"]
    ab = alg_bytes("nec", N, D, CR, 8)
    achieved = ab / (h["kernel_ms"] * 1e-3) / 1e9
    traffic = traffic_from_profile("gen_rastrigin_nec_fp64_2048x1000")
    out = {
        "metric": "pop*dim*gen/s (shifted Rastrigin D=1000 N=2048, NEC, FP64)",
        "value": h["pop_dim_gen_s"], "unit": "pop*dim*gen/s", "n_gpus": 1, "steps": K,
        "warmup": W, "ms_per_step": h["ms_per_gen"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "shifted Rastrigin, D=1000, N=2048, F=0.5, CR=0.9, "
                               "DE/rand/1/NEC, FP64, x~U[-5.12,5.12], o~U[-4,4], Philox seed 0",
                   "N": N, "D": D, "generation": "one generation per step",
                   "launch": "one kernel per generation, stream-ordered"},
        "graph_replay_ms_per_step": h_graph["ms_per_gen"],
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_generation<double, RASTRIGIN, NEC>",
                     "kernel_ms": h["kernel_ms"], "alg_bytes_per_launch": ab,
                     "lower_bound_bytes_per_launch": lower_bytes("nec", N, D, CR, 8, win),
                     "winner_fraction": win},
    }

    if "variants" in secs:
        var = {}
        for dtype in ("fp64", "fp32"):
            es = 8 if dtype == "fp64" else 4
            for xo, impl in (("nec", "lane"), ("bin", "lane"), ("exp", "scan"), ("exp", "lane"),
                             ("exp", "job")):
                cfg = dict(synth.RASTRIGIN_D1000, xo=xo, dtype=dtype, exp_impl=impl)
                kk = K if impl != "job" else max(10, K // 10)
                g2, r = run_variant(cfg, kk, min(W, 10), prof_K=min(kk, 100))
                g2.close()
                name = f"{xo}{'' if xo != 'exp' else '-' + impl}_{dtype}"
                byt = alg_bytes(xo, cfg["N"], cfg["D"], cfg["CR"], es)
                r["hbm_frac_kernel"] = byt / (r["kernel_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS
                var[name] = r
        for dtype in ("fp64", "fp32"):
            nec = var[f"nec_{dtype}"]["ms_per_gen"]
            var[f"ratio_nec_over_bin_time_{dtype}"] = nec / var[f"bin_{dtype}"]["ms_per_gen"]
            var[f"speedup_nec_vs_exp_job_{dtype}"] = var[f"exp-job_{dtype}"]["ms_per_gen"] / nec
            var[f"speedup_nec_vs_exp_scan_{dtype}"] = var[f"exp-scan_{dtype}"]["ms_per_gen"] / nec
        out["variants"] = var

    if "rosenbrock" in secs:
        ros = {}
        for xo, impl in (("nec", "lane"), ("bin", "lane"), ("exp", "scan")):
            cfg = dict(synth.ROSENBROCK_D10000, xo=xo, exp_impl=impl)
            g2, r = run_variant(cfg, 100, 5, prof_K=50)
            g2.close()
            byt = alg_bytes(xo, cfg["N"], cfg["D"], cfg["CR"], 4)
            r["hbm_frac_kernel"] = byt / (r["kernel_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS
            r["alg_bytes_per_gen"] = byt
            ros[xo if xo != "exp" else "exp-scan"] = r
        out["rosenbrock_d10000_n8192_fp32"] = ros

    if "rotated" in secs:
        rot_np = synth.rotation(2048, 0)
        rot = torch.as_tensor(rot_np, dtype=torch.float64, device="cuda:0")
        rr = {}
        for mm, dtype, mdt, mult in (("bf16x6", "fp32", "bf16", 6), ("bf16x3", "fp32", "bf16", 3),
                                     ("fp32", "fp32", "fp32", 1), ("fp64", "fp64", "fp64", 1)):
            cfg = dict(synth.ELLIPSOID_D2048, xo="nec", dtype=dtype, mm=mm, rot=rot)
            g2, r = run_variant(cfg, 20, 2, prof_K=10)
            g2.close()
            flops = 2.0 * cfg["N"] * cfg["D"] ** 2
            tf = flops / (r["kernel_ms"] * 1e-3) / 1e12
            r.update(algorithmic_tflops=tf, executed_tflops=tf * mult,
                     mfma_peak_tflops=MFMA_PEAK_TFLOPS[mdt],
                     mfma_frac=tf * mult / MFMA_PEAK_TFLOPS[mdt])
            rr[mm] = r
        out["rotated_ellipsoid_d2048_n4096"] = rr

    if "batched" in secs:
        cfgs = synth.batch_table(512, seed=0)
        g2 = de.DE(cfgs)
        g2.generation(5)
        kb = 100
        ms = time_gens(g2, kb)
        kms = kernel_ms(g2, 50)
        elems = sum(c["N"] * c["D"] for c in cfgs)
        byt = sum(alg_bytes("nec", c["N"], c["D"], c["CR"], 4) for c in cfgs)
        g2.close()
        # the same generations replayed from captured 64-generation graphs
        g3 = de.DE(cfgs)
        g3.graph(True)
        g3.generation(64)  # capture
        ms_graph = time_gens(g3, 128)
        g3.close()
        out["batched_512_runs_nec_fp32"] = {
            "runs": 512, "elements": elems, "ms_per_gen": ms / kb, "kernel_ms": kms,
            "pop_dim_gen_s": elems * kb / (ms / 1e3),
            "hbm_frac_kernel": byt / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "graph_replay_ms_per_gen": ms_graph / 128}

    if "table1" in secs:
        out["table1_masks"] = table1(torch, de)

    if "fig456" in secs:
        out["fig456_nec_vs_pexp"] = fig456(torch, de)

    if "paper_runs" in secs:
        out["paper_runs"] = paper_runs(torch, de, synth)

    if "tuning" in secs:
        from paper_2101_06599_amd.tune import tune_tpr
        tun = {}
        for name, cfg in (("rastrigin_d1000_n2048_nec_fp64", head),
                          ("rosenbrock_d10000_n8192_nec_fp32",
                           dict(synth.ROSENBROCK_D10000, xo="nec"))):
            best, table = tune_tpr(cfg, gens=64, use_cache=False)
            tun[name] = {"best_tpr": best, "ms_per_gen_by_tpr": table}
        out["tuning"] = tun

    if "copy" in secs:
        # counter calibration: an elementwise kernel that reads and writes a
        # known number of bytes (b = -a over 256 MiB)
        n = 256 << 20
        a = torch.ones(n // 4, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(5):
            torch.neg(a, out=b)
        torch.cuda.synchronize()
        out["copy_calibration"] = {"kernel": "torch.neg over float32", "bytes_read": n,
                                   "bytes_written": n, "launches": 5}

    if "cpu" in secs:
        out["cpu_baseline"] = cpu_baseline(head, args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
