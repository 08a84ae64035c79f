"""Benchmark: throughput of whole DE generations on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--sections ...]

A step is one generation of the headline workload: shifted Rastrigin,
D = 1000, N = 2048, F = 0.5, CR = 0.9, NEC crossover, FP64 (index draws,
crossover mask, masked DE/rand/1 mutation, fitness, greedy selection and the
best-so-far update, with the population resident in device memory).  `value`
is pop*dim*gen/s = N * D * K / (time of K generations launched one kernel at
a time); `graph_replay_ms_per_step` gives the same generations replayed from
captured graphs of 64.

The JSON line (one line on stdout) carries, after the standard fields, the
paper's own experiments in short form (Table 1 masks, Figs 4-6, the Table 2
runs), then the benchmark workloads (C1 sphere, C2 variants, C4 batched, C3
rotated, C5 large Rosenbrock), the roofline of the headline kernel and the CPU
oracle baseline, so that the end of the line holds the main figures.

Byte bases of every `frac_*` figure (fraction of the 8 TB/s HBM peak):
  frac_alg  algorithmic bytes s N D (2 + 3 rho): read the parent row, read the
            three donors where the mask is set, write the trial row;
  frac_min  bytes any design must move, s N D (1 + 3 rho + rho w): parent,
            masked donors, and the masked elements of the w winners;
  frac_ctr  FETCH_SIZE + WRITE_SIZE per launch from rocprofv3 counters
            (profiles/traffic.json, only while the kernel sources are the ones
            the counters were taken on), else null.
frac_alg charges a trial write for every row while the kernels write only
winners, so it can exceed frac_ctr; each is reported with its basis.

Counter summaries: `python bench.py --counters DIR` prints per-kernel averages
of rocprofv3 CSV output found under DIR (used for the files in profiles/).
"""
from __future__ import annotations

import argparse
import csv
import glob
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


def r4(x):
    """Four significant digits (keeps the JSON line short)."""
    if x is None or isinstance(x, (bool, int, str)):
        return x
    if not math.isfinite(x) or x == 0:
        return x
    return float(f"{x:.4g}")


def rho(xo: str, D: int, CR: float) -> float:
    """Expected fraction of crossed elements (mask density)."""
    if xo == "bin":
        return 1.0 / D + (1.0 - 1.0 / D) * CR
    if CR >= 1.0:
        return 1.0
    return (1.0 - CR ** D) / ((1.0 - CR) * D)


def alg_bytes(xo, N, D, CR, esz):
    """Algorithmic bytes of one generation: esz N D (2 + 3 rho)."""
    return esz * N * D * (2.0 + 3.0 * rho(xo, D, CR))


def min_bytes(xo, N, D, CR, esz, win):
    """Bytes any design must move: esz N D (1 + 3 rho + rho w)."""
    r = rho(xo, D, CR)
    return esz * N * D * (1.0 + 3.0 * r + r * win)


def source_sha():
    """Hash of the kernel sources (counter figures are void once it changes)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2101_06599_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        h.update(f.encode())
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


_TRAFFIC = None


def traffic(tag):
    """Counter bytes per launch of a kernel, if measured on these sources."""
    global _TRAFFIC
    if _TRAFFIC is None:
        path = os.path.join(ROOT, "profiles", "traffic.json")
        _TRAFFIC = json.load(open(path)) if os.path.exists(path) else {}
    rec = _TRAFFIC.get(tag)
    if not rec or rec.get("source_sha") != source_sha():
        return None
    return rec.get("bytes_per_launch")


def fracs(tag, xo, N, D, CR, esz, win, kms):
    sec = kms * 1e-3
    ab = alg_bytes(xo, N, D, CR, esz)
    mb = min_bytes(xo, N, D, CR, esz, win) if win is not None else None
    tb = traffic(tag)
    out = {"frac_alg": ab / sec / 1e9 / HBM_PEAK_GBS,
           "frac_min": None if mb is None else mb / sec / 1e9 / HBM_PEAK_GBS,
           "frac_ctr": None if tb is None else tb / sec / 1e9 / HBM_PEAK_GBS}
    return {k: r4(v) for k, v in out.items()}


def device_info(torch):
    """What the box reports about the GPU the figures were taken on."""
    p = torch.cuda.get_device_properties(0)
    return {"arch": p.gcnArchName.split(":")[0], "cus": p.multi_processor_count,
            "hbm_GiB": round(p.total_memory / 2**30), "l2_MiB": round(p.L2_cache_size / 2**20, 1)}


def sync():
    import torch
    torch.cuda.synchronize()


def time_gens(gpu, K):
    """Milliseconds for K generations (HIP events on the launch stream,
    synchronised before and after).  The library is called through the C ABI
    directly, with its arguments prepared before the first event, so that the
    Python binding's own overhead stays out of the timed span."""
    import ctypes as C
    import torch
    import paper_2101_06599_amd as de
    s = torch.cuda.current_stream()
    L, h, st = de.lib(), gpu._h, C.c_void_p(s.cuda_stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s)
    rc = L.de_generation(h, int(K), st)
    e1.record(s)
    torch.cuda.synchronize()
    if rc != 0:
        raise RuntimeError(f"de_generation: {L.de_last_error(h).decode()}")
    return e0.elapsed_time(e1)


def kernel_ms(gpu, K):
    """Average duration of the generation's main kernel (HIP events around the
    launches on the launch stream)."""
    gpu.profile(True)
    gpu.generation(K)
    sync()
    ms, n = gpu.profile_read()
    gpu.profile(False)
    return ms / max(n, 1)


def winners(gpu, K, run=0):
    """Average fraction of rows replaced per generation over K generations."""
    import numpy as np
    wins, n = 0, 0
    fa = gpu.fitness(run)
    for _ in range(K):
        gpu.generation(1)
        fb = gpu.fitness(run)
        wins += int(np.count_nonzero(fb < fa))
        n += len(fa)
        fa = fb
    return wins / n


def run_variant(cfg, K, W, prof_K, win_K=0, best_calls=0):
    import time
    import paper_2101_06599_amd as de
    gpu = de.DE([cfg])
    gpu.generation(W)
    ms = time_gens(gpu, K)
    kms = kernel_ms(gpu, prof_K)
    win = winners(gpu, win_K) if win_K else None
    best_ms = None
    for _ in range(best_calls):  # de_best: FP64 recompute of the best vector, host copy included
        t0 = time.perf_counter()
        gpu.best()
        t = (time.perf_counter() - t0) * 1e3
        best_ms = t if best_ms is None else min(best_ms, t)
    gpu.close()
    return {"ms_per_gen": ms / K, "kernel_ms": kms, "win": win, "best_ms": best_ms,
            "pop_dim_gen_s": cfg["N"] * cfg["D"] * K / (ms / 1e3)}


# ---- the paper's experiments (short form) -----------------------------------

# Table 1: total seconds of mask generation over Cr in {0.2, ..., 1.0} x 100
# repeats, CuPy on a GTX 760: (D, Np) -> (CUDA-nec, CUDA-bin).
PAPER_TABLE1 = {(10, 100): (1.76, 6.99), (10, 1000): (1.18, 0.64), (10, 10000): (1.34, 0.94),
                (100, 100): (1.16, 0.66), (100, 1000): (1.23, 0.64), (100, 10000): (1.11, 1.36),
                (1000, 100): (0.66, 0.56), (1000, 1000): (1.07, 1.00), (1000, 10000): (4.31, 4.56),
                (10000, 100): (1.48, 0.97), (10000, 1000): (4.43, 3.91),
                (10000, 10000): (33.26, 39.14)}


def time_masks(torch, de, run, out, reps):
    """Seconds for masks of generations 1..reps of one run written to `out`
    (the ABI is called directly, so the loop adds little host time)."""
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
    """Table 1's grid: seconds for masks of 100 generations per Cr, summed over
    the five Cr values (nec, bin, exp-scan), with the paper's CUDA times as the
    speed-up basis; and the 100 MB launch at N = D = 10^4 as a fraction of the
    HBM write bandwidth."""
    res, sp = {}, []
    big = {}
    for (D, N), (p_nec, p_bin) in PAPER_TABLE1.items():
        row = []
        out = torch.empty((N, D), dtype=torch.uint8, device="cuda:0")
        for xo in ("nec", "bin", "exp"):
            tot = 0.0
            for CR in (0.2, 0.4, 0.6, 0.8, 1.0):
                t = time_masks(torch, de, dict(N=N, D=D, CR=CR, xo=xo, exp_impl="scan",
                                               fn="sphere", dtype="fp32", seed=0), out, reps)
                tot += t
                if (D, N) == (10000, 10000):
                    big.setdefault(xo, []).append(t / reps)
            row.append(r4(tot))
        del out
        res[f"D{D}_N{N}"] = row
        sp += [p_nec / row[0], p_bin / row[1]]
    per = {xo: sum(v) / len(v) for xo, v in big.items()}
    return {"cols": "nec, bin, exp-scan seconds (5 Cr x 100 generations)", "cells": res,
            "speedup_vs_paper_cuda": [r4(min(sp)), r4(max(sp))],
            "n10000_d10000_us_per_launch": {k: r4(v * 1e6) for k, v in per.items()},
            "n10000_d10000_frac_write": {k: r4(1e8 / v / 1e9 / HBM_PEAK_GBS) for k, v in per.items()}}


def masks10k(torch, de, reps=20):
    """The 100 MB mask launch at N = D = 10^4 alone (Table 1's largest cell),
    per crossover over the five Cr values: microseconds per launch and the
    fraction of the HBM peak on the bytes written, and on the counter bytes
    when they were taken on these sources."""
    out = torch.empty((10000, 10000), dtype=torch.uint8, device="cuda:0")
    res = {}
    for xo in ("nec", "bin", "exp"):
        t = sum(time_masks(torch, de, dict(N=10000, D=10000, CR=CR, xo=xo, exp_impl="scan",
                                           fn="sphere", dtype="fp32", seed=0), out, reps)
                for CR in (0.2, 0.4, 0.6, 0.8, 1.0)) / (5 * reps)
        name = xo if xo != "exp" else "exp-scan"
        tb = traffic(f"masks_{name}")
        res[name] = {"us": r4(t * 1e6), "frac_write": r4(1e8 / t / 1e9 / HBM_PEAK_GBS),
                     "frac_ctr": None if tb is None else r4(tb / t / 1e9 / HBM_PEAK_GBS)}
    # the practical write ceiling beside them: torch's fill of the same 100 MB
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out.fill_(1)
    torch.cuda.synchronize()
    e0.record(s)
    for _ in range(reps):
        out.fill_(1)
    e1.record(s)
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / reps
    res["torch_fill"] = {"us": r4(t * 1e6), "frac_write": r4(1e8 / t / 1e9 / HBM_PEAK_GBS)}
    del out
    return res


def fig456(torch, de, reps=100):
    """Figs 4-6: mask time of the job-per-individual classic exponential
    crossover (p-exp) and of the wavefront-scan one over NEC, N in {100, 1000,
    5000}, D from 2 to 5000 (each point sums Cr in {0.2, ..., 1.0} like
    Table 1)."""
    res = {}
    for N in (100, 1000, 5000):
        ratios = []
        for D in (2, 10, 100, 1000, 5000):
            tt = {}
            out = torch.empty((N, D), dtype=torch.uint8, device="cuda:0")
            for name, xo, impl in (("nec", "nec", "lane"), ("pexp", "exp", "job"),
                                   ("scan", "exp", "scan")):
                tt[name] = sum(time_masks(torch, de, dict(N=N, D=D, CR=CR, xo=xo, exp_impl=impl,
                                                          fn="sphere", dtype="fp32", seed=0),
                                          out, reps) for CR in (0.2, 0.4, 0.6, 0.8, 1.0))
            del out
            ratios.append([D, r4(tt["pexp"] / tt["nec"]), r4(tt["scan"] / tt["nec"])])
        res[f"N{N}"] = ratios
    return {"cols": "D, p-exp/nec, exp-scan/nec (time ratios)", "points": res}


# Tables 3-5 (Sec. 4, GTX 760, CuPy), CUDA-DE rows: (best value, best gen, s).
PAPER_TABLE345 = {
    "ackley": {"nec": (2.62e-05, 29991, 323.97), "bin": (2.28e-04, 29983, 321.45)},
    "griewank": {"nec": (1.73e-16, 19936, 149.03), "bin": (2.22e-16, 6041, 143.95)},
    "rosenbrock": {"nec": (1.16e-07, 9996, 58.92), "bin": (9.93e-10, 10000, 56.72)},
}


def paper_runs(torch, de, synth, seeds=(0, 1, 2, 3, 4)):
    """The three runs of Table 2 end to end (every generation, FP64) over five
    seeds: mean seconds per run, median best value, and the speed-up over the
    paper's CUDA-DE time for the same run (other hardware, other streams).
    Replaying these runs from graphs of 500 generations measured no faster
    (their kernels, not the launches, set the pace)."""
    res = {}
    for name, base in synth.TABLE2.items():
        for xo in ("nec", "bin"):
            times, vals = [], []
            for seed in seeds:
                cfg = dict(base, xo=xo, seed=seed)
                gens = cfg.pop("gens")
                h = de.DE([cfg])
                times.append(time_gens(h, gens) / 1e3)
                vals.append(h.best(0)[0])
                h.close()
            t = sum(times) / len(times)
            res[f"{name}_{xo}"] = [r4(t), r4(sorted(vals)[len(vals) // 2]),
                                   r4(PAPER_TABLE345[name][xo][2] / t)]
    return {"cols": "s per run, median best value, speed-up vs paper CUDA-DE", "runs": res}


# ---- benchmark workloads -------------------------------------------------------

def c1_sphere(synth):
    """C1: sphere D = 10, N = 50, FP64, 100 generations per crossover."""
    import paper_2101_06599_amd as de
    out = {}
    for name, xo, impl in (("bin", "bin", "lane"), ("exp", "exp", "lane"), ("exp-scan", "exp", "scan"),
                           ("nec", "nec", "lane")):
        cfg = dict(synth.SPHERE_D10, xo=xo, exp_impl=impl)
        gpu = de.DE([cfg])
        gpu.generation(10)
        ms = time_gens(gpu, 100)
        f = gpu.best(0)[0]
        gpu.close()
        out[name] = [r4(ms / 100 * 1e3), r4(cfg["N"] * cfg["D"] * 100 / (ms / 1e3)), r4(f)]
    return {"cols": "us per generation, pop*dim*gen/s, best after 110 generations", "runs": out}


def c2_variants(synth, K, W, only=None):
    """C2: the headline shape under every crossover and exp mapping, FP64 and
    FP32 (`only`: a subset of the variant names, for counter runs in which
    each kernel must appear under one variant)."""
    out = {}
    for dtype in ("fp64", "fp32"):
        es = 8 if dtype == "fp64" else 4
        for xo, impl in (("nec", "lane"), ("bin", "lane"), ("exp", "scan"), ("exp", "lane"),
                         ("exp", "job")):
            name = f"{xo}{'' if xo != 'exp' else '-' + impl}_{dtype}"
            if only is not None and name not in only:
                continue
            cfg = dict(synth.RASTRIGIN_D1000, xo=xo, dtype=dtype, exp_impl=impl)
            kk = K if impl != "job" else max(10, K // 10)
            r = run_variant(cfg, kk, min(W, 10), prof_K=100, win_K=10)
            f = fracs(f"c2_{name}", xo, cfg["N"], cfg["D"], cfg["CR"], es, r["win"],
                      r["kernel_ms"])
            out[name] = [r4(r["ms_per_gen"]), r4(r["kernel_ms"]), r4(r["pop_dim_gen_s"]),
                         f["frac_alg"], f["frac_min"], f["frac_ctr"]]
    for dtype in ("fp64", "fp32"):
        if f"nec_{dtype}" not in out:
            continue
        nec = out[f"nec_{dtype}"][0]
        for other, key in (("bin", "nec_over_bin_time"), ("exp-job", "exp-job_over_nec_time"),
                           ("exp-scan", "exp-scan_over_nec_time")):
            if f"{other}_{dtype}" in out:
                t = out[f"{other}_{dtype}"][0]
                out[f"{key}_{dtype}"] = r4(nec / t if other == "bin" else t / nec)
    return dict({"cols": "ms per generation, kernel ms, pop*dim*gen/s, frac_alg, frac_min, "
                         "frac_ctr"}, **out)


def c5_rosenbrock(synth):
    """C5: shifted Rosenbrock D = 10^4, N = 8192, FP32 (2 x 328 MB of
    population: beyond the 256 MB Infinity Cache)."""
    out = {}
    for xo, impl in (("nec", "lane"), ("bin", "lane"), ("exp", "scan")):
        cfg = dict(synth.ROSENBROCK_D10000, xo=xo, exp_impl=impl)
        r = run_variant(cfg, 100, 5, prof_K=50, win_K=5)
        name = xo if xo != "exp" else "exp-scan"
        d = {"ms": r4(r["ms_per_gen"]), "kernel_ms": r4(r["kernel_ms"]),
             "pdg_s": r4(r["pop_dim_gen_s"])}
        d.update(fracs(f"c5_{name}", xo, cfg["N"], cfg["D"], cfg["CR"], 4, r["win"],
                       r["kernel_ms"]))
        out[name] = d
    out["nec_over_bin_time"] = r4(out["nec"]["ms"] / out["bin"]["ms"])
    return out


def c3_rotated(torch, synth):
    """C3: rotated ellipsoid D = 2048, N = 4096: the product's time per
    generation and its rate against the matrix-core peak of the type it
    executes (split-bf16 executes 3 or 6 bf16 products)."""
    rot = torch.as_tensor(synth.rotation(2048, 0), dtype=torch.float64, device="cuda:0")
    out = {}
    for mm, dtype, mdt, mult in (("bf16x6", "fp32", "bf16", 6), ("bf16x3", "fp32", "bf16", 3),
                                 ("fp32", "fp32", "fp32", 1), ("fp64", "fp64", "fp64", 1)):
        cfg = dict(synth.ELLIPSOID_D2048, xo="nec", dtype=dtype, mm=mm, rot=rot)
        r = run_variant(cfg, 20, 2, prof_K=30, best_calls=3)
        flops = 2.0 * cfg["N"] * cfg["D"] ** 2
        tf = flops / (r["kernel_ms"] * 1e-3) / 1e12
        out[mm] = {"ms_per_gen": r4(r["ms_per_gen"]), "product_ms": r4(r["kernel_ms"]),
                   "alg_tflops": r4(tf), "exec_tflops": r4(tf * mult),
                   "mfma_frac": r4(tf * mult / MFMA_PEAK_TFLOPS[mdt]), "de_best_ms": r4(r["best_ms"]),
                   "ctr_MB": None if traffic(f"c3_{mm}") is None else r4(traffic(f"c3_{mm}") / 1e6)}
    return out


def c4_batched(synth):
    """C4: 512 NEC runs of uneven shape, FP32, one launch per generation;
    500 generations replayed from one captured graph, and direct launches."""
    import paper_2101_06599_amd as de
    cfgs = synth.batch_table(512, seed=0)
    elems = sum(c["N"] * c["D"] for c in cfgs)
    g2 = de.DE(cfgs)
    g2.generation(5)
    ms = time_gens(g2, 100)
    kms = kernel_ms(g2, 50)
    g2.close()
    g3 = de.DE(cfgs)
    g3.graph(500)
    g3.generation(500)  # replays the 500-generation graph captured above once
    ms_graph = time_gens(g3, 500)
    g3.close()
    byt = sum(alg_bytes("nec", c["N"], c["D"], c["CR"], 4) for c in cfgs)
    return {"runs": 512, "elements": elems, "ms_direct": r4(ms / 100), "kernel_ms": r4(kms),
            "ms_graph500": r4(ms_graph / 500), "pdg_s_graph500": r4(elems * 500 / (ms_graph / 1e3)),
            "pdg_s_direct": r4(elems * 100 / (ms / 1e3)),
            "frac_alg": r4(byt / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS),
            "frac_ctr": None if traffic("c4_batched") is None
            else r4(traffic("c4_batched") / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS)}


# ---- CPU oracle ------------------------------------------------------------------

def _timed(fn):
    t0 = time.perf_counter()
    fn()
    return time.perf_counter() - t0


def cpu_baseline(synth, head, seconds):
    """The oracle (plain sequential C, OpenMP over individuals) on bounded
    samples: the headline workload with all host threads and with one, and
    per-generation rates of the other workloads on prefixes (C1 whole, C5 one
    generation, C3 one generation of 64 rows, C4 two generations of every run)."""
    import numpy as np

    import oracle
    keys = ("N", "D", "F", "CR", "xo", "fn", "dtype", "lo", "hi", "olo", "ohi", "seed")
    cores = oracle.set_threads(0)

    def rate_head(threads, budget):
        oracle.set_threads(threads)
        r = oracle.Run(**{k: head[k] for k in keys})
        g, t0 = 0, time.perf_counter()
        while True:
            r.generation(1)
            g += 1
            if time.perf_counter() - t0 > budget:
                break
        return head["N"] * head["D"] * g / (time.perf_counter() - t0), g

    all_rate, g_all = rate_head(cores, seconds)
    one_rate, g_one = rate_head(1, seconds / 2)
    oracle.set_threads(cores)
    pre = {}
    c1 = dict(synth.SPHERE_D10, xo="nec")
    r = oracle.Run(**{k: c1[k] for k in keys if k in c1})
    pre["c1_nec_pdg_s"] = r4(c1["N"] * c1["D"] * 100 / _timed(lambda: r.generation(100)))
    c5 = dict(synth.ROSENBROCK_D10000, xo="nec")
    r = oracle.Run(**{k: c5[k] for k in keys if k in c5})
    pre["c5_nec_pdg_s"] = r4(c5["N"] * c5["D"] / _timed(lambda: r.generation(1)))
    del r
    D = 2048
    c3 = dict(synth.ELLIPSOID_D2048, N=64, xo="nec", dtype="fp32")
    r = oracle.Run(rot=synth.rotation(D, 0), **{k: c3[k] for k in keys if k in c3})
    pre["c3_gflops_64rows"] = r4(2.0 * 64 * D * D / _timed(lambda: r.generation(1)) / 1e9)
    del r
    runs = [oracle.Run(run=i, **{k: c[k] for k in keys if k in c})
            for i, c in enumerate(synth.batch_table(512, seed=0))]
    elems = sum(x.N * x.D for x in runs)
    pre["c4_pdg_s"] = r4(elems * 2 / _timed(lambda: [x.generation(2) for x in runs]))
    del runs
    return {"value": r4(all_rate), "unit": "pop*dim*gen/s", "cores": cores, "kind": "oracle",
            "sample": f"headline workload, {g_all} generations with {cores} OpenMP threads "
                      f"(~{seconds:.0f} s); one-thread leg {g_one} generations",
            "one_thread": r4(one_rate), "prefix_rates": pre}


# ---- counter summaries -------------------------------------------------------------

def counters_summary(d):
    """Per-kernel averages of every rocprofv3 CSV under d (counter collection
    and kernel-trace stats), as markdown tables."""
    rows = {}
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        for rec in csv.DictReader(open(f)):
            k = (rec["Kernel_Name"].split("(")[0], rec["Counter_Name"])
            rows.setdefault(k, []).append(float(rec["Counter_Value"]))
    if rows:
        print("| kernel | counter | dispatches | mean |\n|---|---|---|---|")
        for (kn, cn), v in sorted(rows.items()):
            print(f"| `{kn}` | {cn} | {len(v)} | {sum(v) / len(v):.6g} |")
    for f in glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True):
        print(f"\n{os.path.relpath(f, d)}:\n\n| kernel | calls | avg ns | min ns | max ns | % |")
        print("|---|---|---|---|---|---|")
        for rec in csv.DictReader(open(f)):
            print(f"| `{rec['Name'].split('(')[0]}` | {rec['Calls']} | {float(rec['AverageNs']):.1f} | "
                  f"{rec['MinNs']} | {rec['MaxNs']} | {float(rec['Percentage']):.1f} |")


# Kernel of each traffic tag, as rocprofv3 names it (template arguments
# <T, FN, XO, ...>: FN 1 Rastrigin, 2 Rosenbrock, -1 per run; XO 0 bin, 1 exp,
# 2 NEC, -1 per run).  A counter run must hold each of these kernels under one
# workload only: exp-lane and exp-scan share a kernel, so the counter runs
# take the scan variant alone.
TRAFFIC_KERNELS = {
    "c2_nec_fp64": "de::k_generation<double, 1, 2,",
    "c2_bin_fp64": "de::k_generation<double, 1, 0,",
    "c2_exp-scan_fp64": "de::k_generation<double, 1, 1,",
    "c2_nec_fp32": "de::k_generation<float, 1, 2,",
    "c2_bin_fp32": "de::k_generation<float, 1, 0,",
    "c2_exp-scan_fp32": "de::k_generation<float, 1, 1,",
    "c5_nec": "de::k_generation_stream<float, 2, 2,",
    "c5_bin": "de::k_generation<float, 2, 0,",
    "c5_exp-scan": "de::k_generation_stream<float, 2, 1,",
    "c4_batched": "de::k_generation<float, -1, -1,",
    "c3_bf16x6": "de::k_rot_gemm_split<3,",
    "c3_bf16x3": "de::k_rot_gemm_split<2,",
    "c3_fp32": "de::k_rot_gemm<1>",
    "c3_fp64": "de::k_rot_gemm<0>",
    "masks_nec": "de::k_masks<2>",
    "masks_bin": "de::k_masks<0>",
    "masks_exp-scan": "de::k_masks<1>",
}
COPY_KERNEL = "neg_kernel"      # torch.neg of the `copy` section
COPY_BYTES = 256 << 20          # it reads and writes this many bytes per launch


def counter_values(dirs):
    vals = {}
    for d in dirs:
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for rec in csv.DictReader(open(f)):
                name = rec["Kernel_Name"]
                name = name[5:] if name.startswith("void ") else name
                vals.setdefault((name, rec["Counter_Name"]), []).append(float(rec["Counter_Value"]))
    return vals


def record_traffic(dirs, path=None):
    """FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of each tagged kernel,
    scaled by what the same counter reads for the copy kernel, written to
    `path` (profiles/traffic.json) with the hash of the sources they were
    taken on; returns the records written."""
    vals = counter_values(dirs)

    def mean(pat, ctr):
        v = [x for (kn, cn), xs in vals.items() if cn == ctr and pat in kn for x in xs]
        return (sum(v) / len(v) if v else None), len(v)

    scale = {}
    for ctr in ("FETCH_SIZE", "WRITE_SIZE"):
        kib, n = mean(COPY_KERNEL, ctr)
        if not kib:
            sys.exit(f"no {ctr} reading of the copy kernel under {dirs}")
        scale[ctr] = COPY_BYTES / (kib * 1024.0)
    path = path or os.path.join(ROOT, "profiles", "traffic.json")
    rec = json.load(open(path)) if os.path.exists(path) else {}
    sha = source_sha()
    print(f"\ncalibration (bytes per counted byte): fetch {scale['FETCH_SIZE']:.4f}, "
          f"write {scale['WRITE_SIZE']:.4f}\n\n| tag | kernel | fetch MB | write MB | dispatches |")
    print("|---|---|---|---|---|")
    for tag, pat in TRAFFIC_KERNELS.items():
        (f, nf), (w, nw) = mean(pat, "FETCH_SIZE"), mean(pat, "WRITE_SIZE")
        if f is None or w is None:
            continue
        fb, wb = f * 1024.0 * scale["FETCH_SIZE"], w * 1024.0 * scale["WRITE_SIZE"]
        rec[tag] = {"source_sha": sha, "kernel": pat, "fetch_bytes": fb, "write_bytes": wb,
                    "bytes_per_launch": fb + wb, "dispatches": [nf, nw]}
        print(f"| {tag} | `{pat}` | {fb / 1e6:.2f} | {wb / 1e6:.2f} | {nf}, {nw} |")
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1, sort_keys=True)
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--sections", default="all",
                    help="comma list of: head (headline only), c1, variants, c5, c3, c4, table1, "
                         "masks10k, fig456, paper_runs, cpu, tuning, copy (default: all but "
                         "masks10k, tuning and copy)")
    ap.add_argument("--variants", default=None,
                    help="comma list of C2 variant names to run (default: all)")
    ap.add_argument("--cpu-seconds", type=float, default=8.0)
    ap.add_argument("--counters", metavar="DIR", nargs="+",
                    help="summarise rocprofv3 CSV output under DIR(s) and exit")
    ap.add_argument("--record", action="store_true",
                    help="with --counters over a FETCH_SIZE and a WRITE_SIZE run: write "
                         "profiles/traffic.json (calibrated by the torch.neg copy)")
    args = ap.parse_args()
    if args.counters:
        for d in args.counters:
            counters_summary(d)
        if args.record:
            record_traffic(args.counters)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(there is no cross-GPU path)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2101_06599_amd as de
    from paper_2101_06599_amd import synth
    torch.cuda.set_device(0)
    de.lib()
    allsec = {"c1", "variants", "c5", "c3", "c4", "table1", "fig456", "paper_runs", "cpu"}
    # not in the default set: masks10k (a subset of table1), tuning, copy
    secs = allsec if args.sections == "all" else set(args.sections.split(","))
    K, W = args.steps, args.warmup

    head = dict(synth.RASTRIGIN_D1000, xo="nec", dtype="fp64")
    gpu = de.DE([head])
    gpu.generation(W)
    ms = time_gens(gpu, K)
    kms = kernel_ms(gpu, max(200, K))
    win = winners(gpu, 20)
    # the same generations replayed from a captured graph of 64 (two blocks)
    gpu.graph(True)
    ms_graph = time_gens(gpu, 128)
    gpu.close()
    N, D, CR = head["N"], head["D"], head["CR"]
    ab = alg_bytes("nec", N, D, CR, 8)
    achieved = ab / (kms * 1e-3) / 1e9
    tb = traffic("c2_nec_fp64")
    out = {
        "metric": "pop*dim*gen/s (shifted Rastrigin D=1000 N=2048, NEC, FP64)",
        "value": N * D * K / (ms / 1e3), "unit": "pop*dim*gen/s", "n_gpus": 1, "steps": K,
        "warmup": W, "ms_per_step": ms / K, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic (seeded populations and shifts)",
        "config": {"workload": "shifted Rastrigin, D=1000, N=2048, F=0.5, CR=0.9, DE/rand/1/NEC, "
                               "FP64, x~U[-5.12,5.12], o~U[-4,4], Philox seed 0",
                   "N": N, "D": D, "generation": "one generation per step"},
        "graph_replay_ms_per_step": r4(ms_graph / 128),
    }
    if "table1" in secs:
        out["table1_masks"] = table1(torch, de)
    if "masks10k" in secs:
        out["masks_n10000_d10000"] = masks10k(torch, de)
    if "fig456" in secs:
        out["fig456_pexp_scan_vs_nec"] = fig456(torch, de)
    if "paper_runs" in secs:
        out["table2_runs"] = paper_runs(torch, de, synth)
    if "tuning" in secs:
        from paper_2101_06599_amd.tune import tune_tpr
        best, tab = tune_tpr(head, gens=64, use_cache=False)
        out["tuning_headline"] = {"best_tpr": best, "ms_by_tpr": {k: r4(v) for k, v in tab.items()}}
    if "copy" in secs:
        # counter calibration: b = -a over 256 MiB of float32 (reads and
        # writes a known number of bytes)
        n = 256 << 20
        a = torch.ones(n // 4, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(5):
            torch.neg(a, out=b)
        sync()
        out["copy_calibration"] = {"kernel": "torch.neg over float32", "bytes_read": n,
                                   "bytes_written": n, "launches": 5}
    if "c1" in secs:
        out["c1_sphere_d10_n50"] = c1_sphere(synth)
    if "variants" in secs:
        only = None if args.variants is None else set(args.variants.split(","))
        out["frac_bases"] = {
            "frac_alg": "s N D (2 + 3 rho): a trial write charged to every row; the kernels "
                        "write winners only, so it can exceed 1",
            "frac_min": "s N D (1 + 3 rho + rho w), w = measured winner fraction: a lower bound",
            "frac_ctr": "FETCH_SIZE + WRITE_SIZE per launch (profiles/traffic.json), null if "
                        "the kernel sources changed since"}
        out["c2_rastrigin_d1000_n2048"] = c2_variants(synth, K, W, only)
    if "c4" in secs:
        out["c4_batched_512"] = c4_batched(synth)
    if "c3" in secs:
        out["c3_rotated_d2048_n4096"] = c3_rotated(torch, synth)
    if "c5" in secs:
        out["c5_rosenbrock_d10000_n8192"] = c5_rosenbrock(synth)
    # attainable bandwidth beside the datasheet peak: torch's copy of 1 GiB
    # (read + write), beyond every cache
    n = 1 << 28
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    sync()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(10):
        b.copy_(a)
    e1.record(s)
    sync()
    copy_gbs = 2 * 4 * n * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": achieved / HBM_PEAK_GBS, "traffic": tb,
                       "kernel": "k_generation<double, RASTRIGIN, NEC>", "kernel_ms": r4(kms),
                       "alg_bytes_per_launch": r4(ab), "winner_fraction": r4(win),
                       "frac_min": r4(min_bytes("nec", N, D, CR, 8, win) / (kms * 1e-3) / 1e9
                                      / HBM_PEAK_GBS),
                       "frac_ctr": None if tb is None else r4(tb / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS),
                       "copy_GBps": r4(copy_gbs), "frac_of_copy": r4(achieved / copy_gbs),
                       "device": device_info(torch),
                       "note": "33 MB working set: Infinity-Cache resident"}
    if "cpu" in secs:
        out["cpu_baseline"] = cpu_baseline(synth, head, args.cpu_seconds)
    print(json.dumps(out, separators=(",", ":")))


if __name__ == "__main__":
    main()
