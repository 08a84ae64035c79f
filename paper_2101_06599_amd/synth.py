"""Seeded synthetic inputs shared by the tests and the benchmark.

Nothing here computes any part of the method: these are the data a caller
hands to the library (the rotation matrix of the rotated ellipsoid, the
table of runs of a batched launch) and the workload definitions with the
sizes the paper's experiments and the benchmark use."""
from __future__ import annotations

import numpy as np


def rotation(D: int, seed: int = 0) -> np.ndarray:
    """Q of the QR factorisation of a seeded D x D standard Gaussian matrix,
    with column signs fixed by diag(R) > 0 (a Haar-distributed rotation)."""
    rng = np.random.default_rng(seed)
    Q, R = np.linalg.qr(rng.standard_normal((D, D)))
    return np.ascontiguousarray(Q * np.sign(np.diag(R)))


def batch_table(n_runs: int = 512, seed: int = 0, max_D: int = 1000, max_N: int = 512):
    """Independent runs of uneven shape: D ~ U{10..max_D}, N ~ U{20..max_N},
    function from {sphere, shifted Rastrigin, shifted Rosenbrock},
    CR ~ U[0.5, 0.95], F ~ U[0.4, 0.9]; NEC crossover, FP32."""
    rng = np.random.default_rng(seed)
    fns = ("sphere", "rastrigin", "rosenbrock")
    runs = []
    for r in range(n_runs):
        fn = fns[int(rng.integers(0, 3))]
        D = int(rng.integers(10, max_D + 1))
        N = int(rng.integers(20, max_N + 1))
        CR = float(rng.uniform(0.5, 0.95))
        F = float(rng.uniform(0.4, 0.9))
        box = {"sphere": (-100.0, 100.0, 0.0, 0.0), "rastrigin": (-5.12, 5.12, -4.0, 4.0),
               "rosenbrock": (-5.12, 5.12, -4.0, 4.0)}[fn]
        runs.append(dict(N=N, D=D, F=F, CR=CR, xo="nec", fn=fn, dtype="fp32", lo=box[0],
                         hi=box[1], olo=box[2], ohi=box[3], seed=0))
    return runs


# Workloads (population, dimension, parameters, boxes) of the experiments.
SPHERE_D10 = dict(N=50, D=10, F=0.5, CR=0.9, fn="sphere", dtype="fp64", lo=-100.0, hi=100.0,
                  seed=0)
RASTRIGIN_D1000 = dict(N=2048, D=1000, F=0.5, CR=0.9, fn="rastrigin", lo=-5.12, hi=5.12,
                       olo=-4.0, ohi=4.0, seed=0)
ELLIPSOID_D2048 = dict(N=4096, D=2048, F=0.5, CR=0.9, fn="ellipsoid_rot", lo=-100.0, hi=100.0,
                       olo=-80.0, ohi=80.0, seed=0)
ROSENBROCK_D10000 = dict(N=8192, D=10000, F=0.5, CR=0.9, fn="rosenbrock", dtype="fp32",
                         lo=-5.12, hi=5.12, olo=-4.0, ohi=4.0, seed=0)

# The three runs of Table 2 (Sec. 4): function, D, N, F, Cr and generation
# count as listed there, search box as given with each function.  The
# Rosenbrock of Sec. 4 has its optimum at x = 1, which is the shifted form
# z = x - o + 1 with o = 1 (olo = ohi = 1 makes every o_j exactly 1).
ACKLEY_D1000 = dict(N=500, D=1000, F=0.5, CR=0.2, fn="ackley", dtype="fp64", lo=-30.0, hi=30.0,
                    seed=0, gens=30000)
GRIEWANK_D500 = dict(N=300, D=500, F=0.25, CR=0.45, fn="griewank", dtype="fp64", lo=-400.0,
                     hi=400.0, seed=0, gens=20000)
ROSENBROCK_D50 = dict(N=100, D=50, F=0.65, CR=0.95, fn="rosenbrock", dtype="fp64", lo=-5.12,
                      hi=5.12, olo=1.0, ohi=1.0, seed=0, gens=10000)
TABLE2 = {"ackley": ACKLEY_D1000, "griewank": GRIEWANK_D500, "rosenbrock": ROSENBROCK_D50}
