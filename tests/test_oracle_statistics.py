"""Pin of the oracle's whole DE loop (Alg 1 / Alg 2) against an independent
textbook DE/rand/1 written here with numpy's own random streams: the two use
different random numbers, so single runs differ, but over several seeds the
best fitness they reach after a fixed number of generations must agree.  A
reversed selection, for one, moves the oracle far outside the textbook runs'
spread; the masks, indices and trial rows have their own exact pins."""
import numpy as np
import pytest

import oracle


def ackley(X):
    return (-20.0 * np.exp(-0.02 * np.sqrt((X * X).mean(1))) - np.exp(np.cos(2 * np.pi * X).mean(1))
            + 20.0 + np.e)


def sphere(X):
    return (X * X).sum(1)


def textbook(fn, N, D, F, CR, lo, hi, gens, seed, xo):
    rng = np.random.default_rng(seed)
    X = rng.uniform(lo, hi, (N, D))
    f = fn(X)
    rows = np.arange(N)
    for _ in range(gens):
        # three distinct indices per row, all different from the row
        idx = np.argsort(rng.random((N, N - 1)), axis=1)[:, :3]
        idx = idx + (idx >= rows[:, None])
        V = X[idx[:, 0]] + F * (X[idx[:, 1]] - X[idx[:, 2]])
        jr = rng.integers(0, D, N)
        if xo == "bin":
            M = rng.random((N, D)) < CR
            M[rows, jr] = True
        else:  # classic exponential: run of L elements from jr, wrapping
            L = np.ones(N, dtype=np.int64)
            alive = np.ones(N, bool)
            for _k in range(D - 1):
                alive &= rng.random(N) < CR
                L += alive
            M = ((np.arange(D)[None, :] - jr[:, None]) % D) < L[:, None]
        U = np.where(M, V, X)
        fu = fn(U)
        w = fu < f
        X[w] = U[w]
        f[w] = fu[w]
    return float(f.min())


@pytest.mark.parametrize("fn_name,fn,lo,hi,CR,gens", [("ackley", ackley, -30.0, 30.0, 0.2, 300),
                                                     ("sphere", sphere, -100.0, 100.0, 0.9, 150)])
@pytest.mark.parametrize("xo", ["bin", "nec"])
def test_oracle_run_matches_textbook_de(fn_name, fn, lo, hi, CR, gens, xo):
    N, D, F = 40, 30, 0.5
    seeds = range(6)
    tb = [textbook(fn, N, D, F, CR, lo, hi, gens, s, "bin" if xo == "bin" else "exp")
          for s in seeds]
    orc = []
    for s in seeds:
        r = oracle.Run(N=N, D=D, F=F, CR=CR, xo=xo, fn=fn_name, dtype="fp64", lo=lo, hi=hi, seed=s)
        r.generation(gens)
        orc.append(r.best()[0])
    # compare in log space: geometric means within a factor of 3, and the
    # oracle's median inside the textbook runs' range widened by that factor
    lt, lo_ = np.log(tb), np.log(orc)
    assert abs(lt.mean() - lo_.mean()) < np.log(3.0), (tb, orc)
    assert lt.min() - np.log(3.0) < np.median(lo_) < lt.max() + np.log(3.0), (tb, orc)
    # and the oracle improved well beyond the initial population
    start = fn(np.random.default_rng(0).uniform(lo, hi, (N, D))).min()
    assert max(orc) < 0.5 * start
