"""Coefficients of the FP64 sin^2(pi z) polynomial in csrc/de_device.h.

    python -m paper_2101_06599_amd.fit_sinpi

sin(pi r) for |r| <= 1/2 is written r * P(r^2) with P of degree 8; P is the
minimax approximation of sin(pi sqrt(t)) / sqrt(t) on t in [0, 1/4] for the
relative error, found by a Remez exchange in 60-digit arithmetic (mpmath).
Its approximation error is about 2.6e-19, so the rounding of the evaluation
decides the accuracy.  The script prints the coefficients rounded to FP64
(for sin^2 and, multiplied by sqrt(20), for the Rastrigin term 20 sin^2) and
the largest relative error of the evaluated sin^2 over a grid of r, the
evaluation done as the kernels do it (t = r r rounded, Horner steps as fused
multiply-adds rounded once, r P rounded, then squared).
"""
from __future__ import annotations

import mpmath as mp

DEGREE = 8


def _g(t):
    if t == 0:
        return mp.pi
    s = mp.sqrt(t)
    return mp.sin(mp.pi * s) / s


def remez(n: int = DEGREE, iters: int = 12, grid: int = 4000):
    """Coefficients c_0..c_n (mp floats) of the minimax relative-error fit."""
    mp.mp.dps = 60
    m = n + 2
    xs = [mp.mpf(1) / 8 * (1 - mp.cos(mp.pi * k / (m - 1))) for k in range(m)]
    c = None
    for _ in range(iters):
        A = mp.matrix(m, m)
        b = mp.matrix(m, 1)
        for i, t in enumerate(xs):
            gt = _g(t)
            for j in range(n + 1):
                A[i, j] = t ** j / gt
            A[i, n + 1] = (-1) ** i
            b[i] = 1
        sol = mp.lu_solve(A, b)
        c = [sol[j] for j in range(n + 1)]

        def err(t):
            return sum(c[j] * t ** j for j in range(n + 1)) / _g(t) - 1

        pts = [mp.mpf(1) / 4 * k / grid for k in range(grid + 1)]
        ev = [err(t) for t in pts]
        ext = [(pts[k], ev[k]) for k in range(len(pts))
               if k in (0, len(pts) - 1) or (ev[k] - ev[k - 1]) * (ev[k + 1] - ev[k]) <= 0]
        alt: list = []
        for t, e in ext:  # alternating extrema, the larger of equal-signed neighbours
            if alt and mp.sign(alt[-1][1]) == mp.sign(e):
                if abs(e) > abs(alt[-1][1]):
                    alt[-1] = (t, e)
            else:
                alt.append((t, e))
        while len(alt) > m:
            alt.pop(0 if abs(alt[0][1]) < abs(alt[-1][1]) else -1)
        if len(alt) < m:
            break
        xs = [t for t, _ in alt]
    return c


def evaluate_sq(coeffs, r: float) -> float:
    """(r P(r^2))^2 evaluated in FP64 as the kernels do (fma = one rounding)."""
    t = float(mp.mpf(r) * r)
    p = coeffs[-1]
    for ck in reversed(coeffs[:-1]):
        p = float(mp.mpf(p) * t + ck)
    s = float(mp.mpf(r) * p)
    return float(mp.mpf(s) * s)


def worst_relative_error(coeffs, scale, n: int = 4000) -> float:
    mp.mp.dps = 60
    worst = mp.mpf(0)
    for k in range(1, n + 1):
        r = 0.5 * k / n
        ex = scale * mp.sin(mp.pi * r) ** 2
        worst = max(worst, abs((evaluate_sq(coeffs, r) - ex) / ex))
    return float(worst)


def main():
    c = remez()
    sets = {"sinpi_sq": ([float(x) for x in c], 1),
            "sinpi_sq20": ([float(x * mp.sqrt(20)) for x in c], 20)}
    for name, (cd, scale) in sets.items():
        print(f"{name}: highest power first")
        for x in reversed(cd):
            print("  ", float.hex(x))
        print(f"  largest relative error of the evaluated value: "
              f"{worst_relative_error(cd, scale):.3e}")


if __name__ == "__main__":
    main()
