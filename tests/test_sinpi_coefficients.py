"""The sin^2(pi z) polynomials of the fitness kernels, pinned on the CPU to
the mathematics (no GPU): the FP64 coefficients in csrc/de_device.h are the
ones the committed Remez fit produces, and evaluated the way the kernels do
(fused multiply-adds, one rounding each) they stay within a few ulp of
sin^2(pi r) and 20 sin^2(pi r) against 60-digit references; the FP32
coefficients are the Taylor coefficients of sine rounded to FP32."""
import math
import os
import re

import mpmath as mp
import numpy as np
import pytest

from paper_2101_06599_amd import fit_sinpi

HDR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_2101_06599_amd", "csrc", "de_device.h")


def _coeffs(signature: str):
    """Hex literals of one function body, highest power first."""
    src = open(HDR).read()
    start = src.index(signature)
    body = src[start:src.index("\n}", start)]
    return [float.fromhex(h.rstrip("f")) for h in re.findall(r"-?0x1\.[0-9a-f]+p[-+]\d+f?", body)]


FP64_SQ = "__device__ __forceinline__ double sinpi_sq(double z)"
FP64_SQ20 = "__device__ __forceinline__ double sinpi_sq20(double z)"
FP32_SQ = "__device__ __forceinline__ float sinpi_sq(float z)"


def test_fp64_coefficients_are_the_remez_fit():
    c = fit_sinpi.remez()
    assert _coeffs(FP64_SQ) == [float(x) for x in reversed(c)]
    assert _coeffs(FP64_SQ20) == [float(x * mp.sqrt(20)) for x in reversed(c)]


@pytest.mark.parametrize("sig,scale,ulps", [(FP64_SQ, 1, 3.0), (FP64_SQ20, 20, 4.0)])
def test_fp64_polynomial_accuracy(sig, scale, ulps):
    mp.mp.dps = 60
    coeffs = list(reversed(_coeffs(sig)))  # lowest power first, as evaluate_sq takes them
    rng = np.random.default_rng(7)
    rs = np.concatenate([np.linspace(1e-6, 0.5, 1500), rng.uniform(0.0, 0.5, 1500),
                         [0.5, 0.49999999999, 0.25, 1e-3, 2.0 ** -30]])
    worst = 0.0
    for r in rs:
        r = float(r)
        if r == 0.0:
            continue
        ex = scale * mp.sin(mp.pi * r) ** 2
        worst = max(worst, float(abs((fit_sinpi.evaluate_sq(coeffs, r) - ex) / ex)))
    assert worst <= ulps * 2.0 ** -52, worst / 2.0 ** -52


def test_fp32_coefficients_are_the_taylor_series():
    mp.mp.dps = 40
    got = list(reversed(_coeffs(FP32_SQ)))
    want = [float(np.float32((-1) ** k * mp.pi ** (2 * k + 1) / mp.factorial(2 * k + 1)))
            for k in range(len(got))]
    assert got == want
    # the first dropped term, relative to sin(pi r) ~ 2 r at r = 1/2, is tiny
    k = len(got)
    assert float(mp.pi ** (2 * k + 1) / mp.factorial(2 * k + 1) * 0.25 ** k / 2) < 1e-8
    assert math.isclose(got[0], math.pi, rel_tol=2 ** -24)
