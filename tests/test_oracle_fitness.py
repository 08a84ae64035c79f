"""Pins for the oracle's fitness functions (CPU only): known optima, closed-form
points and independent library routines (scipy's Rosenbrock, math.fsum)."""
import math

import numpy as np
import pytest
from scipy.optimize import rosen

import oracle


@pytest.mark.parametrize("D", [1, 10, 1000])
def test_sphere_closed_form_and_fsum(D):
    for c in (0.0, 1.0, -3.0, 7.0):
        assert oracle.fitness("sphere", np.full(D, c)) == D * c * c
    x = np.random.default_rng(D).uniform(-100, 100, D)
    ref = math.fsum(float(v) * float(v) for v in x)
    assert abs(oracle.fitness("sphere", x) - ref) <= 1e-15 * ref


def test_rastrigin_optimum_integer_and_half_points():
    D = 50
    rng = np.random.default_rng(1)
    o = rng.uniform(-4, 4, D)
    assert oracle.fitness("rastrigin", o, o) == 0.0
    z = rng.integers(-5, 6, D).astype(np.float64)
    o2 = np.zeros(D)
    f = oracle.fitness("rastrigin", z, o2)
    assert abs(f - float((z * z).sum())) <= 1e-14 * max(1.0, f)
    h = z + 0.5
    f = oracle.fitness("rastrigin", h, o2)
    ref = float((h * h).sum()) + 20.0 * D
    assert abs(f - ref) <= 1e-14 * ref


def test_rastrigin_matches_cosine_form():
    # f = sum z^2 - 10 cos(2 pi z) + 10, evaluated with numpy's cos
    D = 1000
    rng = np.random.default_rng(2)
    x = rng.uniform(-5.12, 5.12, D)
    o = rng.uniform(-4, 4, D)
    z = x - o
    ref = float(np.sum(z * z - 10.0 * np.cos(2.0 * np.pi * z) + 10.0))
    f = oracle.fitness("rastrigin", x, o)
    # the cosine form loses up to ~20 ulp of 10 per term to cancellation
    assert abs(f - ref) <= 1e-13 * 20.0 * D


@pytest.mark.parametrize("D", [2, 3, 10, 500])
def test_rosenbrock_against_scipy_and_special_points(D):
    rng = np.random.default_rng(D)
    x = rng.uniform(-5.12, 5.12, D)
    ones = np.ones(D)
    # with o = 1 the shifted variable z = x - o + 1 is x itself
    ref = float(rosen(x))
    assert abs(oracle.fitness("rosenbrock", x, ones) - ref) <= 1e-13 * ref
    o = rng.uniform(-4, 4, D)
    assert oracle.fitness("rosenbrock", o, o) == 0.0                      # z = 1
    assert oracle.fitness("rosenbrock", o - 1.0, o) == pytest.approx(D - 1, rel=1e-15)  # z = 0
    assert oracle.fitness_phi("rosenbrock", x, o) >= oracle.fitness("rosenbrock", x, o)


def test_ellipsoid_weights_and_special_points():
    D = 16
    w = oracle.ellipsoid_weights(D)
    assert w[0] == 1.0 and w[-1] == 1e6
    ratios = w[1:] / w[:-1]
    assert np.allclose(ratios, 10 ** (6 / (D - 1)), rtol=1e-14)
    eye = np.eye(D)
    o = np.random.default_rng(3).uniform(-80, 80, D)
    for k in range(D):
        x = o + eye[k]
        assert oracle.fitness("ellipsoid_rot", x, o, eye) == pytest.approx(w[k], rel=1e-15)
    assert oracle.fitness("ellipsoid_rot", o, o, eye) == 0.0
    perm = np.random.default_rng(4).permutation(D)
    P = eye[perm]                        # (P d)_k = d_perm[k]
    d = np.arange(1.0, D + 1.0)
    f = oracle.fitness("ellipsoid_rot", o + d, o, P)
    assert f == pytest.approx(float(np.sum(w * d[perm] ** 2)), rel=1e-15)


def test_ellipsoid_rotated_against_numpy():
    D = 64
    rng = np.random.default_rng(0)
    Q, R = np.linalg.qr(rng.standard_normal((D, D)))
    Q = Q * np.sign(np.diag(R))
    x = rng.uniform(-100, 100, D)
    o = rng.uniform(-80, 80, D)
    w = oracle.ellipsoid_weights(D)
    ref = float(np.sum(w * (Q @ (x - o)) ** 2))
    assert abs(oracle.fitness("ellipsoid_rot", x, o, Q) - ref) <= 1e-12 * ref


def test_nan_is_plus_infinity():
    x = np.array([1.0, np.nan, 2.0])
    assert oracle.fitness("sphere", x) == math.inf
    assert oracle.fitness("rastrigin", x, np.zeros(3)) == math.inf
    assert oracle.fitness("rosenbrock", x, np.zeros(3)) == math.inf


@pytest.mark.parametrize("D", [1, 10, 1000])
def test_ackley_optimum_and_integer_points(D):
    assert abs(oracle.fitness("ackley", np.zeros(D))) <= 1e-15
    for c in (1.0, -3.0, 7.0):
        # cos(2 pi c) = 1 at integers, so f = 20 (1 - exp(-0.02 |c|))
        ref = 20.0 * (1.0 - math.exp(-0.02 * abs(c)))
        assert abs(oracle.fitness("ackley", np.full(D, c)) - ref) <= 1e-14 * ref
    half = np.full(D, 0.5)  # cos(pi) = -1: f = 20 (1 - exp(-0.01)) + e - 1/e
    ref = 20.0 * (1.0 - math.exp(-0.01)) + math.e - 1.0 / math.e
    assert abs(oracle.fitness("ackley", half) - ref) <= 1e-14 * ref


@pytest.mark.parametrize("D", [1, 2, 10, 500])
def test_griewank_optimum_and_cosine_points(D):
    j = np.arange(1, D + 1, dtype=np.float64)
    assert oracle.fitness("griewank", np.zeros(D)) == 0.0
    x = 2.0 * np.pi * np.sqrt(j)      # every cosine is +1
    ref = float(np.sum(x * x)) / 4000.0
    assert abs(oracle.fitness("griewank", x) - ref) <= 1e-13 * ref
    y = np.pi * np.sqrt(j)            # every cosine is -1
    ref = float(np.sum(y * y)) / 4000.0 + 1.0 - (-1.0) ** D
    assert abs(oracle.fitness("griewank", y) - ref) <= 1e-13 * ref
    assert oracle.fitness_phi("griewank", y) >= oracle.fitness("griewank", y)


# ---- Ackley's cancellation-free form and the tolerance scale ----------------

def _ackley_mp(x, dps=60):
    """Sec. 4's Ackley in the printed order, evaluated by mpmath at `dps`
    decimal digits (an independent evaluation of the printed formula)."""
    import mpmath as mp
    with mp.workdps(dps):
        D = len(x)
        sq = mp.fsum(mp.mpf(float(v)) ** 2 for v in x)
        cs = mp.fsum(mp.cos(2 * mp.pi * mp.mpf(float(v))) for v in x)
        f = -20 * mp.exp(mp.mpf("-0.02") * mp.sqrt(sq / D)) - mp.exp(cs / D) + 20 + mp.e
        return f


@pytest.mark.parametrize("scale", [30.0, 1.0, 1e-3, 1e-6, 1e-9])
@pytest.mark.parametrize("D", [1, 7, 1000])
def test_ackley_against_high_precision(D, scale):
    # relative accuracy down to f ~ 1e-10, where the printed order in double
    # precision would keep no correct digit
    rng = np.random.default_rng(int(D * 10 + scale * 7 % 97))
    for _ in range(3):
        x = rng.uniform(-scale, scale, D)
        ref = _ackley_mp(x)
        f = oracle.fitness("ackley", x)
        assert abs(f - float(ref)) <= 4e-16 * float(ref)


def test_ackley_near_nonzero_integers_against_high_precision():
    rng = np.random.default_rng(5)
    c = rng.integers(-20, 21, 50).astype(np.float64)
    x = c + rng.uniform(-1e-7, 1e-7, 50)
    ref = float(_ackley_mp(x))
    assert abs(oracle.fitness("ackley", x) - ref) <= 4e-16 * ref


def test_ackley_equals_printed_order_in_the_box():
    # the two orders agree up to the printed order's cancellation error
    rng = np.random.default_rng(9)
    for D in (3, 100, 1000):
        x = rng.uniform(-30, 30, D)
        f = oracle.fitness("ackley", x)
        assert abs(f - oracle.ackley_printed(x)) <= 4 * np.spacing(f)


@pytest.mark.parametrize("D", [1, 10, 1000])
def test_phi_is_f_for_sums_of_nonnegative_terms(D):
    # the tolerance scale equals f itself where every term is >= 0: a scale
    # that grew (a lost absolute value, an extra term) fails here
    rng = np.random.default_rng(D)
    o = rng.uniform(-4, 4, D)
    for scale in (30.0, 1e-2, 1e-6):
        x = rng.uniform(-scale, scale, D)
        assert oracle.fitness_phi("ackley", x) == oracle.fitness("ackley", x)
        assert oracle.fitness_phi("sphere", x) == oracle.fitness("sphere", x)
        assert oracle.fitness_phi("rastrigin", x, o) == oracle.fitness("rastrigin", x, o)
    assert oracle.fitness_phi("ackley", np.zeros(D)) == 0.0
    for c in (1.0, -3.0):
        ref = 20.0 * (1.0 - math.exp(-0.02 * abs(c)))
        assert abs(oracle.fitness_phi("ackley", np.full(D, c)) - ref) <= 1e-14 * ref
    if D >= 2:
        Q = np.linalg.qr(rng.standard_normal((D, D)))[0]
        x = rng.uniform(-100, 100, D)
        assert oracle.fitness_phi("ellipsoid_rot", x, o, Q) == oracle.fitness("ellipsoid_rot", x, o, Q)


@pytest.mark.parametrize("D", [2, 3, 50])
def test_rosenbrock_phi_closed_points(D):
    # Phi = sum 100 (|z_{j+1}| + z_j^2)^2 + (|z_j| + 1)^2 over the D - 1 pairs
    rng = np.random.default_rng(D)
    o = rng.uniform(-4, 4, D)
    assert oracle.fitness_phi("rosenbrock", o, o) == 404.0 * (D - 1)         # z = 1
    for c in (-2.0, 0.0, 3.0):   # z = c everywhere (exact for these c and o = 0)
        z = np.full(D, c)
        ref = (D - 1) * (100.0 * (abs(c) + c * c) ** 2 + (abs(c) + 1.0) ** 2)
        assert oracle.fitness_phi("rosenbrock", z - 1.0, np.zeros(D)) == ref
    x = rng.uniform(-5.12, 5.12, D)
    z = x - o + 1.0
    ref = float(np.sum(100.0 * (np.abs(z[1:]) + z[:-1] ** 2) ** 2 + (np.abs(z[:-1]) + 1.0) ** 2))
    assert abs(oracle.fitness_phi("rosenbrock", x, o) - ref) <= 1e-13 * ref


@pytest.mark.parametrize("D", [1, 2, 10, 500])
def test_griewank_phi_closed_points(D):
    j = np.arange(1, D + 1, dtype=np.float64)
    assert oracle.fitness_phi("griewank", np.zeros(D)) == 2.0
    x = 2.0 * np.pi * np.sqrt(j)      # every cosine is +1
    ref = float(np.sum(x * x)) / 4000.0 + 2.0
    assert abs(oracle.fitness_phi("griewank", x) - ref) <= 1e-13 * ref
    y = np.pi * np.sqrt(j)            # every cosine is -1: |prod| = 1
    ref = float(np.sum(y * y)) / 4000.0 + 2.0
    assert abs(oracle.fitness_phi("griewank", y) - ref) <= 1e-13 * ref
