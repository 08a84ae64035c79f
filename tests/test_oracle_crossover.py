"""Pins for the oracle's crossover operators (CPU only).

What the paper fixes and these tests check:
* Eq 3/4 (Sec. 3.1): the run length of the classic exponential crossover
  (Alg 8) is geometric, P(L >= k) = Cr^(k-1), truncated at D.
* Eq 9 (Sec. 3.2): NEC samples L with that same law from one uniform; the
  threshold form used by the oracle equals the printed log form.
* Alg 9 and Alg 10 describe the same wrapped run of L elements from j_rand.
* Alg 7 / Eq 2: binomial mask, element j on with probability Cr, plus j_rand.
"""
import itertools
from fractions import Fraction

import numpy as np
import pytest
from scipy.stats import chi2_contingency, chisquare

import oracle


def p_less(CR: float) -> Fraction:
    """Exact P((w + 1/2) 2^-32 < CR) over the 2^32 words."""
    c = Fraction(CR) * 2**32 - Fraction(1, 2)
    n = -((-c.numerator) // c.denominator)  # ceil
    n = min(max(n, 0), 2**32)
    return Fraction(n, 2**32)


def jrand_prob(D):
    return [Fraction(-((-(j + 1) * 2**32) // D) - (-((-j * 2**32) // D)), 2**32)
            for j in range(D)]


def geometric_expected(p: float, D: int, n: int):
    """Expected counts of L = 1..D for P(L >= k) = p^(k-1), truncated at D."""
    tail = [p ** (k - 1) for k in range(1, D + 2)]
    tail[D] = 0.0
    probs = np.array([tail[k - 1] - tail[k] for k in range(1, D + 1)])
    return probs * n


def merged_chisquare(obs, exp, min_exp=5.0):
    obs = np.asarray(obs, float)
    exp = np.asarray(exp, float)
    mo, me, ao, ae = [], [], 0.0, 0.0
    for o, e in zip(obs, exp):
        ao += o
        ae += e
        if ae >= min_exp:
            mo.append(ao); me.append(ae); ao = ae = 0.0
    if ae > 0 or ao > 0:
        if mo:
            mo[-1] += ao; me[-1] += ae
        else:
            mo.append(ao); me.append(ae)
    me = np.array(me) * (sum(mo) / sum(me))
    if len(mo) < 2:
        return 1.0
    return chisquare(mo, me).pvalue


def sample_exp_lengths(D, CR, n, seed=11):
    """Alg 8 run lengths of n individuals, sampled by the oracle's C loop."""
    return oracle.lengths("exp", D, CR, n, seed)


def sample_nec_lengths(D, CR, n, seed=11):
    """NEC (Eq 9) run lengths of n individuals, sampled by the oracle's C loop."""
    return oracle.lengths("nec", D, CR, n, seed)


def test_batch_sampler_is_the_per_individual_draw():
    # the C loop addresses individual k as (generation 1 + k // 4096, position
    # k % 4096) and calls the same per-individual functions
    n = 5000
    a = sample_exp_lengths(37, 0.8, n, seed=5)
    b = sample_nec_lengths(37, 0.8, n, seed=5)
    for k in range(0, n, 7):
        g, i = 1 + k // 4096, k % 4096
        assert a[k] == oracle.exp_length(5, 0, 37, 0.8, g, i)
        w = oracle.word(5, 0, "xo", g, i, 0, 1)
        assert b[k] == oracle.nec_length(oracle.uniform(w), 0.8, 37)


# 10^6 draws per case, as in the L-frequency comparison of Sec. 3.2
N_DRAWS = 1_000_000


@pytest.mark.parametrize("D,CR", [(4, 0.5), (10, 0.2), (10, 0.5), (10, 0.9), (10, 0.95),
                                  (1000, 0.9), (1000, 0.95)])
@pytest.mark.parametrize("kind", ["exp", "nec"])
def test_length_law_geometric_truncated(kind, D, CR):
    n = N_DRAWS
    L = sample_exp_lengths(D, CR, n) if kind == "exp" else sample_nec_lengths(D, CR, n)
    assert L.min() >= 1 and L.max() <= D
    obs = np.bincount(L, minlength=D + 1)[1:]
    exp = geometric_expected(CR, D, n)
    assert merged_chisquare(obs, exp) > 1e-3
    # mean against the closed form E[L] = (1 - Cr^D) / (1 - Cr)
    mean = (1 - CR**D) / (1 - CR)
    sd = np.sqrt(((np.arange(1, D + 1) - mean) ** 2 * exp / n).sum())
    assert abs(L.mean() - mean) < 5 * sd / np.sqrt(n)
    # the tail P(L >= k) = Cr^(k-1) itself at a few k, within 5 binomial sd
    for k in (2, 3, 5, 10):
        if k <= D:
            p = CR ** (k - 1)
            assert abs(np.mean(L >= k) - p) <= 5 * np.sqrt(p * (1 - p) / n) + 1e-12


def test_length_law_detects_a_shifted_law():
    # power check: the 10^6-draw test rejects a law whose ratio is off by 1 %
    n = N_DRAWS
    L = sample_nec_lengths(10, 0.9, n)
    assert merged_chisquare(np.bincount(L, minlength=11)[1:], geometric_expected(0.9 * 1.01, 10, n)) < 1e-3


@pytest.mark.parametrize("D", [1, 4, 10, 1000])
@pytest.mark.parametrize("kind", ["exp", "nec"])
def test_length_special_cases(kind, D):
    f = sample_exp_lengths if kind == "exp" else sample_nec_lengths
    assert set(f(D, 0.0, 300).tolist()) == {1}          # Eq 9 first case
    assert set(f(D, 1.0, 300).tolist()) == {D}          # Eq 9 third case


def test_exp_and_nec_lengths_homogeneous_d10():
    # the claim of the L-frequency comparison for D = 10 in Sec. 3.2, 10^6 draws each
    n = N_DRAWS
    for CR in (0.5, 0.9):
        a = np.bincount(sample_exp_lengths(10, CR, n, seed=3), minlength=11)[1:]
        b = np.bincount(sample_nec_lengths(10, CR, n, seed=4), minlength=11)[1:]
        keep = (a + b) > 10
        assert chi2_contingency(np.vstack([a[keep], b[keep]]))[1] > 1e-3


@pytest.mark.parametrize("CR", [0.2, 0.25, 0.5, 0.9, 0.95, 0.99])
def test_nec_threshold_form_equals_log_form(CR):
    D = 200
    # every threshold boundary on the (w + 1/2) 2^-32 grid
    t = 1.0
    for k in range(2, D + 1):
        t = t * CR
        wb = -((-(Fraction(t) * 2**32 - Fraction(1, 2)).numerator) //
               (Fraction(t) * 2**32 - Fraction(1, 2)).denominator)
        for w in (wb - 1, wb):
            if 0 <= w < 2**32:
                U = oracle.uniform(int(w))
                assert oracle.nec_length(U, CR, D) == oracle.nec_length_log(U, CR, D), (k, w)
        if t * 2**32 < 1:
            break
    rng = np.random.default_rng(5)
    for w in rng.integers(0, 2**32, 20000):
        U = oracle.uniform(int(w))
        assert oracle.nec_length(U, CR, D) == oracle.nec_length_log(U, CR, D)


def test_nec_exact_discrete_law():
    # P(L >= k) = P(U < Cr^(k-1)) exactly, checked on the word grid at small k
    CR, D = 0.5, 10
    t = 1.0
    for k in range(2, D + 1):
        t *= CR
        thr = p_less(t) * 2**32
        assert oracle.nec_length(oracle.uniform(int(thr) - 1), CR, D) >= k
        assert oracle.nec_length(oracle.uniform(int(thr)), CR, D) < k


@pytest.mark.parametrize("D", range(1, 9))
def test_alg10_equals_alg9_bruteforce(D):
    masks = set()
    for j in range(D):
        for L in range(1, D + 1):
            a9 = oracle.alg9_mask(D, j, L)
            a10 = oracle.alg10_mask(D, j, L)
            assert np.array_equal(a9, a10), (D, j, L)
            assert a9.sum() == L
            masks.add(a9.tobytes())
    # D (D - 1) runs shorter than D, plus the single full mask
    assert len(masks) == D * (D - 1) + 1


def test_printed_alg10_comparison_misses_wrapping_runs():
    # Alg 10 as printed, (j <= Seq) XOR (Ls < Seq), does not give Alg 9's run;
    # this is why the oracle states the run elementwise instead.
    bad = 0
    for D in range(2, 9):
        for j in range(D):
            for L in range(1, D + 1):
                printed = np.array([(j <= s) ^ (L < s) for s in range(D)], np.uint8)
                bad += not np.array_equal(printed, oracle.alg9_mask(D, j, L))
    assert bad > 0


@pytest.mark.parametrize("D,CR", [(1, 0.5), (2, 0.3), (3, 0.5), (4, 0.7)])
def test_bin_mask_distribution_enumerated(D, CR):
    p = float(p_less(CR))
    pj = [float(v) for v in jrand_prob(D)]
    exact = {}
    for bits in itertools.product([0, 1], repeat=D):
        pr = 0.0
        for j in range(D):
            if bits[j] != 1:
                continue
            q = pj[j]
            for k in range(D):
                if k != j:
                    q *= p if bits[k] else (1 - p)
            pr += q
        exact[bits] = pr
    n = 40000
    seed = 21
    counts = {b: 0 for b in exact}
    for k in range(n):
        g, i = 1 + k // 1000, k % 1000
        w0 = oracle.word(seed, 0, "xo", g, i, 0, 0)
        jr = oracle.randint(w0, D)
        m = tuple(int(v) for v in oracle.mask_bin(seed, 0, D, CR, g, i, jr))
        counts[m] += 1
    keys = [b for b in exact if exact[b] > 0]
    assert sum(counts[b] for b in exact if exact[b] == 0) == 0
    obs = [counts[b] for b in keys]
    expv = [exact[b] * n for b in keys]
    assert merged_chisquare(obs, expv) > 1e-3


@pytest.mark.parametrize("D", [1, 5, 64])
def test_bin_mask_extremes(D):
    for g in range(1, 20):
        jr = g % D
        m0 = oracle.mask_bin(3, 0, D, 0.0, g, 2, jr)
        assert m0.sum() == 1 and m0[jr] == 1
        m1 = oracle.mask_bin(3, 0, D, 1.0, g, 2, jr)
        assert m1.sum() == D
