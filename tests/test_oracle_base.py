"""Pins for the oracle's base-index schemes (Alg 3, 4, 5 with Alg 6's
offsets), its keyed permutation and the per-generation shuffle (Alg 2):
bijection by brute force, uniformity over many generations, the structural
property each algorithm states, the shuffle as "reorder, then run the plain
generation", and convergence against a textbook DE that uses numpy's own
permutations (CPU only)."""
import numpy as np
import pytest

import oracle
from test_oracle_statistics import sphere


@pytest.mark.parametrize("N", [4, 5, 7, 16, 17, 63, 64, 65, 100, 1000, 4097])
def test_permutation_is_a_bijection(N):
    for tag in ("perm", "shuffle"):
        for g in (1, 2, 999):
            img = [oracle.permute(11, 0, tag, g, N, k) for k in range(N)]
            assert sorted(img) == list(range(N)), (N, tag, g)


def test_permutations_differ_by_generation_tag_seed_and_run():
    N = 50
    ref = [oracle.permute(3, 0, "perm", 1, N, k) for k in range(N)]
    assert ref != [oracle.permute(3, 0, "perm", 2, N, k) for k in range(N)]
    assert ref != [oracle.permute(3, 0, "shuffle", 1, N, k) for k in range(N)]
    assert ref != [oracle.permute(4, 0, "perm", 1, N, k) for k in range(N)]
    assert ref != [oracle.permute(3, 1, "perm", 1, N, k) for k in range(N)]
    assert ref != list(range(N))


@pytest.mark.parametrize("N", [6, 8])
def test_permutation_is_close_to_uniform(N):
    G = 3000
    C = np.zeros((N, N))
    fixed = 0
    for g in range(1, G + 1):
        img = [oracle.permute(5, 0, "shuffle", g, N, k) for k in range(N)]
        for k, v in enumerate(img):
            C[k, v] += 1
        fixed += sum(1 for k, v in enumerate(img) if k == v)
    # every cell ~ G / N; chi-square with (N-1)^2 degrees of freedom
    e = G / N
    chi2 = float(((C - e) ** 2 / e).sum())
    dof = (N - 1) ** 2
    assert chi2 < dof + 6 * np.sqrt(2 * dof), chi2
    # a uniform permutation has one fixed point on average (variance 1)
    assert abs(fixed / G - 1.0) < 0.1


def test_classic_scheme_is_the_distinct_index_rule():
    for g in (1, 7):
        for i in range(20):
            assert np.array_equal(oracle.indices_scheme(2, 0, "classic", 20, g, i),
                                  oracle.indices(2, 0, 20, g, i))


def _offsets(r, N):
    return (r[1] - r[0]) % N, (r[2] - r[1]) % N


@pytest.mark.parametrize("base", ["random", "offset", "perm"])
def test_alg6_offsets_lie_in_1_to_n_minus_1_and_are_uniform(base):
    N = 7
    cnt = np.zeros((2, N))
    for g in range(1, 400):
        for i in range(N):
            r = oracle.indices_scheme(9, 0, base, N, g, i)
            assert all(0 <= v < N for v in r)
            o1, o2 = _offsets(r, N)
            assert 1 <= o1 <= N - 1 and 1 <= o2 <= N - 1
            cnt[0, o1] += 1
            cnt[1, o2] += 1
    assert cnt[:, 0].sum() == 0
    e = 399 * N / (N - 1)
    for row in cnt[:, 1:]:
        assert float(((row - e) ** 2 / e).sum()) < (N - 2) + 6 * np.sqrt(2 * (N - 2))


def test_alg3_random_base_is_uniform_and_may_hit_i():
    N = 9
    cnt = np.zeros(N)
    hits_i = 0
    for g in range(1, 500):
        for i in range(N):
            r0 = oracle.indices_scheme(1, 0, "random", N, g, i)[0]
            cnt[r0] += 1
            hits_i += r0 == i
    e = 499
    assert float(((cnt - e) ** 2 / e).sum()) < (N - 1) + 6 * np.sqrt(2 * (N - 1))
    assert hits_i > 0


def test_alg4_offset_base_is_one_shift_per_generation():
    N = 13
    seen = set()
    for g in range(1, 300):
        shifts = {(oracle.indices_scheme(4, 2, "offset", N, g, i)[0] - i) % N for i in range(N)}
        assert len(shifts) == 1
        s = shifts.pop()
        assert 1 <= s <= N - 1  # ceil((N-1) U) never 0: r0 != i
        seen.add(s)
    assert seen == set(range(1, N))


def test_alg5_permutation_base_is_a_permutation():
    for N in (4, 30, 257):
        for g in (1, 2, 3):
            r0 = [oracle.indices_scheme(8, 0, "perm", N, g, i)[0] for i in range(N)]
            assert sorted(r0) == list(range(N))


@pytest.mark.parametrize("base", ["classic", "offset", "perm"])
@pytest.mark.parametrize("xo", ["bin", "nec"])
def test_shuffle_is_reorder_then_plain_generation(base, xo):
    """Alg 2's shuffle, then the rest of its generation: with the shuffle on, the generation equals
    the plain one run on the population reordered by pi_g, written back to
    the rows the individuals came from."""
    N, D, seed = 24, 9, 6
    kw = dict(N=N, D=D, F=0.7, CR=0.5, xo=xo, fn="rastrigin", lo=-5.0, hi=5.0, olo=-1.0, ohi=1.0,
              seed=seed, base=base)
    A = oracle.Run(shuffle=True, **kw)
    B = oracle.Run(shuffle=False, **kw)
    for g in (1, 2, 3):
        pop, fit, g0 = A.state()
        assert g0 == g - 1
        pi = np.array([oracle.permute(seed, 0, "shuffle", g, N, k) for k in range(N)])
        assert sorted(pi) == list(range(N))
        B.set_state(pop[pi], fit[pi], g - 1, np.inf, -1, 0)
        ta = A.generation(1, trace=True)
        tb = B.generation(1, trace=True)
        pa, fa, _ = A.state()
        pb, fb, _ = B.state()
        assert np.array_equal(pa[pi], pb) and np.array_equal(fa[pi], fb)
        assert np.array_equal(ta["mask"][pi], tb["mask"])
        assert np.array_equal(ta["trial"][pi], tb["trial"])
        assert np.array_equal(ta["idx"][pi][:, :3], pi[tb["idx"][:, :3]])  # rows read
        assert np.array_equal(ta["idx"][pi][:, 3:], tb["idx"][:, 3:])
    # the per-row recomputation finds the same trial for any storage row
    pop, fit, g0 = A.state()
    ta = A.generation(1, trace=True)
    for i in (0, 5, N - 1):
        r = A.individual(pop, g0 + 1, i)
        assert np.array_equal(r["trial"], ta["trial"][i])
        assert np.array_equal(r["idx"][:5], ta["idx"][i, :5])


def textbook_paper_scheme(N, D, F, CR, lo, hi, gens, seed, base):
    """DE/rand/1/bin with Alg 3/4/5 base selection and Alg 6 offsets, numpy RNG."""
    rng = np.random.default_rng(seed)
    X = rng.uniform(lo, hi, (N, D))
    f = sphere(X)
    rows = np.arange(N)
    for _ in range(gens):
        if base == "random":
            r0 = rng.integers(0, N, N)
        elif base == "offset":
            r0 = (rows + rng.integers(1, N)) % N
        else:
            r0 = rng.permutation(N)
        r1 = (r0 + rng.integers(1, N, N)) % N
        r2 = (r1 + rng.integers(1, N, N)) % N
        V = X[r0] + F * (X[r1] - X[r2])
        M = rng.random((N, D)) < CR
        M[rows, rng.integers(0, D, N)] = True
        U = np.where(M, V, X)
        fu = sphere(U)
        w = fu < f
        X[w] = U[w]
        f[w] = fu[w]
    return float(f.min())


@pytest.mark.parametrize("base", ["random", "offset", "perm"])
def test_paper_schemes_converge_like_a_textbook_implementation(base):
    N, D, F, CR, gens = 40, 20, 0.5, 0.9, 150
    tb = [textbook_paper_scheme(N, D, F, CR, -100.0, 100.0, gens, s, base) for s in range(6)]
    orc = []
    for s in range(6):
        r = oracle.Run(N=N, D=D, F=F, CR=CR, xo="bin", fn="sphere", seed=s, base=base)
        r.generation(gens)
        orc.append(r.best()[0])
    lt, lo_ = np.log(tb), np.log(orc)
    assert abs(lt.mean() - lo_.mean()) < np.log(3.0), (tb, orc)
