"""Pins for the oracle's whole generation (CPU only): Alg 2's assembly of
index choice, mask, masked mutation, evaluation and greedy selection."""
import numpy as np
import pytest

import oracle


def small(xo="bin", **kw):
    args = dict(N=50, D=10, F=0.5, CR=0.9, xo=xo, fn="sphere", lo=-100.0, hi=100.0, seed=0)
    args.update(kw)
    return oracle.Run(**args)


@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
def test_init_in_box_and_uniform(dtype):
    from scipy.stats import chisquare
    r = oracle.Run(N=400, D=50, fn="rastrigin", dtype=dtype, lo=-5.12, hi=5.12, olo=-4, ohi=4)
    pop, fit, g = r.state()
    assert g == 0
    assert pop.min() >= -5.12 and pop.max() <= 5.12
    if dtype == "fp32":
        assert np.array_equal(pop.astype(np.float32).astype(np.float64), pop)
    h = np.histogram(pop, bins=16, range=(-5.12, 5.12))[0]
    assert chisquare(h).pvalue > 1e-3
    o = r.shift()
    assert o.min() >= -4 and o.max() <= 4 and np.unique(o).size == 50
    assert np.allclose(fit, oracle.fitness("rastrigin", pop, o), rtol=0, atol=0)


def test_deterministic_and_seed_sensitive():
    a, b, c = small(), small(), small(seed=1)
    for r in (a, b, c):
        r.generation(7)
    pa, fa, _ = a.state()
    pb, fb, _ = b.state()
    pc, _, _ = c.state()
    assert np.array_equal(pa, pb) and np.array_equal(fa, fb)
    assert not np.array_equal(pa, pc)


@pytest.mark.parametrize("xo", ["bin", "exp", "nec"])
def test_masked_mutation_exact_on_integer_population(xo):
    # even integers with F = 0.5: every trial value is exact, so the expected
    # trial follows from the traced indices and mask alone
    N, D = 30, 12
    r = small(xo=xo, N=N, D=D, F=0.5, CR=0.6)
    rng = np.random.default_rng(9)
    pop = 2.0 * rng.integers(-50, 50, (N, D))
    fit = oracle.fitness("sphere", pop)
    r.set_state(pop, fit, 5, float(fit.min()), int(fit.argmin()), 5)
    t = r.generation(1, trace=True)
    idx, mask, trial = t["idx"], t["mask"].astype(bool), t["trial"]
    for i in range(N):
        r0, r1, r2, jr, L, win = idx[i]
        assert len({i, r0, r1, r2}) == 4
        assert mask[i, jr]
        v = pop[r0] + 0.5 * (pop[r1] - pop[r2])
        assert np.array_equal(trial[i], np.where(mask[i], v, pop[i]))
        if xo != "bin":
            assert mask[i].sum() == L
            assert np.array_equal(mask[i], oracle.alg9_mask(D, jr, L).astype(bool))
        assert t["ftrial"][i] == oracle.fitness("sphere", trial[i])
        assert win == (t["ftrial"][i] < fit[i])
    new_pop, new_fit, g = r.state()
    assert g == 6
    for i in range(N):
        exp_row = trial[i] if idx[i, 5] else pop[i]
        assert np.array_equal(new_pop[i], exp_row)


def test_zero_F_copies_base_vector():
    r = small(F=0.0, CR=0.7)
    pop, _, _ = r.state()
    t = r.generation(1, trace=True)
    for i in range(50):
        r0 = t["idx"][i, 0]
        m = t["mask"][i].astype(bool)
        assert np.array_equal(t["trial"][i][m], pop[r0][m])


def test_selection_strict_and_monotone():
    r = small(xo="nec", N=40, D=8)
    _, prev, _ = r.state()
    best_hist = [r.best()[0]]
    for _ in range(30):
        t = r.generation(1, trace=True)
        _, fit, _ = r.state()
        assert np.all(fit <= prev)
        win = t["idx"][:, 5].astype(bool)
        assert np.array_equal(win, t["ftrial"] < prev)
        assert np.array_equal(fit[win], t["ftrial"][win])
        assert np.array_equal(fit[~win], prev[~win])
        prev = fit
        bf, bi, bg, xb = r.best()
        best_hist.append(bf)
        assert bf == fit.min() and bi == int(np.argmin(fit))
        assert oracle.fitness("sphere", xb) == bf
    assert all(a >= b for a, b in zip(best_hist, best_hist[1:]))


def test_ties_keep_parent():
    N, D = 10, 5
    r = small(N=N, D=D)
    pop = np.tile(np.arange(D, dtype=np.float64), (N, 1))
    fit = oracle.fitness("sphere", pop)
    r.set_state(pop, fit, 0, float(fit[0]), 0, 0)
    t = r.generation(3, trace=True)
    assert t["idx"][:, 5].sum() == 0
    assert np.array_equal(r.state()[0], pop)


def test_nan_trial_never_wins():
    N, D = 8, 4
    r = small(N=N, D=D, CR=1.0)
    pop = np.random.default_rng(0).uniform(-1, 1, (N, D))
    pop[3] = np.nan
    fit = oracle.fitness("sphere", pop)
    assert fit[3] == np.inf
    r.set_state(pop, fit, 0, float(np.min(fit)), int(np.argmin(fit)), 0)
    for _ in range(5):
        t = r.generation(1, trace=True)
        bad = np.isnan(t["trial"]).any(axis=1)
        assert not t["idx"][bad, 5].any()
        assert np.all(t["ftrial"][bad] == np.inf)


def test_checkpoint_resume_identity():
    a = small(xo="exp")
    a.generation(20)
    b = small(xo="exp")
    b.generation(9)
    pop, fit, g = b.state()
    bf, bi, bg, _ = b.best()
    c = small(xo="exp", seed=0)
    c.set_state(pop, fit, g, bf, bi, bg)
    c.generation(11)
    pa, fa, ga = a.state()
    pc, fc, gc = c.state()
    assert ga == gc == 20
    assert np.array_equal(pa, pc) and np.array_equal(fa, fc)
    assert a.best()[:3] == c.best()[:3]


@pytest.mark.parametrize("CR", [0.0, 1.0])
def test_crossovers_coincide_at_extreme_cr(CR):
    # Cr = 0: every crossover is the one-hot mask at j_rand; Cr = 1: the full mask
    runs = [small(xo=x, CR=CR) for x in ("bin", "exp", "nec")]
    for r in runs:
        r.generation(25)
    ref = runs[0].state()
    for r in runs[1:]:
        s = r.state()
        assert np.array_equal(ref[0], s[0]) and np.array_equal(ref[1], s[1])


@pytest.mark.parametrize("xo", ["bin", "exp", "nec"])
def test_sphere_d10_converges(xo):
    r = small(xo=xo)
    f0 = r.best()[0]
    r.generation(100)
    f, _, g, _ = r.best()
    assert f < f0 * 1e-3 and 0 < g <= 100


def test_fp32_trials_are_float_values():
    r = small(dtype="fp32", fn="rosenbrock", lo=-5.12, hi=5.12, olo=-4, ohi=4, N=20, D=16)
    t = r.generation(1, trace=True)
    tr = t["trial"]
    assert np.array_equal(tr.astype(np.float32).astype(np.float64), tr)


@pytest.mark.parametrize("xo,fn,base,shuffle", [("nec", "rastrigin", "classic", False),
                                                ("bin", "griewank", "perm", True),
                                                ("exp", "rosenbrock", "offset", True)])
def test_openmp_build_matches_one_thread(xo, fn, base, shuffle):
    """The per-individual loops run in parallel: 1 and 4 threads give the
    same bits (populations, fitness, decisions, best record)."""
    kw = dict(N=37, D=23, F=0.6, CR=0.7, xo=xo, fn=fn, lo=-5.0, hi=5.0, olo=-1.0, ohi=1.0,
              seed=4, base=base, shuffle=shuffle)
    outs = []
    before = oracle.set_threads(0)
    try:
        for n in (1, 4):
            oracle.set_threads(n)
            r = oracle.Run(**kw)
            r.generation(20)
            t = r.generation(1, trace=True)
            outs.append((r.state(), r.best(), t))
    finally:
        oracle.set_threads(before)
    (s1, b1, t1), (s4, b4, t4) = outs
    assert np.array_equal(s1[0], s4[0]) and np.array_equal(s1[1], s4[1]) and s1[2] == s4[2]
    assert b1[:3] == b4[:3] and np.array_equal(b1[3], b4[3])
    for k in t1:
        assert np.array_equal(t1[k], t4[k]), k
