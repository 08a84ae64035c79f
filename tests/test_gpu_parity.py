"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bar:
* integer work bit-exact: r0, r1, r2, j_rand, L, the crossover mask, and
  every selection bit except near-ties (below);
* trial vectors bit-exact (FP64 and FP32: both sides use one fused
  multiply-add on the rounded difference, no other contraction);
* fitness within tol * Phi, Phi = f on absolute sub-terms: tol = 1e-12 (FP64),
  1e-5 (FP32), 1e-6 (rotated, split bf16 into 3 pieces), 1e-4 (2 pieces);
* a selection bit may differ only where |f(u) - f(x)| <= tol * max(Phi); the
  GPU is then re-synchronised from the oracle so a flip does not cascade.
"""
import os

import numpy as np
import pytest

import oracle
from parity_util import compare_generation, gpu_runs, oracle_run, rotation, tol_of

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2101_06599_amd as de
    de.lib()
    yield


def DE(cfgs, rot=None):
    import paper_2101_06599_amd as de
    return de.DE(gpu_runs(cfgs, rot), device="cuda:0")


def c1(xo, **kw):
    d = dict(N=50, D=10, F=0.5, CR=0.9, xo=xo, fn="sphere", dtype="fp64", lo=-100.0, hi=100.0,
             seed=0)
    d.update(kw)
    return d


def rast(**kw):
    d = dict(N=64, D=1000, F=0.5, CR=0.9, xo="nec", fn="rastrigin", dtype="fp64", lo=-5.12,
             hi=5.12, olo=-4.0, ohi=4.0, seed=3)
    d.update(kw)
    return d


def rosen(**kw):
    d = dict(N=12, D=1037, F=0.5, CR=0.9, xo="bin", fn="rosenbrock", dtype="fp32", lo=-5.12,
             hi=5.12, olo=-4.0, ohi=4.0, seed=5)
    d.update(kw)
    return d


def run_parity(cfg, gens, rot=None):
    gpu = DE([cfg], rot)
    ref = oracle_run(cfg, rot=rot)
    pop_g, fit_g, _ = gpu.state(0)
    pop_r, fit_r, _ = ref.state()
    assert np.array_equal(pop_g.astype(np.float64), pop_r), "initial population"
    phi = oracle.fitness_phi(cfg["fn"], pop_r, ref.shift(), rot)
    assert np.all(np.abs(fit_g - fit_r) <= tol_of(cfg) * phi), "initial fitness"
    trace = gpu.trace(0)
    flips = 0
    for _ in range(gens):
        flips += compare_generation(gpu, ref, cfg, rot=rot, trace=trace)
    return gpu, ref, flips


# ---- the sphere workload, D = 10, N = 50, 100 generations ---------------

@pytest.mark.parametrize("xo,impl", [("bin", "lane"), ("exp", "lane"), ("exp", "scan"),
                                     ("exp", "job"), ("nec", "lane")])
def test_sphere_d10_100_generations(xo, impl):
    cfg = c1(xo, exp_impl=impl)
    gpu, ref, flips = run_parity(cfg, 100)
    fb, ib, gb, xb = gpu.best(0)
    rb, rib, rgb, rxb = ref.best()
    assert flips == 0
    assert (ib, gb) == (rib, rgb)
    assert abs(fb - rb) <= 1e-12 * rb
    assert np.array_equal(xb, rxb)


# ---- shifted Rastrigin, D = 1000 ------------------------------------------

@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
@pytest.mark.parametrize("xo,impl", [("nec", "lane"), ("bin", "lane"), ("exp", "lane"),
                                     ("exp", "scan"), ("exp", "job")])
def test_rastrigin_d1000(dtype, xo, impl):
    run_parity(rast(dtype=dtype, xo=xo, exp_impl=impl), 4)


@pytest.mark.parametrize("CR", [0.0, 0.2, 0.5, 1.0])
def test_rastrigin_cr_extremes(CR):
    for xo in ("bin", "exp", "nec"):
        run_parity(rast(N=16, D=300, CR=CR, xo=xo, exp_impl="scan"), 3)


# ---- shifted Rosenbrock: ragged rows on every row shape -------------------

@pytest.mark.parametrize("D", [2, 3, 7, 1037, 4500, 17001])
@pytest.mark.parametrize("xo", ["bin", "nec"])
def test_rosenbrock_row_shapes(D, xo):
    run_parity(rosen(D=D, xo=xo, N=8 if D > 4000 else 12), 2)


@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
def test_rosenbrock_d1000(dtype):
    run_parity(rosen(D=1000, N=40, dtype=dtype, xo="exp", exp_impl="scan"), 3)


# ---- launch shape does not change results ----------------------------------

@pytest.mark.parametrize("cfg", [rast(N=40, D=999, xo="bin"), rosen(D=1001, N=20, xo="nec")])
def test_row_width_invariance(cfg):
    outs = []
    for tpr in (64, 128, 256, 512, 1024):
        gpu = DE([dict(cfg, tpr=tpr)])
        tr = gpu.trace(0)
        gpu.generation(1)
        outs.append((tr["idx"].cpu().numpy().copy(), tr["trial"].cpu().numpy().copy(),
                     tr["ftrial"].cpu().numpy().astype(np.float64)))
        gpu.close()
    tol = tol_of(cfg)
    for o in outs[1:]:
        assert np.array_equal(o[0][:, :5], outs[0][0][:, :5])
        assert np.array_equal(o[1], outs[0][1])
        assert np.all(np.abs(o[2] - outs[0][2]) <= tol * np.abs(outs[0][2]))


# ---- Ackley and Griewank (Sec. 4), the Table 2 runs ----------------------

def table2(name, **kw):
    from paper_2101_06599_amd import synth
    d = dict(synth.TABLE2[name], xo="nec")
    d.pop("gens")
    d.update(kw)
    return d


@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
@pytest.mark.parametrize("xo", ["nec", "bin", "exp"])
@pytest.mark.parametrize("name", ["ackley", "griewank", "rosenbrock"])
def test_table2_runs(name, xo, dtype):
    gens = {"ackley": 3, "griewank": 5, "rosenbrock": 40}[name]
    run_parity(table2(name, xo=xo, dtype=dtype, exp_impl="scan"), gens)


@pytest.mark.parametrize("D", [1, 2, 7, 1037, 4500, 17001])
@pytest.mark.parametrize("name", ["ackley", "griewank"])
def test_two_statistic_row_shapes(name, D):
    run_parity(table2(name, D=D, N=8 if D > 4000 else 12, xo="bin"), 2)


@pytest.mark.parametrize("name", ["ackley", "griewank"])
def test_two_statistic_row_width_invariance(name):
    cfg = table2(name, D=1501, N=24, xo="nec")
    outs = []
    for tpr in (64, 128, 256, 512, 1024):
        gpu = DE([dict(cfg, tpr=tpr)])
        tr = gpu.trace(0)
        gpu.generation(1)
        outs.append((tr["idx"].cpu().numpy().copy(), tr["trial"].cpu().numpy().copy(),
                     tr["ftrial"].cpu().numpy().astype(np.float64)))
        gpu.close()
    ref = oracle_run(cfg)
    rt = ref.generation(1, trace=True)
    phi = oracle.fitness_phi(name, rt["trial"])
    for o in outs:
        assert np.array_equal(o[0][:, :5], rt["idx"][:, :5])
        assert np.array_equal(o[1], rt["trial"])
        assert np.all(np.abs(o[2] - rt["ftrial"]) <= tol_of(cfg) * phi)


@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
@pytest.mark.parametrize("name", ["ackley", "griewank"])
def test_two_statistic_evaluate_special_points(name, dtype):
    """de_evaluate at the optimum, integer / cosine points and random rows."""
    import torch
    D = 777
    cfg = table2(name, D=D, N=8, dtype=dtype)
    gpu = DE([cfg])
    j = np.arange(1, D + 1, dtype=np.float64)
    rows = [np.zeros(D), np.full(D, 3.0), np.full(D, -0.5), 2 * np.pi * np.sqrt(j),
            np.pi * np.sqrt(j)]
    rows += list(np.random.default_rng(4).uniform(cfg["lo"], cfg["hi"], (40, D)))
    dt = torch.float64 if dtype == "fp64" else torch.float32
    Xd = torch.as_tensor(np.array(rows), dtype=dt, device="cuda:0")
    Xr = Xd.cpu().numpy().astype(np.float64)
    f = gpu.evaluate(0, Xd).cpu().numpy().astype(np.float64)
    fr = oracle.fitness(name, Xr)
    phi = oracle.fitness_phi(name, Xr)
    assert np.all(np.abs(f - fr) <= tol_of(cfg) * phi)
    assert f[0] == 0.0 or abs(f[0]) <= 1e-15


@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
def test_ackley_near_optimum_relative_bar(dtype):
    """Near x = 0 the tolerance scale of Ackley is f itself (both terms of its
    cancellation-free form are >= 0), so the bar is tol * f: 1e-12 relative
    in FP64, 1e-5 in FP32.  de_evaluate on rows at shrinking scales, then 30
    generations of a run started in [-1e-4, 1e-4]^D."""
    import torch
    D = 1000
    tol = 1e-12 if dtype == "fp64" else 1e-5
    cfg = table2("ackley", D=D, N=64, dtype=dtype, lo=-1e-4, hi=1e-4)
    gpu = DE([cfg])
    rng = np.random.default_rng(21)
    rows = [rng.uniform(-s, s, D) for s in (1e-1, 1e-3, 1e-5, 1e-7) for _ in range(4)]
    dt = torch.float64 if dtype == "fp64" else torch.float32
    Xd = torch.as_tensor(np.array(rows), dtype=dt, device="cuda:0")
    Xr = Xd.cpu().numpy().astype(np.float64)
    f = gpu.evaluate(0, Xd).cpu().numpy().astype(np.float64)
    fr = oracle.fitness("ackley", Xr)
    assert np.all(oracle.fitness_phi("ackley", Xr) == fr)
    rel = np.abs(f - fr) / fr
    assert np.all(rel <= tol), f"max relative error {rel.max():.3e}"
    gpu.close()
    _, ref, _ = run_parity(cfg, 30)
    _, fit, _ = ref.state()
    assert fit.max() < 1e-3  # the run stayed near the optimum


@pytest.mark.parametrize("name", ["ackley", "griewank"])
def test_two_statistic_best_and_many_generations(name):
    """200 generations at Table 2's F and Cr (smaller N, D): selection and the
    best-so-far stay with the oracle; best f is the FP64 value of the row."""
    cfg = table2(name, D=64, N=40, xo="nec", dtype="fp32")
    gpu, ref, flips = run_parity(cfg, 200)
    f, idx, g, x = gpu.best(0)
    rf, ridx, rg, rx = ref.best()
    fr = oracle.fitness(name, x.astype(np.float64))
    assert abs(f - fr) <= 1e-12 * oracle.fitness_phi(name, x.astype(np.float64))
    if flips == 0:
        assert (idx, g) == (ridx, rg)


# ---- base index schemes (Alg 3-6) and the shuffle of Alg 2 -------------------

@pytest.mark.parametrize("shuffle", [False, True])
@pytest.mark.parametrize("base", ["classic", "random", "offset", "perm"])
@pytest.mark.parametrize("xo,dtype", [("bin", "fp64"), ("nec", "fp32")])
def test_base_schemes_and_shuffle(base, shuffle, xo, dtype):
    run_parity(rast(N=37, D=300, xo=xo, dtype=dtype, base=base, shuffle=shuffle), 4)


@pytest.mark.parametrize("N", [4, 5, 17, 1000])
def test_shuffle_and_permutation_small_and_ragged_populations(N):
    run_parity(rast(N=N, D=40, xo="nec", base="perm", shuffle=True), 3)


def test_shuffle_with_job_exp_and_rotated_paths():
    run_parity(rast(N=30, D=200, xo="exp", exp_impl="job", base="offset", shuffle=True), 3)
    rot = rotation(96, 5)
    run_parity(ell("fp32", "fp32", D=96, N=50, xo="nec", base="perm", shuffle=True), 2, rot=rot)


def test_batched_runs_with_mixed_schemes():
    from paper_2101_06599_amd import synth
    cfgs = synth.batch_table(n_runs=4, seed=3, max_D=200, max_N=50)
    for c, (b, sh) in zip(cfgs, [("random", True), ("offset", False), ("perm", True),
                                 ("classic", True)]):
        c["base"], c["shuffle"] = b, sh
    gpu = DE(cfgs)
    refs = [oracle_run(c, run=r) for r, c in enumerate(cfgs)]
    traces = [gpu.trace(r) for r in range(len(cfgs))]
    for _ in range(3):
        gpu.generation(1)
        for r, c in enumerate(cfgs):
            compare_generation(gpu, refs[r], c, run=r, trace=traces[r], stepped=True)


def test_shuffled_full_size_sampled_rows():
    from paper_2101_06599_amd import synth
    cfg = dict(synth.RASTRIGIN_D1000, xo="nec", dtype="fp64", base="perm", shuffle=True)
    sampled_rows(cfg, gens=3)


def test_shuffled_graph_replay_matches_direct_launches():
    cfgs = [rast(N=40, D=120, xo="bin", base="offset", shuffle=True)]
    a, b = DE(cfgs), DE(cfgs)
    b.graph(True)
    for n in (3, 100, 64):
        a.generation(n)
        b.generation(n)
    pa, fa, ga = a.state(0)
    pb, fb, gb = b.state(0)
    assert ga == gb == 167
    assert np.array_equal(pa, pb) and np.array_equal(fa, fb)
    assert a.best(0)[:3] == b.best(0)[:3]


# ---- exp / NEC rows longer than 4096 elements: streamed, not register-held ---

def streamed(fn, **kw):
    base = {"rastrigin": rast(), "rosenbrock": rosen(), "sphere": c1("nec"),
            "ackley": table2("ackley"), "griewank": table2("griewank")}[fn]
    d = dict(base, D=5003, N=10, CR=0.99, xo="nec")
    d.update(kw)
    return d


@pytest.mark.parametrize("fn", ["rastrigin", "rosenbrock", "sphere", "ackley", "griewank"])
@pytest.mark.parametrize("xo,impl,dtype", [("nec", "lane", "fp32"), ("exp", "scan", "fp64"),
                                           ("nec", "lane", "fp64")])
def test_streamed_rows(fn, xo, impl, dtype):
    # CR 0.99: runs of ~100 elements, many of them wrapping past D - 1
    run_parity(streamed(fn, xo=xo, exp_impl=impl, dtype=dtype), 4)


@pytest.mark.parametrize("fn", ["rastrigin", "rosenbrock"])
def test_streamed_row_width_invariance(fn):
    cfg = streamed(fn, D=4101, N=12, CR=0.9)
    outs = []
    for tpr in (64, 128, 256, 512, 1024):
        gpu = DE([dict(cfg, tpr=tpr)])
        tr = gpu.trace(0)
        gpu.generation(1)
        outs.append((tr["idx"].cpu().numpy().copy(), tr["trial"].cpu().numpy().copy(),
                     tr["ftrial"].cpu().numpy().astype(np.float64)))
        gpu.close()
    ref = oracle_run(cfg)
    rt = ref.generation(1, trace=True)
    phi = oracle.fitness_phi(fn, rt["trial"], ref.shift())
    for o in outs:
        assert np.array_equal(o[0][:, :5], rt["idx"][:, :5])
        assert np.array_equal(o[1], rt["trial"])
        assert np.all(np.abs(o[2] - rt["ftrial"]) <= tol_of(cfg) * phi)


def test_streamed_write_back_modes_agree():
    base = streamed("rosenbrock", D=4500, N=16, CR=0.95, dtype="fp32")
    outs = []
    for wb in ("whole", "partial", "auto"):
        gpu = DE([dict(base, wb=wb)])
        gpu.generation(60)
        outs.append((gpu.state(0), gpu.best(0)[:3]))
        gpu.close()
    for (st, b) in outs[1:]:
        assert np.array_equal(st[0], outs[0][0][0]) and np.array_equal(st[1], outs[0][0][1])
        assert b == outs[0][1]


# ---- partial write-back: winners write only where the buffers differ -------

@pytest.mark.parametrize("xo,impl,dtype", [("nec", "lane", "fp64"), ("exp", "scan", "fp32"),
                                           ("exp", "job", "fp64"), ("bin", "lane", "fp32")])
def test_partial_write_back_many_generations(xo, impl, dtype):
    # CR 0.6 keeps runs short, so most rows are written partially
    run_parity(rast(N=40, D=257, CR=0.6, xo=xo, exp_impl=impl, dtype=dtype, wb="partial"), 30)


def test_partial_write_back_paths():
    # rotated trial-only kernel, the shuffle, a wide row with the register-cache
    # overflow, and a resume (set_state leaves the buffers unrelated)
    rot = rotation(96, 4)
    run_parity(ell("fp32", "fp32", D=96, N=50, xo="nec", wb="partial"), 6, rot=rot)
    run_parity(rast(N=24, D=300, xo="nec", base="perm", shuffle=True, wb="partial"), 8)
    run_parity(rosen(D=4500, N=8, xo="nec", CR=0.99, wb="partial", tpr=64), 4)
    cfg = rast(N=30, D=200, CR=0.7, xo="nec", wb="partial")
    gpu, ref, _ = run_parity(cfg, 5)
    pop, fit, g = ref.state()
    bf, bi, bg, _ = ref.best()
    gpu.set_state(0, pop, fit, g, bf, bi, bg)
    trace = gpu.trace(0)
    for _ in range(10):
        compare_generation(gpu, ref, cfg, trace=trace)


@pytest.mark.parametrize("cfgs", ["single", "batched"])
def test_write_back_modes_agree(cfgs):
    from paper_2101_06599_amd import synth
    if cfgs == "single":
        base = [rast(N=64, D=500, CR=0.8, xo="nec", dtype="fp32")]
    else:
        base = synth.batch_table(n_runs=5, seed=4, max_D=300, max_N=40)
    outs = []
    for wb in ("whole", "partial", "auto"):
        gpu = DE([dict(c, wb=wb) for c in base])
        gpu.generation(150)
        outs.append([gpu.state(r) for r in range(len(base))] + [gpu.best(r)[:3] for r in range(len(base))])
        gpu.close()
    for o in outs[1:]:
        for a, b in zip(o[:len(base)], outs[0][:len(base)]):
            assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]
        assert o[len(base):] == outs[0][len(base):]


# ---- rotated ellipsoid on the matrix cores ---------------------------------

def ell(mm, dtype, **kw):
    d = dict(N=100, D=160, F=0.5, CR=0.9, xo="nec", fn="ellipsoid_rot", dtype=dtype, mm=mm,
             lo=-100.0, hi=100.0, olo=-80.0, ohi=80.0, seed=7)
    d.update(kw)
    return d


@pytest.mark.parametrize("mm,dtype", [("fp64", "fp64"), ("fp32", "fp32"), ("bf16x6", "fp32"),
                                      ("bf16x3", "fp32")])
@pytest.mark.parametrize("xo", ["nec", "bin"])
def test_rotated_ellipsoid(mm, dtype, xo):
    D = 160
    rot = rotation(D, 0)
    run_parity(ell(mm, dtype, xo=xo), 3, rot=rot)


@pytest.mark.parametrize("tile", [1, 2, 3])
@pytest.mark.parametrize("mm", ["bf16x6", "bf16x3"])
@pytest.mark.parametrize("N,D", [(100, 300), (300, 200)])
def test_rotated_tiles(mm, tile, N, D):
    """Every tile shape of the split-bf16 product at shapes ragged against
    the tiles: D against 128- and 256-wide columns and the 32-wide k slices,
    N below one tile of rows or a tile and a part; all shapes use the same
    matrix-core form and k order, so their fitness values agree bit for bit."""
    rot = rotation(D, 6)
    run_parity(ell(mm, "fp32", D=D, N=N, tile=tile), 3, rot=rot)
    if tile == 3:
        outs = []
        for t in (1, 2, 3):
            gpu = DE([ell(mm, "fp32", D=D, N=N, tile=t)], rot)
            tr = gpu.trace(0)
            gpu.generation(2)
            outs.append(tr["ftrial"].cpu().numpy().copy())
            gpu.close()
        assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])


@pytest.mark.parametrize("mm,dtype", [("fp64", "fp64"), ("fp32", "fp32"), ("bf16x6", "fp32"),
                                      ("bf16x3", "fp32")])
@pytest.mark.parametrize("D", [2, 20, 33])
def test_rotated_small_d(mm, dtype, D):
    """Rotated runs whose D is below one K slice of the product (16 or 32
    columns) or one past it, with fewer rows than one tile: the padding of the
    operands and the partial last slice."""
    rot = rotation(D, 8)
    run_parity(ell(mm, dtype, D=D, N=12), 3, rot=rot)


@pytest.mark.parametrize("mm", ["fp32", "bf16x6"])
def test_rotated_ellipsoid_exp_job(mm):
    rot = rotation(96, 1)
    run_parity(ell(mm, "fp32", D=96, N=70, xo="exp", exp_impl="job"), 2, rot=rot)


# ---- several runs in one launch --------------------------------------------

def test_batched_runs_match_independent_oracles():
    from paper_2101_06599_amd import synth
    cfgs = synth.batch_table(n_runs=6, seed=1, max_D=300, max_N=60)
    cfgs[1]["xo"] = "bin"
    cfgs[2]["xo"] = "exp"
    cfgs[2]["exp_impl"] = "scan"
    cfgs[3]["D"] = 1500  # past the register cache of a 64-lane row
    gpu = DE(cfgs)
    refs = [oracle_run(c, run=r) for r, c in enumerate(cfgs)]
    traces = [gpu.trace(r) for r in range(len(cfgs))]
    for _ in range(3):
        gpu.generation(1)
        for r, c in enumerate(cfgs):
            compare_generation(gpu, refs[r], c, run=r, trace=traces[r], stepped=True)


# ---- other entry points -----------------------------------------------------

def test_batched_512_table_sampled_runs():
    """The benchmark's full table of 512 runs in one handle: six runs spread
    over the table are traced and checked, each against its own oracle run,
    for two generations."""
    from paper_2101_06599_amd import synth
    cfgs = synth.batch_table(512, seed=0)
    gpu = DE(cfgs)
    sample = [0, 97, 211, 333, 402, 511]
    refs = {r: oracle_run(cfgs[r], run=r) for r in sample}
    for r in sample:
        pop_g, _, _ = gpu.state(r)
        assert np.array_equal(pop_g.astype(np.float64), refs[r].state()[0]), f"run {r} init"
    traces = {r: gpu.trace(r) for r in sample}
    for _ in range(2):
        gpu.generation(1)
        for r in sample:
            compare_generation(gpu, refs[r], cfgs[r], run=r, trace=traces[r], stepped=True)


@pytest.mark.parametrize("block", [100, 500])
def test_graph_blocks_of_any_length(block):
    """Graphs of `block` generations (best-so-far updated every 64 and at the
    end of a block) give the states and best records of direct launches."""
    from paper_2101_06599_amd import synth
    cfgs = synth.batch_table(n_runs=4, seed=3, max_D=200, max_N=40)
    a, b = DE(cfgs), DE(cfgs)
    b.graph(block)
    for n in (2 * block + 37, block):
        a.generation(n)
        b.generation(n)
    for r in range(len(cfgs)):
        pa, fa, ga = a.state(r)
        pb, fb, gb = b.state(r)
        assert ga == gb == 3 * block + 37
        assert np.array_equal(pa, pb) and np.array_equal(fa, fb)
        assert a.best(r)[:3] == b.best(r)[:3]


@pytest.mark.parametrize("cfg", [rast(dtype="fp64"), rast(dtype="fp32", fn="rosenbrock"),
                                 c1("bin")])
def test_evaluate_matches_oracle(cfg):
    import torch
    gpu = DE([cfg])
    ref = oracle_run(cfg)
    rng = np.random.default_rng(0)
    X = rng.uniform(-5, 5, (33, cfg["D"]))
    dt = torch.float64 if cfg["dtype"] == "fp64" else torch.float32
    Xd = torch.as_tensor(X, dtype=dt, device="cuda:0")
    Xr = Xd.cpu().numpy().astype(np.float64)
    f = gpu.evaluate(0, Xd).cpu().numpy().astype(np.float64)
    o = ref.shift()
    fr = oracle.fitness(cfg["fn"], Xr, o)
    phi = oracle.fitness_phi(cfg["fn"], Xr, o)
    assert np.all(np.abs(f - fr) <= tol_of(cfg) * phi)
    if cfg["fn"] != "sphere":  # the shift is the oracle's to the last bit
        f0 = gpu.evaluate(0, torch.as_tensor(o, dtype=dt, device="cuda:0")[None, :])
        assert float(f0.cpu()[0]) == 0.0


@pytest.mark.parametrize("fn", ["rastrigin", "ackley"])
@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
def test_sin_squared_term_accuracy(fn, dtype):
    """One-element rows across the whole argument range: the polynomial
    sin^2(pi z) keeps each term within a few ulp (far inside the parity bar)."""
    import torch
    cfg = dict(N=8, D=1, F=0.5, CR=0.9, xo="nec", fn=fn, dtype=dtype, lo=-5.0, hi=5.0,
               olo=-4.0, ohi=4.0, seed=2)
    gpu = DE([cfg])
    ref = oracle_run(cfg)
    o = ref.shift()
    rng = np.random.default_rng(5)
    ints = np.arange(-6, 7, dtype=np.float64)
    z = np.concatenate([rng.uniform(-6, 6, 20000), ints,
                        *[ints + d for d in (1e-12, -1e-7, 0.25, 0.5, -0.5, 0.49999)],
                        [1e4 + 0.3, -3e5 - 0.75, 1e-300, 0.0]])
    dt = torch.float64 if dtype == "fp64" else torch.float32
    Xd = torch.as_tensor((z + o[0])[:, None], dtype=dt, device="cuda:0")
    Xr = Xd.cpu().numpy().astype(np.float64)
    f = gpu.evaluate(0, Xd).cpu().numpy().astype(np.float64)
    fr = oracle.fitness(fn, Xr, o)
    phi = oracle.fitness_phi(fn, Xr, o)
    # the argument x - o is rounded once on the GPU: allow its effect on top
    # of a few ulp of the term
    eps = 2.0 ** -52 if dtype == "fp64" else 2.0 ** -23
    zz = np.abs(Xr[:, 0] - (o[0] if fn == "rastrigin" else 0.0))
    bound = eps * (8 * phi + 80 * np.pi * zz * np.maximum(zz, 1.0))
    if fn == "ackley":
        # sum x^2 is formed in the working precision: below the smallest
        # normal square it underflows, which moves -20 expm1(-0.02 sqrt(s1/D))
        # by at most 0.4 sqrt(smallest normal) (x = 1e-300 is such a point)
        bound = bound + 0.4 * np.sqrt(np.finfo(np.float64 if dtype == "fp64" else np.float32).tiny)
    bad = np.nonzero(np.abs(f - fr) > bound)[0]
    assert bad.size == 0, (bad[:5], Xr[bad[:5], 0], f[bad[:5]], fr[bad[:5]])


@pytest.mark.parametrize("mm,dtype,tol", [("fp64", "fp64", 1e-12), ("fp32", "fp32", 1e-5),
                                          ("bf16x6", "fp32", 1e-6), ("bf16x3", "fp32", 1e-4)])
def test_rotated_closed_forms(mm, dtype, tol):
    """Orthogonal M with a known effect, so f has a closed form without the
    oracle: M = I gives sum_k w_k d_k^2 and a permutation matrix P gives
    sum_k w_k d_{perm(k)}^2, with d = x - o."""
    import torch
    D = 200
    w = oracle.ellipsoid_weights(D)
    rng = np.random.default_rng(9)
    perm = rng.permutation(D)
    for permuted, M in ((False, np.eye(D)), (True, np.eye(D)[perm])):
        cfg = ell(mm, dtype, D=D, N=40)
        gpu = DE([cfg], M)
        o = oracle_run(cfg, rot=M, lazy=True).shift()
        dt = torch.float64 if dtype == "fp64" else torch.float32
        Xd = torch.as_tensor(rng.uniform(-100, 100, (60, D)), dtype=dt, device="cuda:0")
        Xr = Xd.cpu().numpy().astype(np.float64)
        f = gpu.evaluate(0, Xd).cpu().numpy().astype(np.float64)
        d = Xr - o
        closed = (w * (d[:, perm] if permuted else d) ** 2).sum(1)
        assert np.all(np.abs(f - closed) <= tol * closed), (mm, float(np.max(np.abs(f - closed) / closed)))
        gpu.close()


def test_evaluate_rotated():
    import torch
    D = 200
    rot = rotation(D, 2)
    for mm, dtype in (("fp64", "fp64"), ("fp32", "fp32"), ("bf16x6", "fp32")):
        cfg = ell(mm, dtype, D=D, N=50)
        gpu = DE([cfg], rot)
        ref = oracle_run(cfg, rot=rot)
        X = np.random.default_rng(1).uniform(-100, 100, (130, D))
        dt = torch.float64 if dtype == "fp64" else torch.float32
        Xd = torch.as_tensor(X, dtype=dt, device="cuda:0")
        Xr = Xd.cpu().numpy().astype(np.float64)
        f = gpu.evaluate(0, Xd).cpu().numpy().astype(np.float64)
        fr = oracle.fitness("ellipsoid_rot", Xr, ref.shift(), rot)
        assert np.all(np.abs(f - fr) <= tol_of(cfg) * fr), mm


@pytest.mark.parametrize("mm", ["bf16x3", "bf16x6"])
@pytest.mark.parametrize("extra", [dict(wb="whole", D=160), dict(wb="partial", D=161),
                                   dict(wb="partial", tpr=64, D=1102),
                                   dict(wb="whole", tpr=64, D=1102),
                                   dict(D=161, base="perm", shuffle=True),
                                   dict(D=161, xo="exp", exp_impl="job")])
def test_rotated_trial_pieces_match_split(mm, extra):
    """In the split-bf16 modes the trial kernel writes the bf16 pieces of
    (trial - o) that the product reads, in place of a split pass over the trial
    rows; de_evaluate still splits its rows.  Every stored fitness (winners'
    trials and kept parents) must therefore equal de_evaluate of the stored
    rows bit for bit.  Covers ragged D (odd last chunk), rows longer than the
    register cache of a 64-lane row (tpr 64, D 1102), both write-back modes,
    the shuffle, and the exp-job trials (which keep the split pass)."""
    import torch
    cfg = ell(mm, "fp32", N=70, CR=0.6)
    cfg.update(extra)
    rot = rotation(cfg["D"], 5)
    gpu = DE([cfg], rot)
    for _ in range(4):
        gpu.generation(1)
        pop, fit, _ = gpu.state(0)
        f = gpu.evaluate(0, torch.as_tensor(pop, device="cuda:0")).cpu().numpy()
        assert np.array_equal(f, fit), (mm, extra, np.nonzero(f != fit)[0][:5])
    gpu.close()


def test_best_is_fp64_recompute_of_best_row():
    cfg = rast(dtype="fp32", N=40, D=200)
    gpu = DE([cfg])
    gpu.generation(5)
    f, idx, g, x = gpu.best(0)
    pop, fit, gen = gpu.state(0)
    assert gen == 5 and 0 <= g <= 5
    assert np.array_equal(pop[idx], x)
    assert fit[idx] == fit.min()
    ref = oracle_run(cfg)
    fr = oracle.fitness("rastrigin", x.astype(np.float64), ref.shift())
    assert abs(f - fr) <= 1e-12 * fr


@pytest.mark.parametrize("mm,dtype,D", [("bf16x6", "fp32", 300), ("fp64", "fp64", 257),
                                        ("fp32", "fp32", 2)])
def test_best_rotated_is_fp64_recompute(mm, dtype, D):
    """de_best on the rotated function: the FP64 value of the best stored row
    with FP64 M and weights (one wavefront per z_k, then a fixed-order sum)."""
    rot = rotation(D, 5)
    cfg = ell(mm, dtype, D=D, N=64)
    gpu = DE([cfg], rot)
    gpu.generation(4)
    f, idx, g, x = gpu.best(0)
    pop, fit, _ = gpu.state(0)
    assert np.array_equal(pop[idx], x) and fit[idx] == fit.min()
    ref = oracle_run(cfg, rot=rot)
    fr = oracle.fitness("ellipsoid_rot", x.astype(np.float64), ref.shift(), rot)
    assert abs(f - fr) <= 1e-12 * fr


def test_determinism_and_resume():
    cfg = rast(N=50, D=500, xo="bin", dtype="fp32")
    a = DE([cfg])
    a.generation(12)
    b = DE([cfg])
    b.generation(5)
    pop, fit, g = b.state(0)
    fb, ib, gb, _ = b.best(0)
    c = DE([cfg])
    _, _, _ = c.state(0)
    fbest_stored = float(fit[ib])
    c.set_state(0, pop, fit, g, fbest_stored, ib, gb)
    c.generation(7)
    pa, fa, ga = a.state(0)
    pc, fc, gc = c.state(0)
    assert ga == gc == 12
    assert np.array_equal(pa, pc) and np.array_equal(fa, fc)
    assert a.best(0)[1:3] == c.best(0)[1:3]


# ---- full sizes, launch shapes of the benchmark, sampled rows ---------------

def sampled_rows(cfg, gens=1, n_sample=24, rot=None, seed=0):
    """Run `gens` generations at full size; check sampled rows of the last
    generation against the oracle's single-individual computation."""
    gpu = DE([cfg], rot)
    ref = oracle_run(cfg, rot=rot, lazy=True)
    if gens > 1:
        gpu.generation(gens - 1)
    pop_before, fit_before, g0 = gpu.state(0)
    tr = gpu.trace(0)
    gpu.generation(1)
    import torch
    torch.cuda.synchronize()
    rows = np.random.default_rng(seed).choice(cfg["N"], n_sample, replace=False)
    gi = tr["idx"].cpu().numpy()
    o = ref.shift()
    tol = tol_of(cfg)
    P = pop_before.astype(np.float64)
    for i in rows:
        r = ref.individual(P, g0 + 1, int(i))
        assert np.array_equal(gi[i, :5], r["idx"][:5]), (i, gi[i], r["idx"])
        assert np.array_equal(tr["mask"][int(i)].cpu().numpy(), r["mask"])
        gt = tr["trial"][int(i)].cpu().numpy().astype(np.float64)
        assert np.array_equal(gt, r["trial"])
        gf = float(tr["ftrial"][int(i)].cpu())
        phi = oracle.fitness_phi(cfg["fn"], r["trial"], o, rot)
        assert abs(gf - r["ftrial"]) <= tol * phi, (i, gf, r["ftrial"])
        win = gi[i, 5] == 1
        if abs(r["ftrial"] - float(fit_before[i])) > tol * phi:
            assert win == (r["ftrial"] < float(fit_before[i]))
    pop_after, fit_after, g1 = gpu.state(0)
    assert g1 == g0 + 1
    assert np.all(fit_after <= fit_before)
    return gpu


@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
@pytest.mark.parametrize("xo", ["nec", "bin", "exp"])
def test_full_size_rastrigin_2048x1000(dtype, xo):
    from paper_2101_06599_amd import synth
    cfg = dict(synth.RASTRIGIN_D1000, dtype=dtype, xo=xo, exp_impl="scan")
    sampled_rows(cfg, gens=3)


@pytest.mark.parametrize("xo", ["nec", "bin", "exp"])
def test_full_size_rosenbrock_8192x10000(xo):
    """The benchmark's three D = 10^4 variants: NEC and exp-scan rows are
    streamed, binomial rows held in registers."""
    from paper_2101_06599_amd import synth
    cfg = dict(synth.ROSENBROCK_D10000, xo=xo, exp_impl="scan")
    sampled_rows(cfg, gens=2, n_sample=12)


@pytest.mark.parametrize("mm,dtype", [("bf16x6", "fp32"), ("bf16x3", "fp32"), ("fp32", "fp32"),
                                      ("fp64", "fp64")])
def test_full_size_rotated_4096x2048(mm, dtype):
    from paper_2101_06599_amd import synth
    cfg = dict(synth.ELLIPSOID_D2048, mm=mm, dtype=dtype, xo="nec")
    sampled_rows(cfg, gens=2, n_sample=6, rot=rotation(2048, 0))


# ---- captured graphs replay the same generations ------------------------------

@pytest.mark.parametrize("kind", ["nec", "nec_partial", "rotated", "batched"])
def test_graph_replay_matches_direct_launches(kind):
    from paper_2101_06599_amd import synth
    rot = None
    if kind == "nec":
        cfgs = [rast(N=64, D=300, xo="nec", dtype="fp64")]
    elif kind == "nec_partial":
        cfgs = [rast(N=64, D=300, CR=0.7, xo="nec", dtype="fp32", wb="partial")]
    elif kind == "rotated":
        rot = rotation(96, 3)
        cfgs = [ell("fp32", "fp32", D=96, N=40, xo="bin")]
    else:
        cfgs = synth.batch_table(n_runs=5, seed=2, max_D=200, max_N=40)
    a, b = DE(cfgs, rot), DE(cfgs, rot)
    b.graph(True)
    for n in (5, 130, 64, 3, 70):
        a.generation(n)
        b.generation(n)
    # resume from a checkpoint in both, then more replayed blocks
    pop, fit, g = a.state(0)
    fb, ib, gb, _ = a.best(0)
    for h in (a, b):
        h.set_state(0, pop, fit, g + 7, float(fit[ib]), ib, gb)
        h.generation(150)
    for r in range(len(cfgs)):
        pa, fa, ga = a.state(r)
        pb, fb2, gb2 = b.state(r)
        assert ga == gb2
        assert np.array_equal(pa, pb) and np.array_equal(fa, fb2)
        assert a.best(r)[:3] == b.best(r)[:3]


def test_autotuned_row_width_gives_same_generations():
    from paper_2101_06599_amd.tune import tune_tpr
    cfg = rast(N=48, D=700, xo="nec", dtype="fp32")
    best, table = tune_tpr(cfg, gens=8, use_cache=False)
    assert best in (64, 128, 256, 512, 1024) and set(table) == {64, 128, 256, 512, 1024}
    assert all(v > 0 for v in table.values())
    a, b = DE([cfg]), DE([dict(cfg, tpr=best)])
    a.generation(20)
    b.generation(20)
    pa, fa, _ = a.state(0)
    pb, fb, _ = b.state(0)
    assert np.array_equal(pa, pb)
    assert np.all(np.abs(fa - fb) <= 1e-5 * np.abs(fa))


def test_autotuned_batch_and_tile_paths():
    """DE(..., tune=True) on a batched table and on a split-bf16 rotated run:
    the tuned widths and tile shapes are valid choices and the tuned handles
    step exactly like the handles they were tuned for."""
    from paper_2101_06599_amd import synth
    from paper_2101_06599_amd.tune import tune_batched, tune_rot_tile
    cfgs = synth.batch_table(n_runs=5, seed=4, max_D=300, max_N=60)
    best, table = tune_batched(cfgs, gens=4, use_cache=False)
    assert best in (64, 128, 256) and set(table) == {64, 128, 256}
    a, b = DE(cfgs), DE([dict(c, tpr=best) for c in cfgs])
    a.generation(10)
    b.generation(10)
    for r in range(len(cfgs)):
        pa, fa, _ = a.state(r)
        pb, fb, _ = b.state(r)
        assert np.array_equal(pa, pb)
        assert np.all(np.abs(fa - fb) <= 1e-5 * np.abs(fa))
    a.close()
    b.close()
    rot = rotation(160, 3)
    cfg = gpu_runs([ell("bf16x6", "fp32", D=160, N=64)], rot)[0]
    tile, ttab = tune_rot_tile(cfg, gens=2, use_cache=False)
    assert tile in (1, 2, 3) and set(ttab) == {1, 2, 3}
    run_parity(ell("bf16x6", "fp32", D=160, N=64, tile=tile), 2, rot=rot)


# ---- edge cases --------------------------------------------------------------

@pytest.mark.parametrize("xo,impl", [("bin", "lane"), ("exp", "scan"), ("exp", "job"),
                                     ("nec", "lane")])
@pytest.mark.parametrize("D", [1, 2])
def test_minimum_population_and_dimension(xo, impl, D):
    # N = 4: r0, r1, r2 are exactly the three other rows, in drawn order
    cfg = c1(xo, N=4, D=D, exp_impl=impl)
    gpu, ref, _ = run_parity(cfg, 30)
    assert gpu.best(0)[1:3] == ref.best()[1:3]


def test_large_population_tiny_dimension():
    cfg = dict(N=1 << 20, D=4, F=0.7, CR=0.5, xo="bin", fn="rastrigin", dtype="fp32",
               lo=-5.12, hi=5.12, olo=-4.0, ohi=4.0, seed=11)
    sampled_rows(cfg, gens=2, n_sample=64)


def test_huge_dimension_minimum_population():
    # rows far beyond the register cache of 1024 lanes, ragged tail
    cfg = dict(N=4, D=(1 << 20) - 3, F=0.5, CR=0.999, xo="nec", fn="rosenbrock",
               dtype="fp32", lo=-5.12, hi=5.12, olo=-4.0, ohi=4.0, seed=12)
    sampled_rows(cfg, gens=2, n_sample=4)


def test_nan_rows_never_win():
    cfg = rast(N=20, D=50, xo="bin", CR=1.0)
    gpu = DE([cfg])
    ref = oracle_run(cfg)
    pop, fit, g = ref.state()
    pop[3] = np.nan
    fit[3] = np.inf
    bf, bi, bg, _ = ref.best()
    ref.set_state(pop, fit, g, bf, bi, bg)
    gpu.set_state(0, pop, fit, g, bf, bi, bg)
    trace = gpu.trace(0)
    for _ in range(5):
        compare_generation(gpu, ref, cfg, trace=trace)
        t = trace["trial"].cpu().numpy()
        win = trace["idx"].cpu().numpy()[:, 5].astype(bool)
        assert not np.any(win & np.isnan(t).any(axis=1))
        assert np.isinf(trace["ftrial"].cpu().numpy()[np.isnan(t).any(axis=1)]).all()


def test_empty_calls():
    import torch
    gpu = DE([c1("nec")])
    before = gpu.state(0)
    gpu.generation(0)
    out = gpu.evaluate(0, torch.zeros((0, 10), dtype=torch.float64, device="cuda:0"))
    assert out.numel() == 0
    after = gpu.state(0)
    assert np.array_equal(before[0], after[0]) and before[2] == after[2] == 0


# ---- crossover masks on their own -----------------------------------------------

def oracle_mask(seed, D, CR, xo, g, i):
    jr = oracle.randint(oracle.word(seed, 0, "xo", g, i, 0, 0), D)
    if xo == "bin":
        return oracle.mask_bin(seed, 0, D, CR, g, i, jr)
    if xo == "exp":
        L = oracle.exp_length(seed, 0, D, CR, g, i)
    else:
        L = oracle.nec_length(oracle.uniform(oracle.word(seed, 0, "xo", g, i, 0, 1)), CR, D)
    return oracle.alg9_mask(D, jr, L)


@pytest.mark.parametrize("xo,impl", [("bin", "lane"), ("exp", "scan"), ("exp", "lane"),
                                     ("exp", "job"), ("nec", "lane")])
@pytest.mark.parametrize("D,N,CR", [(10, 100, 0.2), (13, 37, 0.6), (1000, 64, 0.8),
                                    (100, 30, 1.0), (257, 20, 0.0), (1, 5, 0.5)])
def test_masks_match_oracle(xo, impl, D, N, CR):
    cfg = dict(N=N, D=D, CR=CR, xo=xo, exp_impl=impl, fn="sphere", dtype="fp32", seed=9)
    gpu = DE([cfg])
    for g in (1, 2, 77):
        m = gpu.masks(0, g).cpu().numpy()
        for i in range(N):
            assert np.array_equal(m[i], oracle_mask(9, D, CR, xo, g, i)), (g, i)
    # the same masks the first generation applies
    tr = gpu.trace(0)
    m1 = gpu.masks(0, 1).cpu().numpy()
    gpu.generation(1)
    assert np.array_equal(tr["mask"].cpu().numpy(), m1)


@pytest.mark.parametrize("xo", ["nec", "bin"])
def test_masks_full_size_10000x10000(xo):
    N = D = 10000
    gpu = DE([dict(N=N, D=D, CR=0.6, xo=xo, fn="sphere", dtype="fp32", seed=0)])
    m = gpu.masks(0, 5)
    for i in np.random.default_rng(1).choice(N, 16, replace=False):
        assert np.array_equal(m[int(i)].cpu().numpy(), oracle_mask(0, D, 0.6, xo, 5, int(i)))
