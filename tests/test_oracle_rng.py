"""Pins for the oracle's random-number layer (CPU only).

* Philox4x32-10 against rocRAND's own implementation of the same generator
  (its header-only engine, compiled for the host and used as a black box).
* The integer maps (randint, skip) against exact integer arithmetic and brute
  force on tiny inputs.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_probe(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand"):
        pytest.skip("hipcc / rocRAND headers not available")
    exe = str(tmp_path_factory.mktemp("probe") / "philox_probe")
    subprocess.check_call([hipcc, "-O1", "-x", "hip", "--offload-arch=gfx950",
                           os.path.join(HERE, "philox_rocrand_probe.cpp"), "-o", exe],
                          cwd=str(tmp_path_factory.getbasetemp()))
    return exe


def test_philox_matches_rocrand(rocrand_probe):
    rng = np.random.default_rng(12345)
    n = 3000
    seeds = rng.integers(0, 2**64, n, dtype=np.uint64)
    ctr = rng.integers(0, 2**32, (n, 4), dtype=np.uint64)
    ctr[:, 1] %= 2**30  # the probe passes c1 through a 64-bit offset of 4*(c1:c0)
    ctr[:10] = 0        # include the all-zero counter with assorted keys
    lines = "\n".join(f"{int(s)} {c[0]} {c[1]} {c[2]} {c[3]}" for s, c in zip(seeds, ctr))
    out = subprocess.run([rocrand_probe], input=lines, capture_output=True, text=True,
                         check=True).stdout.split("\n")
    for k in range(n):
        s = int(seeds[k])
        key = [s & 0xFFFFFFFF, s >> 32]
        mine = oracle.philox([int(v) for v in ctr[k]], key)
        ref = [int(v) for v in out[k].split()]
        assert list(mine) == ref, (k, s, ctr[k])


def test_word_layout_addresses_counter_fields():
    # word(seed, run, tag, g, i, block, k) must be word k of philox(block, i, g, tag<<24|run)
    seed = 0x0123456789ABCDEF
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for (run, tag, g, i, block) in [(0, 3, 1, 0, 0), (7, 5, 1000, 2047, 249), (511, 6, 3, 9, 2)]:
        blk = oracle.philox([block, i, g, (tag << 24) | run], key)
        for k in range(4):
            assert oracle.word(seed, run, tag, g, i, block, k) == blk[k]


def test_uniform_open_interval_and_monotone():
    ws = [0, 1, 2, 2**31, 2**32 - 2, 2**32 - 1]
    us = [oracle.uniform(w) for w in ws]
    assert us[0] == 2.0**-33
    assert us[-1] == 1.0 - 2.0**-33
    assert all(0.0 < u < 1.0 for u in us)
    assert all(a < b for a, b in zip(us, us[1:]))


@pytest.mark.parametrize("n", [1, 2, 3, 7, 10, 47, 1000, 2045, 4093, 10000, 2**20 + 7])
def test_randint_boundaries_exact(n):
    # value r is taken exactly for w in [ceil(r 2^32 / n), ceil((r+1) 2^32 / n))
    rs = sorted(set([0, 1, n // 2, n - 2, n - 1] + list(range(0, n, max(1, n // 37)))))
    for r in rs:
        if r < 0 or r >= n:
            continue
        b = -((-r * 2**32) // n)  # ceil
        assert oracle.randint(b, n) == r
        if b > 0:
            assert oracle.randint(b - 1, n) == r - 1
    assert oracle.randint(2**32 - 1, n) == n - 1
    assert oracle.randint(0, n) == 0


def test_skip_is_order_preserving_bijection_bruteforce():
    import itertools
    for n in range(1, 11):
        for size in range(0, 4):
            for S in itertools.combinations(range(n), size):
                if n - size <= 0:
                    continue
                comp = [v for v in range(n) if v not in S]
                for perm in set(itertools.permutations(S)):
                    got = [oracle.skip(r, perm) for r in range(n - size)]
                    assert got == comp, (n, perm)


@pytest.mark.parametrize("N", [4, 5, 50, 2048])
def test_indices_distinct_and_uniform(N):
    from scipy.stats import chisquare
    seed = 7
    counts = np.zeros((3, N), np.int64)
    i = N // 3
    G = 4000 if N <= 50 else 20000
    for g in range(1, G + 1):
        r = oracle.indices(seed, 0, N, g, i)
        assert len({int(r[0]), int(r[1]), int(r[2]), i}) == 4
        assert all(0 <= v < N for v in r)
        counts[np.arange(3), r] += 1
    if N <= 50:
        for k in range(3):
            obs = np.delete(counts[k], i)
            assert chisquare(obs).pvalue > 1e-3
