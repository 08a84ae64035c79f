"""Host-side pieces of the benchmark (CPU only): the byte model behind its
bandwidth fractions, checked against the oracle's own crossover laws; the
calibration of counter bytes; the counter summaries; the one-GPU guard."""
import csv
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("kind,D,CR", [("nec", 1000, 0.9), ("exp", 1000, 0.9),
                                       ("nec", 10000, 0.9), ("nec", 50, 0.5),
                                       ("exp", 10, 0.99), ("nec", 7, 0.0)])
def test_mask_density_is_the_mean_run_length_over_d(kind, D, CR):
    """rho for exp/NEC is E[L]/D of the truncated geometric law (Eq 3-4, Eq 9),
    here against lengths drawn by the oracle."""
    L = oracle.lengths(kind, D, CR, 200_000).astype(np.float64)
    se = L.std() / D / np.sqrt(len(L))
    assert abs(L.mean() / D - bench.rho(kind, D, CR)) <= 5 * se + 1e-12


@pytest.mark.parametrize("D,CR", [(100, 0.9), (10, 0.2), (1000, 0.0)])
def test_binomial_density_matches_oracle_masks(D, CR):
    """rho for bin is 1/D + (1 - 1/D) CR (Eq 2: each element with probability
    CR, and j_rand always), here against masks drawn by the oracle."""
    n = 2000
    m = np.stack([oracle.mask_bin(3, 0, D, CR, 1, i, i % D) for i in range(n)])
    p = bench.rho("bin", D, CR)
    se = np.sqrt(p * (1 - p) / (n * D))
    assert abs(m.mean() - p) <= 5 * se + 1e-12


def test_byte_bases_are_ordered():
    """The minimal bytes never exceed the algorithmic ones (w <= 1)."""
    for xo, D, CR in (("nec", 1000, 0.9), ("bin", 1000, 0.9), ("exp", 10000, 0.5)):
        for w in (0.0, 0.3, 1.0):
            assert bench.min_bytes(xo, 2048, D, CR, 8, w) <= bench.alg_bytes(xo, 2048, D, CR, 8)
    assert bench.alg_bytes("nec", 2048, 1000, 0.9, 8) == pytest.approx(33.26e6, rel=1e-3)


def _counter_csv(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name",
                                          "Counter_Value"])
        w.writeheader()
        for k, (name, ctr, val) in enumerate(rows):
            w.writerow({"Dispatch_Id": k, "Kernel_Name": name, "Counter_Name": ctr,
                        "Counter_Value": val})


def test_record_traffic_scales_by_the_copy_kernel(tmp_path):
    copy = "void at::native::vectorized_elementwise_kernel<4, at::native::neg_kernel_cuda(x)>(int)"
    gen = "void de::k_generation<double, 1, 2, 128, 2, false>(de::RunDev const*, int)"
    _counter_csv(str(tmp_path / "f" / "f_counter_collection.csv"),
                 [(copy, "FETCH_SIZE", 131072.0), (gen, "FETCH_SIZE", 1000.0),
                  (gen, "FETCH_SIZE", 3000.0)])
    _counter_csv(str(tmp_path / "w" / "w_counter_collection.csv"),
                 [(copy, "WRITE_SIZE", 262144.0), (gen, "WRITE_SIZE", 500.0)])
    out = str(tmp_path / "traffic.json")
    rec = bench.record_traffic([str(tmp_path / "f"), str(tmp_path / "w")], out)
    r = rec["c2_nec_fp64"]
    # the copy reads 256 MiB but FETCH_SIZE reports 128 MiB: scale 2; writes scale 1
    assert r["fetch_bytes"] == pytest.approx(2000 * 1024 * 2.0)
    assert r["write_bytes"] == pytest.approx(500 * 1024 * 1.0)
    assert r["bytes_per_launch"] == pytest.approx(r["fetch_bytes"] + r["write_bytes"])
    assert r["dispatches"] == [2, 1]
    assert r["source_sha"] == bench.source_sha()
    assert set(json.load(open(out))) == {"c2_nec_fp64"}


def test_counters_summary_prints_kernel_stats(tmp_path, capsys):
    p = tmp_path / "x_kernel_stats.csv"
    with open(p, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs",
                    "MaxNs", "StdDev"])
        w.writerow(["void de::k_masks<2>(de::RunDev const*, int)", 10, 220000, 22000.0, 50.0,
                    21000, 23000, 1.0])
    bench.counters_summary(str(tmp_path))
    assert "| `void de::k_masks<2>` | 10 | 22000.0 | 21000 | 23000 | 50.0 |" in capsys.readouterr().out


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_tuner_cache_keys_bucket_shapes(monkeypatch, tmp_path):
    """Shapes in the same power-of-two buckets of D and N share one cache
    record; other dtypes, functions or crossovers do not; records round-trip
    through the JSON cache."""
    from paper_2101_06599_amd import tune
    monkeypatch.setattr(tune, "_device", lambda: "gfx950-test")
    monkeypatch.setattr(tune, "CACHE", str(tmp_path / "cache.json"))
    assert [tune.bucket(v) for v in (1, 2, 3, 1000, 1024, 1025)] == [1, 2, 4, 1024, 1024, 2048]
    a = dict(D=1000, N=2048, dtype="fp64", fn="rastrigin", xo="nec")
    assert tune._key(a) == tune._key(dict(a, D=700, N=1500))
    for k, v in (("D", 1100), ("N", 4000), ("dtype", "fp32"), ("fn", "sphere"), ("xo", "bin")):
        assert tune._key(a) != tune._key(dict(a, **{k: v}))
    tune._store(tune._key(a), 128, {64: 0.01, 128: 0.009})
    best, table = tune.tune_tpr(dict(a, D=999), use_cache=True)  # served from the cache
    assert best == 128 and table == {64: 0.01, 128: 0.009}
