"""The allocation-free mask entry point against de_masks (GPU).

de_masks_noalloc keeps its run record and NEC table in the library's static
device array; its bytes must equal those de_masks writes for a handle built
from the same run description, call after call (the second call of each case
is smaller, so stale contents of the array from the first would show), and
for a run at a non-zero position of a batched handle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2101_06599_amd as de
    de.lib()
    yield


def run(xo, impl="lane", **kw):
    d = dict(N=1000, D=777, F=0.5, CR=0.9, xo=xo, exp_impl=impl, fn="sphere", dtype="fp32",
             seed=7)
    d.update(kw)
    return d


def handle_masks(cfgs, r, gen):
    import paper_2101_06599_amd as de
    h = de.DE(cfgs, device="cuda:0")
    try:
        return h.masks(r, gen).cpu().numpy()
    finally:
        h.close()


def noalloc_masks(cfg, gen, run_index=0):
    import torch

    import paper_2101_06599_amd as de
    out = torch.full((cfg["N"], cfg["D"]), 7, dtype=torch.uint8, device="cuda:0")
    de.masks_noalloc(cfg, gen, out, run_index)
    return out.cpu().numpy()


@pytest.mark.parametrize("xo,impl", [("nec", "lane"), ("bin", "lane"), ("exp", "lane"),
                                     ("exp", "scan"), ("exp", "job")])
def test_noalloc_masks_equal_handle_masks_twice(xo, impl):
    big = run(xo, impl)
    small = run(xo, impl, N=37, D=50, CR=0.6, seed=3)
    for cfg, gen in ((big, 5), (small, 2)):
        ref = handle_masks([cfg], 0, gen)
        got = noalloc_masks(cfg, gen)
        assert np.array_equal(got, ref), f"{xo}/{impl} N={cfg['N']} D={cfg['D']}"
        assert set(np.unique(got).tolist()) <= {0, 1}


@pytest.mark.parametrize("CR", [0.0, 0.5, 0.999, 1.0])
def test_noalloc_nec_table_edges(CR):
    # long tables (CR close to 1), and CR = 0, 1 that read no table
    for cfg, gen in ((run("nec", N=64, D=20000, CR=CR), 3), (run("nec", N=64, D=9, CR=CR), 4)):
        assert np.array_equal(noalloc_masks(cfg, gen), handle_masks([cfg], 0, gen))


def test_noalloc_run_index_of_a_batched_handle():
    a = run("nec", N=40, D=300, CR=0.8, fn="rastrigin", olo=-4.0, ohi=4.0)
    b = run("nec", N=90, D=123, CR=0.95, fn="rastrigin", olo=-4.0, ohi=4.0)
    ref = handle_masks([a, b], 1, 6)
    assert np.array_equal(noalloc_masks(b, 6, run_index=1), ref)
    assert not np.array_equal(noalloc_masks(b, 6, run_index=0), ref)


def test_noalloc_rejects_oversized_tables():
    import torch

    import paper_2101_06599_amd as de
    out = torch.empty(8, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(de.DEError) as e:
        de.masks_noalloc(run("nec", N=4, D=131007), 1, out)
    assert e.value.status == de.E_INVALID and "DE_MASKS_NOALLOC_MAX_D" in str(e.value)
