"""Helpers for the GPU parity tests: build the same run on the GPU (through
the C ABI) and in the oracle, and compare one generation at a time.

Bar (see the module docstring of test_gpu_parity.py): integer decisions and
trial vectors bit-exact; fitness within tol * Phi; a selection decision may
differ only where the two fitness values are within that bound, after which
the GPU state is re-synchronised from the oracle."""
from __future__ import annotations

import numpy as np

import oracle

TOL = {"fp64": 1e-12, "fp32": 1e-5, "bf16x6": 1e-6, "bf16x3": 1e-4}
ORACLE_KEYS = ("N", "D", "F", "CR", "xo", "fn", "dtype", "lo", "hi", "olo", "ohi", "seed", "base",
               "shuffle")


def tol_of(cfg) -> float:
    if cfg.get("fn") == "ellipsoid_rot" and cfg.get("mm") in ("bf16x3", "bf16x6"):
        return TOL[cfg["mm"]]
    return TOL[cfg.get("dtype", "fp64")]


def rotation(D: int, seed: int = 0) -> np.ndarray:
    from paper_2101_06599_amd import synth
    return synth.rotation(D, seed)


def oracle_run(cfg, run=0, rot=None, lazy=False):
    kw = {k: cfg[k] for k in ORACLE_KEYS if k in cfg}
    return oracle.Run(run=run, rot=rot, lazy=lazy, **kw)


def gpu_runs(cfgs, rot_np=None):
    """cfg dicts for de.DE (rotation passed as a device tensor)."""
    import torch
    out = []
    for c in cfgs:
        c = dict(c)
        if c.get("fn") == "ellipsoid_rot":
            c["rot"] = torch.as_tensor(rot_np, dtype=torch.float64, device="cuda:0").contiguous()
        out.append(c)
    return out


def phi_rows(cfg, X, o, rot):
    return oracle.fitness_phi(cfg["fn"], X, o, rot)


def compare_generation(gpu, ref, cfg, run=0, resync=True, rot=None, trace=None, stepped=False):
    """Advance both sides one generation and compare.  Returns the number of
    selection flips (re-synchronised)."""
    import torch
    tol = tol_of(cfg)
    o = ref.shift()
    pop_r0, fit_r0, g0 = ref.state()
    if trace is None:
        trace = gpu.trace(run)
    if not stepped:
        gpu.generation(1)
    rt = ref.generation(1, trace=True)
    torch.cuda.synchronize()
    gi = trace["idx"].cpu().numpy()
    gm = trace["mask"].cpu().numpy()
    gt = trace["trial"].cpu().numpy().astype(np.float64)
    gf = trace["ftrial"].cpu().numpy().astype(np.float64)
    ri = rt["idx"]
    assert np.array_equal(gi[:, :5], ri[:, :5]), _first_diff(gi[:, :5], ri[:, :5], "indices/L")
    assert np.array_equal(gm, rt["mask"]), _first_diff(gm, rt["mask"], "mask")
    assert np.array_equal(gt, rt["trial"], equal_nan=True), _first_diff(gt, rt["trial"], "trial")
    phi_u = phi_rows(cfg, rt["trial"], o, rot)
    err = fit_err(gf, rt["ftrial"])
    assert np.all(err <= tol * phi_u), f"trial fitness: max rel {np.max(err / phi_u):.3e}"
    win_g = gi[:, 5].astype(bool)
    win_r = ri[:, 5].astype(bool)
    flips = np.nonzero(win_g != win_r)[0]
    if flips.size:
        phi_x = phi_rows(cfg, pop_r0[flips], o, rot)
        gap = np.abs(rt["ftrial"][flips] - fit_r0[flips])
        assert np.all(gap <= tol * np.maximum(phi_u[flips], phi_x)), (
            f"selection differs outside the tolerance at rows {flips[:8]}")
    pop_g, fit_g, gg = gpu.state(run)
    pop_r, fit_r, gr = ref.state()
    assert gg == gr == g0 + 1
    if flips.size == 0:
        assert np.array_equal(pop_g.astype(np.float64), pop_r, equal_nan=True), "population differs"
        phi_x = phi_rows(cfg, pop_r, o, rot)
        assert np.all(fit_err(fit_g.astype(np.float64), fit_r) <= tol * phi_x)
    elif resync:
        bf, bi, bgen, _ = ref.best()
        gpu.set_state(run, pop_r, fit_r, gr, bf, bi, bgen)
    return int(flips.size)


def fit_err(a, b):
    """|a - b| with equal infinities (NaN fitness counts as +inf) at zero."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    same_inf = np.isinf(a) & np.isinf(b) & (np.sign(a) == np.sign(b))
    with np.errstate(invalid="ignore"):  # inf - inf where same_inf picks 0
        return np.where(same_inf, 0.0, np.abs(a - b))


def _first_diff(a, b, what):
    idx = np.argwhere((a != b) & ~(np.isnan(a) & np.isnan(b)))
    if idx.size == 0:
        return what
    k = tuple(idx[0])
    return f"{what} differs first at {k}: gpu {a[k]!r} oracle {b[k]!r} ({len(idx)} cells)"
