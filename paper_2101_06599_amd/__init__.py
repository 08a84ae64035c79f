"""MI355X (gfx950) parallel differential evolution.

Python binding of the C ABI in ``include/de.h``: argument marshalling only.
Every step of a generation runs in the HIP kernels of ``libde.so``; torch is
used for device memory (the workspace and caller buffers) and for the stream.
Importing this package does not touch the GPU; the library is loaded on first
use and its absence is an error (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libde.so")

OK, E_INVALID, E_UNSUPPORTED, E_HIP, E_WORKSPACE, E_STATE = range(6)
XO = {"bin": 0, "exp": 1, "nec": 2}
EXP_IMPL = {"lane": 0, "job": 1, "scan": 2}
FN = {"sphere": 0, "rastrigin": 1, "rosenbrock": 2, "ellipsoid_rot": 3, "ackley": 4, "griewank": 5}
DTYPE = {"fp64": 0, "fp32": 1}
MM = {"fp64": 0, "fp32": 1, "bf16x3": 2, "bf16x6": 3}
BASE = {"classic": 0, "random": 1, "offset": 2, "perm": 3}
WB = {"auto": 0, "whole": 1, "partial": 2}

ABI_FUNCTIONS = ("de_workspace_size", "de_init", "de_generation", "de_evaluate", "de_best",
                 "de_get_state", "de_set_state", "de_trace", "de_profile", "de_profile_read",
                 "de_graph", "de_masks", "de_masks_noalloc", "de_last_error", "de_destroy")


class DEError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"status {status}: {msg}")
        self.status = status


class RunDesc(C.Structure):
    """Mirror of ``de_run_desc``."""
    _fields_ = [("N", C.c_int64), ("D", C.c_int64), ("F", C.c_double), ("CR", C.c_double),
                ("xo", C.c_int32), ("fn", C.c_int32), ("dtype", C.c_int32), ("mm", C.c_int32),
                ("exp_impl", C.c_int32), ("tpr", C.c_int32), ("base", C.c_int32),
                ("shuffle", C.c_int32), ("wb", C.c_int32), ("tile", C.c_int32),
                ("lo", C.c_double), ("hi", C.c_double), ("olo", C.c_double), ("ohi", C.c_double),
                ("seed", C.c_uint64), ("shift", C.c_void_p), ("rot", C.c_void_p)]


_lib = None


def lib():
    """Load libde.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        L.de_workspace_size.argtypes = [C.POINTER(RunDesc), i32, C.POINTER(C.c_size_t)]
        L.de_init.argtypes = [C.POINTER(vp), C.POINTER(RunDesc), i32, vp, C.c_size_t, vp]
        L.de_generation.argtypes = [vp, i32, vp]
        L.de_evaluate.argtypes = [vp, i32, vp, i64, vp, vp]
        L.de_best.argtypes = [vp, i32, C.POINTER(C.c_double), C.POINTER(i64), C.POINTER(i64), vp, vp]
        L.de_get_state.argtypes = [vp, i32, vp, vp, C.POINTER(i64), vp]
        L.de_set_state.argtypes = [vp, i32, vp, vp, i64, C.c_double, i64, i64, vp]
        L.de_trace.argtypes = [vp, i32, vp, vp, vp, vp]
        L.de_profile.argtypes = [vp, i32]
        L.de_profile_read.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(i64)]
        L.de_graph.argtypes = [vp, i32]
        L.de_masks.argtypes = [vp, i32, i64, vp, vp]
        L.de_masks_noalloc.argtypes = [C.POINTER(RunDesc), i32, i64, vp, vp]
        L.de_last_error.argtypes = [vp]
        L.de_last_error.restype = C.c_char_p
        L.de_destroy.argtypes = [vp]
        L.de_destroy.restype = None
        for name in ABI_FUNCTIONS:
            if name not in ("de_last_error", "de_destroy"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _desc(run: dict, keep: list) -> RunDesc:
    shift = run.get("shift")
    rot = run.get("rot")
    keep += [shift, rot]
    return RunDesc(
        N=int(run["N"]), D=int(run["D"]), F=float(run.get("F", 0.5)), CR=float(run.get("CR", 0.9)),
        xo=XO[run.get("xo", "bin")], fn=FN[run.get("fn", "sphere")],
        dtype=DTYPE[run.get("dtype", "fp64")], mm=MM[run.get("mm", "fp64")],
        exp_impl=EXP_IMPL[run.get("exp_impl", "lane")], tpr=int(run.get("tpr", 0)),
        base=BASE[run.get("base", "classic")], shuffle=1 if run.get("shuffle") else 0,
        wb=WB[run.get("wb", "auto")], tile=int(run.get("tile", 0)),
        lo=float(run.get("lo", -100.0)), hi=float(run.get("hi", 100.0)),
        olo=float(run.get("olo", 0.0)), ohi=float(run.get("ohi", 0.0)),
        seed=int(run.get("seed", 0)),
        shift=None if shift is None else shift.data_ptr(),
        rot=None if rot is None else rot.data_ptr())


def workspace_size(runs: list[dict]) -> int:
    keep: list = []
    arr = (RunDesc * len(runs))(*[_desc(r, keep) for r in runs])
    n = C.c_size_t(0)
    st = lib().de_workspace_size(arr, len(runs), C.byref(n))
    if st != OK:
        raise DEError(st, lib().de_last_error(None).decode())
    return n.value


def masks_noalloc(run: dict, gen: int, out, run_index: int = 0):
    """Crossover masks of generation `gen` for a run without a handle (the
    allocation-free entry point): `out` is a caller-owned N x D uint8 device
    tensor."""
    keep: list = []
    d = _desc(run, keep)
    st = lib().de_masks_noalloc(C.byref(d), int(run_index), int(gen),
                                C.c_void_p(out.data_ptr()), _stream())
    if st != OK:
        raise DEError(st, lib().de_last_error(None).decode())
    return out


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class DE:
    """One handle over one or more runs (all runs step together).

    Each run is a dict with keys N, D, F, CR, xo, fn, dtype, mm, exp_impl,
    tpr, base, shuffle, wb, lo, hi, olo, ohi, seed and optional device tensors
    shift (D values of the run's dtype) and rot (D x D float64, rotated
    function only)."""

    def __init__(self, runs: list[dict], device: str = "cuda:0", tune: bool = False):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.runs = [dict(r) for r in runs]
        if tune and not any(r.get("tpr") for r in self.runs):
            from .tune import tune_batched, tune_tpr
            if len(self.runs) == 1 and self.runs[0].get("fn") == "ellipsoid_rot" and \
                    self.runs[0].get("mm") in ("bf16x3", "bf16x6"):
                from .tune import tune_rot_tile
                self.runs[0]["tile"], self.tuning = tune_rot_tile(self.runs[0])
            elif len(self.runs) == 1:
                self.runs[0]["tpr"], self.tuning = tune_tpr(self.runs[0])
            else:
                t, self.tuning = tune_batched(self.runs)
                self.runs = [dict(r, tpr=t) for r in self.runs]
        self._keep: list = []
        descs = [_desc(r, self._keep) for r in self.runs]
        self._arr = (RunDesc * len(descs))(*descs)
        n = C.c_size_t(0)
        self._check(lib().de_workspace_size(self._arr, len(descs), C.byref(n)), None)
        self.ws_bytes = n.value
        self.workspace = torch.empty(max(n.value, 256), dtype=torch.uint8, device=self.device)
        h = C.c_void_p(0)
        self._check(lib().de_init(C.byref(h), self._arr, len(descs),
                                  C.c_void_p(self.workspace.data_ptr()), n.value, _stream()), None)
        self._h = h
        self._trace_bufs: dict = {}

    # ---- helpers ----
    def _check(self, st, h):
        if st != OK:
            msg = lib().de_last_error(h).decode()
            raise DEError(st, msg)

    def _np_dtype(self, run):
        return np.float64 if self.runs[run].get("dtype", "fp64") == "fp64" else np.float32

    def _t_dtype(self, run):
        t = self.torch
        return t.float64 if self.runs[run].get("dtype", "fp64") == "fp64" else t.float32

    # ---- ABI ----
    def generation(self, n: int = 1):
        self._check(lib().de_generation(self._h, int(n), _stream()), self._h)

    def evaluate(self, run: int, X):
        """f of each row of device tensor X (rows x D, run dtype)."""
        t = self.torch
        X = X.contiguous()
        out = t.empty(X.shape[0], dtype=self._t_dtype(run), device=self.device)
        self._check(lib().de_evaluate(self._h, run, C.c_void_p(X.data_ptr()), X.shape[0],
                                      C.c_void_p(out.data_ptr()), _stream()), self._h)
        return out

    def best(self, run: int = 0):
        f = C.c_double(0)
        idx = C.c_int64(0)
        g = C.c_int64(0)
        x = np.zeros(int(self.runs[run]["D"]), self._np_dtype(run))
        self._check(lib().de_best(self._h, run, C.byref(f), C.byref(idx), C.byref(g),
                                  x.ctypes.data_as(C.c_void_p), _stream()), self._h)
        return f.value, idx.value, g.value, x

    def fitness(self, run: int = 0):
        """Current fitness of every individual of a run (host array)."""
        N = int(self.runs[run]["N"])
        fit = np.zeros(N, self._np_dtype(run))
        g = C.c_int64(0)
        self._check(lib().de_get_state(self._h, run, None, fit.ctypes.data_as(C.c_void_p),
                                       C.byref(g), _stream()), self._h)
        return fit

    def state(self, run: int = 0):
        N, D = int(self.runs[run]["N"]), int(self.runs[run]["D"])
        pop = np.zeros((N, D), self._np_dtype(run))
        fit = np.zeros(N, self._np_dtype(run))
        g = C.c_int64(0)
        self._check(lib().de_get_state(self._h, run, pop.ctypes.data_as(C.c_void_p),
                                       fit.ctypes.data_as(C.c_void_p), C.byref(g), _stream()),
                    self._h)
        return pop, fit, g.value

    def set_state(self, run, pop, fit, gen, best_f=0.0, best_idx=-1, best_gen=0):
        dt = self._np_dtype(run)
        pop = np.ascontiguousarray(pop, dt)
        fit = np.ascontiguousarray(fit, dt)
        self._check(lib().de_set_state(self._h, run, pop.ctypes.data_as(C.c_void_p),
                                       fit.ctypes.data_as(C.c_void_p), int(gen), float(best_f),
                                       int(best_idx), int(best_gen), _stream()), self._h)

    def trace(self, run: int = 0, enable: bool = True):
        """Allocate trace buffers and switch tracing on (or off)."""
        t = self.torch
        if not enable:
            self._check(lib().de_trace(self._h, run, None, None, None, None), self._h)
            self._trace_bufs.pop(run, None)
            return None
        N, D = int(self.runs[run]["N"]), int(self.runs[run]["D"])
        bufs = {"idx": t.zeros((N, 6), dtype=t.int64, device=self.device),
                "mask": t.zeros((N, D), dtype=t.uint8, device=self.device),
                "trial": t.zeros((N, D), dtype=self._t_dtype(run), device=self.device),
                "ftrial": t.zeros(N, dtype=self._t_dtype(run), device=self.device)}
        self._trace_bufs[run] = bufs
        self._check(lib().de_trace(self._h, run, C.c_void_p(bufs["idx"].data_ptr()),
                                   C.c_void_p(bufs["mask"].data_ptr()),
                                   C.c_void_p(bufs["trial"].data_ptr()),
                                   C.c_void_p(bufs["ftrial"].data_ptr())), self._h)
        return bufs

    def profile(self, enable: bool = True):
        self._check(lib().de_profile(self._h, 1 if enable else 0), self._h)

    def profile_read(self):
        ms = C.c_double(0)
        n = C.c_int64(0)
        self._check(lib().de_profile_read(self._h, C.byref(ms), C.byref(n)), self._h)
        return ms.value, n.value

    def masks(self, run: int, gen: int, out=None):
        """Crossover masks of generation `gen` of a run (N x D uint8 device tensor)."""
        t = self.torch
        N, D = int(self.runs[run]["N"]), int(self.runs[run]["D"])
        if out is None:
            out = t.empty((N, D), dtype=t.uint8, device=self.device)
        self._check(lib().de_masks(self._h, run, int(gen), C.c_void_p(out.data_ptr()), _stream()),
                    self._h)
        return out

    def graph(self, enable=True):
        """Replay captured graphs in generation() (same results): True for
        blocks of 64 generations, an int n > 1 for blocks of n, False off."""
        n = (1 if enable else 0) if isinstance(enable, bool) else int(enable)
        self._check(lib().de_graph(self._h, n), self._h)

    def close(self):
        if getattr(self, "_h", None):
            lib().de_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
