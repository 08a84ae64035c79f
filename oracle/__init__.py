"""CPU oracle for parallel differential evolution -- TEST INFRASTRUCTURE ONLY.

A ctypes front end to ``oracle.c``: a plain, sequential FP64 reference of one
DE/rand/1 generation (mutation, bin / classic exp / NEC crossover, fitness,
greedy selection) written from Pan, arXiv:2101.06599 (Alg 1, Alg 2, Alg 7-10,
Eq 1, 2, 9).  Only tests, the smoke check and the benchmark's CPU-baseline leg
may import this package; the GPU library never uses it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

XO = {"bin": 0, "exp": 1, "nec": 2}
FN = {"sphere": 0, "rastrigin": 1, "rosenbrock": 2, "ellipsoid_rot": 3, "ackley": 4,
      "griewank": 5}
DTYPE = {"fp64": 0, "fp32": 1}
TAG = {"init": 1, "shift": 2, "idx": 3, "xo": 4, "bin": 5, "exp": 6, "offset": 7, "perm": 8,
       "shuffle": 9}
BASE = {"classic": 0, "random": 1, "offset": 2, "perm": 3}


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, no fast-math, no contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
             "-fopenmp", "-Wall", "-o", tmp, os.path.join(_HERE, "oracle.c"), "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Desc(C.Structure):
    _fields_ = [("N", C.c_int64), ("D", C.c_int64), ("F", C.c_double), ("CR", C.c_double),
                ("xo", C.c_int32), ("fn", C.c_int32), ("dtype", C.c_int32), ("run", C.c_int32),
                ("lo", C.c_double), ("hi", C.c_double), ("olo", C.c_double), ("ohi", C.c_double),
                ("seed", C.c_uint64), ("shift", C.c_void_p), ("rot", C.c_void_p),
                ("lazy", C.c_int32), ("base", C.c_int32), ("shuffle", C.c_int32),
                ("pad", C.c_int32)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        L = C.CDLL(_LIB_PATH)
        u32p = np.ctypeslib.ndpointer(np.uint32, flags="C")
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C")
        u8p = np.ctypeslib.ndpointer(np.uint8, flags="C")
        L.oracle_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.oracle_word.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32,
                                  C.c_uint32, C.c_int]
        L.oracle_word.restype = C.c_uint32
        L.oracle_uniform.argtypes = [C.c_uint32]
        L.oracle_uniform.restype = C.c_double
        L.oracle_randint.argtypes = [C.c_uint32, C.c_int64]
        L.oracle_randint.restype = C.c_int64
        L.oracle_skip.argtypes = [C.c_int64, i64p, C.c_int]
        L.oracle_skip.restype = C.c_int64
        L.oracle_indices.argtypes = [C.c_uint64, C.c_uint32, C.c_int64, C.c_uint32, C.c_int64, i64p]
        L.oracle_indices_scheme.argtypes = [C.c_uint64, C.c_uint32, C.c_int, C.c_int64, C.c_uint32,
                                            C.c_int64, i64p]
        L.oracle_permute.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_int64,
                                     C.c_int64]
        L.oracle_permute.restype = C.c_int64
        L.oracle_mask_bin.argtypes = [C.c_uint64, C.c_uint32, C.c_int64, C.c_double, C.c_uint32,
                                      C.c_int64, C.c_int64, u8p]
        L.oracle_exp_length.argtypes = [C.c_uint64, C.c_uint32, C.c_int64, C.c_double, C.c_uint32,
                                        C.c_int64]
        L.oracle_exp_length.restype = C.c_int64
        L.oracle_nec_length.argtypes = [C.c_double, C.c_double, C.c_int64]
        L.oracle_nec_length.restype = C.c_int64
        L.oracle_nec_length_log.argtypes = [C.c_double, C.c_double, C.c_int64]
        L.oracle_nec_length_log.restype = C.c_int64
        L.oracle_alg9_mask.argtypes = [C.c_int64, C.c_int64, C.c_int64, u8p]
        L.oracle_alg10_mask.argtypes = [C.c_int64, C.c_int64, C.c_int64, u8p]
        L.oracle_lengths.argtypes = [C.c_int, C.c_uint64, C.c_uint32, C.c_int64, C.c_double,
                                     C.c_int64, i64p]
        L.oracle_ackley_printed.argtypes = [C.c_int64, f64p]
        L.oracle_ackley_printed.restype = C.c_double
        fitargs = [C.c_int, C.c_int64, f64p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.oracle_fitness.argtypes = fitargs
        L.oracle_fitness.restype = C.c_double
        L.oracle_fitness_phi.argtypes = fitargs
        L.oracle_fitness_phi.restype = C.c_double
        L.oracle_ellipsoid_weights.argtypes = [C.c_int64, f64p]
        L.oracle_create.argtypes = [C.POINTER(_Desc)]
        L.oracle_create.restype = C.c_void_p
        L.oracle_destroy.argtypes = [C.c_void_p]
        L.oracle_generation.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.c_void_p]
        L.oracle_generation.restype = C.c_int
        L.oracle_get_state.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.oracle_set_state.argtypes = [C.c_void_p, f64p, f64p, C.c_int64, C.c_double, C.c_int64,
                                       C.c_int64]
        L.oracle_get_best.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.oracle_get_shift.argtypes = [C.c_void_p, f64p]
        L.oracle_set_threads.argtypes = [C.c_int]
        L.oracle_set_threads.restype = C.c_int
        L.oracle_individual.argtypes = [C.c_void_p, f64p, C.c_int64, C.c_int64, i64p, u8p, f64p,
                                        C.POINTER(C.c_double)]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


# ---- element-level functions ------------------------------------------------

def philox(ctr, key) -> np.ndarray:
    out = np.zeros(4, np.uint32)
    lib().oracle_philox4x32_10(np.asarray(ctr, np.uint32), np.asarray(key, np.uint32), out)
    return out


def word(seed, run, tag, g, i, block, k) -> int:
    return int(lib().oracle_word(seed, run, TAG[tag] if isinstance(tag, str) else tag, g, i,
                                 block, k))


def uniform(w: int) -> float:
    return lib().oracle_uniform(w)


def randint(w: int, n: int) -> int:
    return lib().oracle_randint(w, n)


def skip(r: int, excl) -> int:
    e = np.asarray(list(excl), np.int64)
    return lib().oracle_skip(r, e, len(e))


def indices(seed, run, N, g, i):
    r = np.zeros(3, np.int64)
    lib().oracle_indices(seed, run, N, g, i, r)
    return r


def indices_scheme(seed, run, base, N, g, i):
    """r0, r1, r2 of position i under base scheme `base` (BASE name)."""
    r = np.zeros(3, np.int64)
    lib().oracle_indices_scheme(seed, run, BASE[base], N, g, i, r)
    return r


def set_threads(n: int = 0) -> int:
    """Threads for a generation's per-individual loops (0: unchanged); returns
    the count in effect.  Results do not depend on it."""
    return int(lib().oracle_set_threads(int(n)))


def permute(seed, run, tag, g, N, k) -> int:
    """Image of k under the keyed permutation of [0, N) (tag name or number)."""
    t = TAG[tag] if isinstance(tag, str) else int(tag)
    return int(lib().oracle_permute(seed, run, t, g, N, k))


def mask_bin(seed, run, D, CR, g, i, jrand):
    m = np.zeros(D, np.uint8)
    lib().oracle_mask_bin(seed, run, D, CR, g, i, jrand, m)
    return m


def exp_length(seed, run, D, CR, g, i) -> int:
    return lib().oracle_exp_length(seed, run, D, CR, g, i)


def nec_length(U, CR, D) -> int:
    return lib().oracle_nec_length(U, CR, D)


def nec_length_log(U, CR, D) -> int:
    return lib().oracle_nec_length_log(U, CR, D)


def lengths(kind, D, CR, n, seed=11, run=0):
    """Run lengths of n individuals (generation 1 + k // 4096, position
    k % 4096): kind "exp" (Alg 8) or "nec" (Eq 9)."""
    out = np.zeros(int(n), np.int64)
    lib().oracle_lengths(0 if kind == "exp" else 1, seed, run, D, CR, int(n), out)
    return out


def ackley_printed(x) -> float:
    """Ackley in the printed order of Sec. 4 (cross-check of fitness())."""
    x = np.ascontiguousarray(x, np.float64)
    return lib().oracle_ackley_printed(x.shape[-1], x)


def alg9_mask(D, j, L):
    m = np.zeros(D, np.uint8)
    lib().oracle_alg9_mask(D, j, L, m)
    return m


def alg10_mask(D, j, L):
    m = np.zeros(D, np.uint8)
    lib().oracle_alg10_mask(D, j, L, m)
    return m


def ellipsoid_weights(D):
    w = np.zeros(D, np.float64)
    lib().oracle_ellipsoid_weights(D, w)
    return w


def _fit_call(f, fn, x, o, rot, w):
    x = np.ascontiguousarray(x, np.float64)
    D = x.shape[-1]
    o = None if o is None else np.ascontiguousarray(o, np.float64)
    rot = None if rot is None else np.ascontiguousarray(rot, np.float64)
    if FN_NAME(fn) == "ellipsoid_rot" and w is None:
        w = ellipsoid_weights(D)
    w = None if w is None else np.ascontiguousarray(w, np.float64)
    code = FN[fn] if isinstance(fn, str) else fn
    if x.ndim == 1:
        return f(code, D, x, _ptr(o), _ptr(rot), _ptr(w))
    return np.array([f(code, D, np.ascontiguousarray(r), _ptr(o), _ptr(rot), _ptr(w))
                     for r in x])


def FN_NAME(fn):
    if isinstance(fn, str):
        return fn
    return {v: k for k, v in FN.items()}[fn]


def fitness(fn, x, o=None, rot=None, w=None):
    """f(x) for one row (returns float) or for each row of a 2-D array."""
    return _fit_call(lib().oracle_fitness, fn, x, o, rot, w)


def fitness_phi(fn, x, o=None, rot=None, w=None):
    """The tolerance scale: the absolute values of the terms whose rounding
    the evaluation carries (f itself for sums of non-negative terms)."""
    return _fit_call(lib().oracle_fitness_phi, fn, x, o, rot, w)


# ---- a whole run ---------------------------------------------------------

class Run:
    """One DE run in the oracle.  All arrays come back as float64 (FP32 runs
    hold float32 values exactly)."""

    def __init__(self, N, D, F=0.5, CR=0.9, xo="bin", fn="sphere", dtype="fp64", lo=-100.0,
                 hi=100.0, olo=0.0, ohi=0.0, seed=0, run=0, shift=None, rot=None, lazy=False,
                 base="classic", shuffle=False):
        self.N, self.D = int(N), int(D)
        self.dtype = dtype
        self.fn = fn
        self._keep = []
        sh = None if shift is None else np.ascontiguousarray(shift, np.float64)
        rt = None if rot is None else np.ascontiguousarray(rot, np.float64)
        self._keep += [sh, rt]
        d = _Desc(N=self.N, D=self.D, F=F, CR=CR, xo=XO[xo], fn=FN[fn], dtype=DTYPE[dtype], run=run,
                  lo=lo, hi=hi, olo=olo, ohi=ohi, seed=seed,
                  shift=None if sh is None else sh.ctypes.data,
                  rot=None if rt is None else rt.ctypes.data, lazy=1 if lazy else 0,
                  base=BASE[base], shuffle=1 if shuffle else 0)
        self._h = lib().oracle_create(C.byref(d))
        if not self._h:
            raise ValueError("oracle_create rejected the run description")
        self.rot = rt

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().oracle_destroy(h)
            self._h = None

    def generation(self, n=1, trace=False):
        N, D = self.N, self.D
        if not trace:
            lib().oracle_generation(self._h, n, None, None, None, None)
            return None
        ti = np.zeros((N, 6), np.int64)
        tm = np.zeros((N, D), np.uint8)
        tt = np.zeros((N, D), np.float64)
        tf = np.zeros(N, np.float64)
        lib().oracle_generation(self._h, n, _ptr(ti), _ptr(tm), _ptr(tt), _ptr(tf))
        return {"idx": ti, "mask": tm, "trial": tt, "ftrial": tf}

    def state(self):
        pop = np.zeros((self.N, self.D), np.float64)
        fit = np.zeros(self.N, np.float64)
        g = C.c_int64(0)
        lib().oracle_get_state(self._h, _ptr(pop), _ptr(fit), C.byref(g))
        return pop, fit, g.value

    def set_state(self, pop, fit, gen, best_f, best_idx, best_gen):
        lib().oracle_set_state(self._h, np.ascontiguousarray(pop, np.float64),
                               np.ascontiguousarray(fit, np.float64), gen, best_f, best_idx,
                               best_gen)

    def best(self):
        f = C.c_double(0)
        idx = C.c_int64(0)
        g = C.c_int64(0)
        x = np.zeros(self.D, np.float64)
        lib().oracle_get_best(self._h, C.byref(f), C.byref(idx), C.byref(g), _ptr(x))
        return f.value, idx.value, g.value, x

    def individual(self, pop, g, i):
        """Generation g's trial of individual i from population pop (N x D)."""
        idx = np.zeros(6, np.int64)
        m = np.zeros(self.D, np.uint8)
        u = np.zeros(self.D, np.float64)
        f = C.c_double(0)
        lib().oracle_individual(self._h, np.ascontiguousarray(pop, np.float64), int(g), int(i), idx,
                                m, u, C.byref(f))
        return {"idx": idx, "mask": m, "trial": u, "ftrial": f.value}

    def shift(self):
        o = np.zeros(self.D, np.float64)
        lib().oracle_get_shift(self._h, o)
        return o
