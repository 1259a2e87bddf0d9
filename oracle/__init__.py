"""Colour-coding oracle: TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import
this package. The product path (``paper_1804_09764_amd``) never imports, links or calls it, and
the two share no code.

The oracle is a plain CPU implementation of the colour-coding dynamic program of the paper
(Section 2.1, Eq. 1 and Algorithm 1) in C (``oracle.c``), a brute-force embedding enumerator
(``brute.c``) that pins it, and thin ctypes wrappers. See the header of ``oracle.c`` for what is
computed and the readings taken where the paper is silent.

Parity status of every function here: pinned (see tests/test_oracle_pins.py) — by brute force,
by the all-colourings identity, by closed forms on cycles, stars and cliques, and by the Cayley
identity for |Aut|.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from functools import lru_cache

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "liboracle.so")
_SRCS = [os.path.join(_HERE, "oracle.c"), os.path.join(_HERE, "brute.c")]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP). Building the checker is not using it."""
    newest = max(os.path.getmtime(s) for s in _SRCS)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < newest:
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp] + _SRCS)
        os.replace(tmp, _LIB)
    return _LIB


@lru_cache(maxsize=1)
def _lib():
    if not os.path.exists(_LIB):
        build(force=False)
    L = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    L.orc_colour.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int, P]
    L.orc_step.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int64, P, P, P, P, P,
                           ctypes.c_int]
    L.orc_count.argtypes = [ctypes.c_int64, P, P, P, ctypes.c_int, P, ctypes.c_int, ctypes.c_int, P,
                            ctypes.POINTER(ctypes.c_longdouble), ctypes.c_int]
    L.orc_aut.argtypes = [ctypes.c_int, P, ctypes.POINTER(ctypes.c_longdouble)]
    L.orc_estimate.argtypes = [ctypes.c_int, ctypes.c_longdouble, P, ctypes.c_int64,
                               ctypes.POINTER(ctypes.c_longdouble)]
    L.orc_brute_count.argtypes = [ctypes.c_int64, P, P, P, ctypes.c_int, P, ctypes.c_int, P,
                                  ctypes.POINTER(ctypes.c_uint64), ctypes.c_int]
    L.orc_brute_aut.argtypes = [ctypes.c_int, P, ctypes.POINTER(ctypes.c_uint64)]
    L.orc_threads.restype = ctypes.c_int
    return L


def _ptr(a):
    return a.ctypes.data if a is not None and a.size else None


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def threads() -> int:
    return _lib().orc_threads()


def colour(seed: int, it: int, n: int, k: int) -> np.ndarray:
    """The counter-based random colouring (SplitMix64 finaliser + Lemire range reduction)."""
    out = np.empty(n, dtype=np.uint8)
    rc = _lib().orc_colour(seed, it, n, k, out.ctypes.data if n else None)
    if rc:
        raise ValueError(f"orc_colour rc={rc}")
    return out


def count(row_ptr, col, colours, tree_edges, root: int = -1, rule: int = 0, per_vertex: bool = False,
          threads: int = 0, longdouble: bool = False):
    """Colourful labelled embeddings X for one colouring (exact below 2^53).

    Returns X as a Python float (long double rounded; the numpy longdouble if `longdouble`) and,
    if asked, the per-vertex counts C(v, T rooted at `root`, all colours) as float64.
    """
    rp = _c(row_ptr, np.int64)
    cl = _c(col, np.int32)
    co = _c(colours, np.uint8)
    te = _c(tree_edges, np.int32).reshape(-1)
    k = len(te) // 2 + 1
    n = len(rp) - 1
    pv = np.empty(n, dtype=np.float64) if per_vertex else None
    X = ctypes.c_longdouble()
    rc = _lib().orc_count(n, rp.ctypes.data, _ptr(cl), _ptr(co), k, _ptr(te), root, rule, _ptr(pv),
                          ctypes.byref(X), threads)
    if rc:
        raise ValueError(f"orc_count rc={rc}")
    Xv = np.longdouble(X.value) if longdouble else X.value
    return (Xv, pv) if per_vertex else Xv


def count_ld(row_ptr, col, colours, tree_edges, root: int = -1, rule: int = 0, threads: int = 0):
    """As count(), but returns the ctypes long double (64-bit mantissa) unrounded."""
    rp = _c(row_ptr, np.int64)
    cl = _c(col, np.int32)
    co = _c(colours, np.uint8)
    te = _c(tree_edges, np.int32).reshape(-1)
    k = len(te) // 2 + 1
    X = ctypes.c_longdouble()
    rc = _lib().orc_count(len(rp) - 1, rp.ctypes.data, _ptr(cl), _ptr(co), k, _ptr(te), root, rule,
                          None, ctypes.byref(X), threads)
    if rc:
        raise ValueError(f"orc_count rc={rc}")
    return X


def step(k: int, s: int, a: int, nbr_ptr, nbr, act, pas, threads: int = 0) -> np.ndarray:
    """One application of Eq. 1 for a set of centre vertices (see oracle.c: orc_step)."""
    from math import comb
    nptr = _c(nbr_ptr, np.int64)
    nb = _c(nbr, np.int32)
    A = _c(act, np.float64)
    P = _c(pas, np.float64)
    nv = len(nptr) - 1
    out = np.empty((nv, comb(k, s)), dtype=np.float64)
    rc = _lib().orc_step(k, s, a, nv, nptr.ctypes.data, _ptr(nb), _ptr(A), _ptr(P), _ptr(out), threads)
    if rc:
        raise ValueError(f"orc_step rc={rc}")
    return out


def aut(tree_edges) -> int:
    te = _c(tree_edges, np.int32).reshape(-1)
    k = len(te) // 2 + 1
    r = ctypes.c_longdouble()
    rc = _lib().orc_aut(k, _ptr(te), ctypes.byref(r))
    if rc:
        raise ValueError(f"orc_aut rc={rc}")
    return int(r.value)


def brute_aut(tree_edges) -> int:
    te = _c(tree_edges, np.int32).reshape(-1)
    k = len(te) // 2 + 1
    r = ctypes.c_uint64()
    rc = _lib().orc_brute_aut(k, _ptr(te), ctypes.byref(r))
    if rc:
        raise ValueError(f"orc_brute_aut rc={rc}")
    return r.value


def brute_count(row_ptr, col, colours, tree_edges, root: int = 0, per_vertex: bool = False,
                threads: int = 0):
    """Enumerate injective homomorphisms one by one (colourful only unless colours is None)."""
    rp = _c(row_ptr, np.int64)
    cl = _c(col, np.int32)
    co = None if colours is None else _c(colours, np.uint8)
    te = _c(tree_edges, np.int32).reshape(-1)
    k = len(te) // 2 + 1
    n = len(rp) - 1
    pv = np.empty(n, dtype=np.uint64) if per_vertex else None
    tot = ctypes.c_uint64()
    rc = _lib().orc_brute_count(n, rp.ctypes.data, _ptr(cl), _ptr(co), k, _ptr(te), root, _ptr(pv),
                                ctypes.byref(tot), threads)
    if rc:
        raise ValueError(f"orc_brute_count rc={rc}")
    return (tot.value, pv) if per_vertex else tot.value


def estimate(k: int, aut_T: int, X) -> float:
    """mean(X) * k^k / k! / |Aut(T)| (Algorithm 1's scaling of the colourful count)."""
    arr = (ctypes.c_longdouble * len(X))(*[float(x) for x in X])
    r = ctypes.c_longdouble()
    rc = _lib().orc_estimate(k, ctypes.c_longdouble(aut_T), ctypes.addressof(arr), len(X), ctypes.byref(r))
    if rc:
        raise ValueError(f"orc_estimate rc={rc}")
    return r.value
