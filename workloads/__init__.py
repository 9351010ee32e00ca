"""Seeded synthetic workloads: sorted docID lists and query streams.

Holds none of the method's arithmetic; shared by the oracle side and the GPU
side.  The native generator (``gen.cpp``) is built with g++ by ``build()``.

Workload recipes (seed base 14016399; workload k uses seed base + 1000 k):
  plain      A: 2^20, B: 2^14 distinct values uniform without replacement
             from [0, 2^25) (streams 0 and 1).
  bulk       256 lists, length floor(2^u) with u ~ U[12, 24]; even index
             uniform, odd index clustered; universe [0, 2^26).
  pairwise   index of 2^16 clustered lists over [0, 2^26), length of term t
             max(128, floor(2^23 / (t + 1))); 2^18 queries of 2 distinct
             terms, P(term) proportional to sqrt(length).
  multiterm  same index; 2^18 queries of 3..6 terms (uniform count).
  serving    index of 2^20 clustered lists over [0, 2^31), length
             max(128, floor(2^28 / (t + 1))); queries of 2..8 terms; Poisson
             arrivals.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.cpp")
_LIB_PATH = os.path.join(_HERE, "libworkloads.so")

SEED_BASE = 14016399
UNIFORM, CLUSTERED = 0, 1


def config_seed(k: int, stream: int = 0) -> int:
    return SEED_BASE + 1000 * k + stream


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-pthread",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        lib.wl_list.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, u32p]
        lib.wl_lists.argtypes = [ctypes.POINTER(ctypes.c_int32), ctypes.c_uint64, ctypes.c_uint64,
                                 ctypes.c_uint64, u64p, u64p, ctypes.c_uint64, u32p, ctypes.c_int]
        lib.wl_stream_seed.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        lib.wl_stream_seed.restype = ctypes.c_uint64
        lib.wl_queries.argtypes = [ctypes.c_uint64, u64p, ctypes.c_uint64, ctypes.c_uint64,
                                   ctypes.c_uint32, ctypes.c_uint32, u32p, u64p]
        lib.wl_arrivals.argtypes = [ctypes.c_uint64, ctypes.c_double, ctypes.c_uint64,
                                    ctypes.POINTER(ctypes.c_double)]
        lib.wl_queries_alias.argtypes = [ctypes.c_uint64, u64p, ctypes.c_uint64, ctypes.c_uint64,
                                         ctypes.c_uint32, ctypes.c_uint32, u32p, u64p, ctypes.c_int]
        for f in (lib.wl_list, lib.wl_lists, lib.wl_queries, lib.wl_arrivals, lib.wl_queries_alias):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _threads():
    return max(1, min(16, os.cpu_count() or 1))


def sorted_list(kind: int, seed: int, universe: int, n: int) -> np.ndarray:
    """One sorted list of n distinct values in [0, universe)."""
    lib = _load()
    out = np.zeros(max(1, n), dtype=np.uint32)
    rc = lib.wl_list(kind, seed, universe, n, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))
    if rc:
        raise ValueError("list longer than its universe")
    return out[:n]


def lists(kinds, lens, seed: int, universe: int, first_id: int = 0):
    """Many lists at once (multi-threaded).  Returns (flat values, offsets)."""
    lib = _load()
    kinds = np.ascontiguousarray(kinds, dtype=np.int32)
    lens = np.ascontiguousarray(lens, dtype=np.uint64)
    offs = np.zeros(lens.size + 1, dtype=np.uint64)
    np.cumsum(lens, out=offs[1:])
    flat = np.zeros(max(1, int(offs[-1])), dtype=np.uint32)
    rc = lib.wl_lists(kinds.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), seed, first_id, universe,
                      lens.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                      offs.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), lens.size,
                      flat.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), _threads())
    if rc:
        raise ValueError("list longer than its universe")
    return flat[: int(offs[-1])], offs


def list_by_id(kind: int, seed: int, universe: int, n: int, list_id: int) -> np.ndarray:
    """The same list that ``lists(..., first_id=0)`` writes at position list_id."""
    return sorted_list(kind, int(_load().wl_stream_seed(seed, list_id)), universe, n)


def queries(seed: int, lens, nq: int, kmin: int, kmax: int):
    """CSR query stream: (terms uint32[], offsets uint64[nq + 1])."""
    lib = _load()
    lens = np.ascontiguousarray(lens, dtype=np.uint64)
    terms = np.zeros(nq * kmax, dtype=np.uint32)
    offs = np.zeros(nq + 1, dtype=np.uint64)
    rc = lib.wl_queries(seed, lens.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), lens.size, nq,
                        kmin, kmax, terms.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                        offs.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    if rc:
        raise ValueError("bad query parameters")
    return terms[: int(offs[-1])], offs


def queries_fast(seed: int, lens, nq: int, kmin: int, kmax: int):
    """Long CSR query streams of the same law as queries(), drawn in
    parallel with an alias table (a different stream for the same seed)."""
    lib = _load()
    lens = np.ascontiguousarray(lens, dtype=np.uint64)
    terms = np.empty(nq * kmax, dtype=np.uint32)
    offs = np.empty(nq + 1, dtype=np.uint64)
    rc = lib.wl_queries_alias(seed, lens.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), lens.size, nq,
                              kmin, kmax, terms.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                              offs.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), _threads())
    if rc:
        raise ValueError("bad query parameters")
    return terms[: int(offs[-1])], offs


def arrivals(seed: int, rate: float, count: int) -> np.ndarray:
    lib = _load()
    t = np.zeros(count, dtype=np.float64)
    rc = lib.wl_arrivals(seed, rate, count, t.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if rc:
        raise ValueError("bad rate")
    return t


# ---------------------------------------------------------------- recipes

def plain_pair():
    """A (2^20) and B (2^14), uniform without replacement from [0, 2^25)."""
    a = sorted_list(UNIFORM, config_seed(0, 0), 1 << 25, 1 << 20)
    b = sorted_list(UNIFORM, config_seed(0, 1), 1 << 25, 1 << 14)
    return a, b


def bulk_lengths(count: int = 256):
    rng = np.random.Generator(np.random.PCG64(config_seed(1, 999)))
    u = rng.uniform(12.0, 24.0, size=count)
    lens = np.floor(np.exp2(u)).astype(np.uint64)
    kinds = np.array([UNIFORM if i % 2 == 0 else CLUSTERED for i in range(count)], dtype=np.int32)
    return kinds, lens


def bulk_lists(count: int = 256, universe: int = 1 << 26):
    kinds, lens = bulk_lengths(count)
    flat, offs = lists(kinds, lens, config_seed(1, 0), universe)
    return flat, offs, kinds


def index_lengths(nlists: int, total_log2: int) -> np.ndarray:
    t = np.arange(nlists, dtype=np.uint64)
    return np.maximum(np.uint64(128), (np.uint64(1) << np.uint64(total_log2)) // (t + np.uint64(1)))


def pairwise_index(nlists: int = 1 << 16, universe: int = 1 << 26, total_log2: int = 23):
    lens = index_lengths(nlists, total_log2)
    kinds = np.full(nlists, CLUSTERED, dtype=np.int32)
    flat, offs = lists(kinds, lens, config_seed(2, 0), universe)
    return flat, offs


def pairwise_queries(lens, nq: int = 1 << 18):
    return queries(config_seed(2, 1), lens, nq, 2, 2)


def multiterm_queries(lens, nq: int = 1 << 18):
    return queries(config_seed(3, 1), lens, nq, 3, 6)


def length_weighted_queries(seed: int, lens, nq: int, kmin: int, kmax: int):
    """CSR query stream like queries(), with P(t) proportional to lens[t]
    instead of its square root: a term drawn as the term of a random
    posting, so the long (dense) lists that dominate real query logs come
    up often.  queries() weighs by the square root of what it is given, so
    it is given the squared lengths."""
    lv = np.ascontiguousarray(lens, dtype=np.uint64)
    if lv.size and int(lv.max()) >= 1 << 32:
        raise ValueError("lengths must be below 2^32")
    return queries(seed, lv * lv, nq, kmin, kmax)


def serving_queries(lens, nq: int, level: int = 0):
    return queries(config_seed(4, 10 + level), lens, nq, 2, 8)


def serving_trace(lens, nq: int, level: int):
    """The serving workload's query stream for arrival level `level`, long
    traces drawn by queries_fast (2..8 terms, sqrt(length) sampling)."""
    return queries_fast(config_seed(4, 30 + level), lens, nq, 2, 8)


def planted_pair(seed: int, n: int, m: int, frac: float, universe: int = 1 << 26, kind: int = CLUSTERED):
    """A long list f (n values) and a short list r (m values) sharing
    round(frac * m) values: the shared values are drawn from f uniformly,
    the rest of r from outside f, then r is sorted."""
    f = sorted_list(kind, seed, universe, n)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    k = min(int(round(frac * m)), n, m)
    shared = rng.choice(f, size=k, replace=False) if k else np.zeros(0, np.uint32)
    need = m - k
    others = np.zeros(0, np.uint32)
    while others.size < need:
        cand = rng.integers(0, universe, size=2 * (need - others.size) + 16, dtype=np.uint64).astype(np.uint32)
        cand = cand[~np.isin(cand, f)]
        others = np.unique(np.concatenate([others, cand]))
    if others.size > need:
        others = rng.choice(others, size=need, replace=False)
    r = np.sort(np.concatenate([shared.astype(np.uint32), others.astype(np.uint32)]))
    return r, f
