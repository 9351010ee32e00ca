"""The long-trace query generator: same law as the plain one (k uniform in
[kmin, kmax], distinct terms, P(term) proportional to sqrt(length)), and
output independent of the thread count."""
import ctypes

import numpy as np
import pytest

import workloads


def _fast(seed, lens, nq, kmin, kmax, threads):
    lib = workloads._load()
    lens = np.ascontiguousarray(lens, dtype=np.uint64)
    terms = np.empty(nq * kmax, np.uint32)
    offs = np.empty(nq + 1, np.uint64)
    rc = lib.wl_queries_alias(seed, lens.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), lens.size, nq, kmin, kmax,
                              terms.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                              offs.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), threads)
    assert rc == 0
    return terms[: int(offs[-1])], offs


def test_thread_count_does_not_matter():
    lens = workloads.index_lengths(1 << 12, 20)
    a = _fast(7, lens, 200000, 2, 8, 1)
    b = _fast(7, lens, 200000, 2, 8, 8)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_law():
    lens = workloads.index_lengths(1 << 10, 20)
    terms, offs = workloads.queries_fast(11, lens, 400000, 2, 8)
    k = np.diff(offs)
    assert k.min() == 2 and k.max() == 8
    assert abs(k.mean() - 5.0) < 0.02
    counts_k = np.bincount(k.astype(np.int64), minlength=9)[2:]
    assert (np.abs(counts_k / k.size - 1 / 7) < 0.005).all()
    for q in range(0, 400000, 997):
        ts = terms[int(offs[q]): int(offs[q + 1])]
        assert np.unique(ts).size == ts.size
    # one-term draws: the frequency of each term follows sqrt(length)
    t1, o1 = workloads.queries_fast(12, lens, 1 << 21, 1, 1)
    w = np.sqrt(lens.astype(np.float64))
    p = w / w.sum()
    got = np.bincount(t1, minlength=lens.size) / t1.size
    # chi-square over the terms against the law (1023 degrees of freedom)
    e = p * t1.size
    chi2 = float((((got * t1.size) - e) ** 2 / e).sum())
    assert chi2 < 1023 + 6 * np.sqrt(2 * 1023)
    # and the plain generator draws the same law
    t2, _ = workloads.queries(12, lens, 1 << 19, 1, 1)
    got2 = np.bincount(t2, minlength=lens.size) / t2.size
    assert np.abs(got2 - got).max() < 0.002


def test_length_weighted_law():
    """length_weighted_queries: one-term draws follow P(t) = len / sum(len)
    (chi-square over the terms), and lengths of 2^32 or more are refused."""
    lens = workloads.index_lengths(1 << 8, 16)
    t1, o1 = workloads.length_weighted_queries(13, lens, 1 << 19, 1, 1)
    assert np.array_equal(o1, np.arange(o1.size, dtype=np.uint64))
    p = lens.astype(np.float64) / float(lens.sum())
    e = p * t1.size
    got = np.bincount(t1, minlength=lens.size).astype(np.float64)
    chi2 = float(((got - e) ** 2 / e).sum())
    assert chi2 < 255 + 6 * np.sqrt(2 * 255)
    with pytest.raises(ValueError):
        workloads.length_weighted_queries(13, np.array([1 << 32, 5], dtype=np.uint64), 4, 1, 1)
