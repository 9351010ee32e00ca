"""hyb+m2 hybrid index (Sec. 7.7): dense lists held as bitmaps, the rest
compressed.  The representation of every list follows the oracle's rule,
and every query's result equals the oracle's hybrid procedure (and so the
set intersection), whatever mix of bitmap and compressed lists it has."""
import ctypes
import sys

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

UNIVERSE = 1 << 20


def log(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def data(gpu):
    # lengths 2^17 / (t + 1): list t has average gap 8 (t + 1) over 2^20
    lens = workloads.index_lengths(1 << 10, 17)
    kinds = np.full(lens.size, workloads.CLUSTERED, dtype=np.int32)
    kinds[1::2] = workloads.UNIFORM
    flat, offs = workloads.lists(kinds, lens, 9090, UNIVERSE)
    buf, soffs = gpu.encode_many(flat, offs)
    return lens, flat, offs, buf, soffs


def raw(flat, offs, t):
    return flat[int(offs[t]): int(offs[t + 1])]


def dense_queries(rng, nl, count):
    """Queries that lean on the densest lists: all-bitmap pairs and
    triples, dense + sparse, and single dense terms."""
    qs = []
    for _ in range(count):
        k = int(rng.integers(1, 5))
        dense = rng.choice(8, size=min(k, int(rng.integers(1, k + 1))), replace=False)
        rest = rng.choice(np.arange(8, nl), size=k - dense.size, replace=False)
        qs.append(np.concatenate([dense, rest]).astype(np.uint32))
    return qs


def run_and_check(gpu, ix, queries, flat, offs, universe, gap):
    import torch
    terms = np.concatenate(queries).astype(np.uint32)
    qoffs = np.zeros(len(queries) + 1, np.uint64)
    qoffs[1:] = np.cumsum([q.size for q in queries])
    b = gpu.Batch(ix, terms, qoffs)
    b.run()
    torch.cuda.synchronize()
    counts = b.counts.cpu().numpy()
    roffs = b.res_offsets.cpu().numpy()
    res = b.results.cpu().numpy().view(np.uint32)
    for q, ts in enumerate(queries):
        lists = [raw(flat, offs, t) for t in ts]
        want = oracle.hyb_intersect_k(lists, universe, gap)
        got = res[int(roffs[q]): int(roffs[q + 1])]
        assert int(counts[q]) == got.size
        assert np.array_equal(got, want), (q, ts.tolist())
    return b


@pytest.mark.parametrize("gap", [8, 32, 1024, 1 << 20])
def test_hybrid_index_matches_oracle(gpu, data, gap):
    """B = 8 and 32 make the few densest lists bitmaps (the paper's
    settings); B = 1024 most of them; B = 2^20 every list, so every query
    walks a bitmap as its shortest list."""
    lens, flat, offs, buf, soffs = data
    ix = gpu.Index(buf, soffs, universe=UNIVERSE, bitmap_gap=gap)
    kinds = ix.kinds()
    want = np.array([oracle.hyb_is_bitmap(int(n), UNIVERSE, gap) for n in lens], dtype=np.uint8)
    assert np.array_equal(kinds, want)
    nbm = int(want.sum())
    assert ix.bitmap_lists == nbm and ix.universe == UNIVERSE and ix.bitmap_gap == gap
    assert ix.bitmap_bytes == nbm * 4 * ((UNIVERSE + 31) // 32)
    assert ix.select_bytes == sum(4 * ((int(n) + 127) // 128) for n, k in zip(lens, want) if k)
    log(f"B={gap}: {nbm} bitmap lists")
    terms, qoffs = workloads.queries(600 + gap % 97, ix.lengths, 700, 1, 6)
    queries = [terms[int(qoffs[q]): int(qoffs[q + 1])] for q in range(700)]
    queries += dense_queries(np.random.default_rng(gap % 1000), lens.size, 300)
    run_and_check(gpu, ix, queries, flat, offs, UNIVERSE, gap)
    ix.free()


def test_hybrid_ragged_universe_and_edges(gpu):
    """Universe one past the largest value (not a multiple of 32, bit U - 1
    set); lists of 1, 127, 128, 129 and 4096 values; empty list; a
    compressed value above every bitmap's range."""
    rng = np.random.default_rng(77)
    universe = 100_003
    lists = [np.sort(rng.choice(universe - 1, size=n, replace=False)).astype(np.uint32)
             for n in (60000, 50002, 4096, 129, 128, 127, 1)]
    lists[0][-1] = universe - 1
    lists[0] = np.unique(lists[0])
    lists.append(np.zeros(0, np.uint32))
    flat = np.concatenate(lists).astype(np.uint32)
    offs = np.zeros(len(lists) + 1, np.uint64)
    offs[1:] = np.cumsum([l.size for l in lists])
    buf, soffs = gpu.encode_many(flat, offs)
    ix = gpu.Index(buf, soffs, universe=universe, bitmap_gap=2)
    assert ix.kinds().tolist() == [1, 1, 0, 0, 0, 0, 0, 0]
    queries = [np.array(q, np.uint32) for q in
               ([0], [1], [0, 1], [1, 0], [2, 0], [0, 2, 1], [3, 0], [4, 1], [5, 0, 1], [6, 0], [7, 0], [7, 1, 0],
                [6, 5, 4, 3, 2, 1, 0])]
    run_and_check(gpu, ix, queries, flat, offs, universe, 2)
    # a bitmap list has no compressed view
    with pytest.raises(gpu.S4Error) as e:
        ix.list(0)
    assert e.value.code == gpu.EINVAL
    assert ix.list(2).n == 4096
    ix.free()


def test_hybrid_build_errors(gpu):
    vals = np.arange(0, 1000, 2, dtype=np.uint32)
    offs = np.array([0, vals.size], np.uint64)
    buf, soffs = gpu.encode_many(vals, offs)
    with pytest.raises(gpu.S4Error) as e:  # 998 >= universe 900, and the list is a bitmap
        gpu.Index(buf, soffs, universe=900, bitmap_gap=4)
    assert e.value.code == gpu.EINVAL
    h = ctypes.c_void_p()
    rc = gpu.require_library().s4_index_build_hybrid(gpu._ptr(buf, ctypes.c_uint8), gpu._ptr(soffs, ctypes.c_uint64),
                                                     1, 1000, 0, None, ctypes.byref(h))
    assert rc == gpu.EINVAL  # B = 0
    # a list with repeats never becomes a bitmap (a bitmap cannot hold them)
    rep = np.array([1, 1, 2, 3, 5, 8], np.uint32)
    buf2, soffs2 = gpu.encode_many(rep, np.array([0, rep.size], np.uint64))
    ix = gpu.Index(buf2, soffs2, universe=16, bitmap_gap=8)
    assert ix.kinds().tolist() == [0]
    ix.free()


def test_hybrid_server_matches_oracle(gpu, data):
    """The serving loop over a hybrid index (B = 32)."""
    lens, flat, offs, buf, soffs = data
    ix = gpu.Index(buf, soffs, universe=UNIVERSE, bitmap_gap=32)
    terms, qoffs = workloads.queries(41, ix.lengths, 1500, 2, 8)
    srv = gpu.Server(ix, max_slots=1024, pool_bytes=512 << 20, result_bytes=64 << 20)
    try:
        r = srv.replay(terms, qoffs, np.zeros(1500, np.uint64), with_results=True, results_cap=1 << 24)
    finally:
        srv.close()
    for q in range(1500):
        ts = terms[int(qoffs[q]): int(qoffs[q + 1])]
        want = oracle.hyb_intersect_k([raw(flat, offs, t) for t in ts], UNIVERSE, 32)
        got = r["results"][int(r["res_offsets"][q]): int(r["res_offsets"][q + 1])]
        assert np.array_equal(got, want), q
    ix.free()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("kind", ["pairwise", "multiterm"])
def test_full_size_hybrid_batch_sampled(gpu, kind):
    """The batched workloads at full size (2^16 clustered lists over
    [0, 2^26), 2^18 queries) over a hybrid index with B = 32: every query
    run, 3000 sampled results checked with the oracle, every query that
    touches a bitmap list among them."""
    import torch
    flat, offs = workloads.pairwise_index()
    buf, soffs = gpu.encode_many(flat, offs)
    ix = gpu.Index(buf, soffs, universe=1 << 26, bitmap_gap=32)
    log(f"hybrid index: {ix.bitmap_lists} bitmap lists, {ix.bitmap_bytes >> 20} MiB of bitmaps")
    assert ix.bitmap_lists == 4
    if kind == "pairwise":
        terms, qoffs = workloads.pairwise_queries(ix.lengths, 1 << 18)
    else:
        terms, qoffs = workloads.multiterm_queries(ix.lengths, 1 << 18)
    b = gpu.Batch(ix, terms, qoffs)
    b.run(use_graph=True)
    torch.cuda.synchronize()
    roffs = b.res_offsets.cpu().numpy()
    res = b.results.cpu().numpy().view(np.uint32)
    bm = ix.kinds().astype(bool)
    touching = [q for q in range(1 << 18) if bm[terms[int(qoffs[q]): int(qoffs[q + 1])]].any()]
    rng = np.random.default_rng(5)
    sample = sorted(set(rng.choice(1 << 18, size=3000, replace=False).tolist()) | set(touching[:2000]))
    log(f"{len(touching)} queries touch a bitmap list; checking {len(sample)}")
    for q in sample:
        ts = terms[int(qoffs[q]): int(qoffs[q + 1])]
        want = oracle.hyb_intersect_k([raw(flat, offs, t) for t in ts], 1 << 26, 32)
        got = res[int(roffs[q]): int(roffs[q + 1])]
        assert np.array_equal(got, want), (q, ts.tolist())
    ix.free()
