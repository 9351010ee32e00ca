"""Doc-ID partitioned index inside one GPU (the paper's partitioned index,
Sec. 7.7, with one part per XCD): every list split by value range into
parts encoded separately; a batch runs each query part by part and joins
the parts' results in order.  Results equal the oracle's intersection of
the whole lists, and the unpartitioned batch's, query by query."""
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
def lists():
    lens = workloads.index_lengths(1 << 10, 16)
    kinds = np.full(lens.size, workloads.CLUSTERED, dtype=np.int32)
    kinds[1::3] = workloads.UNIFORM
    flat, offs = workloads.lists(kinds, lens, 515, UNIVERSE)
    return flat, offs


def partitioned(gpu, flat, offs, parts, universe, **kw):
    sub = gpu.partition_offsets(flat, offs, parts, universe)
    buf, soffs = gpu.encode_many(flat, sub, **kw)
    return gpu.Index(buf, soffs, parts=parts)


def run(gpu, ix, terms, qoffs, graph=False):
    import torch
    b = gpu.Batch(ix, terms, qoffs)
    b.run(use_graph=graph)
    torch.cuda.synchronize()
    return b.counts.cpu().numpy()[: b.nq], b.res_offsets.cpu().numpy(), b.results.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("parts", [2, 8, 13])
def test_partitioned_batch_matches_oracle(gpu, lists, parts):
    flat, offs = lists
    ix = partitioned(gpu, flat, offs, parts, UNIVERSE)
    assert ix.count == offs.size - 1
    assert np.array_equal(ix.lengths, np.diff(offs))
    terms, qoffs = workloads.queries(parts, ix.lengths, 900, 1, 6)
    counts, roffs, res = run(gpu, ix, terms, qoffs)
    for q in range(900):
        ts = terms[int(qoffs[q]): int(qoffs[q + 1])]
        want = oracle.intersect_k([flat[int(offs[t]): int(offs[t + 1])] for t in ts])
        got = res[int(roffs[q]): int(roffs[q + 1])]
        assert int(counts[q]) == got.size
        assert np.array_equal(got, want), (q, ts.tolist())
    # graph replay of the same plan
    c2, r2, res2 = run(gpu, ix, terms, qoffs, graph=True)
    assert np.array_equal(r2, roffs) and np.array_equal(res2[: int(roffs[-1])], res[: int(roffs[-1])])
    with pytest.raises(gpu.S4Error):
        ix.list(0)


def test_partitioned_patched_lists(gpu, lists):
    """Parts encoded as S4-FastPFOR-D1 (the patched chunk-kernel
    instantiation over a partitioned index)."""
    flat, offs = lists
    ix = partitioned(gpu, flat, offs, 8, UNIVERSE, delta=gpu.DELTA_D1, patched=True)
    terms, qoffs = workloads.queries(99, ix.lengths, 500, 2, 5)
    counts, roffs, res = run(gpu, ix, terms, qoffs)
    for q in range(500):
        ts = terms[int(qoffs[q]): int(qoffs[q + 1])]
        want = oracle.intersect_k([flat[int(offs[t]): int(offs[t + 1])] for t in ts])
        assert np.array_equal(res[int(roffs[q]): int(roffs[q + 1])], want), q


def test_parts_out_of_order_rejected(gpu):
    a = np.array([10, 20, 30], dtype=np.uint32)
    b = np.array([5, 6], dtype=np.uint32)        # part 1 below part 0
    flat = np.concatenate([a, b])
    sub = np.array([0, 3, 5], dtype=np.uint64)
    buf, soffs = gpu.encode_many(flat, sub)
    with pytest.raises(gpu.S4Error) as e:
        gpu.Index(buf, soffs, parts=2)
    assert e.value.code == gpu.EINVAL
    ok = np.concatenate([b, a])                  # ascending parts, one empty part in between
    buf, soffs = gpu.encode_many(ok, np.array([0, 2, 2, 5], dtype=np.uint64))
    ix = gpu.Index(buf, soffs, parts=3)
    assert ix.lengths.tolist() == [5]


def test_server_refuses_partitioned_index(gpu, lists):
    flat, offs = lists
    ix = partitioned(gpu, flat, offs, 4, UNIVERSE)
    with pytest.raises(gpu.S4Error) as e:
        gpu.Server(ix, max_slots=64, pool_bytes=1 << 24)
    assert e.value.code == gpu.EINVAL


@pytest.mark.timeout(600)
@pytest.mark.parametrize("kind", ["pairwise", "multiterm"])
def test_full_size_partitioned_batch(gpu, kind):
    """The batched workloads at full size (2^16 lists over [0, 2^26), 2^18
    queries) over an 8-part index: every query's result identical to the
    unpartitioned index's, and 2000 sampled results equal to the oracle's."""
    flat, offs = workloads.pairwise_index()
    buf, soffs = gpu.encode_many(flat, offs)
    plain = gpu.Index(buf, soffs)
    ix = partitioned(gpu, flat, offs, 8, 1 << 26)
    terms, qoffs = (workloads.pairwise_queries if kind == "pairwise" else workloads.multiterm_queries)(
        plain.lengths, 1 << 18)
    c0, r0, res0 = run(gpu, plain, terms, qoffs)
    c1, r1, res1 = run(gpu, ix, terms, qoffs, graph=True)
    assert np.array_equal(c0, c1) and np.array_equal(r0, r1)
    assert np.array_equal(res0[: int(r0[-1])], res1[: int(r1[-1])])
    rng = np.random.default_rng(8)
    for q in rng.choice(1 << 18, size=2000, replace=False):
        ts = terms[int(qoffs[q]): int(qoffs[q + 1])]
        want = oracle.intersect_k([flat[int(offs[t]): int(offs[t + 1])] for t in ts])
        assert np.array_equal(res1[int(r1[q]): int(r1[q + 1])], want), q
