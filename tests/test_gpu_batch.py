"""Batched conjunctive queries over a device-resident index: every query's
result equals the oracle's k-way intersection of the generated lists."""
import sys
import time

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def small_index(gpu):
    # the pairwise-config length law and generator, scaled down 2^6 x
    lens = workloads.index_lengths(1 << 11, 17)
    kinds = np.full(lens.size, workloads.CLUSTERED, dtype=np.int32)
    flat, offs = workloads.lists(kinds, lens, 4242, 1 << 20)
    buf, soffs = gpu.encode_many(flat, offs)
    ix = gpu.Index(buf, soffs)
    return ix, flat, offs


def raw_list(flat, offs, t):
    return flat[int(offs[t]): int(offs[t + 1])]


def check_batch(gpu, b, terms, qoffs, flat, offs, sample=None):
    import torch
    torch.cuda.synchronize()
    counts = b.counts.cpu().numpy()
    roffs = b.res_offsets.cpu().numpy()
    res = b.results.cpu().numpy().view(np.uint32)
    qs = range(b.nq) if sample is None else sample
    for q in qs:
        ts = terms[int(qoffs[q]): int(qoffs[q + 1])]
        want = oracle.intersect_k([raw_list(flat, offs, t) for t in ts])
        got = res[int(roffs[q]): int(roffs[q + 1])]
        assert int(counts[q]) == got.size
        assert np.array_equal(got, want), (q, ts)
    assert roffs[0] == 0 and np.all(np.diff(roffs) == counts[: b.nq])


@pytest.mark.parametrize("kmin,kmax", [(2, 2), (3, 6), (1, 8)])
def test_batch_matches_oracle(gpu, small_index, kmin, kmax):
    ix, flat, offs = small_index
    terms, qoffs = workloads.queries(77 + kmin * 10 + kmax, ix.lengths, 1500, kmin, kmax)
    b = gpu.Batch(ix, terms, qoffs)
    b.run()
    check_batch(gpu, b, terms, qoffs, flat, offs)


def test_batch_graph_replays(gpu, small_index):
    """Graph replays, with eager runs in between, all match the eager run."""
    import torch
    ix, flat, offs = small_index
    terms, qoffs = workloads.queries(5, ix.lengths, 800, 2, 5)
    b = gpu.Batch(ix, terms, qoffs)
    b.run()
    torch.cuda.synchronize()
    ref = (b.counts.clone(), b.res_offsets.clone(), b.results.clone())
    for rep in range(4):
        b.results.zero_()
        b.counts.zero_()
        b.run(use_graph=True)
        torch.cuda.synchronize()
        assert torch.equal(b.counts, ref[0]) and torch.equal(b.res_offsets, ref[1])
        n = int(ref[1][-1].item())
        assert torch.equal(b.results[:n], ref[2][:n]), rep
        b.run()  # eager work between replays
        torch.cuda.synchronize()
    check_batch(gpu, b, terms, qoffs, flat, offs, sample=range(0, 800, 7))


def test_batch_invariant_under_tuning(gpu, small_index):
    import torch
    ix, flat, offs = small_index
    terms, qoffs = workloads.queries(9, ix.lengths, 600, 2, 6)
    b = gpu.Batch(ix, terms, qoffs)
    old = gpu.get_tuning().as_dict()
    try:
        ref = None
        for g, w, gp, grab in [(64, 4, 8, 1), (1, 1, 1, 1), (512, 8, 16, 4), (4, 2, 2, 2), (16, 4, 4, 3)]:
            gpu.set_tuning(gallop_blocks=g, waves_per_group=w, groups_per_cu=gp, items_per_grab=grab)
            b.run()
            torch.cuda.synchronize()
            n = int(b.res_offsets[-1].item())
            cur = (b.counts.clone(), b.results[:n].clone())
            if ref is None:
                ref = cur
            assert torch.equal(cur[0], ref[0]) and torch.equal(cur[1], ref[1])
        best, ms = b.autotune(reps=1)
        b.run()
        torch.cuda.synchronize()
        n = int(b.res_offsets[-1].item())
        assert torch.equal(b.counts, ref[0]) and torch.equal(b.results[:n], ref[1])
        assert ms > 0 and set(best) >= {"gallop_blocks", "waves_per_group"}
    finally:
        gpu.set_tuning(**old)
    check_batch(gpu, b, terms, qoffs, flat, offs, sample=range(0, 600, 5))


def test_query_ticks(gpu, small_index):
    import torch
    ix, flat, offs = small_index
    terms, qoffs = workloads.queries(11, ix.lengths, 300, 2, 4)
    b = gpu.Batch(ix, terms, qoffs)
    b.run()
    t = b.query_ticks()
    assert t.size == 300 and (t > 0).all()
    assert b.traffic() == (0, 0)  # counting is off by default
    counts, results = b.counts.clone(), b.results.clone()
    b.set_counting(True)
    b.run()
    nbytes, blocks = b.traffic()
    torch.cuda.synchronize()
    assert torch.equal(b.counts, counts) and torch.equal(b.results, results)
    b.set_counting(False)
    b.run()
    assert b.traffic() == (0, 0)
    chunks = sum((int(ix.lengths[min(terms[int(qoffs[q]): int(qoffs[q + 1])], key=lambda x: ix.lengths[x])]) + 127)
                 // 128 for q in range(300))
    assert blocks >= chunks * 0.5 and nbytes > 16 * blocks


def test_counting_through_graph(gpu, small_index):
    # switching counting re-captures the batch's graph: a replay of the old
    # graph would keep the old setting
    import torch
    ix, flat, offs = small_index
    terms, qoffs = workloads.queries(12, ix.lengths, 400, 2, 5)
    b = gpu.Batch(ix, terms, qoffs)
    b.run(use_graph=True)
    b.run(use_graph=True)
    assert b.traffic() == (0, 0)
    counts, results = b.counts.clone(), b.results.clone()
    b.set_counting(True)
    seen = []
    for _ in range(2):
        b.run(use_graph=True)
        seen.append(b.traffic())
    assert seen[0] == seen[1] and seen[0][0] > 0 and seen[0][1] > 0
    b.set_counting(False)
    b.run(use_graph=True)
    assert b.traffic() == (0, 0)
    torch.cuda.synchronize()
    assert torch.equal(b.counts, counts) and torch.equal(b.results, results)
    check_batch(gpu, b, terms, qoffs, flat, offs, sample=range(0, 400, 7))


def test_batch_rejects_bad_queries(gpu, small_index):
    ix, _, _ = small_index
    with pytest.raises(gpu.S4Error):
        gpu.Batch(ix, np.array([0, ix.count], np.uint32), np.array([0, 2], np.uint64))
    with pytest.raises(gpu.S4Error):
        gpu.Batch(ix, np.array([0], np.uint32), np.array([0, 0, 1], np.uint64))


@pytest.mark.parametrize("name", ["pairwise", "multiterm"])
def test_full_size_batch_sampled(gpu, name):
    """The batched-query workloads at full size (index of 2^16 lists,
    2^18 queries) in the configuration the benchmark times; a seeded sample
    of 2^11 queries is checked against the oracle."""
    t0 = time.time()
    flat, offs = workloads.pairwise_index()
    buf, soffs = gpu.encode_many(flat, offs)
    ix = gpu.Index(buf, soffs)
    qfn = workloads.pairwise_queries if name == "pairwise" else workloads.multiterm_queries
    terms, qoffs = qfn(ix.lengths)
    b = gpu.Batch(ix, terms, qoffs)
    b.autotune(reps=1)
    b.run(use_graph=True)
    log(f"{name}: index + batch in {time.time() - t0:.1f} s")
    rng = np.random.default_rng(3)
    sample = np.sort(rng.choice(b.nq, size=1 << 11, replace=False))
    check_batch(gpu, b, terms, qoffs, flat, offs, sample=sample)
