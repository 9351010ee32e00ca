"""The plain path (one single-launch conjunction per query, submitted from
C++) and the serving replay's result selection, against the oracle."""
import sys

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def small_index(gpu):
    lens = workloads.index_lengths(1 << 10, 18)
    kinds = np.full(lens.size, workloads.CLUSTERED, dtype=np.int32)
    flat, offs = workloads.lists(kinds, lens, 4242, 1 << 22)
    buf, soffs = gpu.encode_many(flat, offs)
    return gpu.Index(buf, soffs), flat, offs


def want(flat, offs, ts):
    return oracle.intersect_k([flat[int(offs[t]): int(offs[t + 1])] for t in ts])


@pytest.mark.parametrize("kmin,kmax", [(2, 2), (3, 6), (2, 8)])
@pytest.mark.parametrize("isolate", [False, True])
def test_plain_run_vs_oracle(gpu, small_index, kmin, kmax, isolate):
    ix, flat, offs = small_index
    terms, qoffs = workloads.queries(777 + kmin * 10 + kmax, ix.lengths, 300, kmin, kmax)
    log("plain run", kmin, kmax, isolate)
    counts, results, roffs, ms, lat = gpu.plain_run(ix, terms, qoffs, isolate=isolate)
    counts = counts.cpu().numpy()
    host = results.cpu().numpy().view(np.uint32)
    for q in range(qoffs.size - 1):
        ts = terms[int(qoffs[q]): int(qoffs[q + 1])]
        w = want(flat, offs, ts)
        assert int(counts[q]) == w.size, q
        assert np.array_equal(host[int(roffs[q]): int(roffs[q]) + w.size], w), q
    assert ms > 0
    if isolate:
        assert lat.size == qoffs.size - 1 and (lat > 0).all()


def test_plain_run_rejects(gpu, small_index):
    ix, flat, offs = small_index
    with pytest.raises(gpu.S4Error) as e:
        gpu.plain_run(ix, np.array([1], np.uint32), np.array([0, 1], np.uint64))  # one term
    assert e.value.code == gpu.EINVAL
    with pytest.raises(gpu.S4Error) as e:
        gpu.plain_run(ix, np.array([1, ix.count], np.uint32), np.array([0, 2], np.uint64))
    assert e.value.code == gpu.EINVAL


def test_plain_replay_counts(gpu, small_index):
    ix, flat, offs = small_index
    terms, qoffs = workloads.queries(31337, ix.lengths, 2000, 2, 8)
    arr = (workloads.arrivals(5, 2.0e5, 2000) * 1e9).astype(np.uint64)
    log("plain replay")
    r = gpu.plain_replay(ix, terms, qoffs, arr)
    counts, _, _, _, _ = gpu.plain_run(ix, terms, qoffs)
    assert np.array_equal(r["counts"], counts.cpu().numpy().astype(np.uint64))
    assert r["elapsed_s"] > 0 and r["latency_ns"].size == 2000
    for q in range(0, 2000, 97):
        ts = terms[int(qoffs[q]): int(qoffs[q + 1])]
        assert int(r["counts"][q]) == want(flat, offs, ts).size


def test_server_replay_keep(gpu, small_index):
    """Replay with a selection of queries whose results are returned: those
    equal the oracle, the others come back empty, every count is right."""
    ix, flat, offs = small_index
    nq = 3000
    terms, qoffs = workloads.queries(4711, ix.lengths, nq, 2, 8)
    arr = (workloads.arrivals(6, 1.0e6, nq) * 1e9).astype(np.uint64)
    keep = np.zeros(nq, np.uint8)
    keep[::7] = 1
    srv = gpu.Server(ix, max_slots=512, pool_bytes=1 << 28, result_bytes=1 << 26, max_terms=8)
    try:
        r = srv.replay(terms, qoffs, arr, with_results=True, results_cap=1 << 24, keep=keep)
    finally:
        srv.close()
    ro = r["res_offsets"]
    for q in range(nq):
        ts = terms[int(qoffs[q]): int(qoffs[q + 1])]
        if q % 7 == 0 or q % 101 == 0:
            w = want(flat, offs, ts)
            assert int(r["counts"][q]) == w.size, q
        if keep[q]:
            assert np.array_equal(r["results"][int(ro[q]): int(ro[q + 1])], w), q
        else:
            assert ro[q + 1] == ro[q]
