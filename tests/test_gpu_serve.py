"""The continuous-batching server: every result equals the oracle's, and a
query's result is the same alone and in a concurrent mix."""
import sys
import time

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def served(gpu):
    lens = workloads.index_lengths(1 << 11, 18)
    kinds = np.full(lens.size, workloads.CLUSTERED, dtype=np.int32)
    flat, offs = workloads.lists(kinds, lens, 777, 1 << 23)
    buf, soffs = gpu.encode_many(flat, offs)
    ix = gpu.Index(buf, soffs)
    return ix, flat, offs


def drain(srv, ids, timeout=60.0):
    got = {}
    t0 = time.time()
    while len(got) < len(ids):
        for qid, res, lat in srv.poll():
            got[qid] = (res, lat)
        if time.time() - t0 > timeout:
            raise TimeoutError(f"{len(got)} of {len(ids)} results after {timeout} s")
        time.sleep(0.0005)
    return got


def want(flat, offs, ts):
    return oracle.intersect_k([flat[int(offs[t]): int(offs[t + 1])] for t in ts])


def test_server_results_match_oracle(gpu, served):
    ix, flat, offs = served
    terms, qoffs = workloads.queries(21, ix.lengths, 600, 1, 8)
    srv = gpu.Server(ix, max_slots=256, pool_bytes=64 << 20, result_bytes=32 << 20)
    try:
        ids = {}
        for q in range(600):
            ts = terms[int(qoffs[q]): int(qoffs[q + 1])]
            ids[srv.submit(ts)] = ts
        got = drain(srv, ids)
        for qid, ts in ids.items():
            assert np.array_equal(got[qid][0], want(flat, offs, ts)), ts
            assert got[qid][1] > 0
        st = srv.stats()
        assert st["completed"] == 600 and st["admitted"] == 600 and st["iterations"] >= 1
    finally:
        srv.close()


def test_alone_equals_in_mix(gpu, served):
    ix, flat, offs = served
    terms, qoffs = workloads.queries(22, ix.lengths, 400, 2, 8)
    qs = [terms[int(qoffs[q]): int(qoffs[q + 1])] for q in range(400)]
    srv = gpu.Server(ix, max_slots=512, pool_bytes=128 << 20, result_bytes=64 << 20)
    try:
        alone = {}
        for q in range(0, 400, 20):
            qid = srv.submit(qs[q])
            alone[q] = drain(srv, [qid])[qid][0]
        ids = {srv.submit(ts): q for q, ts in enumerate(qs)}
        mix = drain(srv, ids)
        by_q = {q: mix[qid][0] for qid, q in ids.items()}
        for q, res in alone.items():
            assert np.array_equal(res, by_q[q]), q
            assert np.array_equal(res, want(flat, offs, qs[q]))
        assert srv.stats()["peak_active"] > 1
    finally:
        srv.close()


def test_memory_admission(gpu, served):
    ix, flat, offs = served
    big = int(np.argmax(ix.lengths))
    need = 4 * 128 * ((int(ix.lengths[big]) + 127) // 128)
    # pool holds this query's chunks but not two at once: admission waits
    srv = gpu.Server(ix, max_slots=64, pool_bytes=3 * need + 3 * 512, result_bytes=64 << 20)
    try:
        ids = [srv.submit([big, big]) for _ in range(6)]
        got = drain(srv, ids)
        ref = flat[int(offs[big]): int(offs[big + 1])]
        for qid in ids:
            assert np.array_equal(got[qid][0], ref)
        st = srv.stats()
        assert st["completed"] == 6
    finally:
        srv.close()
    tiny = gpu.Server(ix, max_slots=8, pool_bytes=3 * 4096, result_bytes=1 << 20)
    try:
        with pytest.raises(gpu.S4Error) as e:
            tiny.submit([big, 0])
        assert e.value.code == gpu.ERANGE
        assert tiny.stats()["rejected"] == 1
    finally:
        tiny.close()
