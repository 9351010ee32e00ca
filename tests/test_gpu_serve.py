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


@pytest.mark.parametrize("result_bytes", [32 << 20, 3 * 4 * 128])
def test_server_results_match_oracle(gpu, served, result_bytes):
    """With a roomy result buffer the device writes results straight to
    pinned host memory; with one of 128 values per context most iterations
    go through device memory (an asynchronous copy, or a synchronous one
    when the total exceeds the buffer)."""
    ix, flat, offs = served
    terms, qoffs = workloads.queries(21, ix.lengths, 600, 1, 8)
    srv = gpu.Server(ix, max_slots=256, pool_bytes=64 << 20, result_bytes=result_bytes)
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
        assert 1 <= st["max_batch"] <= 256 // 3 and st["device_ns"] > 0
        if result_bytes > 1 << 20:
            assert st["direct_iterations"] == st["iterations"]
        else:
            assert st["direct_iterations"] < st["iterations"]
    finally:
        srv.close()


def test_single_pass_and_staged_iterations(gpu, served):
    """An iteration of at most one chunk per resident wave runs as one
    single-pass kernel (look-back offsets), a larger one in the staged form;
    with one one-wave group per CU (256 resident waves) a mix of queries
    takes both, and every result still equals the oracle's."""
    ix, flat, offs = served
    terms, qoffs = workloads.queries(23, ix.lengths, 800, 2, 6)
    saved = gpu.get_tuning()
    gpu.set_tuning(waves_per_group=1, groups_per_cu=1)
    srv = gpu.Server(ix, max_slots=3 * 1024, pool_bytes=3 << 30, result_bytes=3 << 26)
    try:
        small = int(np.argmin(ix.lengths[:64]))
        first = srv.submit([small, small])
        drain(srv, [first])
        # all 800 due at once: queued under one lock, so iterations are large
        r = srv.replay(terms, qoffs, np.zeros(800, np.uint64), with_results=True, results_cap=1 << 24)
        for q in range(800):
            ts = terms[int(qoffs[q]): int(qoffs[q + 1])]
            got = r["results"][int(r["res_offsets"][q]): int(r["res_offsets"][q + 1])]
            assert np.array_equal(got, want(flat, offs, ts)), q
        st = srv.stats()
        assert 1 <= st["single_pass_iterations"] < st["iterations"], st
    finally:
        srv.close()
        gpu.set_tuning(**{k: getattr(saved, k) for k, _ in saved._fields_})


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
    # a pool of 8 chunks per iteration: the long query runs 8 chunks at a
    # time, its slices joined in order
    tiny = gpu.Server(ix, max_slots=8, pool_bytes=3 * 4096, result_bytes=1 << 20)
    try:
        qid = tiny.submit([big, 0])
        got = drain(tiny, [qid])
        assert np.array_equal(got[qid][0], want(flat, offs, [big, 0]))
        st = tiny.stats()
        assert st["sliced_queries"] == 1 and st["iterations"] >= (int(ix.lengths[0]) + 1023) // 1024
    finally:
        tiny.close()
    # a pool smaller than one chunk can hold nothing
    none = gpu.Server(ix, max_slots=8, pool_bytes=256, result_bytes=1 << 20)
    try:
        with pytest.raises(gpu.S4Error) as e:
            none.submit([big, 0])
        assert e.value.code == gpu.ERANGE
        assert none.stats()["rejected"] == 1
    finally:
        none.close()


@pytest.mark.parametrize("slice_chunks", [1, 7, 64])
def test_sliced_queries_match_oracle(gpu, served, slice_chunks):
    """Queries longer than a slice run one slice per iteration, interleaved
    with short ones and with each other (several contexts in flight); the
    joined results equal the oracle's, and short queries still finish."""
    ix, flat, offs = served
    terms, qoffs = workloads.queries(24 + slice_chunks, ix.lengths, 500, 1, 6)
    srv = gpu.Server(ix, max_slots=384, pool_bytes=256 << 20, result_bytes=64 << 20, slice_chunks=slice_chunks)
    try:
        r = srv.replay(terms, qoffs, np.zeros(500, np.uint64), with_results=True, results_cap=1 << 24)
        st = srv.stats()
    finally:
        srv.close()
    for q in range(500):
        ts = terms[int(qoffs[q]): int(qoffs[q + 1])]
        got = r["results"][int(r["res_offsets"][q]): int(r["res_offsets"][q + 1])]
        assert np.array_equal(got, want(flat, offs, ts)), q
    long_q = sum(1 for q in range(500)
                 if (min(int(ix.lengths[t]) for t in terms[int(qoffs[q]): int(qoffs[q + 1])]) + 127) // 128
                 > slice_chunks)
    assert st["sliced_queries"] == long_q > 0
    assert st["completed"] == 500


def test_sliced_queries_through_poll(gpu, served):
    """Long queries submitted one by one and drained through s4_server_poll
    a few at a time: the slices' results, handed over in chunk order and
    joined by the poll into the caller's buffer, equal the oracle's."""
    ix, flat, offs = served
    terms, qoffs = workloads.queries(77, ix.lengths, 300, 1, 6)
    srv = gpu.Server(ix, max_slots=256, pool_bytes=256 << 20, result_bytes=64 << 20, slice_chunks=5)
    try:
        ids = {}
        for q in range(300):
            qid = None
            while qid is None:
                qid = srv.submit(terms[int(qoffs[q]): int(qoffs[q + 1])])
            ids[qid] = q
        got = {}
        t0 = time.time()
        while len(got) < 300:
            for qid, res, lat in srv.poll(max_done=7, results_cap=1 << 19):
                got[qid] = res
            assert time.time() - t0 < 60, f"{len(got)} of 300 results"
            time.sleep(0.0005)
        st = srv.stats()
    finally:
        srv.close()
    assert st["sliced_queries"] > 0
    for qid, q in ids.items():
        assert np.array_equal(got[qid], want(flat, offs, terms[int(qoffs[q]): int(qoffs[q + 1])])), q


def test_replay_open_loop(gpu, served):
    ix, flat, offs = served
    nq = 2000
    terms, qoffs = workloads.queries(31, ix.lengths, nq, 2, 8)
    arr = (workloads.arrivals(32, 20000.0, nq) * 1e9).astype(np.uint64)
    srv = gpu.Server(ix, max_slots=1024, pool_bytes=256 << 20)
    try:
        r = srv.replay(terms, qoffs, arr, with_results=True, results_cap=1 << 24)
    finally:
        srv.close()
    assert (r["latency_ns"] > 0).all() and r["elapsed_s"] > 0
    for q in range(0, nq, 13):
        ts = terms[int(qoffs[q]): int(qoffs[q + 1])]
        got = r["results"][int(r["res_offsets"][q]): int(r["res_offsets"][q + 1])]
        assert np.array_equal(got, want(flat, offs, ts)), q
        assert int(r["counts"][q]) == got.size


@pytest.mark.timeout(900)
def test_full_size_serving_sampled(gpu):
    """The serving workload at full size (2^20 clustered lists over
    [0, 2^31), 3.9e9 integers, device-resident), 2^12 queries of 2..8 terms
    replayed open-loop at saturation; every result checked with the oracle."""
    t0 = time.time()
    lens = workloads.index_lengths(1 << 20, 28)
    kinds = np.full(lens.size, workloads.CLUSTERED, dtype=np.int32)
    flat, offs = workloads.lists(kinds, lens, workloads.config_seed(4, 0), 1 << 31)
    buf, soffs = gpu.encode_many(flat, offs)
    ix = gpu.Index(buf, soffs)
    del buf, soffs
    print(f"serving index built in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    nq = 1 << 12
    terms, qoffs = workloads.serving_queries(ix.lengths, nq, level=7)
    srv = gpu.Server(ix, max_slots=1 << 14, pool_bytes=24 << 30, result_bytes=3 << 28)
    try:
        r = srv.replay(terms, qoffs, np.zeros(nq, np.uint64), with_results=True, results_cap=1 << 28)
    finally:
        srv.close()
    for q in range(nq):
        ts = sorted(terms[int(qoffs[q]): int(qoffs[q + 1])], key=lambda t: int(lens[t]))
        w = oracle.intersect_k([flat[int(offs[t]): int(offs[t + 1])] for t in ts])
        got = r["results"][int(r["res_offsets"][q]): int(r["res_offsets"][q + 1])]
        assert np.array_equal(got, w), q


def test_concurrent_submitters(gpu, served):
    """Four threads submit at once (their queries reach the dispatcher in
    batches taken under the server lock) while the main thread drains:
    every id is distinct, every result equals the oracle's, and nothing is
    lost or admitted twice."""
    import threading
    ix, flat, offs = served
    terms, qoffs = workloads.queries(23, ix.lengths, 2000, 1, 8)
    srv = gpu.Server(ix, max_slots=512, pool_bytes=64 << 20, result_bytes=32 << 20)
    ids = {}
    lock = threading.Lock()
    errors = []

    def submitter(part):
        try:
            for q in range(part, 2000, 4):
                ts = terms[int(qoffs[q]): int(qoffs[q + 1])]
                qid = srv.submit(ts)
                with lock:
                    ids[qid] = ts
        except Exception as ex:  # surfaced below
            errors.append(ex)

    try:
        threads = [threading.Thread(target=submitter, args=(p,)) for p in range(4)]
        for t in threads:
            t.start()
        for t in threads:
            t.join(timeout=60)
        assert not errors, errors
        assert len(ids) == 2000
        got = drain(srv, ids)
        assert set(got) == set(ids)
        for qid, ts in ids.items():
            assert np.array_equal(got[qid][0], want(flat, offs, ts)), ts
        st = srv.stats()
        assert st["submitted"] == 2000 and st["admitted"] == 2000 and st["completed"] == 2000
    finally:
        srv.close()


def test_replay_rejects_bad_query_then_serves(gpu, served):
    """A replayed trace whose query 5000 names a term outside the index (in
    the second segment the replay prepares ahead) fails with EINVAL and the
    query's message; the server then serves the next trace normally."""
    ix, flat, offs = served
    terms, qoffs = workloads.queries(29, ix.lengths, 6000, 1, 8)
    terms = np.array(terms, dtype=np.uint32)
    terms[int(qoffs[5000])] = ix.count + 7
    srv = gpu.Server(ix, max_slots=512, pool_bytes=64 << 20, result_bytes=32 << 20)
    try:
        with pytest.raises(gpu.S4Error) as e:
            srv.replay(terms, qoffs, np.zeros(6000, np.uint64))
        assert e.value.code == gpu.EINVAL and "term out of range" in str(e.value)
        terms2, qoffs2 = workloads.queries(31, ix.lengths, 3000, 1, 8)
        r = srv.replay(terms2, qoffs2, np.zeros(3000, np.uint64), with_results=True, results_cap=1 << 24)
        for q in range(0, 3000, 7):
            ts = terms2[int(qoffs2[q]): int(qoffs2[q + 1])]
            got = r["results"][int(r["res_offsets"][q]): int(r["res_offsets"][q + 1])]
            assert np.array_equal(got, want(flat, offs, ts)), ts
    finally:
        srv.close()


def test_staged_iterations_with_chunkless_entries(gpu):
    """Staged iterations whose entries include queries with no chunks (the
    shortest term's list is empty): in the middle of an iteration, several
    in a row, and at its end, where the last tile of the tail kernel writes
    their offsets; entries straddle the tail's tiles of 1024 chunks.  Every
    result equals the oracle's (empty where a term is empty)."""
    lens = workloads.index_lengths(1 << 10, 17).copy()
    lens[::9] = 0
    kinds = np.full(lens.size, workloads.CLUSTERED, dtype=np.int32)
    flat, offs = workloads.lists(kinds, lens, 778, 1 << 22)
    buf, soffs = gpu.encode_many(flat, offs)
    ix = gpu.Index(buf, soffs)
    nq = 900
    terms, qoffs = workloads.queries(24, lens, nq, 2, 6)
    terms = terms.copy()
    empties = np.nonzero(lens == 0)[0].astype(np.uint32)
    rng = np.random.Generator(np.random.PCG64(24))
    # every 7th query, a run of five, and the last four get an empty term
    pick = set(range(0, nq, 7)) | set(range(400, 405)) | set(range(nq - 4, nq))
    for q in pick:
        terms[int(qoffs[q + 1]) - 1] = empties[rng.integers(empties.size)]
    saved = gpu.get_tuning()
    gpu.set_tuning(waves_per_group=1, groups_per_cu=1)
    srv = gpu.Server(ix, max_slots=3 * 1024, pool_bytes=3 << 30, result_bytes=3 << 26)
    try:
        r = srv.replay(terms, qoffs, np.zeros(nq, np.uint64), with_results=True, results_cap=1 << 24)
        for q in range(nq):
            ts = terms[int(qoffs[q]): int(qoffs[q + 1])]
            got = r["results"][int(r["res_offsets"][q]): int(r["res_offsets"][q + 1])]
            assert np.array_equal(got, want(flat, offs, ts)), q
            if q in pick:
                assert got.size == 0, q
        st = srv.stats()
        assert st["single_pass_iterations"] < st["iterations"], st
    finally:
        srv.close()
        gpu.set_tuning(**{k: getattr(saved, k) for k, _ in saved._fields_})
