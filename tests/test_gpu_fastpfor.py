"""GPU parity for patched S4-FastPFOR lists (Sec. 4.4) in every
differential form: bulk decode (unpack, patch and prefix fused in one
pass), the skip index, random block access, intersections mixing patched
and plain lists, batches over a mixed index, hybrid bitmaps built from
patched lists, and the bulk workload at full size."""
import sys

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu
FORMS = [oracle.D4, oracle.DM, oracle.D2, oracle.D1]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def with_outliers(seed, n):
    """Gaps of a few units with sparse jumps of 2^4 .. 2^21: exceptions at
    many widths in many blocks."""
    rng = np.random.default_rng(seed)
    gaps = rng.geometric(0.3, size=n).astype(np.uint64)
    k = max(1, n // 150)
    if n:
        gaps[rng.integers(0, n, size=k)] += np.uint64(1) << rng.integers(4, 22, size=k).astype(np.uint64)
    x = np.cumsum(gaps)
    assert n == 0 or x[-1] < 1 << 32
    return x.astype(np.uint32)


def dense_with_spikes(seed, n):
    """Almost every block patched: gaps of 1..3 with one 2^10..2^16 jump
    every 40 values on average."""
    rng = np.random.default_rng(seed)
    gaps = rng.integers(1, 4, size=n).astype(np.uint64)
    spikes = rng.random(n) < 1 / 40
    gaps[spikes] += np.uint64(1) << rng.integers(10, 17, size=int(spikes.sum())).astype(np.uint64)
    x = np.cumsum(gaps)
    assert n == 0 or x[-1] < 1 << 32
    return x.astype(np.uint32)


@pytest.mark.parametrize("mode", FORMS)
@pytest.mark.parametrize("n", [1, 127, 128, 129, 513, 2049, 128 * 1100 + 77, (1 << 20) + 37])
def test_decode_patched(gpu, mode, n):
    for x in (workloads.sorted_list(workloads.CLUSTERED, 700 + n, 1 << 26, n), with_outliers(n + mode, n),
              dense_with_spikes(n, n)):
        enc = gpu.encode(x, mode, patched=True)
        lst = gpu.DeviceList.upload(enc)
        got = lst.decode().cpu().numpy().view(np.uint32)
        assert np.array_equal(got, x)
        assert np.array_equal(got, oracle.decode(enc))


@pytest.mark.parametrize("mode", [oracle.D4, oracle.D1])
def test_decode_patched_large(gpu, mode):
    """A patched list long enough (2^15 full blocks and a ragged tail) for
    the per-list launch to take 4 passes per wave, where each pass's
    exception records are read a pass ahead."""
    n = (1 << 22) + 77
    rng = np.random.default_rng(900 + mode)
    gaps = rng.geometric(0.3, size=n).astype(np.uint64)
    k = n // 1000
    gaps[rng.integers(0, n, size=k)] += np.uint64(1) << rng.integers(4, 19, size=k).astype(np.uint64)
    sparse_outliers = np.cumsum(gaps)
    assert sparse_outliers[-1] < 1 << 32
    for x in (sparse_outliers.astype(np.uint32),
              workloads.sorted_list(workloads.CLUSTERED, 901 + mode, 1 << 26, n)):
        enc = gpu.encode(x, mode, patched=True)
        got = gpu.DeviceList.upload(enc).decode().cpu().numpy().view(np.uint32)
        assert np.array_equal(got, x)
        assert np.array_equal(got, oracle.decode(enc))


@pytest.mark.parametrize("mode", FORMS)
def test_patched_skip_index_and_blocks(gpu, mode):
    import torch
    x = dense_with_spikes(mode, 128 * 700 + 9)
    enc = gpu.encode(x, mode, patched=True)
    lst = gpu.DeviceList.upload(enc)
    nb = x.size // 128
    bmax, seeds = lst.skip_index()
    assert np.array_equal(bmax, x[127: 128 * nb: 128])
    for k in range(1, nb, 37):
        assert list(seeds[k]) == list(x[128 * k - 4: 128 * k]), k
    rng = np.random.default_rng(mode)
    for _ in range(10):
        first = int(rng.integers(0, lst.nb + 1))
        count = int(rng.integers(1, lst.nb + 2 - first))
        out = torch.zeros(128 * count, dtype=torch.int32, device="cuda")
        lst.decode_blocks_into(first, count, out)
        want = x[128 * first: 128 * (first + count)]
        assert np.array_equal(out.cpu().numpy().view(np.uint32)[: want.size], want)


def test_patched_list_sizes(gpu):
    x = with_outliers(5, 128 * 900 + 3)
    enc = gpu.encode(x, oracle.D1, patched=True)
    lst = gpu.DeviceList.upload(enc)
    nb = x.size // 128
    assert lst.payload_bytes == enc.size - 32 - (((nb + 3) & ~3) - nb)
    assert lst.index_bytes == nb * (24 + 16)


@pytest.mark.parametrize("ratio", [1, 16, 512])
def test_intersect_patched_and_plain(gpu, ratio):
    n = 1 << 17
    r, f = workloads.planted_pair(90 + ratio, n, n // ratio, 0.3)
    want = oracle.intersect(r, f)
    for mr, pr in ((oracle.D4, True), (oracle.D1, True), (oracle.D4, False)):
        for mf, pf in ((oracle.D4, True), (oracle.DM, True), (oracle.D2, False), (oracle.D1, True)):
            a = gpu.DeviceList.upload(gpu.encode(r, mr, patched=pr))
            b = gpu.DeviceList.upload(gpu.encode(f, mf, patched=pf))
            out, cnt = gpu.intersect(a, b)
            c = int(cnt.item())
            assert np.array_equal(out[:c].cpu().numpy().view(np.uint32), want), (mr, pr, mf, pf)


def test_intersect_k_patched(gpu):
    rng = np.random.default_rng(4)
    base = dense_with_spikes(11, 1 << 16)
    lists = [np.sort(rng.choice(base, size=s, replace=False)) for s in (1 << 15, 1 << 14, 1 << 13)] + [base]
    want = oracle.intersect_k(lists)
    handles = [gpu.DeviceList.upload(gpu.encode(l, m, patched=(i % 2 == 0)))
               for i, (l, m) in enumerate(zip(lists, FORMS))]
    out, cnt = gpu.intersect_k(handles)
    assert np.array_equal(out[: int(cnt.item())].cpu().numpy().view(np.uint32), want)


def test_batch_over_patched_index(gpu):
    """Index whose list t is patched when t is even, in form t mod 4."""
    lens = workloads.index_lengths(1 << 10, 16)
    kinds = np.full(lens.size, workloads.CLUSTERED, dtype=np.int32)
    flat, offs = workloads.lists(kinds, lens, 414, 1 << 20)
    streams = [gpu.encode(flat[int(offs[t]): int(offs[t + 1])], t % 4, patched=(t % 2 == 0))
               for t in range(lens.size)]
    soffs = np.zeros(lens.size + 1, np.uint64)
    np.cumsum([s.size for s in streams], out=soffs[1:])
    ix = gpu.Index(np.concatenate(streams), soffs)
    terms, qoffs = workloads.queries(18, ix.lengths, 700, 1, 6)
    b = gpu.Batch(ix, terms, qoffs)
    b.run()
    roffs = b.res_offsets.cpu().numpy()
    res = b.results.cpu().numpy().view(np.uint32)
    for q in range(700):
        ts = terms[int(qoffs[q]): int(qoffs[q + 1])]
        want = oracle.intersect_k([flat[int(offs[t]): int(offs[t + 1])] for t in ts])
        assert np.array_equal(res[int(roffs[q]): int(roffs[q + 1])], want), q
    # the same lists as a hybrid index: bitmaps are built by decoding patched lists
    hx = gpu.Index(np.concatenate(streams), soffs, universe=1 << 20, bitmap_gap=64)
    assert hx.bitmap_lists > 0
    b2 = gpu.Batch(hx, terms, qoffs)
    b2.run()
    roffs2 = b2.res_offsets.cpu().numpy()
    res2 = b2.results.cpu().numpy().view(np.uint32)
    assert np.array_equal(roffs2, roffs) and np.array_equal(res2[: int(roffs[-1])], res[: int(roffs[-1])])


@pytest.mark.parametrize("mode", [oracle.D4, oracle.D1])
def test_bulk_workload_patched_single_launch(gpu, mode):
    """The bulk workload at full size as S4-FastPFOR, decoded by the
    single-launch plan; every value compared with the generated lists."""
    import torch
    flat, offs, kinds = workloads.bulk_lists()
    buf, soffs = gpu.encode_many(flat, offs, delta=mode, patched=True)
    lists = [gpu.DeviceList.upload(buf[int(soffs[i]): int(soffs[i + 1])]) for i in range(len(offs) - 1)]
    out = torch.empty(int(offs[-1]) + 128 * len(lists), dtype=torch.int32, device="cuda")
    outs, pos, p = [], [], 0
    for l in lists:
        outs.append(out[p: p + l.n + 4])
        pos.append(p)
        p += (l.n + 63) // 64 * 64 + 64
    plan = gpu.DecodePlan(lists, outs)
    plan.run()
    torch.cuda.synchronize()
    host = out.cpu().numpy().view(np.uint32)
    for i, l in enumerate(lists):
        assert np.array_equal(host[pos[i]: pos[i] + l.n], flat[int(offs[i]): int(offs[i + 1])]), i


@pytest.mark.parametrize("passes", [1, 2, 4])
def test_mixed_plan_patched_and_plain(gpu, passes):
    """A single-launch plan holding patched and plain lists in every form
    runs the kernel instantiated for patched lists, which decodes its plain
    lists with pipelined rows too; every value compared, at 1, 2 and 4
    passes per wave, with edge lengths (tail only, one block, ragged)."""
    import torch
    lens = [1, 127, 128, 129, 1000, 4096 + 5, 128 * 37, 70001, (1 << 18) + 3]
    xs, lists = [], []
    for i, n in enumerate(lens * 2):
        x = with_outliers(300 + i, n) if i % 2 == 0 else workloads.sorted_list(i % 2, 400 + i, 1 << 26, n)
        xs.append(x)
        lists.append(gpu.DeviceList.upload(gpu.encode(x, FORMS[i % 4], patched=(i % 3 != 1))))
    patched = [(l.flags >> 3) & 1 for l in lists]
    assert any(patched) and not all(patched)
    pos, p = [], 0
    for x in xs:
        pos.append(p)
        p += (x.size + 63) // 64 * 64 + 64
    out = torch.full((p,), -1, dtype=torch.int32, device="cuda")
    outs = [out[q: q + x.size + 4] for q, x in zip(pos, xs)]
    t = gpu.get_tuning()
    try:
        gpu.set_tuning(**{**t.as_dict(), "decode_passes": passes})
        plan = gpu.DecodePlan(lists, outs)
        plan.run()
        torch.cuda.synchronize()
    finally:
        gpu.set_tuning(**t.as_dict())
    host = out.cpu().numpy().view(np.uint32)
    for i, x in enumerate(xs):
        assert np.array_equal(host[pos[i]: pos[i] + x.size], x), (i, lens[i % len(lens)])
