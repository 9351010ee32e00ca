"""GPU decode parity: the HIP decode of every stream equals the oracle's
decode of the same list, bit for bit."""
import struct
import sys

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def gpu_decode(s4, enc):
    lst = s4.DeviceList.upload(enc)
    out = lst.decode()
    return out.cpu().numpy().view(np.uint32), lst


@pytest.mark.parametrize("n", [0, 1, 3, 4, 5, 127, 128, 129, 255, 256, 511, 512, 513, 2047, 2048, 2049,
                               (1 << 20) + 37])
@pytest.mark.parametrize("kind", [workloads.UNIFORM, workloads.CLUSTERED])
def test_decode_edge_lengths(gpu, n, kind):
    log(f"decode edge n={n} kind={kind}")
    x = workloads.sorted_list(kind, 500 + n, 1 << 26, n)
    enc = oracle.encode(x)
    got, lst = gpu_decode(gpu, enc)
    assert got.size == n
    assert np.array_equal(got, oracle.decode(enc))


def test_decode_plain_pair(gpu):
    a, b = workloads.plain_pair()
    for x in (a, b):
        enc = gpu.encode(x)
        got, _ = gpu_decode(gpu, enc)
        assert np.array_equal(got, oracle.decode(oracle.encode(x)))


def synthetic_stream(widths, rng, tail=()):
    nb = len(widths)
    pw = 4 * sum(widths)
    n = 128 * nb + len(tail)
    hdr = struct.pack("<IHHQIIQ", oracle.MAGIC, 1, 0, n, nb, len(tail), pw)
    wb = bytes(widths) + b"\0" * (((nb + 3) & ~3) - nb)
    payload = rng.integers(0, 2**32, size=pw, dtype=np.uint64).astype(np.uint32).tobytes()
    tl = np.array(tail, np.uint32).tobytes()
    return np.frombuffer(hdr + wb + payload + tl, np.uint8).copy()


@pytest.mark.parametrize("seed", range(3))
def test_decode_arbitrary_payload_every_width(gpu, seed):
    """Random payload bits at every width 0..32 in mixed order (sums wrap
    modulo 2^32): unpack and scan must agree with the oracle exactly."""
    rng = np.random.default_rng(seed)
    widths = list(rng.permutation(np.repeat(np.arange(33), 7)))
    enc = synthetic_stream([int(w) for w in widths], rng, tail=list(range(seed * 40)))
    got, _ = gpu_decode(gpu, enc)
    assert np.array_equal(got, oracle.decode(enc))


def test_skip_index_matches_oracle(gpu):
    x = workloads.sorted_list(workloads.CLUSTERED, 77, 1 << 26, 128 * 300 + 17)
    enc = oracle.encode(x)
    lst = gpu.DeviceList.upload(enc)
    bmax, seeds = lst.skip_index()
    ref = oracle.decode(enc)
    nb = ref.size // 128
    assert np.array_equal(bmax, ref[127: 128 * nb: 128])
    want = np.zeros((nb, 4), np.uint32)
    for k in range(1, nb):
        want[k] = ref[128 * k - 4: 128 * k]
    assert np.array_equal(seeds, want)


def test_decode_blocks_random_access(gpu):
    import torch
    x = workloads.sorted_list(workloads.UNIFORM, 91, 1 << 26, 128 * 1000 + 50)
    enc = oracle.encode(x)
    ref = oracle.decode(enc)
    lst = gpu.DeviceList.upload(enc)
    rng = np.random.default_rng(4)
    for _ in range(20):
        first = int(rng.integers(0, lst.nb + 1))
        count = int(rng.integers(1, lst.nb + 2 - first))
        out = torch.zeros(128 * count, dtype=torch.int32, device="cuda")
        lst.decode_blocks_into(first, count, out)
        got = out.cpu().numpy().view(np.uint32)
        want = ref[128 * first: 128 * first + 128 * count]
        assert np.array_equal(got[: want.size], want), (first, count)
    with pytest.raises(gpu.S4Error):
        lst.decode_blocks_into(lst.nb, 2, out)


def test_decode_rejects_small_or_misaligned(gpu):
    import torch
    x = workloads.sorted_list(workloads.UNIFORM, 5, 1 << 20, 1000)
    lst = gpu.DeviceList.upload(oracle.encode(x))
    small = torch.zeros(999, dtype=torch.int32, device="cuda")
    with pytest.raises(gpu.S4Error) as e:
        lst.decode_into(small)
    assert e.value.code == gpu.ERANGE
    big = torch.zeros(1010, dtype=torch.int32, device="cuda")
    with pytest.raises(gpu.S4Error) as e:
        lst.decode_into(big[1:])
    assert e.value.code == gpu.EINVAL


def test_upload_rejects_corrupt(gpu):
    x = workloads.sorted_list(workloads.UNIFORM, 6, 1 << 20, 1000)
    enc = oracle.encode(x)
    bad = enc.copy()
    bad[0] ^= 0xFF
    with pytest.raises(gpu.S4Error) as e:
        gpu.DeviceList.upload(bad)
    assert e.value.code == gpu.ECORRUPT


def test_bulk_workload_full_size(gpu):
    """The bulk-decode workload at full size (256 lists, 2^12..2^24
    integers), one launch per list as timed by the benchmark; every decoded
    value is compared with the generated list, whose oracle round trip is
    pinned separately, and a sample of lists with the oracle's decode."""
    import torch
    flat, offs, kinds = workloads.bulk_lists()
    log(f"bulk lists: {offs[-1]} integers")
    buf, soffs = gpu.encode_many(flat, offs)
    lists = [gpu.DeviceList.upload(buf[int(soffs[i]): int(soffs[i + 1])]) for i in range(len(offs) - 1)]
    out = torch.empty(int(offs[-1]) + 16 * len(lists), dtype=torch.int32, device="cuda")
    pos = []
    p = 0
    for l in lists:
        pos.append(p)
        l.decode_into(out[p: p + l.n + 4] if l.n else out[p: p + 4])
        p += (l.n + 3) // 4 * 4 + 4
    torch.cuda.synchronize()
    host = out.cpu().numpy().view(np.uint32)
    rng = np.random.default_rng(0)
    sample = set(rng.choice(len(lists), size=6, replace=False).tolist())
    for i, l in enumerate(lists):
        x = flat[int(offs[i]): int(offs[i + 1])]
        got = host[pos[i]: pos[i] + l.n]
        assert np.array_equal(got, x), i
        if i in sample:
            assert np.array_equal(got, oracle.decode(oracle.encode(x))), i


def test_decode_timed_matches_and_times(gpu):
    import torch
    x = workloads.sorted_list(workloads.CLUSTERED, 12, 1 << 26, (1 << 20) + 3)
    enc = oracle.encode(x)
    lst = gpu.DeviceList.upload(enc)
    out = torch.zeros(x.size + 4, dtype=torch.int32, device="cuda")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    e1.record()
    lst.decode_timed_into(out, e0, e1)
    torch.cuda.synchronize()
    assert e0.elapsed_time(e1) > 0
    assert np.array_equal(out[: x.size].cpu().numpy().view(np.uint32), oracle.decode(enc))


def _stream_lists(gpu):
    """Lists of 0 .. 2^18 + 77 integers in every differential form, every
    third one patched."""
    rng = np.random.default_rng(31)
    lens = [0, 1, 127, 128, 129, 4096, 70001, (1 << 18) + 77] + [int(2 ** u) for u in rng.uniform(0, 18, size=28)]
    xs, lists = [], []
    for i, n in enumerate(lens):
        x = workloads.sorted_list(i % 2, 900 + i, 1 << 26, n)
        xs.append(x)
        lists.append(gpu.DeviceList.upload(gpu.encode(x, i % 4, patched=(i % 3 == 0))))
    return xs, lists


@pytest.mark.parametrize("nstreams", [1, 8])
def test_decode_lists_streams_and_graph(gpu, nstreams):
    """One launch per list over forked streams: every list decoded exactly,
    nothing written outside [0, n) of its output, eagerly and in each of
    three replays of a captured graph with host checks and refills between
    them."""
    import torch
    xs, lists = _stream_lists(gpu)
    log(f"decode_lists nstreams={nstreams}: {len(lists)} lists, {sum(x.size for x in xs)} integers")
    pos, p = [], 0
    for x in xs:
        pos.append(p)
        p += (x.size + 63) // 64 * 64 + 64
    buf = torch.empty(p, dtype=torch.int32, device="cuda")
    outs = [buf[q: q + x.size + 4] for q, x in zip(pos, xs)]
    sentinel = -0x5A5A5A5B

    def check(tag):
        host = buf.cpu().numpy().view(np.uint32)
        mask = np.ones(host.size, dtype=bool)
        for i, x in enumerate(xs):
            assert np.array_equal(host[pos[i]: pos[i] + x.size], x), (tag, i)
            mask[pos[i]: pos[i] + x.size] = False
        assert np.all(host[mask] == np.uint32(sentinel & 0xFFFFFFFF)), tag

    buf.fill_(sentinel)
    gpu.decode_lists(lists, outs, nstreams=nstreams)
    torch.cuda.synchronize()
    check("eager")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        gpu.decode_lists(lists, outs, nstreams=nstreams)
    torch.cuda.synchronize()
    for r in range(3):
        buf.fill_(sentinel)
        torch.cuda.synchronize()
        with torch.cuda.stream(side):
            g.replay()
        torch.cuda.synchronize()
        check(f"replay {r}")


def test_decode_lists_bulk_workload_graph(gpu):
    """The bulk workload at full size exactly as the benchmark times it: one
    launch per list over 8 forked streams, captured once and replayed; every
    value of every replay compared with the generated lists."""
    import torch
    flat, offs, kinds = workloads.bulk_lists()
    buf, soffs = gpu.encode_many(flat, offs)
    lists = [gpu.DeviceList.upload(buf[int(soffs[i]): int(soffs[i + 1])]) for i in range(len(offs) - 1)]
    out = torch.empty(int(offs[-1]) + 128 * len(lists), dtype=torch.int32, device="cuda")
    outs, pos, p = [], [], 0
    for l in lists:
        outs.append(out[p: p + l.n + 4])
        pos.append(p)
        p += (l.n + 63) // 64 * 64 + 64
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        gpu.decode_lists(lists, outs, nstreams=8)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        gpu.decode_lists(lists, outs, nstreams=8)
    for r in range(2):
        out.zero_()
        torch.cuda.synchronize()
        with torch.cuda.stream(side):
            g.replay()
        torch.cuda.synchronize()
        host = out.cpu().numpy().view(np.uint32)
        log(f"bulk graph replay {r} copied back")
        for i, l in enumerate(lists):
            assert np.array_equal(host[pos[i]: pos[i] + l.n], flat[int(offs[i]): int(offs[i + 1])]), (r, i)


def test_decode_lists_rejects_other_stream_counts(gpu):
    xs, lists = _stream_lists(gpu)
    import torch
    outs = [torch.empty(x.size + 4, dtype=torch.int32, device="cuda") for x in xs]
    for bad in (0, 2, 4, 9):
        with pytest.raises(gpu.S4Error) as e:
            gpu.decode_lists(lists, outs, nstreams=bad)
        assert e.value.code == gpu.EINVAL
