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
