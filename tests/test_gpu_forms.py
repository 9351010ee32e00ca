"""GPU parity for the D1, D2 and DM differential forms (Sec. 5) beside D4:
decode, skip index, random block access, intersections mixing forms."""
import sys

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu
FORMS = [oracle.D4, oracle.DM, oracle.D2, oracle.D1]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def synthetic_stream(mode, widths, rng, tail=()):
    import struct
    nb = len(widths)
    pw = 4 * sum(widths)
    n = 128 * nb + len(tail)
    hdr = struct.pack("<IHHQIIQ", oracle.MAGIC, 1, mode << 1, n, nb, len(tail), pw)
    wb = bytes(widths) + b"\0" * (((nb + 3) & ~3) - nb)
    payload = rng.integers(0, 2**32, size=pw, dtype=np.uint64).astype(np.uint32).tobytes()
    tl = np.array(tail, np.uint32).tobytes()
    return np.frombuffer(hdr + wb + payload + tl, np.uint8).copy()


@pytest.mark.parametrize("mode", FORMS)
@pytest.mark.parametrize("n", [1, 5, 127, 128, 129, 513, 2049, (1 << 20) + 37])
def test_decode_forms(gpu, mode, n):
    x = workloads.sorted_list(workloads.CLUSTERED, 600 + n, 1 << 26, n)
    enc = oracle.encode(x, mode)
    lst = gpu.DeviceList.upload(enc)
    got = lst.decode().cpu().numpy().view(np.uint32)
    assert np.array_equal(got, oracle.decode(enc))


@pytest.mark.parametrize("mode", FORMS)
def test_decode_forms_arbitrary_payload(gpu, mode):
    rng = np.random.default_rng(mode)
    widths = [int(w) for w in rng.permutation(np.repeat(np.arange(33), 5))]
    enc = synthetic_stream(mode, widths, rng, tail=[3, 1, 4, 1, 5])
    lst = gpu.DeviceList.upload(enc)
    got = lst.decode().cpu().numpy().view(np.uint32)
    assert np.array_equal(got, oracle.decode(enc))
    bmax, seeds = lst.skip_index()
    ref = oracle.decode(enc)
    nb = len(widths)
    assert np.array_equal(bmax, ref[127: 128 * nb: 128])
    for k in range(1, nb):
        assert list(seeds[k]) == list(ref[128 * k - 4: 128 * k]), k


@pytest.mark.parametrize("mode", FORMS)
def test_decode_blocks_forms(gpu, mode):
    import torch
    x = workloads.sorted_list(workloads.UNIFORM, 92, 1 << 26, 128 * 300 + 9)
    enc = oracle.encode(x, mode)
    ref = oracle.decode(enc)
    lst = gpu.DeviceList.upload(enc)
    rng = np.random.default_rng(mode)
    for _ in range(10):
        first = int(rng.integers(0, lst.nb + 1))
        count = int(rng.integers(1, lst.nb + 2 - first))
        out = torch.zeros(128 * count, dtype=torch.int32, device="cuda")
        lst.decode_blocks_into(first, count, out)
        want = ref[128 * first: 128 * (first + count)]
        assert np.array_equal(out.cpu().numpy().view(np.uint32)[: want.size], want)


@pytest.mark.parametrize("ratio", [1, 16, 512])
def test_intersect_mixed_forms(gpu, ratio):
    n = 1 << 17
    r, f = workloads.planted_pair(70 + ratio, n, n // ratio, 0.3)
    want = oracle.intersect(r, f)
    for mr in FORMS:
        for mf in FORMS:
            a = gpu.DeviceList.upload(gpu.encode(r, mr))
            b = gpu.DeviceList.upload(gpu.encode(f, mf))
            out, cnt = gpu.intersect(a, b)
            c = int(cnt.item())
            assert np.array_equal(out[:c].cpu().numpy().view(np.uint32), want), (mr, mf)


def test_batch_mixed_form_index(gpu):
    lens = workloads.index_lengths(1 << 10, 16)
    kinds = np.full(lens.size, workloads.CLUSTERED, dtype=np.int32)
    flat, offs = workloads.lists(kinds, lens, 313, 1 << 20)
    # list t uses form t mod 4
    streams = [gpu.encode(flat[int(offs[t]): int(offs[t + 1])], t % 4) for t in range(lens.size)]
    soffs = np.zeros(lens.size + 1, np.uint64)
    np.cumsum([s.size for s in streams], out=soffs[1:])
    ix = gpu.Index(np.concatenate(streams), soffs)
    terms, qoffs = workloads.queries(17, ix.lengths, 700, 1, 6)
    b = gpu.Batch(ix, terms, qoffs)
    b.run()
    roffs = b.res_offsets.cpu().numpy()
    res = b.results.cpu().numpy().view(np.uint32)
    for q in range(700):
        ts = terms[int(qoffs[q]): int(qoffs[q + 1])]
        want = oracle.intersect_k([flat[int(offs[t]): int(offs[t + 1])] for t in ts])
        assert np.array_equal(res[int(roffs[q]): int(roffs[q + 1])], want), q


@pytest.mark.parametrize("mode", [oracle.DM, oracle.D2, oracle.D1])
def test_bulk_workload_forms_single_launch(gpu, mode):
    """The bulk workload at full size in each other form, decoded by the
    single-launch plan; every value compared with the generated lists."""
    import torch
    flat, offs, kinds = workloads.bulk_lists()
    buf, soffs = gpu.encode_many(flat, offs, delta=mode)
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
