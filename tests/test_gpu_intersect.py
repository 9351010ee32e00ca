"""GPU intersection parity against the oracle's two-pointer merge."""
import itertools
import sys

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def dev(s4, x):
    return s4.DeviceList.upload(s4.encode(np.asarray(x, np.uint32)))


def gpu_pair(s4, a, b):
    out, cnt = s4.intersect(dev(s4, a), dev(s4, b))
    c = int(cnt.item())
    return out[:c].cpu().numpy().view(np.uint32)


def test_plain_pair(gpu):
    a, b = workloads.plain_pair()
    got = gpu_pair(gpu, a, b)
    assert np.array_equal(got, oracle.intersect(a, b))


@pytest.mark.parametrize("ratio", [1, 2, 4, 16, 64, 256, 1024, 4096])
@pytest.mark.parametrize("frac", [1 / 3, 0.01])
@pytest.mark.parametrize("kind", [workloads.CLUSTERED, workloads.UNIFORM])
def test_ratio_sweep(gpu, ratio, frac, kind):
    n = 1 << 18
    m = max(1, n // ratio)
    log(f"pair ratio={ratio} frac={frac:.3f} kind={kind}")
    r, f = workloads.planted_pair(1000 + ratio, n, m, frac, kind=kind)
    want = oracle.intersect(r, f)
    assert np.array_equal(gpu_pair(gpu, r, f), want)
    assert np.array_equal(gpu_pair(gpu, f, r), want)


def test_edge_pairs(gpu):
    rng = np.random.default_rng(2)
    base = workloads.sorted_list(workloads.UNIFORM, 8, 1 << 22, 5000)
    cases = [
        (np.zeros(0, np.uint32), base),
        (base, np.zeros(0, np.uint32)),
        (base, base),
        (base[:1], base),
        (base[-1:], base),
        (base[:127], base[100:]),
        (base[::2], base[1::2]),                              # interleaved, disjoint
        (base[:2000], base[3000:]),                           # disjoint ranges
        (np.array([0, 2**32 - 1], np.uint32), np.array([0, 5, 2**32 - 1], np.uint32)),
        # full blocks, then a raw tail ending at the largest value: the key
        # 2^32 - 1 found there, and 2^32 - 2 (below the list's maximum) not
        (np.array([base[7], 2**32 - 1], np.uint32), np.append(base[:300], np.uint32(2**32 - 1))),
        (np.array([base[7], 2**32 - 2], np.uint32), np.append(base[:300], np.uint32(2**32 - 1))),
        (np.append(base[250:300], np.uint32(2**32 - 1)), np.append(base[:300:2], np.uint32(2**32 - 1))),
        # full blocks only, the last one ending at the largest value; and a
        # raw tail below a key of 2^32 - 1 (the key lies past the list)
        (np.array([base[3], 2**32 - 1], np.uint32), np.append(base[:255], np.uint32(2**32 - 1))),
        (np.array([base[3], 2**32 - 2], np.uint32), np.append(base[:255], np.uint32(2**32 - 1))),
        (np.array([base[299], 2**32 - 1], np.uint32), base[:300]),
        (base + np.uint32(1 << 30), base),
        (np.arange(0, 3000, 3, dtype=np.uint32), np.arange(0, 3000, 2, dtype=np.uint32)),
        (rng.choice(base, 300, replace=False), base),
    ]
    for a, b in cases:
        a = np.unique(a).astype(np.uint32)
        b = np.unique(b).astype(np.uint32)
        assert np.array_equal(gpu_pair(gpu, a, b), oracle.intersect(a, b))


@pytest.mark.parametrize("gallop", [1, 2, 8, 64, 512])
@pytest.mark.parametrize("waves", [1, 2, 4, 8])
def test_result_independent_of_tuning(gpu, gallop, waves):
    old = gpu.get_tuning().as_dict()
    try:
        gpu.set_tuning(gallop_blocks=gallop, waves_per_group=waves)
        for ratio in (1, 50, 3000):
            r, f = workloads.planted_pair(77 + ratio, 1 << 17, (1 << 17) // ratio, 0.3)
            assert np.array_equal(gpu_pair(gpu, r, f), oracle.intersect(r, f))
    finally:
        gpu.set_tuning(**old)


def test_unsorted_flag_rejected(gpu):
    dup = gpu.DeviceList.upload(gpu.encode(np.array([1, 1, 2, 3], np.uint32)))
    ok = dev(gpu, np.array([1, 2], np.uint32))
    with pytest.raises(gpu.S4Error) as e:
        gpu.intersect(dup, ok)
    assert e.value.code == gpu.EUNSORTED


def test_small_cap_rejected(gpu):
    import torch
    a = dev(gpu, np.arange(0, 1000, dtype=np.uint32))
    b = dev(gpu, np.arange(0, 2000, 2, dtype=np.uint32))
    with pytest.raises(gpu.S4Error) as e:
        gpu.intersect(a, b, out=torch.zeros(999, dtype=torch.int32, device="cuda"))
    assert e.value.code == gpu.ERANGE


def kway_lists(seed, k, base_n=40000):
    rng = np.random.default_rng(seed)
    common = workloads.sorted_list(workloads.CLUSTERED, seed, 1 << 24, 3000)
    out = []
    for i in range(k):
        n = int(base_n * rng.uniform(0.05, 1.0))
        x = workloads.sorted_list(workloads.CLUSTERED, seed * 31 + i, 1 << 24, n)
        keep = rng.random(common.size) < 0.8
        out.append(np.union1d(x, common[keep]).astype(np.uint32))
    return out


@pytest.mark.parametrize("k", [2, 3, 4])
def test_kway_all_orders(gpu, k):
    lists = kway_lists(10 + k, k)
    want = oracle.intersect_k(lists)
    devs = [dev(gpu, x) for x in lists]
    for perm in itertools.permutations(range(k)):
        out, cnt = gpu.intersect_k([devs[i] for i in perm])
        c = int(cnt.item())
        assert np.array_equal(out[:c].cpu().numpy().view(np.uint32), want), perm


@pytest.mark.parametrize("k", [1, 5, 8])
def test_kway_lengths(gpu, k):
    lists = kway_lists(50 + k, k)
    want = oracle.intersect_k(lists)
    out, cnt = gpu.intersect_k([dev(gpu, x) for x in lists])
    c = int(cnt.item())
    assert np.array_equal(out[:c].cpu().numpy().view(np.uint32), want)


def test_kway_with_empty_and_self(gpu):
    lists = kway_lists(3, 3)
    d = [dev(gpu, x) for x in lists]
    empty = dev(gpu, np.zeros(0, np.uint32))
    out, cnt = gpu.intersect_k(d + [empty])
    assert int(cnt.item()) == 0
    out, cnt = gpu.intersect_k([d[0], d[0], d[0]])
    c = int(cnt.item())
    assert np.array_equal(out[:c].cpu().numpy().view(np.uint32), lists[0])
    with pytest.raises(gpu.S4Error):
        gpu.intersect_k([])


def test_raw_side(gpu):
    import torch
    r, f = workloads.planted_pair(5, 1 << 18, 5000, 0.3)
    rt = torch.from_numpy(r.view(np.int32)).cuda()
    ln = torch.tensor([r.size], dtype=torch.int64, device="cuda")
    out, cnt = gpu.intersect_raw(rt, ln, r.size + 300, dev(gpu, f))
    c = int(cnt.item())
    assert np.array_equal(out[:c].cpu().numpy().view(np.uint32), oracle.intersect(r, f))


def test_single_launch_many_chunks(gpu):
    """One launch, far more chunks than resident waves (2^22 values in the
    shortest list: 32768 chunks): every chunk's offset comes from the
    look-back; results equal the merge."""
    n = 1 << 22
    log("single launch: shortest 2^22")
    a = workloads.sorted_list(workloads.CLUSTERED, 77, 1 << 26, n)
    b = workloads.sorted_list(workloads.CLUSTERED, 78, 1 << 26, n + 12345)
    la, lb = dev(gpu, a), dev(gpu, b)
    out, cnt = gpu.intersect(la, lb)
    c = int(cnt.item())
    assert c != 2**64 - 1 and c < 2**63
    assert np.array_equal(out[:c].cpu().numpy().view(np.uint32), oracle.intersect(a, b))
    # self-intersection: every chunk survives whole
    out, cnt = gpu.intersect(la, la)
    assert int(cnt.item()) == n
    assert np.array_equal(out[:n].cpu().numpy().view(np.uint32), a)


def test_scratch_reused_across_calls(gpu):
    """Calls of different sizes back to back on one scratch buffer, never
    cleared: each call's scan words carry their own epoch, so counts left
    by earlier calls are never read."""
    import torch
    rng = np.random.default_rng(9)
    big = workloads.sorted_list(workloads.UNIFORM, 80, 1 << 24, 1 << 19)
    lbig = dev(gpu, big)
    scratch = torch.zeros(gpu.intersect_k_scratch_bytes([lbig, lbig]) + 4096, dtype=torch.uint8, device="cuda")
    out = torch.empty(1 << 19, dtype=torch.int32, device="cuda")
    cnts = [torch.zeros(1, dtype=torch.int64, device="cuda") for _ in range(12)]
    cases = []
    for i, m in enumerate([1 << 19, 1000, 129, 1 << 17, 1, 5000, 1 << 19, 128, 70000, 3, 1 << 18, 777]):
        r = np.sort(rng.choice(big, size=min(m, big.size), replace=False)).astype(np.uint32) if i % 2 else \
            workloads.sorted_list(workloads.UNIFORM, 90 + i, 1 << 24, m)
        cases.append((r, dev(gpu, r)))
    res = []
    for (r, lr), c in zip(cases, cnts):
        gpu.intersect_k([lr, lbig], out=out, count=c, scratch=scratch)
        k = int(c.item())
        res.append(out[:k].cpu().numpy().view(np.uint32).copy())
    for (r, _), got in zip(cases, res):
        assert np.array_equal(got, oracle.intersect(r, big))
