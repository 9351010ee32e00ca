"""s4_intersect_k_noalloc (scratch from the library's static device array,
no allocation) against s4_intersect_k on the same inputs: two calls in a
row, the second smaller, and a rejection beyond the array's capacity."""
import sys

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def dev(s4, x, mode=None):
    return s4.DeviceList.upload(s4.encode(np.asarray(x, np.uint32)) if mode is None else
                                s4.encode(np.asarray(x, np.uint32), mode))


def both(s4, lists):
    """(no-alloc result, allocating result), both through the C ABI."""
    out1, c1 = s4.intersect_k_noalloc(lists)
    n1 = int(c1.item())
    out2, c2 = s4.intersect_k(lists)
    n2 = int(c2.item())
    return out1[:n1].cpu().numpy().view(np.uint32), out2[:n2].cpu().numpy().view(np.uint32)


def test_noalloc_matches_intersect_k(gpu):
    gpu.init()
    big = [workloads.sorted_list(workloads.CLUSTERED, 500 + i, 1 << 24, (1 << 20) + 1000 * i) for i in range(3)]
    small = [workloads.sorted_list(workloads.UNIFORM, 600 + i, 1 << 16, 3000 + 17 * i) for i in range(3)]
    # first call: a 3-term query whose shortest list has 2^20 values
    log("noalloc call 1: 3 terms, shortest 2^20")
    lb = [dev(gpu, x) for x in big]
    got, ref = both(gpu, lb)
    assert np.array_equal(got, ref)
    assert np.array_equal(got, oracle.intersect_k(big))
    # second call, smaller: the same array holds the first call's words
    log("noalloc call 2: 3 terms, shortest 3000")
    ls = [dev(gpu, x, oracle.D1) for x in small]
    got2, ref2 = both(gpu, ls)
    assert np.array_equal(got2, ref2)
    assert np.array_equal(got2, oracle.intersect_k(small))
    # pairwise and k = 1 through the same entry point
    got3, ref3 = both(gpu, [ls[0], lb[1]])
    assert np.array_equal(got3, ref3)
    got4, ref4 = both(gpu, [ls[2]])
    assert np.array_equal(got4, ref4) and np.array_equal(got4, small[2])


def test_noalloc_rejects_beyond_capacity(gpu):
    m = gpu.intersect_k_noalloc_max_len()
    assert m == 33550336
    x = workloads.sorted_list(workloads.UNIFORM, 700, 1 << 27, m + 1)
    lx = dev(gpu, x)
    with pytest.raises(gpu.S4Error) as e:
        gpu.intersect_k_noalloc([lx, lx])
    assert e.value.code == gpu.ERANGE
