"""Per-list decode through the library's own dispatch queue: every list
decoded exactly as its input (and as the oracle decodes its stream), in one
and in several steps, with ragged, tail-only, empty and multi-pass lists."""
import sys

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build(gpu, specs):
    import torch
    xs, lists = [], []
    for i, (n, mode) in enumerate(specs):
        kind = workloads.CLUSTERED if i % 2 else workloads.UNIFORM
        x = workloads.sorted_list(kind, 600 + i, 1 << 26, n) if n else np.zeros(0, np.uint32)
        xs.append(x)
        lists.append(gpu.DeviceList.upload(gpu.encode(x, mode)))
    pos, p = [], 0
    for x in xs:
        pos.append(p)
        p += (x.size + 63) // 64 * 64 + 64
    out = torch.full((p,), -1, dtype=torch.int32, device="cuda")
    outs = [out[q: q + max(x.size, 1) + 4] for q, x in zip(pos, xs)]
    return xs, lists, out, outs, pos


def check(out, xs, pos):
    host = out.cpu().numpy().view(np.uint32)
    for i, x in enumerate(xs):
        assert np.array_equal(host[pos[i]: pos[i] + x.size], x), i
        # nothing written past the list's end
        assert (host[pos[i] + x.size: pos[i] + x.size + 4] == 0xFFFFFFFF).all(), i


def test_aql_decode_matches_inputs(gpu):
    specs = [(0, oracle.D4), (1, oracle.D4), (127, oracle.D1), (128, oracle.D4), (129, oracle.D1),
             (5000, oracle.D4), (70001, oracle.D1), ((1 << 21) + 5, oracle.D4), ((1 << 22) + 77, oracle.D1)]
    log("building", [n for n, _ in specs])
    xs, lists, out, outs, pos = build(gpu, specs)
    plan = gpu.AqlDecodePlan(lists, outs)
    log("one step")
    ms = plan.run(1)
    assert ms > 0
    check(out, xs, pos)
    assert np.array_equal(out.cpu().numpy().view(np.uint32)[pos[6]: pos[6] + xs[6].size],
                          oracle.decode(gpu.encode(xs[6], oracle.D1)))
    out.fill_(-1)
    log("three steps")
    plan.run(3)
    check(out, xs, pos)


def test_aql_plan_rejects_patched_lists(gpu):
    import torch
    x = workloads.sorted_list(workloads.CLUSTERED, 7, 1 << 26, 3000)
    lst = gpu.DeviceList.upload(gpu.encode(x, oracle.D4, patched=True))
    out = torch.empty(3000 + 4, dtype=torch.int32, device="cuda")
    with pytest.raises(gpu.S4Error) as e:
        gpu.AqlDecodePlan([lst], [out])
    assert e.value.code == gpu.EINVAL
