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


def test_aql_new_plan_after_free_sees_new_lists(gpu):
    """A plan and its lists freed, other lists uploaded (often at the freed
    addresses) and a new plan built: the new run must decode the new inputs,
    not stale cached arguments or payload (every run opens with a
    system-scope acquire)."""
    import gc
    for round_ in range(3):
        specs = [((1 << 16) + 37 * round_, oracle.D4), (5000 + round_, oracle.D1), (129, oracle.D4),
                 ((1 << 19) + 11 * round_, oracle.D4)]
        log("round", round_, [n for n, _ in specs])
        # different seeds each round: different values at possibly reused addresses
        import torch
        xs, lists = [], []
        for i, (n, mode) in enumerate(specs):
            kind = workloads.CLUSTERED if (i + round_) % 2 else workloads.UNIFORM
            x = workloads.sorted_list(kind, 9000 + 17 * round_ + i, 1 << 26, n)
            xs.append(x)
            lists.append(gpu.DeviceList.upload(gpu.encode(x, mode)))
        pos, p = [], 0
        for x in xs:
            pos.append(p)
            p += (x.size + 63) // 64 * 64 + 64
        out = torch.full((p,), -1, dtype=torch.int32, device="cuda")
        outs = [out[q: q + x.size + 4] for q, x in zip(pos, xs)]
        plan = gpu.AqlDecodePlan(lists, outs)
        plan.run(2)
        check(out, xs, pos)
        del plan, lists, outs, out
        gc.collect()


def test_aql_enqueue_is_stream_ordered(gpu):
    """enqueue(): the run starts after the stream's earlier work (a fill of
    the outputs) and the stream's later work (a copy of the outputs) sees
    its results; the caller never synchronises in between."""
    import torch
    specs = [((1 << 20) + 3, oracle.D4), (70001, oracle.D1), (128, oracle.D4), (0, oracle.D4)]
    xs, lists, out, outs, pos = build(gpu, specs)
    plan = gpu.AqlDecodePlan(lists, outs)
    s = torch.cuda.Stream()
    copy = torch.empty_like(out)
    with torch.cuda.stream(s):
        for rep in range(3):
            out.fill_(-1)
            gpu.spin(2_000_000)  # the fill stays in flight while the call returns
            plan.enqueue(2)
            copy.copy_(out)
    s.synchronize()
    plan.status()
    check(copy, xs, pos)


def test_aql_profile_reports_every_dispatch(gpu):
    specs = [(0, oracle.D4), (1, oracle.D4), (5000, oracle.D4), ((1 << 21) + 5, oracle.D4),
             ((1 << 22) + 77, oracle.D1), (127, oracle.D1)]
    xs, lists, out, outs, pos = build(gpu, specs)
    plan = gpu.AqlDecodePlan(lists, outs)
    st, en, ms = plan.profile(2)
    check(out, xs, pos)
    assert st.shape == (2, len(specs))
    for s in range(2):
        for i, x in enumerate(xs):
            if x.size == 0:
                assert st[s, i] == 0 and en[s, i] == 0
            else:
                assert en[s, i] > st[s, i], (s, i)
    # step 1 starts after step 0 has ended on every queue
    live = [i for i, x in enumerate(xs) if x.size]
    assert st[1, live].min() >= en[0, live].max()
    # the device span fits in the host's wall time of the run
    assert (en.max() - st[0, live].min()) / 1e6 <= ms * 1.05 + 0.05
