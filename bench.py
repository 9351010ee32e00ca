#!/usr/bin/env python3
"""Benchmark of the S4-BP128-D4 decode + intersection engine on one MI355X.

Headline workload (bulk decode): 256 lists, lengths floor(2^u), u ~ U[12, 24],
universe [0, 2^26), even lists uniform and odd lists clustered, encoded as
S4-BP128-D4 and resident in HBM; one step decodes every list with one
kernel launch per list, each a dispatch packet the library writes into one of
its four HSA queues (s4_aql_plan; steps separated by barrier packets).
value = decoded integers per second (Gint/s), end to end.  The same
launches through HIP (forked streams, the step replayed as one hipGraph) are
reported beside it.

Also reported:
  roofline      the decode kernel's algorithmic bytes (width bytes + packed
                payload + raw tail read, 4 bytes per integer written) over its
                average launch duration, measured with HIP events around each
                launch on its own stream, against 8 TB/s HBM peak;
  single_launch the same lists decoded by one multi-list launch;
  batched       two-term and multi-term query batches (one persistent
                decode-fused launch) against the plain one-launch-per-query
                path, with p50 / p99 query latency;
  cpu_baseline  the oracle's decode timed on the host cores.

Prints one JSON line.  --gpus N with N > 1 exits: the engine runs on one GPU
(sharding by document-ID range across GPUs is a design, not code).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "decoded Gint/s; batched queries/s + p50/p99 vs plain path; % HBM peak"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--nstreams", type=int, default=8, choices=(1, 8))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--cpu-passes", type=int, default=16)
    ap.add_argument("--decode-only", action="store_true", help="skip the batched and CPU legs (for profiling)")
    ap.add_argument("--batched-only", action="store_true",
                    help="run only the batched leg and print its JSON (for profiling)")
    ap.add_argument("--no-aql", action="store_true",
                    help="time the per-list step through HIP only (for counter passes: the library's own queues "
                         "run launches concurrently, so counters cannot be read per dispatch there)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy 1 GiB three times with a plain copy kernel (counter calibration)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="turn rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE CSVs into profiles/decode_traffic.json")
    ap.add_argument("--serve", action="store_true",
                    help="run the serving workload instead (index of 2^20 lists, Poisson arrivals at 3 levels)")
    ap.add_argument("--serve-queries", type=int, default=1 << 20)
    ap.add_argument("--serve-lists", type=int, default=1 << 20)
    ap.add_argument("--serve-check", type=int, default=1 << 12,
                    help="queries per level checked against the oracle (0: none)")
    ap.add_argument("--calib-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="rocprofv3 CSVs of --calibrate-copy, for the counter scale factors")
    ap.add_argument("--batch-queries", type=int, default=1 << 18)
    ap.add_argument("--plain-sample", type=int, default=4096)
    return ap.parse_args()


def build_bulk(s4, workloads, torch):
    import numpy as np
    t0 = time.time()
    flat, offs, kinds = workloads.bulk_lists()
    buf, soffs = s4.encode_many(flat, offs)
    lists = [s4.DeviceList.upload(buf[int(soffs[i]): int(soffs[i + 1])]) for i in range(len(offs) - 1)]
    total = int(offs[-1])
    out = torch.empty(total + 128 * len(lists), dtype=torch.int32, device="cuda")
    # every list's output starts on a 256-byte boundary, so each 512-byte
    # block of output covers whole cache lines
    outs, p = [], 0
    for l in lists:
        outs.append(out[p: p + l.n + 4])
        p += (l.n + 63) // 64 * 64 + 64
    torch.cuda.synchronize()
    log(f"bulk workload: {len(lists)} lists, {total} ints, built in {time.time() - t0:.1f} s")
    return flat, offs, kinds, buf, soffs, lists, outs, out


def time_graph(torch, fn, stream, steps, warmup):
    """Capture fn() into a graph on `stream`; time `steps` replays."""
    with torch.cuda.stream(stream):
        fn()  # eager warm-up outside capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        fn()
    with torch.cuda.stream(stream):
        for _ in range(warmup):
            g.replay()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        e0.record()
        for _ in range(steps):
            g.replay()
        e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps, g


def time_graph_gated(torch, s4, g, stream, steps):
    """Replays of graph g timed on the device after a spin kernel has held
    the stream long enough for the host to queue all of them; also the
    host's wall time per replay launch, taken while the device is held."""
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        s4.spin(max(20_000_000, 3_000_000 * steps))
        e0.record()
        t0 = time.perf_counter()
        for _ in range(steps):
            g.replay()
        t1 = time.perf_counter()
        e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps, (t1 - t0) * 1e3 / steps


def per_launch_ms(torch, s4, lists, outs, stream, reps=3):
    """Duration of every decode launch, from HIP events on the launch stream
    that the launch itself records at the kernel's start and end
    (hipExtLaunchKernel); a clock-bounded spin kernel first holds the stream
    so the host has queued every launch before any runs."""
    import numpy as np
    acc = np.zeros(len(lists))
    for _ in range(reps):
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in lists]
        with torch.cuda.stream(stream):
            for a, b in evs:  # create the events
                a.record()
                b.record()
            torch.cuda.synchronize()
            s4.spin(40_000_000)
            for (a, b), l, o in zip(evs, lists, outs):
                l.decode_timed_into(o, a, b)
        torch.cuda.synchronize()
        acc += np.array([a.elapsed_time(b) for a, b in evs])
    return acc / reps


def cpu_baseline(flat, offs, passes):
    """The oracle's decode over the bulk lists, all host threads."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    import oracle

    threads = max(1, min(16, os.cpu_count() or 1))
    n = len(offs) - 1
    with ThreadPoolExecutor(threads) as ex:
        encs = list(ex.map(lambda i: oracle.encode(flat[int(offs[i]): int(offs[i + 1])]), range(n)))
    order = sorted(range(n), key=lambda i: -int(offs[i + 1] - offs[i]))
    done = 0
    t0, c0 = time.perf_counter(), time.process_time()
    for _ in range(passes):
        with ThreadPoolExecutor(threads) as ex:
            for r in ex.map(lambda i: oracle.decode(encs[i]).size, order):
                done += r
    dt, cpu = time.perf_counter() - t0, time.process_time() - c0
    # one thread, one pass over the same lists
    t1 = time.perf_counter()
    one = sum(oracle.decode(encs[i]).size for i in order)
    dt1 = time.perf_counter() - t1
    return {"value": round(done / dt / 1e9, 4), "unit": "Gint/s", "cores": threads, "kind": "oracle",
            "sample": f"oracle decode of all {n} bulk lists ({int(offs[-1])} ints), {passes} passes, "
                      f"{threads} threads, {dt:.1f} s wall, {cpu:.1f} s CPU",
            "single_thread_value": round(one / dt1 / 1e9, 4),
            "single_thread_sample": f"one pass over the same lists on one thread, {dt1:.1f} s",
            "host": host_info()}


def host_info():
    """CPU model and thread counts of the host the oracle ran on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_threads": aff}


def device_info(torch):
    """The GPU's properties as the runtime reports them."""
    p = torch.cuda.get_device_properties(0)
    return {"name": p.name, "arch": getattr(p, "gcnArchName", None), "compute_units": p.multi_processor_count,
            "l2_bytes": getattr(p, "L2_cache_size", None), "hbm_bytes": p.total_memory}


def copy_ceiling(torch, stream, reps=10):
    """Bandwidth of a plain device-to-device copy of 1 GiB (read + write
    bytes per second): what a kernel that only moves data reaches here."""
    n = (1 << 30) // 4
    a = torch.ones(n, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    with torch.cuda.stream(stream):
        for _ in range(2):
            b.copy_(a)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            b.copy_(a)
        e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    gbs = 2 * 4 * n / (ms / 1e3) / 1e9
    return {"gbs": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4), "bytes": 2 * 4 * n,
            "ms": round(ms, 4)}


def delta_forms(s4, torch, flat, offs, outs, stream, steps, warmup, patched=False):
    """The bulk workload in each differential form (Sec. 5), as S4-BP128 or,
    with patched, as S4-FastPFOR (Sec. 4.4): payload bits per integer and
    the single-launch decode rate (unpack, patch and prefix in one pass)."""
    import numpy as np
    res = {}
    for name, delta in (("D4", s4.DELTA_D4), ("DM", s4.DELTA_DM), ("D2", s4.DELTA_D2), ("D1", s4.DELTA_D1)):
        buf, soffs = s4.encode_many(flat, offs, delta=delta, patched=patched)
        lists = [s4.DeviceList.upload(buf[int(soffs[i]): int(soffs[i + 1])]) for i in range(len(offs) - 1)]
        n = float(sum(l.n for l in lists))
        pb = float(sum(l.payload_bytes for l in lists))
        plan = s4.DecodePlan(lists, outs)
        ms, _ = time_graph(torch, lambda: plan.run(), stream, steps, warmup)
        res[name] = {"bits_per_int": round(8 * pb / n, 3), "single_launch_gints": round(n / (ms / 1e3) / 1e9, 1),
                     "single_launch_frac": round((pb + 4 * n) / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
        del plan, lists
    return res


def batched(s4, workloads, torch, nq, plain_sample):
    """Batched pairwise / multi-term queries vs the plain per-query path."""
    import numpy as np
    out = {}
    t0 = time.time()
    flat, offs = workloads.pairwise_index()
    buf, soffs = s4.encode_many(flat, offs)
    index = s4.Index(buf, soffs)
    del flat
    log(f"index: {index.count} lists, {index.total_ints} ints, built in {time.time() - t0:.1f} s")
    dev = torch.cuda.current_device()
    for name, qfn in (("pairwise", workloads.pairwise_queries), ("multiterm", workloads.multiterm_queries)):
        terms, qoffs = qfn(index.lengths, nq)
        b = s4.Batch(index, terms, qoffs)
        best, tune_ms = b.autotune(reps=2)
        stream = torch.cuda.Stream()
        ms, _ = time_graph(torch, lambda: b.run(use_graph=False), stream, steps=5, warmup=2)
        ticks = b.query_ticks().astype(np.float64) / 100.0  # 100 MHz clock -> us
        abytes, ablocks = counted_traffic(b)
        # plain path: one intersect_k call per query, on a sample
        lists = [index.list(i) for i in range(index.count)] if name == "pairwise" else lists
        sample = np.arange(min(plain_sample, b.nq))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        lat = []
        scratch = torch.empty(1 << 26, dtype=torch.uint8, device="cuda")
        res = torch.empty(1 << 24, dtype=torch.int32, device="cuda")
        cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for q in sample:
            ts = terms[int(qoffs[q]): int(qoffs[q + 1])]
            s4.intersect_k([lists[t] for t in ts], out=res, count=cnt, scratch=scratch)
        torch.cuda.synchronize()
        plain_s = time.perf_counter() - t1
        for q in sample[:256]:
            ts = terms[int(qoffs[q]): int(qoffs[q + 1])]
            e0.record()
            s4.intersect_k([lists[t] for t in ts], out=res, count=cnt, scratch=scratch)
            e1.record()
            torch.cuda.synchronize()
            lat.append(e0.elapsed_time(e1) * 1e3)
        out[name] = {
            "queries": int(b.nq),
            "batched_qps": round(b.nq / (ms / 1e3), 1),
            "batched_ms": round(ms, 3),
            "batch_p50_us": round(float(np.percentile(ticks, 50)), 1),
            "batch_p99_us": round(float(np.percentile(ticks, 99)), 1),
            "plain_qps": round(sample.size / plain_s, 1),
            "plain_p50_us": round(float(np.percentile(lat, 50)), 1),
            "plain_p99_us": round(float(np.percentile(lat, 99)), 1),
            "speedup_vs_plain": round((b.nq / (ms / 1e3)) / (sample.size / plain_s), 2),
            "algorithmic_mb": round(abytes / 1e6, 2),
            "blocks_decoded": int(ablocks),
            "achieved_gbs": round(abytes / (ms / 1e3) / 1e9, 1),
            "hbm_frac": round(abytes / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
            "tuning": best,
        }
        log(f"{name}: {out[name]}")
        del b
    out["hybrid"] = hybrid(s4, workloads, torch, index, buf, soffs, nq, {k: out[k] for k in ("pairwise", "multiterm")})
    out["partitioned"] = partitioned(s4, workloads, torch, nq, {k: out[k] for k in ("pairwise", "multiterm")})
    out["fastpfor_index"] = fastpfor_index(s4, workloads, torch, nq, {k: out[k] for k in ("pairwise", "multiterm")})
    return out


def fastpfor_index(s4, workloads, torch, nq, plain):
    """The same index encoded as S4-FastPFOR-D1 (Sec. 4.4, patched blocks,
    the densest form) and the same queries, autotuned, replayed as a
    graph: storage against query time."""
    flat, offs = workloads.pairwise_index()
    buf, soffs = s4.encode_many(flat, offs, delta=s4.DELTA_D1, patched=True)
    ix = s4.Index(buf, soffs)
    del flat
    row = {"bits_per_int": round(8 * ix.payload_bytes / ix.total_ints, 3)}
    for name, qfn in (("pairwise", workloads.pairwise_queries), ("multiterm", workloads.multiterm_queries)):
        terms, qoffs = qfn(ix.lengths, nq)
        b = s4.Batch(ix, terms, qoffs)
        best, _ = b.autotune(reps=2)
        stream = torch.cuda.Stream()
        ms, _ = time_graph(torch, lambda: b.run(use_graph=False), stream, steps=5, warmup=2)
        row[f"{name}_qps"] = round(b.nq / (ms / 1e3), 1)
        row[f"{name}_ms"] = round(ms, 3)
        row[f"{name}_time_vs_s4bp128_d4"] = round(ms / plain[name]["batched_ms"], 3)
        del b
    log(f"S4-FastPFOR-D1 index: {row}")
    return row


def partitioned(s4, workloads, torch, nq, plain):
    """Doc-ID partitioned index (Sec. 7.7's partitioning, one part per XCD
    and finer): every list split by value range and each part encoded
    alone; a query runs part by part in each part's own length order, chunks
    queued per part and drained XCD-first.  Same queries, results identical
    to the unpartitioned batch (checked by the tests); each workload
    autotuned, replayed as a graph."""
    flat, offs = workloads.pairwise_index()
    res = {}
    for parts in (8, 16):
        sub = s4.partition_offsets(flat, offs, parts, 1 << 26)
        buf, soffs = s4.encode_many(flat, sub)
        ix = s4.Index(buf, soffs, parts=parts)
        row = {"bits_per_int": round(8 * ix.payload_bytes / ix.total_ints, 3)}
        for name, qfn in (("pairwise", workloads.pairwise_queries), ("multiterm", workloads.multiterm_queries)):
            terms, qoffs = qfn(ix.lengths, nq)
            b = s4.Batch(ix, terms, qoffs)
            best, _ = b.autotune(reps=2)
            stream = torch.cuda.Stream()
            ms, _ = time_graph(torch, lambda: b.run(use_graph=False), stream, steps=5, warmup=2)
            abytes, _ = counted_traffic(b)
            row[f"{name}_qps"] = round(b.nq / (ms / 1e3), 1)
            row[f"{name}_ms"] = round(ms, 3)
            row[f"{name}_algorithmic_mb"] = round(abytes / 1e6, 2)
            row[f"{name}_speedup_vs_one_part"] = round(plain[name]["batched_ms"] / ms, 3)
            row[f"{name}_tuning"] = best
            del b
        res[f"parts={parts}"] = row
        log(f"partitioned {parts}: {row}")
        del ix
    return res


def hybrid(s4, workloads, torch, index, buf, soffs, nq, plain):
    """hyb+m2 (Sec. 7.7): the same index and queries with the lists of
    average gap <= B held as bitmaps over [0, 2^26), B = 8, 16, 32; each
    index and workload autotuned on its own, replayed as a graph.
    Storage in bits/int counts packed payload + width bytes + tails +
    bitmaps (skip index and select samples apart)."""
    res = {"none": {"bitmap_lists": 0, "bits_per_int": round(8 * index.payload_bytes / index.total_ints, 3),
                    **{f"{k}_qps": plain[k]["batched_qps"] for k in plain}}}
    queries = {"pairwise": workloads.pairwise_queries(index.lengths, nq),
               "multiterm": workloads.multiterm_queries(index.lengths, nq)}
    for gap in (8, 16, 32):
        hx = s4.Index(buf, soffs, universe=1 << 26, bitmap_gap=gap)
        row = {"bitmap_lists": hx.bitmap_lists, "bitmap_mib": round(hx.bitmap_bytes / 2**20, 1),
               "bits_per_int": round(8 * hx.payload_bytes / hx.total_ints, 3)}
        for name, (terms, qoffs) in queries.items():
            b = s4.Batch(hx, terms, qoffs)
            b.autotune(reps=2)
            stream = torch.cuda.Stream()
            ms, _ = time_graph(torch, lambda: b.run(use_graph=False), stream, steps=5, warmup=2)
            abytes, _ = counted_traffic(b)
            row[f"{name}_qps"] = round(b.nq / (ms / 1e3), 1)
            row[f"{name}_ms"] = round(ms, 3)
            row[f"{name}_algorithmic_mb"] = round(abytes / 1e6, 2)
            row[f"{name}_speedup_vs_no_bitmaps"] = round(plain[name]["batched_ms"] / ms, 3)
            del b
        res[f"B={gap}"] = row
        log(f"hyb+m2 B={gap}: {row}")
        hx.free()
    return res


def run_steps(plan, steps):
    """Host wall time (ms) of `steps` per-list decodes on the library's
    queues, in runs of at most 64 steps."""
    t = 0.0
    while steps > 0:
        k = min(steps, 64)
        t += plan.run(k)
        steps -= k
    return t


def check_decoded(out, lists, flat, offs):
    """Every list's decoded values equal its input (outputs laid out as
    build_bulk lays them out)."""
    import numpy as np
    host = out.cpu().numpy().view(np.uint32)
    p = 0
    for i, l in enumerate(lists):
        if not np.array_equal(host[p: p + l.n], flat[int(offs[i]): int(offs[i + 1])]):
            raise SystemExit(f"decoded list {i} differs from its input")
        p += (l.n + 63) // 64 * 64 + 64


def counted_traffic(b):
    """Algorithmic traffic of one extra, untimed run with counting on (the
    timed runs leave it off: it slows the chunk kernels by 4-15%)."""
    b.set_counting(True)
    b.run(use_graph=False)
    out = b.traffic()
    b.set_counting(False)
    return out


def kernel_source_sha():
    import hashlib
    h = hashlib.sha256()
    for f in ("s4_kernels.h", "s4_device.hip"):
        with open(os.path.join(ROOT, "paper_1401_6399_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def pmc_values(path, kernel_substr, counter):
    import csv
    out = []
    with open(path) as f:
        for r in csv.DictReader(f):
            if kernel_substr in r["Kernel_Name"] and r["Counter_Name"] == counter:
                out.append(float(r["Counter_Value"]))
    return out


def traffic_json(args):
    """Per-launch HBM traffic of the decode kernel from two counter passes,
    scaled by what the same counters read for a copy of 1 GiB."""
    import numpy as np
    one_gib_kib = float(1 << 20)
    cf = np.mean(pmc_values(args.calib_from[0], "copyBuffer", "FETCH_SIZE"))
    cw = np.mean(pmc_values(args.calib_from[1], "copyBuffer", "WRITE_SIZE"))
    sf, sw = one_gib_kib / cf, one_gib_kib / cw
    fetch = np.array(pmc_values(args.traffic_from[0], "k_decode<", "FETCH_SIZE"))
    write = np.array(pmc_values(args.traffic_from[1], "k_decode<", "WRITE_SIZE"))
    n = min(fetch.size, write.size)
    per_launch = float((fetch[:n].mean() * sf + write[:n].mean() * sw) * 1024.0)
    res = {"bytes_per_launch": round(per_launch, 1), "launches": int(n),
           "fetch_kib_per_launch": round(float(fetch[:n].mean()), 2),
           "write_kib_per_launch": round(float(write[:n].mean()), 2),
           "fetch_scale": round(float(sf), 4), "write_scale": round(float(sw), 4),
           "kernel_source_sha": kernel_source_sha()}
    path = os.path.join(ROOT, "profiles", "decode_traffic.json")
    with open(path, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res))


def calibrate_copy():
    import torch
    torch.cuda.set_device(0)
    n = (1 << 30) // 4
    a = torch.ones(n, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copied_bytes": 4 * n, "times": 3}))


def serving(args):
    """Serving workload: device-resident index of 2^20 clustered lists over
    [0, 2^31) (length max(128, 2^28 / (t + 1))), 2..8-term queries, open-loop
    Poisson arrivals at 0.5, 0.8 and 0.95 of the saturated rate."""
    import numpy as np
    import torch
    import workloads
    import paper_1401_6399_amd as s4

    s4.require_library()
    torch.cuda.set_device(0)
    t0 = time.time()
    nl = args.serve_lists
    lens = workloads.index_lengths(nl, 28 - (20 - nl.bit_length() + 1))
    kinds = np.full(nl, workloads.CLUSTERED, dtype=np.int32)
    flat, offs = workloads.lists(kinds, lens, workloads.config_seed(4, 0), 1 << 31)
    log(f"serving index: {nl} lists, {int(offs[-1])} ints generated in {time.time() - t0:.1f} s")
    buf, soffs = s4.encode_many(flat, offs)
    ix = s4.Index(buf, soffs)
    del buf, soffs
    log(f"index resident: {ix.payload_bytes / 2**30:.2f} GiB payload + {ix.index_bytes / 2**30:.2f} GiB skip "
        f"index, {8 * ix.payload_bytes / ix.total_ints:.2f} bits/int; built in {time.time() - t0:.1f} s")
    srv = s4.Server(ix, max_slots=1 << 15, pool_bytes=24 << 30, result_bytes=3 << 28, max_terms=8)
    nq = args.serve_queries
    terms, qoffs = workloads.serving_queries(ix.lengths, nq, level=0)
    sat = srv.replay(terms, qoffs, np.zeros(nq, np.uint64))
    qstar = nq / sat["elapsed_s"]
    log(f"saturated: {qstar:.0f} queries/s over {nq} queries")
    levels = []
    for lv, frac in enumerate((0.5, 0.8, 0.95)):
        terms, qoffs = workloads.serving_queries(ix.lengths, nq, level=lv + 1)
        arr = (workloads.arrivals(workloads.config_seed(4, 20 + lv), frac * qstar, nq) * 1e9).astype(np.uint64)
        chk = args.serve_check > 0
        r = srv.replay(terms, qoffs, arr, with_results=chk, results_cap=1 << 28)
        lat = r["latency_ns"].astype(np.float64) / 1e3
        span = (float(arr[-1]) / 1e9) if nq else 0.0
        lev = {"offered_qps": round(frac * qstar, 1), "achieved_qps": round(nq / max(r["elapsed_s"], 1e-9), 1),
               "queries": nq, "trace_s": round(span, 3),
               "p50_us": round(float(np.percentile(lat, 50)), 1), "p99_us": round(float(np.percentile(lat, 99)), 1),
               "p999_us": round(float(np.percentile(lat, 99.9)), 1)}
        if chk:
            import oracle
            rng = np.random.default_rng(lv)
            sample = rng.choice(nq, size=min(args.serve_check, nq), replace=False)
            bad = 0
            for q in sample:
                ts = sorted(terms[int(qoffs[q]): int(qoffs[q + 1])], key=lambda t: int(lens[t]))
                want = oracle.intersect_k([flat[int(offs[t]): int(offs[t + 1])] for t in ts])
                got = r["results"][int(r["res_offsets"][q]): int(r["res_offsets"][q + 1])]
                bad += not np.array_equal(got, want)
            lev["oracle_checked"] = int(sample.size)
            lev["oracle_mismatches"] = int(bad)
        levels.append(lev)
        log(f"level {lv}: {lev}")
    st = srv.stats()
    srv.close()
    print(json.dumps({"metric": "served queries/s + p50/p99/p999 latency", "unit": "queries/s",
                      "n_gpus": 1, "data": "synthetic",
                      "config": {"workload": f"serving: {nl} clustered lists over [0,2^31), "
                                             f"{int(offs[-1])} ints, 2..8-term queries, sqrt(len) term sampling, "
                                             "open-loop Poisson arrivals", "queries_per_level": nq},
                      "saturated_qps": round(qstar, 1), "levels": levels,
                      "index": {"payload_gib": round(ix.payload_bytes / 2**30, 3),
                                "skip_index_gib": round(ix.index_bytes / 2**30, 3),
                                "bits_per_int": round(8 * ix.payload_bytes / ix.total_ints, 3)},
                      "server_stats": st}), flush=True)


def main():
    args = parse()
    if args.serve:
        return serving(args)
    if args.traffic_from:
        return traffic_json(args)
    if args.calibrate_copy:
        return calibrate_copy()
    if args.gpus != 1:
        print(json.dumps({"error": "the engine runs on one GPU; sharding across GPUs (by document-ID range) "
                                   "is not implemented", "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch
    import workloads
    import paper_1401_6399_amd as s4

    s4.require_library()
    torch.cuda.set_device(0)
    if args.batched_only:
        print(json.dumps({"batched": batched(s4, workloads, torch, args.batch_queries, args.plain_sample)}),
              flush=True)
        return
    flat, offs, kinds, buf, soffs, lists, outs, out = build_bulk(s4, workloads, torch)
    ns = np.array([l.n for l in lists], dtype=np.float64)
    rbytes = np.array([l.payload_bytes for l in lists], dtype=np.float64)
    wbytes = 4.0 * ns
    abytes = rbytes + wbytes
    total = int(ns.sum())
    bits = float(rbytes.sum() * 8 / ns.sum())

    stream = torch.cuda.Stream()
    # headline: one launch per list, forked over streams, replayed as a graph
    torch.cuda.synchronize()
    graph_ms, g = time_graph(torch, lambda: s4.decode_lists(lists, outs, nstreams=args.nstreams), stream,
                             args.steps, args.warmup)
    log(f"per-list launches through HIP (graph): {graph_ms:.3f} ms/step, "
        f"{total / (graph_ms / 1e3) / 1e9:.1f} Gint/s")
    # diagnostic only (never `value`): the same replays with the stream held
    # until the host has queued them all, i.e. the device's time per step
    # when launching the 256-kernel graph does not limit it
    # (at most 30 replays queued at once, so the hardware queues never fill)
    gated_ms, host_ms = time_graph_gated(torch, s4, g, stream, min(args.steps, 30))
    log(f"per-list, device time with launches queued ahead: {gated_ms:.3f} ms/step; "
        f"host time to launch one replay: {host_ms:.3f} ms")

    # headline: the same launches written by the library into its own queues
    if args.no_aql:
        ms = graph_ms
        launch = f"one k_decode launch per list over {args.nstreams} forked streams, hipGraph replay"
    else:
        plan_q = s4.AqlDecodePlan(lists, outs)
        run_steps(plan_q, args.warmup)
        out.fill_(-1)
        ms = run_steps(plan_q, args.steps) / args.steps
        check_decoded(out, lists, flat, offs)
        del plan_q
        launch = ("one k_decode dispatch per list, written by the library into four HSA queues "
                  "(s4_aql_plan); steps separated by barrier packets")
    value = total / (ms / 1e3) / 1e9
    log(f"per-list launches ({launch}): {ms:.3f} ms/step, {value:.1f} Gint/s (outputs checked)")

    # roofline of the decode kernel: events around each launch
    dur = per_launch_ms(torch, s4, lists, outs, stream)
    achieved = abytes.sum() / (dur.sum() / 1e3) / 1e9
    big = ns >= (1 << 22)
    achieved_big = abytes[big].sum() / (dur[big].sum() / 1e3) / 1e9
    log(f"decode kernel: avg {dur.mean() * 1e3:.2f} us/launch, {achieved:.0f} GB/s; lists >= 2^22: "
        f"{achieved_big:.0f} GB/s")

    # single multi-list launch
    plan = s4.DecodePlan(lists, outs)
    ms1, _ = time_graph(torch, lambda: plan.run(), stream, args.steps, args.warmup)
    single = total / (ms1 / 1e3) / 1e9
    log(f"single launch: {ms1:.3f} ms/step, {single:.1f} Gint/s, {abytes.sum() / (ms1 / 1e3) / 1e9:.0f} GB/s")

    # correctness of the last decode timed (the single launch)
    check_decoded(out, lists, flat, offs)

    # counter-measured HBM bytes per launch, valid only for the kernel
    # source the counters were taken on
    traffic = None
    tf = os.path.join(ROOT, "profiles", "decode_traffic.json")
    if os.path.exists(tf):
        with open(tf) as f:
            tj = json.load(f)
        if tj.get("kernel_source_sha") == kernel_source_sha():
            traffic = tj.get("bytes_per_launch")

    result = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "Gint/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": "bulk decode: 256 S4-BP128-D4 lists, lengths floor(2^u) u~U[12,24], universe 2^26, "
                        "even lists uniform / odd clustered; one kernel launch per list",
            "lists": len(lists),
            "total_ints": total,
            "bits_per_int": round(bits, 3),
            "launch": launch,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "kernel": "k_decode",
            "avg_launch_us": round(float(dur.mean() * 1e3), 3),
            "bytes_per_launch": round(float(abytes.mean()), 1),
            "frac_lists_ge_2p22": round(achieved_big / HBM_PEAK_GBS, 4),
        },
        "per_list_hip_graph": {"ms_per_step": round(graph_ms, 4), "gint_s": round(total / (graph_ms / 1e3) / 1e9, 2),
                               "device_ms_per_step": round(gated_ms, 4),
                               "host_ms_per_launch_of_step": round(host_ms, 4),
                               "note": f"the same launches through HIP over {args.nstreams} forked streams, replayed "
                                       "as a hipGraph: end to end, and with the stream held until the host has "
                                       "queued every replay (the device's time per step)"},
        "single_launch": {"value": round(single, 2), "unit": "Gint/s", "ms_per_step": round(ms1, 4),
                          "frac": round(abytes.sum() / (ms1 / 1e3) / 1e9 / HBM_PEAK_GBS, 4)},
        "whole_job_hbm_frac": round(abytes.sum() / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
        "paper_context": "0.7 cycles/int, 5.4 Gint/s: Xeon E5-1620 3.6 GHz, 1 thread, cache-resident",
        "device": device_info(torch),
    }
    if not args.decode_only:
        cc = copy_ceiling(torch, stream)
        cc["decode_single_launch_vs_copy"] = round(abytes.sum() / (ms1 / 1e3) / 1e9 / cc["gbs"], 4)
        result["copy_ceiling"] = cc
        log(f"copy ceiling: {cc}")
    if not args.decode_only:
        result["delta_forms"] = delta_forms(s4, torch, flat, offs, outs, stream, 20, 3)
        log(f"delta forms: {result['delta_forms']}")
        result["fastpfor_forms"] = delta_forms(s4, torch, flat, offs, outs, stream, 20, 3, patched=True)
        log(f"S4-FastPFOR forms: {result['fastpfor_forms']}")
    if not args.no_batched and not args.decode_only:
        try:
            result["batched"] = batched(s4, workloads, torch, args.batch_queries, args.plain_sample)
        except Exception as ex:  # reported, never hidden
            result["batched"] = {"error": str(ex)}
    if not args.no_cpu_baseline and not args.decode_only:
        result["cpu_baseline"] = cpu_baseline(flat, offs, args.cpu_passes)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
