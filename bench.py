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
  roofline      the step's algorithmic bytes (width bytes + packed payload +
                raw tail read, 4 bytes per integer written) over its time in
                the timed run, against 8 TB/s HBM peak; beside it a profiled
                breakdown (device timestamp of every dispatch) and the same
                kernel launched serially through HIP;
  single_launch the same lists decoded by one multi-list launch;
  plain_config  the CPU-sized configuration (A = 2^20, B = 2^14): host
                encode, GPU decode and intersect, and the oracle on one thread;
  batched       two-term and multi-term query batches (one persistent
                decode-fused launch) against the plain path (one
                single-launch conjunction per query, submitted from C++),
                with the oracle's queries/s on a sample;
  cpu_baseline  the oracle's decode timed on the host cores;
  serving       the serving workload: sustained rate, three Poisson levels
                with latency percentiles, the plain path and the oracle
                beside each.

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
    ap.add_argument("--serve-lists", type=int, default=1 << 20)
    ap.add_argument("--serve-check", type=int, default=1 << 12,
                    help="queries per level checked against the oracle (0: none)")
    ap.add_argument("--calib-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="rocprofv3 CSVs of --calibrate-copy, for the counter scale factors")
    ap.add_argument("--batch-queries", type=int, default=1 << 18)
    ap.add_argument("--plain-sample", type=int, default=4096,
                    help="queries whose isolated latency the plain path measures")
    ap.add_argument("--cpu-queries", type=int, default=1 << 15,
                    help="sample of the batched workloads the oracle's queries/s is timed on")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving leg")
    ap.add_argument("--serve-level-s", type=float, default=30.0,
                    help="length of each Poisson level of the serving leg (at least 2^16 queries)")
    ap.add_argument("--serve-saturate", type=int, default=1 << 24,
                    help="queries submitted at once to measure the serving burst rate")
    ap.add_argument("--serve-saturate-s", type=float, default=30.0,
                    help="length of the overloaded open-loop trace that measures the sustained rate Q*")
    ap.add_argument("--serve-plain", type=int, default=1 << 14,
                    help="queries of each level's trace replayed through the plain path")
    ap.add_argument("--step-only", action="store_true",
                    help="only the headline's per-list steps on the library's queues (for rocprofv3)")
    ap.add_argument("--profile-steps", type=int, default=8,
                    help="untimed steps run with per-dispatch device timestamps for the roofline")
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


def cpu_queries(encs, terms, qoffs, sample):
    """The oracle's queries/s on a sample of a batch, all host threads:
    each query decodes its lists from their (oracle-encoded) streams and
    intersects them shortest first."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    threads = max(1, min(16, os.cpu_count() or 1))

    def one(q):
        ts = terms[int(qoffs[q]): int(qoffs[q + 1])]
        return oracle.intersect_k(sorted((oracle.decode(encs[t]) for t in ts), key=len)).size

    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        total = sum(ex.map(one, sample))
    dt = time.perf_counter() - t0
    return {"value": round(len(sample) / dt, 1), "unit": "queries/s", "cores": threads, "kind": "oracle",
            "sample": f"the first {len(sample)} queries: oracle decode of every term's list from its stream, "
                      f"then intersect_k (two-pointer merge, shortest first); {threads} threads, {dt:.2f} s",
            "results": int(total)}


def batched(s4, workloads, torch, nq, plain_sample, cpu_sample):
    """Batched pairwise / multi-term queries vs the plain per-query path."""
    import numpy as np
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    out = {}
    t0 = time.time()
    flat, offs = workloads.pairwise_index()
    buf, soffs = s4.encode_many(flat, offs)
    index = s4.Index(buf, soffs)
    log(f"index: {index.count} lists, {index.total_ints} ints, built in {time.time() - t0:.1f} s")
    # the oracle's own streams of every list (for its queries/s baseline)
    threads = max(1, min(16, os.cpu_count() or 1))
    with ThreadPoolExecutor(threads) as ex:
        encs = list(ex.map(lambda i: oracle.encode(flat[int(offs[i]): int(offs[i + 1])]), range(index.count)))
    del flat
    for name, qfn in (("pairwise", workloads.pairwise_queries), ("multiterm", workloads.multiterm_queries)):
        terms, qoffs = qfn(index.lengths, nq)
        b = s4.Batch(index, terms, qoffs)
        best, tune_ms = b.autotune(reps=2)
        stream = torch.cuda.Stream()
        ms, _ = time_graph(torch, lambda: b.run(use_graph=False), stream, steps=5, warmup=2)
        ticks = b.query_ticks().astype(np.float64) / 100.0  # 100 MHz clock -> us
        abytes, ablocks = counted_traffic(b)
        # plain path: every query its own single-launch conjunction, all of
        # them back to back from C++, then a sample one at a time
        pc, _, _, plain_ms, _ = s4.plain_run(index, terms, qoffs)
        same = bool(torch.equal(pc, b.counts[: b.nq]))
        ns_ = min(plain_sample, b.nq)
        _, _, _, _, lat = s4.plain_run(index, terms[: int(qoffs[ns_])], qoffs[: ns_ + 1], isolate=True)
        lat = lat.astype(np.float64) / 1e3
        cpu = cpu_queries(encs, terms, qoffs, np.arange(min(cpu_sample, b.nq)))
        out[name] = {
            "queries": int(b.nq),
            "batched_qps": round(b.nq / (ms / 1e3), 1),
            "batched_ms": round(ms, 3),
            "batch_completion_p50_us": round(float(np.percentile(ticks, 50)), 1),
            "batch_completion_p99_us": round(float(np.percentile(ticks, 99)), 1),
            "plain_qps": round(b.nq / (plain_ms / 1e3), 1),
            "plain_ms": round(plain_ms, 2),
            "plain_isolated_p50_us": round(float(np.percentile(lat, 50)), 1),
            "plain_isolated_p99_us": round(float(np.percentile(lat, 99)), 1),
            "plain_counts_match_batch": same,
            "speedup_vs_plain": round(plain_ms / ms, 2),
            "algorithmic_mb": round(abytes / 1e6, 2),
            "blocks_decoded": int(ablocks),
            "achieved_gbs": round(abytes / (ms / 1e3) / 1e9, 1),
            "hbm_frac": round(abytes / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
            "tuning": best,
            "cpu_baseline": cpu,
            "note": "batch_completion_*: when each query's last chunk finished inside the batch, from the batch's "
                    "start; plain_isolated_*: one query launched and waited for alone (launch to completion); "
                    "plain_qps: all queries, one launch each, submitted back to back from C++",
        }
        log(f"{name}: {out[name]}")
        del b
    del encs
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
    bitmaps (skip index and select samples apart).  Besides the sqrt(length)
    queries, a second set draws terms with probability proportional to
    length (2^14 pairs, 2^16 queries of 3..6 terms), so that the dense
    lists, which the bitmaps replace, take part in many queries; each
    index's counts are checked equal to the compressed index's."""
    import numpy as np

    def timed(ix, terms, qoffs):
        b = s4.Batch(ix, terms, qoffs)
        b.autotune(reps=2)
        stream = torch.cuda.Stream()
        ms, _ = time_graph(torch, lambda: b.run(use_graph=False), stream, steps=5, warmup=2)
        abytes, _ = counted_traffic(b)
        counts = b.counts[: b.nq].clone()
        del b
        return ms, abytes, counts

    queries = {"pairwise": workloads.pairwise_queries(index.lengths, nq),
               "multiterm": workloads.multiterm_queries(index.lengths, nq)}
    dense = {"pairwise_by_length": workloads.length_weighted_queries(workloads.config_seed(2, 7), index.lengths,
                                                                     1 << 14, 2, 2),
             "multiterm_by_length": workloads.length_weighted_queries(workloads.config_seed(3, 7), index.lengths,
                                                                      1 << 16, 3, 6)}
    base = {}
    res = {"none": {"bitmap_lists": 0, "bits_per_int": round(8 * index.payload_bytes / index.total_ints, 3),
                    **{f"{k}_qps": plain[k]["batched_qps"] for k in plain}}}
    for name, (terms, qoffs) in dense.items():
        ms, abytes, counts = timed(index, terms, qoffs)
        base[name] = (ms, counts)
        nqd = int(qoffs.size - 1)
        res["none"][f"{name}_queries"] = nqd
        res["none"][f"{name}_qps"] = round(nqd / (ms / 1e3), 1)
        res["none"][f"{name}_ms"] = round(ms, 3)
        res["none"][f"{name}_algorithmic_mb"] = round(abytes / 1e6, 2)
    log(f"hyb+m2 none: {res['none']}")
    for gap in (8, 16, 32):
        hx = s4.Index(buf, soffs, universe=1 << 26, bitmap_gap=gap)
        row = {"bitmap_lists": hx.bitmap_lists, "bitmap_mib": round(hx.bitmap_bytes / 2**20, 1),
               "bits_per_int": round(8 * hx.payload_bytes / hx.total_ints, 3)}
        for name, (terms, qoffs) in {**queries, **dense}.items():
            ms, abytes, counts = timed(hx, terms, qoffs)
            ref_ms = plain[name]["batched_ms"] if name in plain else base[name][0]
            row[f"{name}_qps"] = round(int(qoffs.size - 1) / (ms / 1e3), 1)
            row[f"{name}_ms"] = round(ms, 3)
            row[f"{name}_algorithmic_mb"] = round(abytes / 1e6, 2)
            row[f"{name}_speedup_vs_no_bitmaps"] = round(ref_ms / ms, 3)
            if name in base:
                row[f"{name}_counts_match_no_bitmaps"] = bool(torch.equal(counts, base[name][1]))
        res[f"B={gap}"] = row
        log(f"hyb+m2 B={gap}: {row}")
        hx.free()
    frac = {}
    for name, (terms, qoffs) in {**queries, **dense}.items():
        lens = np.asarray(index.lengths, dtype=np.float64)
        ql = np.maximum.reduceat(lens[terms], qoffs[:-1].astype(np.int64))
        frac[name] = {f"B={g}": round(float(np.mean(ql * g >= float(1 << 26))), 4) for g in (8, 16, 32)}
    res["queries_with_a_bitmap_list"] = frac
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


def pct(x, q):
    import numpy as np
    return round(float(np.percentile(x, q)), 1) if len(x) else None


def serving_leg(s4, workloads, torch, args):
    """Serving workload: device-resident index of 2^20 clustered lists over
    [0, 2^31) (length max(128, 2^28 / (t + 1))), 2..8-term queries.  The
    saturated rate Q* (every query of a long trace submitted at once), then
    open-loop Poisson arrivals at 0.5, 0.8 and 0.95 Q*, each level lasting
    at least --serve-level-s seconds and 2^16 queries; latency percentiles
    from arrival to result; the plain path (one single-launch conjunction
    per query, submitted from C++) replaying the first --serve-plain
    arrivals of the same trace; a sample of each level's results checked
    against the oracle, whose own queries/s on that sample is timed on the
    host cores."""
    import numpy as np
    import oracle
    from concurrent.futures import ThreadPoolExecutor

    # the server's iterations launch with the library's default tuning, not
    # with whatever the batch legs' autotuning last set
    s4.set_tuning(**args.default_tuning)
    t0 = time.time()
    nl = args.serve_lists
    lens = workloads.index_lengths(nl, 28 - (20 - nl.bit_length() + 1))
    kinds = np.full(nl, workloads.CLUSTERED, dtype=np.int32)
    flat, offs = workloads.lists(kinds, lens, workloads.config_seed(4, 0), 1 << 31)
    log(f"serving index: {nl} lists, {int(offs[-1])} ints generated in {time.time() - t0:.1f} s")
    buf, soffs = s4.encode_many(flat, offs)
    ix = s4.Index(buf, soffs)
    del buf, soffs
    build_s = time.time() - t0
    log(f"index resident: {ix.payload_bytes / 2**30:.2f} GiB payload + {ix.index_bytes / 2**30:.2f} GiB skip "
        f"index, {8 * ix.payload_bytes / ix.total_ints:.2f} bits/int; built in {build_s:.1f} s")
    srv = s4.Server(ix, max_slots=1 << 15, pool_bytes=24 << 30, result_bytes=3 << 28, max_terms=8)
    # saturated rate: first every query of a trace submitted at once (a
    # burst), then an open-loop trace offered well above that rate (1.5x)
    # for --serve-saturate-s seconds, as long as a level: what the server
    # sustains under arrivals for that long is Q*, and the levels are
    # fractions of it
    nsat = args.serve_saturate
    terms, qoffs = workloads.serving_trace(ix.lengths, nsat, 0)
    sat = srv.replay(terms, qoffs, np.zeros(nsat, np.uint64))
    q_burst = nsat / sat["elapsed_s"]
    log(f"burst: {q_burst:.0f} queries/s over {nsat} queries")
    over = 1.5 * q_burst
    nov = max(1 << 16, int(over * args.serve_saturate_s))
    terms, qoffs = workloads.serving_trace(ix.lengths, nov, 9)
    arr = (workloads.arrivals(workloads.config_seed(4, 29), over, nov) * 1e9).astype(np.uint64)
    ov = srv.replay(terms, qoffs, arr, timeout_s=max(600.0, 8 * args.serve_saturate_s))
    qstar = nov / ov["elapsed_s"]
    log(f"sustained under {over:.0f}/s offered: {qstar:.0f} queries/s over {nov} queries")
    del terms, qoffs, arr, ov
    threads = max(1, min(16, os.cpu_count() or 1))

    def raw(t):
        return flat[int(offs[t]): int(offs[t + 1])]

    levels = []
    for lv, frac in ((1, 0.5), (2, 0.8), (3, 0.95)):
        rate = frac * qstar
        nq = max(1 << 16, int(np.ceil(rate * args.serve_level_s)))
        tg = time.time()
        terms, qoffs = workloads.serving_trace(ix.lengths, nq, lv)
        arr = (workloads.arrivals(workloads.config_seed(4, 20 + lv), rate, nq) * 1e9).astype(np.uint64)
        rng = np.random.default_rng(lv)
        sample = np.sort(rng.choice(nq, size=min(args.serve_check, nq), replace=False))
        keep = np.zeros(nq, np.uint8)
        keep[sample] = 1
        log(f"level {lv}: {nq} queries at {rate:.0f}/s generated in {time.time() - tg:.1f} s")
        r = srv.replay(terms, qoffs, arr, with_results=True, results_cap=1 << 27, keep=keep,
                       timeout_s=max(600.0, 4 * args.serve_level_s))
        lat = r["latency_ns"].astype(np.float64) / 1e3
        lev = {"offered_qps": round(rate, 1), "achieved_qps": round(nq / max(r["elapsed_s"], 1e-9), 1),
               "queries": nq, "trace_s": round(float(arr[-1]) / 1e9, 3), "elapsed_s": round(r["elapsed_s"], 3),
               "p50_us": pct(lat, 50), "p99_us": pct(lat, 99), "p999_us": pct(lat, 99.9)}
        del lat
        # the sample against the oracle, and the oracle's own rate on it
        qs = [sorted(terms[int(qoffs[q]): int(qoffs[q + 1])].tolist(), key=lambda t: int(lens[t])) for q in sample]
        tc = time.perf_counter()
        with ThreadPoolExecutor(threads) as ex:
            wants = list(ex.map(lambda ts: oracle.intersect_k([raw(t) for t in ts]), qs))
        cpu_s = time.perf_counter() - tc
        bad = 0
        for q, w in zip(sample, wants):
            got = r["results"][int(r["res_offsets"][q]): int(r["res_offsets"][q + 1])]
            bad += int(r["counts"][q]) != w.size or not np.array_equal(got, w)
        lev["oracle_checked"] = int(sample.size)
        lev["oracle_mismatches"] = int(bad)
        lev["cpu_baseline"] = {"value": round(sample.size / cpu_s, 1), "unit": "queries/s", "cores": threads,
                               "kind": "oracle",
                               "sample": f"oracle intersect_k (two-pointer merge, shortest first) of the "
                                         f"{sample.size} checked queries over their uncompressed lists "
                                         f"(decoding not counted), {threads} threads, {cpu_s:.2f} s"}
        # the plain path under the first arrivals of the same trace
        npl = min(args.serve_plain, nq)
        pl = s4.plain_replay(ix, terms[: int(qoffs[npl])], qoffs[: npl + 1], arr[:npl],
                             timeout_s=max(600.0, 4 * args.serve_level_s))
        plat = pl["latency_ns"].astype(np.float64) / 1e3
        lev["plain"] = {"queries": npl, "offered_qps": round(rate, 1),
                        "achieved_qps": round(npl / max(pl["elapsed_s"], 1e-9), 1),
                        "p50_us": pct(plat, 50), "p99_us": pct(plat, 99), "p999_us": pct(plat, 99.9),
                        "counts_match_server": bool(np.array_equal(pl["counts"], r["counts"][:npl]))}
        levels.append(lev)
        log(f"level {lv}: {lev}")
        del terms, qoffs, arr, r, keep, pl
    st = srv.stats()
    srv.close()
    out = {"workload": f"serving: {nl} clustered lists over [0,2^31), {int(offs[-1])} ints resident, 2..8-term "
                       "queries, sqrt(len) term sampling, open-loop Poisson arrivals at 0.5/0.8/0.95 Q*",
           "unit": "queries/s", "saturated_qps": round(qstar, 1),
           "saturated": {"qps": round(qstar, 1), "offered_qps": round(over, 1), "queries": nov,
                         "burst_qps": round(q_burst, 1), "burst_queries": nsat,
                         "note": "Q* is what the server sustains under open-loop arrivals offered at 1.5x the rate "
                                 "of a burst (every query of a trace submitted at once); the levels are fractions "
                                 "of Q*"},
           "levels": levels,
           "tuning": s4.get_tuning().as_dict(),
           "index": {"payload_gib": round(ix.payload_bytes / 2**30, 3),
                     "skip_index_gib": round(ix.index_bytes / 2**30, 3),
                     "bits_per_int": round(8 * ix.payload_bytes / ix.total_ints, 3), "build_s": round(build_s, 1)},
           "server_stats": st}
    ix.free()
    return out


def serving(args):
    """--serve: the serving leg alone, printed as its own JSON line."""
    import torch
    import workloads
    import paper_1401_6399_amd as s4

    s4.require_library()
    args.default_tuning = s4.get_tuning().as_dict()
    torch.cuda.set_device(0)
    res = serving_leg(s4, workloads, torch, args)
    print(json.dumps({"metric": "served queries/s + p50/p99/p999 latency", "n_gpus": 1, "data": "synthetic",
                      "serving": res}), flush=True)


def step_profile(plan_q, ns, abytes, steps):
    """Device timestamps of every dispatch in `steps` untimed per-list steps
    on the library's queues (HSA dispatch profiling): per step, its device
    span (first start to last end), the summed kernel time, and bytes over
    span for each class of list length; medians over the steps."""
    import numpy as np
    st, en, host_ms = plan_q.profile(steps)
    st = st.astype(np.float64)
    en = en.astype(np.float64)
    live = ns > 0
    classes = {"lt_2p18": ns < 2**18, "2p18_to_2p22": (ns >= 2**18) & (ns < 2**22), "ge_2p22": ns >= 2**22}
    spans, ksums, durs = [], [], []
    per = {k: {"span": [], "dur": []} for k in classes}
    for i in range(steps):
        a, b = st[i, live], en[i, live]
        spans.append(b.max() - a.min())
        ksums.append((b - a).sum())
        durs.append((b - a).mean())
        for k, m in classes.items():
            mm = m & live
            if mm.any():
                per[k]["span"].append(en[i, mm].max() - st[i, mm].min())
                per[k]["dur"].append((en[i, mm] - st[i, mm]).mean())
    span_ns = float(np.median(spans))
    by = {}
    for k, m in classes.items():
        mm = m & live
        if not mm.any():
            continue
        sp = float(np.median(per[k]["span"]))
        by[k] = {"lists": int(mm.sum()), "bytes": round(float(abytes[mm].sum()), 1),
                 "span_us": round(sp / 1e3, 2), "avg_dispatch_us": round(float(np.median(per[k]["dur"])) / 1e3, 2),
                 "gbs_over_span": round(float(abytes[mm].sum()) / sp, 1)}
    return {"span_ns": span_ns, "kernel_sum_ns": float(np.median(ksums)), "avg_dispatch_ns": float(np.median(durs)),
            "host_ms": host_ms, "by_size_class": by, "spans_us": [round(x / 1e3, 2) for x in spans]}


def plain_config(s4, workloads, torch, reps=20):
    """The plain CPU-sized configuration: A = 2^20 and B = 2^14 values drawn
    uniformly from [0, 2^25); encode both (host library), decode both and
    intersect them on the GPU (kernel time from events on the stream, and
    end to end from the first launch to the synchronised result), every
    output checked against the oracle; beside it the oracle's encode, decode
    and merge on one host thread.  Medians."""
    import numpy as np
    import oracle
    a, b = workloads.plain_pair()
    med = lambda v: round(float(np.median(v)), 2)
    enc_us = []
    for _ in range(reps // 4):
        t0 = time.perf_counter()
        ea, eb = s4.encode(a), s4.encode(b)
        enc_us.append((time.perf_counter() - t0) * 1e6)
    la, lb = s4.DeviceList.upload(ea), s4.DeviceList.upload(eb)
    oa = torch.empty(a.size + 4, dtype=torch.int32, device="cuda")
    ob = torch.empty(b.size + 4, dtype=torch.int32, device="cuda")
    res = torch.empty(b.size, dtype=torch.int32, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    scratch = torch.empty(max(256, s4.intersect_k_scratch_bytes([la, lb])), dtype=torch.uint8, device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    dec_a, dec_b, inter, e2e = [], [], [], []
    for i in range(reps + 3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev[0].record()
        la.decode_into(oa)
        ev[1].record()
        lb.decode_into(ob)
        ev[2].record()
        s4.intersect(la, lb, out=res, count=cnt, scratch=scratch)
        ev[3].record()
        ev[3].synchronize()
        t1 = time.perf_counter()
        if i >= 3:
            dec_a.append(ev[0].elapsed_time(ev[1]) * 1e3)
            dec_b.append(ev[1].elapsed_time(ev[2]) * 1e3)
            inter.append(ev[2].elapsed_time(ev[3]) * 1e3)
            e2e.append((t1 - t0) * 1e6)
    c = int(cnt.item())
    ok = (np.array_equal(oa[: a.size].cpu().numpy().view(np.uint32), a) and
          np.array_equal(ob[: b.size].cpu().numpy().view(np.uint32), b) and
          np.array_equal(res[:c].cpu().numpy().view(np.uint32), oracle.intersect(a, b)) and
          np.array_equal(ea, oracle.encode(a)) and np.array_equal(eb, oracle.encode(b)))
    # the oracle on one thread
    o_enc, o_dec, o_mrg = [], [], []
    for _ in range(5):
        t0 = time.perf_counter()
        xa, xb = oracle.encode(a), oracle.encode(b)
        t1 = time.perf_counter()
        da, db = oracle.decode(xa), oracle.decode(xb)
        t2 = time.perf_counter()
        oracle.intersect(da, db)
        t3 = time.perf_counter()
        o_enc.append((t1 - t0) * 1e6)
        o_dec.append((t2 - t1) * 1e6)
        o_mrg.append((t3 - t2) * 1e6)
    n = a.size + b.size
    return {"workload": "plain: A = 2^20, B = 2^14 distinct values uniform from [0, 2^25); S4-BP128-D4",
            "intersection": c, "bits_per_int_a": round(8 * la.payload_bytes / a.size, 3),
            "bits_per_int_b": round(8 * lb.payload_bytes / b.size, 3), "outputs_match_oracle": bool(ok),
            "gpu_us": {"host_encode_a_b": med(enc_us), "decode_a": med(dec_a), "decode_b": med(dec_b),
                       "intersect": med(inter), "decode_both_and_intersect_end_to_end": med(e2e)},
            "gpu_decode_gints": round(n / ((np.median(dec_a) + np.median(dec_b)) * 1e3), 2),
            "cpu_baseline": {"kind": "oracle", "cores": 1, "unit": "us",
                             "encode_a_b": med(o_enc), "decode_a_b": med(o_dec), "merge": med(o_mrg),
                             "decode_gints": round(n / (np.median(o_dec) * 1e3), 3),
                             "sample": "the whole plain workload, one host thread, median of 5"},
            "note": "fits in L2/MALL and is launch-bound: a correctness configuration, not a roofline one"}


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
    args.default_tuning = s4.get_tuning().as_dict()  # before any autotuning
    torch.cuda.set_device(0)
    if args.batched_only:
        print(json.dumps({"batched": batched(s4, workloads, torch, args.batch_queries, args.plain_sample,
                                             args.cpu_queries)}), flush=True)
        return
    flat, offs, kinds, buf, soffs, lists, outs, out = build_bulk(s4, workloads, torch)
    ns = np.array([l.n for l in lists], dtype=np.float64)
    rbytes = np.array([l.payload_bytes for l in lists], dtype=np.float64)
    wbytes = 4.0 * ns
    abytes = rbytes + wbytes
    total = int(ns.sum())
    bits = float(rbytes.sum() * 8 / ns.sum())
    launch = ("one k_decode dispatch per list, written by the library into four HSA queues "
              "(s4_aql_plan); steps separated by barrier packets")

    if args.step_only:
        # the headline's steps alone (what rocprofv3 traces for the roofline)
        plan_q = s4.AqlDecodePlan(lists, outs)
        run_steps(plan_q, args.warmup)
        ms = run_steps(plan_q, args.steps) / args.steps
        check_decoded(out, lists, flat, offs)
        line = {"ms_per_step": round(ms, 4), "gint_s": round(total / (ms / 1e3) / 1e9, 2),
                "dispatches_per_step": len(lists), "steps": args.warmup + args.steps}
        if args.profile_steps:
            prof = step_profile(plan_q, ns, abytes, args.profile_steps)
            line.update({"device_span_us": round(prof["span_ns"] / 1e3, 2),
                         "avg_dispatch_us": round(prof["avg_dispatch_ns"] / 1e3, 3),
                         "steps": args.warmup + args.steps + args.profile_steps,
                         "by_size_class": prof["by_size_class"]})
        print(json.dumps(line), flush=True)
        return

    stream = torch.cuda.Stream()
    # the same launches through HIP, forked over streams, replayed as a graph
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
    del g

    # headline: the launches written by the library into its own queues
    if args.no_aql:
        ms = graph_ms
        launch = f"one k_decode launch per list over {args.nstreams} forked streams, hipGraph replay"
        prof = None
    else:
        plan_q = s4.AqlDecodePlan(lists, outs)
        run_steps(plan_q, args.warmup)
        out.fill_(-1)
        torch.cuda.synchronize()
        ms = run_steps(plan_q, args.steps) / args.steps
        check_decoded(out, lists, flat, offs)
        # roofline of the timed mode: one more, untimed run with a device
        # timestamp on every dispatch
        prof = step_profile(plan_q, ns, abytes, args.profile_steps)
        check_decoded(out, lists, flat, offs)
        del plan_q
    value = total / (ms / 1e3) / 1e9
    log(f"per-list launches ({launch}): {ms:.3f} ms/step, {value:.1f} Gint/s (outputs checked)")

    # the kernel launched serially through HIP: events around each launch
    dur = per_launch_ms(torch, s4, lists, outs, stream)
    achieved_serial = abytes.sum() / (dur.sum() / 1e3) / 1e9
    big = ns >= (1 << 22)
    achieved_big = abytes[big].sum() / (dur[big].sum() / 1e3) / 1e9
    log(f"decode kernel, serial launches: avg {dur.mean() * 1e3:.2f} us/launch, {achieved_serial:.0f} GB/s; "
        f"lists >= 2^22: {achieved_big:.0f} GB/s")

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

    serial = {"achieved": round(achieved_serial, 1), "frac": round(achieved_serial / HBM_PEAK_GBS, 4),
              "avg_launch_us": round(float(dur.mean() * 1e3), 3), "bytes_per_launch": round(float(abytes.mean()), 1),
              "frac_lists_ge_2p22": round(achieved_big / HBM_PEAK_GBS, 4), "traffic_per_launch": traffic,
              "note": "the same kernel launched one list at a time through HIP, each launch timed by events it "
                      "records at its kernel's start and end"}
    if prof is not None:
        step_bytes = float(abytes.sum())
        # the timed run writes every step's packets ahead and returns when
        # the last step is complete, so its wall time per step is the
        # device's time per step
        achieved = step_bytes / (ms / 1e3) / 1e9
        roofline = {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": round(traffic * len(lists), 1) if traffic else None,
            "kernel": "k_decode",
            "unit_of_work": "one step of the headline: all 256 per-list dispatches on the library's four queues",
            "bytes_per_step": round(step_bytes, 1), "step_us": round(ms * 1e3, 2),
            "profiled": {
                "note": "untimed steps with a device timestamp on every dispatch (HSA dispatch profiling, which "
                        "slows a step by about 7%): the step's device span, the summed dispatch durations "
                        "(four queues run concurrently) and bytes over span per class of list length",
                "steps": args.profile_steps, "device_span_us": round(prof["span_ns"] / 1e3, 2),
                "kernel_time_sum_us": round(prof["kernel_sum_ns"] / 1e3, 2),
                "avg_dispatch_us": round(prof["avg_dispatch_ns"] / 1e3, 3), "dispatches_per_step": len(lists),
                "by_size_class": prof["by_size_class"],
                "host_ms_per_step": round(prof["host_ms"] / args.profile_steps, 4)},
            "serial": serial,
        }
    else:
        roofline = {"bound": "hbm", "achieved": serial["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": serial["frac"], "traffic": traffic, "kernel": "k_decode", "serial": serial}

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
        "roofline": roofline,
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
        result["plain_config"] = plain_config(s4, workloads, torch)
        log(f"plain config: {result['plain_config']}")
    if not args.no_batched and not args.decode_only:
        try:
            result["batched"] = batched(s4, workloads, torch, args.batch_queries, args.plain_sample,
                                        args.cpu_queries)
        except Exception as ex:  # reported, never hidden
            result["batched"] = {"error": str(ex)}
    if not args.no_cpu_baseline and not args.decode_only:
        result["cpu_baseline"] = cpu_baseline(flat, offs, args.cpu_passes)
    if not args.no_serving and not args.decode_only:
        del lists, outs, out
        torch.cuda.empty_cache()
        try:
            result["serving"] = serving_leg(s4, workloads, torch, args)
        except Exception as ex:  # reported, never hidden
            result["serving"] = {"error": str(ex)}
    print(json.dumps(result, default=float), flush=True)


if __name__ == "__main__":
    main()
