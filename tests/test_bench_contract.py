"""The benchmark script's host-side contract: it refuses more than one GPU
with a message, and its CPU baseline (the oracle's decode, timed) reports
what it measured and on which host."""
import json
import os
import subprocess
import sys

import numpy as np

import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert p.returncode == 2
    line = json.loads(p.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_cpu_baseline_fields():
    sys.path.insert(0, ROOT)
    import bench
    lens = np.array([300, 4096, 129], np.uint64)
    kinds = np.array([workloads.UNIFORM, workloads.CLUSTERED, workloads.UNIFORM], np.int32)
    flat, offs = workloads.lists(kinds, lens, 5, 1 << 20)
    cb = bench.cpu_baseline(flat, offs, 1)
    assert cb["unit"] == "Gint/s" and cb["kind"] == "oracle"
    assert cb["value"] > 0 and cb["single_thread_value"] > 0 and cb["cores"] >= 1
    assert str(int(offs[-1])) in cb["sample"]
    host = cb["host"]
    assert host["nproc"] >= 1 and set(host) == {"cpu_model", "nproc", "usable_threads"}


def test_cpu_queries_fields():
    """The oracle's queries/s baseline decodes and intersects every sampled
    query; the result total equals the plain fold on the raw lists."""
    sys.path.insert(0, ROOT)
    import bench
    import oracle
    lens = np.array([5000, 3000, 700, 129, 4096], np.uint64)
    kinds = np.full(lens.size, workloads.CLUSTERED, np.int32)
    flat, offs = workloads.lists(kinds, lens, 11, 1 << 16)
    encs = [oracle.encode(flat[int(offs[i]): int(offs[i + 1])]) for i in range(lens.size)]
    terms, qoffs = workloads.queries(3, lens, 40, 2, 4)
    cb = bench.cpu_queries(encs, terms, qoffs, np.arange(40))
    assert cb["unit"] == "queries/s" and cb["kind"] == "oracle" and cb["value"] > 0 and cb["cores"] >= 1
    want = sum(oracle.intersect_k([flat[int(offs[t]): int(offs[t + 1])] for t in terms[int(qoffs[q]): int(qoffs[q + 1])]]).size
               for q in range(40))
    assert cb["results"] == want
