"""CPU-side checks of the C-ABI library: it loads, exports every declared
symbol, and its host encoder writes the same bytes as the oracle."""
import os
import re

import numpy as np
import pytest

import oracle
import workloads
import paper_1401_6399_amd as s4

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "s4.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(s4_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = s4.require_library()
    names = declared_functions()
    assert len(names) >= 30
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(s4.SIGNATURES), set(names) ^ set(s4.SIGNATURES)


@pytest.mark.parametrize("n", [0, 1, 3, 4, 5, 127, 128, 129, 2047, 2048, 2049, 65536 + 5])
@pytest.mark.parametrize("kind", [workloads.UNIFORM, workloads.CLUSTERED])
def test_encode_bytes_match_oracle(n, kind):
    x = workloads.sorted_list(kind, 300 + n, 1 << 26, n)
    assert np.array_equal(s4.encode(x), oracle.encode(x))


def test_encode_plain_pair_matches_oracle():
    a, b = workloads.plain_pair()
    assert np.array_equal(s4.encode(a), oracle.encode(a))
    assert np.array_equal(s4.encode(b), oracle.encode(b))


def test_encode_extreme_values_and_duplicates():
    xs = [np.array([0, 2**32 - 1] * 1, np.uint32),
          np.sort(np.random.default_rng(1).integers(0, 2**32, size=1000, dtype=np.uint64)).astype(np.uint32),
          np.repeat(np.arange(300, dtype=np.uint32), 3),
          np.full(1000, 7, np.uint32)]
    for x in xs:
        assert np.array_equal(s4.encode(x), oracle.encode(x))


def test_encode_many_matches_single():
    kinds, lens = workloads.bulk_lengths(16)
    lens = (lens // 64).astype(np.uint64)
    flat, offs = workloads.lists(kinds, lens, 99, 1 << 26)
    buf, soffs = s4.encode_many(flat, offs, nthreads=4)
    for i in range(len(lens)):
        x = flat[int(offs[i]): int(offs[i + 1])]
        assert np.array_equal(buf[int(soffs[i]): int(soffs[i + 1])], oracle.encode(x))


def test_encode_rejects_unsorted():
    with pytest.raises(s4.S4Error) as e:
        s4.encode(np.array([5, 4], np.uint32))
    assert e.value.code == s4.EUNSORTED


def test_decoded_length_rejects_corrupt():
    x = workloads.sorted_list(workloads.UNIFORM, 3, 1 << 20, 1000)
    enc = s4.encode(x)
    assert s4.decoded_length(enc) == 1000
    for bad in (enc[:-4], np.concatenate([enc, np.zeros(4, np.uint8)])):
        with pytest.raises(s4.S4Error) as e:
            s4.decoded_length(bad)
        assert e.value.code == s4.ECORRUPT
    bad = enc.copy()
    bad[32] = 40
    with pytest.raises(s4.S4Error):
        s4.decoded_length(bad)


def test_tuning_validation():
    t = s4.get_tuning()
    with pytest.raises(s4.S4Error):
        s4.set_tuning(gallop_blocks=0)
    with pytest.raises(s4.S4Error):
        s4.set_tuning(waves_per_group=3)
    s4.set_tuning(**t.as_dict())
    assert s4.get_tuning().as_dict() == t.as_dict()


@pytest.mark.parametrize("delta", [0, 1, 2, 3])
@pytest.mark.parametrize("n", [0, 5, 128, 129, 4097, 70001])
def test_encode_forms_match_oracle(delta, n):
    x = workloads.sorted_list(workloads.CLUSTERED, 400 + n, 1 << 26, n)
    assert np.array_equal(s4.encode(x, delta), oracle.encode(x, delta))


def test_encode_many_forms_match_oracle():
    kinds, lens = workloads.bulk_lengths(8)
    lens = (lens // 32).astype(np.uint64)
    flat, offs = workloads.lists(kinds, lens, 98, 1 << 26)
    for delta in range(4):
        buf, soffs = s4.encode_many(flat, offs, nthreads=3, delta=delta)
        for i in range(len(lens)):
            x = flat[int(offs[i]): int(offs[i + 1])]
            assert np.array_equal(buf[int(soffs[i]): int(soffs[i + 1])], oracle.encode(x, delta))


def _with_outliers(seed, n, universe=1 << 31):
    """Clustered-like gaps with sparse large jumps (exceptions at many
    widths), strictly increasing below the universe."""
    rng = np.random.default_rng(seed)
    gaps = rng.geometric(0.3, size=n).astype(np.uint64)
    k = max(1, n // 150)
    if n:
        gaps[rng.integers(0, n, size=k)] += (np.uint64(1) << rng.integers(4, 22, size=k).astype(np.uint64))
    x = np.cumsum(gaps)
    assert n == 0 or x[-1] < universe
    return x.astype(np.uint32)


@pytest.mark.parametrize("delta", [0, 1, 2, 3])
@pytest.mark.parametrize("n", [0, 5, 128, 129, 4097, 70001, 128 * 1100 + 77])
def test_encode_patched_matches_oracle(delta, n):
    """S4-FastPFOR streams (Sec. 4.4) are byte-identical to the oracle's,
    over several 512-block pages, for clustered data and for data with
    exceptions at many widths."""
    x = workloads.sorted_list(workloads.CLUSTERED, 500 + n, 1 << 26, n)
    assert np.array_equal(s4.encode(x, delta, patched=True), oracle.encode(x, delta, patched=True))
    y = _with_outliers(n + delta, n)
    enc = s4.encode(y, delta, patched=True)
    assert np.array_equal(enc, oracle.encode(y, delta, patched=True))
    assert enc.size <= s4.encoded_bound(n)


def test_encode_many_patched_matches_oracle():
    kinds, lens = workloads.bulk_lengths(8)
    lens = (lens // 32).astype(np.uint64)
    flat, offs = workloads.lists(kinds, lens, 99, 1 << 26)
    for delta in (0, 3):
        buf, soffs = s4.encode_many(flat, offs, nthreads=3, delta=delta, patched=True)
        for i in range(len(lens)):
            x = flat[int(offs[i]): int(offs[i + 1])]
            assert np.array_equal(buf[int(soffs[i]): int(soffs[i + 1])], oracle.encode(x, delta, patched=True))


def test_patched_bound_holds_for_worst_blocks():
    """Blocks whose every delta needs 32 bits, and blocks of one huge delta
    among zeros, stay within s4_encoded_bound."""
    n = 128 * 600
    for y in (np.sort(np.random.default_rng(3).integers(0, 1 << 32, size=n, dtype=np.uint64)).astype(np.uint32),
              np.repeat(np.arange(n // 128, dtype=np.uint64) * (1 << 22), 128).astype(np.uint32)):
        for delta in range(4):
            enc = s4.encode(y, delta, patched=True)
            assert enc.size <= s4.encoded_bound(n)
            assert np.array_equal(enc, oracle.encode(y, delta, patched=True))


def test_encode_rejects_unknown_form():
    with pytest.raises(s4.S4Error) as e:
        s4.encode(np.arange(10, dtype=np.uint32), 4)
    assert e.value.code == s4.EINVAL


@pytest.mark.parametrize("parts", [1, 2, 8, 13])
def test_partition_offsets(parts):
    """Each part of each sorted list starts at the first value >= floor(p U / parts)."""
    universe = 1 << 20
    lens = np.array([0, 1, 5, 1000, 77777, 3], dtype=np.uint64)
    kinds = np.full(lens.size, workloads.CLUSTERED, dtype=np.int32)
    flat, offs = workloads.lists(kinds, lens, 31, universe)
    sub = s4.partition_offsets(flat, offs, parts, universe)
    assert sub.size == lens.size * parts + 1 and sub[-1] == offs[-1]
    for t in range(lens.size):
        a, b = int(offs[t]), int(offs[t + 1])
        edges = [p * universe // parts for p in range(parts)]
        want = a + np.searchsorted(flat[a:b], np.array(edges, dtype=np.uint64), side="left")
        assert np.array_equal(sub[t * parts: t * parts + parts], want)
        for p in range(parts):
            part = flat[int(sub[t * parts + p]): int(sub[t * parts + p + 1])]
            lo, hi = p * universe // parts, (p + 1) * universe // parts
            assert part.size == 0 or (part[0] >= lo and part[-1] < hi)


def test_partition_offsets_errors():
    flat = np.array([1, 5, 1 << 20], dtype=np.uint32)
    offs = np.array([0, 3], dtype=np.uint64)
    with pytest.raises(s4.S4Error) as e:
        s4.partition_offsets(flat, offs, 4, 1 << 20)  # a value reaches the universe
    assert e.value.code == s4.EINVAL
    with pytest.raises(s4.S4Error):
        s4.partition_offsets(flat[:2], np.array([0, 2], np.uint64), 0, 1 << 20)


def test_decode_lists_stream_count_checked_before_any_device_work():
    """nstreams other than 1 and 8 is refused before the library touches a
    device (an empty call still validates it)."""
    lib = s4.require_library()
    assert lib.s4_decode_lists_dev(None, None, None, 0, 1, None) == 0
    assert lib.s4_decode_lists_dev(None, None, None, 0, 8, None) == 0
    for bad in (0, 2, 3, 4, 5, 6, 7, 9):
        assert lib.s4_decode_lists_dev(None, None, None, 0, bad, None) == s4.EINVAL, bad


def test_batch_calls_refuse_a_null_batch():
    """The batch entry points that take a handle check it before any device
    work."""
    import ctypes
    lib = s4.require_library()
    assert lib.s4_batch_set_counting(None, 1) == s4.EINVAL
    assert lib.s4_batch_set_counting(None, 0) == s4.EINVAL
    b, k = ctypes.c_uint64(0), ctypes.c_uint64(0)
    assert lib.s4_batch_traffic(None, ctypes.byref(b), ctypes.byref(k), None) == s4.EINVAL


@pytest.mark.parametrize("delta", [0, 1, 2, 3])
@pytest.mark.parametrize("patched", [False, True])
@pytest.mark.parametrize("n", [0, 1, 127, 128, 129, 4097, 128 * 1100 + 77])
def test_host_decode_matches_oracle(delta, patched, n):
    """s4_decode (the library's host decoder) on streams of every form,
    plain and patched (several pages), equals the oracle's decode and the
    input; extreme values and duplicates too."""
    for x in (workloads.sorted_list(workloads.CLUSTERED, 800 + n, 1 << 26, n), _with_outliers(n + 3 * delta, n)):
        enc = oracle.encode(x, delta, patched=patched)
        got = s4.decode_host(enc)
        assert np.array_equal(got, oracle.decode(enc))
        assert np.array_equal(got, x)
    y = np.repeat(np.array([0, 5, 2**31, 2**32 - 1], np.uint32), 100)
    enc = oracle.encode(y, delta, patched=patched)
    assert np.array_equal(s4.decode_host(enc), y)


def test_host_decode_errors():
    x = workloads.sorted_list(workloads.UNIFORM, 5, 1 << 20, 1000)
    enc = s4.encode(x)
    lib = s4.require_library()
    import ctypes
    out = np.zeros(999, np.uint32)
    n = ctypes.c_uint64(0)
    rc = lib.s4_decode(enc.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), enc.size,
                       out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), 999, ctypes.byref(n))
    assert rc == s4.ERANGE and n.value == 1000
    bad = enc.copy()
    bad[0] ^= 1
    with pytest.raises(s4.S4Error) as e:
        s4.decode_host(bad)
    assert e.value.code == s4.ECORRUPT
