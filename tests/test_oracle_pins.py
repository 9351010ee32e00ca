"""Pins for the CPU oracle: each test checks it against something the paper or
mathematics fixes independently of the oracle's own code (worked examples,
closed forms, invariants, brute force), never against a retyping of the
oracle itself."""
import itertools
import struct

import numpy as np
import pytest

import oracle
import workloads
from conftest import read_golden


def lane_words(enc, block_word_base, b, lane):
    """The b payload words of one lane of a block, in stream order."""
    nb = struct.unpack_from("<I", enc.tobytes(), 16)[0]
    payload_off = 32 + ((nb + 3) & ~3)
    base = payload_off + 4 * block_word_base
    return [struct.unpack_from("<I", enc.tobytes(), base + 4 * (4 * m + lane))[0] for m in range(b)]


def header(enc):
    magic, ver, flags, n, nb, t, pw = struct.unpack_from("<IHHQIIQ", enc.tobytes(), 0)
    return dict(magic=magic, version=ver, flags=flags, n=n, nb=nb, t=t, pw=pw)


# ------------------------------------------------------------- worked examples

def test_fig1c_bytes_are_one_lane_stream():
    """Fig. 1(c): 1, 3840, 131073, 2 at b = 18 are the 9 bytes printed in the
    figure.  Every lane of the block carries these deltas (each value is
    repeated four times, so the D4 deltas of every lane are the same), so
    lane 0's stream must start with exactly those bytes."""
    rows = {r[0]: r[1:] for r in read_golden("fig1c_packed.txt")}
    vals = [int(v) for v in rows["values"]]
    b = int(rows["bits"][0])
    want = bytes(int(h, 16) for h in rows["bytes"])
    x, acc = [], 0
    for v in vals:
        acc += v
        x += [acc] * 4
    x += [acc] * (128 - len(x))            # zero deltas afterwards
    enc = oracle.encode(np.array(x, np.uint32))
    assert list(oracle.widths(enc)) == [b]
    words = lane_words(enc, 0, b, lane=0)
    stream = b"".join(struct.pack("<I", w) for w in words)
    assert stream[:9] == want
    assert set(stream[9:]) == {0}
    for lane in range(1, 4):
        assert lane_words(enc, 0, b, lane) == words


def test_fig2_interleaved_layout():
    """Fig. 2 at b = 18: placement of x1..x9 in the interleaved words."""
    rows = read_golden("fig2_interleave.txt")
    b = int(rows[0][1])
    rng = np.random.default_rng(7)
    # sorted list: first quad 0,0,0,1, then consecutive gaps in [2^14, 2^16),
    # so every later D4 delta (a sum of four gaps) lies in [2^16, 2^18)
    gaps = rng.integers(1 << 14, 1 << 16, size=128).astype(np.int64)
    gaps[:4] = [0, 0, 0, 1]
    gaps[4] = 1 << 15
    x = np.cumsum(gaps).astype(np.uint32)
    d = [int(x[i]) - (int(x[i - 4]) if i >= 4 else 0) for i in range(128)]
    assert max(d).bit_length() == b
    enc = oracle.encode(x)
    assert list(oracle.widths(enc)) == [b]
    nb = header(enc)["nb"]
    payload_off = 32 + ((nb + 3) & ~3)
    words = struct.unpack_from(f"<{4 * b}I", enc.tobytes(), payload_off)
    for r in rows[1:]:
        xi = int(r[0][1:]) - 1
        wi = int(r[1][4:]) - 1
        bit = int(r[2][3:])
        ln = int(r[3][3:])
        frm = int(r[4][4:])
        got = (words[wi] >> bit) & ((1 << ln) - 1)
        assert got == (d[xi] >> frm) & ((1 << ln) - 1), r


# ---------------------------------------------------------- two decoders agree

def synthetic_stream(widths, rng, tail=()):
    """A valid stream with arbitrary payload bits (not produced by encode)."""
    nb = len(widths)
    pw = 4 * sum(widths)
    n = 128 * nb + len(tail)
    hdr = struct.pack("<IHHQIIQ", oracle.MAGIC, 1, 0, n, nb, len(tail), pw)
    wb = bytes(widths) + b"\0" * (((nb + 3) & ~3) - nb)
    payload = rng.integers(0, 2**32, size=pw, dtype=np.uint64).astype(np.uint32).tobytes()
    tl = np.array(tail, np.uint32).tobytes()
    return np.frombuffer(hdr + wb + payload + tl, np.uint8).copy()


@pytest.mark.parametrize("b", range(33))
def test_random_access_matches_alg1_walk(b):
    """The random-access extractor and the Alg. 1 vector walk are written
    differently; on arbitrary payload bits at every width they must agree."""
    rng = np.random.default_rng(100 + b)
    enc = synthetic_stream([b, b, (b * 7) % 33, b], rng, tail=[5, 9])
    assert np.array_equal(oracle.decode(enc), oracle.decode_alg1(enc))


def test_mixed_widths_all_values():
    rng = np.random.default_rng(3)
    enc = synthetic_stream(list(range(33)) + list(range(32, -1, -1)), rng)
    assert np.array_equal(oracle.decode(enc), oracle.decode_alg1(enc))


def test_b32_block_is_raw_words():
    """At b = 32 each lane word holds one delta verbatim (mask = all ones)."""
    rng = np.random.default_rng(5)
    enc = synthetic_stream([32], rng)
    nb = 1
    words = np.frombuffer(enc.tobytes()[32 + 4: 32 + 4 + 512], np.uint32)
    out = oracle.decode(enc).astype(np.uint64)
    # D4 inverse of raw deltas: out[p] = sum of words of lane p%4 up to q
    d = words.reshape(32, 4).astype(np.uint64)
    assert np.array_equal(out.reshape(32, 4), np.cumsum(d, axis=0) % (1 << 32))


def test_b0_block_repeats_seed():
    """b = 0 (reading A4): 128 zero deltas, every lane keeps its seed."""
    x = np.full(256, 3, np.uint32)
    enc = oracle.encode(x)
    assert list(oracle.widths(enc)) == [2, 0]
    assert np.array_equal(oracle.decode(enc), x)
    assert np.array_equal(oracle.decode_alg1(enc), x)


# ------------------------------------------------------------ round trips

def recipe_list(b, n=4096, seed=0):
    """Sec. 7.4 recipe: 4096 integers whose D4 gaps are below 2^b, built
    as a sorted list (each consecutive gap below 2^b / 4)."""
    rng = np.random.default_rng(seed + b)
    g = max(1, (1 << b) // 4) if b >= 2 else 1
    if b == 0:
        return np.zeros(n, np.uint32)
    if b == 1:
        gaps = np.zeros(n, np.uint64)
        gaps[::4] = rng.integers(0, 2, size=(n + 3) // 4)
        gaps[:4] = 0
    else:
        gaps = rng.integers(0, g, size=n).astype(np.uint64)
    x = np.cumsum(gaps) % (1 << 32)
    x.sort()
    return x.astype(np.uint32)


@pytest.mark.parametrize("b", range(33))
def test_round_trip_per_width(b):
    x = recipe_list(b)
    enc = oracle.encode(x)
    w = oracle.widths(enc)
    assert w.max() <= max(b, 1) or b == 32
    assert np.array_equal(oracle.decode(enc), x)
    assert np.array_equal(oracle.decode_alg1(enc), x)


@pytest.mark.parametrize("n", [0, 1, 3, 4, 5, 127, 128, 129, 255, 256, 2047, 2048, 2049, 4096 + 77])
def test_round_trip_edge_lengths(n):
    x = workloads.sorted_list(workloads.UNIFORM, 42 + n, 1 << 25, n)
    enc = oracle.encode(x)
    h = header(enc)
    assert h["n"] == n and h["nb"] == n // 128 and h["t"] == n % 128
    assert h["flags"] == 1
    assert np.array_equal(oracle.decode(enc), x)
    assert np.array_equal(oracle.decode_alg1(enc), x)


def test_round_trip_full_range_values():
    x = np.array(sorted({0, 1, 2**31, 2**32 - 1, 2**32 - 2} | set(range(5, 700, 3))), np.uint32)
    enc = oracle.encode(x)
    assert np.array_equal(oracle.decode(enc), x)


# ------------------------------------------------ size formula and widths

def brute_width(vals):
    """Sec. 4.3 definition, by search: smallest b with all values < 2^b."""
    for b in range(33):
        if all(v < 2**b for v in vals):
            return b
    raise AssertionError


@pytest.mark.parametrize("seed", range(4))
def test_bits_per_block_formula_and_widths(seed):
    """Encoded size = header + width bytes (padded to 4) + 16 b bytes per
    block (Sec. 4.2) + 4 bytes per tail integer; every width is the
    smallest b that holds the block's D4 deltas (Sec. 4.3, Sec. 5)."""
    n = 128 * 37 + seed * 31
    kind = workloads.CLUSTERED if seed % 2 else workloads.UNIFORM
    x = workloads.sorted_list(kind, 1000 + seed, 1 << (20 + 3 * seed), n)
    xi = [int(v) for v in x]
    enc = oracle.encode(x)
    w = [int(v) for v in oracle.widths(enc)]
    nb = n // 128
    assert len(w) == nb
    for k in range(nb):
        deltas = [xi[i] - (xi[i - 4] if i >= 4 else 0) for i in range(128 * k, 128 * k + 128)]
        assert w[k] == brute_width(deltas)
    expect = 32 + ((nb + 3) // 4) * 4 + sum(16 * b for b in w) + 4 * (n % 128)
    assert enc.size == expect
    assert oracle.stream_bytes(n, np.array(w, np.uint8)) == expect


@pytest.mark.parametrize("c,s", [(0, 1), (7, 3), (1000, 255), (5, 1 << 20), (0, (1 << 30) // 700)])
def test_arithmetic_progression_closed_form(c, s):
    """x_i = c + s i: every D4 delta past the first quad is 4s, so blocks
    k >= 1 have width bitlen(4s); block 0 also holds x_0..x_3."""
    n = 128 * 5 + 9
    x = (c + s * np.arange(n, dtype=np.uint64))
    assert x[-1] < 2**32
    enc = oracle.encode(x.astype(np.uint32))
    w = oracle.widths(enc)
    assert int(w[0]) == max((c + 3 * s).bit_length(), (4 * s).bit_length())
    assert all(int(b) == (4 * s).bit_length() for b in w[1:])
    assert np.array_equal(oracle.decode(enc), x.astype(np.uint32))


@pytest.mark.parametrize("p", [0, 3, 61, 124, 127])
def test_width_reaches_every_position(p):
    """A single jump of J at position p raises only the D4 deltas at
    p..p+3 to 4 + J: the block width must follow it wherever it sits,
    including the last delta of the block."""
    J = 1000
    x = np.arange(128, dtype=np.uint32)
    x[p:] += J
    w = oracle.widths(oracle.encode(x))
    assert int(w[0]) == (4 + J).bit_length()
    assert np.array_equal(oracle.decode(oracle.encode(x)), x)


def test_width_floor_strictly_increasing():
    """Strictly increasing input: every D4 delta after the first quad is
    >= 4, so every block after the first has width >= 3."""
    for seed in range(5):
        x = workloads.sorted_list(workloads.CLUSTERED, 77 + seed, 1 << 26, 128 * 50)
        w = oracle.widths(oracle.encode(x))
        assert w[1:].min() >= 3


def test_first_block_width_uses_zero_seed():
    """The first quad's deltas are the values themselves (seed 0)."""
    x = np.arange(128, dtype=np.uint32) + np.uint32(1 << 20)
    w = oracle.widths(oracle.encode(x))
    assert int(w[0]) == 21


# ------------------------------------------------------------- errors

def test_unsorted_rejected():
    with pytest.raises(oracle.OracleError) as e:
        oracle.encode(np.array([1, 2, 3, 2], np.uint32))
    assert e.value.code == oracle.EUNSORTED


def test_corrupt_streams_rejected():
    x = workloads.sorted_list(workloads.UNIFORM, 9, 1 << 20, 300)
    enc = oracle.encode(x)
    bad = [enc[:-1], enc.copy(), enc.copy(), enc.copy(), np.concatenate([enc, [0, 0, 0, 0]])]
    bad[1][0] ^= 1                     # magic
    bad[2][32] = 33                    # width > 32
    bad[3][8] ^= 1                     # n inconsistent with nb, t
    for e in bad:
        with pytest.raises(oracle.OracleError) as ex:
            oracle.decode(e)
        assert ex.value.code == oracle.ECORRUPT


def test_duplicates_allowed_by_codec_flag_cleared():
    x = np.array([1, 1, 2, 3, 3, 3, 9] * 40, np.uint32)
    x.sort()
    enc = oracle.encode(x)
    assert header(enc)["flags"] == 0
    assert np.array_equal(oracle.decode(enc), x)


# ------------------------------------------------------- intersection

def brute_intersection(a, b):
    """O(mn): keep each element of a that equals some element of b."""
    out = []
    for u in a:
        for v in b:
            if u == v:
                out.append(u)
                break
    return out


def test_intersect_exhaustive_small_universe():
    """Every pair of subsets of [0, 7)."""
    subsets = [list(c) for r in range(8) for c in itertools.combinations(range(7), r)]
    for a in subsets:
        for b in subsets:
            got = oracle.intersect(np.array(a, np.uint32), np.array(b, np.uint32)).tolist()
            assert got == brute_intersection(a, b)


def test_intersect_random_subsets_of_12():
    rng = np.random.default_rng(11)
    for _ in range(3000):
        a = np.flatnonzero(rng.random(12) < rng.random())
        b = np.flatnonzero(rng.random(12) < rng.random())
        got = oracle.intersect(a.astype(np.uint32), b.astype(np.uint32)).tolist()
        assert got == brute_intersection(a.tolist(), b.tolist())


def test_intersect_matches_numpy_set_routine():
    a, b = workloads.plain_pair()
    got = oracle.intersect(a, b)
    assert np.array_equal(got, np.intersect1d(a, b, assume_unique=True))
    assert np.array_equal(got, oracle.intersect(b, a))


def test_plain_pair_intersection_size_is_plausible():
    """E|A n B| = 2^20 2^14 / 2^25 = 512, sd about 22 (hypergeometric)."""
    a, b = workloads.plain_pair()
    c = oracle.intersect(a, b).size
    assert abs(c - 512) < 6 * 23


def test_intersect_rejects_unsorted_and_duplicates():
    with pytest.raises(oracle.OracleError):
        oracle.intersect(np.array([1, 1, 2], np.uint32), np.array([1], np.uint32))
    with pytest.raises(oracle.OracleError):
        oracle.intersect(np.array([3, 2], np.uint32), np.array([1], np.uint32))


def test_intersect_k_invariants():
    rng = np.random.default_rng(5)
    lists = [np.unique(rng.integers(0, 300, size=rng.integers(0, 200))).astype(np.uint32)
             for _ in range(4)]
    ref = set(lists[0].tolist())
    for l in lists[1:]:
        ref &= set(l.tolist())
    ref = sorted(ref)
    for perm in itertools.permutations(range(4)):
        assert oracle.intersect_k([lists[i] for i in perm]).tolist() == ref
    assert oracle.intersect_k([lists[0]]).tolist() == lists[0].tolist()
    assert oracle.intersect_k([lists[1], lists[1]]).tolist() == lists[1].tolist()
    assert oracle.intersect_k([lists[2], np.zeros(0, np.uint32)]).tolist() == []


# ---------------------------------------------------- other differential forms

MODES = {"D4": oracle.D4, "DM": oracle.DM, "D2": oracle.D2, "D1": oracle.D1}


def mode_stream(mode, widths, rng, tail=()):
    """synthetic_stream with the differential form in flag bits 1-2."""
    enc = synthetic_stream(widths, rng, tail)
    enc[6] = (mode << 1) & 0xFF
    return enc


@pytest.mark.parametrize("name", sorted(MODES))
@pytest.mark.parametrize("b", [0, 1, 5, 17, 31, 32])
def test_modes_random_access_matches_alg1_walk(name, b):
    """The definition-based inverse and the Sec. 5 SIMD step lists (applied
    per 4-vector in the Alg. 1 walk) agree on arbitrary payload bits."""
    rng = np.random.default_rng(300 + b)
    enc = mode_stream(MODES[name], [b, (b + 9) % 33, b], rng, tail=[1, 2, 3])
    assert np.array_equal(oracle.decode(enc), oracle.decode_alg1(enc))


def test_sec5_worked_prefix_steps():
    """The Sec. 5 step lists, instantiated by hand (golden file): a stream
    whose second 4-vector of deltas is (3, 5, 7, 11) after a first vector
    decoding to (100, 110, 120, 130)."""
    rows = {r[0]: [int(v) for v in r[1:]] for r in read_golden("sec5_prefix_steps.txt")}
    prev, deltas = rows["prev"], rows["deltas"]
    for name, mode in MODES.items():
        # the list (x1..x8, then x8 repeated) encoded with the form must
        # pack exactly the deltas (d5..d8) at positions 4..7 and decode back
        x = np.array(prev + rows[name] + [rows[name][-1]] * 120, np.uint32)
        enc = oracle.encode(x, mode)
        got = oracle.decode(enc)
        assert list(got[4:8]) == rows[name]
        # the stream's packed deltas for positions 4..7 are the Sec. 5 deltas
        d = payload_deltas(enc)
        assert list(d[4:8]) == deltas, name


def payload_deltas(enc, block=0):
    """Unpack the packed values of one block with the pinned Fig. 2 layout:
    lane j's words are 4m + j, read as one least-significant-first bit
    stream."""
    w = oracle.widths(enc)
    b = int(w[block])
    nb = header(enc)["nb"]
    off = 32 + ((nb + 3) & ~3) + 16 * int(sum(int(v) for v in w[:block]))
    words = struct.unpack_from(f"<{4 * b}I", enc.tobytes(), off) if b else ()
    out = [0] * 128
    for j in range(4):
        stream = 0
        for m in range(b):
            stream |= words[4 * m + j] << (32 * m)
        for q in range(32):
            out[4 * q + j] = (stream >> (q * b)) & ((1 << b) - 1)
    return out


@pytest.mark.parametrize("c,s", [(7, 3), (1000, 255), (5, 1 << 20)])
def test_modes_arithmetic_progression_widths(c, s):
    """x_i = c + s i: after the first block every D1 delta is s, every D2
    delta 2s, DM deltas are s, 2s, 3s, 4s within each quad, D4 deltas 4s."""
    n = 128 * 4 + 3
    x = (c + s * np.arange(n, dtype=np.uint64)).astype(np.uint32)
    expect = {"D1": s, "D2": 2 * s, "DM": 4 * s, "D4": 4 * s}
    for name, mode in MODES.items():
        enc = oracle.encode(x, mode)
        w = oracle.widths(enc)
        assert all(int(b) == expect[name].bit_length() for b in w[1:]), name
        assert np.array_equal(oracle.decode(enc), x)
        d = payload_deltas(enc)
        if name == "DM":
            assert d[4:8] == [s, 2 * s, 3 * s, 4 * s]


def test_table3_relative_delta_sizes():
    """Table 3: the deltas of D2, DM and D4 are on average 2, 2.5 and 4
    times those of D1 (a D1 delta spans one gap, D2 two, DM one to four,
    D4 four), read back from the packed payload of every block."""
    x = workloads.sorted_list(workloads.UNIFORM, 5, 1 << 30, 128 * 48)
    mean = {}
    for name, m in MODES.items():
        enc = oracle.encode(x, m)
        d = [v for k in range(1, 48) for v in payload_deltas(enc, k)]
        mean[name] = float(np.mean(d))
    for name, ratio in (("D2", 2.0), ("DM", 2.5), ("D4", 4.0)):
        assert abs(mean[name] / mean["D1"] - ratio) < 0.05 * ratio, (name, mean)


@pytest.mark.parametrize("name", sorted(MODES))
@pytest.mark.parametrize("n", [0, 1, 5, 127, 128, 129, 2049, 70001])
def test_modes_round_trip(name, n):
    x = workloads.sorted_list(workloads.CLUSTERED, 900 + n, 1 << 26, n)
    enc = oracle.encode(x, MODES[name])
    assert header(enc)["flags"] >> 1 == MODES[name]
    assert np.array_equal(oracle.decode(enc), x)
    assert np.array_equal(oracle.decode_alg1(enc), x)


# ------------------------------------------------------ hyb+m2 (Sec. 7.7)

@pytest.mark.parametrize("n, universe, gap, want", [
    (128, 1024, 8, True),      # average gap exactly B: a bitmap (at most B)
    (127, 1024, 8, False),     # just above B
    (64, 1024, 16, True), (63, 1024, 16, False),
    (32, 1000, 32, True),      # 1000 / 32 = 31.25
    (31, 1000, 32, False),     # 32.3
    (1, 1, 1, True), (5, 40, 8, True), (5, 41, 8, False),
    (0, 1024, 8, False),       # an empty list is never a bitmap
    (1 << 20, 1 << 20, 0, False),  # B = 0: no bitmaps
    ((1 << 32) - 1, 1 << 32, 2, True),
])
def test_hyb_bitmap_rule(n, universe, gap, want):
    """The representation rule: a bitmap exactly when universe / n <= B,
    checked on boundaries in exact rational arithmetic."""
    from fractions import Fraction
    assert oracle.hyb_is_bitmap(n, universe, gap) == want
    if n and gap:
        assert (Fraction(universe, n) <= gap) == want


def _hyb_brute(lists):
    s = set(int(v) for v in lists[0])
    for l in lists[1:]:
        s &= set(int(v) for v in l)
    return np.array(sorted(s), dtype=np.uint32)


@pytest.mark.parametrize("seed", range(40))
def test_hyb_equals_set_intersection(seed):
    """Whatever lists become bitmaps, the hybrid procedure (SvS over the
    compressed lists, then bit probes) returns exactly the set
    intersection; every mix of representations is drawn, including all
    compressed and all bitmaps, and universes that are not a multiple of 32
    with the last value U - 1 present."""
    rng = np.random.default_rng(4400 + seed)
    universe = int(rng.choice([61, 96, 1000, 4096, 5003]))
    k = int(rng.integers(1, 6))
    lists = []
    for _ in range(k):
        n = int(rng.integers(0, universe + 1)) if rng.random() < 0.8 else int(rng.integers(universe // 2, universe + 1))
        v = np.sort(rng.choice(universe, size=n, replace=False)).astype(np.uint32)
        if n and rng.random() < 0.3:
            v[-1] = universe - 1 if universe - 1 not in v[:-1] else v[-1]
            v = np.unique(v)
        lists.append(v)
    for gap in (0, 1, 2, 4, 8, 16, 32, 1 << 20):
        kinds = [oracle.hyb_is_bitmap(l.size, universe, gap) for l in lists]
        got = oracle.hyb_intersect_k(lists, universe, gap)
        assert np.array_equal(got, _hyb_brute(lists)), (seed, gap, kinds)


def test_hyb_all_bitmaps_and_mixed_by_hand():
    """Hand-checked cases: multiples of 2 and 3 below 100 (50 and 34
    values) are bitmaps at B = 4 (gaps 2 and 2.94); {6, 12, 99, 100} stays
    compressed; 100 >= U has no bit."""
    m2 = np.arange(0, 100, 2, dtype=np.uint32)
    m3 = np.arange(0, 100, 3, dtype=np.uint32)
    few = np.array([6, 12, 99, 100], dtype=np.uint32)
    assert oracle.hyb_is_bitmap(m2.size, 100, 4) and oracle.hyb_is_bitmap(m3.size, 100, 4)
    assert not oracle.hyb_is_bitmap(few.size, 100, 4)
    assert oracle.hyb_intersect_k([m2, m3], 100, 4).tolist() == list(range(0, 100, 6))
    assert oracle.hyb_intersect_k([few, m2, m3], 100, 4).tolist() == [6, 12]
    assert oracle.hyb_intersect_k([m3, few], 100, 4).tolist() == [6, 12, 99]
    assert oracle.hyb_intersect_k([m2], 100, 4).tolist() == m2.tolist()
    with pytest.raises(oracle.OracleError):  # a bitmap list reaching the universe
        oracle.hyb_intersect_k([np.arange(0, 101, 2, dtype=np.uint32)], 100, 4)


# -------------------------------------------------- S4-FastPFOR (Sec. 4.4)

def _fig3_block():
    rows = {r[0]: [int(v) for v in r[1:]] for r in read_golden("fig3_fastpfor.txt")}
    first, filler = rows["first"], rows["filler"]
    blk = first + [filler[i % 9] for i in range(len(first), 128)]
    return np.array(blk, dtype=np.uint32), rows


def test_fig3_fastpfor_choice():
    """Fig. 3's block: b = 28 (the printed 27 corrected by the width rule),
    b' = 2, one exception."""
    blk, rows = _fig3_block()
    assert oracle.fp_choose(blk) == (rows["b"][0], rows["bprime"][0], rows["exceptions"][0])


def test_fig3_fastpfor_stream_bytes():
    """The same block as the first block of a D1 stream (x = running sums of
    the block, so the D1 deltas are the block): the stored width is b', the
    packed low bits are those of the figure, the page metadata records b, one
    exception at position 3, and the array for 26 holds 134217729 >> 2."""
    blk, rows = _fig3_block()
    x = np.cumsum(blk.astype(np.uint64)).astype(np.uint32)
    enc = oracle.encode(x, oracle.D1, patched=True)
    # zero deltas repeat values: not strictly increasing (bit 0 clear)
    assert int.from_bytes(enc[6:8].tobytes(), "little") == (oracle.D1 << 1) | 8
    assert enc[32] == rows["bprime"][0]
    pw = int.from_bytes(enc[24:32].tobytes(), "little")
    assert pw == 4 * rows["bprime"][0]
    words = np.frombuffer(enc[36: 36 + 4 * pw].tobytes(), dtype="<u4")
    b = rows["bprime"][0]
    low = []
    for i in range(9):  # Fig. 2 layout: lane i % 4, position i // 4, LSB first
        lane, q = i % 4, i // 4
        bit = q * b
        low.append(int(words[4 * (bit // 32) + lane] >> (bit % 32)) & ((1 << b) - 1))
    assert low == rows["low"]
    p = 36 + 4 * pw  # no tail: 128 values
    meta_len = int.from_bytes(enc[p: p + 4].tobytes(), "little")
    meta = enc[p + 4: p + 4 + meta_len].tolist()
    assert meta == [rows["b"][0], 1, rows["position"][0]]
    q = p + 4 + ((meta_len + 3) & ~3)
    present = int.from_bytes(enc[q: q + 4].tobytes(), "little")
    assert present == 1 << (rows["array"][0] - 1)
    count = int.from_bytes(enc[q + 4: q + 8].tobytes(), "little")
    first_word = int.from_bytes(enc[q + 8: q + 12].tobytes(), "little")
    assert count == 1 and first_word == rows["high"][0]
    assert enc.size == q + 8 + 4 * rows["array"][0]  # 26 words: one padded group of 32 values
    assert np.array_equal(oracle.decode(enc), x) and np.array_equal(oracle.decode_alg1(enc), x)


@pytest.mark.parametrize("blk, want", [
    ([5] * 128, (3, 3, 0)),                       # no outlier: b' = b
    ([0] * 128, (0, 0, 0)),
    ([0] * 127 + [1 << 31], (32, 0, 1)),          # one 32-bit outlier among zeros: b' = 0, 40 bits
    ([7] * 120 + [1 << 20] * 8, (21, 3, 8)),      # 8 exceptions of 18 + 8 bits beat 18 bits a value
])
def test_fastpfor_choice_by_hand(blk, want):
    assert oracle.fp_choose(np.array(blk, dtype=np.uint32)) == want


def test_fastpfor_tie_goes_to_larger_width():
    """b = 11 with 8 values in [2^10, 2^11), 12 in [2^9, 2^10) and 108 in
    [2^8, 2^9): b' = 10 costs 1280 + 8 * 9 and b' = 9 costs 1152 + 20 * 10,
    both 1352, every other b' more; the reading breaks the tie toward 10."""
    blk = np.array([1500] * 8 + [700] * 12 + [300] * 108, dtype=np.uint32)
    assert oracle.fp_choose(blk) == (11, 10, 8)


def _deltas(x, mode):
    x = x.astype(np.int64)
    ref = np.zeros_like(x)
    if mode == oracle.D1:
        ref[1:] = x[:-1]
    elif mode == oracle.D2:
        ref[2:] = x[:-2]
    elif mode == oracle.D4:
        ref[4:] = x[:-4]
    else:
        q = np.arange(x.size) // 4
        ref[q >= 1] = x[4 * q[q >= 1] - 1]
    return (x - ref).astype(np.uint32)


@pytest.mark.parametrize("mode", [oracle.D4, oracle.DM, oracle.D2, oracle.D1])
@pytest.mark.parametrize("n", [128 * 512 * 2 + 300, 128 * 700])
def test_fastpfor_stream_size_and_pages(mode, n):
    """Round trip through both decoders over several pages (512 blocks
    each); the stream is exactly header + b' widths + 16 b' per block + raw
    tail + per page (meta length, 2 bytes + positions per block padded to 4,
    presence mask, per present d a count and d words per 32 values); every
    block's chosen cost stays within plain packing's 128 b."""
    rng = np.random.default_rng(n + mode)
    gaps = rng.geometric(0.25, size=n).astype(np.uint64)
    k = n // 97
    gaps[rng.integers(0, n, size=k)] += rng.integers(1, 1 << 20, size=k).astype(np.uint64)
    x = np.cumsum(gaps)
    assert x[-1] < 1 << 32
    x = x.astype(np.uint32)
    enc = oracle.encode(x, mode, patched=True)
    assert np.array_equal(oracle.decode(enc), x)
    assert np.array_equal(oracle.decode_alg1(enc), x)
    nb, t = n // 128, n % 128
    d = _deltas(x, mode)
    choice = [oracle.fp_choose(d[128 * kb: 128 * kb + 128]) for kb in range(nb)]
    size = 32 + ((nb + 3) & ~3) + sum(16 * bp for _, bp, _ in choice) + 4 * t
    for k0 in range(0, nb, 512):
        page = choice[k0: k0 + 512]
        meta = sum(2 + c for _, _, c in page)
        size += 4 + ((meta + 3) & ~3) + 4
        cnt = {}
        for b, bp, c in page:
            if c:
                cnt[b - bp] = cnt.get(b - bp, 0) + c
        size += sum(4 + 4 * dd * ((cc + 31) // 32) for dd, cc in cnt.items())
    assert enc.size == size
    for b, bp, c in choice:
        assert 128 * bp + c * (b - bp + 8) <= 128 * b
        assert (c > 0) == (bp < b)


def test_fastpfor_compresses_at_least_as_well_on_clustered_data():
    """Table 5's direction: on clustered lists S4-FastPFOR never needs more
    bits per integer than S4-BP128 in the same form (D1: 4.4 vs 5.0 bits on
    the paper's dense ClusterData)."""
    x = workloads.sorted_list(workloads.CLUSTERED, 77, 1 << 26, 1 << 18)
    for mode in (oracle.D4, oracle.DM, oracle.D2, oracle.D1):
        plain = oracle.encode(x, mode).size
        patched = oracle.encode(x, mode, patched=True).size
        assert patched < plain, mode
        assert np.array_equal(oracle.decode(oracle.encode(x, mode, patched=True)), x)


def test_fastpfor_corrupt_streams_rejected():
    x = np.cumsum(np.array([1] * 300 + [1 << 20] + [2] * 400, dtype=np.uint64)).astype(np.uint32)
    enc = oracle.encode(x, oracle.D1, patched=True)
    assert np.array_equal(oracle.decode(enc), x)
    with pytest.raises(oracle.OracleError):
        oracle.decode(enc[:-4])                  # truncated array
    bad = enc.copy()
    bad[6] = bad[6] & 0xF7                       # patched flag cleared: trailing bytes
    with pytest.raises(oracle.OracleError):
        oracle.decode(bad)
    pw = int.from_bytes(enc[24:32].tobytes(), "little")
    p = 32 + 8 + 4 * pw + 4 * (x.size % 128)      # 5 blocks: widths padded to 8
    bad = enc.copy()
    bad[p + 4 + 1] = 129                         # exception count > 128
    with pytest.raises(oracle.OracleError):
        oracle.decode(bad)
