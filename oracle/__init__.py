"""Python access to the plain C oracle (``oracle/oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the CPU-baseline leg of the benchmark.  The product library never imports,
links or calls anything here.

Every function returns numpy arrays and raises ``OracleError`` on a
non-zero status.  The shared object is built by ``oracle.build()`` (plain
gcc, no GPU toolchain).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

OK, EINVAL, EUNSORTED, ERANGE, ECORRUPT, ENOMEM = 0, -1, -2, -3, -4, -5
D4, DM, D2, D1 = 0, 1, 2, 3  # differential forms (stream flag bits 1-2)
HEADER_BYTES = 32
MAGIC = 0x34443453


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc -O2 (scalar C only)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None
_variants = {}


def _bind(path):
    lib = ctypes.CDLL(path)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    sz = ctypes.c_size_t
    lib.orc_encode.argtypes = [u32p, ctypes.c_uint64, u8p, sz, ctypes.POINTER(sz)]
    lib.orc_encode_mode.argtypes = [u32p, ctypes.c_uint64, ctypes.c_uint32, u8p, sz, ctypes.POINTER(sz)]
    lib.orc_decode.argtypes = [u8p, sz, u32p, ctypes.c_uint64, u64p]
    lib.orc_decode_alg1.argtypes = [u8p, sz, u32p, ctypes.c_uint64, u64p]
    lib.orc_decoded_length.argtypes = [u8p, sz, u64p]
    lib.orc_widths.argtypes = [u8p, sz, u8p, ctypes.c_uint64, u64p]
    lib.orc_stream_bytes.argtypes = [ctypes.c_uint64, u8p]
    lib.orc_stream_bytes.restype = sz
    lib.orc_intersect.argtypes = [u32p, ctypes.c_uint64, u32p, ctypes.c_uint64, u32p, u64p]
    lib.orc_encode_fp.argtypes = [u32p, ctypes.c_uint64, ctypes.c_uint32, u8p, sz, ctypes.POINTER(sz)]
    lib.orc_fp_choose.argtypes = [u32p, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint32),
                                  ctypes.POINTER(ctypes.c_uint32)]
    lib.orc_fp_choose.restype = None
    lib.orc_hyb_is_bitmap.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32]
    lib.orc_hyb_intersect_k.argtypes = [ctypes.POINTER(u32p), u64p, ctypes.c_uint32, ctypes.c_uint64,
                                        ctypes.c_uint32, u32p, ctypes.c_uint64, u64p]
    lib.orc_intersect_k.argtypes = [ctypes.POINTER(u32p), u64p, ctypes.c_uint32, u32p,
                                    ctypes.c_uint64, u64p]
    for f in (lib.orc_encode, lib.orc_encode_mode, lib.orc_encode_fp, lib.orc_decode, lib.orc_decode_alg1, lib.orc_decoded_length,
              lib.orc_widths, lib.orc_intersect, lib.orc_intersect_k):
        f.restype = ctypes.c_int
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = _bind(_LIB_PATH)
    return _lib


_current = None  # set while a variant library is active (tests only)


def _active():
    return _current if _current is not None else _load()


class use_variant:
    """Context manager: route every oracle call to another build of oracle.c.

    Used only by the mutation tests, which compile deliberately broken copies
    of the oracle and check that the pins reject them."""

    def __init__(self, path):
        self.path = path

    def __enter__(self):
        global _current
        if self.path not in _variants:
            _variants[self.path] = _bind(self.path)
        _current = _variants[self.path]
        return self

    def __exit__(self, *exc):
        global _current
        _current = None
        return False


def _u32(a):
    a = np.ascontiguousarray(a, dtype=np.uint32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def _u8(a):
    a = np.ascontiguousarray(a, dtype=np.uint8)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def encode(x, mode: int = D4, patched: bool = False) -> np.ndarray:
    """Serialized S4-BP128 stream of a non-decreasing uint32 list with the
    given differential form (D4 by default); patched=True gives the
    S4-FastPFOR stream (Sec. 4.4)."""
    lib = _active()
    x, xp = _u32(x)
    n = x.size
    nb = n // 128
    bound = HEADER_BYTES + ((nb + 3) & ~3) + 514 * nb + 4 * (n % 128) + 16
    if patched:  # per page: 2 headers, padding of up to 32 arrays
        bound += ((nb + 511) // 512) * (16 + 4 * 33 + 32 * 32 * 4)
    out = np.zeros(bound, dtype=np.uint8)
    nbytes = ctypes.c_size_t(0)
    fn = lib.orc_encode_fp if patched else lib.orc_encode_mode
    rc = fn(xp, n, mode, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), bound, ctypes.byref(nbytes))
    if rc:
        raise OracleError(rc, "encode")
    return out[: nbytes.value].copy()


def fp_choose(block):
    """FastPFOR's (b, b', exceptions) for one block of 128 deltas."""
    lib = _active()
    blk, bp = _u32(block)
    if blk.size != 128:
        raise ValueError("a block has 128 deltas")
    b, p, c = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
    lib.orc_fp_choose(bp, ctypes.byref(b), ctypes.byref(p), ctypes.byref(c))
    return b.value, p.value, c.value


def decode(enc) -> np.ndarray:
    """Decode by random-access extraction + running D4 sums."""
    return _decode(enc, "orc_decode")


def decode_alg1(enc) -> np.ndarray:
    """Decode by the vector-walk procedure of the paper's Alg. 1."""
    return _decode(enc, "orc_decode_alg1")


def _decode(enc, fname):
    lib = _active()
    enc, ep = _u8(enc)
    n = ctypes.c_uint64(0)
    rc = lib.orc_decoded_length(ep, enc.size, ctypes.byref(n))
    if rc:
        raise OracleError(rc, "decoded_length")
    out = np.zeros(max(1, n.value), dtype=np.uint32)
    rc = getattr(lib, fname)(ep, enc.size, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                             n.value, ctypes.byref(n))
    if rc:
        raise OracleError(rc, fname)
    return out[: n.value].copy()


def widths(enc) -> np.ndarray:
    lib = _active()
    enc, ep = _u8(enc)
    n = ctypes.c_uint64(0)
    rc = lib.orc_decoded_length(ep, enc.size, ctypes.byref(n))
    if rc:
        raise OracleError(rc, "decoded_length")
    out = np.zeros(max(1, n.value // 128), dtype=np.uint8)
    nb = ctypes.c_uint64(0)
    rc = lib.orc_widths(ep, enc.size, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), out.size,
                        ctypes.byref(nb))
    if rc:
        raise OracleError(rc, "widths")
    return out[: nb.value].copy()


def stream_bytes(n: int, w) -> int:
    lib = _active()
    w, wp = _u8(w if len(w) else np.zeros(1, np.uint8))
    return int(lib.orc_stream_bytes(n, wp))


def intersect(a, b) -> np.ndarray:
    """Two-pointer merge of strictly increasing lists."""
    lib = _active()
    a, ap = _u32(a)
    b, bp = _u32(b)
    out = np.zeros(max(1, min(a.size, b.size)), dtype=np.uint32)
    c = ctypes.c_uint64(0)
    rc = lib.orc_intersect(ap, a.size, bp, b.size, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                           ctypes.byref(c))
    if rc:
        raise OracleError(rc, "intersect")
    return out[: c.value].copy()


def intersect_k(lists) -> np.ndarray:
    """Left fold of the pairwise merge over the lists in the order given."""
    lib = _active()
    arrs = [np.ascontiguousarray(l, dtype=np.uint32) for l in lists]
    k = len(arrs)
    ptrs = (ctypes.POINTER(ctypes.c_uint32) * max(1, k))()
    keep = []
    for i, a in enumerate(arrs):
        if a.size == 0:
            a = np.zeros(1, np.uint32)[:0]
        keep.append(a)
        ptrs[i] = a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
    lens = (ctypes.c_uint64 * max(1, k))(*[a.size for a in arrs])
    cap = arrs[0].size if k else 0
    out = np.zeros(max(1, cap), dtype=np.uint32)
    c = ctypes.c_uint64(0)
    rc = lib.orc_intersect_k(ptrs, lens, k, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), cap,
                             ctypes.byref(c))
    if rc:
        raise OracleError(rc, "intersect_k")
    return out[: c.value].copy()


def hyb_is_bitmap(n: int, universe: int, gap: int) -> bool:
    """hyb+m2 rule: a list of n > 0 values is a bitmap when universe / n <= gap."""
    return bool(_active().orc_hyb_is_bitmap(int(n), int(universe), int(gap)))


def hyb_intersect_k(lists, universe: int, gap: int) -> np.ndarray:
    """Conjunctive query under hyb+m2: SvS over the compressed lists, then
    bit probes of the bitmap lists (AND of the bitmaps when all are)."""
    lib = _active()
    arrs = [np.ascontiguousarray(l, dtype=np.uint32) for l in lists]
    k = len(arrs)
    ptrs = (ctypes.POINTER(ctypes.c_uint32) * max(1, k))()
    keep = []
    for i, a in enumerate(arrs):
        if a.size == 0:
            a = np.zeros(1, np.uint32)[:0]
        keep.append(a)
        ptrs[i] = a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
    lens = (ctypes.c_uint64 * max(1, k))(*[a.size for a in arrs])
    cap = min(a.size for a in arrs) if k else 0
    out = np.zeros(max(1, cap), dtype=np.uint32)
    c = ctypes.c_uint64(0)
    rc = lib.orc_hyb_intersect_k(ptrs, lens, k, int(universe), int(gap),
                                 out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), cap, ctypes.byref(c))
    if rc:
        raise OracleError(rc, "hyb_intersect_k")
    return out[: c.value].copy()
