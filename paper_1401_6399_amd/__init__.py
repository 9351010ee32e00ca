"""Python binding of libs4.so (the C ABI declared in include/s4.h).

Argument marshalling only: every step of decode and intersection runs in
the library's HIP kernels.  Device buffers are torch tensors on the current
CUDA (HIP) device; the library enqueues on torch's current stream.  If the
shared library has not been built this module raises on first use: there is
no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libs4.so")

OK, EINVAL, EUNSORTED, ERANGE, ECORRUPT, ENOMEM, EDEVICE, EAGAIN = 0, -1, -2, -3, -4, -5, -6, -7
DELTA_D4, DELTA_DM, DELTA_D2, DELTA_D1 = 0, 1, 2, 3
CODEC_FASTPFOR = 0x100  # OR into `delta`: patched (S4-FastPFOR) stream

# every symbol declared in include/s4.h, with (restype, argtypes)
_vp = ctypes.c_void_p
_u8p = ctypes.POINTER(ctypes.c_uint8)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_sz = ctypes.c_size_t
_i = ctypes.c_int
_u32 = ctypes.c_uint32
_u64 = ctypes.c_uint64


class Tuning(ctypes.Structure):
    _fields_ = [("gallop_blocks", ctypes.c_uint32), ("waves_per_group", ctypes.c_uint32),
                ("groups_per_cu", ctypes.c_uint32), ("items_per_grab", ctypes.c_uint32),
                ("decode_passes", ctypes.c_uint32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class ServerConfig(ctypes.Structure):
    _fields_ = [("max_slots", ctypes.c_uint32), ("pool_bytes", ctypes.c_uint64),
                ("result_bytes", ctypes.c_uint64), ("max_terms", ctypes.c_uint32),
                ("slice_chunks", ctypes.c_uint32)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("admitted", ctypes.c_uint64),
                ("completed", ctypes.c_uint64), ("rejected", ctypes.c_uint64),
                ("iterations", ctypes.c_uint64), ("peak_active", ctypes.c_uint64),
                ("peak_pool_bytes", ctypes.c_uint64), ("waits_for_memory", ctypes.c_uint64),
                ("max_batch", ctypes.c_uint64), ("direct_iterations", ctypes.c_uint64),
                ("single_pass_iterations", ctypes.c_uint64), ("sliced_queries", ctypes.c_uint64),
                ("device_ns", ctypes.c_uint64), ("host_ns", ctypes.c_uint64), ("retire_ns", ctypes.c_uint64),
                ("admit_ns", ctypes.c_uint64), ("launch_ns", ctypes.c_uint64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


SIGNATURES = {
    "s4_last_error": (ctypes.c_char_p, []),
    "s4_version": (_i, []),
    "s4_init": (_i, []),
    "s4_encoded_bound": (_sz, [_u64]),
    "s4_encode": (_i, [_u32p, _u64, _u8p, _sz, ctypes.POINTER(_sz)]),
    "s4_encode_ex": (_i, [_u32p, _u64, _u32, _u8p, _sz, ctypes.POINTER(_sz)]),
    "s4_encode_many": (_i, [_u32p, _u64p, _u64, _u32, _u8p, _u64p, _u64p, _i]),
    "s4_decoded_length": (_i, [_u8p, _sz, _u64p]),
    "s4_decode": (_i, [_u8p, _sz, _u32p, _u64, _u64p]),
    "s4_list_upload": (_i, [_u8p, _sz, _vp, ctypes.POINTER(_vp)]),
    "s4_list_free": (_i, [_vp]),
    "s4_list_info": (_i, [_vp, _u64p, _u32p, _u32p, _u64p, _u64p]),
    "s4_list_skip_index": (_i, [_vp, _u32p, _u32p, _vp]),
    "s4_decode_dev": (_i, [_vp, _vp, _u64, _vp]),
    "s4_decode_blocks_dev": (_i, [_vp, _u32, _u32, _vp, _vp]),
    "s4_decode_timed_dev": (_i, [_vp, _vp, _u64, _vp, _vp, _vp]),
    "s4_decode_lists_dev": (_i, [ctypes.POINTER(_vp), ctypes.POINTER(_vp), _u64p, _u32, _u32, _vp]),
    "s4_decode_plan_create": (_i, [ctypes.POINTER(_vp), ctypes.POINTER(_vp), _u64p, _u32, _vp,
                                   ctypes.POINTER(_vp)]),
    "s4_decode_plan_run": (_i, [_vp, _vp]),
    "s4_decode_plan_free": (_i, [_vp]),
    "s4_aql_plan_create": (_i, [ctypes.POINTER(_vp), ctypes.POINTER(_vp), _u64p, _u32, ctypes.POINTER(_vp)]),
    "s4_aql_plan_create_placed": (_i, [ctypes.POINTER(_vp), ctypes.POINTER(_vp), _u64p, _u32, _u32p, _u32p,
                                       ctypes.POINTER(_vp)]),
    "s4_aql_plan_run": (_i, [_vp, _u32, _u64p]),
    "s4_aql_plan_enqueue": (_i, [_vp, _u32, _vp]),
    "s4_aql_plan_status": (_i, [_vp]),
    "s4_aql_plan_profile": (_i, [_vp, _u32, _u64p, _u64p, _u64p]),
    "s4_aql_plan_layout": (_i, [_vp, _u32p, _u32p]),
    "s4_aql_plan_free": (_i, [_vp]),
    "s4_spin_dev": (_i, [_u64, _vp]),
    "s4_intersect_scratch_bytes": (_sz, [_u64, _u64]),
    "s4_intersect": (_i, [_vp, _vp, _vp, _u64, _vp, _vp, _sz, _vp]),
    "s4_intersect_k_scratch_bytes": (_sz, [ctypes.POINTER(_vp), _u32]),
    "s4_intersect_k": (_i, [ctypes.POINTER(_vp), _u32, _vp, _u64, _vp, _vp, _sz, _vp]),
    "s4_intersect_raw_scratch_bytes": (_sz, [_u64]),
    "s4_intersect_k_noalloc_max_len": (_u64, []),
    "s4_intersect_k_noalloc": (_i, [ctypes.POINTER(_vp), _u32, _vp, _u64, _vp, _vp]),
    "s4_intersect_raw": (_i, [_vp, _vp, _u64, _vp, _vp, _u64, _vp, _vp, _sz, _vp]),
    "s4_get_tuning": (_i, [ctypes.POINTER(Tuning)]),
    "s4_set_tuning": (_i, [ctypes.POINTER(Tuning)]),
    "s4_index_build": (_i, [_u8p, _u64p, _u64, _vp, ctypes.POINTER(_vp)]),
    "s4_index_free": (_i, [_vp]),
    "s4_index_lengths": (_i, [_vp, _u64p]),
    "s4_index_info": (_i, [_vp, _u64p, _u64p, _u64p, _u64p]),
    "s4_index_list": (_i, [_vp, _u64, ctypes.POINTER(_vp)]),
    "s4_index_build_hybrid": (_i, [_u8p, _u64p, _u64, _u64, _u32, _vp, ctypes.POINTER(_vp)]),
    "s4_index_kinds": (_i, [_vp, _u8p]),
    "s4_index_build_parts": (_i, [_u8p, _u64p, _u64, _u32, _vp, ctypes.POINTER(_vp)]),
    "s4_partition_offsets": (_i, [_u32p, _u64p, _u64, _u32, _u64, _u64p]),
    "s4_index_hybrid_info": (_i, [_vp, _u64p, ctypes.POINTER(_u32), _u64p, _u64p, _u64p]),
    "s4_batch_plan": (_i, [_vp, _u32p, _u64p, _u64, _vp, ctypes.POINTER(_vp)]),
    "s4_batch_free": (_i, [_vp]),
    "s4_batch_results_bound": (_u64, [_vp]),
    "s4_batch_run": (_i, [_vp, _vp, _vp, _vp, _u64, _i, _vp]),
    "s4_batch_query_ticks": (_i, [_vp, _u64p, _vp]),
    "s4_batch_set_counting": (_i, [_vp, _i]),
    "s4_batch_traffic": (_i, [_vp, _u64p, _u64p, _vp]),
    "s4_batch_autotune": (_i, [_vp, _vp, _vp, _vp, _u64, _i, _vp, ctypes.POINTER(Tuning),
                               ctypes.POINTER(ctypes.c_double)]),
    "s4_server_create": (_i, [_vp, ctypes.POINTER(ServerConfig), ctypes.POINTER(_vp)]),
    "s4_server_submit": (_i, [_vp, _u32p, _u32, _u64p]),
    "s4_server_poll": (_i, [_vp, _u64p, _u64p, _u64p, _u32p, _u64, _u64p, _u32, _u32p]),
    "s4_server_stats_get": (_i, [_vp, ctypes.POINTER(ServerStats)]),
    "s4_server_destroy": (_i, [_vp]),
    "s4_server_replay": (_i, [_vp, _u32p, _u64p, _u64, _u64p, _u64p, _u64p, _u32p, _u64, _u64p, _u8p,
                              ctypes.c_double, ctypes.POINTER(ctypes.c_double)]),
    "s4_plain_run": (_i, [_vp, _u32p, _u64p, _u64, _vp, _u64, _u64p, _vp, _vp, _sz, _u64p, _u64p, _vp]),
    "s4_plain_replay": (_i, [_vp, _u32p, _u64p, _u64, _u64p, _u64p, _vp, _u64, _vp, _vp, _sz, ctypes.c_double,
                             ctypes.POINTER(ctypes.c_double), _vp]),
}


class S4Error(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"s4 error {code}: {msg}")
        self.code = code


_lib = None


def library_built() -> bool:
    return os.path.exists(LIB_PATH)


def require_library():
    """Load libs4.so or raise: there is no CPU fallback."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(rc, what=""):
    if rc != OK:
        msg = require_library().s4_last_error()
        raise S4Error(rc, (what + ": " if what else "") + (msg.decode() if msg else ""))


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _dptr(t):
    """Raw device address of a torch tensor (or None)."""
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


# ------------------------------------------------------------------ codec

def init():
    """Set up the current device (s4_init): checks it and looks up the
    static scratch of intersect_k_noalloc."""
    _check(require_library().s4_init(), "s4_init")


def encoded_bound(n: int) -> int:
    return int(require_library().s4_encoded_bound(n))


def encode(x, delta: int = DELTA_D4, patched: bool = False) -> np.ndarray:
    """Host encode of a non-decreasing uint32 list (s4_encode_ex); patched
    selects S4-FastPFOR."""
    lib = require_library()
    x = np.ascontiguousarray(x, dtype=np.uint32)
    cap = encoded_bound(x.size)
    out = np.zeros(cap, dtype=np.uint8)
    nbytes = ctypes.c_size_t(0)
    code = delta | (CODEC_FASTPFOR if patched else 0)
    _check(lib.s4_encode_ex(_ptr(x, ctypes.c_uint32), x.size, code, _ptr(out, ctypes.c_uint8), cap,
                            ctypes.byref(nbytes)), "s4_encode_ex")
    return out[: nbytes.value].copy()


def partition_offsets(flat, offsets, parts: int, universe: int) -> np.ndarray:
    """Where each part of each sorted list starts in `flat` (s4_partition_offsets):
    sub-list t * parts + p holds list t's values in part p of [0, universe)."""
    lib = require_library()
    flat = np.ascontiguousarray(flat, dtype=np.uint32)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    count = offsets.size - 1
    sub = np.zeros(count * parts + 1, dtype=np.uint64)
    _check(lib.s4_partition_offsets(_ptr(flat if flat.size else np.zeros(1, np.uint32), ctypes.c_uint32),
                                    _ptr(offsets, ctypes.c_uint64), count, int(parts), int(universe),
                                    _ptr(sub, ctypes.c_uint64)), "s4_partition_offsets")
    return sub


def encode_many(flat, offsets, nthreads: int = 0, delta: int = DELTA_D4, patched: bool = False):
    """Encode many lists at once: returns (streams buffer, stream offsets)."""
    delta = delta | (CODEC_FASTPFOR if patched else 0)
    lib = require_library()
    flat = np.ascontiguousarray(flat, dtype=np.uint32)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    count = offsets.size - 1
    lens = np.diff(offsets)
    bounds = np.array([encoded_bound(int(n)) for n in lens], dtype=np.uint64) if count else np.zeros(0, np.uint64)
    out_offs = np.zeros(count + 1, dtype=np.uint64)
    np.cumsum(bounds, out=out_offs[1:])
    buf = np.zeros(max(1, int(out_offs[-1])), dtype=np.uint8)
    sizes = np.zeros(max(1, count), dtype=np.uint64)
    _check(lib.s4_encode_many(_ptr(flat if flat.size else np.zeros(1, np.uint32), ctypes.c_uint32),
                              _ptr(offsets, ctypes.c_uint64), count, delta, _ptr(buf, ctypes.c_uint8),
                              _ptr(out_offs, ctypes.c_uint64), _ptr(sizes, ctypes.c_uint64), nthreads),
           "s4_encode_many")
    # compact the streams back to back
    sizes = sizes[:count]
    offs = np.zeros(count + 1, dtype=np.uint64)
    np.cumsum(sizes, out=offs[1:])
    packed = np.empty(max(1, int(offs[-1])), dtype=np.uint8)
    for i in range(count):
        s, n = int(out_offs[i]), int(sizes[i])
        packed[int(offs[i]): int(offs[i]) + n] = buf[s: s + n]
    return packed[: int(offs[-1])], offs


def decode_host(enc) -> np.ndarray:
    """Host decode of a stream (s4_decode): a scalar loop in the library,
    for tools and checks; the decoding path is the device one."""
    lib = require_library()
    enc = np.ascontiguousarray(enc, dtype=np.uint8)
    n = decoded_length(enc)
    out = np.zeros(max(1, n), np.uint32)
    got = ctypes.c_uint64(0)
    _check(lib.s4_decode(_ptr(enc, ctypes.c_uint8), enc.size, _ptr(out, ctypes.c_uint32), n, ctypes.byref(got)),
           "s4_decode")
    return out[:n]


def decoded_length(enc) -> int:
    lib = require_library()
    enc = np.ascontiguousarray(enc, dtype=np.uint8)
    n = ctypes.c_uint64(0)
    _check(lib.s4_decoded_length(_ptr(enc, ctypes.c_uint8), enc.size, ctypes.byref(n)), "s4_decoded_length")
    return n.value


# ----------------------------------------------------------------- lists

class DeviceList:
    """A list resident in device memory (s4_list)."""

    def __init__(self, handle, owner=None):
        self.h = ctypes.c_void_p(handle) if not isinstance(handle, ctypes.c_void_p) else handle
        self._owner = owner
        n = ctypes.c_uint64(0)
        nb = ctypes.c_uint32(0)
        fl = ctypes.c_uint32(0)
        pb = ctypes.c_uint64(0)
        ib = ctypes.c_uint64(0)
        _check(require_library().s4_list_info(self.h, ctypes.byref(n), ctypes.byref(nb), ctypes.byref(fl),
                                              ctypes.byref(pb), ctypes.byref(ib)), "s4_list_info")
        self.n, self.nb, self.flags = n.value, nb.value, fl.value
        self.payload_bytes, self.index_bytes = pb.value, ib.value

    @classmethod
    def upload(cls, enc, stream=None):
        lib = require_library()
        enc = np.ascontiguousarray(enc, dtype=np.uint8)
        h = ctypes.c_void_p()
        _check(lib.s4_list_upload(_ptr(enc, ctypes.c_uint8), enc.size, _stream(stream), ctypes.byref(h)),
               "s4_list_upload")
        return cls(h)

    def free(self):
        if self.h:
            _check(require_library().s4_list_free(self.h), "s4_list_free")
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            if self.h and require_library() is not None:
                require_library().s4_list_free(self.h)
                self.h = ctypes.c_void_p()
        except Exception:
            pass

    def skip_index(self, stream=None):
        bmax = np.zeros(max(1, self.nb), np.uint32)
        seeds = np.zeros(max(1, 4 * self.nb), np.uint32)
        _check(require_library().s4_list_skip_index(self.h, _ptr(bmax, ctypes.c_uint32),
                                                    _ptr(seeds, ctypes.c_uint32), _stream(stream)),
               "s4_list_skip_index")
        return bmax[: self.nb], seeds[: 4 * self.nb].reshape(-1, 4)

    def decode_into(self, out, stream=None):
        _check(require_library().s4_decode_dev(self.h, _dptr(out), out.numel(), _stream(stream)), "s4_decode_dev")

    def decode_timed_into(self, out, start_event, stop_event, stream=None):
        """Decode with torch timing events recorded by the launch itself at
        the kernel's start and end (the events must have been recorded once,
        so that they exist)."""
        _check(require_library().s4_decode_timed_dev(self.h, _dptr(out), out.numel(),
                                                     ctypes.c_void_p(start_event.cuda_event),
                                                     ctypes.c_void_p(stop_event.cuda_event), _stream(stream)),
               "s4_decode_timed_dev")

    def decode(self, stream=None):
        import torch
        out = torch.empty(max(1, self.n), dtype=torch.int32, device="cuda")
        self.decode_into(out, stream)
        return out[: self.n]

    def decode_blocks_into(self, first, count, out, stream=None):
        _check(require_library().s4_decode_blocks_dev(self.h, first, count, _dptr(out), _stream(stream)),
               "s4_decode_blocks_dev")


def _out_arrays(lists, outs):
    hs = _handles(lists)
    ptrs = (ctypes.c_void_p * max(1, len(outs)))(*[o.data_ptr() for o in outs])
    caps = np.array([o.numel() for o in outs] or [0], dtype=np.uint64)
    return hs, ptrs, caps


def decode_lists(lists, outs, nstreams=1, stream=None):
    """One decode launch per list, spread over nstreams forked streams."""
    hs, ptrs, caps = _out_arrays(lists, outs)
    _check(require_library().s4_decode_lists_dev(hs, ptrs, _ptr(caps, ctypes.c_uint64), len(lists), nstreams,
                                                 _stream(stream)), "s4_decode_lists_dev")


class DecodePlan:
    """Single-launch decode of many lists (s4_decode_plan)."""

    def __init__(self, lists, outs, stream=None):
        hs, ptrs, caps = _out_arrays(lists, outs)
        self._keep = (lists, outs)
        self.h = ctypes.c_void_p()
        _check(require_library().s4_decode_plan_create(hs, ptrs, _ptr(caps, ctypes.c_uint64), len(lists),
                                                       _stream(stream), ctypes.byref(self.h)),
               "s4_decode_plan_create")

    def run(self, stream=None):
        _check(require_library().s4_decode_plan_run(self.h, _stream(stream)), "s4_decode_plan_run")

    def __del__(self):
        try:
            if self.h:
                require_library().s4_decode_plan_free(self.h)
                self.h = ctypes.c_void_p()
        except Exception:
            pass


class AqlDecodePlan:
    """Per-list decode, one dispatch per list, on the library's own queues
    (s4_aql_plan).  run() is host-synchronous and not ordered with torch's
    streams (the device is synchronised before it); enqueue() orders a run
    after the work of a stream and returns at once."""

    def __init__(self, lists, outs, queue_of=None, rank=None):
        import torch
        hs, ptrs, caps = _out_arrays(lists, outs)
        self._keep = (lists, outs)
        self.count = len(lists)
        self.h = ctypes.c_void_p()
        torch.cuda.synchronize()
        if queue_of is None:
            _check(require_library().s4_aql_plan_create(hs, ptrs, _ptr(caps, ctypes.c_uint64), len(lists),
                                                        ctypes.byref(self.h)), "s4_aql_plan_create")
        else:
            qo = np.ascontiguousarray(queue_of, dtype=np.uint32)
            rk = np.ascontiguousarray(rank, dtype=np.uint32) if rank is not None else None
            _check(require_library().s4_aql_plan_create_placed(
                hs, ptrs, _ptr(caps, ctypes.c_uint64), len(lists), _ptr(qo, ctypes.c_uint32),
                _ptr(rk, ctypes.c_uint32) if rk is not None else None, ctypes.byref(self.h)),
                "s4_aql_plan_create_placed")

    def run(self, steps=1):
        """Decode every list `steps` times; returns the host wall time in ms."""
        import torch
        torch.cuda.synchronize()
        ns = ctypes.c_uint64(0)
        _check(require_library().s4_aql_plan_run(self.h, int(steps), ctypes.byref(ns)), "s4_aql_plan_run")
        return ns.value / 1e6

    def enqueue(self, steps=1, stream=None):
        """Decode every list `steps` times after the work already on `stream`
        (torch's current stream by default); later work on the stream waits
        for it."""
        _check(require_library().s4_aql_plan_enqueue(self.h, int(steps), _stream(stream)), "s4_aql_plan_enqueue")

    def status(self):
        """Raise if an enqueued run has failed."""
        _check(require_library().s4_aql_plan_status(self.h), "s4_aql_plan_status")

    def layout(self):
        """(queue of each list, its position in that queue's step order)."""
        q = np.zeros(max(1, self.count), np.uint32)
        p = np.zeros(max(1, self.count), np.uint32)
        _check(require_library().s4_aql_plan_layout(self.h, _ptr(q, ctypes.c_uint32), _ptr(p, ctypes.c_uint32)),
               "s4_aql_plan_layout")
        return q[: self.count], p[: self.count]

    def profile(self, steps=1):
        """One profiled run: per-list device start and end (ns after the
        run's first dispatch started), arrays [steps, count], and the host
        wall time in ms."""
        import torch
        torch.cuda.synchronize()
        st = np.zeros(steps * self.count, np.uint64)
        en = np.zeros(steps * self.count, np.uint64)
        ns = ctypes.c_uint64(0)
        _check(require_library().s4_aql_plan_profile(self.h, int(steps), _ptr(st, ctypes.c_uint64),
                                                     _ptr(en, ctypes.c_uint64), ctypes.byref(ns)),
               "s4_aql_plan_profile")
        return st.reshape(steps, self.count), en.reshape(steps, self.count), ns.value / 1e6

    def __del__(self):
        try:
            if self.h:
                require_library().s4_aql_plan_free(self.h)
                self.h = ctypes.c_void_p()
        except Exception:
            pass


def spin(ns, stream=None):
    _check(require_library().s4_spin_dev(int(ns), _stream(stream)), "s4_spin_dev")


def _device_u64():
    import torch
    return torch.zeros(1, dtype=torch.int64, device="cuda")


def _scratch(nbytes):
    import torch
    return torch.empty(max(256, int(nbytes)), dtype=torch.uint8, device="cuda")


def intersect(a: DeviceList, b: DeviceList, out=None, count=None, scratch=None, stream=None):
    """Decode-fused pairwise intersection; returns (out tensor, device count)."""
    import torch
    lib = require_library()
    m = min(a.n, b.n)
    if out is None:
        out = torch.empty(max(1, m), dtype=torch.int32, device="cuda")
    if count is None:
        count = _device_u64()
    need = int(lib.s4_intersect_scratch_bytes(a.n, b.n))
    if scratch is None:
        scratch = _scratch(need)
    _check(lib.s4_intersect(a.h, b.h, _dptr(out), out.numel(), _dptr(count), _dptr(scratch),
                            scratch.numel(), _stream(stream)), "s4_intersect")
    return out, count


def _handles(lists):
    arr = (ctypes.c_void_p * max(1, len(lists)))()
    for i, l in enumerate(lists):
        arr[i] = l.h.value if isinstance(l.h, ctypes.c_void_p) else l.h
    return arr


def intersect_k_scratch_bytes(lists) -> int:
    return int(require_library().s4_intersect_k_scratch_bytes(_handles(lists), len(lists)))


def intersect_k(lists, out=None, count=None, scratch=None, stream=None):
    import torch
    lib = require_library()
    m = min(l.n for l in lists) if lists else 0
    if out is None:
        out = torch.empty(max(1, m), dtype=torch.int32, device="cuda")
    if count is None:
        count = _device_u64()
    if scratch is None:
        scratch = _scratch(intersect_k_scratch_bytes(lists))
    _check(lib.s4_intersect_k(_handles(lists), len(lists), _dptr(out), out.numel(), _dptr(count),
                              _dptr(scratch), scratch.numel(), _stream(stream)), "s4_intersect_k")
    return out, count


def intersect_k_noalloc(lists, out=None, count=None, stream=None):
    """intersect_k with the library's static device scratch (no allocation
    in the library; out and count are allocated here when not given)."""
    import torch
    lib = require_library()
    m = min(l.n for l in lists) if lists else 0
    if out is None:
        out = torch.empty(max(1, m), dtype=torch.int32, device="cuda")
    if count is None:
        count = _device_u64()
    _check(lib.s4_intersect_k_noalloc(_handles(lists), len(lists), _dptr(out), out.numel(), _dptr(count),
                                      _stream(stream)), "s4_intersect_k_noalloc")
    return out, count


def intersect_k_noalloc_max_len() -> int:
    return int(require_library().s4_intersect_k_noalloc_max_len())


def intersect_raw(r, r_len, cap_r, f: DeviceList, out=None, count=None, scratch=None, stream=None):
    import torch
    lib = require_library()
    if out is None:
        out = torch.empty(max(1, min(cap_r, f.n)), dtype=torch.int32, device="cuda")
    if count is None:
        count = _device_u64()
    if scratch is None:
        scratch = _scratch(int(lib.s4_intersect_raw_scratch_bytes(cap_r)))
    _check(lib.s4_intersect_raw(_dptr(r), _dptr(r_len), cap_r, f.h, _dptr(out), out.numel(), _dptr(count),
                                _dptr(scratch), scratch.numel(), _stream(stream)), "s4_intersect_raw")
    return out, count


def get_tuning() -> Tuning:
    t = Tuning()
    _check(require_library().s4_get_tuning(ctypes.byref(t)), "s4_get_tuning")
    return t


def set_tuning(**kw):
    t = get_tuning()
    for k, v in kw.items():
        setattr(t, k, int(v))
    _check(require_library().s4_set_tuning(ctypes.byref(t)), "s4_set_tuning")
    return t


# ----------------------------------------------------------------- index

class Index:
    """Many device-resident lists (s4_index).  With bitmap_gap = B > 0 the
    index is a hyb+m2 hybrid: lists with universe / n <= B are bitmaps over
    [0, universe) (s4_index_build_hybrid)."""

    def __init__(self, streams, offsets, stream=None, universe=0, bitmap_gap=0, parts=1):
        lib = require_library()
        streams = np.ascontiguousarray(streams, dtype=np.uint8)
        offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
        self.h = ctypes.c_void_p()
        self.parts = int(parts)
        sp = _ptr(streams if streams.size else np.zeros(1, np.uint8), ctypes.c_uint8)
        if parts > 1:
            if bitmap_gap:
                raise ValueError("a partitioned index has no bitmap lists")
            _check(lib.s4_index_build_parts(sp, _ptr(offsets, ctypes.c_uint64), (offsets.size - 1) // parts,
                                            int(parts), _stream(stream), ctypes.byref(self.h)),
                   "s4_index_build_parts")
        elif bitmap_gap:
            _check(lib.s4_index_build_hybrid(sp, _ptr(offsets, ctypes.c_uint64), offsets.size - 1, int(universe),
                                             int(bitmap_gap), _stream(stream), ctypes.byref(self.h)),
                   "s4_index_build_hybrid")
        else:
            _check(lib.s4_index_build(sp, _ptr(offsets, ctypes.c_uint64), offsets.size - 1, _stream(stream),
                                      ctypes.byref(self.h)), "s4_index_build")
        self.count = (offsets.size - 1) // max(1, self.parts)
        self.lengths = np.zeros(max(1, self.count), np.uint64)
        _check(lib.s4_index_lengths(self.h, _ptr(self.lengths, ctypes.c_uint64)), "s4_index_lengths")
        self.lengths = self.lengths[: self.count]
        c, ti, pb, ib = (ctypes.c_uint64() for _ in range(4))
        _check(lib.s4_index_info(self.h, ctypes.byref(c), ctypes.byref(ti), ctypes.byref(pb), ctypes.byref(ib)),
               "s4_index_info")
        self.total_ints, self.payload_bytes, self.index_bytes = ti.value, pb.value, ib.value
        u, nbm, bb, sb = (ctypes.c_uint64() for _ in range(4))
        g = ctypes.c_uint32()
        _check(lib.s4_index_hybrid_info(self.h, ctypes.byref(u), ctypes.byref(g), ctypes.byref(nbm),
                                        ctypes.byref(bb), ctypes.byref(sb)), "s4_index_hybrid_info")
        self.universe, self.bitmap_gap = u.value, g.value
        self.bitmap_lists, self.bitmap_bytes, self.select_bytes = nbm.value, bb.value, sb.value

    def kinds(self) -> np.ndarray:
        """1 where the list is held as a bitmap, else 0."""
        k = np.zeros(max(1, self.count), np.uint8)
        _check(require_library().s4_index_kinds(self.h, _ptr(k, ctypes.c_uint8)), "s4_index_kinds")
        return k[: self.count]

    def list(self, i) -> DeviceList:
        h = ctypes.c_void_p()
        _check(require_library().s4_index_list(self.h, i, ctypes.byref(h)), "s4_index_list")
        return DeviceList(h, owner=self)

    def free(self):
        if self.h:
            _check(require_library().s4_index_free(self.h), "s4_index_free")
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            if self.h:
                require_library().s4_index_free(self.h)
                self.h = ctypes.c_void_p()
        except Exception:
            pass


class Batch:
    """A planned batch of conjunctive queries over an Index (s4_batch)."""

    def __init__(self, index: Index, terms, q_offsets, stream=None):
        import torch
        lib = require_library()
        terms = np.ascontiguousarray(terms, dtype=np.uint32)
        q_offsets = np.ascontiguousarray(q_offsets, dtype=np.uint64)
        self.index = index
        self.nq = q_offsets.size - 1
        self.h = ctypes.c_void_p()
        _check(lib.s4_batch_plan(index.h, _ptr(terms if terms.size else np.zeros(1, np.uint32), ctypes.c_uint32),
                                 _ptr(q_offsets, ctypes.c_uint64), self.nq, _stream(stream),
                                 ctypes.byref(self.h)), "s4_batch_plan")
        self.results_bound = int(lib.s4_batch_results_bound(self.h))
        self.counts = torch.zeros(max(1, self.nq), dtype=torch.int64, device="cuda")
        self.res_offsets = torch.zeros(self.nq + 1, dtype=torch.int64, device="cuda")
        self.results = torch.zeros(max(1, self.results_bound), dtype=torch.int32, device="cuda")

    def run(self, use_graph=False, stream=None):
        _check(require_library().s4_batch_run(self.h, _dptr(self.counts), _dptr(self.res_offsets),
                                              _dptr(self.results), self.results.numel(), int(bool(use_graph)),
                                              _stream(stream)), "s4_batch_run")

    def query_ticks(self, stream=None):
        t = np.zeros(max(1, self.nq), np.uint64)
        _check(require_library().s4_batch_query_ticks(self.h, _ptr(t, ctypes.c_uint64), _stream(stream)),
               "s4_batch_query_ticks")
        return t[: self.nq]

    def set_counting(self, on):
        """Count algorithmic traffic in later runs (off by default: it slows
        the kernels)."""
        _check(require_library().s4_batch_set_counting(self.h, 1 if on else 0), "s4_batch_set_counting")

    def traffic(self, stream=None):
        """(algorithmic bytes, blocks decoded) of the last run, zeros if it
        did not count (see set_counting)."""
        b, k = ctypes.c_uint64(0), ctypes.c_uint64(0)
        _check(require_library().s4_batch_traffic(self.h, ctypes.byref(b), ctypes.byref(k), _stream(stream)),
               "s4_batch_traffic")
        return b.value, k.value

    def autotune(self, reps=3, stream=None):
        best = Tuning()
        ms = ctypes.c_double(0)
        _check(require_library().s4_batch_autotune(self.h, _dptr(self.counts), _dptr(self.res_offsets),
                                                   _dptr(self.results), self.results.numel(), reps,
                                                   _stream(stream), ctypes.byref(best), ctypes.byref(ms)),
               "s4_batch_autotune")
        return best.as_dict(), ms.value

    def result(self, q):
        """Host copy of query q's result (synchronises)."""
        offs = self.res_offsets.cpu().numpy()
        return self.results[int(offs[q]): int(offs[q + 1])].cpu().numpy().view(np.uint32)

    def free(self):
        if self.h:
            _check(require_library().s4_batch_free(self.h), "s4_batch_free")
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            if self.h:
                require_library().s4_batch_free(self.h)
                self.h = ctypes.c_void_p()
        except Exception:
            pass


# ------------------------------------------------------------- plain path

def plain_run(index: "Index", terms, q_offsets, isolate=False, stream=None):
    """Every query as its own single-launch conjunction, back to back
    (s4_plain_run).  Returns (counts tensor, results tensor, res_offsets
    numpy, elapsed ms, per-query isolated latency in ns or None)."""
    import torch
    lib = require_library()
    terms = np.ascontiguousarray(terms, dtype=np.uint32)
    q_offsets = np.ascontiguousarray(q_offsets, dtype=np.uint64)
    nq = q_offsets.size - 1
    lens = index.lengths
    # sizes only (terms are checked by the library)
    tl = lens[np.minimum(terms, max(0, lens.size - 1))] if lens.size else np.zeros(terms.size, np.uint64)
    mins = np.minimum.reduceat(tl, q_offsets[:-1].astype(np.int64)) if nq and tl.size else np.zeros(nq, np.uint64)
    total = int(mins.sum()) if nq else 0
    need = int(lib.s4_intersect_raw_scratch_bytes(int(mins.max()) if nq else 0))
    results = torch.empty(max(1, total), dtype=torch.int32, device="cuda")
    counts = torch.zeros(max(1, nq), dtype=torch.int64, device="cuda")
    scratch = _scratch(need)
    roffs = np.zeros(nq + 1, np.uint64)
    lat = np.zeros(max(1, nq), np.uint64) if isolate else None
    ns = ctypes.c_uint64(0)
    _check(lib.s4_plain_run(index.h, _ptr(terms if terms.size else np.zeros(1, np.uint32), ctypes.c_uint32),
                            _ptr(q_offsets, ctypes.c_uint64), nq, _dptr(results), results.numel(),
                            _ptr(roffs, ctypes.c_uint64), _dptr(counts), _dptr(scratch), scratch.numel(),
                            _ptr(lat, ctypes.c_uint64) if isolate else None, ctypes.byref(ns), _stream(stream)),
           "s4_plain_run")
    return counts[:nq], results, roffs, ns.value / 1e6, (lat[:nq] if isolate else None)


def plain_replay(index: "Index", terms, q_offsets, arrival_ns, timeout_s=600.0, stream=None):
    """The plain path under an open-loop arrival trace (s4_plain_replay):
    {'latency_ns', 'counts', 'elapsed_s'}."""
    import torch
    lib = require_library()
    terms = np.ascontiguousarray(terms, dtype=np.uint32)
    q_offsets = np.ascontiguousarray(q_offsets, dtype=np.uint64)
    arrival_ns = np.ascontiguousarray(arrival_ns, dtype=np.uint64)
    nq = q_offsets.size - 1
    lens = index.lengths
    tl = lens[np.minimum(terms, max(0, lens.size - 1))] if lens.size else np.zeros(terms.size, np.uint64)
    mins = np.minimum.reduceat(tl, q_offsets[:-1].astype(np.int64)) if nq and tl.size else np.zeros(1, np.uint64)
    m = int(mins.max()) if nq else 0
    results = torch.empty(max(1, m), dtype=torch.int32, device="cuda")
    counts = torch.zeros(max(1, nq), dtype=torch.int64, device="cuda")
    scratch = _scratch(int(lib.s4_intersect_raw_scratch_bytes(m)))
    lat = np.zeros(max(1, nq), np.uint64)
    el = ctypes.c_double(0)
    _check(lib.s4_plain_replay(index.h, _ptr(terms if terms.size else np.zeros(1, np.uint32), ctypes.c_uint32),
                               _ptr(q_offsets, ctypes.c_uint64), nq, _ptr(arrival_ns, ctypes.c_uint64),
                               _ptr(lat, ctypes.c_uint64), _dptr(results), results.numel(), _dptr(counts),
                               _dptr(scratch), scratch.numel(), timeout_s, ctypes.byref(el), _stream(stream)),
           "s4_plain_replay")
    return {"latency_ns": lat[:nq], "counts": counts[:nq].cpu().numpy().astype(np.uint64), "elapsed_s": el.value}


# ----------------------------------------------------------------- server

class Server:
    """Continuous-batching query server (s4_server)."""

    def __init__(self, index: Index, max_slots=4096, pool_bytes=1 << 30, result_bytes=1 << 28, max_terms=8,
                 slice_chunks=0):
        cfg = ServerConfig(max_slots, pool_bytes, result_bytes, max_terms, slice_chunks)
        self.index = index
        self.h = ctypes.c_void_p()
        _check(require_library().s4_server_create(index.h, ctypes.byref(cfg), ctypes.byref(self.h)),
               "s4_server_create")

    def submit(self, terms):
        terms = np.ascontiguousarray(terms, dtype=np.uint32)
        qid = ctypes.c_uint64(0)
        rc = require_library().s4_server_submit(self.h, _ptr(terms, ctypes.c_uint32), terms.size, ctypes.byref(qid))
        if rc == EAGAIN:
            return None
        _check(rc, "s4_server_submit")
        return qid.value

    def poll(self, max_done=4096, results_cap=1 << 24):
        ids = np.zeros(max_done, np.uint64)
        counts = np.zeros(max_done, np.uint64)
        lat = np.zeros(max_done, np.uint64)
        res = np.zeros(results_cap, np.uint32)
        roffs = np.zeros(max_done + 1, np.uint64)
        done = ctypes.c_uint32(0)
        _check(require_library().s4_server_poll(self.h, _ptr(ids, ctypes.c_uint64), _ptr(counts, ctypes.c_uint64),
                                                _ptr(lat, ctypes.c_uint64), _ptr(res, ctypes.c_uint32), results_cap,
                                                _ptr(roffs, ctypes.c_uint64), max_done, ctypes.byref(done)),
               "s4_server_poll")
        d = done.value
        out = []
        for i in range(d):
            out.append((int(ids[i]), res[int(roffs[i]): int(roffs[i + 1])].copy(), int(lat[i])))
        return out

    def replay(self, terms, q_offsets, arrival_ns, with_results=False, results_cap=1 << 26, timeout_s=600.0,
               keep=None):
        """Open-loop replay of an arrival trace (s4_server_replay); with
        keep (bool per query) only those queries' results are returned."""
        terms = np.ascontiguousarray(terms, dtype=np.uint32)
        q_offsets = np.ascontiguousarray(q_offsets, dtype=np.uint64)
        arrival_ns = np.ascontiguousarray(arrival_ns, dtype=np.uint64)
        nq = q_offsets.size - 1
        lat = np.zeros(max(1, nq), np.uint64)
        counts = np.zeros(max(1, nq), np.uint64)
        res = np.zeros(results_cap if with_results else 1, np.uint32)
        roffs = np.zeros(nq + 1, np.uint64)
        el = ctypes.c_double(0)
        kp = None
        if keep is not None:
            keep = np.ascontiguousarray(keep, dtype=np.uint8)
            if keep.size != nq:
                raise ValueError("keep needs one entry per query")
            kp = _ptr(keep if keep.size else np.zeros(1, np.uint8), ctypes.c_uint8)
        _check(require_library().s4_server_replay(
            self.h, _ptr(terms if terms.size else np.zeros(1, np.uint32), ctypes.c_uint32),
            _ptr(q_offsets, ctypes.c_uint64), nq, _ptr(arrival_ns, ctypes.c_uint64), _ptr(lat, ctypes.c_uint64),
            _ptr(counts, ctypes.c_uint64), _ptr(res, ctypes.c_uint32) if with_results else None,
            results_cap if with_results else 0, _ptr(roffs, ctypes.c_uint64), kp, timeout_s, ctypes.byref(el)),
            "s4_server_replay")
        out = {"latency_ns": lat[:nq], "counts": counts[:nq], "elapsed_s": el.value}
        if with_results:
            out["results"] = res
            out["res_offsets"] = roffs
        return out

    def stats(self):
        st = ServerStats()
        _check(require_library().s4_server_stats_get(self.h, ctypes.byref(st)), "s4_server_stats_get")
        return st.as_dict()

    def close(self):
        if self.h:
            _check(require_library().s4_server_destroy(self.h), "s4_server_destroy")
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
