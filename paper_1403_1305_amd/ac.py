"""ctypes binding of libac.so (include/ac.h), one Python function per C entry point.

Arguments are marshalled only: device buffers may be torch tensors (their
``data_ptr()``) or integer addresses, streams may be ``torch.cuda.Stream``
objects, raw integer handles or None (torch's current stream). Every step of
the scan runs in the library's HIP kernels; there is no Python or CPU path.
A failing call raises ``AcError`` carrying the library's status and message.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch  # torch's HIP runtime must be the one libac.so binds to: load it first

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libac.so")

AC_OK = 0
AC_ERR_INVALID = -1
AC_ERR_NOMEM = -2
AC_ERR_TOO_LARGE = -3
AC_ERR_OVERFLOW = -4
AC_ERR_HIP = -5
AC_ERR_BUSY = -6

AC_PLACE_AUTO = 0
AC_PLACE_GLOBAL = 1
AC_PLACE_LDS_FULL = 2
AC_PLACE_LDS_HOT = 3

AC_ALGO_AUTO = 0
AC_ALGO_DFA = 1
AC_ALGO_PFAC = 2
AC_ALGO_GATED = 3

AC_BUILD_GOTO_ONLY = 1
AC_BUILD_PAIR_ROWS = 2
AC_BUILD_NO_GATE = 4
AC_PAIR_AUTO, AC_PAIR_OFF = 0, 1

AC_TABLE_DFA, AC_TABLE_GO, AC_TABLE_OUT_OFF, AC_TABLE_OUT_IDS, AC_TABLE_OWN_OFF, \
    AC_TABLE_OWN_IDS, AC_TABLE_HOT_DFA, AC_TABLE_HOT_GO, AC_TABLE_CMAP, AC_TABLE_PAIR, \
    AC_TABLE_GATE_BITS, AC_TABLE_GATE_NODE, AC_TABLE_PATH_OFF, AC_TABLE_PATH_IDS, \
    AC_TABLE_GATE2_BITS, AC_TABLE_QGATE_BITS, AC_TABLE_QGATE_TAB, AC_TABLE_OWN_ONE, \
    AC_TABLE_PATH_ONE = range(19)

_TABLE_DTYPE = {AC_TABLE_HOT_DFA: np.uint16, AC_TABLE_HOT_GO: np.uint16, AC_TABLE_CMAP: np.uint8}


class AcError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"[{status}] {message}")
        self.status = status
        self.message = message


class ac_build_opts(ctypes.Structure):
    _fields_ = [("placement", ctypes.c_uint32), ("hot_states", ctypes.c_uint32),
                ("lds_bytes", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("threads", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class ac_info_t(ctypes.Structure):
    _fields_ = [("n_states", ctypes.c_uint64), ("n_patterns", ctypes.c_uint32),
                ("sigma", ctypes.c_uint32), ("n_cols", ctypes.c_uint32),
                ("m_max", ctypes.c_uint32), ("placement", ctypes.c_uint32),
                ("hot_states", ctypes.c_uint32), ("class_shift", ctypes.c_uint32),
                ("class_hashed", ctypes.c_uint32), ("table_bytes", ctypes.c_uint64),
                ("out_entries", ctypes.c_uint64), ("build_ms", ctypes.c_double),
                ("goto_only", ctypes.c_uint32), ("pair_states", ctypes.c_uint32),
                ("has_gate", ctypes.c_uint32), ("gate_pass", ctypes.c_double),
                ("match_rate", ctypes.c_double)]


class ac_scan_opts(ctypes.Structure):
    _fields_ = [("algo", ctypes.c_uint32), ("chunk", ctypes.c_uint32),
                ("block", ctypes.c_uint32), ("placement", ctypes.c_uint32),
                ("walkers", ctypes.c_uint32), ("block_bytes", ctypes.c_uint32),
                ("pair_steps", ctypes.c_uint32), ("append", ctypes.c_uint32)]


class ac_batch_tune(ctypes.Structure):
    _fields_ = [("placement", ctypes.c_uint32), ("walkers", ctypes.c_uint32),
                ("chunk", ctypes.c_uint32), ("algo", ctypes.c_uint32)]


class ac_batch_info_t(ctypes.Structure):
    _fields_ = [("placement", ctypes.c_uint32), ("walkers", ctypes.c_uint32),
                ("block_bytes", ctypes.c_uint32), ("chunk", ctypes.c_uint32),
                ("threads", ctypes.c_uint32), ("grid", ctypes.c_uint32),
                ("n_items", ctypes.c_uint32), ("n_tasks", ctypes.c_uint32),
                ("text_bytes", ctypes.c_uint64), ("algo", ctypes.c_uint32), ("pad", ctypes.c_uint32)]


class ac_serve_opts(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_uint64), ("max_inflight", ctypes.c_uint32),
                ("piece_bytes", ctypes.c_uint32), ("match_ppm", ctypes.c_uint32),
                ("flags", ctypes.c_uint32), ("max_large", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class ac_serve_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("automaton", ctypes.c_uint32), ("n", ctypes.c_uint64),
                ("d_matches", ctypes.c_void_p), ("n_matches", ctypes.c_uint64),
                ("t_submit_ns", ctypes.c_uint64), ("t_admit_ns", ctypes.c_uint64),
                ("t_done_ns", ctypes.c_uint64), ("pieces", ctypes.c_uint32), ("rescans", ctypes.c_uint32)]


class ac_serve_stats_t(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint64) for k in ("submitted", "completed", "failed", "queued", "running",
                                               "rescans", "pool_bytes", "pool_used", "pool_peak",
                                               "running_peak", "bytes_done")] + \
               [("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double), ("gbps", ctypes.c_double)]


_vp = ctypes.c_void_p
_u64 = ctypes.c_uint64
_u32 = ctypes.c_uint32

# name -> (restype, argtypes); every symbol include/ac.h declares
SIGNATURES = {
    "ac_build": (ctypes.c_int, [_vp, _vp, _u32, ctypes.POINTER(ac_build_opts), _vp,
                                ctypes.POINTER(_vp)]),
    "ac_build_host": (ctypes.c_int, [_vp, _vp, _u32, ctypes.POINTER(ac_build_opts),
                                     ctypes.POINTER(_vp)]),
    "ac_get_table": (ctypes.c_int, [_vp, _u32, _vp, _u64, ctypes.POINTER(_u64)]),
    "ac_free": (None, [_vp]),
    "ac_info": (ctypes.c_int, [_vp, ctypes.POINTER(ac_info_t)]),
    "ac_scan": (ctypes.c_int, [_vp, _vp, _u64, _vp, _u64, _vp, ctypes.POINTER(ac_scan_opts), _vp]),
    "ac_scan_sync": (ctypes.c_int, [_vp, _vp, _u64, _vp, _u64, _vp, ctypes.POINTER(ac_scan_opts),
                                    _vp, ctypes.POINTER(_u64)]),
    "ac_scan_stream": (ctypes.c_int, [_vp, _vp, _u64, _u64, _vp, _vp, _vp, _u64, _vp, ctypes.c_int,
                                      ctypes.POINTER(ac_scan_opts), _vp]),
    "ac_sort_scratch_bytes": (_u64, [_u64]),
    "ac_sort_matches": (ctypes.c_int, [_vp, _u64, _vp, _u64, _vp]),
    "ac_hbm_read": (ctypes.c_int, [_vp, _u64, _vp, _u32, _vp]),
    "ac_hbm_copy": (ctypes.c_int, [_vp, _vp, _u64, _u32, _vp]),
    "ac_batch_create": (ctypes.c_int, [_vp, _u32, _vp, _vp, _vp, _u32, ctypes.POINTER(ac_batch_tune),
                                       _vp, ctypes.POINTER(_vp)]),
    "ac_batch_info": (ctypes.c_int, [_vp, ctypes.POINTER(ac_batch_info_t)]),
    "ac_batch_scan": (ctypes.c_int, [_vp, _vp, _vp, _u64, _vp, ctypes.c_int, _vp]),
    "ac_batch_free": (None, [_vp]),
    "ac_scan_batch": (ctypes.c_int, [_vp, _u32, _vp, _vp, _vp, _u32, _vp, _vp, _u64, _vp,
                                     ctypes.POINTER(ac_batch_tune), _vp]),
    "ac_scan_batch_noalloc": (ctypes.c_int, [_vp, _u32, _vp, _vp, _vp, _u32, _vp, _vp, _u64, _vp,
                                             ctypes.POINTER(ac_batch_tune), _vp]),
    "ac_serve_create": (ctypes.c_int, [_vp, _u32, ctypes.POINTER(ac_serve_opts), ctypes.POINTER(_vp)]),
    "ac_serve_add": (ctypes.c_int, [_vp, _vp, ctypes.POINTER(_u32)]),
    "ac_serve_submit": (ctypes.c_int, [_vp, _u32, _vp, _u64, ctypes.c_int, _u64, ctypes.POINTER(_u64)]),
    "ac_serve_now_ns": (_u64, [_vp]),
    "ac_serve_wait": (ctypes.c_int, [_vp, _u64, ctypes.c_int64, ctypes.POINTER(ac_serve_result)]),
    "ac_serve_release": (ctypes.c_int, [_vp, _u64]),
    "ac_serve_stats": (ctypes.c_int, [_vp, ctypes.POINTER(ac_serve_stats_t)]),
    "ac_serve_destroy": (None, [_vp]),
    "ac_last_error": (ctypes.c_char_p, []),
}

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libac.so (raising if it is not built) and declare its signatures."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: build it with "
                              "`python -m paper_1403_1305_amd.build_lib` (or __graft_entry__.build())")
        lib = ctypes.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(rc: int):
    if rc != AC_OK:
        raise AcError(rc, (_lib.ac_last_error() or b"").decode())


def _ptr(x) -> int | None:
    if x is None:
        return None
    if isinstance(x, torch.Tensor):
        return x.data_ptr()
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    return int(x)


def _stream(s) -> int | None:
    if s is None:
        return torch.cuda.current_stream().cuda_stream if torch.cuda.is_available() else None
    if isinstance(s, torch.cuda.Stream):
        return s.cuda_stream
    return int(s)


def patterns_csr(patterns) -> tuple[np.ndarray, np.ndarray]:
    """Concatenated pattern bytes (uint8) and n+1 offsets (uint64)."""
    pats = [bytes(p) for p in patterns]
    off = np.zeros(len(pats) + 1, dtype=np.uint64)
    if pats:
        off[1:] = np.cumsum([len(p) for p in pats], dtype=np.uint64)
    data = np.frombuffer(b"".join(pats) or b"\0", dtype=np.uint8).copy()
    return data, off


class Automaton:
    """Owning handle of an ac_automaton*; freed with ac_free."""

    def __init__(self, handle: int, on_device: bool):
        self.handle = handle
        self.on_device = on_device

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.ac_free(self.handle)
            self.handle = None

    @property
    def _as_parameter_(self):
        return ctypes.c_void_p(self.handle)


def _opts(placement=AC_PLACE_AUTO, hot_states=0, lds_bytes=0, flags=0, threads=0):
    return ac_build_opts(placement, hot_states, lds_bytes, flags, threads, 0)


def ac_build(pat_bytes, pat_off, n_patterns: int | None = None, opts: ac_build_opts | None = None,
             stream=None) -> Automaton:
    lib = load_library()
    pat_bytes = np.ascontiguousarray(pat_bytes, dtype=np.uint8)
    pat_off = np.ascontiguousarray(pat_off, dtype=np.uint64)
    n = len(pat_off) - 1 if n_patterns is None else n_patterns
    h = _vp()
    _check(lib.ac_build(pat_bytes.ctypes.data, pat_off.ctypes.data, n,
                        ctypes.byref(opts) if opts is not None else None, _stream(stream),
                        ctypes.byref(h)))
    return Automaton(h.value, True)


def ac_build_host(pat_bytes, pat_off, n_patterns: int | None = None,
                  opts: ac_build_opts | None = None) -> Automaton:
    lib = load_library()
    pat_bytes = np.ascontiguousarray(pat_bytes, dtype=np.uint8)
    pat_off = np.ascontiguousarray(pat_off, dtype=np.uint64)
    n = len(pat_off) - 1 if n_patterns is None else n_patterns
    h = _vp()
    _check(lib.ac_build_host(pat_bytes.ctypes.data, pat_off.ctypes.data, n,
                             ctypes.byref(opts) if opts is not None else None, ctypes.byref(h)))
    return Automaton(h.value, False)


def ac_free(a: Automaton):
    if a.handle:
        load_library().ac_free(a.handle)
        a.handle = None


def ac_info(a: Automaton) -> dict:
    info = ac_info_t()
    _check(load_library().ac_info(a.handle, ctypes.byref(info)))
    return {name: getattr(info, name) for name, _ in ac_info_t._fields_}


def ac_get_table(a: Automaton, which: int) -> np.ndarray:
    lib = load_library()
    size = _u64()
    _check(lib.ac_get_table(a.handle, which, None, 0, ctypes.byref(size)))
    dt = _TABLE_DTYPE.get(which, np.uint32)
    out = np.zeros(max(1, size.value // np.dtype(dt).itemsize), dtype=dt)
    _check(lib.ac_get_table(a.handle, which, out.ctypes.data, out.nbytes, ctypes.byref(size)))
    return out[: size.value // np.dtype(dt).itemsize]


def _scan_opts(algo=AC_ALGO_DFA, chunk=0, block=0, placement=0, walkers=0, block_bytes=0, pair_steps=0, append=0):
    return ac_scan_opts(algo, chunk, block, placement, walkers, block_bytes, pair_steps, append)


def ac_scan(a: Automaton, d_text, n: int, d_matches, capacity: int, d_count,
            opts: ac_scan_opts | None = None, stream=None) -> None:
    _check(load_library().ac_scan(a.handle, _ptr(d_text), n, _ptr(d_matches), capacity,
                                  _ptr(d_count), ctypes.byref(opts) if opts is not None else None,
                                  _stream(stream)))


def ac_scan_sync(a: Automaton, d_text, n: int, d_matches, capacity: int, d_count,
                 opts: ac_scan_opts | None = None, stream=None) -> int:
    """Returns the total match count; raises AcError(AC_ERR_OVERFLOW) if it
    exceeds capacity (the error carries the count in its message)."""
    h = _u64()
    _check(load_library().ac_scan_sync(a.handle, _ptr(d_text), n, _ptr(d_matches), capacity,
                                       _ptr(d_count),
                                       ctypes.byref(opts) if opts is not None else None,
                                       _stream(stream), ctypes.byref(h)))
    return h.value


def ac_scan_stream(a: Automaton, d_text, n: int, base: int, d_state_in, d_state_out, d_matches,
                   capacity: int, d_count, append: bool = False, opts: ac_scan_opts | None = None,
                   stream=None) -> None:
    _check(load_library().ac_scan_stream(a.handle, _ptr(d_text), n, base, _ptr(d_state_in),
                                         _ptr(d_state_out), _ptr(d_matches), capacity, _ptr(d_count),
                                         int(bool(append)),
                                         ctypes.byref(opts) if opts is not None else None,
                                         _stream(stream)))


def ac_sort_scratch_bytes(count: int) -> int:
    return load_library().ac_sort_scratch_bytes(count)


def ac_sort_matches(d_keys, count: int, d_tmp, tmp_bytes: int, stream=None) -> None:
    _check(load_library().ac_sort_matches(_ptr(d_keys), count, _ptr(d_tmp), tmp_bytes,
                                          _stream(stream)))


class Batch:
    """Owning handle of an ac_batch* plan (keeps its automata alive)."""

    def __init__(self, handle: int, autos):
        self.handle = handle
        self.autos = list(autos)

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.ac_batch_free(self.handle)
            self.handle = None


def ac_batch_create(autos, text_off, text_len, text_auto, tune: ac_batch_tune | None = None,
                    stream=None) -> Batch:
    lib = load_library()
    arr = (ctypes.c_void_p * len(autos))(*[a.handle for a in autos])
    off = np.ascontiguousarray(text_off, dtype=np.uint64)
    ln = np.ascontiguousarray(text_len, dtype=np.uint64)
    au = np.ascontiguousarray(text_auto, dtype=np.uint32)
    h = _vp()
    _check(lib.ac_batch_create(arr, len(autos), off.ctypes.data, ln.ctypes.data, au.ctypes.data,
                               len(off), ctypes.byref(tune) if tune is not None else None,
                               _stream(stream), ctypes.byref(h)))
    return Batch(h.value, autos)


def ac_batch_info(b: Batch) -> dict:
    info = ac_batch_info_t()
    _check(load_library().ac_batch_info(b.handle, ctypes.byref(info)))
    return {name: getattr(info, name) for name, _ in ac_batch_info_t._fields_}


def ac_batch_scan(b: Batch, d_texts, d_matches, capacity: int, d_count, use_graph: bool = False,
                  stream=None) -> None:
    _check(load_library().ac_batch_scan(b.handle, _ptr(d_texts), _ptr(d_matches), capacity,
                                        _ptr(d_count), int(bool(use_graph)), _stream(stream)))


def ac_batch_free(b: Batch) -> None:
    if b.handle:
        load_library().ac_batch_free(b.handle)
        b.handle = None


class Server:
    """Owning handle of an ac_server* (keeps its automata alive)."""

    def __init__(self, autos, hbm_budget: int = 0, max_inflight: int = 0, piece_bytes: int = 0,
                 match_ppm: int = 0, flags: int = 0, max_large: int = 0):
        lib = load_library()
        self.autos = list(autos)
        self._texts = {}  # ticket -> the submitted text object, alive until release
        arr = (ctypes.c_void_p * len(self.autos))(*[a.handle for a in self.autos])
        o = ac_serve_opts(hbm_budget, max_inflight, piece_bytes, match_ppm, flags, max_large, 0)
        h = _vp()
        _check(lib.ac_serve_create(arr, len(self.autos), ctypes.byref(o), ctypes.byref(h)))
        self.handle = h.value

    def submit(self, automaton: int, text, n: int | None = None, on_device: bool | None = None,
               arrival_ns: int = 0) -> int:
        """Queue a scan; `text` is a uint8 torch tensor (device or host) or a
        numpy array (host); `arrival_ns` schedules its arrival on the server's
        clock (0 = now). Returns the ticket."""
        if isinstance(text, torch.Tensor):
            n = text.numel() if n is None else n
            on_device = text.is_cuda if on_device is None else on_device
        elif isinstance(text, np.ndarray):
            n = text.size if n is None else n
            on_device = False
        t = _u64()
        _check(load_library().ac_serve_submit(self.handle, automaton, _ptr(text), n, int(bool(on_device)),
                                              arrival_ns, ctypes.byref(t)))
        self._texts[t.value] = text  # the server reads it until the request is done
        return t.value

    def add(self, automaton: Automaton) -> int:
        """Make another automaton resident; returns its index."""
        i = _u32()
        _check(load_library().ac_serve_add(self.handle, automaton.handle, ctypes.byref(i)))
        self.autos.append(automaton)
        return i.value

    def now_ns(self) -> int:
        return load_library().ac_serve_now_ns(self.handle)

    def wait(self, ticket: int, timeout_ms: int = -1) -> ac_serve_result:
        r = ac_serve_result()
        _check(load_library().ac_serve_wait(self.handle, ticket, timeout_ms, ctypes.byref(r)))
        return r

    @staticmethod
    def keys_tensor(res: ac_serve_result) -> torch.Tensor:
        """The request's match keys as an int64 device tensor that aliases the
        server's list (bit pattern of the uint64 keys; valid until release)."""
        n = int(res.n_matches)
        if n == 0:
            return torch.empty(0, dtype=torch.int64, device="cuda")

        class _View:
            __cuda_array_interface__ = {"shape": (n,), "typestr": "<i8", "data": (int(res.d_matches), False),
                                        "version": 2, "strides": None}

        return torch.as_tensor(_View(), device="cuda")

    def keys(self, res: ac_serve_result) -> np.ndarray:
        """The request's match keys copied to the host (unordered)."""
        return keys_to_numpy(self.keys_tensor(res)).copy()

    def release(self, ticket: int) -> None:
        _check(load_library().ac_serve_release(self.handle, ticket))
        self._texts.pop(ticket, None)

    def stats(self) -> dict:
        st = ac_serve_stats_t()
        _check(load_library().ac_serve_stats(self.handle, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in ac_serve_stats_t._fields_}

    def close(self) -> None:
        if getattr(self, "handle", None) and _lib is not None:
            _lib.ac_serve_destroy(self.handle)
            self.handle = None
            self._texts = {}

    __del__ = close


def _scan_batch(fn: str, autos, d_texts, d_text_off, d_text_auto, d_matches, capacity: int, d_count,
                d_match_text=None, tune: ac_batch_tune | None = None, stream=None) -> None:
    lib = load_library()
    arr = (ctypes.c_void_p * len(autos))(*[a.handle for a in autos])
    n_texts = int(d_text_auto.numel()) if isinstance(d_text_auto, torch.Tensor) else len(d_text_auto)
    _check(getattr(lib, fn)(arr, len(autos), _ptr(d_texts), _ptr(d_text_off), _ptr(d_text_auto), n_texts,
                            _ptr(d_match_text), _ptr(d_matches), capacity, _ptr(d_count),
                            ctypes.byref(tune) if tune is not None else None, _stream(stream)))


def ac_scan_batch(autos, d_texts, d_text_off, d_text_auto, d_matches, capacity: int, d_count,
                  d_match_text=None, tune: ac_batch_tune | None = None, stream=None) -> None:
    """One-shot batch; the descriptors are device tensors: d_text_off (int64,
    n_texts + 1, text t is bytes [off[t], off[t+1]) of d_texts) and
    d_text_auto (int32, n_texts). d_match_text (int32, capacity) receives
    each key's text index when given."""
    _scan_batch("ac_scan_batch", autos, d_texts, d_text_off, d_text_auto, d_matches, capacity, d_count,
                d_match_text, tune, stream)


def ac_scan_batch_noalloc(autos, d_texts, d_text_off, d_text_auto, d_matches, capacity: int, d_count,
                          d_match_text=None, tune: ac_batch_tune | None = None, stream=None) -> None:
    """ac_scan_batch with the plan in the library's fixed scratch array (no
    device allocation; at most 65,536 texts; calls on one GPU must not overlap)."""
    _scan_batch("ac_scan_batch_noalloc", autos, d_texts, d_text_off, d_text_auto, d_matches, capacity, d_count,
                d_match_text, tune, stream)


def ac_hbm_read(d, n: int, d_fold, blocks: int = 0, stream=None) -> None:
    """Stream n bytes of device tensor d once, XOR-folding 32-bit words into
    d_fold (one int64 element); its time is the HBM read ceiling."""
    _check(load_library().ac_hbm_read(_ptr(d), n, _ptr(d_fold), blocks, _stream(stream)))


def ac_hbm_copy(dst, src, n: int, blocks: int = 0, stream=None) -> None:
    """Copy n bytes between device tensors with the scans' load shape (a
    kernel of known traffic for scaling byte counters)."""
    _check(load_library().ac_hbm_copy(_ptr(dst), _ptr(src), n, blocks, _stream(stream)))


def pack_texts(texts, align: int = 16) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Concatenate host texts into one buffer, each starting at a multiple of
    `align`; returns (buffer uint8, offsets uint64, lengths uint64)."""
    lens = np.array([len(t) for t in texts], dtype=np.uint64)
    offs = np.zeros(len(texts), dtype=np.uint64)
    pos = 0
    for i, t in enumerate(texts):
        offs[i] = pos
        pos += (len(t) + align - 1) // align * align
    buf = np.zeros(max(align, pos), dtype=np.uint8)
    for i, t in enumerate(texts):
        buf[int(offs[i]):int(offs[i]) + len(t)] = np.frombuffer(bytes(t), dtype=np.uint8) \
            if isinstance(t, (bytes, bytearray)) else t
    return buf, offs, lens


def ac_last_error() -> str:
    return (load_library().ac_last_error() or b"").decode()


# ---------------------------------------------------------------- conveniences

def scan_text(a: Automaton, d_text: torch.Tensor, capacity: int | None = None,
              opts: ac_scan_opts | None = None, stream=None) -> torch.Tensor:
    """Scan a 1-D uint8 device tensor; returns the match keys as an int64
    device tensor (bit pattern of the uint64 keys), in unspecified order. The
    output buffer is sized by ``capacity`` and regrown once on overflow."""
    n = d_text.numel()
    dev = d_text.device
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    cap = capacity if capacity is not None else max(1024, n // 256)
    for _ in range(2):
        out = torch.empty(max(1, cap), dtype=torch.int64, device=dev)
        try:
            total = ac_scan_sync(a, d_text, n, out, cap, count, opts, stream)
            return out[:total]
        except AcError as e:
            if e.status != AC_ERR_OVERFLOW:
                raise
            cap = int(count.item())
    raise AcError(AC_ERR_OVERFLOW, "match count changed between two scans")


def sort_keys(keys: torch.Tensor, stream=None) -> torch.Tensor:
    """Sort int64-stored uint64 keys ascending in place on the device."""
    n = keys.numel()
    if n > 1:
        tmp = torch.empty(ac_sort_scratch_bytes(n), dtype=torch.uint8, device=keys.device)
        ac_sort_matches(keys, n, tmp, tmp.numel(), stream)
    return keys


def keys_to_numpy(keys: torch.Tensor) -> np.ndarray:
    return keys.cpu().numpy().view(np.uint64)
