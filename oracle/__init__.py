"""CPU oracle for multi-pattern exact matching -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package. The GPU library never imports, links or calls it,
and it shares no code with the GPU library.

Contents:
  * ``ac_oracle.c``: Aho-Corasick with failure links (the paper's Sec. II.A) and
    the failure-less per-start-position walk (Sec. II.B / IV.A), in plain C,
    loaded here through ctypes.
  * ``naive.py``: the definition of the match set written out as a brute-force
    double loop, for tiny inputs.

Every result is an ascending ``numpy.uint64`` array of keys ``(e << 32) | k``:
pattern ``k`` (its index in the input list) ends at text position ``e``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ac_oracle.c")
_LIB_DIR = os.path.join(_HERE, "_build")
_LIB = os.path.join(_LIB_DIR, "libacoracle.so")

_u8p = ctypes.POINTER(ctypes.c_uint8)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_i32p = ctypes.POINTER(ctypes.c_int32)


def compile_source(src: str, out: str) -> str:
    """gcc -O2 a C file of the oracle into a shared library at ``out``."""
    os.makedirs(os.path.dirname(out), exist_ok=True)
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.run(["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-shared", "-fPIC",
                    "-o", tmp, src], check=True)
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    """Compile ac_oracle.c with gcc into oracle/_build/libacoracle.so."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    return compile_source(_SRC, _LIB)


_lib = None


def load_library(path: str):
    """ctypes handle with the oracle's signatures declared."""
    lib = ctypes.CDLL(path)
    lib.oracle_ac_build.restype = ctypes.c_void_p
    lib.oracle_ac_build.argtypes = [_u8p, _u64p, ctypes.c_uint32]
    lib.oracle_ac_free.argtypes = [ctypes.c_void_p]
    lib.oracle_ac_states.restype = ctypes.c_int32
    lib.oracle_ac_states.argtypes = [ctypes.c_void_p]
    lib.oracle_ac_m_max.restype = ctypes.c_int32
    lib.oracle_ac_m_max.argtypes = [ctypes.c_void_p]
    lib.oracle_ac_fail.restype = ctypes.c_int32
    lib.oracle_ac_fail.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    lib.oracle_ac_goto.restype = ctypes.c_int32
    lib.oracle_ac_goto.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32]
    lib.oracle_ac_scan.restype = ctypes.c_int64
    lib.oracle_ac_scan.argtypes = [ctypes.c_void_p, _u8p, ctypes.c_uint64,
                                   ctypes.POINTER(_u64p), _i32p]
    lib.oracle_pfac_scan.restype = ctypes.c_int64
    lib.oracle_pfac_scan.argtypes = [ctypes.c_void_p, _u8p, ctypes.c_uint64,
                                     ctypes.POINTER(_u64p)]
    lib.oracle_pfac_walk.restype = ctypes.c_int64
    lib.oracle_pfac_walk.argtypes = [ctypes.c_void_p, _u8p, ctypes.c_uint64,
                                     ctypes.c_uint64, _i32p, ctypes.c_int64]
    lib.oracle_buf_free.argtypes = [_u64p]
    return lib


def _load():
    global _lib
    if _lib is None:
        _lib = load_library(build(force=False))
    return _lib


def _as_u8(text) -> np.ndarray:
    if isinstance(text, (bytes, bytearray, memoryview)):
        return np.frombuffer(bytes(text), dtype=np.uint8)
    a = np.ascontiguousarray(text, dtype=np.uint8)
    return a


def _ptr(a: np.ndarray, t=_u8p):
    if a.size == 0:
        a = np.zeros(1, dtype=a.dtype)
    return a.ctypes.data_as(t), a


class OracleAC:
    """The Aho-Corasick machine of a pattern list (ids = list positions)."""

    def __init__(self, patterns, lib=None):
        pats = [bytes(p) for p in patterns]
        lib = lib if lib is not None else _load()
        self._lib = lib
        off = np.zeros(len(pats) + 1, dtype=np.uint64)
        off[1:] = np.cumsum([len(p) for p in pats], dtype=np.uint64) if pats else []
        data = np.frombuffer(b"".join(pats) or b"\0", dtype=np.uint8).copy()
        self._h = lib.oracle_ac_build(data.ctypes.data_as(_u8p), off.ctypes.data_as(_u64p),
                                      len(pats))
        if not self._h:
            raise ValueError("oracle: empty pattern list, empty pattern or out of memory")
        self.n_patterns = len(pats)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and getattr(self, "_lib", None) is not None:
            self._lib.oracle_ac_free(h)
            self._h = None

    @property
    def n_states(self) -> int:
        return self._lib.oracle_ac_states(self._h)

    @property
    def m_max(self) -> int:
        return self._lib.oracle_ac_m_max(self._h)

    def fail(self, s: int) -> int:
        return self._lib.oracle_ac_fail(self._h, s)

    def goto(self, s: int, a: int) -> int:
        return self._lib.oracle_ac_goto(self._h, s, a)

    def _take(self, res, n) -> np.ndarray:
        if n < 0:
            raise MemoryError("oracle: out of memory")
        if n == 0:
            if res:
                self._lib.oracle_buf_free(res)
            return np.zeros(0, dtype=np.uint64)
        out = np.ctypeslib.as_array(res, shape=(n,)).copy()
        self._lib.oracle_buf_free(res)
        return out

    def scan(self, text) -> np.ndarray:
        """All matches, via failure links (Sec. II.A); sorted keys."""
        a = _as_u8(text)
        t, keep = _ptr(a)
        res = _u64p()
        n = self._lib.oracle_ac_scan(self._h, t, a.size, ctypes.byref(res), None)
        return np.sort(self._take(res, n))

    def trace(self, text) -> list[int]:
        """The state after each byte of a failure-link scan."""
        a = _as_u8(text)
        t, keep = _ptr(a)
        tr = np.zeros(max(1, a.size), dtype=np.int32)
        res = _u64p()
        n = self._lib.oracle_ac_scan(self._h, t, a.size, ctypes.byref(res), tr.ctypes.data_as(_i32p))
        self._take(res, n)
        return tr[:a.size].tolist()

    def pfac_scan(self, text) -> np.ndarray:
        """All matches, via a failure-less walk from every start (Sec. IV.A)."""
        a = _as_u8(text)
        t, keep = _ptr(a)
        res = _u64p()
        n = self._lib.oracle_pfac_scan(self._h, t, a.size, ctypes.byref(res))
        return np.sort(self._take(res, n))

    def pfac_walk(self, text, p: int) -> list[int]:
        """States entered by the failure-less walk started at position p."""
        a = _as_u8(text)
        t, keep = _ptr(a)
        cap = self.m_max + 1
        st = np.zeros(cap, dtype=np.int32)
        n = self._lib.oracle_pfac_walk(self._h, t, a.size, p, st.ctypes.data_as(_i32p), cap)
        return st[:min(n, cap)].tolist()


def oracle_match(text, patterns) -> np.ndarray:
    """Sorted (e << 32) | k keys of every occurrence, via failure-link AC."""
    return OracleAC(patterns).scan(text)


def window_matches(ac: OracleAC, text: np.ndarray, lo: int, hi: int) -> np.ndarray:
    """Matches whose end position lies in [lo, hi), computed by scanning only
    text[max(0, lo - m_max + 1) : hi]: an occurrence ending at e >= lo starts
    at e - len + 1 >= lo - m_max + 1, so it lies wholly inside that slice."""
    start = max(0, lo - ac.m_max + 1)
    keys = ac.scan(text[start:hi])
    ends = (keys >> np.uint64(32)) + np.uint64(start)
    ids = keys & np.uint64(0xFFFFFFFF)
    keep = ends >= np.uint64(lo)
    return (ends[keep] << np.uint64(32)) | ids[keep]


def split_keys(keys: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    keys = np.asarray(keys, dtype=np.uint64)
    return (keys >> np.uint64(32)).astype(np.int64), (keys & np.uint64(0xFFFFFFFF)).astype(np.int64)
