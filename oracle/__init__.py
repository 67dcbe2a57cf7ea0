"""CPU oracle for the kernel-actor pipelines (TEST INFRASTRUCTURE ONLY).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg use
this package.  It wraps ``liboracle.so`` (built from ``oracle.cpp`` by
``oracle/build.py``) with numpy marshalling and shares nothing with the HIP
implementation.  See ``oracle.cpp`` for the paper passages each function
follows and the word conventions.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_U32P = ctypes.POINTER(ctypes.c_uint32)
_U64P = ctypes.POINTER(ctypes.c_uint64)
_lib_cache: dict[str, ctypes.CDLL] = {}


def load(path: str | None = None) -> ctypes.CDLL:
    """Load the oracle library (building it on first use if absent)."""
    path = path or _build.LIB
    if path in _lib_cache:
        return _lib_cache[path]
    if not os.path.exists(path):
        if path != _build.LIB:
            raise FileNotFoundError(path)
        _build.build()
    lib = ctypes.CDLL(path)
    for name, argt in {
        "ora_sort_pairs": [_U32P, _U32P, ctypes.c_uint64, _U32P, _U32P],
        "ora_wah_groups": [_U32P, _U32P, ctypes.c_uint64, _U32P, _U32P, _U32P, _U64P],
        "ora_wah_fills": [_U32P, _U32P, ctypes.c_uint64, _U32P],
        "ora_wah_interleave": [_U32P, _U32P, ctypes.c_uint64, _U32P],
        "ora_compact_nonzero": [_U32P, ctypes.c_uint64, _U32P, _U64P],
        "ora_wah_table": [_U32P, _U32P, ctypes.c_uint64, _U32P, _U32P, _U64P],
        "ora_wah_index": [_U32P, ctypes.c_uint64, _U32P, _U32P, _U32P, _U64P, _U64P],
        "ora_wah_encode_sorted": [_U32P, _U32P, ctypes.c_uint64, _U32P, _U32P, _U32P, _U64P, _U64P],
        "ora_wah_encode_groups": [_U32P, _U32P, _U32P, ctypes.c_uint64, ctypes.c_uint32, _U32P, _U32P, _U32P,
                                  _U64P, _U64P],
        "ora_wah_index_format": [_U32P, ctypes.c_uint64, ctypes.c_uint32, _U32P, _U32P, _U32P, _U64P, _U64P],
        "ora_wah_lookup": [_U32P, ctypes.c_uint64, _U32P, ctypes.c_uint64, _U32P],
        "ora_wah_decode": [_U32P, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, _U32P],
        "ora_wah_combine": [_U32P, ctypes.c_uint64, _U32P, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64,
                            ctypes.c_uint32, ctypes.c_uint32, _U32P, _U64P],
        "ora_exclusive_scan": [_U32P, ctypes.c_uint64, _U32P],
        "ora_affine_chain": [_U32P, ctypes.c_uint64, _U32P, _U32P, ctypes.c_uint32],
    }.items():
        f = getattr(lib, name)
        f.argtypes = argt
        f.restype = ctypes.c_int
    _lib_cache[path] = lib
    return lib


def _p(a: np.ndarray | None):
    if a is None:
        return None
    assert a.dtype == np.uint32 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_U32P)


def _u32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint32))


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


class Oracle:
    """numpy front end of one oracle library build."""

    def __init__(self, path: str | None = None):
        self.lib = load(path)

    def sort_pairs(self, keys, rows=None):
        keys = _u32(keys)
        n = keys.size
        sk = np.empty(n, np.uint32)
        sr = np.empty(n, np.uint32)
        r = None if rows is None else _u32(rows)
        _check(self.lib.ora_sort_pairs(_p(keys), _p(r), n, _p(sk), _p(sr)), "sort_pairs")
        return sk, sr

    def wah_groups(self, skeys, srows):
        skeys, srows = _u32(skeys), _u32(srows)
        n = skeys.size
        gk, gc, gl = (np.empty(n, np.uint32) for _ in range(3))
        k = ctypes.c_uint64()
        _check(self.lib.ora_wah_groups(_p(skeys), _p(srows), n, _p(gk), _p(gc), _p(gl), ctypes.byref(k)),
               "wah_groups")
        k = k.value
        return gk[:k].copy(), gc[:k].copy(), gl[:k].copy()

    def wah_fills(self, gkey, gchunk):
        gkey, gchunk = _u32(gkey), _u32(gchunk)
        out = np.empty(gkey.size, np.uint32)
        _check(self.lib.ora_wah_fills(_p(gkey), _p(gchunk), gkey.size, _p(out)), "wah_fills")
        return out

    def wah_interleave(self, gfill, glit):
        gfill, glit = _u32(gfill), _u32(glit)
        out = np.empty(2 * gfill.size, np.uint32)
        _check(self.lib.ora_wah_interleave(_p(gfill), _p(glit), gfill.size, _p(out)), "wah_interleave")
        return out

    def compact_nonzero(self, x):
        x = _u32(x)
        out = np.empty(x.size, np.uint32)
        kept = ctypes.c_uint64()
        _check(self.lib.ora_compact_nonzero(_p(x), x.size, _p(out), ctypes.byref(kept)), "compact_nonzero")
        return out[: kept.value].copy()

    def wah_table(self, gkey, index):
        gkey, index = _u32(gkey), _u32(index)
        k = gkey.size
        keys = np.empty(max(k, 1), np.uint32)
        offs = np.empty(k + 1, np.uint32)
        D = ctypes.c_uint64()
        _check(self.lib.ora_wah_table(_p(gkey), _p(index), k, _p(keys), _p(offs), ctypes.byref(D)), "wah_table")
        return keys[: D.value].copy(), offs[: D.value + 1].copy()

    def wah_index(self, values):
        """Full index build.  Returns (keys[D], offsets[D+1], words[W])."""
        values = _u32(values)
        n = values.size
        keys = np.empty(max(n, 1), np.uint32)
        offs = np.empty(n + 1, np.uint32)
        words = np.empty(max(2 * n, 1), np.uint32)
        D, W = ctypes.c_uint64(), ctypes.c_uint64()
        _check(self.lib.ora_wah_index(_p(values), n, _p(keys), _p(offs), _p(words), ctypes.byref(D),
                                      ctypes.byref(W)), "wah_index")
        return keys[: D.value].copy(), offs[: D.value + 1].copy(), words[: W.value].copy()

    def wah_encode_sorted(self, skeys, srows):
        skeys, srows = _u32(skeys), _u32(srows)
        n = skeys.size
        keys = np.empty(max(n, 1), np.uint32)
        offs = np.empty(n + 1, np.uint32)
        words = np.empty(max(2 * n, 1), np.uint32)
        D, W = ctypes.c_uint64(), ctypes.c_uint64()
        _check(self.lib.ora_wah_encode_sorted(_p(skeys), _p(srows), n, _p(keys), _p(offs), _p(words),
                                              ctypes.byref(D), ctypes.byref(W)), "wah_encode_sorted")
        return keys[: D.value].copy(), offs[: D.value + 1].copy(), words[: W.value].copy()

    def wah_index_format(self, values, fmt: int):
        """Index build in an encoder format (0 paper form, 1 canonical WAH,
        2 PLWAH).  Returns (keys[D], offsets[D+1], words[W])."""
        values = _u32(values)
        n = values.size
        keys = np.empty(max(n, 1), np.uint32)
        offs = np.empty(n + 1, np.uint32)
        words = np.empty(max(2 * n, 1), np.uint32)
        D, W = ctypes.c_uint64(), ctypes.c_uint64()
        _check(self.lib.ora_wah_index_format(_p(values), n, fmt, _p(keys), _p(offs), _p(words), ctypes.byref(D),
                                             ctypes.byref(W)), "wah_index_format")
        return keys[: D.value].copy(), offs[: D.value + 1].copy(), words[: W.value].copy()

    def wah_encode_groups(self, gkey, gchunk, glit, fmt: int):
        gkey, gchunk, glit = _u32(gkey), _u32(gchunk), _u32(glit)
        k = gkey.size
        keys = np.empty(max(k, 1), np.uint32)
        offs = np.empty(k + 1, np.uint32)
        words = np.empty(max(2 * k, 1), np.uint32)
        D, W = ctypes.c_uint64(), ctypes.c_uint64()
        _check(self.lib.ora_wah_encode_groups(_p(gkey), _p(gchunk), _p(glit), k, fmt, _p(keys), _p(offs), _p(words),
                                              ctypes.byref(D), ctypes.byref(W)), "wah_encode_groups")
        return keys[: D.value].copy(), offs[: D.value + 1].copy(), words[: W.value].copy()

    def wah_lookup(self, keys, queries):
        keys, queries = _u32(keys), _u32(queries)
        out = np.empty(queries.size, np.uint32)
        _check(self.lib.ora_wah_lookup(_p(keys), keys.size, _p(queries), queries.size, _p(out)), "wah_lookup")
        return out

    def wah_decode(self, words, fmt: int, ngroups: int):
        words = _u32(words)
        out = np.empty(ngroups, np.uint32)
        _check(self.lib.ora_wah_decode(_p(words), words.size, fmt, ngroups, _p(out)), "wah_decode")
        return out

    def wah_combine(self, a, b, in_fmt: int, ngroups: int, op: int, out_fmt: int):
        """AND (op 0) / OR (op 1) of two bitmaps, re-encoded in out_fmt."""
        a, b = _u32(a), _u32(b)
        out = np.empty(max(2 * ngroups, 1), np.uint32)
        m = ctypes.c_uint64()
        _check(self.lib.ora_wah_combine(_p(a), a.size, _p(b), b.size, in_fmt, ngroups, op, out_fmt, _p(out),
                                        ctypes.byref(m)), "wah_combine")
        return out[: m.value].copy()

    def exclusive_scan(self, x):
        x = _u32(x)
        out = np.empty(x.size, np.uint32)
        _check(self.lib.ora_exclusive_scan(_p(x), x.size, _p(out)), "exclusive_scan")
        return out

    def affine_chain(self, x, a, b):
        x = _u32(x).copy()
        a, b = _u32(a), _u32(b)
        _check(self.lib.ora_affine_chain(_p(x), x.size, _p(a), _p(b), a.size), "affine_chain")
        return x


_default: Oracle | None = None


def default() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default
