"""CPU oracle for the GPU LSM dictionary (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this package; the product library never does.  It shares no code with the HIP
path: the arithmetic lives in ``lsm_oracle.cpp`` (plain C++ over std::map,
std::sort and std::merge), reached through ctypes with numpy arrays.

* :class:`MapOracle` -- the dictionary of sec. I-B applied one operation at a
  time (the plain definition of every query answer).
* :class:`CascadeOracle` -- the level layout produced by the insertion
  algorithm of Fig. 2(a) / Fig. 3, step by step, and by the cleanup of
  sec. III-E / IV-D.

Every function is pinned by ``tests/test_oracle_pins.py`` against brute force
on tiny inputs, a closed form of the layout, the building invariants of
sec. III-D, the worked cascade of Fig. 1 and special cases that reduce to a
sorted array.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lsm_oracle.cpp")
_LIB = os.path.join(_HERE, "liblsm_oracle.so")

_u32p = ctypes.POINTER(ctypes.c_uint32)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_u8p = ctypes.POINTER(ctypes.c_uint8)


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (in place). Returns the library path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        # LSM_ORACLE_LIB lets the mutation tests load a copy of the oracle
        # with a planted mistake, to show that the pins catch it.
        lib = ctypes.CDLL(os.environ.get("LSM_ORACLE_LIB") or build())
        vp = ctypes.c_void_p
        sig = {
            "om_create": (vp, []),
            "om_destroy": (None, [vp]),
            "om_insert": (None, [vp, _u32p, _u32p, ctypes.c_uint64]),
            "om_delete": (None, [vp, _u32p, ctypes.c_uint64]),
            "om_mixed": (None, [vp, _u32p, _u32p, _u8p, ctypes.c_uint64]),
            "om_lookup": (None, [vp, _u32p, ctypes.c_uint64, _u32p, _u8p]),
            "om_count": (None, [vp, _u32p, _u32p, ctypes.c_uint64, _u32p]),
            "om_range": (ctypes.c_uint64, [vp, _u32p, _u32p, ctypes.c_uint64, _u64p, _u32p, _u32p, ctypes.c_uint64]),
            "om_successor": (None, [vp, _u32p, ctypes.c_uint64, _u32p, _u32p, _u8p]),
            "om_predecessor": (None, [vp, _u32p, ctypes.c_uint64, _u32p, _u32p, _u8p]),
            "om_size": (ctypes.c_uint64, [vp]),
            "om_items": (None, [vp, _u32p, _u32p]),
            "oc_create": (vp, [ctypes.c_uint32]),
            "oc_destroy": (None, [vp]),
            "oc_insert": (ctypes.c_int, [vp, _u32p, _u32p, _u8p, ctypes.c_uint32]),
            "oc_insert_ordered": (ctypes.c_int, [vp, _u32p, _u32p, _u8p, ctypes.c_uint32]),
            "oc_cleanup": (ctypes.c_uint64, [vp]),
            "oc_num_batches": (ctypes.c_uint64, [vp]),
            "oc_merged_last": (ctypes.c_uint64, [vp]),
            "oc_merged_total": (ctypes.c_uint64, [vp]),
            "oc_level_size": (ctypes.c_uint64, [vp, ctypes.c_uint32]),
            "oc_level": (None, [vp, ctypes.c_uint32, _u32p, _u32p]),
        }
        for name, (res, args) in sig.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def _u32(a) -> np.ndarray:
    a = np.ascontiguousarray(a)
    if a.dtype != np.uint32:
        a = np.ascontiguousarray(a.astype(np.int64).astype(np.uint32))
    return a


def _p32(a: np.ndarray):
    return a.ctypes.data_as(_u32p)


class MapOracle:
    """std::map dictionary; one operation at a time, batches in call order."""

    def __init__(self):
        self._lib = _load()
        self._h = self._lib.om_create()

    def __del__(self):
        h, self._h = getattr(self, "_h", None), None
        if h:
            self._lib.om_destroy(h)

    def insert(self, keys, vals) -> None:
        k, v = _u32(keys), _u32(vals)
        assert k.shape == v.shape
        self._lib.om_insert(self._h, _p32(k), _p32(v), k.size)

    def delete(self, keys) -> None:
        k = _u32(keys)
        self._lib.om_delete(self._h, _p32(k), k.size)

    def mixed(self, keys, vals, is_delete) -> None:
        k, v = _u32(keys), _u32(vals)
        d = np.ascontiguousarray(is_delete, dtype=np.uint8)
        assert k.shape == v.shape == d.shape
        self._lib.om_mixed(self._h, _p32(k), _p32(v), d.ctypes.data_as(_u8p), k.size)

    def lookup(self, q):
        q = _u32(q)
        vals = np.zeros(q.size, np.uint32)
        found = np.zeros(q.size, np.uint8)
        self._lib.om_lookup(self._h, _p32(q), q.size, _p32(vals), found.ctypes.data_as(_u8p))
        return vals, found

    def count(self, lo, hi):
        lo, hi = _u32(lo), _u32(hi)
        out = np.zeros(lo.size, np.uint32)
        self._lib.om_count(self._h, _p32(lo), _p32(hi), lo.size, _p32(out))
        return out

    def range(self, lo, hi):
        """Returns (offsets[nq+1] u64, keys u32, vals u32)."""
        lo, hi = _u32(lo), _u32(hi)
        nq = lo.size
        offsets = np.zeros(nq + 1, np.uint64)
        total = self._lib.om_range(self._h, _p32(lo), _p32(hi), nq,
                                   offsets.ctypes.data_as(_u64p), None, None, 0)
        keys = np.zeros(total, np.uint32)
        vals = np.zeros(total, np.uint32)
        if total:
            self._lib.om_range(self._h, _p32(lo), _p32(hi), nq,
                               offsets.ctypes.data_as(_u64p), _p32(keys), _p32(vals), total)
        return offsets, keys, vals

    def _order(self, fn, q):
        q = _u32(q)
        keys = np.zeros(q.size, np.uint32)
        vals = np.zeros(q.size, np.uint32)
        found = np.zeros(q.size, np.uint8)
        fn(self._h, _p32(q), q.size, _p32(keys), _p32(vals), found.ctypes.data_as(_u8p))
        return keys, vals, found

    def successor(self, q):
        """(keys, vals, found): the pair with the smallest key > q."""
        return self._order(self._lib.om_successor, q)

    def predecessor(self, q):
        """(keys, vals, found): the pair with the largest key < q."""
        return self._order(self._lib.om_predecessor, q)

    def __len__(self) -> int:
        return int(self._lib.om_size(self._h))

    def items(self):
        n = len(self)
        k = np.zeros(n, np.uint32)
        v = np.zeros(n, np.uint32)
        if n:
            self._lib.om_items(self._h, _p32(k), _p32(v))
        return k, v


class CascadeOracle:
    """Level layout from the insertion algorithm of Fig. 2(a) / Fig. 3."""

    def __init__(self, b: int):
        self.b = int(b)
        self._lib = _load()
        self._h = self._lib.oc_create(self.b)

    def __del__(self):
        h, self._h = getattr(self, "_h", None), None
        if h:
            self._lib.oc_destroy(h)

    def insert(self, keys, vals=None, status=None) -> None:
        """One batch of 1..b elements; status 1 = regular, 0 = tombstone."""
        k = _u32(keys)
        v = None if vals is None else _u32(vals)
        s = None if status is None else np.ascontiguousarray(status, dtype=np.uint8)
        rc = self._lib.oc_insert(self._h, _p32(k), None if v is None else _p32(v),
                                 None if s is None else s.ctypes.data_as(_u8p), k.size)
        if rc != 0:
            raise ValueError("batch size must be in [1, b]")

    def delete(self, keys) -> None:
        k = _u32(keys)
        self.insert(k, None, np.zeros(k.size, np.uint8))

    def insert_ordered(self, keys, vals, status) -> None:
        """A coalesced batch of 1..b elements: user batches packed in arrival
        order; the newest operation on a key wins whatever its type."""
        k, v = _u32(keys), _u32(vals)
        s = np.ascontiguousarray(status, dtype=np.uint8)
        rc = self._lib.oc_insert_ordered(self._h, _p32(k), _p32(v), s.ctypes.data_as(_u8p), k.size)
        if rc != 0:
            raise ValueError("batch size must be in [1, b]")

    def cleanup(self) -> int:
        """Cleanup of sec. III-E / IV-D; returns the number of valid elements."""
        return int(self._lib.oc_cleanup(self._h))

    @property
    def r(self) -> int:
        return int(self._lib.oc_num_batches(self._h))

    @property
    def merged_last(self) -> int:
        return int(self._lib.oc_merged_last(self._h))

    @property
    def merged_total(self) -> int:
        return int(self._lib.oc_merged_total(self._h))

    def level(self, i: int):
        """(kv, vals) of level i as uint32 arrays (empty when the level is empty)."""
        n = int(self._lib.oc_level_size(self._h, i))
        kv = np.zeros(n, np.uint32)
        v = np.zeros(n, np.uint32)
        if n:
            self._lib.oc_level(self._h, i, _p32(kv), _p32(v))
        return kv, v

    def occupied(self):
        r, out, i = self.r, [], 0
        while (r >> i) != 0:
            if (r >> i) & 1:
                out.append(i)
            i += 1
        return out
