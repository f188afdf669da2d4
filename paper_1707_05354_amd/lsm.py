"""Thin ctypes binding of the C ABI in include/lsm.h.

Argument marshalling only: every step of every operation runs in the HIP
kernels of liblsm_hip.so.  Tensors are torch tensors on the handle's GPU
(int32 or uint32 storage; keys and values are reinterpreted as uint32 and
never interpreted by torch).  If the library is missing this module raises;
there is no fallback path.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import re
import weakref
from typing import Optional, Tuple

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "liblsm_hip.so")
HEADER = os.path.join(os.path.dirname(_PKG), "include", "lsm.h")

LSM_OK, LSM_EINVAL, LSM_EKEY, LSM_EBATCH, LSM_ENOMEM, LSM_ECAPACITY, LSM_EHIP = range(7)
LSM_CHECKED = 0x1


def LSM_KEY_BITS(k: int) -> int:
    return (int(k) & 0x3F) << 8


class LSMError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = int(status)
        super().__init__("%s failed: %s (%d)" % (where, _strerror(status), status))


class Stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in (
        "num_batches", "resident_elems", "merged_elems_last", "merged_elems_total",
        "sorted_elems_total", "device_bytes", "sorts_top_digit", "sorts_digit_passes")]


KERNEL_NAMES = ("k_sort_hist", "k_sort_pass", "k_merge", "k_lookup", "k_count", "k_scan",
                "k_range_emit", "k_order", "k_clean", "(unused)", "k_msd_scatter",
                "k_local_sort", "k_sort_step")
# rocprofv3 kernel names behind each profiler kind that covers several kernels.
KERNEL_TRACE_NAMES = {"k_order": ("k_successor", "k_predecessor"),
                      "k_clean": ("k_clean_count", "k_clean_scatter", "k_clean_pad"),
                      "k_merge": ("k_merge<4>", "k_merge<8>", "k_merge<16>")}
_NK = len(KERNEL_NAMES)
PROF_SIZES = 40  # LSM_PROF_SIZES


class Profile(ctypes.Structure):
    _fields_ = [("update_calls", ctypes.c_uint64), ("query_calls", ctypes.c_uint64 * 3),
                ("query_items", ctypes.c_uint64 * 3), ("launches", ctypes.c_uint64 * _NK),
                ("elems", ctypes.c_uint64 * _NK), ("kernel_ms", ctypes.c_double * _NK),
                ("kernel_bytes", ctypes.c_double * _NK), ("update_ms", ctypes.c_double),
                ("update_p50_ms", ctypes.c_double), ("update_p99_ms", ctypes.c_double),
                ("update_max_ms", ctypes.c_double), ("query_ms", ctypes.c_double * 3),
                ("merge_launches_by_size", ctypes.c_uint64 * PROF_SIZES),
                ("merge_ms_by_size", ctypes.c_double * PROF_SIZES),
                ("merge_bytes_by_size", ctypes.c_double * PROF_SIZES)]


_lib = None
_vp = ctypes.c_void_p
_u32 = ctypes.c_uint32
_u64 = ctypes.c_uint64

_SIGNATURES = {
    "lsm_create": (ctypes.c_int, [ctypes.POINTER(_vp), _u32, _u32, _vp]),
    "lsm_set_stream": (ctypes.c_int, [_vp, _vp]),
    "lsm_insert_batch": (ctypes.c_int, [_vp, _vp, _vp, _u32]),
    "lsm_delete_batch": (ctypes.c_int, [_vp, _vp, _u32]),
    "lsm_update_batch": (ctypes.c_int, [_vp, _vp, _vp, _vp, _u32]),
    "lsm_lookup": (ctypes.c_int, [_vp, _vp, _u32, _vp, _vp]),
    "lsm_count": (ctypes.c_int, [_vp, _vp, _vp, _u32, _vp]),
    "lsm_range": (ctypes.c_int, [_vp, _vp, _vp, _u32, _vp, _vp, _vp, _u64, ctypes.POINTER(_u64)]),
    "lsm_successor": (ctypes.c_int, [_vp, _vp, _u32, _vp, _vp, _vp]),
    "lsm_predecessor": (ctypes.c_int, [_vp, _vp, _u32, _vp, _vp, _vp]),
    "lsm_cleanup": (ctypes.c_int, [_vp, ctypes.POINTER(_u64)]),
    "lsm_bulk_insert": (ctypes.c_int, [_vp, _vp, _vp, _u64]),
    "lsm_set_sort_path": (ctypes.c_int, [_vp, ctypes.c_int]),
    "lsm_set_fusion": (ctypes.c_int, [_vp, ctypes.c_int]),
    "lsm_set_max_inflight": (ctypes.c_int, [_vp, ctypes.c_int]),
    "lsm_set_grouping": (ctypes.c_int, [_vp, ctypes.c_int]),
    "lsm_destroy": (ctypes.c_int, [_vp]),
    "lsm_clear": (ctypes.c_int, [_vp]),
    "lsm_sync": (ctypes.c_int, [_vp]),
    "lsm_profile_enable": (ctypes.c_int, [_vp, ctypes.c_int]),
    "lsm_profile_read": (ctypes.c_int, [_vp, ctypes.POINTER(Profile), ctypes.c_int]),
    "lsm_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "lsm_num_batches": (_u64, [_vp]),
    "lsm_batch_size": (_u32, [_vp]),
    "lsm_level_view": (ctypes.c_int, [_vp, _u32, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                      ctypes.POINTER(_u64)]),
    "lsm_level_copy": (ctypes.c_int, [_vp, _u32, _vp, _vp, ctypes.POINTER(_u64)]),
    "lsm_get_stats": (ctypes.c_int, [_vp, ctypes.POINTER(Stats)]),
    "lsm_submit": (ctypes.c_int, [_vp, _vp, _vp, _u32, ctypes.c_int]),
    "lsm_flush": (ctypes.c_int, [_vp]),
    "lsm_submit_mixed": (ctypes.c_int, [_vp, _vp, _vp, _vp, _u32]),
    "lsm_range_async": (ctypes.c_int, [_vp, _vp, _vp, _u32, _vp, _vp, _vp, _u64]),
    "lsm_range_async_noalloc": (ctypes.c_int, [_vp, _vp, _vp, _u32, _vp, _vp, _vp, _u64]),
    "lsm_pending": (_u32, [_vp]),
    "lsm_autotune": (ctypes.c_int, [_vp, _u32, _u32]),
    "lsm_get_tuning": (ctypes.c_int, [_vp, _u32, ctypes.POINTER(_u32), ctypes.POINTER(ctypes.c_float)]),
    "lsm_set_tuning": (ctypes.c_int, [_vp, _u32, _u32]),
    "lsm_fail_alloc_after": (ctypes.c_int, [_vp, ctypes.c_int64]),
    "lsm_struct_sizes": (None, [ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]),
}


def header_symbols(path: str = HEADER):
    """Names of every function the public header declares."""
    text = open(path).read()
    return re.findall(r"^LSM_API\s+[\w\s\*]+?\b(lsm_\w+)\s*\(", text, flags=re.M)


def load_library(path: str = LIB_PATH):
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError("HIP library %s is not built (python -m paper_1707_05354_amd.build)"
                               % path)
        lib = ctypes.CDLL(path)
        for name, (res, args) in _SIGNATURES.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        ss, ps = ctypes.c_size_t(), ctypes.c_size_t()
        lib.lsm_struct_sizes(ctypes.byref(ss), ctypes.byref(ps))
        if (ss.value, ps.value) != (ctypes.sizeof(Stats), ctypes.sizeof(Profile)):
            raise RuntimeError("lsm_stats_t / lsm_profile_t layout differs from the binding: "
                               "%s vs %s" % ((ss.value, ps.value),
                                             (ctypes.sizeof(Stats), ctypes.sizeof(Profile))))
        _lib = lib
    return _lib


def _strerror(status: int) -> str:
    try:
        return load_library().lsm_strerror(int(status)).decode()
    except Exception:  # library missing: still report the number
        return "status"


def _dev(t: torch.Tensor, name: str, dtypes=(torch.int32, torch.uint32)) -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype not in dtypes:
        raise TypeError("%s must have dtype in %s, got %s" % (name, dtypes, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return t.data_ptr()


def _check(rc: int, where: str) -> None:
    if rc != LSM_OK:
        raise LSMError(rc, where)


# Every open handle, so that the ones still open when the interpreter exits
# are destroyed by an atexit hook, while the HIP runtime is still fully up,
# instead of by __del__ during interpreter teardown.
_OPEN = weakref.WeakSet()


@atexit.register
def _close_open_handles() -> None:
    for g in list(_OPEN):
        try:
            g.close()
        except Exception:
            pass


class LSM:
    """A batched LSM dictionary resident on one GPU (see include/lsm.h)."""

    def __init__(self, b: int, checked: bool = False, key_bits: int = 31,
                 stream: Optional[torch.cuda.Stream] = None):
        self._lib = load_library()
        self.b = int(b)
        self.device = torch.cuda.current_device()
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        flags = (LSM_CHECKED if checked else 0) | LSM_KEY_BITS(key_bits)
        h = _vp()
        _check(self._lib.lsm_create(ctypes.byref(h), self.b, flags, _vp(self.stream.cuda_stream)),
               "lsm_create")
        self._h = h
        self._last_total = 0
        _OPEN.add(self)

    # -- lifetime -----------------------------------------------------------
    def close(self) -> None:
        h, self._h = getattr(self, "_h", None), None
        _OPEN.discard(self)
        if h:
            _check(self._lib.lsm_destroy(h), "lsm_destroy")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def sync(self) -> None:
        """Wait for the handle's stream; raises if a device-side wait ran out."""
        _check(self._lib.lsm_sync(self._h), "lsm_sync")

    def clear(self) -> None:
        """Empty the dictionary, keeping its device memory."""
        _check(self._lib.lsm_clear(self._h), "lsm_clear")

    def profile(self, on: bool = True) -> None:
        _check(self._lib.lsm_profile_enable(self._h, 1 if on else 0), "lsm_profile_enable")

    def profile_read(self, reset: bool = True) -> Profile:
        p = Profile()
        _check(self._lib.lsm_profile_read(self._h, ctypes.byref(p), 1 if reset else 0),
               "lsm_profile_read")
        return p

    # -- updates ------------------------------------------------------------
    def insert(self, keys: torch.Tensor, vals: torch.Tensor) -> None:
        if keys.numel() != vals.numel():
            raise ValueError("keys and vals differ in length")
        _check(self._lib.lsm_insert_batch(self._h, _dev(keys, "keys"), _dev(vals, "vals"),
                                          keys.numel()), "lsm_insert_batch")

    def delete(self, keys: torch.Tensor) -> None:
        _check(self._lib.lsm_delete_batch(self._h, _dev(keys, "keys"), keys.numel()),
               "lsm_delete_batch")

    def update(self, keys: torch.Tensor, vals: torch.Tensor, is_delete: torch.Tensor) -> None:
        if not (keys.numel() == vals.numel() == is_delete.numel()):
            raise ValueError("keys, vals and is_delete differ in length")
        _check(self._lib.lsm_update_batch(
            self._h, _dev(keys, "keys"), _dev(vals, "vals"),
            _dev(is_delete, "is_delete", (torch.uint8, torch.bool)), keys.numel()),
            "lsm_update_batch")

    # -- batching form --------------------------------------------------------
    def submit(self, keys: torch.Tensor, vals: Optional[torch.Tensor] = None,
               delete: bool = False) -> None:
        """One user batch of any size, packed into LSM batches of b."""
        n = keys.numel()
        if not delete and (vals is None or vals.numel() != n):
            raise ValueError("an insert batch needs one value per key")
        vp = _dev(vals, "vals") if (vals is not None and not delete) else None
        _check(self._lib.lsm_submit(self._h, _dev(keys, "keys"), vp, n, 1 if delete else 0),
               "lsm_submit")

    def submit_mixed(self, keys: torch.Tensor, vals: torch.Tensor,
                     is_delete: torch.Tensor) -> None:
        """Arrival-ordered operations of both types: element j deletes
        keys[j] when is_delete[j] != 0, else inserts (keys[j], vals[j])."""
        if not (keys.numel() == vals.numel() == is_delete.numel()):
            raise ValueError("keys, vals and is_delete differ in length")
        _check(self._lib.lsm_submit_mixed(
            self._h, _dev(keys, "keys"), _dev(vals, "vals"),
            _dev(is_delete, "is_delete", (torch.uint8, torch.bool)), keys.numel()),
            "lsm_submit_mixed")

    def range_async(self, lo, hi, offsets, keys, vals, cap: int) -> None:
        _check(self._lib.lsm_range_async(self._h, _dev(lo, "lo"), _dev(hi, "hi"), lo.numel(),
                                         _dev(offsets, "offsets", (torch.int64,)),
                                         keys.data_ptr() if keys is not None else None,
                                         vals.data_ptr() if vals is not None else None, int(cap)),
               "lsm_range_async")

    def flush(self) -> None:
        _check(self._lib.lsm_flush(self._h), "lsm_flush")

    @property
    def pending(self) -> int:
        return int(self._lib.lsm_pending(self._h))

    def autotune(self, max_level: int, reps: int = 5) -> None:
        _check(self._lib.lsm_autotune(self._h, int(max_level), int(reps)), "lsm_autotune")

    def tuning(self, level: int):
        """(chosen merge variant, [us per launch of each of the 6 variants])."""
        v = _u32()
        us = (ctypes.c_float * 6)()
        _check(self._lib.lsm_get_tuning(self._h, int(level), ctypes.byref(v), us), "lsm_get_tuning")
        return int(v.value), [float(x) for x in us]

    SORT_AUTO, SORT_TOP_DIGIT, SORT_DIGIT_PASSES = 0, 1, 2

    def set_sort_path(self, mode: int) -> None:
        """LSM.SORT_AUTO (default), LSM.SORT_TOP_DIGIT or LSM.SORT_DIGIT_PASSES."""
        _check(self._lib.lsm_set_sort_path(self._h, int(mode)), "lsm_set_sort_path")

    def set_fusion(self, max_levels: int) -> None:
        """Deepest cascade fused into the top-digit sort (0 off, -1 default)."""
        _check(self._lib.lsm_set_fusion(self._h, int(max_levels)), "lsm_set_fusion")

    def set_max_inflight(self, launches: int) -> None:
        """Update launches the host may queue ahead of the device (0: no pacing)."""
        _check(self._lib.lsm_set_max_inflight(self._h, int(launches)), "lsm_set_max_inflight")

    def set_grouping(self, max_batches: int) -> None:
        """Sort up to max_batches (1, 2 or 4) consecutive batches together."""
        _check(self._lib.lsm_set_grouping(self._h, int(max_batches)), "lsm_set_grouping")

    def set_tuning(self, level: int, variant: int) -> None:
        _check(self._lib.lsm_set_tuning(self._h, int(level), int(variant)), "lsm_set_tuning")

    # -- queries ------------------------------------------------------------
    def lookup(self, q: torch.Tensor, out: Optional[Tuple[torch.Tensor, torch.Tensor]] = None):
        nq = q.numel()
        if out is None:
            vals = torch.empty(nq, dtype=torch.int32, device=q.device)
            found = torch.empty(nq, dtype=torch.uint8, device=q.device)
        else:
            vals, found = out
        _check(self._lib.lsm_lookup(self._h, _dev(q, "q"), nq, _dev(vals, "vals"),
                                    _dev(found, "found", (torch.uint8, torch.bool))), "lsm_lookup")
        return vals, found

    def _order(self, fn, name, q):
        nq = q.numel()
        keys = torch.empty(nq, dtype=torch.int32, device=q.device)
        vals = torch.empty(nq, dtype=torch.int32, device=q.device)
        found = torch.empty(nq, dtype=torch.uint8, device=q.device)
        _check(fn(self._h, _dev(q, "q"), nq, _dev(keys, "keys"), _dev(vals, "vals"),
                  _dev(found, "found", (torch.uint8,))), name)
        return keys, vals, found

    def successor(self, q: torch.Tensor):
        """(keys, vals, found): per query the live pair with the smallest key > q."""
        return self._order(self._lib.lsm_successor, "lsm_successor", q)

    def predecessor(self, q: torch.Tensor):
        """(keys, vals, found): per query the live pair with the largest key < q."""
        return self._order(self._lib.lsm_predecessor, "lsm_predecessor", q)

    def bulk_insert(self, keys: torch.Tensor, vals: torch.Tensor) -> None:
        """keys.numel() pairs as consecutive insert batches of b (the last one
        partial); synchronises the stream."""
        n = keys.numel()
        if vals.numel() != n:
            raise ValueError("keys and vals differ in length")
        _check(self._lib.lsm_bulk_insert(self._h, _dev(keys, "keys"), _dev(vals, "vals"), n),
               "lsm_bulk_insert")

    def cleanup(self) -> int:
        """Cleanup (drop stale elements, rebuild the levels); returns the
        number of valid pairs.  Synchronises the stream."""
        v = _u64(0)
        _check(self._lib.lsm_cleanup(self._h, ctypes.byref(v)), "lsm_cleanup")
        return int(v.value)

    def count(self, lo: torch.Tensor, hi: torch.Tensor, out: Optional[torch.Tensor] = None):
        nq = lo.numel()
        if hi.numel() != nq:
            raise ValueError("lo and hi differ in length")
        counts = out if out is not None else torch.empty(nq, dtype=torch.int32, device=lo.device)
        _check(self._lib.lsm_count(self._h, _dev(lo, "lo"), _dev(hi, "hi"), nq,
                                   _dev(counts, "counts")), "lsm_count")
        return counts

    def range_raw(self, lo, hi, offsets, keys, vals, cap: int) -> int:
        """One lsm_range call; returns the total (raises on any error)."""
        total = _u64(0)
        kp = _dev(keys, "keys") if keys is not None else None
        vp = _dev(vals, "vals") if vals is not None else None
        rc = self._lib.lsm_range(self._h, _dev(lo, "lo"), _dev(hi, "hi"), lo.numel(),
                                 _dev(offsets, "offsets", (torch.int64, torch.uint64)), kp, vp,
                                 int(cap), ctypes.byref(total))
        _check(rc, "lsm_range")
        return int(total.value)

    def range(self, lo: torch.Tensor, hi: torch.Tensor, cap: Optional[int] = None):
        """Returns (offsets[nq+1] int64, keys int32, vals int32); two-phase
        when the first output guess is too small."""
        nq = lo.numel()
        if hi.numel() != nq:
            raise ValueError("lo and hi differ in length")
        offsets = torch.empty(nq + 1, dtype=torch.int64, device=lo.device)
        guess = int(cap) if cap is not None else max(1024, 2 * self._last_total)
        keys = torch.empty(max(guess, 1), dtype=torch.int32, device=lo.device)
        vals = torch.empty(max(guess, 1), dtype=torch.int32, device=lo.device)
        total = _u64(0)
        rc = self._lib.lsm_range(self._h, _dev(lo, "lo"), _dev(hi, "hi"), nq,
                                 _dev(offsets, "offsets", (torch.int64,)), keys.data_ptr(),
                                 vals.data_ptr(), guess, ctypes.byref(total))
        if rc == LSM_ECAPACITY and cap is None:
            need = int(total.value)
            keys = torch.empty(need, dtype=torch.int32, device=lo.device)
            vals = torch.empty(need, dtype=torch.int32, device=lo.device)
            rc = self._lib.lsm_range(self._h, _dev(lo, "lo"), _dev(hi, "hi"), nq,
                                     _dev(offsets, "offsets", (torch.int64,)), keys.data_ptr(),
                                     vals.data_ptr(), need, ctypes.byref(total))
        _check(rc, "lsm_range")
        n = int(total.value)
        self._last_total = n
        return offsets, keys[:n], vals[:n]

    def fail_alloc_after(self, n: int) -> None:
        """Tests: the next n allocations succeed, later ones fail (n < 0: off)."""
        _check(self._lib.lsm_fail_alloc_after(self._h, int(n)), "lsm_fail_alloc_after")

    # -- introspection ------------------------------------------------------
    @property
    def num_batches(self) -> int:
        return int(self._lib.lsm_num_batches(self._h))

    def stats(self) -> Stats:
        s = Stats()
        _check(self._lib.lsm_get_stats(self._h, ctypes.byref(s)), "lsm_get_stats")
        return s

    def occupied(self):
        r, out, i = self.num_batches, [], 0
        while (r >> i) != 0:
            if (r >> i) & 1:
                out.append(i)
            i += 1
        return out

    def level(self, i: int):
        """Copies of level i's key variables and values (int32 tensors),
        enqueued on the handle's stream."""
        kp, vp, n = _vp(), _vp(), _u64()
        _check(self._lib.lsm_level_view(self._h, int(i), ctypes.byref(kp), ctypes.byref(vp),
                                        ctypes.byref(n)), "lsm_level_view")
        n = int(n.value)
        dev = torch.device("cuda", self.device)
        kv = torch.empty(n, dtype=torch.int32, device=dev)
        val = torch.empty(n, dtype=torch.int32, device=dev)
        if n:
            got = _u64()
            _check(self._lib.lsm_level_copy(self._h, int(i), kv.data_ptr(), val.data_ptr(),
                                            ctypes.byref(got)), "lsm_level_copy")
        return kv, val
