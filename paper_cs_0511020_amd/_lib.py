"""ctypes binding of libpbit.so (the C ABI in include/pbit.h).

Argument marshalling only: every step of the sort runs in the HIP kernels of
the library.  torch tensors supply device memory and the HIP stream.  There is
no CPU fallback: if the library is missing the import of a function raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpbit.so")

NIL = 0xFFFFFFFF
MAX_NODES = (1 << 32) - 2
OK, EINVAL, EMALFORMED, ENOMEM, EHIP = 0, -1, -2, -3, -4
ASCENDING, DESCENDING, SIGNED, FLOAT, SHARED = 0, 1, 2, 4, 8

# name -> (restype, argtypes)
_SIGNATURES = {
    "pbit_workspace_bytes": (ctypes.c_size_t, [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32]),
    "pbit_sort_list_async": (ctypes.c_int, [
        ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
        ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p,
        ctypes.c_size_t, ctypes.c_void_p]),
    "pbit_sort_list_noalloc": (ctypes.c_int, [
        ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
        ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p]),
    "pbit_sort_list": (ctypes.c_int64, [
        ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32,
        ctypes.c_uint32]),
    "pbit_sort_list_profiled": (ctypes.c_int, [
        ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
        ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p,
        ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
        ctypes.POINTER(ctypes.c_int)]),
    "pbit_stage_name": (ctypes.c_char_p, [ctypes.c_int]),
    "pbit_lists_workspace_bytes": (ctypes.c_size_t, [ctypes.c_uint64, ctypes.c_uint32,
                                                     ctypes.c_uint32, ctypes.c_uint32]),
    "pbit_sort_lists": (ctypes.c_int, [
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "pbit_sort_lists_gather": (ctypes.c_int, [
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "pbit_sort_lists_profiled": (ctypes.c_int, [
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
    "pbit_sort_list_aos_async": (ctypes.c_int, [
        ctypes.c_uint32, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
        ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p,
        ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "pbit_repair_prev_async": (ctypes.c_int, [
        ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
        ctypes.c_void_p, ctypes.c_void_p]),
    "pbit_set_lookback_spin_limit": (ctypes.c_uint32, [ctypes.c_uint32]),
    "pbit_tune_set": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64,
                                     ctypes.c_uint32, ctypes.c_uint32]),
    "pbit_tune_clear": (None, []),
    "pbit_tune_reset": (None, []),
    "pbit_tune_lookup": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64,
                                        ctypes.POINTER(ctypes.c_uint32),
                                        ctypes.POINTER(ctypes.c_uint32)]),
    "pbit_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "pbit_version": (ctypes.c_char_p, []),
}

_lib = None


def load() -> ctypes.CDLL:
    """Load libpbit.so (built by ``paper_cs_0511020_amd.build``); raise if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                "libpbit.so is not built (run __graft_entry__.build() or "
                "python -m paper_cs_0511020_amd.build); there is no fallback path")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def status_string(code: int) -> str:
    return load().pbit_status_string(int(code)).decode()


def version() -> str:
    return load().pbit_version().decode()


def tune_set(kind: int, M: int, n_max: int, K: int, cutoff: int) -> int:
    """Add or replace a tuning entry (kind 0: one list, 1: many lists)."""
    return int(load().pbit_tune_set(int(kind), int(M), int(n_max), int(K), int(cutoff)))


def tune_reset() -> None:
    """Back to the built-in table."""
    load().pbit_tune_reset()


def tune_clear() -> None:
    """An empty table: K = 8 (4 for M = 8) and cutoff 2048 everywhere."""
    load().pbit_tune_clear()


def tune_lookup(kind: int, M: int, n: int):
    """(K, cutoff) the library picks for a sort of this kind, width and size."""
    k, c = ctypes.c_uint32(0), ctypes.c_uint32(0)
    st = load().pbit_tune_lookup(int(kind), int(M), int(n), ctypes.byref(k), ctypes.byref(c))
    if st != OK:
        raise ValueError("bad tuning query")
    return int(k.value), int(c.value)


def set_lookback_spin_limit(sleeps: int) -> int:
    """Look-back wait bound for digit passes queued from now on (diagnostic;
    0 sends every waiting tile down its counting path).  Returns the old one."""
    return int(load().pbit_set_lookback_spin_limit(int(sleeps)))


def workspace_bytes(n: int, M: int, K: int = 0) -> int:
    return int(load().pbit_workspace_bytes(n, M, K))


def _ptr(t) -> int:
    if t is None:
        return 0
    return int(t.data_ptr())


def _stream_handle(stream) -> int:
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def sort_list_async(head: int, next_in, next_out, keys, n: int, M: int, K: int, flags: int,
                    result, ws, ws_bytes: int, stream=None) -> int:
    """Raw C-ABI call with device tensors; returns the host-side status."""
    return int(load().pbit_sort_list_async(
        int(head) & 0xFFFFFFFF, _ptr(next_in), _ptr(next_out), _ptr(keys), int(n), int(M),
        int(K), int(flags), _ptr(result), _ptr(ws), int(ws_bytes), _stream_handle(stream)))


NOALLOC_SCRATCH_BYTES = 64 << 20


def sort_list_noalloc(head: int, next_in, next_out, keys, n: int, M: int, K: int, flags: int,
                      result, stream=None) -> int:
    """Raw C-ABI call of the form that allocates nothing (a fixed per-device
    workspace of NOALLOC_SCRATCH_BYTES; concurrent calls on one device race)."""
    return int(load().pbit_sort_list_noalloc(
        int(head) & 0xFFFFFFFF, _ptr(next_in), _ptr(next_out), _ptr(keys), int(n), int(M),
        int(K), int(flags), _ptr(result), _stream_handle(stream)))


def lists_workspace_bytes(total: int, num_lists: int, M: int, K: int = 0) -> int:
    return int(load().pbit_lists_workspace_bytes(total, num_lists, M, K))


def sort_lists(heads, offsets, num_lists: int, total: int, next_in, next_out, keys, M: int,
               K: int, flags: int, new_heads, status, ws, ws_bytes: int, stream=None) -> int:
    """Raw C-ABI call of the batched form with device tensors."""
    return int(load().pbit_sort_lists(
        _ptr(heads), _ptr(offsets), int(num_lists), int(total), _ptr(next_in), _ptr(next_out),
        _ptr(keys), int(M), int(K), int(flags), _ptr(new_heads), _ptr(status), _ptr(ws),
        int(ws_bytes), _stream_handle(stream)))


def sort_lists_gather(heads, offsets, num_lists: int, total: int, next_in_ptrs, next_out_ptrs,
                      key_ptrs, M: int, K: int, flags: int, new_heads, status, ws,
                      ws_bytes: int, stream=None) -> int:
    """Raw C-ABI call of the gather form: the three pointer tables are device
    int64 tensors holding each list's array addresses."""
    return int(load().pbit_sort_lists_gather(
        _ptr(heads), _ptr(offsets), int(num_lists), int(total), _ptr(next_in_ptrs),
        _ptr(next_out_ptrs), _ptr(key_ptrs), int(M), int(K), int(flags), _ptr(new_heads),
        _ptr(status), _ptr(ws), int(ws_bytes), _stream_handle(stream)))


def sort_list(head: int, next_, keys, M: int, K: int = 0) -> int:
    """Synchronous in-place C-ABI call (library-owned workspace, default stream)."""
    n = int(next_.numel())
    return int(load().pbit_sort_list(int(head) & 0xFFFFFFFF, _ptr(next_), _ptr(keys), n,
                                      int(M), int(K)))


def repair_prev(heads, num_lists: int, next_, prev, n: int, status=None, status_offset: int = 0,
                stream=None) -> int:
    """Raw C-ABI call of the backward-link repair (``status_offset`` bytes into
    ``status``: 4 selects the status word of a single-list result)."""
    st_ptr = _ptr(status) + status_offset if status is not None else 0
    return int(load().pbit_repair_prev_async(
        _ptr(heads), int(num_lists), _ptr(next_), _ptr(prev), int(n), st_ptr,
        _stream_handle(stream)))


def sort_list_aos_async(head: int, nodes, stride: int, next_off: int, key_off: int, n: int,
                        M: int, K: int, flags: int, result, ws, ws_bytes: int,
                        stream=None) -> int:
    """Raw C-ABI call for nodes stored as records of ``stride`` bytes."""
    return int(load().pbit_sort_list_aos_async(
        int(head) & 0xFFFFFFFF, _ptr(nodes), int(stride), int(next_off), int(key_off), int(n),
        int(M), int(K), int(flags), _ptr(result), _ptr(ws), int(ws_bytes),
        _stream_handle(stream)))
