"""Python access to the Pbit CPU oracle (``pbit_oracle.c``).

Test infrastructure only: the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this package; the product package never does.

The oracle follows the paper (Planeta, arXiv cs/0511020) Sec. 3-6: a
recursive most-significant-pattern-first split of the list into 2^K groups per
level, first-in-first-out groups so equal keys keep list order, and the
concatenation of the final groups by the merge of Sec. 5.1.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

NIL = 0xFFFFFFFF
FLAG_LIFO = 1
FLAG_DESCENDING = 2
FLAG_SIGNED = 4
FLAG_FLOAT = 8

OK, EINVAL, EMALFORMED, ENOMEM = 0, -1, -2, -3

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pbit_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_KEY_DTYPES = {8: np.uint8, 16: np.uint16, 32: np.uint32, 64: np.uint64}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/liboracle.so``."""
    if force or not os.path.exists(_LIB_PATH) or (
        os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)
    ):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-D_DEFAULT_SOURCE", "-Wall", "-Wextra", "-shared",
             "-fPIC", "-pthread", _SRC, "-o", tmp]
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        lib.pbit_oracle_sort.restype = ctypes.c_int64
        lib.pbit_oracle_sort.argtypes = [
            ctypes.c_uint32, u32p, ctypes.c_void_p, ctypes.c_uint64,
            ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
            ctypes.POINTER(ctypes.c_uint64)]
        lib.pbit_oracle_sort_threads.restype = ctypes.c_int64
        lib.pbit_oracle_sort_threads.argtypes = [
            ctypes.c_uint32, u32p, ctypes.c_void_p, ctypes.c_uint64,
            ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32]
        lib.pbit_oracle_sort_lists.restype = ctypes.c_int
        lib.pbit_oracle_sort_lists.argtypes = [
            u32p, ctypes.POINTER(ctypes.c_uint64), ctypes.c_uint32, u32p,
            ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, u32p]
        lib.pbit_oracle_list_order.restype = ctypes.c_int64
        lib.pbit_oracle_list_order.argtypes = [
            ctypes.c_uint32, u32p, ctypes.c_uint64, u32p]
        lib.pbit_oracle_repair_prev.restype = ctypes.c_int64
        lib.pbit_oracle_repair_prev.argtypes = [
            ctypes.c_uint32, u32p, ctypes.c_uint64, u32p]
        _lib = lib
    return _lib


def _u32p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def _check_keys(keys: np.ndarray, M: int) -> np.ndarray:
    keys = np.ascontiguousarray(keys)
    if M not in _KEY_DTYPES or keys.dtype != _KEY_DTYPES[M]:
        # signed storage of the same width is reinterpreted, never converted
        if M in _KEY_DTYPES and keys.dtype.itemsize * 8 == M:
            keys = keys.view(_KEY_DTYPES[M])
        else:
            raise ValueError("keys dtype %s does not match M=%d" % (keys.dtype, M))
    return keys


def sort_list(head: int, next_: np.ndarray, keys: np.ndarray, M: int, K: int,
              flags: int = 0, counters: bool = False):
    """Sort one list; returns (new_head_or_status, relinked_next[, counters]).

    ``next_`` is not modified; a relinked copy is returned.  counters =
    (merge steps, split visits, recursive calls, deepest level).
    """
    lib = _load()
    nxt = np.array(next_, dtype=np.uint32, copy=True)
    keys = _check_keys(keys, M)
    if keys.shape[0] != nxt.shape[0]:
        raise ValueError("keys and next differ in length")
    cnt = (ctypes.c_uint64 * 4)()
    h = lib.pbit_oracle_sort(int(head) & 0xFFFFFFFF, _u32p(nxt), keys.ctypes.data,
                             nxt.shape[0], M, K, flags, cnt)
    if counters:
        return int(h), nxt, tuple(int(c) for c in cnt)
    return int(h), nxt


def sort_list_threads(head: int, next_: np.ndarray, keys: np.ndarray, M: int, K: int,
                      flags: int = 0, threads: int = 0):
    """The same sort with the groups below the top levels sorted on host
    threads (0 = every online core); unsigned keys, ascending or descending.
    Returns (new_head_or_status, relinked_next)."""
    lib = _load()
    nxt = np.array(next_, dtype=np.uint32, copy=True)
    keys = _check_keys(keys, M)
    if keys.shape[0] != nxt.shape[0]:
        raise ValueError("keys and next differ in length")
    h = lib.pbit_oracle_sort_threads(int(head) & 0xFFFFFFFF, _u32p(nxt), keys.ctypes.data,
                                     nxt.shape[0], M, K, flags, int(threads))
    return int(h), nxt


def sort_lists(heads: np.ndarray, offsets: np.ndarray, next_: np.ndarray, keys: np.ndarray,
               M: int, K: int, flags: int = 0):
    """Segmented form: returns (status, relinked_next, new_heads)."""
    lib = _load()
    heads = np.ascontiguousarray(heads, dtype=np.uint32)
    offs = np.ascontiguousarray(offsets, dtype=np.uint64)
    nxt = np.array(next_, dtype=np.uint32, copy=True)
    keys = _check_keys(keys, M)
    new_heads = np.full(heads.shape[0], NIL, dtype=np.uint32)
    st = lib.pbit_oracle_sort_lists(
        _u32p(heads), offs.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
        heads.shape[0], _u32p(nxt), keys.ctypes.data, M, K, flags, _u32p(new_heads))
    return int(st), nxt, new_heads


def list_order(head: int, next_: np.ndarray) -> np.ndarray:
    """Nodes in list order (walk from head); raises on a malformed list."""
    lib = _load()
    nxt = np.ascontiguousarray(next_, dtype=np.uint32)
    out = np.empty(nxt.shape[0], dtype=np.uint32)
    t = lib.pbit_oracle_list_order(int(head) & 0xFFFFFFFF, _u32p(nxt), nxt.shape[0], _u32p(out))
    if t < 0:
        raise ValueError("malformed list (status %d)" % t)
    return out[:t]


def repair_prev(head: int, next_: np.ndarray, prev: np.ndarray | None = None) -> np.ndarray:
    """Backward links of the list (Sec. 13): returns a prev[] array (a copy of
    ``prev`` or, by default, all NIL) with every node on the list pointed at
    the node before it; raises on a malformed list."""
    lib = _load()
    nxt = np.ascontiguousarray(next_, dtype=np.uint32)
    out = (np.full(nxt.shape[0], NIL, dtype=np.uint32) if prev is None
           else np.array(prev, dtype=np.uint32, copy=True))
    t = lib.pbit_oracle_repair_prev(int(head) & 0xFFFFFFFF, _u32p(nxt), nxt.shape[0], _u32p(out))
    if t < 0:
        raise ValueError("malformed list (status %d)" % t)
    return out
