"""Device-resident list sorting on top of the C ABI.

``ListSorter`` owns a workspace and a result word on one device and sorts
lists held in torch device tensors (``next`` uint32 as int32 storage, keys of
8/16/32/64 bits).  Every step runs in libpbit's HIP kernels; this module only
allocates device memory through torch and passes pointers.
"""
from __future__ import annotations

import torch

from . import _lib

_KEY_BITS = {torch.uint8: 8, torch.int8: 8, torch.int16: 16, torch.uint16: 16,
             torch.int32: 32, torch.uint32: 32, torch.int64: 64, torch.uint64: 64,
             torch.float16: 16, torch.bfloat16: 16, torch.float32: 32, torch.float64: 64}


def key_bits(keys: torch.Tensor) -> int:
    try:
        return _KEY_BITS[keys.dtype]
    except KeyError:
        raise TypeError("unsupported key dtype %s" % keys.dtype) from None


def key_flags(keys: torch.Tensor, descending: bool, signed: bool, shared: bool = False) -> int:
    """Flag word for a key tensor: floating-point dtypes sort by value;
    ``shared``: other sorts may run on the device at the same time."""
    flags = _lib.DESCENDING if descending else 0
    if shared:
        flags |= _lib.SHARED
    if keys.is_floating_point():
        if signed:
            raise ValueError("signed applies to integer keys only")
        flags |= _lib.FLOAT
    elif signed:
        flags |= _lib.SIGNED
    return flags


def _retire(ws, streams):
    """Before a workspace grown on demand is dropped: sorts queued on side
    streams may still use it, so the caching allocator must not hand its
    memory out again before those streams pass this point."""
    if ws is not None:
        for s in streams:
            ws.record_stream(s)
    streams.clear()


def _note_stream(streams, stream, *tensors):
    """A call queued on a stream other than the current one: remember the
    stream for the workspace and keep the result words alive for it."""
    if stream is None or stream == torch.cuda.current_stream(stream.device):
        return
    if all(s != stream for s in streams):
        streams.append(stream)
    for t in tensors:
        t.record_stream(stream)


class PbitError(RuntimeError):
    def __init__(self, code: int):
        super().__init__("%s (%d)" % (_lib.status_string(code), code))
        self.code = code


class ListSorter:
    """Sort singly-linked lists stored as device arrays.

    next: int32/uint32 tensor of n node indices (0xFFFFFFFF ends the list).
    keys: n unsigned (or, with ``signed=True``, two's-complement) integers, or
    floating-point values (float16/bfloat16/float32/float64), sorted by value.

    A sorter holds one workspace and one result word, so sorts that may run at
    the same time (queued on different streams) need a sorter each.  A sort
    queued on a side stream keeps the workspace it used alive for that stream
    when a later, larger sort replaces it.
    """

    def __init__(self, device="cuda"):
        self.device = torch.device(device)
        self._ws = None
        self._ws_bytes = 0
        self._ws_streams = []
        self.result = torch.zeros(2, dtype=torch.int32, device=self.device)

    def workspace(self, n: int, M: int, K: int = 0) -> torch.Tensor:
        need = _lib.workspace_bytes(n, M, K)
        if need == 0:
            raise PbitError(_lib.EINVAL)
        if self._ws is None or self._ws_bytes < need:
            _retire(self._ws, self._ws_streams)
            self._ws = None
            self._ws = torch.empty(need, dtype=torch.uint8, device=self.device)
            self._ws_bytes = need
        return self._ws

    def sort_async(self, head: int, next_in: torch.Tensor, keys: torch.Tensor, K: int = 0,
                   descending: bool = False, signed: bool = False,
                   next_out: torch.Tensor | None = None, result: torch.Tensor | None = None,
                   stream=None, prev_out: torch.Tensor | None = None,
                   shared: bool = False) -> torch.Tensor:
        """Queue the sort; returns the 2-word device result {head, status}.

        With ``prev_out`` (n uint32 entries, not the next array) the list is
        treated as doubly linked and its backward links are rebuilt after the
        relink."""
        n = int(next_in.numel())
        M = key_bits(keys)
        if int(keys.numel()) != n:
            raise ValueError("keys and next differ in length")
        if next_out is None:
            next_out = next_in
        if result is None:
            result = self.result
        ws = self.workspace(n, M, K)
        _note_stream(self._ws_streams, stream, result)
        flags = key_flags(keys, descending, signed, shared)
        st = _lib.sort_list_async(head, next_in, next_out, keys, n, M, K, flags, result, ws,
                                  self._ws_bytes, stream)
        if st == _lib.OK and prev_out is not None:
            st = _lib.repair_prev(result, 1, next_out, prev_out, n, result, 4, stream)
        if st != _lib.OK:
            raise PbitError(st)
        return result

    def sort(self, head: int, next_in: torch.Tensor, keys: torch.Tensor, K: int = 0,
             descending: bool = False, signed: bool = False,
             next_out: torch.Tensor | None = None,
             prev_out: torch.Tensor | None = None) -> int:
        """Sort and wait; returns the new head (0xFFFFFFFF if empty)."""
        res = self.sort_async(head, next_in, keys, K, descending, signed, next_out,
                              prev_out=prev_out)
        h, st = (int(x) for x in res.cpu().tolist())
        if st != 0:
            raise PbitError(st)
        return h & 0xFFFFFFFF


    def sort_aos_async(self, head: int, nodes: torch.Tensor, n: int, stride: int, next_off: int,
                       key_off: int, M: int, K: int = 0, descending: bool = False,
                       signed: bool = False, floating: bool = False, result=None,
                       stream=None) -> torch.Tensor:
        """Sort nodes stored as records of ``stride`` bytes in ``nodes`` (any
        dtype; byte offsets): the next index is the uint32 at ``next_off``, the
        key the M-bit value at ``key_off``.  Links are rewritten in place."""
        if result is None:
            result = self.result
        if int(nodes.numel()) * nodes.element_size() < n * stride:
            raise ValueError("nodes holds fewer than n records")
        ws = self.workspace(n, M, K)
        _note_stream(self._ws_streams, stream, result)
        flags = ((_lib.DESCENDING if descending else 0) | (_lib.SIGNED if signed else 0)
                 | (_lib.FLOAT if floating else 0))
        st = _lib.sort_list_aos_async(head, nodes, stride, next_off, key_off, n, M, K, flags,
                                      result, ws, self._ws_bytes, stream)
        if st != _lib.OK:
            raise PbitError(st)
        return result

    def sort_aos(self, head: int, nodes: torch.Tensor, n: int, stride: int, next_off: int,
                 key_off: int, M: int, K: int = 0, **kw) -> int:
        res = self.sort_aos_async(head, nodes, n, stride, next_off, key_off, M, K, **kw)
        h, st = (int(x) for x in res.cpu().tolist())
        if st != 0:
            raise PbitError(st)
        return h & 0xFFFFFFFF


class ListsSorter:
    """Sort many lists in one launch sequence (lists in contiguous node slabs).

    heads: int32/uint32 tensor [L]; offsets: int64 tensor [L+1] of slab bounds;
    next/keys: shared device arrays over all slabs.
    Like ``ListSorter``: one sorter per stream for sorts that may overlap.
    """

    def __init__(self, device="cuda"):
        self.device = torch.device(device)
        self._ws = None
        self._ws_bytes = 0
        self._ws_streams = []
        self.status = torch.zeros(1, dtype=torch.int32, device=self.device)

    def workspace(self, total: int, num_lists: int, M: int, K: int = 0) -> torch.Tensor:
        need = _lib.lists_workspace_bytes(total, num_lists, M, K)
        if need == 0:
            raise PbitError(_lib.EINVAL)
        if self._ws is None or self._ws_bytes < need:
            _retire(self._ws, self._ws_streams)
            self._ws = None
            self._ws = torch.empty(need, dtype=torch.uint8, device=self.device)
            self._ws_bytes = need
        return self._ws

    def sort_async(self, heads, offsets, next_in, keys, K: int = 0, descending: bool = False,
                   signed: bool = False, next_out=None, new_heads=None, status=None,
                   stream=None, prev_out=None, shared: bool = False):
        L = int(heads.numel())
        total = int(next_in.numel())
        M = key_bits(keys)
        if next_out is None:
            next_out = next_in
        if new_heads is None:
            new_heads = torch.empty(L, dtype=torch.int32, device=self.device)
        if status is None:
            status = self.status
        ws = self.workspace(total, L, M, K)
        _note_stream(self._ws_streams, stream, new_heads, status)
        flags = key_flags(keys, descending, signed, shared)
        st = _lib.sort_lists(heads, offsets, L, total, next_in, next_out, keys, M, K, flags,
                             new_heads, status, ws, self._ws_bytes, stream)
        if st == _lib.OK and prev_out is not None:
            st = _lib.repair_prev(new_heads, L, next_out, prev_out, total, status, 0, stream)
        if st != _lib.OK:
            raise PbitError(st)
        return new_heads, status

    def sort(self, heads, offsets, next_in, keys, K: int = 0, descending: bool = False,
             signed: bool = False, next_out=None, prev_out=None):
        new_heads, status = self.sort_async(heads, offsets, next_in, keys, K, descending, signed,
                                            next_out, prev_out=prev_out)
        st = int(status.item())
        if st != 0:
            raise PbitError(st)
        return new_heads
