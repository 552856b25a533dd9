"""MI355X (gfx950) Pbit list sort: a singly-linked list, stored as device
arrays, is re-linked into stable key order by hand-written HIP kernels behind
the C ABI of include/pbit.h (Planeta, arXiv cs/0511020).
"""
from ._lib import (ASCENDING, DESCENDING, EHIP, EINVAL, EMALFORMED, ENOMEM, NIL, OK,  # noqa: F401
                   SIGNED, load, status_string, version, workspace_bytes)

__all__ = ["ListSorter", "load", "workspace_bytes", "status_string", "version", "NIL"]


def __getattr__(name):
    if name in ("ListSorter", "PbitError"):
        from . import sorter
        return getattr(sorter, name)
    raise AttributeError(name)
