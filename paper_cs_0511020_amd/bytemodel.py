"""Algorithmic byte counts of the sort, per node.

Two models are kept apart:

* ``path_bytes_per_node`` is the fixed model of the whole sort used for the
  path-level roofline: walk-1 reads next (4 B); walk-2 reads next and key and
  writes key and node index in list order (8 + 2w); every pass but the last
  reads and writes (key, index) (2(w + 4)); the last pass reads (key, index)
  and writes the index (w + 8 counting the index read and write of the
  relink input); the relink reads the order and writes next (8).
  B = 28 + 3w + (P - 1)(2w + 8), w = key bytes, P = executed passes.
  Every element access counts once at its element size, random ones included.

* ``kernel_bytes_per_node`` counts, for one kernel of this implementation,
  the element bytes it reads and writes once each; a kernel's roofline uses
  it with the number of nodes one launch processes.
"""
from __future__ import annotations

MI355X_HBM_PEAK_GBS = 8000.0  # GB/s, published HBM3E peak


def record_bytes(w: int) -> int:
    """Packed node record (next + key): 8 bytes up to 32-bit keys, else 16."""
    return 16 if w == 8 else 8


def entry_bytes(w: int) -> int:
    """Walk buffer entry (key + node index): 8 bytes up to 32-bit keys, else 16."""
    return 16 if w == 8 else 8


def path_bytes_per_node(w: int, passes: int) -> int:
    return 28 + 3 * w + (passes - 1) * (2 * w + 8)


def kernel_bytes_per_node(stage: str, w: int, last_pass: bool = False) -> int:
    if stage == "pack":
        return 4 + w + record_bytes(w)
    if stage == "walk0":
        return record_bytes(w) + entry_bytes(w)
    if stage == "unchain":
        return entry_bytes(w) + w + 4
    if stage == "digit_pass":
        return (w + 4) + (4 if last_pass else w + 4)
    if stage == "relink":
        return 8
    raise KeyError(stage)
