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
  it with the number of nodes one launch processes.  A digit pass reads and
  writes (key, index) pairs, except that the last pass writes indices only
  and, when node indices fit below one K-bit digit in 32 bits, the pass
  before it writes one 4-byte word (the last pass's digit over the index)
  that the last pass reads.
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


def kernel_bytes_per_node(stage: str, w: int, last_pass: bool = False,
                          packed_in: bool = False, packed_out: bool = False) -> int:
    if stage == "pack":
        return 4 + w + record_bytes(w)
    if stage == "walk0":
        return record_bytes(w) + entry_bytes(w)
    if stage == "unchain":
        return entry_bytes(w) + w + 4
    if stage == "digit_pass":
        return (4 if packed_in else w + 4) + (4 if last_pass or packed_out else w + 4)
    if stage == "relink":
        return 8
    raise KeyError(stage)


def packs_last_pass(n: int, K: int, executed: int) -> bool:
    """Whether the last two executed passes of one list exchange packed words:
    node indices (below n) must fit in 32 - K bits."""
    return executed >= 2 and n <= (1 << (32 - K))


def digit_pass_bytes_per_node(w: int, executed: int, n: int, K: int) -> float:
    """Mean element bytes per node of one digit-pass launch over a sort's
    executed passes (one list, no pattern skipped).  With 64-bit keys the
    passes over the high 32 bits move (high half, index) pairs of 8 bytes,
    which the last pass over the low half writes."""
    if executed <= 0:
        return 0.0
    pair = w + 4
    packed = packs_last_pass(n, K, executed)
    hi_from = executed // 2 if w == 8 else executed
    total = 0
    for p in range(executed):
        rd = 8 if p >= hi_from and p > 0 else pair
        if p == executed - 1:
            wr = 4
            if packed:
                rd = 4
        elif packed and p == executed - 2:
            wr = 4
        elif p + 1 >= hi_from:
            wr = 8
        else:
            wr = pair
        total += rd + wr
    return total / executed
