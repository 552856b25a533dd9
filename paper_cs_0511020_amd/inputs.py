"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle runs.

This module only draws random lists and keys; it holds none of the sorting
method's arithmetic.  Every generator takes a numpy ``Generator`` (PCG64) or a
seed so that the CPU oracle and the GPU path see byte-identical inputs.

A list over nodes 0..n-1 is stored structure-of-arrays: ``next[i]`` is the
index of the node after i (NIL = 0xFFFFFFFF ends the list) and ``head`` is the
first node.  The list order is a uniformly random permutation of the nodes, so
node order in memory is unrelated to list order (a random single cycle cut
open in front of a random head).
"""
from __future__ import annotations

import numpy as np

NIL = np.uint32(0xFFFFFFFF)

KEY_DTYPES = {8: np.uint8, 16: np.uint16, 32: np.uint32, 64: np.uint64}

# The paper's 8-node example (Sec. 3): one-byte keys in list order 0 -> 7.
WORKED_EXAMPLE_KEYS = np.array([21, 3, 209, 14, 156, 47, 3, 214], dtype=np.uint8)


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def links_from_order(order: np.ndarray, n: int | None = None):
    """next[] and head for the list visiting ``order`` (node ids) in sequence."""
    order = np.asarray(order, dtype=np.uint32)
    if n is None:
        n = order.shape[0]
    nxt = np.full(n, NIL, dtype=np.uint32)
    if order.shape[0] == 0:
        return nxt, int(NIL)
    nxt[order[:-1]] = order[1:]
    nxt[order[-1]] = NIL
    return nxt, int(order[0])


def random_list(n: int, rng: np.random.Generator):
    """Random layout: (next, head, order) with order a uniform permutation."""
    order = rng.permutation(n).astype(np.uint32)
    nxt, head = links_from_order(order, n)
    return nxt, head, order


def identity_list(n: int):
    """next[i] = i + 1: list order equals memory order."""
    order = np.arange(n, dtype=np.uint32)
    nxt, head = links_from_order(order, n)
    return nxt, head, order


def uniform_keys(n: int, M: int, rng: np.random.Generator) -> np.ndarray:
    dt = KEY_DTYPES[M]
    info = np.iinfo(dt)
    return rng.integers(0, int(info.max), size=n, dtype=dt, endpoint=True)


def zipf_keys(n: int, rng: np.random.Generator, s: float = 1.1,
              distinct: int = 1 << 16) -> np.ndarray:
    """u32 keys: ``distinct`` values drawn without repeats, rank r picked with
    probability proportional to r^-s (truncated table, inverse CDF)."""
    values = rng.choice(np.uint64(1) << np.uint64(32), size=distinct, replace=False)
    values = values.astype(np.uint32)
    ranks = np.arange(1, distinct + 1, dtype=np.float64)
    cdf = np.cumsum(ranks ** (-s))
    cdf /= cdf[-1]
    u = rng.random(n)
    r = np.searchsorted(cdf, u, side="right")
    r = np.minimum(r, distinct - 1)
    perm = rng.permutation(distinct)
    return values[perm[r]]


def few_distinct_keys(n: int, rng: np.random.Generator, count: int = 8,
                      M: int = 32) -> np.ndarray:
    dt = KEY_DTYPES[M]
    info = np.iinfo(dt)
    values = rng.choice(int(info.max) + 1 if M < 64 else (1 << 63), size=count, replace=False)
    values = np.asarray(values).astype(dt)
    return values[rng.integers(0, count, size=n)]


FLOAT_DTYPES = {16: np.float16, 32: np.float32, 64: np.float64}


def float_keys(n: int, M: int, rng: np.random.Generator, specials: bool = True) -> np.ndarray:
    """IEEE-754 keys of width M (binary16/32/64), returned as their bit
    patterns in the unsigned M-bit dtype.  Values of both signs spread over the
    whole exponent range (log-uniform magnitudes), a pool of repeated values,
    and, with ``specials``, a sprinkling of +-0, subnormals, +-inf and NaNs of
    both signs."""
    ft = FLOAT_DTYPES[M]
    fi = np.finfo(ft)
    lo, hi = np.log2(float(fi.tiny)), np.log2(float(fi.max)) - 1.0
    mag = np.exp2(rng.uniform(lo, hi, size=n))
    sign = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    vals = (sign * mag).astype(ft)
    pool = vals[rng.integers(0, max(1, n), size=max(1, n // 16))] if n else vals
    rep = rng.random(n) < 0.25
    if n:
        vals[rep] = pool[rng.integers(0, pool.shape[0], size=int(rep.sum()))]
    bits = vals.view(KEY_DTYPES[M]).copy()
    if specials and n:
        one = KEY_DTYPES[M](1)
        top = KEY_DTYPES[M](one << KEY_DTYPES[M](M - 1))
        nm = fi.nmant
        exp_all = KEY_DTYPES[M](((1 << (M - 1 - nm)) - 1) << nm)
        choices = [
            KEY_DTYPES[M](0), top,                          # +0, -0
            one, top | one,                                 # smallest subnormals
            exp_all, top | exp_all,                         # +inf, -inf
            exp_all | one, top | exp_all | one,             # NaNs of both signs
            exp_all | KEY_DTYPES[M](1 << (nm - 1)),         # quiet NaN
            top | exp_all | KEY_DTYPES[M]((1 << nm) - 1),   # NaN, all mantissa bits
        ]
        sp = rng.random(n) < 0.02
        bits[sp] = np.asarray(choices, dtype=KEY_DTYPES[M])[rng.integers(0, len(choices),
                                                                          size=int(sp.sum()))]
    return bits


def keys_by_distribution(dist: str, n: int, rng: np.random.Generator) -> np.ndarray:
    if dist == "uniform":
        return uniform_keys(n, 32, rng)
    if dist == "zipf":
        return zipf_keys(n, rng)
    if dist == "distinct8":
        return few_distinct_keys(n, rng, 8, 32)
    raise ValueError(dist)


def log_uniform_lengths(count: int, lo_log2: float, hi_log2: float,
                        rng: np.random.Generator, lo: int, hi: int) -> np.ndarray:
    u = rng.random(count)
    lens = np.floor(2.0 ** (lo_log2 + (hi_log2 - lo_log2) * u)).astype(np.int64)
    return np.clip(lens, lo, hi)


def slab_lists(lengths, rng: np.random.Generator):
    """Many lists in contiguous node slabs; each slab gets its own random layout.

    Returns (next, heads, offsets) with global node indices inside each slab.
    """
    lengths = np.asarray(lengths, dtype=np.int64)
    offsets = np.zeros(lengths.shape[0] + 1, dtype=np.uint64)
    offsets[1:] = np.cumsum(lengths)
    total = int(offsets[-1])
    nxt = np.full(total, NIL, dtype=np.uint32)
    heads = np.full(lengths.shape[0], NIL, dtype=np.uint32)
    for l, ln in enumerate(lengths):
        if ln == 0:
            continue
        lo = int(offsets[l])
        order = (rng.permutation(int(ln)) + lo).astype(np.uint32)
        nxt[order[:-1]] = order[1:]
        nxt[order[-1]] = NIL
        heads[l] = order[0]
    return nxt, heads, offsets


def slab_lists_device(lengths, seed: int, M: int = 32, device="cuda", local_copy: bool = False):
    """The same recipe as ``slab_lists`` generated on the GPU with torch
    (for batches too large to build on the host): each slab gets its own
    uniformly random list order (torch.randperm) and a random head; keys are
    uniform M-bit values.

    Returns dict(next, heads, offsets, keys[, next_local]) of device tensors
    (int32/int64 storage); ``next_local`` holds slab-local indices, for
    sorting one list at a time with the single-list entry point.
    """
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    lengths = np.asarray(lengths, dtype=np.int64)
    offsets = np.zeros(lengths.shape[0] + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(lengths)
    total = int(offsets[-1])
    nxt = torch.full((total,), -1, dtype=torch.int32, device=device)
    loc = torch.full((total,), -1, dtype=torch.int32, device=device) if local_copy else None
    heads = np.full(lengths.shape[0], 0xFFFFFFFF, dtype=np.uint32)
    for l, ln in enumerate(lengths):
        ln = int(ln)
        if ln == 0:
            continue
        lo = int(offsets[l])
        perm = torch.randperm(ln, generator=g, device=device, dtype=torch.int64)
        seg = nxt[lo:lo + ln]
        seg[perm[:-1]] = (perm[1:] + lo).to(torch.int32)
        if loc is not None:
            lseg = loc[lo:lo + ln]
            lseg[perm[:-1]] = perm[1:].to(torch.int32)
        heads[l] = lo + int(perm[0].item())
    if M == 8:
        keys = torch.randint(0, 256, (total,), generator=g, device=device, dtype=torch.uint8)
    elif M == 16:
        keys = torch.randint(-(1 << 15), 1 << 15, (total,), generator=g, device=device,
                             dtype=torch.int16)
    elif M == 32:
        keys = torch.randint(-(1 << 31), 1 << 31, (total,), generator=g, device=device,
                             dtype=torch.int32)
    else:
        hi = torch.randint(-(1 << 31), 1 << 31, (total,), generator=g, device=device,
                           dtype=torch.int64)
        lo = torch.randint(0, 1 << 32, (total,), generator=g, device=device, dtype=torch.int64)
        keys = (hi << 32) | lo
    out = {
        "next": nxt,
        "heads": torch.from_numpy(heads.view(np.int32)).to(device),
        "heads_host": heads,
        "offsets": torch.from_numpy(offsets).to(device),
        "offsets_host": offsets,
        "keys": keys,
    }
    if loc is not None:
        out["next_local"] = loc
    return out
