"""Pins of the CPU oracle against facts fixed outside the oracle itself.

- the paper's worked example (Sec. 3), stored in tests/golden/worked_example.json;
- exhaustive brute force on tiny lists against Python's stable ``sorted``;
- numpy's stable argsort on random lists (the plain definition of the result:
  walk, stable sort by key, relink);
- invariants the paper states: every node is walked exactly once by the merges
  (Sec. 5.1), every node is visited once per level (Sec. 3, f(n) = (M/K) n + n),
  recursion depth M/K;
- the push-front reading: the printed listings reverse equal keys once per
  level, so they agree with the stable result exactly when M/K is even.
"""
import itertools
import json
import os

import numpy as np
import pytest

from paper_cs_0511020_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))
NIL = 0xFFFFFFFF


def walk(head, nxt):
    out = []
    i = head
    while i != NIL:
        out.append(int(i))
        i = int(nxt[i])
        assert len(out) <= len(nxt)
    return out


def expected_order(order, keys, descending=False, signed=False):
    """Stable sort of the list order by key (the definition of the result)."""
    vals = [int(k) for k in keys]
    if signed:
        bits = keys.dtype.itemsize * 8
        vals = [v - (1 << bits) if v >> (bits - 1) else v for v in vals]
    if descending:
        return sorted(order, key=lambda i: -vals[i])
    return sorted(order, key=lambda i: vals[i])


def golden():
    with open(os.path.join(HERE, "golden", "worked_example.json")) as f:
        return json.load(f)


def test_worked_example_ascending(oracle_mod):
    g = golden()
    keys = np.array(g["keys_in_list_order"], dtype=np.uint8)
    nxt, head = inputs.links_from_order(np.arange(8))
    h, out, cnt = oracle_mod.sort_list(head, nxt, keys, g["M"], g["K"], counters=True)
    assert h == g["ascending_head"]
    assert out.tolist() == g["ascending_next"]
    assert walk(h, out) == g["ascending_node_order"]
    sorted_keys = [int(keys[i]) for i in walk(h, out)]
    flat = [k for grp in g["paper_second_level_groups"] for k in grp]
    assert sorted_keys == flat
    assert cnt[0] == 8  # merge walks every node once


def test_worked_example_first_level_groups(oracle_mod):
    """Sorting on the high pattern only reproduces the printed first split,
    including the list order {3,14,3} inside the first group."""
    g = golden()
    keys = np.array(g["keys_in_list_order"], dtype=np.uint8)
    high_only = (keys & 0xF0).astype(np.uint8)
    nxt, head = inputs.links_from_order(np.arange(8))
    h, out = oracle_mod.sort_list(head, nxt, high_only, 8, 4)
    order = walk(h, out)
    assert order == g["first_level_node_order"]
    groups = []
    for i in order:
        d = int(keys[i]) >> 4
        if not groups or groups[-1][0] != d:
            groups.append((d, []))
        groups[-1][1].append(int(keys[i]))
    assert [grp for _, grp in groups] == g["paper_first_level_groups"]


def test_worked_example_descending(oracle_mod):
    g = golden()
    keys = np.array(g["keys_in_list_order"], dtype=np.uint8)
    nxt, head = inputs.links_from_order(np.arange(8))
    h, out = oracle_mod.sort_list(head, nxt, keys, 8, 4, flags=oracle_mod.FLAG_DESCENDING)
    assert h == g["descending_head"]
    assert out.tolist() == g["descending_next"]
    # the printed listing (push-front groups, descending) gives the same here: M/K = 2
    h2, out2 = oracle_mod.sort_list(head, nxt, keys, 8, 4,
                                    flags=oracle_mod.FLAG_DESCENDING | oracle_mod.FLAG_LIFO)
    assert h2 == h and out2.tolist() == out.tolist()


def _alphabet(M):
    top = (1 << M) - 1
    return [0, 1, 1 << (M - 1), top]


@pytest.mark.parametrize("M,K", [(8, 4), (8, 8), (8, 2), (8, 1), (16, 4), (16, 16),
                                 (32, 8), (32, 4), (64, 8), (64, 16)])
def test_bruteforce_all_layouts(oracle_mod, M, K):
    """Every list order of n<=5 nodes, key tuples from an alphabet holding the
    extreme values, against Python's stable sort."""
    dt = inputs.KEY_DTYPES[M]
    alpha = _alphabet(M)
    rng = inputs.rng_for(7 + M + K)
    for n in range(1, 6):
        tuples = list(itertools.product(alpha[:3], repeat=n)) if n <= 4 else \
            [tuple(alpha[j] for j in rng.integers(0, len(alpha), size=n)) for _ in range(12)]
        for kt in tuples[:40]:
            keys = np.array(kt, dtype=dt)
            for order in itertools.permutations(range(n)):
                nxt, head = inputs.links_from_order(np.array(order))
                h, out = oracle_mod.sort_list(head, nxt, keys, M, K)
                got = walk(h, out)
                assert got == expected_order(list(order), keys), (M, K, kt, order)


@pytest.mark.parametrize("M", [8, 16, 32, 64])
def test_random_against_numpy_stable_argsort(oracle_mod, M):
    rng = inputs.rng_for(100 + M)
    for n, span in [(1, 3), (2, 3), (37, 5), (1000, 7), (5000, None)]:
        nxt, head, order = inputs.random_list(n, rng)
        if span is None:
            keys = inputs.uniform_keys(n, M, rng)
        else:
            keys = rng.integers(0, span, size=n).astype(inputs.KEY_DTYPES[M])
            keys = keys << (M - 3)  # duplicates spread over the top patterns
        for K in [k for k in (1, 2, 4, 8, 16) if M % k == 0 and k <= M]:
            h, out = oracle_mod.sort_list(head, nxt, keys, M, K)
            lk = keys[order]
            exp = order[np.argsort(lk, kind="stable")]
            assert walk(h, out) == exp.tolist()


def test_counters_match_paper_invariants(oracle_mod):
    rng = inputs.rng_for(3)
    n = 3000
    nxt, head, _ = inputs.random_list(n, rng)
    for M in (8, 16, 32, 64):
        keys = inputs.uniform_keys(n, M, rng)
        for K in (1, 4, 8):
            h, out, (merges, visits, calls, depth) = oracle_mod.sort_list(
                head, nxt, keys, M, K, counters=True)
            assert merges == n             # Sec. 5.1: merge walks n nodes in all
            assert visits == n * (M // K)  # Sec. 3: (M/K) n split visits
            assert depth == M // K


@pytest.mark.parametrize("M,K", [(8, 8), (16, 4), (32, 4), (32, 8), (64, 8), (16, 8), (32, 16)])
def test_push_front_reading(oracle_mod, M, K):
    """Push-front groups (the printed code) equal FIFO groups when M/K is even
    and list the ties in reverse when M/K is odd."""
    rng = inputs.rng_for(11)
    n = 400
    nxt, head, order = inputs.random_list(n, rng)
    keys = rng.integers(0, 6, size=n).astype(inputs.KEY_DTYPES[M]) << (M - 3)
    h, out = oracle_mod.sort_list(head, nxt, keys, M, K)
    hl, outl = oracle_mod.sort_list(head, nxt, keys, M, K, flags=oracle_mod.FLAG_LIFO)
    fifo, lifo = walk(h, out), walk(hl, outl)
    if (M // K) % 2 == 0:
        assert fifo == lifo
    else:
        assert fifo != lifo
        # same key sequence, each run of equal keys reversed
        assert [keys[i] for i in fifo] == [keys[i] for i in lifo]
        i = 0
        while i < n:
            j = i
            while j < n and keys[fifo[j]] == keys[fifo[i]]:
                j += 1
            assert lifo[i:j] == fifo[i:j][::-1]
            i = j


def test_descending_and_signed(oracle_mod):
    rng = inputs.rng_for(5)
    for M in (8, 16, 32, 64):
        n = 700
        nxt, head, order = inputs.random_list(n, rng)
        keys = rng.integers(0, 9, size=n).astype(inputs.KEY_DTYPES[M])
        keys = keys * inputs.KEY_DTYPES[M]((1 << (M - 3)) - 1)
        for flags, desc, sgn in [(0, False, False), (oracle_mod.FLAG_DESCENDING, True, False),
                                 (oracle_mod.FLAG_SIGNED, False, True),
                                 (oracle_mod.FLAG_SIGNED | oracle_mod.FLAG_DESCENDING, True, True)]:
            h, out = oracle_mod.sort_list(head, nxt, keys, M, 4, flags=flags)
            assert walk(h, out) == expected_order(order.tolist(), keys, desc, sgn)


def test_special_cases(oracle_mod):
    rng = inputs.rng_for(9)
    n = 2000
    # all keys equal: the list is unchanged
    nxt, head, _ = inputs.random_list(n, rng)
    keys = np.full(n, 77, dtype=np.uint32)
    h, out = oracle_mod.sort_list(head, nxt, keys, 32, 4)
    assert h == head and np.array_equal(out, nxt)
    # already sorted: unchanged
    keys = np.sort(inputs.uniform_keys(n, 32, rng))
    order = rng.permutation(n)
    keys_by_node = np.empty_like(keys)
    keys_by_node[order] = keys
    nxt2, head2 = inputs.links_from_order(order)
    h, out = oracle_mod.sort_list(head2, nxt2, keys_by_node, 32, 8)
    assert h == head2 and np.array_equal(out, nxt2)
    # identity layout reduces to array stable sort
    nxt3, head3, _ = inputs.identity_list(n)
    keys3 = rng.integers(0, 50, size=n).astype(np.uint16)
    h, out = oracle_mod.sort_list(head3, nxt3, keys3, 16, 4)
    assert walk(h, out) == np.argsort(keys3, kind="stable").tolist()
    # single node: head kept, next untouched
    h, out = oracle_mod.sort_list(0, np.array([NIL], np.uint32), np.array([5], np.uint8), 8, 4)
    assert h == 0 and out.tolist() == [NIL]


def test_layout_invariance(oracle_mod):
    """Renaming the nodes commutes with the sort."""
    rng = inputs.rng_for(21)
    n = 1500
    nxt, head, order = inputs.random_list(n, rng)
    keys = rng.integers(0, 40, size=n).astype(np.uint32)
    h, out = oracle_mod.sort_list(head, nxt, keys, 32, 8)
    sigma = rng.permutation(n).astype(np.uint32)
    nxt_r, head_r = inputs.links_from_order(sigma[order], n)
    keys_r = np.empty_like(keys)
    keys_r[sigma] = keys
    h_r, out_r = oracle_mod.sort_list(head_r, nxt_r, keys_r, 32, 8)
    assert walk(h_r, out_r) == [int(sigma[i]) for i in walk(h, out)]


def test_malformed_and_empty(oracle_mod):
    keys = np.arange(6, dtype=np.uint32)
    good, head = inputs.links_from_order(np.array([3, 1, 4, 0, 5, 2]))
    # cycle
    bad = good.copy(); bad[2] = 3
    st, out = oracle_mod.sort_list(head, bad, keys, 32, 4)
    assert st == oracle_mod.EMALFORMED and np.array_equal(out, bad)
    # index out of range
    bad = good.copy(); bad[5] = 17
    assert oracle_mod.sort_list(head, bad, keys, 32, 4)[0] == oracle_mod.EMALFORMED
    # too short (a node not reachable from head)
    bad = good.copy(); bad[4] = NIL
    assert oracle_mod.sort_list(head, bad, keys, 32, 4)[0] == oracle_mod.EMALFORMED
    # bad shapes
    assert oracle_mod.sort_list(head, good, keys, 32, 3)[0] == oracle_mod.EINVAL
    assert oracle_mod.sort_list(9, good, keys, 32, 4)[0] == oracle_mod.EINVAL
    # empty list
    st, out = oracle_mod.sort_list(NIL, np.zeros(0, np.uint32), np.zeros(0, np.uint32), 32, 4)
    assert st == NIL


def test_segmented_equals_alone(oracle_mod):
    rng = inputs.rng_for(31)
    lengths = [0, 1, 5, 300, 17, 0, 2048]
    nxt, heads, offs = inputs.slab_lists(lengths, rng)
    keys = rng.integers(0, 30, size=nxt.shape[0]).astype(np.uint32)
    st, out, new_heads = oracle_mod.sort_lists(heads, offs, nxt, keys, 32, 4)
    assert st == 0
    for l, ln in enumerate(lengths):
        lo = int(offs[l])
        if ln == 0:
            assert new_heads[l] == NIL
            continue
        local_next = np.where(nxt[lo:lo + ln] == NIL, NIL, nxt[lo:lo + ln] - lo).astype(np.uint32)
        h, o = oracle_mod.sort_list(int(heads[l]) - lo, local_next, keys[lo:lo + ln], 32, 4)
        assert new_heads[l] == h + lo
        exp = np.where(o == NIL, NIL, o + lo).astype(np.uint32)
        assert np.array_equal(out[lo:lo + ln], exp)


def test_list_order(oracle_mod):
    rng = inputs.rng_for(41)
    nxt, head, order = inputs.random_list(999, rng)
    assert np.array_equal(oracle_mod.list_order(head, nxt), order)
