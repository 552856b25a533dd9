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


def float_value_key(b, M):
    """The order the floating-point reading defines, computed from the values:
    numeric order, -0 before +0, NaNs outside the infinities on the side of
    their sign bit (a larger payload further out)."""
    import math
    ft = inputs.FLOAT_DTYPES[M]
    b = int(b)
    v = float(np.array([b], dtype=inputs.KEY_DTYPES[M]).view(ft)[0])
    neg = (b >> (M - 1)) & 1
    if math.isnan(v):
        payload = b & ((1 << (M - 1)) - 1)
        return (0, -payload, 0) if neg else (2, payload, 0)
    return (1, v, 0 if neg else 1)


@pytest.mark.parametrize("M", [16, 32, 64])
def test_float_keys_against_value_order(oracle_mod, M):
    rng = inputs.rng_for(700 + M)
    n = 3000
    nxt, head, order = inputs.random_list(n, rng)
    keys = inputs.float_keys(n, M, rng)
    vk = [float_value_key(k, M) for k in keys]
    for K in (4, 8):
        for flags, desc in [(oracle_mod.FLAG_FLOAT, False),
                            (oracle_mod.FLAG_FLOAT | oracle_mod.FLAG_DESCENDING, True)]:
            h, out = oracle_mod.sort_list(head, nxt, keys, M, K, flags=flags)
            exp = sorted(order.tolist(), key=lambda i: vk[i], reverse=desc)
            assert walk(h, out) == exp, (M, K, desc)


def test_float_finite_against_numpy(oracle_mod):
    """Finite non-zero values: numpy's stable argsort of the values themselves."""
    rng = inputs.rng_for(711)
    for M in (16, 32, 64):
        n = 2000
        nxt, head, order = inputs.random_list(n, rng)
        keys = inputs.float_keys(n, M, rng, specials=False)
        vals = keys.view(inputs.FLOAT_DTYPES[M])[order]
        assert np.all(np.isfinite(vals)) and np.all(vals != 0)
        h, out = oracle_mod.sort_list(head, nxt, keys, M, 8, flags=oracle_mod.FLAG_FLOAT)
        assert walk(h, out) == order[np.argsort(vals, kind="stable")].tolist()
        h, out = oracle_mod.sort_list(head, nxt, keys, M, 8,
                                      flags=oracle_mod.FLAG_FLOAT | oracle_mod.FLAG_DESCENDING)
        assert walk(h, out) == order[np.argsort(-vals, kind="stable")].tolist()


def test_float_hand_order(oracle_mod):
    """binary32 specials in a fixed scrambled list; the expected order is written out."""
    pats = {
        "-nan": 0xFFC00000, "-inf": 0xFF800000, "-3.5": 0xC0600000, "-den": 0x80000001,
        "-0": 0x80000000, "+0": 0x00000000, "+den": 0x00000001, "2": 0x40000000,
        "+inf": 0x7F800000, "+nan": 0x7FC00000,
    }
    names = ["2", "-0", "+nan", "-3.5", "+den", "-inf", "+0", "-nan", "+inf", "-den"]
    keys = np.array([pats[x] for x in names], dtype=np.uint32)
    nxt, head, _ = inputs.identity_list(len(names))
    h, out = oracle_mod.sort_list(head, nxt, keys, 32, 8, flags=oracle_mod.FLAG_FLOAT)
    assert [names[i] for i in walk(h, out)] == [
        "-nan", "-inf", "-3.5", "-den", "-0", "+0", "+den", "2", "+inf", "+nan"]
    h, out = oracle_mod.sort_list(head, nxt, keys, 32, 4,
                                  flags=oracle_mod.FLAG_FLOAT | oracle_mod.FLAG_DESCENDING)
    assert [names[i] for i in walk(h, out)] == [
        "+nan", "+inf", "2", "+den", "+0", "-0", "-den", "-3.5", "-inf", "-nan"]


@pytest.mark.parametrize("M", [16, 32, 64])
def test_float_two_pass_reading(oracle_mod, M):
    """Sec. 14 sorts non-negative floats on the mantissa, then stably on the
    characteristic; two unsigned sorts on those fields give the same list as
    one floating-point sort."""
    rng = inputs.rng_for(720 + M)
    n = 2500
    nxt, head, order = inputs.random_list(n, rng)
    keys = inputs.float_keys(n, M, rng)
    top = inputs.KEY_DTYPES[M](1) << inputs.KEY_DTYPES[M](M - 1)
    keys = keys & ~top  # non-negative: clear the sign bit
    nm = np.finfo(inputs.FLOAT_DTYPES[M]).nmant
    mant = keys & inputs.KEY_DTYPES[M]((1 << nm) - 1)
    char_w = {16: 8, 32: 8, 64: 16}[M]
    char = (keys >> inputs.KEY_DTYPES[M](nm)).astype(inputs.KEY_DTYPES[char_w])
    h1, o1 = oracle_mod.sort_list(head, nxt, mant, M, 8)
    h2, o2 = oracle_mod.sort_list(h1, o1, char, char_w, 8)
    hf, of = oracle_mod.sort_list(head, nxt, keys, M, 8, flags=oracle_mod.FLAG_FLOAT)
    assert h2 == hf and np.array_equal(o2, of)
    assert walk(hf, of) == sorted(order.tolist(), key=lambda i: float_value_key(keys[i], M))


def test_float_and_signed_rejected(oracle_mod):
    nxt, head, _ = inputs.identity_list(4)
    keys = np.arange(4, dtype=np.uint32)
    h, _ = oracle_mod.sort_list(head, nxt, keys, 32, 8,
                                flags=oracle_mod.FLAG_FLOAT | oracle_mod.FLAG_SIGNED)
    assert h == oracle_mod.EINVAL


def test_repair_prev_reverses_the_walk(oracle_mod):
    """Sec. 13: after the repair, walking backward from the tail meets the
    nodes of the forward walk in reverse, and the head's backward link is NIL."""
    rng = inputs.rng_for(730)
    for n in (1, 2, 3, 50, 4097):
        nxt, head, order = inputs.random_list(n, rng)
        keys = inputs.uniform_keys(n, 16, rng)
        h, out = oracle_mod.sort_list(head, nxt, keys, 16, 4)
        prev = oracle_mod.repair_prev(h, out)
        fwd = walk(h, out)
        back, i = [], fwd[-1]
        while i != NIL:
            back.append(i)
            i = int(prev[i])
            assert len(back) <= n
        assert back == fwd[::-1]
        assert prev[h] == NIL
        # brute force: the predecessor of j is the one node whose next is j
        for j in fwd[1:]:
            assert np.nonzero(out == j)[0].tolist() == [int(prev[j])]


def test_repair_prev_hand_case_and_errors(oracle_mod):
    # list 2 -> 0 -> 3 -> 1; node 4 is not on it and keeps its value
    nxt = np.array([3, NIL, 0, 1, NIL], dtype=np.uint32)
    prev = oracle_mod.repair_prev(2, nxt, prev=np.full(5, 77, dtype=np.uint32))
    assert prev.tolist() == [2, 3, NIL, 0, 77]
    with pytest.raises(ValueError):
        oracle_mod.repair_prev(0, np.array([1, 0], dtype=np.uint32))   # cycle
    with pytest.raises(ValueError):
        oracle_mod.repair_prev(0, np.array([5, NIL], dtype=np.uint32))  # index out of range
    assert oracle_mod.repair_prev(NIL, np.zeros(0, dtype=np.uint32)).shape == (0,)


@pytest.mark.parametrize("M,K", [(8, 4), (16, 2), (32, 8), (32, 4), (64, 8)])
def test_threaded_variant_against_numpy(oracle_mod, M, K):
    """The multi-threaded form (top levels split on the caller's thread, the
    groups below sorted on worker threads and joined in pattern order) gives
    the definition's result: numpy's stable argsort of the list order, either
    direction, for any thread count; heavy ties included."""
    rng = inputs.rng_for(660 + M + K)
    for n, threads in [(1, 1), (2, 3), (300, 2), (20000, 5), (100003, 0)]:
        nxt, head, order = inputs.random_list(n, rng)
        keys = inputs.uniform_keys(n, M, rng)
        keys[::3] = keys[0]
        h, out = oracle_mod.sort_list_threads(head, nxt, keys, M, K, threads=threads)
        exp = order[np.argsort(keys[order], kind="stable")]
        assert h == exp[0] and walk(h, out) == exp.tolist()
        h, out = oracle_mod.sort_list_threads(head, nxt, keys, M, K,
                                              flags=oracle_mod.FLAG_DESCENDING, threads=threads)
        expd = order[np.argsort(~keys[order], kind="stable")]
        assert h == expd[0] and walk(h, out) == expd.tolist()


def test_threaded_variant_rejections(oracle_mod):
    nxt, head, _ = inputs.random_list(10, inputs.rng_for(3))
    keys = np.arange(10, dtype=np.uint32)
    for f in (oracle_mod.FLAG_SIGNED, oracle_mod.FLAG_FLOAT, oracle_mod.FLAG_LIFO):
        assert oracle_mod.sort_list_threads(head, nxt, keys, 32, 8, flags=f)[0] == -1
    assert oracle_mod.sort_list_threads(head, nxt, keys, 32, 3)[0] == -1
    bad = nxt.copy()
    bad[head] = head
    assert oracle_mod.sort_list_threads(head, bad, keys, 32, 8)[0] == -2
