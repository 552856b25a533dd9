"""GPU parity of the batched form: many lists in node slabs sorted in one
launch sequence, bit-exact against the oracle's per-list sort and against the
single-list entry point run on each list alone."""
import numpy as np
import pytest

from paper_cs_0511020_amd import inputs

from .gpu_util import NIL, keys_to_dev, oracle_flags, to_dev

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_cs_0511020_amd import _lib
    _lib.load()


def gpu_sort_lists(heads, offsets, nxt, keys, K, flags=0, inplace=False, shared=False):
    import torch
    from paper_cs_0511020_amd.sorter import ListsSorter
    s = ListsSorter()
    ht = to_dev(heads.astype(np.uint32), torch)
    ot = torch.from_numpy(np.asarray(offsets, dtype=np.int64)).to("cuda")
    nt = to_dev(nxt.astype(np.uint32), torch)
    kt = keys_to_dev(keys, flags, torch)
    out = None if inplace else torch.full_like(nt, -1)
    new_heads, status = s.sort_async(ht, ot, nt, kt, K, descending=bool(flags & 1),
                                     signed=bool(flags & 2), next_out=out, shared=shared)
    torch.cuda.synchronize()
    st = int(status.item())
    got = (nt if inplace else out).cpu().numpy().view(np.uint32)
    return st, new_heads.cpu().numpy().view(np.uint32), got


def oracle_lists(oracle_mod, heads, offsets, nxt, keys, K, flags=0):
    M = keys.dtype.itemsize * 8
    f = oracle_flags(flags, oracle_mod)
    st, out, nh = oracle_mod.sort_lists(heads, offsets, nxt, keys, M, K, flags=f)
    assert st == 0
    return nh, out


def check(oracle_mod, heads, offsets, nxt, keys, K, flags=0, inplace=False, shared=False):
    st, nh, got = gpu_sort_lists(heads, offsets, nxt, keys, K, flags, inplace, shared)
    assert st == 0
    enh, enext = oracle_lists(oracle_mod, heads, offsets, nxt, keys, K, flags)
    assert np.array_equal(nh, enh)
    assert np.array_equal(got, enext)


def test_small_mixed_lengths(oracle_mod):
    rng = inputs.rng_for(4101)
    lengths = [0, 1, 2, 3, 15, 16, 17, 0, 31, 100, 1000, 4097, 1, 0, 20000]
    nxt, heads, offs = inputs.slab_lists(lengths, rng)
    keys = rng.integers(0, 50, size=nxt.shape[0]).astype(np.uint32)
    for K in (4, 8):
        say("small mixed K=%d" % K)
        check(oracle_mod, heads, offs, nxt, keys, K)
    check(oracle_mod, heads, offs, nxt, keys, 8, inplace=True)


def test_single_list_batch_equals_plain(oracle_mod):
    rng = inputs.rng_for(4102)
    nxt, heads, offs = inputs.slab_lists([65536], rng)
    keys = inputs.uniform_keys(65536, 32, rng)
    check(oracle_mod, heads, offs, nxt, keys, 8)


def test_many_lists_shape_reduced(oracle_mod):
    """Log-uniform lengths like the 20 000-list batch, scaled down."""
    rng = inputs.rng_for(4001)
    lengths = inputs.log_uniform_lengths(1500, 4, 14, rng, 16, 1 << 14)
    nxt, heads, offs = inputs.slab_lists(lengths, rng)
    keys = inputs.uniform_keys(nxt.shape[0], 32, rng)
    say("many lists, reduced, total=%d" % nxt.shape[0])
    check(oracle_mod, heads, offs, nxt, keys, 8)


@pytest.mark.parametrize("M,K", [(8, 4), (8, 8), (16, 4), (32, 4), (64, 8), (64, 4), (16, 2)])
def test_key_widths(oracle_mod, M, K):
    rng = inputs.rng_for(4200 + M + K)
    lengths = inputs.log_uniform_lengths(200, 0, 12, rng, 0, 1 << 12)
    nxt, heads, offs = inputs.slab_lists(lengths, rng)
    keys = inputs.uniform_keys(nxt.shape[0], M, rng)
    keys[::4] = keys[2]
    say("batched M=%d K=%d" % (M, K))
    check(oracle_mod, heads, offs, nxt, keys, K)
    if M == 32:
        check(oracle_mod, heads, offs, nxt, keys, K, flags=3)
    if M >= 16:
        fkeys = inputs.float_keys(nxt.shape[0], M, rng)
        check(oracle_mod, heads, offs, nxt, fkeys, K, flags=4)
        check(oracle_mod, heads, offs, nxt, fkeys, K, flags=5)


def test_70000_tiny_lists(oracle_mod):
    """More than 2^16 lists of 0 to 3 nodes: all sorted in LDS, many empty."""
    rng = inputs.rng_for(4301)
    lengths = rng.integers(0, 4, size=70000)
    nxt, heads, offs = inputs.slab_lists(lengths, rng)
    keys = rng.integers(0, 7, size=nxt.shape[0]).astype(np.uint16)
    say("many lists total=%d" % nxt.shape[0])
    check(oracle_mod, heads, offs, nxt, keys, 8)


def test_long_chains_in_batch(oracle_mod):
    """Slabs whose level-0 chains exceed their stored slot."""
    from .test_gpu_parity import long_chain_order
    rng = inputs.rng_for(4300)
    lengths = np.array([40000, 17, 0, 25000, 3000, 1], dtype=np.int64)
    offs = np.zeros(len(lengths) + 1, dtype=np.uint64)
    offs[1:] = np.cumsum(lengths)
    nxt = np.full(int(offs[-1]), NIL, dtype=np.uint32)
    heads = np.full(len(lengths), NIL, dtype=np.uint32)
    for l, ln in enumerate(lengths):
        if ln == 0:
            continue
        lo = int(offs[l])
        order = long_chain_order(int(ln), rng, max(1, int(ln) // 250)) + lo
        nxt[order[:-1]] = order[1:]
        heads[l] = order[0]
    keys = inputs.uniform_keys(nxt.shape[0], 32, rng)
    say("batched long chains")
    check(oracle_mod, heads, offs, nxt, keys, 8)


def test_batched_equals_alone():
    """Each list of a batch sorts exactly as the single-list entry point
    sorts it alone."""
    import torch
    from paper_cs_0511020_amd.sorter import ListSorter
    from .gpu_util import gpu_sort
    rng = inputs.rng_for(4401)
    lengths = inputs.log_uniform_lengths(60, 4, 16, rng, 16, 1 << 16)
    nxt, heads, offs = inputs.slab_lists(lengths, rng)
    keys = rng.integers(0, 1 << 20, size=nxt.shape[0]).astype(np.uint32)
    st, nh, got = gpu_sort_lists(heads, offs, nxt, keys, 8)
    assert st == 0
    sorter = ListSorter()
    for l, ln in enumerate(lengths):
        lo = int(offs[l])
        local = np.where(nxt[lo:lo + ln] == NIL, NIL, nxt[lo:lo + ln] - lo).astype(np.uint32)
        h, st1, g1 = gpu_sort(int(heads[l]) - lo, local, keys[lo:lo + ln], 8, sorter=sorter)
        assert st1 == 0 and h + lo == nh[l]
        exp = np.where(g1 == NIL, NIL, g1 + lo).astype(np.uint32)
        assert np.array_equal(got[lo:lo + ln], exp)


def test_batched_rejects_malformed():
    rng = inputs.rng_for(4501)
    lengths = [50, 70, 0, 40]
    nxt, heads, offs = inputs.slab_lists(lengths, rng)
    keys = rng.integers(0, 9, size=nxt.shape[0]).astype(np.uint32)
    # swap two next pointers across slabs: every node keeps one predecessor
    bad = nxt.copy()
    a = int(heads[0]); b = int(heads[1])
    bad[a], bad[b] = nxt[b], nxt[a]
    st, nh, got = gpu_sort_lists(heads, offs, bad, keys, 8)
    assert st == -2 and np.array_equal(got, np.full_like(bad, NIL))
    # a cycle inside one slab
    bad = nxt.copy()
    tail = [i for i in range(50) if nxt[i] == NIL][0]
    bad[tail] = heads[0]
    st, _, _ = gpu_sort_lists(heads, offs, bad, keys, 8, inplace=True)
    assert st == -2
    # bad slab bounds or head
    bad_offs = offs.copy(); bad_offs[2] = bad_offs[3] + 1
    st, _, _ = gpu_sort_lists(heads, bad_offs, nxt, keys, 8)
    assert st == -1
    bad_heads = heads.copy(); bad_heads[2] = 5
    st, _, _ = gpu_sort_lists(bad_heads, offs, nxt, keys, 8)
    assert st == -1


def gpu_sort_lists_gather(heads_local, offsets, nexts, keys_list, K):
    """The gather form: each list in arrays of its own, list-local indices.
    Outputs start as all ones so that untouched entries can be seen."""
    import torch
    from paper_cs_0511020_amd import _lib
    L = len(nexts)
    M = keys_list[0].dtype.itemsize * 8
    nt = [to_dev(x.astype(np.uint32), torch) for x in nexts]
    kt = [to_dev(x, torch) for x in keys_list]
    outs = [torch.full_like(x, -1) for x in nt]
    ptrs = lambda ts: torch.tensor([t.data_ptr() for t in ts], dtype=torch.int64, device="cuda")
    p_in, p_out, p_key = ptrs(nt), ptrs(outs), ptrs(kt)
    ht = to_dev(np.asarray(heads_local, dtype=np.uint32), torch)
    ot = torch.from_numpy(np.asarray(offsets, dtype=np.int64)).to("cuda")
    total = int(sum(int(x.shape[0]) for x in nexts))
    new_heads = torch.full((L,), -1, dtype=torch.int32, device="cuda")
    status = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    wsb = _lib.lists_workspace_bytes(total, L, M, K)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    st = _lib.sort_lists_gather(ht, ot, L, total, p_in, p_out, p_key, M, K, 0, new_heads, status,
                                ws, wsb)
    assert st == 0
    torch.cuda.synchronize()
    return (int(status.item()), new_heads.cpu().numpy().view(np.uint32),
            [o.cpu().numpy().view(np.uint32) for o in outs])


def test_gather_form_and_its_rejections(oracle_mod):
    """Gather-form batch against the oracle; then slab bounds that are not
    monotone, that end below the node count, or a head outside its list:
    status PBIT_EINVAL, no output or head written, nothing read out of
    bounds."""
    rng = inputs.rng_for(4601)
    lengths = [300, 1, 0, 7000, 45]
    nexts, heads, keys_list = [], [], []
    for ln in lengths:
        if ln:
            nx, h, _ = inputs.random_list(ln, rng)
        else:
            nx, h = np.zeros(0, dtype=np.uint32), NIL
        nexts.append(nx)
        heads.append(h)
        keys_list.append(rng.integers(0, 40, size=ln).astype(np.uint32))
    offs = np.zeros(len(lengths) + 1, dtype=np.int64)
    offs[1:] = np.cumsum(lengths)
    st, nh, outs = gpu_sort_lists_gather(heads, offs, nexts, keys_list, 8)
    assert st == 0
    for l, ln in enumerate(lengths):
        if ln == 0:
            assert nh[l] == NIL
            continue
        eh, enext = oracle_mod.sort_list(heads[l], nexts[l], keys_list[l], 32, 8)
        assert nh[l] == eh and np.array_equal(outs[l], enext)

    def rejected(h, o):
        st, nh, outs = gpu_sort_lists_gather(h, o, nexts, keys_list, 8)
        assert st == -1
        assert np.all(nh == NIL)
        assert all(np.all(x == NIL) for x in outs)

    bad = offs.copy(); bad[2] = bad[4] + 3          # list 1 ends after list 3 starts
    rejected(heads, bad)
    bad = offs.copy(); bad[-1] -= 10                # last slab ends below the node count
    rejected(heads, bad)
    bad = offs.copy(); bad[1], bad[2] = bad[2], bad[1]  # decreasing bounds
    rejected(heads, bad)
    bad_heads = list(heads); bad_heads[3] = 7000    # head past its list's end
    rejected(bad_heads, offs)
    bad_heads = list(heads); bad_heads[2] = 0       # head given for an empty list
    rejected(bad_heads, offs)


@pytest.fixture
def cutoff_setter():
    """Set the short-list cutoff of many-list sorts through the tuning table;
    the built-in table is restored afterwards."""
    from paper_cs_0511020_amd import _lib

    def set_cutoff(M, K, cutoff):
        _lib.tune_clear()  # no entry of the built-in table may win over this one
        assert _lib.tune_set(1, M, 0xFFFFFFFF, K, cutoff) == 0
        assert _lib.tune_lookup(1, M, 1000) == (K, cutoff)
    yield set_cutoff
    _lib.tune_reset()


@pytest.mark.parametrize("cutoff", [1024, 2048, 4096])
@pytest.mark.parametrize("M,K", [(32, 8), (8, 4), (64, 8), (16, 4)])
def test_lists_straddling_the_cutoff(oracle_mod, cutoff_setter, cutoff, M, K):
    """Lists one node either side of the cutoff take different paths (LDS
    sort or segment passes); all must equal the oracle, with ties."""
    cutoff_setter(M, K, cutoff)
    rng = inputs.rng_for(4700 + cutoff + M + K)
    lengths = [cutoff - 1, cutoff, cutoff + 1, 1, 0, 2 * cutoff + 7, 16, cutoff + 1, 3,
               cutoff, 9000, 2, cutoff - 1]
    nxt, heads, offs = inputs.slab_lists(lengths, rng)
    keys = inputs.uniform_keys(nxt.shape[0], M, rng)
    keys[::3] = keys[1]
    say("straddle cutoff=%d M=%d K=%d" % (cutoff, M, K))
    check(oracle_mod, heads, offs, nxt, keys, K)
    check(oracle_mod, heads, offs, nxt, keys, K, flags=3 if M != 8 else 1)


def test_tiles_spanning_many_segments(oracle_mod, cutoff_setter):
    """Segments just above the smallest cutoff: a digit-pass tile (6144 or
    8192 positions) spans up to 8 of them, each with its own digit bases."""
    cutoff_setter(32, 8, 1024)
    rng = inputs.rng_for(4801)
    lengths = rng.integers(1025, 1300, size=300)
    lengths[::7] = rng.integers(1, 1024, size=len(lengths[::7]))
    nxt, heads, offs = inputs.slab_lists(lengths, rng)
    keys = inputs.uniform_keys(nxt.shape[0], 32, rng)
    keys[::2] = keys[5]
    say("tiles over many segments, %d nodes" % nxt.shape[0])
    check(oracle_mod, heads, offs, nxt, keys, 8)
    check(oracle_mod, heads, offs, nxt, keys, 4)
    k64 = inputs.uniform_keys(nxt.shape[0], 64, rng)
    cutoff_setter(64, 8, 1024)
    check(oracle_mod, heads, offs, nxt, k64, 8)


def test_batches_of_one_path_only(oracle_mod):
    """Every list short (no segment passes at all) or every list long."""
    rng = inputs.rng_for(4901)
    nxt, heads, offs = inputs.slab_lists(rng.integers(0, 2048, size=500), rng)
    keys = rng.integers(0, 1000, size=nxt.shape[0]).astype(np.uint32)
    check(oracle_mod, heads, offs, nxt, keys, 8)
    nxt, heads, offs = inputs.slab_lists(rng.integers(4097, 30000, size=40), rng)
    keys = rng.integers(0, 1000, size=nxt.shape[0]).astype(np.uint32)
    check(oracle_mod, heads, offs, nxt, keys, 8)
    # constant keys inside every list: every pass is skipped for the segments
    per = np.repeat(np.arange(40, dtype=np.uint32), np.diff(offs.astype(np.int64)))
    check(oracle_mod, heads, offs, nxt, per * np.uint32(7919), 8)


def test_short_list_malformations_leave_outputs(cutoff_setter):
    """A cycle, a link out of the slab, or a second list inside one short
    list's slab: PBIT_EMALFORMED, nothing written."""
    cutoff_setter(32, 8, 2048)
    rng = inputs.rng_for(5001)
    lengths = [100, 1500, 3000, 7]
    nxt, heads, offs = inputs.slab_lists(lengths, rng)
    keys = rng.integers(0, 9, size=nxt.shape[0]).astype(np.uint32)
    lo = int(offs[1])
    order = [int(heads[1])]
    while int(nxt[order[-1]]) != NIL:
        order.append(int(nxt[order[-1]]))
    cases = []
    bad = nxt.copy(); bad[order[-1]] = order[500]                 # cycle
    cases.append(bad)
    bad = nxt.copy(); bad[order[10]] = int(offs[2]) + 3            # into the next slab
    cases.append(bad)
    bad = nxt.copy(); bad[order[700]] = NIL                        # list cut in two
    cases.append(bad)
    bad = nxt.copy(); bad[order[3]] = 0xFFFFFFF0                   # index out of range
    cases.append(bad)
    for bad in cases:
        st, nh, got = gpu_sort_lists(heads, offs, bad, keys, 8)
        assert st == -2
        assert np.array_equal(got, np.full_like(bad, NIL))


def test_shared_flag_batched(oracle_mod):
    """PBIT_SHARED (tiles claimed in block start order) changes no result."""
    rng = inputs.rng_for(4951)
    lengths = inputs.log_uniform_lengths(400, 4, 16, rng, 16, 1 << 16)
    nxt, heads, offs = inputs.slab_lists(lengths, rng)
    keys = inputs.uniform_keys(nxt.shape[0], 32, rng)
    keys[::3] = keys[0]
    check(oracle_mod, heads, offs, nxt, keys, 8, shared=True)
    check(oracle_mod, heads, offs, nxt, inputs.uniform_keys(nxt.shape[0], 64, rng), 4,
          shared=True)
