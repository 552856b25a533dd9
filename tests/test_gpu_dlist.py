"""Doubly-linked lists (Sec. 13): sort, then rebuild the backward links on the
device; prev[] must equal the oracle's repair walk over the oracle's sorted
list, element by element."""
import numpy as np
import pytest

from paper_cs_0511020_amd import inputs

from .gpu_util import NIL, keys_to_dev, oracle_flags, to_dev

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _single(oracle_mod, n, M, K, flags, seed):
    import torch
    from paper_cs_0511020_amd.sorter import ListSorter
    rng = inputs.rng_for(seed)
    nxt, head, _ = inputs.random_list(n, rng)
    keys = inputs.float_keys(n, M, rng) if flags & 4 else inputs.uniform_keys(n, M, rng)
    if n > 4:
        keys[::3] = keys[1]
    nt = to_dev(nxt, torch)
    prev = torch.full_like(nt, 0x5A5A5A5A)
    s = ListSorter()
    h = s.sort(head, nt, keys_to_dev(keys, flags, torch), K, descending=bool(flags & 1),
               signed=bool(flags & 2), prev_out=prev)
    eh, enext = oracle_mod.sort_list(head, nxt, keys, M, K, flags=oracle_flags(flags, oracle_mod))
    eprev = oracle_mod.repair_prev(eh, enext)
    assert h == eh
    assert np.array_equal(nt.cpu().numpy().view(np.uint32), enext)
    assert np.array_equal(prev.cpu().numpy().view(np.uint32), eprev)


@pytest.mark.parametrize("n", [1, 2, 3, 1000, 65537, 300007])
def test_single_list_prev(oracle_mod, n):
    say("dlist n=%d" % n)
    _single(oracle_mod, n, 32, 8, 0, 9100 + n)


def test_single_list_prev_flags(oracle_mod):
    for M, K, flags in [(16, 4, 1), (64, 8, 2), (32, 4, 5), (64, 8, 4)]:
        say("dlist M=%d K=%d flags=%d" % (M, K, flags))
        _single(oracle_mod, 50001, M, K, flags, 9200 + M + flags)


def test_batched_prev(oracle_mod):
    import torch
    from paper_cs_0511020_amd.sorter import ListsSorter
    rng = inputs.rng_for(9300)
    lengths = inputs.log_uniform_lengths(400, 0, 13, rng, 0, 1 << 13)
    nxt, heads, offs = inputs.slab_lists(lengths, rng)
    keys = inputs.uniform_keys(nxt.shape[0], 32, rng)
    nt = to_dev(nxt, torch)
    prev = torch.full_like(nt, 0x5A5A5A5A)
    s = ListsSorter()
    nh = s.sort(to_dev(heads, torch), torch.from_numpy(offs.astype(np.int64)).to("cuda"), nt,
                to_dev(keys, torch), 8, prev_out=prev)
    st, enext, enh = oracle_mod.sort_lists(heads, offs, nxt, keys, 32, 8)
    assert st == 0
    eprev = np.full(nxt.shape[0], NIL, dtype=np.uint32)
    for l in range(len(lengths)):
        if enh[l] != NIL:
            eprev = oracle_mod.repair_prev(int(enh[l]), enext, eprev)
    assert np.array_equal(nh.cpu().numpy().view(np.uint32), enh)
    assert np.array_equal(nt.cpu().numpy().view(np.uint32), enext)
    assert np.array_equal(prev.cpu().numpy().view(np.uint32), eprev)


def test_repair_after_failed_sort_writes_nothing():
    import torch
    from paper_cs_0511020_amd import _lib
    from paper_cs_0511020_amd.sorter import ListSorter, PbitError
    n = 5000
    nxt, head, order = inputs.random_list(n, inputs.rng_for(9400))
    nxt[order[n // 2]] = order[n // 4]          # a cycle: the sort reports it
    nt = to_dev(nxt, torch)
    keys = to_dev(np.arange(n, dtype=np.uint32), torch)
    prev = torch.full_like(nt, 0x5A5A5A5A)
    with pytest.raises(PbitError) as e:
        ListSorter().sort(head, nt, keys, 8, prev_out=prev)
    assert e.value.code == _lib.EMALFORMED
    assert bool((prev == 0x5A5A5A5A).all())
    assert np.array_equal(nt.cpu().numpy().view(np.uint32), nxt)


def test_repair_only_hand_case_and_bad_index():
    import torch
    from paper_cs_0511020_amd import _lib
    # two lists over 6 nodes: 2 -> 0 -> 3 and 5 -> 1 -> 4
    nxt = np.array([3, 4, 0, NIL, NIL, 1], dtype=np.uint32)
    nt = to_dev(nxt, torch)
    heads = to_dev(np.array([2, 5], dtype=np.uint32), torch)
    prev = torch.full_like(nt, 7)
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    assert _lib.repair_prev(heads, 2, nt, prev, 6, status) == _lib.OK
    torch.cuda.synchronize()
    assert prev.cpu().numpy().view(np.uint32).tolist() == [2, 5, NIL, 0, 1, NIL]
    assert int(status.item()) == 0
    bad = to_dev(np.array([3, 4, 0, 99, NIL, 1], dtype=np.uint32), torch)
    assert _lib.repair_prev(heads, 2, bad, prev, 6, status) == _lib.OK
    torch.cuda.synchronize()
    assert int(status.item()) == _lib.EMALFORMED
