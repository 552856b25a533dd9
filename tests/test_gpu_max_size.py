"""Single lists beyond the sizes the oracle can sort in a test, with 8-bit
keys (so many ties): n = 2^30 - 1, the largest list whose digit passes chain
tiles with 32-bit look-back words (2 flag bits and a 30-bit count), and
n = 2^30 + 2^20, which takes the 64-bit words.  The result is checked on the
device by properties that together fix the stable sort:

* every node but one (the head) has exactly one predecessor and exactly one
  node links to NIL;
* along every link the pair (key, position in the input list) strictly
  increases -- positions are unique, so this is a strict order: no cycle can
  exist, the links form one path from the head over all n nodes, and that
  path is the list sorted by key with ties in input order, i.e. the unique
  stable sort;
* the head holds the smallest pair.
"""
import pytest

pytestmark = pytest.mark.gpu



@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("n", [(1 << 30) - 1, (1 << 30) + (1 << 20)])
def test_largest_lists_u8_keys(n):
    import torch
    from paper_cs_0511020_amd.sorter import ListSorter
    print("large list n=%d u8 keys" % n, flush=True)
    dev = torch.device("cuda")
    g = torch.Generator(device=dev)
    g.manual_seed(3030 + n)
    order = torch.randperm(n, generator=g, device=dev, dtype=torch.int64)  # list order
    nxt = torch.full((n,), -1, dtype=torch.int32, device=dev)
    nxt[order[:-1]] = order[1:].to(torch.int32)
    head = int(order[0].item())
    pos = torch.empty(n, dtype=torch.int64, device=dev)  # position in the input list
    pos[order] = torch.arange(n, device=dev)
    del order
    keys = torch.randint(0, 256, (n,), generator=g, device=dev, dtype=torch.uint8)
    s = ListSorter()
    h = s.sort(head, nxt, keys, K=4)  # in place
    s._ws = None
    torch.cuda.empty_cache()
    nil = nxt == -1
    assert int(nil.sum().item()) == 1
    tgt = nxt[~nil].to(torch.int64) & 0xFFFFFFFF
    assert bool((tgt < n).all().item())
    indeg = torch.bincount(tgt, minlength=n)
    assert bool((indeg <= 1).all().item())
    assert int(indeg[h].item()) == 0 and int((indeg == 0).sum().item()) == 1
    src = torch.nonzero(~nil).flatten()
    del indeg, nil
    k64 = keys.to(torch.int64)
    a = k64[src] * (1 << 31) + pos[src]          # (key, position) as one integer
    b = k64[tgt] * (1 << 31) + pos[tgt]
    assert bool((b > a).all().item())
    del a, b, src, tgt
    kp = k64 * (1 << 31) + pos
    assert int(kp[h].item()) == int(kp.min().item())
    print("max size ok", flush=True)
