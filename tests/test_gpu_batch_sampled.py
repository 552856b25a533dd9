"""The batched form at the two 20 000-list shapes: lengths log-uniform in
[16, 2^16] (about 1.6e8 nodes, the shape the benchmark times by default) and
in [16, 2^20] (about 1.9e9 nodes, the stated count and range), uint32 keys,
K = 8, one launch sequence.  A sample of lists (the longest, the shortest and
random ones) is compared element by element with the oracle sorting each list
alone; every list is checked on the device for the structure of a relinked
slab (one NIL per non-empty list, every other node with exactly one
predecessor, all links inside the slab, non-decreasing keys along every
link)."""
import numpy as np
import pytest

from paper_cs_0511020_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _local(x, lo):
    x = x.astype(np.int64)
    return np.where(x == 0xFFFFFFFF, 0xFFFFFFFF, x - lo).astype(np.uint32)


@pytest.mark.parametrize("hi_log2", [16, 20])
def test_20000_lists_sampled(oracle_mod, hi_log2):
    import torch
    from paper_cs_0511020_amd.sorter import ListsSorter
    rng = inputs.rng_for(4001)
    lengths = inputs.log_uniform_lengths(20000, 4, hi_log2, rng, 16, 1 << hi_log2)
    print("20000 lists up to 2^%d: %d nodes" % (hi_log2, int(lengths.sum())), flush=True)
    d = inputs.slab_lists_device(lengths, seed=4001, M=32)
    nxt0 = d["next"].clone()
    offs = d["offsets_host"]
    total = int(offs[-1])
    sorter = ListsSorter()
    new_heads = sorter.sort(d["heads"], d["offsets"], d["next"], d["keys"], K=8)
    torch.cuda.synchronize()
    sorter._ws = None
    print("sorted; checking every slab on the device", flush=True)
    out = d["next"]
    # structure of every slab, on the device
    nil = out == -1
    assert int(nil.sum().item()) == len(lengths)
    tgt = out[~nil].to(torch.int64) & 0xFFFFFFFF
    src = torch.nonzero(~nil).flatten()
    del nil
    lens_t = torch.from_numpy(lengths).to("cuda")
    slab_of = torch.repeat_interleave(torch.arange(len(lengths), device="cuda"), lens_t)
    assert bool((slab_of[tgt] == slab_of[src]).all().item())
    del slab_of
    indeg = torch.bincount(tgt, minlength=total)
    assert bool((indeg <= 1).all().item())
    assert int((indeg == 0).sum().item()) == len(lengths)
    del indeg
    k = d["keys"].to(torch.int64) & 0xFFFFFFFF
    assert bool((k[tgt] >= k[src]).all().item())
    del tgt, src, k
    # sampled lists against the oracle
    sample = {int(np.argmax(lengths)), int(np.argmin(lengths))}
    sample |= set(int(x) for x in inputs.rng_for(4002).choice(len(lengths), 38, replace=False))
    nh = new_heads.cpu().numpy().view(np.uint32)
    heads = d["heads_host"]
    for l in sorted(sample):
        lo, hi = int(offs[l]), int(offs[l + 1])
        nx = _local(nxt0[lo:hi].cpu().numpy().view(np.uint32), lo)
        keys = d["keys"][lo:hi].cpu().numpy().view(np.uint32)
        eh, en = oracle_mod.sort_list(int(heads[l]) - lo, nx, keys, 32, 8)
        got = _local(out[lo:hi].cpu().numpy().view(np.uint32), lo)
        assert int(nh[l]) - lo == eh, l
        assert np.array_equal(got, en), l
    print("sampled %d lists ok (longest %d nodes)" % (len(sample), int(lengths.max())),
          flush=True)
