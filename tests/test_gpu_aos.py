"""Nodes stored as records (the paper's node structure: link and data side by
side).  The sort must rewrite exactly the link field of every record, to the
oracle's result on the records' (next, key) projection, and leave every other
byte alone."""
import numpy as np
import pytest

from paper_cs_0511020_amd import inputs

from .gpu_util import NIL

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def field(rec, n, stride, off, dtype):
    return np.ndarray(shape=(n,), dtype=dtype, buffer=rec, offset=off, strides=(stride,))


def make_records(n, stride, next_off, key_off, keys, rng, nxt):
    rec = rng.integers(0, 256, size=n * stride, dtype=np.uint8)  # payload / padding bytes
    field(rec, n, stride, next_off, np.uint32)[:] = nxt
    field(rec, n, stride, key_off, keys.dtype)[:] = keys
    return rec


def run_case(oracle_mod, n, stride, next_off, key_off, keys, K, flags=0, seed=0, layout=None):
    import torch
    from paper_cs_0511020_amd.sorter import ListSorter
    rng = inputs.rng_for(seed)
    if layout is None:
        nxt, head, _ = inputs.random_list(n, rng)
    else:
        nxt, head = layout
    rec = make_records(n, stride, next_off, key_off, keys, rng, nxt)
    M = keys.dtype.itemsize * 8
    dev = torch.from_numpy(rec.copy()).to("cuda")
    h = ListSorter().sort_aos(head, dev, n, stride, next_off, key_off, M, K,
                              descending=bool(flags & 1), signed=bool(flags & 2),
                              floating=bool(flags & 4))
    of = ((oracle_mod.FLAG_DESCENDING if flags & 1 else 0) | (oracle_mod.FLAG_SIGNED if flags & 2 else 0)
          | (oracle_mod.FLAG_FLOAT if flags & 4 else 0))
    eh, enext = oracle_mod.sort_list(head, nxt, keys, M, K, flags=of)
    got = dev.cpu().numpy()
    assert h == eh
    assert np.array_equal(field(got, n, stride, next_off, np.uint32), enext)
    # every byte outside the link fields is unchanged
    mask = np.ones(n * stride, dtype=bool)
    for b in range(4):
        mask[next_off + b::stride] = False
    assert np.array_equal(got[mask], rec[mask])


def test_paper_node_struct(oracle_mod):
    """{next, key} records of 8 bytes, u32 keys."""
    rng = inputs.rng_for(9500)
    for n in (1, 2, 1000, 100003):
        say("aos {next,key} n=%d" % n)
        keys = inputs.uniform_keys(n, 32, rng)
        if n > 10:
            keys[::3] = keys[1]
        run_case(oracle_mod, n, 8, 0, 4, keys, 8, seed=n)


@pytest.mark.parametrize("stride,next_off,key_off,M,K,flags", [
    (24, 0, 8, 64, 4, 0),      # {next, pad, u64 key, u64 payload}
    (16, 12, 8, 16, 4, 1),     # {u64 payload, u16 key, pad, next}, descending
    (8, 4, 0, 8, 4, 0),        # {u8 key, pad, next}
    (12, 8, 0, 32, 8, 4),      # {f32 key, payload, next}, floating point
    (32, 28, 16, 64, 8, 2),    # payload, i64 key, more payload, next; signed
])
def test_record_layouts(oracle_mod, stride, next_off, key_off, M, K, flags):
    rng = inputs.rng_for(9600 + stride + M)
    n = 70001
    say("aos stride=%d next@%d key@%d M=%d flags=%d" % (stride, next_off, key_off, M, flags))
    if flags & 4:
        keys = inputs.float_keys(n, M, rng)
    else:
        keys = inputs.uniform_keys(n, M, rng)
        keys[::5] = keys[2]
    run_case(oracle_mod, n, stride, next_off, key_off, keys, K, flags, seed=stride)


def test_aos_long_chains(oracle_mod):
    from .test_gpu_parity import long_chain_order
    rng = inputs.rng_for(9700)
    n = 300000
    order = long_chain_order(n, rng, 600)
    nxt, head = inputs.links_from_order(order)
    keys = inputs.uniform_keys(n, 32, rng)
    say("aos long chains")
    run_case(oracle_mod, n, 16, 0, 8, keys, 8, seed=5, layout=(nxt, head))


def test_aos_malformed_untouched():
    import torch
    from paper_cs_0511020_amd import _lib
    from paper_cs_0511020_amd.sorter import ListSorter, PbitError
    rng = inputs.rng_for(9800)
    n = 20000
    nxt, head, order = inputs.random_list(n, rng)
    nxt[order[n // 2]] = order[n // 5]
    keys = inputs.uniform_keys(n, 32, rng)
    rec = make_records(n, 16, 4, 8, keys, rng, nxt)
    dev = torch.from_numpy(rec.copy()).to("cuda")
    with pytest.raises(PbitError) as e:
        ListSorter().sort_aos(head, dev, n, 16, 4, 8, 32, 8)
    assert e.value.code == _lib.EMALFORMED
    assert np.array_equal(dev.cpu().numpy(), rec)


def test_aos_empty():
    import torch
    from paper_cs_0511020_amd.sorter import ListSorter
    dev = torch.zeros(16, dtype=torch.uint8, device="cuda")
    assert ListSorter().sort_aos(NIL, dev, 0, 8, 0, 4, 32, 8) == NIL
