"""The digit pass's look-back fallback, run on purpose.

A tile whose predecessor has not yet published its digit counts waits a
bounded number of sleeps and then counts that predecessor's digits in the
pass input itself.  At test sizes predecessors are nearly always running, so
the parity tests seldom take that branch.  Here the bound is set to zero, so
every tile that finds a predecessor unpublished takes it (with more than 16
tiles some always do: tiles are handed to the chip's dies in chunks of 16, so
tile 16 runs before tile 15).  Every kernel still ends normally; the results
must still equal the oracle's bit for bit."""
import numpy as np
import pytest

from paper_cs_0511020_amd import inputs

from .gpu_util import gpu_sort

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _fallback_only():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_cs_0511020_amd import _lib
    old = _lib.set_lookback_spin_limit(0)
    yield
    _lib.set_lookback_spin_limit(old)


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("M,K,tile", [(32, 8, 6144), (32, 4, 6144), (64, 8, 8192),
                                      (16, 2, 6144)])
def test_single_list_fallback(oracle_mod, M, K, tile):
    for n in (tile + 1, 3 * tile + 5, 20 * tile - 1, 33 * tile + 17):
        say("look-back fallback M=%d K=%d n=%d" % (M, K, n))
        rng = inputs.rng_for(9700 + n + M + K)
        nxt, head, _ = inputs.random_list(n, rng)
        keys = inputs.uniform_keys(n, M, rng)
        keys[::5] = keys[1]
        h, st, got = gpu_sort(head, nxt, keys, K)
        eh, enext = oracle_mod.sort_list(head, nxt, keys, M, K)
        assert st == 0 and h == eh
        assert np.array_equal(got, enext)


def test_batched_fallback_with_list_id_passes(oracle_mod):
    from .test_gpu_batched import check
    rng = inputs.rng_for(9801)
    lengths = inputs.log_uniform_lengths(3000, 0, 12, rng, 0, 1 << 12)
    nxt, heads, offs = inputs.slab_lists(lengths, rng)
    say("batched look-back fallback, %d lists, %d nodes" % (len(lengths), nxt.shape[0]))
    keys = inputs.uniform_keys(nxt.shape[0], 32, rng)
    keys[::3] = keys[0]
    check(oracle_mod, heads, offs, nxt, keys, 8)
    keys64 = inputs.uniform_keys(nxt.shape[0], 64, rng)
    check(oracle_mod, heads, offs, nxt, keys64, 4)
