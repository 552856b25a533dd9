"""GPU: a single list short enough for one workgroup (at most the tuned
cutoff, and at most 4096 nodes) is sorted entirely in LDS by one launch.
Its result must equal the oracle and the device-wide path, bit for bit, and
a malformed short list must be rejected with nothing written."""
import numpy as np
import pytest

from paper_cs_0511020_amd import inputs

from .gpu_util import NIL, gpu_sort, oracle_flags

pytestmark = pytest.mark.gpu

SIZES = [1, 2, 3, 63, 64, 65, 511, 512, 513, 1023, 1024, 1025, 2047, 2048, 2049, 4095, 4096]


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture
def single_cutoff():
    """Set the one-list short-sort cutoff through the tuning table; the
    built-in table is restored afterwards."""
    from paper_cs_0511020_amd import _lib
    _lib.load()

    def set_cutoff(M, K, cutoff):
        _lib.tune_clear()  # no entry of the built-in table may win over this one
        assert _lib.tune_set(0, M, 0xFFFFFFFF, K, cutoff) == 0
        assert _lib.tune_lookup(0, M, 100) == (K, cutoff)
    yield set_cutoff
    _lib.tune_reset()


def oracle_check(oracle_mod, head, nxt, keys, K, flags=0, inplace=True):
    M = keys.dtype.itemsize * 8
    h, st, got = gpu_sort(head, nxt, keys, K, flags, inplace)
    eh, enext = oracle_mod.sort_list(head, nxt, keys, M, K, flags=oracle_flags(flags, oracle_mod))
    assert st == 0
    assert h == eh
    assert np.array_equal(got, enext)


@pytest.mark.parametrize("M,K", [(8, 4), (8, 8), (16, 8), (32, 8), (32, 4), (64, 8), (32, 1)])
def test_short_single_lists_equal_oracle(oracle_mod, single_cutoff, M, K):
    single_cutoff(M, K, 4096)
    for n in SIZES:
        say("short list M=%d K=%d n=%d" % (M, K, n))
        rng = inputs.rng_for(9500 + 7 * n + M + K)
        nxt, head, _ = inputs.random_list(n, rng)
        keys = inputs.uniform_keys(n, M, rng)
        keys[::4] = keys[0]
        oracle_check(oracle_mod, head, nxt, keys, K)
        oracle_check(oracle_mod, head, nxt, keys, K, flags=3 if M != 8 else 1, inplace=False)


@pytest.mark.parametrize("M", [16, 32, 64])
def test_short_float_keys(oracle_mod, single_cutoff, M):
    """IEEE keys with specials, both orders, on the one-workgroup path."""
    single_cutoff(M, 8, 4096)
    rng = inputs.rng_for(9600 + M)
    for n in (5, 700, 4096):
        nxt, head, _ = inputs.random_list(n, rng)
        keys = inputs.float_keys(n, M, rng)
        for flags in (4, 5):
            say("short float M=%d n=%d flags=%d" % (M, n, flags))
            oracle_check(oracle_mod, head, nxt, keys, 8, flags=flags)


@pytest.mark.parametrize("n", [1500, 2048, 4096])
def test_short_and_device_wide_paths_agree(single_cutoff, n):
    """The same list through the LDS path (cutoff 4096) and the device-wide
    path (cutoff 1024) gives identical links and head."""
    rng = inputs.rng_for(9700 + n)
    nxt, head, _ = inputs.random_list(n, rng)
    keys = inputs.uniform_keys(n, 32, rng)
    keys[::3] = keys[2]
    single_cutoff(32, 8, 1024)
    h1, st1, got1 = gpu_sort(head, nxt, keys, 8, inplace=False)
    single_cutoff(32, 8, 4096)
    h2, st2, got2 = gpu_sort(head, nxt, keys, 8, inplace=False)
    assert st1 == 0 and st2 == 0
    assert h1 == h2
    assert np.array_equal(got1, got2)


@pytest.mark.parametrize("inplace", [True, False])
def test_short_malformed_lists_rejected_untouched(single_cutoff, inplace):
    single_cutoff(32, 8, 4096)
    rng = inputs.rng_for(9800)
    n = 3000
    nxt, head, order = inputs.random_list(n, rng)
    keys = inputs.uniform_keys(n, 32, rng)
    cases = {}
    bad = nxt.copy(); bad[order[n // 2]] = order[n // 3]; cases["cycle"] = bad
    bad = nxt.copy(); bad[order[100]] = n + 5; cases["index out of range"] = bad
    bad = nxt.copy(); bad[order[n - 10]] = NIL; cases["short list"] = bad
    bad = nxt.copy(); bad[order[-1]] = order[0]; cases["cycle through head"] = bad
    bad = nxt.copy(); bad[order[n // 2 - 1]] = NIL; bad[order[-1]] = order[n // 2]
    cases["path plus disjoint cycle"] = bad
    bad = nxt.copy(); bad[order[7]] = order[7]; cases["self loop"] = bad
    for name, b in cases.items():
        say("short malformed:", name, "in place" if inplace else "out of place")
        h, st, got = gpu_sort(head, b, keys, 8, inplace=inplace)
        assert st == -2, name
        assert h == NIL
        if inplace:
            assert np.array_equal(got, b), name
        else:
            assert np.all(got == NIL), name  # the output array keeps its fill
