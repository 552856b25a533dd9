"""GPU: lists of 2^18 .. 2^25 nodes relink through node ranges held in LDS
(pairs grouped by node range per tile, then one workgroup per range writes
its links in node order).  The result must equal the oracle at sizes on both
sides of the thresholds and range widths, when no pass runs (the order is
read from the pairs buffer), for records, and a malformed list must be
rejected with nothing written."""
import numpy as np
import pytest

from paper_cs_0511020_amd import inputs

from .gpu_util import NIL, gpu_sort, oracle_flags

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def check(oracle_mod, head, nxt, keys, K, flags=0, inplace=True):
    M = keys.dtype.itemsize * 8
    h, st, got = gpu_sort(head, nxt, keys, K, flags, inplace)
    eh, enext = oracle_mod.sort_list(head, nxt, keys, M, K, flags=oracle_flags(flags, oracle_mod))
    assert st == 0
    assert h == eh
    assert np.array_equal(got, enext)


# below the range path, its smallest size, ragged sizes with 2^14-node
# ranges, the largest size with 2^14-node ranges, 2^15-node ranges, and the
# largest range-path size
@pytest.mark.parametrize("n", [(1 << 18) - 1, 1 << 18, (1 << 18) + 1, 3 * (1 << 20) + 7,
                               1 << 24, (1 << 24) + 1, (1 << 25) - 3, 1 << 25])
def test_range_relink_sizes(oracle_mod, n):
    say("range relink n=%d" % n)
    rng = inputs.rng_for(9900 + n % 1000)
    nxt, head, _ = inputs.random_list(n, rng)
    keys = inputs.uniform_keys(n, 32, rng)
    keys[::11] = keys[5]
    check(oracle_mod, head, nxt, keys, 8, inplace=(n % 2 == 0))


def test_range_relink_u64_and_descending(oracle_mod):
    rng = inputs.rng_for(9910)
    n = (1 << 19) + 13
    nxt, head, _ = inputs.random_list(n, rng)
    keys = inputs.uniform_keys(n, 64, rng)
    keys[::7] = keys[3]
    say("range relink u64 n=%d" % n)
    check(oracle_mod, head, nxt, keys, 8)
    check(oracle_mod, head, nxt, keys, 4, flags=3, inplace=False)


def test_range_relink_when_no_pass_runs():
    """All keys equal: every pass is skipped and the order is read from the
    pairs buffer the range relink must not overwrite; the list comes back
    unchanged."""
    rng = inputs.rng_for(9920)
    n = 1 << 20
    nxt, head, _ = inputs.random_list(n, rng)
    keys = np.full(n, 777, dtype=np.uint32)
    say("range relink, no pass, n=%d" % n)
    h, st, got = gpu_sort(head, nxt, keys, 8, inplace=False)
    assert st == 0 and h == head
    assert np.array_equal(got, nxt)


@pytest.mark.parametrize("inplace", [True, False])
def test_range_relink_malformed_untouched(inplace):
    rng = inputs.rng_for(9930)
    n = 1 << 19
    nxt, head, order = inputs.random_list(n, rng)
    keys = inputs.uniform_keys(n, 32, rng)
    cases = {}
    bad = nxt.copy(); bad[order[n // 2]] = order[n // 3]; cases["cycle"] = bad
    bad = nxt.copy(); bad[order[n - 10]] = NIL; cases["short list"] = bad
    bad = nxt.copy(); bad[order[n // 2 - 1]] = NIL; bad[order[-1]] = order[n // 2]
    cases["path plus disjoint cycle"] = bad
    for name, b in cases.items():
        say("range relink malformed:", name)
        h, st, got = gpu_sort(head, b, keys, 8, inplace=inplace)
        assert st == -2, name
        assert h == NIL
        if inplace:
            assert np.array_equal(got, b), name
        else:
            assert np.all(got == NIL), name


def test_range_relink_records(oracle_mod):
    """Records of 16 bytes: the range relink writes the link field of each
    record at the record stride and leaves the other bytes alone."""
    from .test_gpu_aos import run_case
    rng = inputs.rng_for(9940)
    n = (1 << 19) + 5
    keys = inputs.uniform_keys(n, 32, rng)
    say("range relink records n=%d" % n)
    run_case(oracle_mod, n, 16, 0, 4, keys, 8, seed=9941)
