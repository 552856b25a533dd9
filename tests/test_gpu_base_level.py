"""GPU: the last ranking level, ranked by one workgroup in LDS by pointer
jumping (at most 8192 elements).  Cases: list sizes whose last level holds
exactly the most elements or one more (then one more level is built), and
malformed lists that only the last level's length check catches."""
import numpy as np
import pytest

from paper_cs_0511020_amd import inputs

from .gpu_util import NIL, gpu_sort

pytestmark = pytest.mark.gpu

BASE_MAX = 8192


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def say(*a):
    print(*a, flush=True)


def level_sizes(n):
    """Elements per ranking level: 1 + ceil(n / 16) chains at level 1, then
    1 + ceil(m / 4) per level until at most BASE_MAX remain."""
    m = 1 + -(-n // 16)
    sizes = [m]
    while m > BASE_MAX:
        m = 1 + -(-m // 4)
        sizes.append(m)
    return sizes


def largest_n_with_last_level(levels):
    """The largest n whose ranking has `levels` levels and a full last one."""
    lo, hi = 1, 1 << 32
    while hi - lo > 1:  # level count and last size grow with n
        mid = (lo + hi) // 2
        s = level_sizes(mid)
        if len(s) < levels or (len(s) == levels and s[-1] <= BASE_MAX):
            lo = mid
        else:
            hi = mid
    return lo


LIMITS = [largest_n_with_last_level(1), largest_n_with_last_level(2)]


def parity(oracle_mod, head, nxt, keys, K=8):
    M = keys.dtype.itemsize * 8
    h, st, got = gpu_sort(head, nxt, keys, K, inplace=False)
    eh, enext = oracle_mod.sort_list(head, nxt, keys, M, K)
    assert st == 0
    assert h == eh
    assert np.array_equal(got, enext)


def test_level_sizes_of_the_cases():
    assert LIMITS == [16 * (BASE_MAX - 1), 16 * (4 * (BASE_MAX - 1) - 1)]
    assert level_sizes(LIMITS[0]) == [BASE_MAX]
    assert level_sizes(LIMITS[0] + 1) == [BASE_MAX + 1, 2050]
    assert level_sizes(LIMITS[1]) == [4 * (BASE_MAX - 1), BASE_MAX]
    assert level_sizes(LIMITS[1] + 1)[-1] == 2050
    assert level_sizes(1 << 24) == [1048577, 262146, 65538, 16386, 4098]


@pytest.mark.parametrize("n", [LIMITS[0], LIMITS[0] + 1, LIMITS[1], LIMITS[1] + 1])
def test_last_level_at_its_limit(oracle_mod, n):
    say("last level limit n=%d levels=%s" % (n, level_sizes(n)))
    rng = inputs.rng_for(13000 + n % 1000)
    nxt, head, _ = inputs.random_list(n, rng)
    keys = inputs.uniform_keys(n, 32, rng)
    keys[::6] = keys[1]
    parity(oracle_mod, head, nxt, keys)


@pytest.mark.parametrize("n", [LIMITS[0], 300000])
def test_malformed_caught_at_the_last_level(n):
    """Every node keeps at most one predecessor and exactly one link is NIL,
    so the pack-time checks pass; the ranking finds a path from the head that
    weighs fewer than n nodes and rejects the list with nothing written."""
    rng = inputs.rng_for(13200 + n % 997)
    nxt, head, order = inputs.random_list(n, rng)
    keys = inputs.uniform_keys(n, 32, rng)
    cases = {}
    bad = nxt.copy(); bad[order[n // 2 - 1]] = NIL; bad[order[-1]] = order[n // 2]
    cases["path plus disjoint cycle"] = bad
    bad = nxt.copy(); bad[order[100]] = NIL; bad[order[-1]] = order[101]
    cases["short path plus long cycle"] = bad
    bad = nxt.copy(); bad[order[n - 3]] = NIL; bad[order[-1]] = order[n - 2]
    cases["long path plus two-node cycle"] = bad
    for name, b in cases.items():
        say("malformed n=%d: %s" % (n, name))
        for inplace in (True, False):
            h, st, got = gpu_sort(head, b, keys, 8, inplace=inplace)
            assert st == -2, name
            assert h == NIL
            if inplace:
                assert np.array_equal(got, b), name
            else:
                assert np.all(got == NIL), name
