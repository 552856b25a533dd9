"""GPU: one list of 64-bit keys.  Once the patterns of the low 32 key bits are
done, the passes over the high 32 bits run as 32-bit-key passes over
(high half, node) pairs, which the last running pass over the low half
writes.  Which passes run is decided on the device (constant patterns are
skipped), so these cases fix the constant patterns: no pass over the low
half (the first high pass then reads the full pairs), none over the high
half, one on each side, the boundary passes alone; below 2^24 nodes the
last two passes also exchange packed words, above it they do not.  Every
result is compared with the oracle bit for bit."""
import numpy as np
import pytest

from paper_cs_0511020_amd import inputs

from .gpu_util import gpu_sort, oracle_flags
from .test_gpu_packed_pass import keys_with_constant_patterns

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def say(*a):
    print(*a, flush=True)


def check(oracle_mod, head, nxt, keys, K, flags=0):
    h, st, got = gpu_sort(head, nxt, keys, K, flags, inplace=False)
    eh, enext = oracle_mod.sort_list(head, nxt, keys, 64, K, flags=oracle_flags(flags, oracle_mod))
    assert st == 0
    assert h == eh
    assert np.array_equal(got, enext)


def running(K, constant):
    return [p for p in range(64 // K) if p not in constant]


# K = 8: passes 0-3 cover the low half, 4-7 the high half
CASES_K8 = [
    [0, 1, 2, 3],              # high half only: the first high pass reads the full pairs
    [4, 5, 6, 7],              # low half only
    [0, 1, 2, 5, 6, 7],        # passes 3 and 4: the boundary
    [1, 2, 3, 4, 5, 6],        # passes 0 and 7
    [0, 1, 2, 3, 4, 5, 6],     # pass 7 alone, reading the full pairs
    [1, 2, 4, 5, 6],           # passes 0, 3 and 7
    [2, 6],
    [],
]


@pytest.mark.parametrize("constant", CASES_K8)
def test_u64_k8_constant_patterns(oracle_mod, constant):
    n = 3 * 8192 + 5
    rng = inputs.rng_for(14000 + sum(1 << p for p in constant))
    nxt, head, _ = inputs.random_list(n, rng)
    keys = keys_with_constant_patterns(n, 64, 8, constant, rng)
    keys[::7] = keys[3]
    for flags in (0, 1, 2):
        say("u64 K=8 running %s flags=%d" % (running(8, constant), flags))
        check(oracle_mod, head, nxt, keys, 8, flags)


@pytest.mark.parametrize("constant", [list(range(8)), list(range(8, 16)),
                                      [p for p in range(16) if p not in (7, 8)],
                                      [p for p in range(16) if p not in (0, 15)],
                                      list(range(1, 15, 2))])
def test_u64_k4_constant_patterns(oracle_mod, constant):
    n = 2 * 8192 + 6144 + 1
    rng = inputs.rng_for(14100 + len(constant) + constant[0])
    nxt, head, _ = inputs.random_list(n, rng)
    keys = keys_with_constant_patterns(n, 64, 4, constant, rng)
    say("u64 K=4 running %s" % running(4, constant))
    check(oracle_mod, head, nxt, keys, 4)
    check(oracle_mod, head, nxt, keys, 4, flags=1)


def test_u64_float_and_signed_keys(oracle_mod):
    n = 40000
    rng = inputs.rng_for(14200)
    nxt, head, _ = inputs.random_list(n, rng)
    fkeys = inputs.float_keys(n, 64, rng)
    for flags in (4, 5):
        say("u64 float flags=%d" % flags)
        h, st, got = gpu_sort(head, nxt, fkeys, 8, flags, inplace=False)
        eh, enext = oracle_mod.sort_list(head, nxt, fkeys, 64, 8,
                                         flags=oracle_flags(flags, oracle_mod))
        assert st == 0 and h == eh and np.array_equal(got, enext)
    skeys = inputs.uniform_keys(n, 64, rng)
    say("u64 signed")
    check(oracle_mod, head, nxt, skeys, 8, flags=2)


@pytest.mark.parametrize("constant", [[1, 2, 3, 4, 5, 6], [0, 1, 2, 3, 5, 6]])
def test_u64_above_the_packing_limit(oracle_mod, constant):
    """2^24 + 5 nodes: node indices no longer fit below an 8-bit digit, so
    the last high pass reads the (high half, node) pairs themselves."""
    n = (1 << 24) + 5
    rng = inputs.rng_for(14300 + constant[0])
    nxt, head, _ = inputs.random_list(n, rng)
    keys = keys_with_constant_patterns(n, 64, 8, constant, rng)
    say("u64 K=8 n=2^24+5 running %s" % running(8, constant))
    check(oracle_mod, head, nxt, keys, 8)
