"""GPU: the last digit pass reads one packed word per element (its digit over
the node index) that the pass before it wrote, when node indices fit below
the digit.  Which passes run is decided on the device (a pass whose pattern
is one value for every key is skipped), so the packing pass and the last pass
need not be adjacent.  These cases fix the constant patterns and compare
with the oracle bit for bit, and cover list sizes on both sides of the
packing limit (2^(32 - K) nodes)."""
import numpy as np
import pytest

from paper_cs_0511020_amd import inputs

from .gpu_util import gpu_sort, oracle_flags

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def say(*a):
    print(*a, flush=True)


def keys_with_constant_patterns(n, M, K, constant, rng):
    """Uniform M-bit keys whose K-bit patterns listed in `constant` are one
    fixed value in every key (those passes are skipped)."""
    keys = inputs.uniform_keys(n, M, rng).astype(np.uint64)
    for p in constant:
        field = np.uint64(((1 << K) - 1) << (p * K))
        fixed = np.uint64(((0x5A5A5A5A5A5A5A5A >> (p * K)) & ((1 << K) - 1)) << (p * K))
        keys = (keys & ~field) | fixed
    return keys.astype(np.dtype("uint%d" % M))


def check(oracle_mod, head, nxt, keys, K, flags=0):
    M = keys.dtype.itemsize * 8
    h, st, got = gpu_sort(head, nxt, keys, K, flags, inplace=False)
    eh, enext = oracle_mod.sort_list(head, nxt, keys, M, K, flags=oracle_flags(flags, oracle_mod))
    assert st == 0
    assert h == eh
    assert np.array_equal(got, enext)


@pytest.mark.parametrize("mask", range(16))
def test_u32_k8_every_set_of_constant_patterns(oracle_mod, mask):
    constant = [p for p in range(4) if mask >> p & 1]
    n = 3 * 6144 + 17
    rng = inputs.rng_for(12000 + mask)
    nxt, head, _ = inputs.random_list(n, rng)
    keys = keys_with_constant_patterns(n, 32, 8, constant, rng)
    keys[::9] = keys[4]
    for flags in (0, 1):
        say("u32 K=8 constant patterns %s flags=%d" % (constant, flags))
        check(oracle_mod, head, nxt, keys, 8, flags)


@pytest.mark.parametrize("M,K,constant", [
    (32, 4, [0, 2, 4, 6]), (32, 4, [1, 2, 3, 4, 5, 6]), (32, 4, [0, 1, 2, 3, 4, 5, 7]),
    (64, 8, [2, 3, 4, 5, 6, 7]), (64, 8, [0, 7]), (64, 4, list(range(1, 15))),
    (16, 8, []), (16, 8, [1]), (8, 2, [1]), (8, 1, [0, 2, 3, 4, 5, 6]),
])
def test_other_widths_with_constant_patterns(oracle_mod, M, K, constant):
    n = 5 * 6144 + 3
    rng = inputs.rng_for(12100 + M * 7 + K + len(constant))
    nxt, head, _ = inputs.random_list(n, rng)
    keys = keys_with_constant_patterns(n, M, K, constant, rng)
    keys[::11] = keys[2]
    say("M=%d K=%d constant patterns %s" % (M, K, constant))
    check(oracle_mod, head, nxt, keys, K)
    check(oracle_mod, head, nxt, keys, K, flags=1)


@pytest.mark.parametrize("n,K", [((1 << 24) - 1, 8), ((1 << 24) + 1, 8), ((1 << 24) + 1, 4)])
def test_packing_limit(oracle_mod, n, K):
    """Node indices of 2^24 - 1 lists fit below an 8-bit digit; one node more
    and the last pass reads pairs instead (4-bit digits still pack)."""
    rng = inputs.rng_for(12200 + K + (n & 7))
    nxt, head, _ = inputs.random_list(n, rng)
    keys = inputs.uniform_keys(n, 32, rng)
    say("packing limit n=%d K=%d" % (n, K))
    check(oracle_mod, head, nxt, keys, K)
