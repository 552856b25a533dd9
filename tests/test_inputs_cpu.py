"""The seeded input generators against the recipe they implement.

Checked independently of the generator code: list layouts by walking them,
the Zipf frequencies against the truncated harmonic sums p(r) = r^-s / H,
the batch totals against the mean of a log-uniform length, and the float
generator's specials and repeats by classifying the bit patterns."""
import math

import numpy as np
import pytest

from paper_cs_0511020_amd import inputs

NIL = 0xFFFFFFFF


def walk(nxt, head):
    out, cur, n = [], head, len(nxt)
    while cur != NIL and len(out) <= n:
        out.append(cur)
        cur = int(nxt[cur])
    return out


@pytest.mark.parametrize("n", [1, 2, 17, 1000])
def test_random_list_is_one_list_over_all_nodes(n):
    nxt, head, order = inputs.random_list(n, inputs.rng_for(11 + n))
    visited = walk(nxt, head)
    assert visited == [int(x) for x in order]
    assert sorted(visited) == list(range(n))
    assert int((nxt == NIL).sum()) == 1


def test_random_layout_is_unrelated_to_memory_order():
    n = 1 << 16
    nxt, head, _ = inputs.random_list(n, inputs.rng_for(5))
    # in a uniformly random layout, next[i] == i + 1 has probability about 1/n
    assert int((nxt[:-1] == np.arange(1, n, dtype=np.uint32)).sum()) < 8


def test_zipf_frequencies_follow_the_truncated_table():
    n, s, distinct = 1 << 20, 1.1, 1 << 16
    keys = inputs.zipf_keys(n, inputs.rng_for(2002), s=s, distinct=distinct)
    _, counts = np.unique(keys, return_counts=True)
    assert counts.shape[0] <= distinct
    counts = np.sort(counts)[::-1]
    H = math.fsum(r ** -s for r in range(1, distinct + 1))
    p1 = 1.0 / H
    p10 = math.fsum(r ** -s for r in range(1, 11)) / H
    assert abs(p1 - 0.137) < 0.001 and abs(p10 - 0.368) < 0.001  # the plan's figures
    for got, p in ((counts[0] / n, p1), (counts[:10].sum() / n, p10)):
        sigma = math.sqrt(p * (1 - p) / n)
        assert abs(got - p) < 6 * sigma


def test_eight_distinct_values_about_equally_often():
    n = 1 << 18
    keys = inputs.few_distinct_keys(n, inputs.rng_for(2003), 8, 32)
    vals, counts = np.unique(keys, return_counts=True)
    assert vals.shape[0] == 8
    sigma = math.sqrt(n * (1 / 8) * (7 / 8))
    assert np.all(np.abs(counts - n / 8) < 6 * sigma)


@pytest.mark.parametrize("hi,total", [(16, 161_533_792), (20, 1_944_927_695)])
def test_batch_lengths(hi, total):
    lens = inputs.log_uniform_lengths(20000, 4, hi, inputs.rng_for(4001), 16, 1 << hi)
    assert lens.min() >= 16 and lens.max() <= (1 << hi)
    # the realized totals the batched runs report
    assert int(lens.sum()) == total
    # and consistent with the mean of 2^(4 + (hi - 4) u), u uniform:
    # (2^hi - 2^4) / ((hi - 4) ln 2), within a few standard errors
    mean = ((1 << hi) - 16) / ((hi - 4) * math.log(2))
    second = ((1 << (2 * hi)) - 256) / (2 * (hi - 4) * math.log(2))
    sigma = math.sqrt((second - mean * mean) / 20000)
    assert abs(lens.mean() - mean) < 5 * sigma


@pytest.mark.parametrize("M", [16, 32, 64])
def test_float_keys_specials_and_repeats(M):
    n = 1 << 16
    bits = inputs.float_keys(n, M, inputs.rng_for(300 + M), specials=True)
    assert bits.dtype == inputs.KEY_DTYPES[M]
    vals = bits.view(inputs.FLOAT_DTYPES[M])
    assert np.isnan(vals).any() and np.isinf(vals).any()
    assert (np.signbit(vals) & ~np.isnan(vals)).any() and (~np.signbit(vals)).any()
    assert (vals == 0).any()
    # about 25 % of the values repeat an earlier draw: far more repeats than
    # independent draws over the whole exponent range would give
    _, counts = np.unique(bits, return_counts=True)
    assert (counts > 1).sum() > n // 64
    plain = inputs.float_keys(n, M, inputs.rng_for(300 + M), specials=False)
    assert not np.isnan(plain.view(inputs.FLOAT_DTYPES[M])).any()
