"""The algorithmic byte model behind every roofline figure.

The path totals are pinned to the per-configuration table of the measurement
plan (u32 and u64 keys, K = 8 and K = 4) and to the sum of its per-kernel
terms: the first walk reads next (4 B), the second reads next and key and
writes key and node (8 + 2w), every pass but the last reads and writes
(key, node) (2(w + 4)), the last reads (key, node) and writes the node
(w + 8), and the relink reads the order and writes next (8)."""
import pytest

from paper_cs_0511020_amd import bytemodel


@pytest.mark.parametrize("w,passes,expected", [(4, 4, 88), (4, 8, 152), (8, 8, 220), (8, 16, 412)])
def test_path_bytes_match_the_plan_table(w, passes, expected):
    assert bytemodel.path_bytes_per_node(w, passes) == expected


@pytest.mark.parametrize("w", [1, 2, 4, 8])
@pytest.mark.parametrize("passes", [1, 2, 4, 8, 16, 64])
def test_path_bytes_are_the_sum_of_the_kernel_terms(w, passes):
    terms = [4, 8 + 2 * w] + [2 * (w + 4)] * (passes - 1) + [w + 8, 8]
    assert bytemodel.path_bytes_per_node(w, passes) == sum(terms)


def test_kernel_bytes_per_node():
    # u32 keys: pack reads next + key and writes an 8-byte record; the walk
    # reads a record and writes an entry; unchain reads an entry and writes a
    # (key, node) pair; a pass moves a pair in and a pair out (the last one
    # writes the node only); the relink reads a node and writes a link
    assert bytemodel.kernel_bytes_per_node("pack", 4) == 16
    assert bytemodel.kernel_bytes_per_node("walk0", 4) == 16
    assert bytemodel.kernel_bytes_per_node("unchain", 4) == 16
    assert bytemodel.kernel_bytes_per_node("digit_pass", 4) == 16
    assert bytemodel.kernel_bytes_per_node("digit_pass", 4, last_pass=True) == 12
    assert bytemodel.kernel_bytes_per_node("relink", 4) == 8
    # u64 keys: 16-byte records and entries
    assert bytemodel.kernel_bytes_per_node("pack", 8) == 28
    assert bytemodel.kernel_bytes_per_node("walk0", 8) == 32
    assert bytemodel.kernel_bytes_per_node("digit_pass", 8) == 24
    with pytest.raises(KeyError):
        bytemodel.kernel_bytes_per_node("nonesuch", 4)


def test_packed_digit_passes():
    # the pass before the last writes one 4-byte word per node, which the last
    # pass reads: u32 keys, K = 8, four passes at 2^24 nodes move
    # 16 + 16 + (8 + 4) + (4 + 4) bytes per node
    assert bytemodel.kernel_bytes_per_node("digit_pass", 4, packed_out=True) == 12
    assert bytemodel.kernel_bytes_per_node("digit_pass", 4, last_pass=True, packed_in=True) == 8
    assert bytemodel.digit_pass_bytes_per_node(4, 4, 1 << 24, 8) == (16 + 16 + 12 + 8) / 4
    # one node more and the indices no longer fit below an 8-bit digit
    assert not bytemodel.packs_last_pass((1 << 24) + 1, 8, 4)
    assert bytemodel.digit_pass_bytes_per_node(4, 4, (1 << 24) + 1, 8) == (16 * 3 + 12) / 4
    # 4-bit digits pack up to 2^28 nodes
    assert bytemodel.packs_last_pass(1 << 28, 4, 16)
    # a single executed pass reads pairs and writes indices
    assert bytemodel.digit_pass_bytes_per_node(4, 1, 1000, 8) == 12
    assert bytemodel.digit_pass_bytes_per_node(4, 0, 1000, 8) == 0


def test_u64_passes_over_the_high_half():
    # u64, K = 8, 2^26 nodes: passes 0-2 move 12-byte pairs, pass 3 writes
    # 8-byte (high half, index) pairs, passes 4-6 move those, pass 7 reads
    # them and writes indices
    assert bytemodel.digit_pass_bytes_per_node(8, 8, 1 << 26, 8) == (24 * 3 + 20 + 16 * 3 + 12) / 8
    # at 2^24 nodes the last two passes exchange packed words as well
    assert bytemodel.digit_pass_bytes_per_node(8, 8, 1 << 24, 8) == (24 * 3 + 20 + 16 * 2 + 12 + 8) / 8
