"""The tuner's table logic (no GPU): choices become table entries that
cover size ranges, the rendered header parses back, and the committed
built-in table holds only entries the library accepts."""
import os

from paper_cs_0511020_amd import _lib, tune

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_entries_cover_sizes_and_merge_equal_neighbours():
    best = [(1 << 12, 4, 2048), (1 << 16, 8, 2048), (1 << 20, 8, 2048), (1 << 24, 4, 1024)]
    e = tune.entries_from_best(1, 32, best)
    assert [x["K"] for x in e] == [4, 8, 4]
    assert e[0]["n_max"] == 1 << 14          # midpoint of 2^12 and 2^16
    assert e[1]["n_max"] == 1 << 22          # merged 2^16 and 2^20 up to their next midpoint
    assert e[2]["n_max"] == tune.NMAX and e[2]["cutoff"] == 1024
    assert all(x["kind"] == 1 and x["M"] == 32 for x in e)


def test_header_round_trip():
    e = tune.entries_from_best(0, 8, [(4096, 2, 2048), (1 << 20, 8, 2048)])
    assert tune.parse_header(tune.render_header(e)) == e


def test_committed_table_is_valid_and_applied():
    with open(os.path.join(ROOT, "paper_cs_0511020_amd", "csrc", "pbit_tuning.h")) as f:
        entries = tune.parse_header(f.read())
    assert entries
    for kind in (0, 1):
        for M in (8, 16, 32, 64):
            mine = [x for x in entries if x["kind"] == kind and x["M"] == M]
            assert mine and max(x["n_max"] for x in mine) == tune.NMAX
    _lib.tune_reset()
    for x in entries:
        assert x["K"] in (1, 2, 4, 8) and x["M"] % x["K"] == 0
        assert x["cutoff"] in (1024, 2048, 4096)
        # the library answers with the entry that covers its own n_max
        assert _lib.tune_lookup(x["kind"], x["M"], x["n_max"]) == (x["K"], x["cutoff"])


def test_single_list_ties_prefer_the_larger_cutoff():
    # at 2048 nodes cutoffs 2048 and 4096 both take the one-workgroup path:
    # only noise separates them, and the larger one must win
    t = {(8, 1024): 0.064, (8, 2048): 0.0270, (8, 4096): 0.0272, (4, 4096): 0.0326}
    assert tune.pick_single(t) == (8, 4096)
    # a real difference is kept
    t = {(8, 1024): 0.020, (8, 4096): 0.030}
    assert tune.pick_single(t) == (8, 1024)


def test_table_rebuilt_from_saved_timings(tmp_path):
    """The committed table is what the committed timings give."""
    with open(os.path.join(ROOT, "paper_cs_0511020_amd", "csrc", "pbit_tuning.h")) as f:
        committed = tune.parse_header(f.read())
    entries = tune.write_from_record(os.path.join(ROOT, "paper_cs_0511020_amd", "tuning.json"),
                                     str(tmp_path))
    assert entries == committed
    # every single-list entry sends lists of up to 4096 nodes to one workgroup
    assert all(e["cutoff"] == 4096 for e in entries if e["kind"] == 0)
