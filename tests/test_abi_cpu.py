"""The C-ABI library loads and exports every declared symbol; host-side
argument checks reject bad calls before any device work (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_cs_0511020_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_cs_0511020_amd import build
        build.build()
    return _lib.load()


def declared_functions():
    names = []
    for h in os.listdir(os.path.join(ROOT, "include")):
        if not h.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"\b(pbit_[a-z_0-9]+)\s*\(", text)
    return sorted(set(names))


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert "pbit_sort_list_async" in names and "pbit_sort_list" in names
    for name in names:
        assert hasattr(lib, name), name
        assert name in _lib._SIGNATURES, "binding misses " + name


def test_version_and_status_strings(lib):
    assert "gfx950" in _lib.version()
    for code in (0, -1, -2, -3, -4):
        assert _lib.status_string(code) != "unknown status"


def test_workspace_bytes_shapes(lib):
    assert _lib.workspace_bytes(1 << 16, 32, 4) > (1 << 16) * 16
    assert _lib.workspace_bytes(1 << 16, 32, 0) > 0
    for M, K in [(8, 1), (8, 2), (8, 4), (8, 8), (16, 8), (64, 4), (64, 8)]:
        assert _lib.workspace_bytes(1000, M, K) > 0
    # rejected shapes
    assert _lib.workspace_bytes(1000, 12, 4) == 0
    assert _lib.workspace_bytes(1000, 32, 3) == 0
    assert _lib.workspace_bytes(1000, 32, 16) == 0
    assert _lib.workspace_bytes(1000, 8, 16) == 0
    assert _lib.workspace_bytes((1 << 32) - 1, 32, 4) == 0
    # from 2^30 nodes on the look-back words are 8 bytes: the look-back array
    # grows by (passes x tiles x radix x 4) bytes at that step
    below, above = _lib.workspace_bytes((1 << 30) - 1, 8, 4), _lib.workspace_bytes(1 << 30, 8, 4)
    assert above - below >= 2 * ((1 << 30) // 6144) * 16 * 4
    assert _lib.workspace_bytes((1 << 32) - 2, 8, 8) > 0
    # the workspace grows linearly with n
    a, b = _lib.workspace_bytes(1 << 20, 32, 8), _lib.workspace_bytes(1 << 21, 32, 8)
    assert 1.8 < b / a < 2.2


def test_workspace_sizes_match_the_header(lib):
    # include/pbit.h: about 94 bytes per node for 32-bit keys up to 2^26
    # nodes, about 62 beyond, about 174 for 64-bit keys
    per = lambda n, M, K: _lib.workspace_bytes(n, M, K) / n  # noqa: E731
    assert 90 < per(1 << 24, 32, 8) < 98
    assert 90 < per(1 << 26, 32, 8) < 98
    assert 58 < per(1 << 28, 32, 8) < 66
    assert 168 < per(1 << 26, 64, 8) < 180
    # the batched form: about 63 bytes per node at the 20 000-list batch
    assert 58 < _lib.lists_workspace_bytes(1_944_927_695, 20000, 32, 8) / 1_944_927_695 < 68


def _call(lib, head=0, nxt=0x1000, nout=0x1000, keys=0x1000, n=8, M=32, K=4, flags=0,
          res=0x2000, ws=0x100000, ws_bytes=1 << 40):
    return lib.pbit_sort_list_async(head, nxt, nout, keys, n, M, K, flags, res, ws, ws_bytes,
                                    None)


def test_host_argument_checks(lib):
    E = _lib.EINVAL
    assert _call(lib, M=12) == E
    assert _call(lib, K=3) == E
    assert _call(lib, M=8, K=16) == E
    assert _call(lib, flags=16) == E         # unknown flag bit
    assert _call(lib, flags=_lib.SIGNED | _lib.FLOAT) == E
    assert _call(lib, res=0) == E
    assert _call(lib, res=0x2002) == E            # misaligned result
    assert _call(lib, head=8, n=8) == E           # head out of range
    assert _call(lib, head=_lib.NIL, n=8) == E    # empty head with nodes
    assert _call(lib, nxt=0) == E
    assert _call(lib, keys=0) == E
    assert _call(lib, ws=0) == E
    assert _call(lib, keys=0x1002, M=32) == E     # misaligned keys
    assert _call(lib, ws=0x100010) == E           # misaligned workspace
    assert _call(lib, n=(1 << 32) - 1) == E
    assert _call(lib, ws_bytes=16) == _lib.ENOMEM
    # the synchronous form checks the same way before touching a device
    assert lib.pbit_sort_list(0, 0x1000, 0x1000, 8, 12, 4) == E
    assert lib.pbit_sort_list(9, 0x1000, 0x1000, 8, 32, 4) == E
    assert lib.pbit_sort_list(0, 0, 0x1000, 8, 32, 4) == E
    assert lib.pbit_sort_list(_lib.NIL, 0, 0, 0, 32, 4) == _lib.NIL


def test_aos_host_checks(lib):
    E = _lib.EINVAL
    f = lib.pbit_sort_list_aos_async

    def call(head=0, nodes=0x10000, stride=8, next_off=0, key_off=4, n=8, M=32, K=8, flags=0,
             res=0x2000, ws=0x100000, wsb=1 << 40):
        return f(head, nodes, stride, next_off, key_off, n, M, K, flags, res, ws, wsb, None)
    assert call(stride=2) == E                   # too short for a link
    assert call(stride=10) == E                  # not a multiple of 4
    assert call(key_off=2) == E                  # key overlaps the link
    assert call(next_off=6, stride=12) == E      # misaligned link
    assert call(key_off=6, M=32, stride=12) == E  # misaligned key
    assert call(key_off=8) == E                  # key past the record
    assert call(M=64, key_off=4, stride=16) == E  # 8-byte key not 8-aligned
    assert call(stride=1 << 32) == E
    assert call(nodes=0) == E
    assert call(head=8) == E
    assert call(K=3) == E
    assert call(wsb=16) == _lib.ENOMEM


def test_repair_prev_host_checks(lib):
    E = _lib.EINVAL
    f = lib.pbit_repair_prev_async
    assert f(0x1000, 1, 0x2000, 0x3000, 1 << 32, 0, None) == E      # n too large
    assert f(0, 1, 0x2000, 0x3000, 8, 0, None) == E                 # heads missing
    assert f(0x1000, 1, 0, 0x3000, 8, 0, None) == E                 # next missing
    assert f(0x1000, 1, 0x2000, 0x2000, 8, 0, None) == E            # prev aliases next
    assert f(0x1000, 1, 0x2002, 0x3000, 8, 0, None) == E            # misaligned next
    assert f(0x1000, 1, 0x2000, 0x3000, 8, 0x4001, None) == E       # misaligned status
    assert f(0, 0, 0, 0, 0, 0, None) == _lib.OK                     # nothing to do


def test_lists_host_checks(lib):
    E = _lib.EINVAL
    assert _lib.lists_workspace_bytes(1 << 20, 100, 32, 8) > 0
    assert _lib.lists_workspace_bytes(1 << 20, 0, 32, 8) == 0
    assert _lib.lists_workspace_bytes(1 << 20, 100, 32, 3) == 0
    assert _lib.lists_workspace_bytes(0xFFFFFFFF, 100, 32, 8) == 0

    def call(heads=0x1000, offs=0x2000, L=4, total=100, nin=0x3000, nout=0x3000, keys=0x4000,
             M=32, K=8, flags=0, nh=0x5000, st=0x6000, ws=0x100000, wsb=1 << 40):
        return lib.pbit_sort_lists(heads, offs, L, total, nin, nout, keys, M, K, flags, nh, st,
                                   ws, wsb, None)
    assert call(L=0) == E
    assert call(M=24) == E
    assert call(heads=0) == E
    assert call(offs=0x2004) == E      # offsets must be 8-byte aligned
    assert call(st=0) == E
    assert call(nin=0) == E
    assert call(flags=16) == E
    assert call(flags=_lib.SIGNED | _lib.FLOAT) == E
    assert call(wsb=100) == _lib.ENOMEM


def test_tuning_table_is_read_and_applied(lib):
    """K = 0 takes the tuning table's choice: the workspace a K = 0 call asks
    for equals the one for the table's K, an added entry overrides the
    built-in one for sizes up to its n_max only, and reset restores it."""
    _lib.tune_reset()
    try:
        k0, c0 = _lib.tune_lookup(0, 32, 1 << 20)
        assert k0 in (4, 8) and c0 in (1024, 2048, 4096)
        assert _lib.workspace_bytes(1 << 20, 32, 0) == _lib.workspace_bytes(1 << 20, 32, k0)
        other = 12 - k0
        assert _lib.tune_set(0, 32, 1 << 21, other, 2048) == 0
        assert _lib.tune_lookup(0, 32, 1 << 20) == (other, 2048)
        assert _lib.tune_lookup(0, 32, (1 << 21) + 1) == (k0, c0)
        assert _lib.workspace_bytes(1 << 20, 32, 0) == _lib.workspace_bytes(1 << 20, 32, other)
        kb, cb = _lib.tune_lookup(1, 16, 5000)
        assert _lib.tune_set(1, 16, 1 << 30, 4, 4096) == 0
        assert _lib.tune_lookup(1, 16, 5000) == (4, 4096)
        assert (_lib.lists_workspace_bytes(1 << 20, 100, 16, 0)
                == _lib.lists_workspace_bytes(1 << 20, 100, 16, 4))
        # rejected entries
        assert _lib.tune_set(2, 32, 1, 8, 2048) == _lib.EINVAL
        assert _lib.tune_set(0, 32, 1, 3, 2048) == _lib.EINVAL
        assert _lib.tune_set(0, 8, 1, 16, 2048) == _lib.EINVAL
        assert _lib.tune_set(1, 32, 1, 8, 512) == _lib.EINVAL
        _lib.tune_clear()
        assert _lib.tune_lookup(1, 32, 5000) == (8, 2048)
        assert _lib.tune_lookup(0, 8, 5000) == (4, 2048)
        _lib.tune_reset()
        assert _lib.tune_lookup(0, 32, 1 << 20) == (k0, c0)
        assert _lib.tune_lookup(1, 16, 5000) == (kb, cb)
    finally:
        _lib.tune_reset()
