"""The entry point that allocates nothing (pbit_sort_list_noalloc): called
through the C ABI twice in a row, the second time with a smaller list of
another key width, each result bit-exact against pbit_sort_list_async (the
entry point with a caller workspace) and the oracle; a list too large for its
fixed workspace is refused with PBIT_ENOMEM and nothing written."""
import numpy as np
import pytest

from paper_cs_0511020_amd import inputs

from .gpu_util import from_dev, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _case(torch, oracle_mod, n, M, K, seed):
    from paper_cs_0511020_amd import _lib
    print("no-alloc case n=%d M=%d K=%d" % (n, M, K), flush=True)
    rng = inputs.rng_for(seed)
    nxt, head, _ = inputs.random_list(n, rng)
    keys = inputs.uniform_keys(n, M, rng)
    keys[::4] = keys[1]  # ties
    nt, kt = to_dev(nxt, torch), to_dev(keys, torch)
    out_na = torch.full_like(nt, -1)
    res_na = torch.full((2,), -7, dtype=torch.int32, device="cuda")
    st = _lib.sort_list_noalloc(head, nt, out_na, kt, n, M, K, 0, res_na)
    assert st == _lib.OK
    out_ws = torch.full_like(nt, -1)
    res_ws = torch.full((2,), -7, dtype=torch.int32, device="cuda")
    wsb = _lib.workspace_bytes(n, M, K)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    assert _lib.sort_list_async(head, nt, out_ws, kt, n, M, K, 0, res_ws, ws, wsb) == _lib.OK
    torch.cuda.synchronize()
    assert torch.equal(res_na, res_ws) and int(res_na[1].item()) == 0
    assert torch.equal(out_na, out_ws)
    eh, enext = oracle_mod.sort_list(head, nxt, keys, M, K if K else 8)
    assert int(res_na[0].item()) & 0xFFFFFFFF == eh
    assert np.array_equal(from_dev(out_na), enext)


def test_noalloc_twice_then_smaller(oracle_mod):
    import torch
    _case(torch, oracle_mod, 600000, 32, 0, 6101)
    _case(torch, oracle_mod, 70001, 64, 4, 6102)


def test_noalloc_refuses_lists_beyond_its_workspace():
    import torch
    from paper_cs_0511020_amd import _lib
    n = 800000
    assert _lib.workspace_bytes(n, 32, 8) > _lib.NOALLOC_SCRATCH_BYTES
    rng = inputs.rng_for(6103)
    nxt, head, _ = inputs.random_list(n, rng)
    nt = to_dev(nxt, torch)
    kt = to_dev(inputs.uniform_keys(n, 32, rng), torch)
    out = torch.full_like(nt, -1)
    res = torch.full((2,), -7, dtype=torch.int32, device="cuda")
    assert _lib.sort_list_noalloc(head, nt, out, kt, n, 32, 8, 0, res) == _lib.ENOMEM
    torch.cuda.synchronize()
    assert bool((out == -1).all().item()) and bool((res == -7).all().item())
