"""The sort entry points queue no allocation, no memset and no host sync, so
they can be captured in a HIP graph: every replay (with eager work and
synchronisations in between) must equal the eager result."""
import numpy as np
import pytest

from paper_cs_0511020_amd import inputs

from .gpu_util import to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _capture(torch, fn):
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.graph(g, stream=side):
        fn(int(torch.cuda.current_stream().cuda_stream))
    torch.cuda.current_stream().wait_stream(side)
    return g


def test_graph_replay_single_list():
    import torch
    from paper_cs_0511020_amd import _lib
    rng = inputs.rng_for(6001)
    n = 300000
    nxt, head, _ = inputs.random_list(n, rng)
    keys = inputs.uniform_keys(n, 32, rng)
    nt, kt = to_dev(nxt, torch), to_dev(keys, torch)
    out = torch.full_like(nt, -1)
    res = torch.zeros(2, dtype=torch.int32, device="cuda")
    wsb = _lib.workspace_bytes(n, 32, 8)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    lib = _lib.load()

    def call(stream):
        st = lib.pbit_sort_list_async(head, nt.data_ptr(), out.data_ptr(), kt.data_ptr(), n, 32,
                                      8, 0, res.data_ptr(), ws.data_ptr(), wsb, stream)
        assert st == 0

    call(int(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    eager_out, eager_res = out.clone(), res.clone()
    g = _capture(torch, call)
    for i in range(4):
        out.fill_(-1)
        res.zero_()
        ws.random_(0, 255)  # eager work that scrambles the workspace between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager_out), "replay %d" % i
        assert torch.equal(res, eager_res), "replay %d" % i


def test_graph_replay_batched():
    import torch
    from paper_cs_0511020_amd import _lib
    rng = inputs.rng_for(6002)
    lengths = inputs.log_uniform_lengths(300, 4, 14, rng, 16, 1 << 14)
    nxt, heads, offs = inputs.slab_lists(lengths, rng)
    keys = inputs.uniform_keys(nxt.shape[0], 32, rng)
    ht = to_dev(heads, torch)
    ot = torch.from_numpy(offs.astype(np.int64)).to("cuda")
    nt, kt = to_dev(nxt, torch), to_dev(keys, torch)
    out = torch.full_like(nt, -1)
    nh = torch.zeros(len(lengths), dtype=torch.int32, device="cuda")
    st_t = torch.zeros(1, dtype=torch.int32, device="cuda")
    total, L = int(nxt.shape[0]), len(lengths)
    wsb = _lib.lists_workspace_bytes(total, L, 32, 8)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    lib = _lib.load()

    def call(stream):
        st = lib.pbit_sort_lists(ht.data_ptr(), ot.data_ptr(), L, total, nt.data_ptr(),
                                 out.data_ptr(), kt.data_ptr(), 32, 8, 0, nh.data_ptr(),
                                 st_t.data_ptr(), ws.data_ptr(), wsb, stream)
        assert st == 0

    call(int(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    assert int(st_t.item()) == 0
    eager_out, eager_nh = out.clone(), nh.clone()
    g = _capture(torch, call)
    for i in range(4):
        out.fill_(-1)
        nh.zero_()
        st_t.fill_(7)
        ws.random_(0, 255)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert int(st_t.item()) == 0
        assert torch.equal(out, eager_out), "replay %d" % i
        assert torch.equal(nh, eager_nh), "replay %d" % i
