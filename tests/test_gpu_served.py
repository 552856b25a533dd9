"""GPU serving: requests of mixed sizes and key widths, admitted by slots and
memory and batched continuously, come out exactly as each request sorted
alone; a few are also checked against the oracle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _alone(torch, r):
    from paper_cs_0511020_amd.sorter import ListSorter
    out = torch.empty_like(r.next)
    h = ListSorter().sort(r.head, r.next, r.keys, next_out=out)
    return h, out


@pytest.mark.parametrize("rate", [None, 2e8])
def test_served_results_identical_alone_and_in_mix(oracle_mod, rate):
    import torch
    from paper_cs_0511020_amd.serve import GpuExecutor, SortServer, make_requests_device
    reqs = make_requests_device(48, seed=5001, lo_log2=4, hi_log2=16, rate_nodes_s=rate)
    server = SortServer(GpuExecutor(streams=2), slots=12, budget_bytes=256 << 20)
    st = server.run(reqs)
    torch.cuda.synchronize()
    print("served", st.as_dict(), flush=True)
    assert st.requests == 48 and st.batches > 1
    assert len({r.M for r in reqs}) == 4
    for r in reqs:
        assert r.status == 0
        h, out = _alone(torch, r)
        assert r.new_head == h, r.rid
        assert torch.equal(r.out, out), r.rid
    for r in reqs[:6]:
        nxt = r.next.cpu().numpy().view(np.uint32)
        keys = r.keys.cpu().numpy().view({8: np.uint8, 16: np.uint16, 32: np.uint32,
                                          64: np.uint64}[r.M])
        K = 4 if r.M == 8 else 8
        eh, enext = oracle_mod.sort_list(r.head, nxt, keys, r.M, K)
        assert r.new_head == eh
        assert np.array_equal(r.out.cpu().numpy().view(np.uint32), enext)


def test_fifo_baseline_executor():
    import torch
    from paper_cs_0511020_amd.serve import PlainExecutor, SortServer, make_requests_device
    reqs = make_requests_device(16, seed=5002, lo_log2=4, hi_log2=14)
    st = SortServer(PlainExecutor(), slots=1, budget_bytes=1 << 30).run(reqs)
    torch.cuda.synchronize()
    assert st.batches == 16
    for r in reqs:
        h, out = _alone(torch, r)
        assert r.new_head == h and torch.equal(r.out, out)


def test_served_full_size_mix(oracle_mod):
    """Requests of 2^10..2^24 nodes over all four key widths, all arriving at
    once, so the first ticks batch requests of very different sizes through
    the gather form.  Every request must equal the single-list sort of it
    alone; per key width the largest request up to 2^23 nodes is checked
    against the oracle."""
    import torch
    from paper_cs_0511020_amd.serve import GpuExecutor, SortServer, make_requests_device
    reqs = make_requests_device(40, seed=5003, lo_log2=10, hi_log2=24)
    print("full-size mix: %d requests, %d nodes, largest %d" % (
        len(reqs), sum(r.n for r in reqs), max(r.n for r in reqs)), flush=True)
    server = SortServer(GpuExecutor(streams=2), slots=16, budget_bytes=96 << 30)
    st = server.run(reqs)
    torch.cuda.synchronize()
    print("served", st.as_dict(), flush=True)
    assert st.requests == 40
    assert len({r.M for r in reqs}) == 4
    assert max(r.n for r in reqs) > (1 << 22)
    sizes = {}
    for r in reqs:
        sizes.setdefault(r.batch, []).append(r.n)
    # a request above 2^20 nodes went through the gather form with others
    assert any(len(v) > 1 and max(v) > (1 << 20) for v in sizes.values())
    for r in reqs:
        assert r.status == 0
        h, out = _alone(torch, r)
        assert r.new_head == h, r.rid
        assert torch.equal(r.out, out), r.rid
    dt = {8: np.uint8, 16: np.uint16, 32: np.uint32, 64: np.uint64}
    for M in (8, 16, 32, 64):
        cand = [r for r in reqs if r.M == M and r.n <= (1 << 23)]
        r = max(cand, key=lambda x: x.n)
        print("oracle check M=%d n=%d" % (M, r.n), flush=True)
        nxt = r.next.cpu().numpy().view(np.uint32)
        keys = r.keys.cpu().numpy().view(dt[M])
        eh, enext = oracle_mod.sort_list(r.head, nxt, keys, M, 4 if M == 8 else 8)
        assert r.new_head == eh
        assert np.array_equal(r.out.cpu().numpy().view(np.uint32), enext)
