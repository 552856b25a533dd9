"""Scheduler logic of the request server on the CPU: a fake executor backed
by the oracle and a small memory budget; no GPU involved."""
import time

import numpy as np

from paper_cs_0511020_amd import inputs
from paper_cs_0511020_amd.serve import NIL, Request, SortServer


class CpuExecutor:
    """Runs every batch on the CPU oracle; a batch completes `delay` seconds
    after it was launched."""

    def __init__(self, K=4, delay=0.0):
        import oracle
        self.oracle = oracle
        self.K = K
        self.delay = delay
        self.t0 = None

    def start_clock(self):
        self.t0 = time.perf_counter()

    def launch(self, batch, batch_id):
        for r in batch:
            h, out = self.oracle.sort_list(r.head, r.next, r.keys, r.M, self.K)
            r.out[:] = out
            r.new_head = h & 0xFFFFFFFF if h >= 0 else h
            r.status = 0 if h >= 0 or h == NIL else h
        return {"batch": batch, "ready": time.perf_counter() + self.delay, "id": batch_id}

    def poll(self, h):
        return time.perf_counter() >= h["ready"]

    def finish(self, h):
        t = time.perf_counter() - self.t0
        for r in h["batch"]:
            r.done = t


def make_host_requests(count, seed, rate=None):
    rng = inputs.rng_for(seed)
    reqs = []
    t = 0.0
    for i in range(count):
        n = int(rng.integers(1, 3000))
        M = int(rng.choice([8, 16, 32, 64]))
        nxt, head, _ = inputs.random_list(n, rng)
        keys = inputs.uniform_keys(n, M, rng)
        if rate:
            t += float(rng.exponential(1.0 / rate))
        reqs.append(Request(rid=i, arrival=t, n=n, M=M, head=head, next=nxt, keys=keys,
                            out=np.zeros(n, dtype=np.uint32)))
    return reqs


def fixed_share(n, M, K):
    return n * 10


def test_every_request_served_like_alone(oracle_mod):
    reqs = make_host_requests(60, 7001, rate=3000.0)
    server = SortServer(CpuExecutor(K=4, delay=0.002), slots=8, budget_bytes=40000,
                        share=fixed_share)
    st = server.run(reqs)
    assert st.requests == 60 and st.batches >= 1
    for r in reqs:
        h, out = oracle_mod.sort_list(r.head, r.next, r.keys, r.M, 4)
        assert r.new_head == h and np.array_equal(r.out, out)
        assert r.done >= r.arrival
    # admission never exceeded the budget (a lone request may use it whole)
    assert st.max_inflight_bytes <= max(40000, max(fixed_share(r.n, 0, 0) for r in reqs))


def test_admission_is_fifo_and_batches_group_widths():
    reqs = make_host_requests(40, 7002)  # all arrive at t = 0
    server = SortServer(CpuExecutor(K=4, delay=0.001), slots=5, budget_bytes=10 ** 9,
                        share=fixed_share)
    server.run(reqs)
    # admission follows arrival order
    order = sorted(reqs, key=lambda r: (r.admitted, r.rid))
    assert [r.rid for r in order] == sorted(r.rid for r in reqs)
    # every batch holds one key width and at most `slots` requests
    by_batch = {}
    for r in reqs:
        by_batch.setdefault(r.batch, []).append(r)
    for b in by_batch.values():
        assert len({r.M for r in b}) == 1
        assert len(b) <= 5


def test_budget_blocks_until_memory_frees():
    reqs = make_host_requests(12, 7003)
    big = max(fixed_share(r.n, 0, 0) for r in reqs)
    server = SortServer(CpuExecutor(K=4, delay=0.003), slots=64, budget_bytes=big,
                        share=fixed_share)
    st = server.run(reqs)
    assert st.max_inflight_bytes <= big
    assert st.batches >= 2
