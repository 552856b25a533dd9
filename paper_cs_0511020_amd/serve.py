"""A sort-request server with continuous batching.

Requests are lists already resident in device memory (next[] in list-local
indices plus keys of 8, 16, 32 or 64 bits).  A request arrives at its
arrival time; it is admitted, in arrival order, when a slot is free and the
free-HBM budget covers its share of workspace.  On every scheduler tick the
requests admitted in that tick are grouped by key width and each group is
launched as ONE batched sort (the gather form of the C ABI, which reads every
list in place), alternating over several streams; batches admitted while
others run overlap with them on the device.  Completion is detected from HIP
events, and each request's latency is measured from its arrival to the
device-side end of its batch.

Executors:
  GpuExecutor    the library on one device (one batched call per launch)
  PlainExecutor  one single-list call per request, one stream: the FIFO
                 baseline that serves requests one at a time
An executor provides start_clock(), launch(batch, id) -> handle, poll(handle)
and finish(handle); the scheduler tests plug in a CPU executor of their own.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field
from typing import Any

import numpy as np

from . import _lib

NIL = 0xFFFFFFFF


@dataclass
class Request:
    rid: int
    arrival: float            # seconds after the start of the run
    n: int
    M: int
    head: int                 # list-local
    next: Any                 # device int32 tensor (or numpy array for the CPU executor)
    keys: Any
    out: Any = None           # receives the relinked next[] (list-local)
    new_head: int = -1
    status: int = 0
    admitted: float = -1.0
    done: float = -1.0
    batch: int = -1
    share: int = 0            # workspace bytes reserved while admitted
    order: Any = None         # optional: the input list order (node at each position)

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def workspace_share(n: int, M: int, K: int = 0) -> int:
    """Workspace bytes a request adds to a batch (its single-list estimate)."""
    return max(_lib.lists_workspace_bytes(max(n, 1), 1, M, K), 1)


class GpuExecutor:
    """Launch a batch as one gather-form batched sort on one of `streams`."""

    def __init__(self, device="cuda", streams: int = 2, K: int = 0):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(streams)]
        self.K = K
        # sorts on several streams run at the same time: tiles in start order
        self.flags = _lib.SHARED if streams > 1 else 0
        self.next_stream = 0
        self.t0_event = None
        self.lib = _lib.load()

    def start_clock(self):
        torch = self.torch
        self.t0_event = torch.cuda.Event(enable_timing=True)
        self.t0_event.record(torch.cuda.current_stream(self.device))

    def launch(self, batch, batch_id):
        torch = self.torch
        M = batch[0].M
        L = len(batch)
        if L == 1:
            return self._launch_single(batch, batch_id)
        lens = np.array([r.n for r in batch], dtype=np.int64)
        offs = np.zeros(L + 1, dtype=np.int64)
        offs[1:] = np.cumsum(lens)
        total = int(offs[-1])
        meta = np.zeros((5, L), dtype=np.int64)
        meta[0] = [r.head for r in batch]
        meta[1] = [r.next.data_ptr() for r in batch]
        meta[2] = [r.out.data_ptr() for r in batch]
        meta[3] = [r.keys.data_ptr() for r in batch]
        stream = self.streams[self.next_stream]
        self.next_stream = (self.next_stream + 1) % len(self.streams)
        wsb = _lib.lists_workspace_bytes(total, L, M, self.K)
        # pinned staging so that the small metadata copies are queued on the
        # stream instead of stalling the host until the stream drains
        h_meta = torch.empty((6, L + 1), dtype=torch.int64, pin_memory=True)
        h_meta[:5, :L] = torch.from_numpy(meta)
        h_meta[5] = torch.from_numpy(offs)
        with torch.cuda.stream(stream):
            d_all = h_meta.to(self.device, non_blocking=True)
            d_meta = d_all[:5, :L]
            d_heads = d_meta[0].to(torch.int32)
            d_offs = d_all[5]
            ws = torch.empty(wsb, dtype=torch.uint8, device=self.device)
            new_heads = torch.empty(L, dtype=torch.int32, device=self.device)
            status = torch.zeros(1, dtype=torch.int32, device=self.device)
            st = self.lib.pbit_sort_lists_gather(
                d_heads.data_ptr(), d_offs.data_ptr(), L, total, d_meta[1].data_ptr(),
                d_meta[2].data_ptr(), d_meta[3].data_ptr(), M, self.K, self.flags,
                new_heads.data_ptr(),
                status.data_ptr(), ws.data_ptr(), wsb, int(stream.cuda_stream))
            if st != 0:
                raise RuntimeError("batched launch failed: " + _lib.status_string(st))
            end = torch.cuda.Event(enable_timing=True)
            end.record(stream)
        return {"batch": batch, "end": end, "keep": (h_meta, d_all, d_heads, ws),
                "new_heads": new_heads, "status": status, "ws_bytes": wsb, "id": batch_id}

    def _launch_single(self, batch, batch_id):
        """A batch of one request takes the single-list call: fewer kernels
        than the batched form, which pays off when requests arrive apart."""
        torch = self.torch
        r = batch[0]
        stream = self.streams[self.next_stream]
        self.next_stream = (self.next_stream + 1) % len(self.streams)
        wsb = _lib.workspace_bytes(r.n, r.M, self.K)
        with torch.cuda.stream(stream):
            ws = torch.empty(wsb, dtype=torch.uint8, device=self.device)
            res = torch.zeros(2, dtype=torch.int32, device=self.device)
            st = self.lib.pbit_sort_list_async(r.head, r.next.data_ptr(), r.out.data_ptr(),
                                               r.keys.data_ptr(), r.n, r.M, self.K, self.flags,
                                               res.data_ptr(), ws.data_ptr(), wsb,
                                               int(stream.cuda_stream))
            if st != 0:
                raise RuntimeError("single launch failed: " + _lib.status_string(st))
            end = torch.cuda.Event(enable_timing=True)
            end.record(stream)
        return {"batch": batch, "end": end, "keep": (ws,), "single": res, "id": batch_id}

    def poll(self, h) -> bool:
        return h["end"].query()

    def finish(self, h):
        h["end"].synchronize()
        t = self.t0_event.elapsed_time(h["end"]) * 1e-3
        if "single" in h:
            head, st = (int(x) for x in h["single"].cpu().tolist())
            r = h["batch"][0]
            r.new_head = head & 0xFFFFFFFF
            r.status = st
            r.done = t
            h["keep"] = None
            return
        nh = h["new_heads"].cpu().numpy().view(np.uint32)
        st = int(h["status"].item())
        for r, x in zip(h["batch"], nh):
            r.new_head = int(x)
            r.status = st
            r.done = t
        h["keep"] = None


class PlainExecutor(GpuExecutor):
    """Baseline: every request is sorted alone by the single-list call on one
    stream (a FIFO queue without batching)."""

    def __init__(self, device="cuda", K: int = 0):
        super().__init__(device, streams=1, K=K)

    def launch(self, batch, batch_id):
        torch = self.torch
        stream = self.streams[0]
        handles = []
        with torch.cuda.stream(stream):
            for r in batch:
                wsb = _lib.workspace_bytes(r.n, r.M, self.K)
                ws = torch.empty(wsb, dtype=torch.uint8, device=self.device)
                res = torch.zeros(2, dtype=torch.int32, device=self.device)
                st = self.lib.pbit_sort_list_async(r.head, r.next.data_ptr(), r.out.data_ptr(),
                                                   r.keys.data_ptr(), r.n, r.M, self.K, 0,
                                                   res.data_ptr(), ws.data_ptr(), wsb,
                                                   int(stream.cuda_stream))
                if st != 0:
                    raise RuntimeError("plain launch failed: " + _lib.status_string(st))
                handles.append((r, res, ws))
            end = torch.cuda.Event(enable_timing=True)
            end.record(stream)
        return {"items": handles, "end": end, "id": batch_id}

    def finish(self, h):
        h["end"].synchronize()
        t = self.t0_event.elapsed_time(h["end"]) * 1e-3
        for r, res, _ in h["items"]:
            head, st = (int(x) for x in res.cpu().tolist())
            r.new_head = head & 0xFFFFFFFF
            r.status = st
            r.done = t
        h["items"] = None


@dataclass
class ServerStats:
    requests: int
    nodes: int
    wall_s: float
    throughput_mnodes_s: float
    p50_ms: float
    p99_ms: float
    mean_ms: float
    batches: int
    mean_batch: float
    max_inflight_bytes: int
    budget_bytes: int
    events: list = field(default_factory=list)

    def as_dict(self):
        d = dict(self.__dict__)
        d.pop("events", None)
        return d


class SortServer:
    """Admission by slots and free-HBM budget, continuous batching per tick."""

    def __init__(self, executor, slots: int = 64, budget_bytes: int = 8 << 30,
                 max_batch_nodes: int = 1 << 28, K: int = 0, share=workspace_share):
        self.ex = executor
        self.slots = slots
        self.budget = int(budget_bytes)
        self.max_batch_nodes = max_batch_nodes
        self.K = K
        self.share = share

    def run(self, requests, idle_sleep: float = 20e-6) -> ServerStats:
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        waiting = collections.deque()
        inflight = []
        nxt = 0
        done = 0
        slots_free = self.slots
        budget_free = self.budget
        max_used = 0
        batches = 0
        batch_sizes = []
        events = []
        self.ex.start_clock()
        t0 = time.perf_counter()
        while done < len(reqs):
            now = time.perf_counter() - t0
            while nxt < len(reqs) and reqs[nxt].arrival <= now:
                waiting.append(reqs[nxt])
                nxt += 1
            progressed = False
            still = []
            for h in inflight:
                if self.ex.poll(h):
                    self.ex.finish(h)
                    for r in h["reqs"]:
                        slots_free += 1
                        budget_free += r.share
                        done += 1
                    events.append(("done", h["id"], time.perf_counter() - t0))
                    progressed = True
                else:
                    still.append(h)
            inflight = still
            # admit in arrival order while a slot and the budget allow
            groups = collections.OrderedDict()
            gnodes = collections.Counter()
            while waiting and slots_free > 0:
                r = waiting[0]
                need = self.share(r.n, r.M, self.K)
                if need > budget_free and (inflight or groups):
                    break  # wait for memory to free up
                if gnodes[r.M] + r.n > self.max_batch_nodes and groups.get(r.M):
                    break
                waiting.popleft()
                r.share = need
                r.admitted = now
                slots_free -= 1
                budget_free -= need
                groups.setdefault(r.M, []).append(r)
                gnodes[r.M] += r.n
            max_used = max(max_used, self.budget - budget_free)
            for M, batch in groups.items():
                h = self.ex.launch(batch, batches)
                h["reqs"] = batch
                for r in batch:
                    r.batch = batches
                events.append(("launch", batches, now, len(batch), sum(r.n for r in batch)))
                batches += 1
                batch_sizes.append(len(batch))
                inflight.append(h)
                progressed = True
            if not progressed:
                if idle_sleep > 0:
                    time.sleep(idle_sleep)
        wall = time.perf_counter() - t0
        lat = np.sort(np.array([r.latency for r in reqs]))
        nodes = int(sum(r.n for r in reqs))
        span = max(r.done for r in reqs) - min(r.arrival for r in reqs)
        return ServerStats(
            requests=len(reqs), nodes=nodes, wall_s=wall,
            throughput_mnodes_s=nodes / max(span, 1e-9) / 1e6,
            p50_ms=float(np.percentile(lat, 50) * 1e3), p99_ms=float(np.percentile(lat, 99) * 1e3),
            mean_ms=float(lat.mean() * 1e3), batches=batches,
            mean_batch=float(np.mean(batch_sizes)) if batch_sizes else 0.0,
            max_inflight_bytes=int(max_used), budget_bytes=self.budget, events=events)


def make_requests_device(count: int, seed: int, lo_log2: float = 10, hi_log2: float = 24,
                         widths=(8, 16, 32, 64), rate_nodes_s: float | None = None,
                         device="cuda", keep_order: bool = False):
    """Seeded request mix kept in device memory: length log-uniform in
    [2^lo, 2^hi], key width uniform over `widths`, uniform keys, random list
    layout; Poisson arrivals at `rate_nodes_s` offered nodes per second (all
    at time 0 when None).  With keep_order each request also keeps its input
    list order (int32 device tensor), for checking results."""
    import torch

    from . import inputs
    rng = inputs.rng_for(seed)
    lens = inputs.log_uniform_lengths(count, lo_log2, hi_log2, rng, 1 << int(lo_log2),
                                      1 << int(hi_log2))
    Ms = rng.choice(np.array(widths), size=count)
    if rate_nodes_s:
        lam = rate_nodes_s / float(lens.mean())
        arrivals = np.cumsum(rng.exponential(1.0 / lam, size=count))
    else:
        arrivals = np.zeros(count)
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    reqs = []
    for i in range(count):
        n, M = int(lens[i]), int(Ms[i])
        perm = torch.randperm(n, generator=g, device=device, dtype=torch.int64)
        nxt = torch.full((n,), -1, dtype=torch.int32, device=device)
        nxt[perm[:-1]] = perm[1:].to(torch.int32)
        if M == 8:
            keys = torch.randint(0, 256, (n,), generator=g, device=device, dtype=torch.uint8)
        elif M == 16:
            keys = torch.randint(-(1 << 15), 1 << 15, (n,), generator=g, device=device,
                                 dtype=torch.int16)
        elif M == 32:
            keys = torch.randint(-(1 << 31), 1 << 31, (n,), generator=g, device=device,
                                 dtype=torch.int32)
        else:
            hi = torch.randint(-(1 << 31), 1 << 31, (n,), generator=g, device=device,
                               dtype=torch.int64)
            lo = torch.randint(0, 1 << 32, (n,), generator=g, device=device, dtype=torch.int64)
            keys = (hi << 32) | lo
        reqs.append(Request(rid=i, arrival=float(arrivals[i]), n=n, M=M,
                            head=int(perm[0].item()), next=nxt, keys=keys,
                            out=torch.empty_like(nxt),
                            order=perm.to(torch.int32) if keep_order else None))
    return reqs
