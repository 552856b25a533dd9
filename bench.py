#!/usr/bin/env python3
"""Benchmark of the MI355X Pbit list sort.

Default run (the headline): one step = one whole sort (pack, list ranking,
every digit pass, relink) of a single list of n = 2^24 nodes with uint32 keys
and a random-permutation next[] layout, inputs resident in HBM.  The sort
reads next_in and writes next_out (out of place, same traffic as in place),
so every step sorts the same input.  Each kernel stage is bracketed by HIP
events on the stream the library launches on; the dominant stage's
algorithmic bytes per launch over its mean launch time give the roofline
figure.

Beside the warm back-to-back rate (`value`) the line carries the same sort's
latency when L2 and the last-level cache are flushed before it (a 1 GiB write
on the stream, outside the sort's events), its HIP-graph replay time, and
extras: binary32 keys, nodes stored as records, the backward-link repair and
the paper's own input shape (10^7 nodes, keys below 2^15).

A "batched" section sorts 20 000 lists with log-uniform lengths by one
batched call (direct and replayed from a HIP graph), against the same lists
sorted by 20 000 single-list calls; a "served" section runs the request
server under Poisson arrivals.

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Mnodes/s at n=2^24 u32 (plain vs batched), %HBM roofline; p50/p99 sort latency"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=1 << 24)
    ap.add_argument("--K", type=int, default=0,
                    help="pattern bits (1, 2, 4 or 8; 0 = the library's tuned choice)")
    ap.add_argument("--M", type=int, default=32, choices=[32, 64], help="key bits")
    ap.add_argument("--dist", default="uniform", choices=["uniform", "zipf", "distinct8"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-n", type=int, default=1 << 24,
                    help="nodes in the list the CPU oracle sorts once")
    ap.add_argument("--batched", default="long", choices=["none", "short", "long"],
                    help="batched section: 20 000 lists of 16..2^16 nodes (short) or 16..2^20 (long)")
    ap.add_argument("--batched-steps", type=int, default=5)
    ap.add_argument("--no-plain-compare", action="store_true",
                    help="skip the 20 000 single-list calls of the batched comparison")
    ap.add_argument("--served", default="full", choices=["none", "small", "full"],
                    help="served section: 300 requests up to 2^20 nodes (small) or 2000 up "
                         "to 2^24 (full)")
    ap.add_argument("--no-cold", action="store_true",
                    help="skip the sorts timed after a 1 GiB cache flush")
    ap.add_argument("--no-graph", action="store_true",
                    help="skip the graph-replay timing of the single-list sort")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the float-key sort and the backward-link repair timings")
    ap.add_argument("--no-other-k", action="store_true",
                    help="skip the same list sorted with the other pattern width (4 vs 8)")
    ap.add_argument("--no-c3", action="store_true",
                    help="skip the 2^26-node list with 64-bit keys and a 64-bit payload")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="threads of the all-core oracle baseline (0 = every core)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    return ap.parse_args()


def source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_cs_0511020_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str, src_hash: str, config: dict):
    """HBM bytes per launch from committed rocprofv3 counter summaries, if they
    were taken on the current kernel sources and the same workload."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % kernel)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_hash") != src_hash or d.get("config") != config:
        return None
    return d.get("hbm_bytes_per_launch")


def percentile(sorted_vals, q):
    return sorted_vals[min(len(sorted_vals) - 1, int(round(q * (len(sorted_vals) - 1))))]


def unsigned_order(torch, keys):
    """int64 tensor whose signed order is the unsigned order of the stored keys
    (keys arrive in signed storage of their width)."""
    if keys.dtype == torch.uint8:
        return keys.to(torch.int64)
    if keys.dtype == torch.int16:
        return keys.to(torch.int64) & 0xFFFF
    if keys.dtype == torch.int32:
        return keys.to(torch.int64) & 0xFFFFFFFF
    if keys.dtype == torch.int64:
        return keys ^ (-(1 << 63))
    raise TypeError(keys.dtype)


def relinked_ok(torch, head, nxt, keys, order):
    """On the device, the properties that together fix the stable sort of a
    list whose input order (node at each position) is `order`: exactly one
    NIL; every node but the head has exactly one predecessor; along every link
    the pair (key, input position) strictly increases, so the links form one
    path from the head over all nodes, sorted by key with ties in input
    order."""
    n = int(nxt.numel())
    if n == 0:
        return head == 0xFFFFFFFF
    if not 0 <= head < n:
        return False
    nil = nxt == -1
    if int(nil.sum().item()) != 1:
        return False
    src = torch.nonzero(~nil).flatten()
    tgt = nxt[src].to(torch.int64) & 0xFFFFFFFF
    if not bool((tgt < n).all().item()):
        return False
    indeg = torch.bincount(tgt, minlength=n)
    if not bool((indeg <= 1).all().item()) or int(indeg[head].item()) != 0:
        return False
    pos = torch.empty(n, dtype=torch.int64, device=nxt.device)
    pos[order.to(torch.int64)] = torch.arange(n, device=nxt.device)
    k = unsigned_order(torch, keys)
    ks, kt = k[src], k[tgt]
    return bool(((kt > ks) | ((kt == ks) & (pos[tgt] > pos[src]))).all().item())


def stage_table(lib, pools, counts):
    """Per-stage mean time per step and launches per step from event pools."""
    names, per_stage, launches, lat = {}, {}, {}, []
    for p, c in zip(pools, counts):
        lat.append(p.elapsed_ms(0, c - 1))
        tot, cnt = {}, {}
        for i in range(c - 1):
            sid = p.ids[i]
            name = names.setdefault(sid, lib.pbit_stage_name(sid).decode())
            tot[name] = tot.get(name, 0.0) + p.elapsed_ms(i, i + 1)
            cnt[name] = cnt.get(name, 0) + 1
        for name, v in tot.items():
            per_stage.setdefault(name, []).append(v)
            launches[name] = cnt[name]
    return {k: statistics.mean(v) for k, v in per_stage.items()}, launches, sorted(lat)


def run_plain(args, lib, torch, np, inputs, bytemodel, EventPool):
    dev = torch.device("cuda:0")
    n, K, M = args.n, args.K, args.M
    from paper_cs_0511020_amd import _lib
    Keff = K if K else _lib.tune_lookup(0, M, n)[0]
    passes = M // Keff
    seed = {"uniform": 2001, "zipf": 2002, "distinct8": 2003}[args.dist]
    rng = inputs.rng_for(seed)
    nxt, head, order = inputs.random_list(n, rng)
    if M == 64:
        keys = inputs.uniform_keys(n, 64, rng)
        keys_d = torch.from_numpy(keys.view(np.int64)).to(dev)
    else:
        keys = inputs.keys_by_distribution(args.dist, n, rng)
        keys_d = torch.from_numpy(keys.view(np.int32)).to(dev)
    next_in = torch.from_numpy(nxt.view(np.int32)).to(dev)
    next_out = torch.empty_like(next_in)
    from paper_cs_0511020_amd import _lib
    ws_bytes = _lib.workspace_bytes(n, M, K)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    result = torch.zeros(2, dtype=torch.int32, device=dev)
    sh = int(torch.cuda.current_stream().cuda_stream)
    max_ev = 64
    pools = [EventPool(max_ev) for _ in range(args.steps)]
    warm = EventPool(max_ev)
    rec = ctypes.c_int(0)

    def run(pool):
        st = lib.pbit_sort_list_profiled(
            head, next_in.data_ptr(), next_out.data_ptr(), keys_d.data_ptr(), n, M, K, 0,
            result.data_ptr(), ws.data_ptr(), ws_bytes, sh, pool.ptr(), pool.ids_ptr(),
            max_ev, ctypes.byref(rec))
        if st != 0:
            raise RuntimeError("sort failed: " + _lib.status_string(st))
        return rec.value

    for _ in range(args.warmup):
        run(warm)
    torch.cuda.synchronize()
    h0, st0 = (int(x) & 0xFFFFFFFF for x in result.cpu().tolist())
    if st0 != 0:
        raise RuntimeError("device status %d" % st0)
    counts = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        counts.append(run(pools[k]))
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3 / args.steps
    stage_ms, launches, lat = stage_table(lib, pools, counts)
    p50, p99 = statistics.median(lat), percentile(lat, 0.99)

    got = next_out.cpu().numpy().view(np.uint32)
    exp_order = order[np.argsort(keys[order], kind="stable")]
    ok = (h0 == int(exp_order[0])) and bool(np.array_equal(got[exp_order[:-1]], exp_order[1:]))

    # the other pattern width on the same input (K = 4 beside K = 8)
    other = None
    if Keff in (4, 8) and not args.no_other_k:
        K2 = 12 - Keff
        ws2_bytes = _lib.workspace_bytes(n, M, K2)
        ws2 = torch.empty(ws2_bytes, dtype=torch.uint8, device=dev)
        out2 = torch.empty_like(next_in)
        res2 = torch.zeros(2, dtype=torch.int32, device=dev)
        pools2 = [EventPool(max_ev) for _ in range(args.steps)]

        def run2(pool):
            st = lib.pbit_sort_list_profiled(
                head, next_in.data_ptr(), out2.data_ptr(), keys_d.data_ptr(), n, M, K2, 0,
                res2.data_ptr(), ws2.data_ptr(), ws2_bytes, sh, pool.ptr(), pool.ids_ptr(),
                max_ev, ctypes.byref(rec))
            if st != 0:
                raise RuntimeError("sort failed: " + _lib.status_string(st))
            return rec.value

        for _ in range(2):
            run2(warm)
        torch.cuda.synchronize()
        cnt2 = [run2(pools2[k]) for k in range(args.steps)]
        torch.cuda.synchronize()
        st2, ln2, lat2 = stage_table(lib, pools2, cnt2)
        h2 = int(res2[0].item()) & 0xFFFFFFFF
        g2 = out2.cpu().numpy().view(np.uint32)
        ok2 = h2 == int(exp_order[0]) and bool(np.array_equal(g2[exp_order[:-1]], exp_order[1:]))
        ex2 = ln2.get("digit_pass", M // K2)
        pass2 = st2.get("digit_pass", 0.0) / max(ex2, 1)
        w2 = M // 8
        pb2 = bytemodel.digit_pass_bytes_per_node(w2, ex2, n, K2)
        other = {"K": K2, "p50_ms": round(statistics.median(lat2), 4),
                 "Mnodes_s_at_p50": round(n / (statistics.median(lat2) * 1e-3) / 1e6, 1),
                 "digit_passes": ex2, "digit_pass_ms": round(pass2, 5),
                 "digit_pass_frac": round(pb2 * n / (pass2 * 1e-3) / 1e9
                                          / bytemodel.MI355X_HBM_PEAK_GBS, 4) if pass2 else None,
                 "correct": ok2}
        for p_ in pools2:
            p_.close()
        del ws2, out2

    # the same sort captured once in a HIP graph and replayed (no per-kernel
    # launch work on the host); reported beside the eager rate
    graph_ms = None
    if not args.no_graph:
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=side):
            st = lib.pbit_sort_list_async(head, next_in.data_ptr(), next_out.data_ptr(),
                                          keys_d.data_ptr(), n, M, K, 0, result.data_ptr(),
                                          ws.data_ptr(), ws_bytes,
                                          int(torch.cuda.current_stream().cuda_stream))
            if st != 0:
                raise RuntimeError("capture failed: " + _lib.status_string(st))
        torch.cuda.current_stream().wait_stream(side)
        for _ in range(2):
            g.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            g.replay()
        torch.cuda.synchronize()
        graph_ms = (time.perf_counter() - t0) * 1e3 / args.steps
        ok = ok and bool(np.array_equal(next_out.cpu().numpy().view(np.uint32), got))
        del g

    # cold: L2 and the last-level cache flushed (1 GiB written on the same
    # stream) before each sort; the flush lies outside the sort's events
    cold = None
    if not args.no_cold:
        scratch = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        cold_pools = [EventPool(max_ev) for _ in range(args.steps)]
        cold_counts = []
        for k in range(args.steps):
            scratch.fill_(k & 0x7F)
            cold_counts.append(run(cold_pools[k]))
        torch.cuda.synchronize()
        _, _, cold_lat = stage_table(lib, cold_pools, cold_counts)
        cold = {"p10_ms": round(percentile(cold_lat, 0.10), 4),
                "p50_ms": round(statistics.median(cold_lat), 4),
                "p90_ms": round(percentile(cold_lat, 0.90), 4),
                "Mnodes_s_at_p50": round(n / (statistics.median(cold_lat) * 1e-3) / 1e6, 1),
                "flush_bytes": 1 << 30}
        ok = ok and bool(np.array_equal(next_out.cpu().numpy().view(np.uint32), got))
        for p in cold_pools:
            p.close()
        del scratch

    w = M // 8
    executed = launches.get("digit_pass", passes)
    path_bpn = bytemodel.path_bytes_per_node(w, executed)
    path_frac = path_bpn * n / (p50 * 1e-3) / 1e9 / bytemodel.MI355X_HBM_PEAK_GBS
    cand = {k: v for k, v in stage_ms.items()
            if k in ("pack", "walk0", "unchain", "digit_pass", "relink")}
    src_hash = source_hash()

    def stage_roofline(st):
        launch_ms = stage_ms[st] / launches[st]
        if st == "digit_pass":
            per_node = bytemodel.digit_pass_bytes_per_node(w, executed, n, Keff)
        else:
            per_node = bytemodel.kernel_bytes_per_node(st, w)
        nbytes = per_node * n
        achieved = nbytes / (launch_ms * 1e-3) / 1e9
        return {
            "bound": "hbm", "kernel": st, "achieved": round(achieved, 1),
            "peak": bytemodel.MI355X_HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / bytemodel.MI355X_HBM_PEAK_GBS, 4),
            "traffic": load_traffic(st, src_hash, {"n": n, "M": M, "K": Keff, "dist": args.dist}),
            "algorithmic_bytes_per_launch": int(nbytes),
            "launch_ms": round(launch_ms, 5),
        }

    # the dominant stage, and the next one for context
    ranked = sorted(cand, key=cand.get, reverse=True)
    roofline = stage_roofline(ranked[0])
    roofline_second = stage_roofline(ranked[1]) if len(ranked) > 1 else None
    for p in pools + [warm]:
        p.close()
    del ws, next_in, next_out, keys_d
    return {
        "value": n / (wall_ms * 1e-3) / 1e6, "wall_ms": wall_ms, "p50": p50, "p99": p99,
        "roofline": roofline, "roofline_second": roofline_second, "stage_ms": stage_ms,
        "launches": launches, "correct": ok,
        "path_bpn": path_bpn, "path_frac": path_frac, "Keff": Keff, "src_hash": src_hash,
        "graph_ms": graph_ms, "cold": cold, "other_k": other,
    }


def run_extras(args, lib, torch, np, inputs, bytemodel):
    """Floating-point keys (binary32, both signs, repeats) through the whole
    path, the backward-link repair kernel of doubly-linked lists on the sorted
    result, and a list stored as records; each timed with events on the stream
    it runs on and checked against numpy."""
    from paper_cs_0511020_amd import _lib
    dev = torch.device("cuda:0")
    n, K = args.n, args.K
    Kshow = K if K else _lib.tune_lookup(0, 32, n)[0]
    rng = inputs.rng_for(2301)
    nxt, head, order = inputs.random_list(n, rng)
    keys = inputs.float_keys(n, 32, rng, specials=False)
    next_in = torch.from_numpy(nxt.view(np.int32)).to(dev)
    next_out = torch.empty_like(next_in)
    prev = torch.empty_like(next_in)
    keys_d = torch.from_numpy(keys.view(np.float32)).to(dev)
    ws_bytes = _lib.workspace_bytes(n, 32, K)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    result = torch.zeros(2, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    steps = max(3, args.steps // 3)

    def sort():
        st = _lib.sort_list_async(head, next_in, next_out, keys_d, n, 32, K, _lib.FLOAT, result,
                                  ws, ws_bytes, stream)
        if st != 0:
            raise RuntimeError("float sort failed: " + _lib.status_string(st))

    def repair():
        st = _lib.repair_prev(result, 1, next_out, prev, n, result, 4, stream)
        if st != 0:
            raise RuntimeError("repair failed: " + _lib.status_string(st))

    def timed(fn):
        for _ in range(2):
            fn()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * steps)]
        for k in range(steps):
            ev[2 * k].record(stream)
            fn()
            ev[2 * k + 1].record(stream)
        torch.cuda.synchronize()
        return statistics.median(ev[2 * k].elapsed_time(ev[2 * k + 1]) for k in range(steps))

    sort_ms = timed(sort)
    rep_ms = timed(repair)
    h = int(result[0].item()) & 0xFFFFFFFF
    got = next_out.cpu().numpy().view(np.uint32)
    vals = keys.view(np.float32)
    exp = order[np.argsort(vals[order], kind="stable")]
    ok_sort = h == int(exp[0]) and bool(np.array_equal(got[exp[:-1]], exp[1:]))
    pv = prev.cpu().numpy().view(np.uint32)
    ok_prev = bool(np.array_equal(pv[exp[1:]], exp[:-1])) and int(pv[exp[0]]) == 0xFFFFFFFF
    del next_out, prev, keys_d

    # nodes as 16-byte records {next, u32 key, u64 payload}: links rewritten in place
    ukeys = inputs.uniform_keys(n, 32, rng)
    rec = np.zeros((n, 4), dtype=np.uint32)
    rec[:, 0] = nxt
    rec[:, 1] = ukeys
    rec[:, 2] = np.arange(n, dtype=np.uint32)
    pristine = torch.from_numpy(rec.view(np.int32)).to(dev)
    recs = torch.empty_like(pristine)

    def sort_aos():
        recs.copy_(pristine)
        st = _lib.sort_list_aos_async(head, recs, 16, 0, 4, n, 32, K, 0, result, ws, ws_bytes,
                                      stream)
        if st != 0:
            raise RuntimeError("record sort failed: " + _lib.status_string(st))

    def copy_only():
        recs.copy_(pristine)

    aos_ms = timed(sort_aos)
    copy_ms = timed(copy_only)
    sort_aos()
    torch.cuda.synchronize()
    ha = int(result[0].item()) & 0xFFFFFFFF
    ra = recs.cpu().numpy().view(np.uint32).reshape(n, 4)
    expa = order[np.argsort(ukeys[order], kind="stable")]
    ok_aos = (ha == int(expa[0]) and bool(np.array_equal(ra[expa[:-1], 0], expa[1:]))
              and bool(np.array_equal(ra[:, 1:], rec[:, 1:])))
    del recs, pristine

    # the paper's own input shape: 10^7 nodes, keys uniform below 2^15 (its
    # rand() range); the patterns above bit 15 are constant, so their passes
    # are skipped
    pn = 10 ** 7
    prng = inputs.rng_for(2401)
    pnxt, phead, porder = inputs.random_list(pn, prng)
    pkeys = prng.integers(0, 1 << 15, pn, dtype=np.uint32)
    pnext_in = torch.from_numpy(pnxt.view(np.int32)).to(dev)
    pnext_out = torch.empty_like(pnext_in)
    pkeys_d = torch.from_numpy(pkeys.view(np.int32)).to(dev)
    pexp = porder[np.argsort(pkeys[porder], kind="stable")]
    paper_shape = {}
    for pk in (8, 4):
        pws_bytes = _lib.workspace_bytes(pn, 32, pk)
        pws = torch.empty(pws_bytes, dtype=torch.uint8, device=dev)

        def sort_paper():
            st = _lib.sort_list_async(phead, pnext_in, pnext_out, pkeys_d, pn, 32, pk, 0, result,
                                      pws, pws_bytes, stream)
            if st != 0:
                raise RuntimeError("paper-shape sort failed: " + _lib.status_string(st))

        pms = timed(sort_paper)
        hp = int(result[0].item()) & 0xFFFFFFFF
        gotp = pnext_out.cpu().numpy().view(np.uint32)
        okp = hp == int(pexp[0]) and bool(np.array_equal(gotp[pexp[:-1]], pexp[1:]))
        skipped = sum(1 for sh in range(0, 32, pk) if sh >= 15)
        paper_shape["K%d" % pk] = {"ms": round(pms, 4),
                                   "Mnodes_per_s": round(pn / (pms * 1e-3) / 1e6, 1),
                                   "passes": 32 // pk, "constant_patterns_skipped": skipped,
                                   "correct": okp}
        del pws
    del pnext_in, pnext_out, pkeys_d
    # short single lists: one workgroup sorts the whole list in LDS (lists of
    # at most the tuned cutoff); each size also timed on the device-wide path
    # (a cutoff below the size, through the tuning table) for comparison
    short = {}
    try:
        for sn in (1024, 4096):
            srng = inputs.rng_for(2501 + sn)
            snxt, shead, sorder = inputs.random_list(sn, srng)
            skeys = inputs.uniform_keys(sn, 32, srng)
            sn_in = torch.from_numpy(snxt.view(np.int32)).to(dev)
            sn_out = torch.empty_like(sn_in)
            sk_d = torch.from_numpy(skeys.view(np.int32)).to(dev)
            sws_bytes = _lib.workspace_bytes(sn, 32, 8)
            sws = torch.empty(sws_bytes, dtype=torch.uint8, device=dev)
            sexp = sorder[np.argsort(skeys[sorder], kind="stable")]
            row = {}
            for name, cut in (("one_workgroup", 4096), ("device_wide", 1024 if sn > 1024 else None)):
                if cut is None:
                    continue
                _lib.tune_clear()
                if _lib.tune_set(0, 32, 0xFFFFFFFF, 8, cut) != 0:
                    raise RuntimeError("tuning entry rejected")

                def sort_short():
                    st = _lib.sort_list_async(shead, sn_in, sn_out, sk_d, sn, 32, 8, 0, result,
                                              sws, sws_bytes, stream)
                    if st != 0:
                        raise RuntimeError("short sort failed: " + _lib.status_string(st))

                sms = timed(sort_short)
                hs = int(result[0].item()) & 0xFFFFFFFF
                gots = sn_out.cpu().numpy().view(np.uint32)
                oks = hs == int(sexp[0]) and bool(np.array_equal(gots[sexp[:-1]], sexp[1:]))
                row[name] = {"us": round(sms * 1e3, 1), "correct": oks}
            short["n%d" % sn] = row
            del sws, sn_in, sn_out, sk_d
    finally:
        _lib.tune_reset()
    rep_bytes = 8 * n + 4
    rep_gbs = rep_bytes / (rep_ms * 1e-3) / 1e9
    del ws, next_in
    return {
        "short_lists": dict(workload="single lists of 1024 and 4096 nodes, u32 uniform keys, "
                                     "K=8: the one-workgroup sort in LDS (cutoff 4096) and, at "
                                     "4096, the device-wide path (cutoff 1024)", **short),
        "float32_keys": {"workload": "single list n=%d binary32 keys, log-uniform magnitudes of "
                                     "both signs, 25%% repeats, K=%d" % (n, Kshow),
                         "ms": round(sort_ms, 4), "Mnodes_per_s": round(n / (sort_ms * 1e-3) / 1e6, 1),
                         "correct": ok_sort},
        "records": {"workload": "single list n=%d stored as 16-byte records {next, u32 key, "
                                "u64 payload}, links rewritten in place, K=%d" % (n, Kshow),
                    "ms": round(aos_ms - copy_ms, 4),
                    "Mnodes_per_s": round(n / ((aos_ms - copy_ms) * 1e-3) / 1e6, 1),
                    "note": "time of a restore copy of the records subtracted",
                    "correct": ok_aos},
        "paper_shape": dict(workload="single list n=10^7, u32 keys uniform on [0, 2^15), "
                                     "random-permutation layout", **paper_shape),
        "repair_prev": {"workload": "backward links of the sorted %d-node list" % n,
                        "ms": round(rep_ms, 4), "bytes_per_node": 8,
                        "achieved_GBs": round(rep_gbs, 1),
                        "frac": round(rep_gbs / bytemodel.MI355X_HBM_PEAK_GBS, 4),
                        "correct": ok_prev},
    }


def run_c3(args, lib, torch, np, bytemodel):
    """One list of 2^26 nodes with uniform 64-bit keys and a 64-bit payload per
    node (nodes never move, so the payload needs no handling), random layout,
    K = 8 and K = 4; inputs built on the device from a seeded generator;
    checked on the device by the properties that fix the stable sort."""
    from paper_cs_0511020_amd import _lib
    dev = torch.device("cuda:0")
    n, M = 1 << 26, 64
    g = torch.Generator(device=dev)
    g.manual_seed(3001)
    order = torch.randperm(n, generator=g, device=dev, dtype=torch.int64)
    nxt = torch.full((n,), -1, dtype=torch.int32, device=dev)
    nxt[order[:-1]] = order[1:].to(torch.int32)
    head = int(order[0].item())
    hi = torch.randint(-(1 << 31), 1 << 31, (n,), generator=g, device=dev, dtype=torch.int64)
    lo = torch.randint(0, 1 << 32, (n,), generator=g, device=dev, dtype=torch.int64)
    keys = (hi << 32) | lo
    del hi, lo
    payload = torch.randint(-(1 << 62), 1 << 62, (n,), generator=g, device=dev,
                            dtype=torch.int64)
    out = torch.empty_like(nxt)
    res = torch.zeros(2, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    steps = max(3, args.steps // 4)
    rows = {}
    for K in (8, 4):
        wsb = _lib.workspace_bytes(n, M, K)
        ws = torch.empty(wsb, dtype=torch.uint8, device=dev)

        def sort():
            st = _lib.sort_list_async(head, nxt, out, keys, n, M, K, 0, res, ws, wsb, stream)
            if st != 0:
                raise RuntimeError("u64 sort failed: " + _lib.status_string(st))

        sort()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * steps)]
        for k in range(steps):
            ev[2 * k].record(stream)
            sort()
            ev[2 * k + 1].record(stream)
        torch.cuda.synchronize()
        ms = statistics.median(ev[2 * k].elapsed_time(ev[2 * k + 1]) for k in range(steps))
        h = int(res[0].item()) & 0xFFFFFFFF
        ok = int(res[1].item()) == 0 and relinked_ok(torch, h, out, keys, order)
        passes = M // K
        bpn = bytemodel.path_bytes_per_node(8, passes)
        rows["K%d" % K] = {"ms": round(ms, 4), "Mnodes_per_s": round(n / (ms * 1e-3) / 1e6, 1),
                           "path_frac": round(bpn * n / (ms * 1e-3) / 1e9
                                              / bytemodel.MI355X_HBM_PEAK_GBS, 4),
                           "correct": ok}
        del ws
        torch.cuda.empty_cache()
    del order, nxt, keys, payload, out
    torch.cuda.empty_cache()
    return dict(workload="single list n=2^26, uint64 keys uniform, a uint64 payload per node, "
                         "random-permutation layout", **rows)


def run_batched(args, lib, torch, np, inputs, EventPool):
    """20 000 lists, log-uniform lengths in [16, 2^hi]: one batched call vs
    one single-list call per list, same inputs, same stream."""
    from paper_cs_0511020_amd import _lib
    dev = torch.device("cuda:0")
    hi = 20 if args.batched == "long" else 16
    rng = inputs.rng_for(4001)
    lengths = inputs.log_uniform_lengths(20000, 4, hi, rng, 16, 1 << hi)
    compare = not args.no_plain_compare
    d = inputs.slab_lists_device(lengths, seed=4001, M=32, local_copy=compare)
    L = int(lengths.shape[0])
    total = int(d["offsets_host"][-1])
    M, K = 32, 0  # the tuned pattern width and cutoff
    Keff, cutoff = _lib.tune_lookup(1, M, total)
    ws_bytes = _lib.lists_workspace_bytes(total, L, M, K)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    next_out = torch.empty_like(d["next"])
    new_heads = torch.empty(L, dtype=torch.int32, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    sh = int(stream.cuda_stream)
    max_ev = 96
    steps = max(1, args.batched_steps)
    pools = [EventPool(max_ev) for _ in range(steps)]
    warm = EventPool(max_ev)
    rec = ctypes.c_int(0)

    def call_profiled(pool):
        st = lib.pbit_sort_lists_profiled(
            d["heads"].data_ptr(), d["offsets"].data_ptr(), L, total, d["next"].data_ptr(),
            next_out.data_ptr(), d["keys"].data_ptr(), M, K, 0, new_heads.data_ptr(),
            status.data_ptr(), ws.data_ptr(), ws_bytes, sh, pool.ptr(), pool.ids_ptr(), max_ev,
            ctypes.byref(rec))
        if st != 0:
            raise RuntimeError("batched sort failed: " + _lib.status_string(st))
        return rec.value

    def call_plain_api():
        st = lib.pbit_sort_lists(
            d["heads"].data_ptr(), d["offsets"].data_ptr(), L, total, d["next"].data_ptr(),
            next_out.data_ptr(), d["keys"].data_ptr(), M, K, 0, new_heads.data_ptr(),
            status.data_ptr(), ws.data_ptr(), ws_bytes, sh)
        if st != 0:
            raise RuntimeError("batched sort failed: " + _lib.status_string(st))

    call_profiled(warm)
    torch.cuda.synchronize()
    if int(status.item()) != 0:
        raise RuntimeError("batched device status %d" % int(status.item()))
    counts = []
    t0 = time.perf_counter()
    for k in range(steps):
        counts.append(call_profiled(pools[k]))
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3 / steps
    stage_ms, launches, lat = stage_table(lib, pools, counts)

    # the same call captured once in a HIP graph and replayed
    graph_ms = None
    graph_ok = None
    try:
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            with torch.cuda.graph(g, stream=side):
                st = lib.pbit_sort_lists(
                    d["heads"].data_ptr(), d["offsets"].data_ptr(), L, total,
                    d["next"].data_ptr(), next_out.data_ptr(), d["keys"].data_ptr(), M, K, 0,
                    new_heads.data_ptr(), status.data_ptr(), ws.data_ptr(), ws_bytes,
                    int(torch.cuda.current_stream().cuda_stream))
        stream.wait_stream(side)
        ref = next_out.clone()
        g.replay()
        torch.cuda.synchronize()
        graph_ok = bool(torch.equal(next_out, ref)) and st == 0
        t0 = time.perf_counter()
        for _ in range(steps):
            g.replay()
        torch.cuda.synchronize()
        graph_ms = (time.perf_counter() - t0) * 1e3 / steps
        del g
    except Exception as exc:  # graph capture is optional for the measurement
        graph_ok = "unavailable: %s" % exc

    # sampled lists against the oracle (the longest and seven seeded picks)
    import oracle
    offs_h = d["offsets_host"]
    heads_h = d["heads_host"]
    picks = [int(np.argmax(lengths))] + [int(x) for x in inputs.rng_for(4003).choice(L, 7, replace=False)]
    nh_h = new_heads.cpu().numpy().view(np.uint32)
    oracle_ok = int(status.item()) == 0

    def local(x, lo):
        x = x.astype(np.int64)
        return np.where(x == 0xFFFFFFFF, 0xFFFFFFFF, x - lo).astype(np.uint32)

    for l in picks:
        lo, hi_ = int(offs_h[l]), int(offs_h[l + 1])
        eh, en = oracle.sort_list(int(heads_h[l]) - lo,
                                  local(d["next"][lo:hi_].cpu().numpy().view(np.uint32), lo),
                                  d["keys"][lo:hi_].cpu().numpy().view(np.uint32), 32, 8)
        oracle_ok = oracle_ok and int(nh_h[l]) - lo == eh and bool(np.array_equal(
            local(next_out[lo:hi_].cpu().numpy().view(np.uint32), lo), en))

    out = {
        "workload": "20000 lists, lengths log-uniform in [16, 2^%d], %d nodes, uint32 keys, "
                    "random layout per slab, K=%d (tuned), short-list cutoff %d (tuned)"
                    % (hi, total, Keff, cutoff),
        "K": Keff, "cutoff": cutoff,
        "oracle_sampled_lists": len(picks),
        "oracle_equal": oracle_ok,
        "lists": L, "nodes": total,
        "batched_ms": round(wall_ms, 3),
        "batched_Mnodes_s": round(total / (wall_ms * 1e-3) / 1e6, 1),
        "batched_p50_ms": round(statistics.median(lat), 3),
        "graph_replay_ms": None if graph_ms is None else round(graph_ms, 3),
        "graph_replay_equal": graph_ok,
        "stages_ms": {k: round(v, 3) for k, v in sorted(stage_ms.items(), key=lambda x: -x[1])},
    }

    if compare:
        # single-list calls over the same lists (slab-local indices), one stream
        maxlen = int(lengths.max())
        pws_bytes = _lib.workspace_bytes(maxlen, M, K)
        pws = torch.empty(pws_bytes, dtype=torch.uint8, device=dev)
        pout = torch.empty_like(d["next_local"])
        pres = torch.zeros(2 * L, dtype=torch.int32, device=dev)
        offs = d["offsets_host"]
        heads_h = d["heads_host"]
        nl = d["next_local"].data_ptr()
        po = pout.data_ptr()
        kp = d["keys"].data_ptr()
        rp = pres.data_ptr()
        wp = pws.data_ptr()
        fn = lib.pbit_sort_list_async
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for l in range(L):
            lo = int(offs[l])
            ln = int(offs[l + 1]) - lo
            st = fn(int(heads_h[l]) - lo, nl + 4 * lo, po + 4 * lo, kp + 4 * lo, ln, M, K, 0,
                    rp + 8 * l, wp, pws_bytes, sh)
            if st != 0:
                raise RuntimeError("plain call failed for list %d" % l)
        torch.cuda.synchronize()
        plain_ms = (time.perf_counter() - t0) * 1e3
        # every list identical alone and in the batch
        lens_t = torch.from_numpy(lengths).to(dev)
        base = torch.repeat_interleave(d["offsets"][:-1], lens_t).to(torch.int32)
        glob = torch.where(pout == -1, pout, pout + base)
        same_next = bool(torch.equal(glob, next_out))
        ph = pres.view(L, 2)
        same_heads = bool(torch.equal(ph[:, 0] + d["offsets"][:-1].to(torch.int32), new_heads))
        ok_status = bool(torch.all(ph[:, 1] == 0).item())
        out.update({
            "plain_calls_ms": round(plain_ms, 1),
            "plain_Mnodes_s": round(total / (plain_ms * 1e-3) / 1e6, 1),
            "speedup_batched_vs_plain": round(plain_ms / wall_ms, 2),
            "identical_alone_and_batched": same_next and same_heads and ok_status,
        })
        del pws, pout, pres
    for p in pools + [warm]:
        p.close()
    del ws, next_out, d
    torch.cuda.empty_cache()
    return out


def run_served(args, torch, np, inputs):
    """Poisson request stream, key widths {8,16,32,64}, lengths log-uniform:
    saturated throughput X first (all requests at t = 0), then open loop at
    0.7 X offered node rate with continuous batching, and the FIFO baseline
    (one single-list call per request, one stream) at the same offered load."""
    from paper_cs_0511020_amd.serve import (GpuExecutor, PlainExecutor, SortServer,
                                            make_requests_device)
    full = args.served == "full"
    count, hi = (2000, 24) if full else (300, 20)
    reqs = make_requests_device(count, seed=5001, lo_log2=10, hi_log2=hi, keep_order=True)

    def all_relinked():
        """Every request's result has the properties of its stable sort."""
        return all(r.status == 0 and relinked_ok(torch, r.new_head, r.out, r.keys, r.order)
                   for r in reqs)
    torch.cuda.synchronize()
    free = torch.cuda.mem_get_info()[0]
    budget = int(free * 0.6)
    mean_len = float(np.mean([r.n for r in reqs]))

    def reset(arrivals):
        for r, a in zip(reqs, arrivals):
            r.arrival = float(a)
            r.done = r.admitted = -1.0
            r.batch = -1
            r.new_head = -1

    def summary(st):
        d = st.as_dict()
        return {k: (round(v, 3) if isinstance(v, float) else v) for k, v in d.items()}

    # warm the allocator and kernels once
    SortServer(GpuExecutor(streams=2), slots=64, budget_bytes=budget).run(reqs[: min(40, count)])
    reset(np.zeros(count))
    sat = SortServer(GpuExecutor(streams=2), slots=64, budget_bytes=budget).run(reqs)
    X = sat.throughput_mnodes_s * 1e6
    checked = 1
    ok = all_relinked()
    # a few requests of every key width against the oracle
    import oracle
    dt = {8: np.uint8, 16: np.uint16, 32: np.uint32, 64: np.uint64}
    srng = inputs.rng_for(5003)
    sample = []
    for M in (8, 16, 32, 64):
        cand = [r for r in reqs if r.M == M and r.n <= (1 << 18)]
        sample += [cand[int(i)] for i in srng.choice(len(cand), min(2, len(cand)),
                                                      replace=False)]
    for r in sample:
        eh, en = oracle.sort_list(r.head, r.next.cpu().numpy().view(np.uint32),
                                  r.keys.cpu().numpy().view(dt[r.M]), r.M, 4 if r.M == 8 else 8)
        ok = ok and eh == r.new_head and bool(
            np.array_equal(r.out.cpu().numpy().view(np.uint32), en))
    loads = {}
    for frac in ((0.5, 0.7, 0.9) if full else (0.7,)):
        rng = inputs.rng_for(5002)
        lam = frac * X / mean_len
        arrivals = np.cumsum(rng.exponential(1.0 / lam, size=count))
        reset(arrivals)
        opened = SortServer(GpuExecutor(streams=2), slots=64, budget_bytes=budget).run(reqs)
        ok = ok and all_relinked()
        reset(arrivals)
        fifo = SortServer(PlainExecutor(), slots=1, budget_bytes=budget).run(reqs)
        ok = ok and all_relinked()
        checked += 2
        loads[frac] = (summary(opened), summary(fifo))
    opened_s, fifo_s = loads[0.7]
    out = {
        "workload": "%d requests, lengths log-uniform in [2^10, 2^%d], key widths uniform over "
                    "{8,16,32,64}, uniform keys, device-resident, Poisson arrivals at %s of the "
                    "saturated rate" % (count, hi, "0.5/0.7/0.9" if full else "0.7"),
        "nodes": int(sum(r.n for r in reqs)),
        "saturated": summary(sat),
        "offered_mnodes_s": round(0.7 * X / 1e6, 1),
        "batched_open_loop": opened_s,
        "fifo_plain_open_loop": fifo_s,
        "by_load": {"%.1f" % f: {"offered_mnodes_s": round(f * X / 1e6, 1), "batched": b,
                                 "fifo_plain": p} for f, (b, p) in loads.items()},
        "all_ok": ok,
        "checks": "after each of the %d runs every request's result is checked on the device "
                  "for the properties of its stable sort (one path from the head over all "
                  "nodes, (key, input position) increasing along every link); %d requests "
                  "(two per key width, up to 2^18 nodes) are compared with the oracle"
                  % (checked, len(sample)),
    }
    del reqs
    torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: measures one GPU only (the sort runs on a single device; no "
              "multi-GPU path exists); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_cs_0511020_amd import _lib, bytemodel, inputs
    from paper_cs_0511020_amd.hipevents import EventPool

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    lib = _lib.load()

    r = run_plain(args, lib, torch, np, inputs, bytemodel, EventPool)
    torch.cuda.empty_cache()

    extras = None
    if not args.no_extras:
        extras = run_extras(args, lib, torch, np, inputs, bytemodel)
        torch.cuda.empty_cache()

    c3 = None
    if not args.no_c3:
        c3 = run_c3(args, lib, torch, np, bytemodel)

    batched = None
    if args.batched != "none":
        batched = run_batched(args, lib, torch, np, inputs, EventPool)
    served = None
    if args.served != "none":
        served = run_served(args, torch, np, inputs)

    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.int32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        cn = min(args.cpu_sample_n, args.n)
        seed = {"uniform": 2001, "zipf": 2002, "distinct8": 2003}[args.dist]
        crng = inputs.rng_for(seed + 100)
        cnxt, chead, _ = inputs.random_list(cn, crng)
        ckeys = inputs.keys_by_distribution(args.dist, cn, crng)
        oracle.build(force=False)
        if args.M == 64:
            ckeys = inputs.uniform_keys(cn, 64, crng)
        tc0 = time.perf_counter()
        ch, cout = oracle.sort_list(chead, cnxt, ckeys, args.M, r["Keff"])
        tc1 = time.perf_counter()
        # (ii) the same oracle with the groups below its top levels on every core
        threads = args.cpu_threads or (os.cpu_count() or 1)
        tp0 = time.perf_counter()
        ph, pout = oracle.sort_list_threads(chead, cnxt, ckeys, args.M, r["Keff"],
                                            threads=threads)
        tp1 = time.perf_counter()
        # (iii) context: walk the list, stable-sort its keys (numpy), relink
        tw0 = time.perf_counter()
        corder = oracle.list_order(chead, cnxt)
        sorted_nodes = corder[np.argsort(ckeys[corder], kind="stable")]
        wout = np.empty_like(cnxt)
        wout[sorted_nodes[:-1]] = sorted_nodes[1:]
        wout[sorted_nodes[-1]] = 0xFFFFFFFF
        tw1 = time.perf_counter()
        agree = (ch == ph == int(sorted_nodes[0]) and bool(np.array_equal(cout, pout))
                 and bool(np.array_equal(cout, wout)))
        cpu_model = ""
        try:
            with open("/proc/cpuinfo") as f:
                for line in f:
                    if line.startswith("model name"):
                        cpu_model = line.split(":", 1)[1].strip()
                        break
        except OSError:
            pass
        cpu = {"value": round(cn / (tc1 - tc0) / 1e6, 3), "unit": "Mnodes/s", "cores": 1,
               "kind": "oracle",
               "sample": "one sort of a %d-node list, same key distribution and layout recipe, "
                         "K=%d, single-threaded C oracle, %.1f s" % (cn, r["Keff"], tc1 - tc0),
               "nproc": os.cpu_count(), "cpu_model": cpu_model,
               "all_cores": {"value": round(cn / (tp1 - tp0) / 1e6, 3), "unit": "Mnodes/s",
                             "cores": threads, "kind": "oracle",
                             "sample": "the same list; top pattern levels split on one thread, "
                                       "the groups below sorted on %d threads, %.1f s"
                                       % (threads, tp1 - tp0)},
               "walk_stable_sort_relink": {"value": round(cn / (tw1 - tw0) / 1e6, 3),
                                           "unit": "Mnodes/s", "cores": 1, "kind": "context",
                                           "sample": "the same list walked, its keys stably "
                                                     "sorted by numpy, relinked, %.1f s"
                                                     % (tw1 - tw0)},
               "variants_agree": agree}

    out = {
        "metric": METRIC,
        "value": round(r["value"], 2),
        "unit": "Mnodes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["wall_ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u%d" % args.M,
        "data": "synthetic",
        "config": {"workload": "single list n=%d uint%d keys (%s), random-permutation next[] "
                               "layout, K=%d, plain per-list launch"
                               % (args.n, args.M, args.dist if args.M == 32 else "uniform",
                                  r["Keff"]),
                   "n": args.n, "M": args.M, "K": r["Keff"], "dist": args.dist, "mode": "plain"},
        "timing": "value and ms_per_step: warm, %d back-to-back sorts of the same resident "
                  "input (out of place) after %d warm-up sorts, wall clock around them; "
                  "latency_ms from HIP events per sort; cold_latency_ms: each sort after a "
                  "1 GiB write that flushes L2 and the last-level cache" % (args.steps,
                                                                            args.warmup),
        "roofline": r["roofline"],
        "roofline_second": r["roofline_second"],
        "cpu_baseline": cpu,
        "latency_ms": {"p50": round(r["p50"], 4), "p99": round(r["p99"], 4)},
        "graph_replay_ms_per_step": (round(r["graph_ms"], 4) if r["graph_ms"] is not None
                                     else None),
        "cold_latency_ms": r["cold"],
        "path_roofline": {"bytes_per_node": r["path_bpn"], "frac_at_p50": round(r["path_frac"], 4)},
        "stages_ms": {k: round(v, 4) for k, v in sorted(r["stage_ms"].items(), key=lambda x: -x[1])},
        "stage_launches": r["launches"],
        "correct": r["correct"],
        "other_k": r["other_k"],
        "c3_u64_payload": c3,
        "extras": extras,
        "batched": batched,
        "served": served,
        "source_hash": r["src_hash"],
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
