#!/usr/bin/env python3
"""Benchmark of the MI355X Pbit list sort.

One step = one whole sort (pack, list ranking, every digit pass, relink) of a
single list of n = 2^24 nodes with uint32 keys and a random-permutation
next[] layout, inputs resident in HBM.  The sort reads next_in and writes
next_out (out of place, same traffic as in place), so every step sorts the
same input.  Each kernel stage is bracketed by HIP events on the stream the
library launches on; the dominant stage's algorithmic bytes per launch over
its mean launch time give the roofline figure.

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
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
    ap.add_argument("--K", type=int, default=8, help="pattern bits (4 or 8; 0 = library choice)")
    ap.add_argument("--dist", default="uniform", choices=["uniform", "zipf", "distinct8"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-n", type=int, default=1 << 24,
                    help="nodes in the list the CPU oracle sorts once")
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


def load_traffic(kernel: str, src_hash: str):
    """HBM bytes per launch from committed rocprofv3 counter summaries, if they
    were taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % kernel)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_hash") != src_hash:
        return None
    return d.get("hbm_bytes_per_launch")


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only (the sort runs on a single "
              "device; no multi-GPU path exists); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import ctypes

    import numpy as np
    import torch

    from paper_cs_0511020_amd import _lib, bytemodel, inputs
    from paper_cs_0511020_amd.hipevents import EventPool

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    lib = _lib.load()
    dev = torch.device("cuda:0")
    n, K, M = args.n, args.K, 32
    Keff = K if K else 8
    passes = M // Keff
    seed = {"uniform": 2001, "zipf": 2002, "distinct8": 2003}[args.dist]

    rng = inputs.rng_for(seed)
    nxt, head, order = inputs.random_list(n, rng)
    keys = inputs.c2_keys(args.dist, n, rng)
    next_in = torch.from_numpy(nxt.view(np.int32)).to(dev)
    keys_d = torch.from_numpy(keys.view(np.int32)).to(dev)
    next_out = torch.empty_like(next_in)
    ws_bytes = _lib.workspace_bytes(n, M, K)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    result = torch.zeros(2, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    sh = int(stream.cuda_stream)

    max_ev = 64
    pools = [EventPool(max_ev) for _ in range(args.steps)]
    warm_pool = EventPool(max_ev)
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
        run(warm_pool)
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
    t1 = time.perf_counter()
    wall_ms = (t1 - t0) * 1e3 / args.steps

    # per-step latency (first to last event) and per-stage times
    stage_names = {}
    per_stage = {}
    launches = {}
    lat = []
    for k in range(args.steps):
        p, c = pools[k], counts[k]
        lat.append(p.elapsed_ms(0, c - 1))
        step_tot, step_cnt = {}, {}
        for i in range(c - 1):
            sid = p.ids[i]
            name = stage_names.setdefault(sid, lib.pbit_stage_name(sid).decode())
            step_tot[name] = step_tot.get(name, 0.0) + p.elapsed_ms(i, i + 1)
            step_cnt[name] = step_cnt.get(name, 0) + 1
        for name, v in step_tot.items():
            per_stage.setdefault(name, []).append(v)
            launches[name] = step_cnt[name]
    stage_ms = {k: statistics.mean(v) for k, v in per_stage.items()}
    lat_sorted = sorted(lat)
    p50 = statistics.median(lat_sorted)
    p99 = lat_sorted[min(len(lat_sorted) - 1, int(round(0.99 * (len(lat_sorted) - 1))))]

    # correctness of the timed configuration against the definition (cheap)
    got = next_out.cpu().numpy().view(np.uint32)
    exp_order = order[np.argsort(keys[order], kind="stable")]
    ok = (h0 == int(exp_order[0])) and bool(np.array_equal(got[exp_order[:-1]], exp_order[1:]))

    w = 4
    executed_passes = launches.get("digit_pass", passes)
    value = n / (wall_ms * 1e-3) / 1e6
    path_bytes = bytemodel.path_bytes_per_node(w, passes) * n
    path_frac = path_bytes / (p50 * 1e-3) / 1e9 / bytemodel.MI355X_HBM_PEAK_GBS

    # dominant kernel: largest share of the step
    roof_candidates = {k: v for k, v in stage_ms.items()
                       if k in ("pack", "walk0", "unchain", "digit_pass", "relink")}
    dom = max(roof_candidates, key=roof_candidates.get)
    dom_launch_ms = stage_ms[dom] / launches[dom]
    if dom == "digit_pass":
        # mean bytes per launch over the executed passes (the last writes no keys)
        per_node = (bytemodel.kernel_bytes_per_node(dom, w) * (executed_passes - 1)
                    + bytemodel.kernel_bytes_per_node(dom, w, last_pass=True)) / executed_passes
    else:
        per_node = bytemodel.kernel_bytes_per_node(dom, w)
    dom_bytes = per_node * n
    achieved = dom_bytes / (dom_launch_ms * 1e-3) / 1e9
    src_hash = source_hash()
    roofline = {
        "bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
        "peak": bytemodel.MI355X_HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / bytemodel.MI355X_HBM_PEAK_GBS, 4),
        "traffic": load_traffic(dom, src_hash),
        "algorithmic_bytes_per_launch": int(dom_bytes),
        "launch_ms": round(dom_launch_ms, 5),
    }

    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.int32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        cn = min(args.cpu_sample_n, n)
        crng = inputs.rng_for(seed + 100)
        cnxt, chead, _ = inputs.random_list(cn, crng)
        ckeys = inputs.c2_keys(args.dist, cn, crng)
        oracle.build(force=False)
        tc0 = time.perf_counter()
        hh, _ = oracle.sort_list(chead, cnxt, ckeys, M, Keff)
        tc1 = time.perf_counter()
        cpu = {"value": round(cn / (tc1 - tc0) / 1e6, 3), "unit": "Mnodes/s", "cores": 1,
               "kind": "oracle",
               "sample": "one sort of a %d-node list, same key distribution and layout recipe, "
                         "K=%d, single-threaded C oracle, %.1f s" % (cn, Keff, tc1 - tc0)}

    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "Mnodes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall_ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "single list n=2^24 uint32 keys (%s), random-permutation next[] "
                               "layout, K=%d, plain per-list launch" % (args.dist, Keff),
                   "n": n, "M": M, "K": Keff, "dist": args.dist, "mode": "plain"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "latency_ms": {"p50": round(p50, 4), "p99": round(p99, 4)},
        "path_roofline": {"bytes_per_node": bytemodel.path_bytes_per_node(w, passes),
                          "frac_at_p50": round(path_frac, 4)},
        "stages_ms": {k: round(v, 4) for k, v in sorted(stage_ms.items(), key=lambda x: -x[1])},
        "stage_launches": launches,
        "correct": ok,
        "source_hash": src_hash,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
