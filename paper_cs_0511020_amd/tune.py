"""Device autotuner: pattern width K and the short-list cutoff.

The paper weighs the pattern length (Sec. 10): a longer pattern means fewer
passes over the list but more groups per pass.  On the GPU a pass moves every
(key, node) pair once, so fewer passes usually win, but a wider pattern also
means larger per-tile tables and, for many lists, larger per-list digit
tables.  The cutoff (Sec. 9 weighs methods by list length) decides which
lists are sorted by one workgroup in on-chip memory and which take the
device-wide path: the short lists of a batch, and a single list of at most
that many nodes.  This module times the library on the device for each
candidate and writes the fastest choices:

* ``pbit_tuning.h`` -- the library's built-in table (entries
  {kind, M, n_max, K, cutoff}; kind 0 one list, 1 many lists), compiled into
  libpbit by the next build;
* ``tuning.json`` -- the same choices with every timing behind them.

Workloads: single lists of 2^10, 2^11, 2^12, 2^16, 2^20 and 2^24 nodes,
uniform keys, random layout (the cutoff is timed on the lists of at most
4096 nodes, the largest one workgroup takes); batches of lists with lengths
log-uniform in [16, 2^16] (the batched benchmark's distribution) at about
2^20, 2^24 and 2^27 nodes.
Every input is generated on the device from fixed seeds.  Times are medians
of HIP-event intervals around the sort on its stream.

Run on a GPU:  python -m paper_cs_0511020_amd.tune --out-dir DIR [--quick]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import time

from . import _lib

NMAX = 0xFFFFFFFF
SINGLE_SIZES = (1 << 10, 1 << 11, 1 << 12, 1 << 16, 1 << 20, 1 << 24)
SHORT_MAX = 4096  # the longest single list one workgroup sorts
BATCH_NODES = (1 << 20, 1 << 24, 1 << 27)
CUTOFFS = (1024, 2048, 4096)
WIDTHS = (8, 16, 32, 64)


def k_candidates(M: int):
    return (2, 4, 8) if M == 8 else (4, 8)


def _keys(torch, n, M, g, dev):
    if M == 8:
        return torch.randint(0, 256, (n,), generator=g, device=dev, dtype=torch.uint8)
    if M == 16:
        return torch.randint(-(1 << 15), 1 << 15, (n,), generator=g, device=dev,
                             dtype=torch.int16)
    if M == 32:
        return torch.randint(-(1 << 31), 1 << 31, (n,), generator=g, device=dev,
                             dtype=torch.int32)
    hi = torch.randint(-(1 << 31), 1 << 31, (n,), generator=g, device=dev, dtype=torch.int64)
    lo = torch.randint(0, 1 << 32, (n,), generator=g, device=dev, dtype=torch.int64)
    return (hi << 32) | lo


def _median_ms(torch, fn, reps: int, warm: int = 2) -> float:
    stream = torch.cuda.current_stream()
    for _ in range(warm):
        fn()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * reps)]
    for k in range(reps):
        ev[2 * k].record(stream)
        fn()
        ev[2 * k + 1].record(stream)
    torch.cuda.synchronize()
    return statistics.median(ev[2 * k].elapsed_time(ev[2 * k + 1]) for k in range(reps))


def time_single(torch, M: int, n: int, reps: int):
    """{(K, cutoff): ms} for one list of n nodes with uniform M-bit keys.  The
    cutoff only matters up to SHORT_MAX nodes; above, the largest one is
    recorded (it keeps neighbouring table entries mergeable)."""
    dev = torch.device("cuda")
    g = torch.Generator(device=dev)
    g.manual_seed(7000 + M + n)
    order = torch.randperm(n, generator=g, device=dev, dtype=torch.int64)
    nxt = torch.full((n,), -1, dtype=torch.int32, device=dev)
    nxt[order[:-1]] = order[1:].to(torch.int32)
    head = int(order[0].item())
    del order
    keys = _keys(torch, n, M, g, dev)
    out = torch.empty_like(nxt)
    res = torch.zeros(2, dtype=torch.int32, device=dev)
    times = {}
    cuts = CUTOFFS if n <= SHORT_MAX else (CUTOFFS[-1],)
    try:
        for K in k_candidates(M):
            wsb = _lib.workspace_bytes(n, M, K)
            ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
            for cut in cuts:
                # an entry for exactly this size wins over any wider one
                if _lib.tune_set(0, M, n, K, cut) != _lib.OK:
                    raise RuntimeError("tuning entry rejected")

                def run():
                    st = _lib.sort_list_async(head, nxt, out, keys, n, M, K, 0, res, ws, wsb)
                    if st != _lib.OK:
                        raise RuntimeError(_lib.status_string(st))

                times[(K, cut)] = _median_ms(torch, run, reps)
                if int(res[1].item()) != 0:
                    raise RuntimeError("device status %d" % int(res[1].item()))
            del ws
    finally:
        _lib.tune_reset()
    return times


TIE = 0.02  # timings this close are treated as equal


def pick_single(times):
    """The (K, cutoff) of a single-list timing: the fastest, except that
    choices within TIE of it count as equal and the largest cutoff among them
    wins.  At a size below two cutoffs both send the list down the same path,
    so only noise tells them apart; the larger one keeps the next sizes on
    the one-workgroup path too."""
    best = min(times.values())
    near = [kc for kc, v in times.items() if v <= best * (1 + TIE)]
    return max(near, key=lambda kc: (kc[1], -times[kc]))


def _parse_ms(ms):
    import re
    out = {}
    for key, v in ms.items():
        m = re.fullmatch(r"K(\d+)_cut(\d+)", key)
        out[(int(m.group(1)), int(m.group(2)))] = float(v)
    return out


def entries_from_record(record):
    """Table entries from a saved timing record (tuning.json)."""
    entries = []
    for kind, rows, size_key, pick in ((0, record["single"], "n", pick_single),
                                       (1, record["batched"], "nodes",
                                        lambda t: min(t, key=t.get))):
        for M in WIDTHS:
            best = []
            for r in rows:
                if r["M"] == M:
                    r["K"], r["cutoff"] = pick(_parse_ms(r["ms"]))
                    best.append((r[size_key], r["K"], r["cutoff"]))
            if best:
                entries += entries_from_best(kind, M, best)
    return entries


def batch_lengths(total: int, seed: int):
    """Lengths log-uniform in [16, 2^16] adding up to about `total` nodes."""
    import numpy as np
    rng = np.random.Generator(np.random.PCG64(seed))
    mean = (65536 - 16) / math.log(65536 / 16)
    count = max(1, int(round(total / mean)))
    u = rng.random(count)
    return np.clip(np.floor(2.0 ** (4 + 12 * u)).astype(np.int64), 16, 65536)


def time_batched(torch, M: int, total: int, reps: int):
    """{(K, cutoff): ms} for a batch of about `total` nodes."""
    import numpy as np
    from .inputs import slab_lists_device
    dev = torch.device("cuda")
    lengths = batch_lengths(total, 8000 + M + total % 997)
    d = slab_lists_device(lengths, seed=8100 + M, M=M)
    L = int(lengths.shape[0])
    n = int(d["offsets_host"][-1])
    out = torch.empty_like(d["next"])
    heads = torch.empty(L, dtype=torch.int32, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    times = {}
    try:
        for K in k_candidates(M):
            for cut in CUTOFFS:
                # an entry for exactly this size wins over any wider one
                if _lib.tune_set(1, M, n, K, cut) != _lib.OK:
                    raise RuntimeError("tuning entry rejected")
                wsb = _lib.lists_workspace_bytes(n, L, M, K)
                ws = torch.empty(wsb, dtype=torch.uint8, device=dev)

                def run():
                    st = _lib.sort_lists(d["heads"], d["offsets"], L, n, d["next"], out,
                                         d["keys"], M, K, 0, heads, status, ws, wsb)
                    if st != _lib.OK:
                        raise RuntimeError(_lib.status_string(st))

                times[(K, cut)] = _median_ms(torch, run, reps)
                if int(status.item()) != 0:
                    raise RuntimeError("device status %d" % int(status.item()))
                del ws
    finally:
        _lib.tune_reset()
    del d, out
    torch.cuda.empty_cache()
    return times, n, L


def entries_from_best(kind: int, M: int, best):
    """best: [(n, K, cutoff)] by increasing n -> table entries, each
    covering sizes up to the geometric midpoint to the next measured size
    (the last one up to every size), neighbours with equal choices merged."""
    best = sorted(best)
    out = []
    for i, (n, K, cut) in enumerate(best):
        n_max = NMAX if i + 1 == len(best) else int(math.sqrt(n * best[i + 1][0]))
        if out and out[-1]["K"] == K and out[-1]["cutoff"] == cut:
            out[-1]["n_max"] = n_max
        else:
            out.append({"kind": kind, "M": M, "n_max": n_max, "K": K, "cutoff": cut})
    return out


def render_header(entries) -> str:
    lines = [
        "// Built-in tuning table of libpbit (included once, by pbit_capi.hip).",
        "// Entries: {kind (0 one list, 1 many lists), key bits M, largest node count",
        "// n_max, pattern bits K, short-list cutoff}.  Written by",
        "// paper_cs_0511020_amd/tune.py from device measurements (tuning.json beside",
        "// the package holds the timings).",
        "static const TuneEntry kBuiltinTuning[] = {",
    ]
    for e in entries:
        lines.append("    {%d, %d, 0x%Xull, %d, %d}," % (e["kind"], e["M"], e["n_max"], e["K"],
                                                          e["cutoff"]))
    lines.append("};")
    return "\n".join(lines) + "\n"


def parse_header(text: str):
    """Entries of a pbit_tuning.h (for checks of the committed table)."""
    import re
    out = []
    for m in re.finditer(r"\{(\d+), (\d+), 0x([0-9A-F]+)ull, (\d+), (\d+)\}", text):
        out.append({"kind": int(m.group(1)), "M": int(m.group(2)),
                    "n_max": int(m.group(3), 16), "K": int(m.group(4)),
                    "cutoff": int(m.group(5))})
    return out


def run(out_dir: str, quick: bool = False):
    import torch
    _lib.load()
    _lib.tune_reset()
    reps = 5 if quick else 10
    single_sizes = SINGLE_SIZES[:5] if quick else SINGLE_SIZES
    batch_nodes = BATCH_NODES[:2] if quick else BATCH_NODES
    record = {"single": [], "batched": [], "device": torch.cuda.get_device_name(0),
              "when": time.strftime("%Y-%m-%d %H:%M:%S")}
    entries = []
    for M in WIDTHS:
        best = []
        for n in single_sizes:
            t = time_single(torch, M, n, reps)
            K, cut = pick_single(t)
            best.append((n, K, cut))
            record["single"].append({"M": M, "n": n,
                                     "ms": {"K%d_cut%d" % kc: round(v, 4) for kc, v in t.items()},
                                     "K": K, "cutoff": cut})
            print("single M=%d n=%d %s -> K=%d cutoff=%d" % (M, n, t, K, cut), flush=True)
        entries += entries_from_best(0, M, best)
    for M in WIDTHS:
        best = []
        for total in batch_nodes:
            t, n, L = time_batched(torch, M, total, max(3, reps // 2))
            K, cut = min(t, key=t.get)
            best.append((n, K, cut))
            record["batched"].append({"M": M, "nodes": n, "lists": L,
                                      "ms": {"K%d_cut%d" % kc: round(v, 4)
                                             for kc, v in t.items()},
                                      "K": K, "cutoff": cut})
            print("batched M=%d n=%d L=%d %s -> K=%d cutoff=%d" % (M, n, L, t, K, cut),
                  flush=True)
        entries += entries_from_best(1, M, best)
    record["entries"] = entries
    os.makedirs(out_dir, exist_ok=True)
    with open(os.path.join(out_dir, "pbit_tuning.h"), "w") as f:
        f.write(render_header(entries))
    with open(os.path.join(out_dir, "tuning.json"), "w") as f:
        json.dump(record, f, indent=1)
    return record


def write_from_record(json_path: str, out_dir: str):
    """Rewrite pbit_tuning.h from a saved record, without a GPU."""
    with open(json_path) as f:
        record = json.load(f)
    entries = entries_from_record(record)
    record["entries"] = entries
    os.makedirs(out_dir, exist_ok=True)
    with open(os.path.join(out_dir, "pbit_tuning.h"), "w") as f:
        f.write(render_header(entries))
    with open(os.path.join(out_dir, "tuning.json"), "w") as f:
        json.dump(record, f, indent=1)
    return entries


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--out-dir", default="tuning_out")
    ap.add_argument("--quick", action="store_true", help="fewer sizes and repetitions")
    ap.add_argument("--from-json", help="rebuild the table from a saved tuning.json instead")
    args = ap.parse_args()
    if args.from_json:
        write_from_record(args.from_json, args.out_dir)
    else:
        run(args.out_dir, args.quick)


if __name__ == "__main__":
    main()
