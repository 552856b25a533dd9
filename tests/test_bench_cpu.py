"""bench.py's command-line contract that needs no GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_help_lists_the_options():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0
    for opt in ("--gpus", "--steps", "--warmup", "--K", "--M", "--dist", "--batched", "--served",
                "--no-cold", "--no-graph", "--no-extras"):
        assert opt in r.stdout


def test_device_property_check_on_host_tensors():
    """The benchmark's result check (run on the GPU there) accepts the stable
    sort and rejects a relinked list with two links swapped, with equal keys
    out of input order, or with a cycle cut off."""
    import numpy as np
    import torch
    import bench
    from paper_cs_0511020_amd import inputs
    rng = inputs.rng_for(77)
    n = 5000
    nxt, head, order = inputs.random_list(n, rng)
    keys = rng.integers(0, 50, size=n).astype(np.uint32)
    srt = order[np.argsort(keys[order], kind="stable")]
    out = np.full(n, 0xFFFFFFFF, dtype=np.uint32)
    out[srt[:-1]] = srt[1:]
    t = lambda a: torch.from_numpy(a.view(np.int32).copy())
    kt = torch.from_numpy(keys.view(np.int32))
    ot = torch.from_numpy(order.astype(np.int32))
    assert bench.relinked_ok(torch, int(srt[0]), t(out), kt, ot)
    bad = out.copy()
    bad[srt[10]], bad[srt[20]] = out[srt[20]], out[srt[10]]
    assert not bench.relinked_ok(torch, int(srt[0]), t(bad), kt, ot)
    # two equal keys in reverse input order
    i = int(np.nonzero(keys[srt[1:]] == keys[srt[:-1]])[0][0])
    rev = srt.copy()
    rev[i], rev[i + 1] = srt[i + 1], srt[i]
    bad = np.full(n, 0xFFFFFFFF, dtype=np.uint32)
    bad[rev[:-1]] = rev[1:]
    assert not bench.relinked_ok(torch, int(rev[0]), t(bad), kt, ot)
    # the last three nodes cut off into a cycle
    bad = out.copy()
    bad[srt[-4]] = 0xFFFFFFFF
    bad[srt[-1]] = srt[-3]
    assert not bench.relinked_ok(torch, int(srt[0]), t(bad), kt, ot)
    # 64-bit keys compare unsigned
    k64 = np.array([1, 2 ** 63, 5], dtype=np.uint64)
    nx = np.array([2, 0xFFFFFFFF, 1], dtype=np.uint32)
    assert bench.relinked_ok(torch, 0, t(nx), torch.from_numpy(k64.view(np.int64)),
                             torch.tensor([0, 1, 2], dtype=torch.int32))
