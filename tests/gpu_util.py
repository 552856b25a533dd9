"""Helpers shared by the GPU tests: move seeded numpy inputs to the device,
run the library, and check results against the oracle or the definition."""
import numpy as np

NIL = 0xFFFFFFFF
SIGNED_VIEW = {np.dtype(np.uint8): np.uint8, np.dtype(np.uint16): np.int16,
               np.dtype(np.uint32): np.int32, np.dtype(np.uint64): np.int64}


def to_dev(arr, torch):
    arr = np.ascontiguousarray(arr)
    view = SIGNED_VIEW.get(arr.dtype, None)
    if view is not None:
        arr = arr.view(view)
    return torch.from_numpy(arr).to("cuda")


def from_dev(t, dtype=np.uint32):
    return t.cpu().numpy().view(dtype)


FLOAT_VIEW = {np.dtype(np.uint16): np.float16, np.dtype(np.uint32): np.float32,
              np.dtype(np.uint64): np.float64}


def keys_to_dev(keys, flags, torch):
    """Device keys; with the floating-point flag (4) the bit patterns are
    handed over as the float dtype of the same width, which is what selects
    floating-point order in the binding."""
    keys = np.ascontiguousarray(keys)
    if flags & 4:
        return torch.from_numpy(keys.view(FLOAT_VIEW[keys.dtype])).to("cuda")
    return to_dev(keys, torch)


def gpu_sort(head, nxt, keys, K, flags=0, inplace=True, sorter=None, shared=False):
    import torch
    from paper_cs_0511020_amd.sorter import ListSorter
    sorter = sorter or ListSorter()
    nt = to_dev(nxt.astype(np.uint32), torch)
    kt = keys_to_dev(keys, flags, torch)
    out = None if inplace else torch.full_like(nt, -1)
    res = sorter.sort_async(head, nt, kt, K, descending=bool(flags & 1),
                            signed=bool(flags & 2), next_out=out, shared=shared)
    torch.cuda.synchronize()
    h, st = (int(x) & 0xFFFFFFFF for x in res.cpu().tolist())
    st = st - (1 << 32) if st >> 31 else st
    got = from_dev(nt if inplace else out)
    return h, st, got


def oracle_flags(flags, oracle):
    f = 0
    if flags & 1:
        f |= oracle.FLAG_DESCENDING
    if flags & 2:
        f |= oracle.FLAG_SIGNED
    if flags & 4:
        f |= oracle.FLAG_FLOAT
    return f


def definition_order(order, keys):
    """Stable sort of the list order by key (numpy's stable argsort)."""
    return order[np.argsort(keys[order], kind="stable")]


def check_properties(head, nxt_out, keys, orig_order, list_order_fn):
    """Checks that hold at any size and together fix the stable sort:
    the output visits every node once, keys never decrease along it, and
    equal keys keep their original list order."""
    n = keys.shape[0]
    out_order = list_order_fn(head, nxt_out)
    assert out_order.shape[0] == n
    k = keys[out_order]
    assert np.all(k[1:] >= k[:-1]), "keys decrease"
    rank = np.empty(n, dtype=np.int64)
    rank[orig_order] = np.arange(n)
    r = rank[out_order]
    ties = k[1:] == k[:-1]
    assert np.all(r[1:][ties] > r[:-1][ties]), "equal keys out of list order"
    return out_order
