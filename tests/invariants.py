"""Checks that pin a stable sort's output without any reference sort.

Sorted (non-decreasing keys) + permutation (the index payload names every
input position once and carries its key) + stable (indices increase inside
every run of equal keys) together determine the output uniquely.
"""
import numpy as np


def check_stable_sorted(keys_in, keys_out, idx_out):
    """Raises AssertionError naming the first violated property."""
    keys_in = np.asarray(keys_in, dtype=np.uint64)
    keys_out = np.asarray(keys_out, dtype=np.uint64)
    idx = np.asarray(idx_out).astype(np.int64)
    n = keys_in.size
    assert keys_out.size == n and idx.size == n, "size changed"
    if n == 0:
        return
    assert np.all(keys_out[1:] >= keys_out[:-1]), "keys not non-decreasing"
    assert idx.min() >= 0 and idx.max() < n, "index out of range"
    seen = np.zeros(n, dtype=bool)
    seen[idx] = True
    assert seen.all(), "index payload is not a permutation"
    assert np.array_equal(keys_in[idx], keys_out), "key does not match its index"
    eq = keys_out[1:] == keys_out[:-1]
    assert np.all(idx[1:][eq] > idx[:-1][eq]), "equal keys out of input order"


def stable_reference(keys, payload=None):
    """numpy's stable argsort: a library routine used as a special case."""
    order = np.argsort(np.asarray(keys, dtype=np.uint64), kind="stable")
    k = np.asarray(keys, dtype=np.uint64)[order]
    p = None if payload is None else np.asarray(payload)[order]
    return k, p


# ---------------------------------------------------------------------------
# The same three properties checked on the device (torch ops on CUDA tensors),
# for arrays too large to copy to the host and check there: keys are u64 bits
# in int64 tensors, ordered as unsigned numbers; the payload is the index of
# each key (u32 bits in an int32 tensor, or int64).
# ---------------------------------------------------------------------------
def _unsigned_order(k):
    import torch
    return k ^ torch.tensor(-(2**63), dtype=torch.int64, device=k.device)


def _as_index(p):
    import torch
    return p.long() & 0xFFFFFFFF if p.dtype == torch.int32 else p.long()


def check_stable_sorted_device(k_in, k_out, idx_out):
    """Sorted, a permutation whose index carries its key, stable (device)."""
    import torch
    ks = _unsigned_order(k_out)
    n = k_out.numel()
    assert k_in.numel() == n, "size changed"
    if n == 0:
        return
    assert bool((ks[1:] >= ks[:-1]).all()), "keys not non-decreasing"
    if idx_out is None:
        return
    idx = _as_index(idx_out)
    assert int(idx.min()) >= 0 and int(idx.max()) < n, "index out of range"
    seen = torch.zeros(n, dtype=torch.int8, device=k_out.device)
    seen.index_fill_(0, idx, 1)
    assert int(seen.sum(dtype=torch.int64)) == n, "index payload is not a permutation"
    assert bool((k_in[idx] == k_out).all()), "key does not match its index"
    eq = ks[1:] == ks[:-1]
    assert bool((idx[1:][eq] > idx[:-1][eq]).all()), "equal keys out of input order"


def check_stable_sorted128_device(k_in, k_out, idx_out):
    """128-bit keys as (n, 2) int64 tensors, low word first, ordered as
    unsigned 128-bit numbers: sorted, a permutation whose index carries its
    key (both words), stable."""
    import torch
    n = k_out.shape[0]
    assert k_in.shape[0] == n, "size changed"
    if n == 0:
        return
    hi = _unsigned_order(k_out[:, 1])
    lo = _unsigned_order(k_out[:, 0])
    same_hi = hi[1:] == hi[:-1]
    assert bool(((hi[1:] > hi[:-1]) | (same_hi & (lo[1:] >= lo[:-1]))).all()), \
        "keys not non-decreasing"
    if idx_out is None:
        return
    idx = _as_index(idx_out)
    assert int(idx.min()) >= 0 and int(idx.max()) < n, "index out of range"
    seen = torch.zeros(n, dtype=torch.int8, device=k_out.device)
    seen.index_fill_(0, idx, 1)
    assert int(seen.sum(dtype=torch.int64)) == n, "index payload is not a permutation"
    # each word gathered on its own: torch's row gather of an (n, 2) tensor
    # (k_in[idx], index_select) returns wrong rows past the first n - 2^26 on
    # this ROCm build once n exceeds 2^26, where one-dimensional gathers are right
    for w in (0, 1):
        assert bool((k_in[:, w].contiguous()[idx] == k_out[:, w]).all()), \
            "key does not match its index"
    eq = same_hi & (lo[1:] == lo[:-1])
    assert bool((idx[1:][eq] > idx[:-1][eq]).all()), "equal keys out of input order"


def check_segmented_stable_sorted_device(k_in, k_out, idx_out, offsets):
    """The three properties inside every segment [off[i], off[i+1]): the
    payload is each key's index within its own segment."""
    import torch
    dev = k_out.device
    n = k_out.numel()
    off = offsets.to(dev).long()
    lens = off[1:] - off[:-1]
    assert int(off[0]) == 0 and int(off[-1]) == n and bool((lens >= 0).all()), "bad offsets"
    sid = torch.repeat_interleave(torch.arange(lens.numel(), device=dev), lens)
    ks = _unsigned_order(k_out)
    same = sid[1:] == sid[:-1]
    assert bool(((ks[1:] >= ks[:-1]) | ~same).all()), "keys not non-decreasing in a segment"
    loc = _as_index(idx_out)
    assert bool((loc < lens[sid]).all()) and int(loc.min()) >= 0, "index outside its segment"
    gidx = off[:-1][sid] + loc
    seen = torch.zeros(n, dtype=torch.int8, device=dev)
    seen.index_fill_(0, gidx, 1)
    assert int(seen.sum(dtype=torch.int64)) == n, "index payload is not a permutation"
    assert bool((k_in[gidx] == k_out).all()), "key does not match its index"
    eq = (ks[1:] == ks[:-1]) & same
    assert bool((loc[1:][eq] > loc[:-1][eq]).all()), "equal keys out of input order"
