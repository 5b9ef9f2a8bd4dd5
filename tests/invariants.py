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
