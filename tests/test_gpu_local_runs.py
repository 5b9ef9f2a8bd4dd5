"""Leaf groups with runs of duplicate keys (Section III: duplicate handling),
through the C-ABI, against the CPU oracle.

A one-wave group whose bucket pass puts more than 128 keys into one bucket is
still sorted on the fast path when every such bucket holds one key value: the
words are then placed in input order and a run needs no ranking.  A bucket
that mixes values keeps going to the fallback sort.  Small arrays go straight
to the local sort, so each array here is one leaf group; the call's
`fallback_groups` statistic shows which path each kind of group took.
"""
import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")
zs = pytest.importorskip("paper_2605_14419_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
CFG = dict(k=1024, cutoff=2048, max_zlevels=8, chunk=16384)


def say(*a):
    print(*a, flush=True)


def group(rng, kind, n):
    """one array of n keys (n <= 1024).
    run    one value repeated 129..n/2 times; the other keys 2^33 apart, so
           that each bucket of the pass holds one value
    narrow keys within a range below n (a bucket per value), one of them
           repeated 129..n/2 times
    mixed  two neighbouring values 100 times each (one bucket, two values),
           the other keys 2^33 apart
    small  runs of about 50 copies of random values
    equal  a single value"""
    base = np.uint64(rng.integers(0, 2**40))
    apart = base + (np.uint64(2) + rng.permutation(n).astype(np.uint64)) * np.uint64(2**33)
    if kind == "equal":
        return np.full(n, base, dtype=np.uint64)
    if kind == "run":
        m = int(rng.integers(129, max(130, n // 2)))
        apart[rng.choice(n, size=m, replace=False)] = base
        return apart
    if kind == "narrow":
        x = base + rng.integers(0, n // 2, size=n).astype(np.uint64)
        m = int(rng.integers(129, max(130, n // 2)))
        x[rng.choice(n, size=m, replace=False)] = base + np.uint64(n // 4)
        return x
    if kind == "mixed":
        pos = rng.choice(n, size=200, replace=False)
        apart[pos[:100]] = base
        apart[pos[100:]] = base + np.uint64(1)
        return apart
    vals = rng.integers(0, 2**40, size=max(2, n // 50), dtype=np.uint64)
    return vals[rng.integers(0, vals.size, size=n)]


def build(seed, kinds, lo, hi, count):
    rng = np.random.default_rng(seed)
    parts, off = [], [0]
    for i in range(count):
        n = int(rng.integers(lo, hi + 1))
        parts.append(group(rng, kinds[i % len(kinds)], n))
        off.append(off[-1] + n)
    return np.concatenate(parts), np.array(off, dtype=np.int64)


@pytest.mark.parametrize("pw", [0, 4, 8])
def test_duplicate_runs_in_wave_groups_vs_oracle(pw):
    """wave-sized groups (up to 512 keys with 8-byte payloads, else 640):
    runs of one value stay on the fast path, and every group is the
    oracle's"""
    cap = 512 if pw == 8 else 640
    keys, off = build(17 + pw, ["run", "small", "equal", "narrow"], 300, cap, 400)
    n = keys.size
    pay = None
    if pw:
        pay = np.arange(n, dtype=np.uint32 if pw == 4 else np.uint64)
    tk = torch.from_numpy(keys.view(np.int64)).to(DEV)
    tp = None if pay is None else torch.from_numpy(
        pay.view(np.int32 if pw == 4 else np.int64)).to(DEV)
    say(f"case duplicate runs pw={pw} n={n}")
    zs.zsort_stable_segmented(tk, torch.from_numpy(off).to(DEV), tp, CFG)
    torch.cuda.synchronize()
    st = zs.zsort_get_last_stats()
    assert st["device_error"] == 0, st
    assert st["fallback_groups"] == 0, st
    ok, op = oracle.sort_segmented(keys, off, pay, k=1024, cutoff=2048, max_zlevels=8)
    assert np.array_equal(tk.cpu().numpy().view(np.uint64), ok)
    if pw:
        assert np.array_equal(tp.cpu().numpy().view(pay.dtype), op)


def test_mixed_buckets_fall_back_vs_oracle():
    """a bucket holding two values (100 keys each) is left to the fallback
    sort, which orders it like the oracle"""
    keys, off = build(29, ["mixed", "run"], 400, 640, 200)
    idx = np.arange(keys.size, dtype=np.uint32)
    tk = torch.from_numpy(keys.view(np.int64)).to(DEV)
    tp = torch.from_numpy(idx.view(np.int32)).to(DEV)
    say(f"case mixed buckets n={keys.size}")
    zs.zsort_stable_segmented(tk, torch.from_numpy(off).to(DEV), tp, CFG)
    torch.cuda.synchronize()
    st = zs.zsort_get_last_stats()
    assert st["device_error"] == 0, st
    assert st["fallback_groups"] == 100, st   # the mixed groups, and only those
    ok, oi = oracle.sort_segmented(keys, off, idx, k=1024, cutoff=2048, max_zlevels=8)
    assert np.array_equal(tk.cpu().numpy().view(np.uint64), ok)
    assert np.array_equal(tp.cpu().numpy().view(np.uint32), oi)


def test_duplicate_runs_in_one_wave_mid_groups_vs_oracle():
    """groups of 641..1024 keys (one wave of the mid-size kernel, 16 keys a
    lane) with runs of one value: the fast path, and the oracle's order"""
    keys, off = build(41, ["run", "narrow", "small"], 641, 1024, 150)
    idx = np.arange(keys.size, dtype=np.uint32)
    tk = torch.from_numpy(keys.view(np.int64)).to(DEV)
    tp = torch.from_numpy(idx.view(np.int32)).to(DEV)
    say(f"case mid-size duplicate runs n={keys.size}")
    zs.zsort_stable_segmented(tk, torch.from_numpy(off).to(DEV), tp, CFG)
    torch.cuda.synchronize()
    st = zs.zsort_get_last_stats()
    assert st["device_error"] == 0, st
    assert st["fallback_groups"] == 0, st
    ok, oi = oracle.sort_segmented(keys, off, idx, k=1024, cutoff=2048, max_zlevels=8)
    assert np.array_equal(tk.cpu().numpy().view(np.uint64), ok)
    assert np.array_equal(tp.cpu().numpy().view(np.uint32), oi)


def test_duplicate_runs_in_largest_block_groups_vs_oracle():
    """groups of 2049..4096 keys (cutoff 4096: a 512-thread workgroup each)
    with runs of one value: these workgroup jobs leave every group with an
    overfull bucket to the fallback sort (placing their words stably wave by
    wave cost more than the fallback), which orders them like the oracle"""
    cfg = dict(k=1024, cutoff=4096, max_zlevels=8, chunk=16384)
    keys, off = build(53, ["run", "narrow", "small", "equal"], 2049, 4096, 60)
    idx = np.arange(keys.size, dtype=np.uint32)
    tk = torch.from_numpy(keys.view(np.int64)).to(DEV)
    tp = torch.from_numpy(idx.view(np.int32)).to(DEV)
    say(f"case block duplicate runs n={keys.size}")
    zs.zsort_stable_segmented(tk, torch.from_numpy(off).to(DEV), tp, cfg)
    torch.cuda.synchronize()
    st = zs.zsort_get_last_stats()
    assert st["device_error"] == 0, st
    assert st["fallback_groups"] == 30, st   # the run and narrow groups
    ok, oi = oracle.sort_segmented(keys, off, idx, k=1024, cutoff=4096, max_zlevels=8)
    assert np.array_equal(tk.cpu().numpy().view(np.uint64), ok)
    assert np.array_equal(tp.cpu().numpy().view(np.uint32), oi)
