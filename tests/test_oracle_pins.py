"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: each check is a closed form,
an invariant stated in the paper, a hand-derived example, brute force, or a
library routine (numpy's stable argsort, Python's correctly rounded int ->
float conversion) used as a special case.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth
from tests.invariants import check_stable_sorted, stable_reference

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
U64 = 2**64 - 1
ALPHABET = [0, 1, 2, 2**63 - 1, 2**63, 2**64 - 2, 2**64 - 1]


# --------------------------------------------------------------------------
# brute force and the final output
# --------------------------------------------------------------------------
def test_brute_force_matches_python_sorted():
    rng = np.random.default_rng(7)
    for n in [0, 1, 2, 5, 17, 64]:
        for alpha in [2, 5, 1000]:
            x = rng.integers(0, alpha, size=n).astype(np.uint64) * np.uint64(2**50)
            idx = np.arange(n, dtype=np.uint32)
            bk, bi = oracle.brute_stable_sort(x, idx)
            order = sorted(range(n), key=lambda i: int(x[i]))  # Python's sort is stable
            assert bi.tolist() == order
            assert bk.tolist() == [int(x[i]) for i in order]


@pytest.mark.parametrize("k,cutoff,maxz", [(2, 1, 8), (4, 1, 8), (3, 2, 1), (1024, 1, 0)])
def test_exhaustive_tiny_vs_brute(k, cutoff, maxz):
    """every array of length <= 5 over an alphabet of extreme values"""
    for n in range(0, 6):
        arrays = list(itertools.product(ALPHABET, repeat=n)) if n else [()]
        for tup in arrays:
            x = np.array(tup, dtype=np.uint64)
            idx = np.arange(n, dtype=np.uint32)
            ok, oi, _ = oracle.sort(x, idx, k=k, cutoff=cutoff, max_zlevels=maxz)
            bk, bi = oracle.brute_stable_sort(x, idx)
            assert np.array_equal(ok, bk) and np.array_equal(oi, bi), (tup, k, cutoff)


def test_exhaustive_len6_segmented_vs_lexsort():
    """all 7^6 arrays of length 6 at once through the segmented entry, against
    numpy's lexsort of (segment, key, position)"""
    arrays = np.array(list(itertools.product(ALPHABET, repeat=6)), dtype=np.uint64)
    nseg = arrays.shape[0]
    x = arrays.reshape(-1)
    off = np.arange(0, x.size + 1, 6, dtype=np.int64)
    idx = np.tile(np.arange(6, dtype=np.uint32), nseg)
    ok, oi = oracle.sort_segmented(x, off, idx, k=4, cutoff=1, max_zlevels=8)
    seg = np.repeat(np.arange(nseg), 6)
    order = np.lexsort((np.arange(x.size), x, seg))
    assert np.array_equal(ok, x[order])
    assert np.array_equal(oi, idx[order])


@pytest.mark.parametrize("seed", range(6))
def test_random_small_alphabet(seed):
    rng = np.random.default_rng(100 + seed)
    for _ in range(40):
        n = int(rng.integers(0, 2000))
        alpha = int(rng.choice([1, 2, 3, 10, 100, 10**6]))
        base = rng.integers(0, 2**64, size=alpha, dtype=np.uint64, endpoint=False)
        x = base[rng.integers(0, alpha, size=n)]
        idx = np.arange(n, dtype=np.uint32)
        k = int(rng.choice([2, 3, 16, 256, 1024]))
        cutoff = int(rng.choice([1, 8, 96]))
        maxz = int(rng.choice([0, 1, 3, 8]))
        ok, oi, _ = oracle.sort(x, idx, k=k, cutoff=cutoff, max_zlevels=maxz)
        check_stable_sorted(x, ok, oi)
        rk, ri = stable_reference(x, idx)
        assert np.array_equal(ok, rk) and np.array_equal(oi, ri)


WORKLOAD_NAMES = ["uniform_2p20", "uniform", "normal", "dup_heavy", "partial", "descending",
                  "lognormal", "zipf", "gmm", "gmm_identity"]


@pytest.mark.parametrize("name", WORKLOAD_NAMES)
@pytest.mark.parametrize("mode", ["gpu_like", "paper"])
def test_workloads_reduced(name, mode):
    n = 1 << 16
    x, idx = synth.make(name, n, payload_bytes=4)
    if mode == "paper":
        prm = oracle.paper_params(n)
    else:
        prm = dict(k=1024, cutoff=256, max_zlevels=8)
    ok, oi, info = oracle.sort(x, idx, **prm)
    check_stable_sorted(x, ok, oi)
    rk, ri = stable_reference(x, idx)
    assert np.array_equal(ok, rk) and np.array_equal(oi, ri)


def test_payload_widths():
    x, _ = synth.make("dup_heavy", 5000, payload_bytes=0)
    for dt in [np.uint32, np.uint64]:
        p = np.arange(x.size, dtype=dt) * dt(3)
        ok, op, _ = oracle.sort(x, p, k=64, cutoff=8)
        rk, rp = stable_reference(x, p)
        assert np.array_equal(ok, rk) and np.array_equal(op, rp)
    ok, op, _ = oracle.sort(x, None, k=64, cutoff=8)
    assert op is None and np.array_equal(ok, np.sort(x))


def test_paper_mode_equals_parity_mode():
    x, idx = synth.make("normal", 200000)
    a = oracle.sort(x, idx, **oracle.paper_params(x.size))
    b = oracle.sort(x, idx, **oracle.paper_params(x.size, alpha=0.6))
    c = oracle.sort(x, idx, k=1024, cutoff=4096, max_zlevels=8)
    for r in (b, c):
        assert np.array_equal(a[0], r[0]) and np.array_equal(a[1], r[1])


def test_counting_sort_heuristic():
    rng = np.random.default_rng(3)
    x = (rng.integers(0, 60000, size=50000) + 10**15).astype(np.uint64)
    idx = np.arange(x.size, dtype=np.uint32)
    ok, oi, info, tr, _ = oracle.sort(x, idx, k=64, cutoff=96, counting_range=65000, trace=True)
    assert tr[0]["kind"] == oracle.KIND_COUNT
    check_stable_sorted(x, ok, oi)


def test_segmented_oracle():
    keys, off, idx = synth.segments(64, 11, median=2000, hi=20000)
    ok, oi = oracle.sort_segmented(keys, off, idx, k=256, cutoff=64)
    for s in range(64):
        a, b = off[s], off[s + 1]
        rk, ri = stable_reference(keys[a:b], idx[a:b])
        assert np.array_equal(ok[a:b], rk) and np.array_equal(oi[a:b], ri)


# --------------------------------------------------------------------------
# exact integers and their conversion
# --------------------------------------------------------------------------
def test_u256_to_double_correctly_rounded():
    """CPython converts int -> float with correct rounding (ties to even)."""
    rng = np.random.default_rng(5)
    vals = [0, 1, 2**53 - 1, 2**53, 2**53 + 1, 2**64 - 1, 2**64, 2**64 + 1, 2**255 + 2**202,
            2**200 + 2**147, 2**200 + 2**147 + 1, 2**200 + 3 * 2**147, (2**53 + 1) << 100,
            ((2**53 + 1) << 100) + 1, (1 << 256) - 1]
    for bits in range(1, 257):
        for _ in range(8):
            v = int(rng.integers(0, 2**63)) << 193
            v |= sum(int(rng.integers(0, 2**63)) << (63 * i) for i in range(4))
            vals.append(v % (1 << bits) | (1 << (bits - 1)))
    # exact ties: 54 significant bits ending in 1 -> halfway between doubles
    for s in [11, 40, 100, 150, 199]:
        for m in [(1 << 53) | 1, (1 << 53) | 3, (1 << 53) | 0x155555]:
            vals.append(m << s)
    for v in vals:
        if v >= 1 << 256:
            continue
        assert oracle.u256_to_double(v) == float(v), hex(v)


def test_moments_closed_forms():
    rng = np.random.default_rng(9)
    for n in [1, 2, 3, 10, 1000, 65537]:
        for c in [0, 12345, 2**64 - n]:
            x = (np.arange(n, dtype=np.uint64) + np.uint64(c))
            x = x[rng.permutation(n)]
            o, M, s1, s2 = oracle.moments(x)
            assert o == c and M == c + n - 1
            assert s1 == n * (n - 1) // 2
            assert s2 == (n - 1) * n * (2 * n - 1) // 6
    # extreme two-valued arrays: a zeros and b maxima
    for a, b in [(1, 1), (3, 5), (1000, 1)]:
        x = np.array([0] * a + [U64] * b, dtype=np.uint64)
        o, M, s1, s2 = oracle.moments(x[rng.permutation(x.size)])
        assert (o, M) == (0, U64)
        assert s1 == b * U64 and s2 == b * U64 * U64
    # constant arrays
    o, M, s1, s2 = oracle.moments(np.full(77, 2**63 + 5, dtype=np.uint64))
    assert o == M == 2**63 + 5 and s1 == 0 and s2 == 0


def test_moments_order_independent_bits():
    """Section III: mean and standard deviation do not depend on the input
    order -- with exact moments the statistics are bit-identical."""
    x, _ = synth.make("lognormal", 100000)
    rng = np.random.default_rng(1)
    ref = None
    for _ in range(4):
        o, M, s1, s2 = oracle.moments(x[rng.permutation(x.size)])
        st = oracle.zstats(x.size, s1, s2, 1024)
        if ref is None:
            ref = (o, M, s1, s2, st)
        assert (o, M, s1, s2, st) == ref


# --------------------------------------------------------------------------
# statistics and the map
# --------------------------------------------------------------------------
@pytest.mark.parametrize("k", [4, 1024, 4096])
def test_two_point_set(k):
    """n/2 copies of a and of b, b - a a power of two: mean (a+b)/2,
    std (b-a)/2, Zmin 1; h(a) = 0, h(b) = min(2*scale, k-1)."""
    for p in [1, 20, 52, 63]:
        a = 2**61 + 12345
        b = a + 2**p
        x = np.array([a, b] * 500, dtype=np.uint64)
        o, M, s1, s2 = oracle.moments(x)
        ok, m, var, sigma, zmin, A, B = oracle.zstats(x.size, s1, s2, k)
        assert ok
        assert m == 2.0 ** (p - 1) and sigma == 2.0 ** (p - 1) and var == 4.0 ** (p - 1)
        assert zmin == 1.0
        assert oracle.zbucket(a, o, m, A, B, k) == 0
        assert oracle.zbucket(b, o, m, A, B, k) == min(k // 2, k - 1)


def test_arithmetic_progression_variance():
    """x = 0..n-1: population variance (n^2 - 1)/12, exact for n = 4097."""
    n = 4097
    x = np.arange(n, dtype=np.uint64) + np.uint64(99)
    o, M, s1, s2 = oracle.moments(x)
    ok, m, var, sigma, zmin, A, B = oracle.zstats(n, s1, s2, 256)
    assert m == 2048.0 and var == (n * n - 1) / 12 == 1398784.0
    assert sigma == math.sqrt(1398784.0)
    assert zmin == 2048.0 / math.sqrt(1398784.0)


def test_fig1_setting_hand_example():
    g = json.load(open(os.path.join(GOLDEN, "fig1_setting_k4.json")))
    x = np.array(g["keys"], dtype=np.uint64)
    idx = np.arange(x.size, dtype=np.uint32)
    tol = g["tolerance"]
    ck, ci, rec, hist = oracle.level0(x, idx, k=g["k"], cutoff=g["cutoff"])
    assert hist.tolist() == g["root_hist"]
    assert ck.tolist() == g["root_cluster_keys"] and ci.tolist() == g["root_cluster_index"]
    assert abs(rec["m"] - g["root_m"]) < tol
    assert abs(rec["sigma"] - g["root_sigma"]) < tol
    assert abs(rec["zmin"] - g["root_zmin"]) < tol
    sk, si, info, tr, hs = oracle.sort(x, idx, k=g["k"], cutoff=g["cutoff"], trace=True)
    assert sk.tolist() == g["sorted_keys"] and si.tolist() == g["sorted_index"]
    child = [r for r in tr if r["depth"] == 1]
    assert len(child) == 1
    c = child[0]
    assert (int(c["start"]), int(c["count"])) == (g["child_start"], g["child_count"])
    assert c["kind"] == oracle.KIND_ZMAP
    h = hs[c["hist_off"]: c["hist_off"] + g["k"]]
    assert h.tolist() == g["child_hist"]
    assert abs(c["m"] - g["child_m"]) < tol
    assert abs(c["sigma"] - g["child_sigma"]) < tol
    assert abs(c["zmin"] - g["child_zmin"]) < tol
    ident = sorted((int(r["start"]), int(r["count"])) for r in tr if r["kind"] == oracle.KIND_IDENT)
    assert ident == [tuple(v) for v in g["identical"]]


def test_mean_est_inverts_h():
    """Recursive phase: h(meanEst_j) = j + 0.5 (the mid-point of cluster j)."""
    for name in ["uniform", "normal", "lognormal"]:
        x, _ = synth.make(name, 50000)
        o, M, s1, s2 = oracle.moments(x)
        k = 1024
        ok, m, var, sigma, zmin, A, B = oracle.zstats(x.size, s1, s2, k)
        scale = k / 4.0
        for j in [0, 1, 7, 100, 511, 1023]:
            e = oracle.mean_est(j, scale, zmin, sigma, m)
            h_real = (e - m) / sigma * scale + zmin * scale
            assert abs(h_real - (j + 0.5)) < 1e-9 * (j + 1)


def test_map_monotone_clipped_and_min_at_zero():
    """Ordering invariant max(C_j) < min(C_j+1) needs h monotone; the clip keeps
    j in [0, k-1]; the shift by |Zmin| puts the root's minimum in cluster 0."""
    for name in ["uniform", "normal", "lognormal", "zipf", "gmm"]:
        x, _ = synth.make(name, 20000)
        xs = np.unique(x)
        o, M, s1, s2 = oracle.moments(x)
        for k in [4, 1000, 4096]:
            ok, m, var, sigma, zmin, A, B = oracle.zstats(x.size, s1, s2, k)
            assert ok
            h = np.array([oracle.zbucket(int(v), o, m, A, B, k) for v in xs])
            assert h.min() >= 0 and h.max() <= k - 1
            assert np.all(np.diff(h) >= 0)
            assert h[0] == 0


def test_uniform_nonempty_fraction():
    """uniform data: Zmin ~ sqrt(3), so about sqrt(3)/2 of the k clusters are
    reached (statistical sanity of the map's scale)."""
    x, idx = synth.make("uniform_2p20", 1 << 20)
    _, _, rec, hist = oracle.level0(x, idx, k=1024, cutoff=4096)
    assert abs(rec["zmin"] - math.sqrt(3)) < 5e-3
    nonempty = int((hist > 0).sum())
    assert abs(nonempty - math.sqrt(3) / 2 * 1024) < 4


def test_level0_is_stable_bucket_sort():
    """After one pass the array equals a stable sort by cluster index, the
    histogram is the count of each index, and clusters are ordered."""
    for name in ["normal", "dup_heavy", "descending"]:
        x, idx = synth.make(name, 6000)
        k = 256
        ck, ci, rec, hist = oracle.level0(x, idx, k=k, cutoff=64)
        h = np.array([oracle.zbucket(int(v), int(rec["o"]), rec["m"], rec["A"], rec["B"], k)
                      for v in x])
        order = np.argsort(h, kind="stable")
        assert np.array_equal(ck, x[order]) and np.array_equal(ci, idx[order])
        assert np.array_equal(hist, np.bincount(h, minlength=k))
        starts = np.concatenate([[0], np.cumsum(hist.astype(np.int64))]).astype(np.int64)
        prev_max = None
        for j in range(k):
            if hist[j]:
                seg = ck[starts[j]:starts[j + 1]]
                if prev_max is not None:
                    assert prev_max < seg.min()
                prev_max = seg.max()


def test_range_map_splits():
    """Progress guard: the range map sends min and max to different clusters
    whenever max > min, and stays in [0, k)."""
    rng = np.random.default_rng(2)
    for k in [2, 3, 256, 1000, 4096]:
        for _ in range(200):
            o = int(rng.integers(0, 2**63))
            R = int(rng.integers(1, 2**63)) >> int(rng.integers(0, 63))
            R = max(R, 1)
            s = oracle.rshift(R, k)
            b0, b1 = oracle.rbucket(o, o, s), oracle.rbucket(o + R, o, s)
            assert b0 == 0 and 1 <= b1 < k


def test_forced_range_map_only():
    x, idx = synth.make("gmm", 30000)
    ok, oi, info, tr, _ = oracle.sort(x, idx, k=256, cutoff=32, max_zlevels=0, trace=True)
    assert set(np.unique(tr["kind"])) <= {oracle.KIND_RMAP, oracle.KIND_IDENT}
    check_stable_sorted(x, ok, oi)
    assert info[2] <= 8 + 1  # 64 bits / 8 bits per pass, plus the leaf level


def test_trace_consistency_and_guard():
    """Every pass: histogram sums to the subproblem; clusters > cutoff appear
    as subproblems one level deeper at the right offset; a pass that put all
    keys in one cluster hands a range-mapped child."""
    for name in ["normal", "zipf", "lognormal", "dup_heavy", "gmm"]:
        x, idx = synth.make(name, 1 << 15)
        k, cutoff = 64, 16
        ok, oi, info, tr, hs = oracle.sort(x, idx, k=k, cutoff=cutoff, max_zlevels=8, trace=True)
        by_pos = {(int(r["depth"]), int(r["start"])): r for r in tr}
        for r in tr:
            if r["kind"] not in (oracle.KIND_ZMAP, oracle.KIND_RMAP):
                continue
            h = hs[r["hist_off"]: r["hist_off"] + k].astype(np.int64)
            assert h.sum() == r["count"]
            assert r["nonempty"] == int((h > 0).sum())
            start = int(r["start"])
            for j in range(k):
                if h[j] > cutoff:
                    ch = by_pos[(int(r["depth"]) + 1, start)]
                    assert int(ch["count"]) == h[j]
                    if h[j] == r["count"] or r["kind"] == oracle.KIND_RMAP:
                        assert ch["kind"] in (oracle.KIND_RMAP, oracle.KIND_IDENT)
                start += int(h[j])


def test_invariant_checker_rejects_errors():
    x = np.array([5, 3, 5, 1], dtype=np.uint64)
    good_k, good_i = np.array([1, 3, 5, 5], dtype=np.uint64), np.array([3, 1, 0, 2])
    check_stable_sorted(x, good_k, good_i)
    with pytest.raises(AssertionError):
        check_stable_sorted(x, good_k, np.array([3, 1, 2, 0]))       # unstable
    with pytest.raises(AssertionError):
        check_stable_sorted(x, np.array([1, 3, 5, 4], dtype=np.uint64), good_i)
    with pytest.raises(AssertionError):
        check_stable_sorted(x, good_k, np.array([3, 1, 0, 0]))       # not a permutation


def test_device_checkers_reject_planted_mistakes_on_cpu_tensors():
    """The torch forms of the three properties (used at 10^8 keys on the
    device) accept a correct stable sort and reject each planted mistake."""
    torch = pytest.importorskip("torch")
    from tests.invariants import (check_segmented_stable_sorted_device,
                                  check_stable_sorted_device)
    rng = np.random.default_rng(5)
    x = rng.integers(0, 6, size=400).astype(np.uint64) * np.uint64(2**62 // 3)
    order = np.argsort(x, kind="stable")
    kin = torch.from_numpy(x.view(np.int64))
    kout = torch.from_numpy(x[order].view(np.int64))
    iout = torch.from_numpy(order.astype(np.int32))
    check_stable_sorted_device(kin, kout, iout)
    bad_unstable = iout.clone()
    eqpos = np.nonzero(x[order][1:] == x[order][:-1])[0][0]
    bad_unstable[eqpos], bad_unstable[eqpos + 1] = iout[eqpos + 1], iout[eqpos]
    bad_keys = kout.clone()
    bad_keys[0], bad_keys[-1] = kout[-1], kout[0]
    bad_perm = iout.clone()
    bad_perm[3] = bad_perm[4]
    for k, i, what in [(kout, bad_unstable, "order"), (bad_keys, iout, "non-decreasing"),
                       (kout, bad_perm, "permutation")]:
        with pytest.raises(AssertionError, match=what):
            check_stable_sorted_device(kin, k, i)
    # segmented: two segments, each sorted on its own
    off = torch.tensor([0, 150, 400])
    parts_k, parts_i = [], []
    for a, b in [(0, 150), (150, 400)]:
        o = np.argsort(x[a:b], kind="stable")
        parts_k.append(x[a:b][o])
        parts_i.append(o.astype(np.int32))
    sk = torch.from_numpy(np.concatenate(parts_k).view(np.int64))
    si = torch.from_numpy(np.concatenate(parts_i))
    check_segmented_stable_sorted_device(kin, sk, si, off)
    with pytest.raises(AssertionError):   # sorted as one array is not per segment
        check_segmented_stable_sorted_device(kin, kout, iout, off)


def test_device_checker128_rejects_planted_mistakes_on_cpu_tensors():
    """The 128-bit form: (high, low) order with the high word deciding, the
    index carrying both words, equal keys in input order."""
    torch = pytest.importorskip("torch")
    from tests.invariants import check_stable_sorted128_device
    rng = np.random.default_rng(6)
    hi = rng.integers(0, 3, size=300).astype(np.uint64) * np.uint64(2**63 // 2)
    lo = rng.integers(0, 4, size=300).astype(np.uint64) * np.uint64(2**62)
    order = np.lexsort((lo, hi))          # stable: equal keys keep input order
    k2 = np.stack([lo, hi], axis=1)
    kin = torch.from_numpy(k2.view(np.int64))
    kout = torch.from_numpy(np.ascontiguousarray(k2[order]).view(np.int64))
    iout = torch.from_numpy(order.astype(np.int32))
    check_stable_sorted128_device(kin, kout, iout)
    sk = k2[order]
    eqpos = np.nonzero((sk[1:] == sk[:-1]).all(axis=1))[0][0]
    bad_unstable = iout.clone()
    bad_unstable[eqpos], bad_unstable[eqpos + 1] = iout[eqpos + 1], iout[eqpos]
    # low words out of order inside a run of equal high words
    run = np.nonzero((sk[1:, 1] == sk[:-1, 1]) & (sk[1:, 0] != sk[:-1, 0]))[0][0]
    bad_lo = kout.clone()
    bad_lo[run, 0], bad_lo[run + 1, 0] = kout[run + 1, 0], kout[run, 0]
    bad_perm = iout.clone()
    bad_perm[3] = bad_perm[4]
    # a key whose low word differs from its index's key (still sorted: the
    # last low word 0 becomes 1, below every other nonzero low word)
    bad_word = kout.clone()
    j = int(np.nonzero(sk[:, 0] == 0)[0][-1])
    bad_word[j, 0] = 1
    for k, i, what in [(kout, bad_unstable, "order"), (bad_lo, iout, "non-decreasing"),
                       (kout, bad_perm, "permutation"), (bad_word, iout, "match")]:
        with pytest.raises(AssertionError, match=what):
            check_stable_sorted128_device(kin, k, i)


# ---------------------------------------------------------------------------
# 128-bit keys: the oracle's definition against brute force and a library sort
# ---------------------------------------------------------------------------
ALPHA128 = [(0, 0), (1, 0), (0, 1), (2**64 - 1, 0), (0, 2**64 - 1), (2**64 - 1, 2**64 - 1),
            (5, 2**63), (5, 2**63 - 1)]


def _brute128(keys, signed):
    """selection of the least remaining key, first occurrence on ties"""
    def val(k):
        hi = int(k[1]) ^ (1 << 63) if signed else int(k[1])
        return (hi << 64) | int(k[0])
    rest = list(range(len(keys)))
    out = []
    while rest:
        best = min(rest, key=lambda i: (val(keys[i]), i))
        out.append(best)
        rest.remove(best)
    return out


@pytest.mark.parametrize("signed", [False, True])
def test_sort128_exhaustive_tiny_vs_brute_force(signed):
    import itertools
    for combo in itertools.product(range(len(ALPHA128)), repeat=3):
        keys = np.array([ALPHA128[c] for c in combo], dtype=np.uint64)
        idx = np.arange(3, dtype=np.uint32)
        k, p = oracle.sort128(keys, idx, signed=signed)
        order = _brute128(keys, signed)
        assert p.tolist() == order
        assert np.array_equal(k, keys[order])


def test_sort128_random_vs_lexsort_and_structure():
    rng = np.random.default_rng(9)
    for n in (0, 1, 2, 17, 1000, 4097):
        hi = rng.integers(0, 4, size=n).astype(np.uint64) * np.uint64(2**62)
        lo = rng.integers(0, 5, size=n).astype(np.uint64) * np.uint64(2**61)
        keys = np.stack([lo, hi], axis=1)
        idx = np.arange(n, dtype=np.uint32)
        k, p = oracle.sort128(keys, idx)
        order = np.lexsort((lo, hi))          # stable, last key primary
        assert np.array_equal(p, order.astype(np.uint32))
        assert np.array_equal(k, keys[order])
        # signed: the high word's sign bit decides first
        ks, ps = oracle.sort128(keys, idx, signed=True)
        order_s = np.lexsort((lo, hi ^ np.uint64(2**63)))
        assert np.array_equal(ps, order_s.astype(np.uint32))
    # keys that differ only in the low word order as 64-bit keys do
    lo = rng.integers(0, 2**64, size=3000, dtype=np.uint64)
    keys = np.stack([lo, np.full(3000, 7, dtype=np.uint64)], axis=1)
    k, p = oracle.sort128(keys, np.arange(3000, dtype=np.uint32))
    assert np.array_equal(k[:, 0], np.sort(lo, kind="stable"))
