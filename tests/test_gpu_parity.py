"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle.

Integer work is compared bit for bit: the sorted keys and payloads, the exact
moments, the histograms and the cluster array after a pass.  The binary64
statistics are compared bit for bit too, because both sides evaluate the same
correctly rounded operations in the same order.
"""
import itertools

import numpy as np
import pytest

import oracle
import synth
from tests.invariants import check_stable_sorted

torch = pytest.importorskip("torch")
zs = pytest.importorskip("paper_2605_14419_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
ALPHABET = [0, 1, 2, 2**63 - 1, 2**63, 2**64 - 2, 2**64 - 1]


def say(*a):
    print(*a, flush=True)


def to_dev(keys, pay=None):
    tk = torch.from_numpy(np.ascontiguousarray(keys).view(np.int64)).to(DEV)
    tp = None
    if pay is not None:
        v = pay.view(np.int32) if pay.dtype.itemsize == 4 else pay.view(np.int64)
        tp = torch.from_numpy(np.ascontiguousarray(v)).to(DEV)
    return tk, tp


def from_dev(tk, tp, pdtype=np.uint32):
    k = tk.cpu().numpy().view(np.uint64)
    p = None if tp is None else tp.cpu().numpy().view(pdtype)
    return k, p


def gpu_sort(keys, pay, cfg):
    tk, tp = to_dev(keys, pay)
    zs.zsort_stable_ex(tk, tp, cfg)
    torch.cuda.synchronize()
    st = zs.zsort_get_last_stats() if keys.size > 1 else {"device_error": 0}
    k, p = from_dev(tk, tp, None if pay is None else pay.dtype)
    return k, p, st


CFG = dict(k=1024, cutoff=2048, max_zlevels=8, chunk=16384)


@pytest.mark.parametrize("n", [0, 1, 2, 3, 7, 64, 65, 2047, 2048, 2049, 4097, 16385, 40000])
def test_small_sizes_and_ragged_tails(n):
    say(f"case small n={n}")
    x, idx = synth.make("dup_heavy", max(n, 1))
    x, idx = x[:n], idx[:n]
    for cfg in [CFG, dict(CFG, cutoff=16, k=16, chunk=2048)]:
        k, p, st = gpu_sort(x, idx, cfg)
        assert st["device_error"] == 0, st
        ok, oi, _ = oracle.sort(x, idx, k=cfg["k"], cutoff=cfg["cutoff"], max_zlevels=8)
        assert np.array_equal(k, ok) and np.array_equal(p, oi), cfg


def test_exhaustive_tiny_segmented():
    """every array of length 4 over extreme values, one segmented call,
    cutoff 1 so every array of >= 2 keys is distributed"""
    arrays = np.array(list(itertools.product(ALPHABET, repeat=4)), dtype=np.uint64)
    x = arrays.reshape(-1)
    off = np.arange(0, x.size + 1, 4, dtype=np.int64)
    idx = np.tile(np.arange(4, dtype=np.uint32), arrays.shape[0])
    for cfg in [dict(k=16, cutoff=1, max_zlevels=8, chunk=2048),
                dict(k=16, cutoff=1, max_zlevels=0, chunk=2048),
                dict(k=4096, cutoff=1, max_zlevels=1, chunk=2048)]:
        say(f"case exhaustive4 {cfg}")
        tk, tp = to_dev(x, idx)
        toff = torch.from_numpy(off).to(DEV)
        zs.zsort_stable_segmented(tk, toff, tp, cfg)
        torch.cuda.synchronize()
        assert zs.zsort_get_last_stats()["device_error"] == 0
        k, p = from_dev(tk, tp)
        ok, oi = oracle.sort_segmented(x, off, idx, k=cfg["k"], cutoff=1,
                                       max_zlevels=cfg["max_zlevels"])
        assert np.array_equal(k, ok) and np.array_equal(p, oi)


WORKLOADS = ["uniform", "normal", "dup_heavy", "partial", "descending", "lognormal", "zipf",
             "gmm"]


@pytest.mark.parametrize("name", WORKLOADS)
def test_workloads_vs_oracle(name):
    n = 3 * 10**5 + 17
    x, idx = synth.make(name, n)
    say(f"case workload {name} n={n}")
    k, p, st = gpu_sort(x, idx, CFG)
    assert st["device_error"] == 0, st
    ok, oi, _ = oracle.sort(x, idx, **{kk: CFG[kk] for kk in ("k", "cutoff", "max_zlevels")})
    assert np.array_equal(k, ok) and np.array_equal(p, oi)


@pytest.mark.parametrize("cfg", [dict(k=16, cutoff=64, max_zlevels=8, chunk=2048),
                                 dict(k=256, cutoff=256, max_zlevels=2, chunk=4096),
                                 dict(k=4096, cutoff=2048, max_zlevels=8, chunk=32768),
                                 dict(k=1000, cutoff=100, max_zlevels=0, chunk=16384),
                                 dict(k=3162, cutoff=96, max_zlevels=16, chunk=2048)])
def test_configs_trace_parity(cfg):
    """level by level: every subproblem's moments, statistics bits, kind and
    histogram agree with the oracle under the same k / cutoff / depth guard"""
    for name in ["uniform", "normal", "zipf", "gmm", "dup_heavy"]:
        n = 200_003
        x, idx = synth.make(name, n)
        say(f"case trace {name} {cfg}")
        tk, tp = to_dev(x, idx)
        rec, hist = zs.zsort_stable_traced(tk, tp, cfg)
        k, p = from_dev(tk, tp)
        ok, oi, info, otr, ohist = oracle.sort(
            x, idx, k=cfg["k"], cutoff=cfg["cutoff"], max_zlevels=cfg["max_zlevels"], trace=True)
        assert np.array_equal(k, ok) and np.array_equal(p, oi)
        assert len(rec) == len(otr) == info[0]
        g = {(int(r["depth"]), int(r["start"])): r for r in rec}
        assert len(g) == len(rec)
        kk = cfg["k"]
        for r in otr:
            q = g[(int(r["depth"]), int(r["start"]))]
            for f in ["kind", "count", "o", "M", "shift"]:
                assert q[f] == r[f], (f, r, q)
            assert np.array_equal(q["s1"], r["s1"]) and np.array_equal(q["s2"], r["s2"])
            for f in ["m", "sigma", "zmin", "A", "B"]:
                assert np.float64(q[f]).tobytes() == np.float64(r[f]).tobytes(), (f, r, q)
            if r["kind"] in (oracle.KIND_ZMAP, oracle.KIND_RMAP):
                assert q["nonempty"] == r["nonempty"]
                gh = hist[q["hist_off"]: q["hist_off"] + kk]
                oh = ohist[r["hist_off"]: r["hist_off"] + kk]
                assert np.array_equal(gh, oh)


@pytest.mark.parametrize("name", ["uniform_2p20", "normal", "dup_heavy"])
def test_level0_cluster_array(name):
    n = 1 << 20
    x, idx = synth.make(name, n)
    say(f"case level0 {name}")
    for cfg in [CFG, dict(CFG, k=4096, chunk=32768), dict(CFG, max_zlevels=0)]:
        tk, tp = to_dev(x, idx)
        ck, cp = zs.zsort_debug_level0(tk, tp, cfg)
        gk, gp = from_dev(ck, cp)
        assert np.array_equal(from_dev(tk, tp)[0], x)   # input untouched
        ok, oi, rec, hist = oracle.level0(x, idx, k=cfg["k"], cutoff=cfg["cutoff"],
                                          max_zlevels=cfg["max_zlevels"])
        assert np.array_equal(gk, ok) and np.array_equal(gp, oi)


@pytest.mark.parametrize("pw", [0, 4, 8])
def test_payload_widths(pw):
    n = 123_457
    x, pay = synth.make("zipf", n, payload_bytes=pw)
    say(f"case payload {pw}")
    k, p, st = gpu_sort(x, pay, CFG)
    ok, op, _ = oracle.sort(x, pay, k=1024, cutoff=2048, max_zlevels=8)
    assert np.array_equal(k, ok)
    if pw:
        assert np.array_equal(p, op)


def test_segmented_vs_oracle():
    keys, off, idx = synth.segments(512, 77, median=3000, hi=200_000)
    say(f"case segmented n={keys.size}")
    tk, tp = to_dev(keys, idx)
    toff = torch.from_numpy(off).to(DEV)
    zs.zsort_stable_segmented(tk, toff, tp, CFG)
    torch.cuda.synchronize()
    assert zs.zsort_get_last_stats()["device_error"] == 0
    k, p = from_dev(tk, tp)
    ok, oi = oracle.sort_segmented(keys, off, idx, k=1024, cutoff=2048, max_zlevels=8)
    assert np.array_equal(k, ok) and np.array_equal(p, oi)


def test_segmented_malformed_offsets_move_nothing():
    keys, idx = synth.make("uniform", 10_000)
    off = np.array([0, 5000, 4000, 10_000], dtype=np.int64)  # decreasing
    say("case segmented malformed")
    tk, tp = to_dev(keys, idx)
    zs.zsort_stable_segmented(tk, torch.from_numpy(off).to(DEV), tp, CFG)
    torch.cuda.synchronize()
    assert zs.zsort_get_last_stats()["device_error"] & 0x100
    k, p = from_dev(tk, tp)
    assert np.array_equal(k, keys) and np.array_equal(p, idx)


def test_repeat_calls_identical():
    x, idx = synth.make("lognormal", 500_000)
    say("case repeat")
    outs = [gpu_sort(x, idx, CFG)[:2] for _ in range(3)]
    for k, p in outs[1:]:
        assert np.array_equal(k, outs[0][0]) and np.array_equal(p, outs[0][1])


@pytest.mark.parametrize("name,pw", [("lognormal", 8), ("normal", 4), ("dup_heavy", 8),
                                     ("uniform", 0), ("zipf", 4)])
def test_cutoff_4096_vs_oracle(name, pw):
    # leaves of 2049..4096 keys: the block jobs of their own kernel, and (wide
    # ranges, duplicates) its fallback to the merge / radix sort
    n = 3_000_000
    x, pay = synth.make(name, n, payload_bytes=pw)
    cfg = dict(k=256, cutoff=4096, max_zlevels=8, chunk=16384)
    say("case cutoff 4096", name, pw)
    k, p, st = gpu_sort(x, pay, cfg)
    assert st["device_error"] == 0
    ok, op, _ = oracle.sort(x, pay, k=256, cutoff=4096, max_zlevels=8)
    assert np.array_equal(k, ok)
    if pw:
        assert np.array_equal(p, op)


@pytest.mark.parametrize("nch,chunk,tile", [(2, 2048, 2048), (8, 2048, 2048), (9, 2048, 2048),
                                           (64, 2048, 2048), (65, 2048, 2048), (257, 2048, 2048),
                                           (1025, 2048, 2048), (65, 16384, 8192),
                                           (300, 32768, 8192)])
def test_cross_chunk_scan_unit_boundaries_vs_oracle(nch, chunk, tile):
    # the root's chunks fall into scan units of 8..256 chunks (a power of two
    # near sqrt(nch)); counts just at and past unit boundaries, ragged tail
    n = nch * chunk - 777
    x, idx = synth.make("normal", n)
    cfg = dict(k=256, cutoff=2048, max_zlevels=8, chunk=chunk, tile=tile)
    say("case scan units", nch, chunk, tile)
    k, p, st = gpu_sort(x, idx, cfg)
    assert st["device_error"] == 0
    ok, oi, _ = oracle.sort(x, idx, k=256, cutoff=2048, max_zlevels=8)
    assert np.array_equal(k, ok) and np.array_equal(p, oi)


def test_profiling_one_kernel_kind_leaves_the_sort_unchanged():
    x, idx = synth.make("lognormal", 300_000)
    ok, oi, _ = oracle.sort(x, idx, **{kk: CFG[kk] for kk in ("k", "cutoff", "max_zlevels")})
    say("case profile stages")
    tk, tp = to_dev(x, idx)
    zs.zsort_profile_begin(stages=["scatter"])
    zs.zsort_stable_ex(tk, tp, CFG)
    kt = zs.zsort_profile_end()
    k, p = from_dev(tk, tp, idx.dtype)
    assert np.array_equal(k, ok) and np.array_equal(p, oi)
    assert kt["scatter"][1] >= 1 and kt["scatter"][0] > 0
    assert all(kt[s] == (0.0, 0) for s in zs.STAGES if s != "scatter")
    tk, tp = to_dev(x, idx)
    zs.zsort_profile_begin()
    zs.zsort_stable_ex(tk, tp, CFG)
    kt = zs.zsort_profile_end()
    assert all(kt[s][1] >= 1 for s in ("moments", "finalize", "hist", "scatter", "local"))


@pytest.mark.parametrize("name", ["uniform", "normal", "dup_heavy", "partial", "descending"])
def test_ten_million_vs_oracle(name):
    """the five 10^7 arrays of the plain-path workload, full size"""
    n = 10**7
    x, idx = synth.make(name, n)
    say(f"case 1e7 {name}")
    k, p, st = gpu_sort(x, idx, CFG)
    assert st["device_error"] == 0, st
    ok, oi, _ = oracle.sort(x, idx, k=1024, cutoff=2048, max_zlevels=8)
    assert np.array_equal(k, ok) and np.array_equal(p, oi)


@pytest.mark.parametrize("tile,k,pw", [(t, k, pw) for t in (4096, 8192) for k in (256, 512, 1024)
                                        for pw in (0, 4, 8)])
def test_tiles_vs_oracle(tile, k, pw):
    """tiles larger than the staging window (8192 keys: two windows), every
    bucket-count instance and payload width, several work items and a ragged
    last tile"""
    n = 3 * 32768 + 12_345
    x, pay = synth.make("lognormal" if k != 512 else "dup_heavy", n, payload_bytes=pw)
    cfg = dict(k=k, cutoff=256, max_zlevels=8, chunk=32768, tile=tile)
    say(f"case tile {cfg} pw={pw}")
    kk, p, st = gpu_sort(x, pay, cfg)
    assert st["device_error"] == 0, st
    ok, op, _ = oracle.sort(x, pay, k=k, cutoff=256, max_zlevels=8)
    assert np.array_equal(kk, ok)
    if pw:
        assert np.array_equal(p, op)


@pytest.mark.parametrize("name,pw", [("lognormal", 8), ("uniform_1e8", 4)])
def test_full_size_bench_configuration(name, pw):
    """10^8 keys in the configuration the benchmark times (the library's
    autotuner picks it): sorted, the index payload a permutation carrying its
    key, equal keys in input order -- together these fix the output"""
    n = 10**8
    x, idx = synth.make(name, n, payload_bytes=pw)
    tk, tp = to_dev(x, idx)
    cfg = zs.zsort_autotune(tk, tp)
    say(f"case full size {name} {cfg}")
    zs.zsort_stable_ex(tk, tp, cfg)
    torch.cuda.synchronize()
    assert zs.zsort_get_last_stats()["device_error"] == 0
    k, p = from_dev(tk, tp, idx.dtype)
    del tk, tp
    check_stable_sorted(x, k, p)


@pytest.mark.parametrize("chunk", [8192, 16384, 65536])
def test_segmented_tile8192_vs_oracle(chunk):
    """8192-key tiles as work items of their own (one, two per chunk) across
    many segments, each segment's starts taken from the histogram pass"""
    keys, off, idx = synth.segments(300, 91, median=20_000, hi=120_000)
    cfg = dict(k=512, cutoff=512, max_zlevels=8, chunk=chunk, tile=8192)
    say(f"case segmented tile 8192 n={keys.size} {cfg}")
    tk, tp = to_dev(keys, idx)
    zs.zsort_stable_segmented(tk, torch.from_numpy(off).to(DEV), tp, cfg)
    torch.cuda.synchronize()
    assert zs.zsort_get_last_stats()["device_error"] == 0
    k, p = from_dev(tk, tp)
    ok, oi = oracle.sort_segmented(keys, off, idx, k=512, cutoff=512, max_zlevels=8)
    assert np.array_equal(k, ok) and np.array_equal(p, oi)


@pytest.mark.parametrize("k,pw", [(256, 8), (1024, 4)])
def test_eight_tiles_per_work_item_vs_oracle(k, pw):
    """chunks of 65536 keys: each work item has eight 8192-key tiles whose
    starts come from the histogram pass's per-tile counts"""
    n = 2 * 65536 + 12_345
    x, pay = synth.make("lognormal", n, payload_bytes=pw)
    cfg = dict(k=k, cutoff=256, max_zlevels=8, chunk=65536, tile=8192)
    say(f"case eight tiles {cfg} pw={pw}")
    kk, p, st = gpu_sort(x, pay, cfg)
    assert st["device_error"] == 0, st
    ok, op, _ = oracle.sort(x, pay, k=k, cutoff=256, max_zlevels=8)
    assert np.array_equal(kk, ok) and np.array_equal(p, op)


SIGN = np.uint64(1 << 63)


def signed_expected(x, idx, k, off=None):
    """the oracle on the order-preserving map int64 -> u64 (flip the sign
    bit), mapped back"""
    xu = x ^ SIGN
    if off is None:
        ok, oi, _ = oracle.sort(xu, idx, k=k, cutoff=2048, max_zlevels=8)
    else:
        ok, oi = oracle.sort_segmented(xu, off, idx, k=k, cutoff=2048, max_zlevels=8)
    return ok ^ SIGN, oi


@pytest.mark.parametrize("name,flags", [("uniform", 2), ("normal", 2), ("dup_heavy", 3)])
def test_signed_keys_vs_oracle(name, flags):
    """ZSORT_FLAG_SIGNED: keys ordered as two's-complement int64 (with and
    without the captured graph)"""
    n = 300_007
    x, idx = synth.make(name, n)
    x = x - np.uint64(1 << 62)          # wraps: about a quarter negative as int64
    cfg = dict(CFG, flags=flags)
    say(f"case signed {name} flags={flags}")
    for rep in range(2 if flags & 1 else 1):   # graph: capture, then replay
        k, p, st = gpu_sort(x, idx, cfg)
        assert st["device_error"] == 0, st
        ek, ep = signed_expected(x, idx, 1024)
        assert np.array_equal(k, ek) and np.array_equal(p, ep), rep
    s = k.view(np.int64)
    assert np.all(s[1:] >= s[:-1]) and s[0] < 0


def test_signed_segmented_vs_oracle():
    keys, off, idx = synth.segments(64, 33, median=5000, hi=50_000)
    keys = keys ^ SIGN                   # the upper half of each array's range turns negative
    say(f"case signed segmented n={keys.size}")
    tk, tp = to_dev(keys, idx)
    zs.zsort_stable_segmented(tk, torch.from_numpy(off).to(DEV), tp,
                              dict(CFG, flags=zs.ZSORT_FLAG_SIGNED))
    torch.cuda.synchronize()
    assert zs.zsort_get_last_stats()["device_error"] == 0
    k, p = from_dev(tk, tp)
    ek, ep = signed_expected(keys, idx, 1024, off)
    assert np.array_equal(k, ek) and np.array_equal(p, ep)


def test_signed_flag_rejected_where_unsupported():
    x, idx = synth.make("uniform", 5000)
    tk, tp = to_dev(x, idx)
    with pytest.raises(zs.ZsortError) as ei:
        zs.zsort_debug_level0(tk, tp, dict(CFG, flags=zs.ZSORT_FLAG_SIGNED))
    assert ei.value.code == -5


@pytest.mark.parametrize("cfg", [dict(k=256, cutoff=256, max_zlevels=8, chunk=4096, count_range=256),
                                 dict(k=1024, cutoff=64, max_zlevels=8, chunk=2048, count_range=1000),
                                 dict(k=4096, cutoff=2048, max_zlevels=8, chunk=32768,
                                      count_range=4096)])
def test_counting_pass_trace_parity(cfg):
    """Counting-sort termination (small key ranges, Section III's heuristic):
    the same subproblems take a counting pass (record kind 4) as in the oracle's
    counting_range mode, every record agrees, the output is the oracle's, and
    the recursion is no deeper than without the counting pass."""
    for name in ["small_range", "clustered_ranges", "dup_heavy", "zipf"]:
        n = 200_003
        x, idx = synth.make(name, n)
        say(f"case counting {name} {cfg}")
        tk, tp = to_dev(x, idx)
        rec, hist = zs.zsort_stable_traced(tk, tp, cfg)
        k, p = from_dev(tk, tp)
        ok, oi, info, otr, ohist = oracle.sort(
            x, idx, k=cfg["k"], cutoff=cfg["cutoff"], max_zlevels=cfg["max_zlevels"],
            counting_range=cfg["count_range"], trace=True)
        assert np.array_equal(k, ok) and np.array_equal(p, oi)
        assert len(rec) == len(otr) == info[0]
        g = {(int(r["depth"]), int(r["start"])): r for r in rec}
        for r in otr:
            q = g[(int(r["depth"]), int(r["start"]))]
            for f in ["kind", "count", "o", "M", "shift"]:
                assert q[f] == r[f], (f, r, q)
            assert np.array_equal(q["s1"], r["s1"]) and np.array_equal(q["s2"], r["s2"])
        counted = int(np.count_nonzero(otr["kind"] == oracle.KIND_COUNT))
        if name in ("small_range", "clustered_ranges"):
            assert counted > 0
        # the same sort through the plain entry point: stats and depth
        tk, tp = to_dev(x, idx)
        zs.zsort_stable_ex(tk, tp, cfg)
        torch.cuda.synchronize()
        st = zs.zsort_get_last_stats()
        assert st["device_error"] == 0 and st["counted"] == counted
        assert np.array_equal(from_dev(tk, tp)[0], ok)
        tk, tp = to_dev(x, idx)
        zs.zsort_stable_ex(tk, tp, dict(cfg, count_range=0))
        torch.cuda.synchronize()
        assert zs.zsort_get_last_stats()["levels"] >= st["levels"]


@pytest.mark.parametrize("pw", [0, 4, 8])
def test_wide_range_leaves_vs_oracle(pw):
    # Leaves whose keys span 2^53 .. 2^64, each array one leaf sorted in place
    # (cutoff 4096): the fallback kernel's bucket sort (offset in a bucket up
    # to 52 bits), and its radix sort where the counters cannot hold the
    # buckets (a wave's share spanning 2^64, three keys spanning 2^63) or a
    # bucket overflows (five values repeated ~400 times)
    keys, off = synth.wide_range_arrays(synth.seed_for(40))
    seg = np.repeat(np.arange(off.size - 1), np.diff(off))
    if pw == 4:
        pay = (np.arange(keys.size, dtype=np.int64) - off[seg]).astype(np.uint32)
    elif pw == 8:
        pay = np.random.default_rng(synth.seed_for(40, 1)).integers(
            0, 2**64 - 1, size=keys.size, dtype=np.uint64, endpoint=True)
    else:
        pay = None
    cfg = dict(k=256, cutoff=4096, max_zlevels=8, chunk=16384)
    say(f"case wide-range leaves pw={pw} n={keys.size}")
    tk, tp = to_dev(keys, pay)
    zs.zsort_stable_segmented(tk, torch.from_numpy(off).to(DEV), tp, cfg)
    torch.cuda.synchronize()
    assert zs.zsort_get_last_stats()["device_error"] == 0
    k, p = from_dev(tk, tp, None if pay is None else pay.dtype)
    ok, op = oracle.sort_segmented(keys, off, pay, k=256, cutoff=4096, max_zlevels=8)
    assert np.array_equal(k, ok)
    if pw:
        assert np.array_equal(p, op)


@pytest.mark.parametrize("k,pw,name", [(256, 4, "uniform"), (2048, 8, "uniform"),
                                       (2048, 0, "uniform"), (2048, 4, "dup_heavy")])
def test_wide_range_leaves_after_a_pass_vs_oracle(k, pw, name):
    # one level over uniform 64-bit keys: leaves of ~3900 (k 256) or ~490
    # (k 2048) keys spanning ~2^56 or ~2^53, sorted from the other buffer; the
    # k 2048 groups go straight to the wide wave jobs.  dup_heavy: 5000 values
    # repeated ~200 times, groups of two or three of them, which overflow a
    # bucket and go on to the fallback kernel
    n = 1_000_000
    x, pay = synth.make(name, n, payload_bytes=pw)
    if name == "dup_heavy":
        x = synth.dup_heavy(n, synth.seed_for(41), distinct=5000)
    cfg = dict(k=k, cutoff=4096, max_zlevels=1, chunk=16384)
    say(f"case wide-range leaves after a pass k={k} pw={pw} {name}")
    kk, p, st = gpu_sort(x, pay, cfg)
    assert st["device_error"] == 0
    ok, op, _ = oracle.sort(x, pay, k=k, cutoff=4096, max_zlevels=1)
    assert np.array_equal(kk, ok)
    if pw:
        assert np.array_equal(p, op)


def test_release_then_sort_again():
    """zsort_release waits for the library's streams, frees its workspaces
    and drops its graphs; the next calls lay everything out anew and sort
    like the oracle (plain, with the local sorts beside the next level, and
    through a captured graph)"""
    x, idx = synth.make("lognormal", 300_007, payload_bytes=4)
    cfg = dict(k=256, cutoff=1024, max_zlevels=8, chunk=32768, tile=8192)
    ok, oi, _ = oracle.sort(x, idx, k=256, cutoff=1024, max_zlevels=8)
    for rep in range(2):
        say(f"case release then sort {rep}")
        k, p, st = gpu_sort(x, idx, cfg)
        assert st["device_error"] == 0, st
        assert np.array_equal(k, ok) and np.array_equal(p, oi)
        k, p, st = gpu_sort(x, idx, dict(cfg, flags=zs.ZSORT_FLAG_GRAPH))
        assert np.array_equal(k, ok) and np.array_equal(p, oi)
        zs.zsort_release()


def test_results_ordered_on_the_callers_stream():
    """The local sorts of a level may run on the library's second stream; the
    caller's stream waits for them. Work queued on the caller's (non-default)
    stream right after the call, with no synchronisation in between, sees
    the finished sort: a copy made there equals the oracle's output."""
    x, idx = synth.make("lognormal", 2_000_003, payload_bytes=4)
    cfg = dict(k=256, cutoff=4096, max_zlevels=8, chunk=32768, tile=8192)
    ok, oi, _ = oracle.sort(x, idx, k=256, cutoff=4096, max_zlevels=8)
    s = torch.cuda.Stream()
    tk, tp = to_dev(x, idx)
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        for rep in range(3):
            say(f"case caller stream {rep}")
            ck, cp = tk.clone(), tp.clone()
            zs.zsort_stable_ex(ck, cp, cfg, stream=s)
            snap_k, snap_p = ck.clone(), cp.clone()   # queued on s right behind the sort
            s.synchronize()
            assert np.array_equal(snap_k.cpu().numpy().view(np.uint64), ok)
            assert np.array_equal(snap_p.cpu().numpy().view(np.uint32), oi)
