"""Fused child statistics (ZSORT_FLAG_FUSED_STATS), through the C-ABI.

With the flag, a distribution pass accumulates each child's statistics (the
exact min, max and sums of x and x^2 of Section III's per-subproblem
statistics, Algorithm 1's mean and variance loops) while it scatters the
child's keys, and no moments pass reads those keys again at the next level.
The sums are exact integers, so every subproblem's record -- its moments, the
binary64 statistics derived from them, its kind and histogram -- must equal the
oracle's bit for bit, and the output must be the oracle's.  Each test also
checks from the call's statistics that the fusion really ran: below level 0 no
moments pass read a key, yet the recursion has the same levels and the same
keys per level as without the flag.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
zs = pytest.importorskip("paper_2605_14419_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
FUSED = 4


def say(*a):
    print(*a, flush=True)


def to_dev(keys, pay=None):
    tk = torch.from_numpy(np.ascontiguousarray(keys).view(np.int64)).to(DEV)
    tp = None
    if pay is not None:
        v = pay.view(np.int32) if pay.dtype.itemsize == 4 else pay.view(np.int64)
        tp = torch.from_numpy(np.ascontiguousarray(v)).to(DEV)
    return tk, tp


def from_dev(t, dtype=np.uint64):
    return t.cpu().numpy().view(dtype)


def check_fused_stats(st, ref, n):
    """st: stats of the fused call, ref: of the same call without the flag"""
    assert zs.ZSORT_FLAG_FUSED_STATS == FUSED
    assert st["device_error"] == 0, st
    assert st["levels"] == ref["levels"], (st, ref)
    assert st["keys_per_level"] == ref["keys_per_level"]
    assert st["segs_per_level"] == ref["segs_per_level"]
    assert st["local_keys"] == ref["local_keys"]
    if ref["levels"] > 0:
        assert st["mkeys_per_level"][0] == ref["mkeys_per_level"][0] == n
    assert sum(st["mkeys_per_level"][1:]) == 0, st["mkeys_per_level"]
    assert st["model_bytes"] <= ref["model_bytes"]


def sort_pair(x, pay, cfg):
    """the same sort with and without the flag: outputs and statistics"""
    out = []
    for flags in (FUSED, 0):
        tk, tp = to_dev(x, pay)
        zs.zsort_stable_ex(tk, tp, dict(cfg, flags=flags))
        torch.cuda.synchronize()
        st = zs.zsort_get_last_stats()
        out.append((from_dev(tk), None if tp is None else from_dev(tp, pay.dtype), st))
    return out


TRACE_CFGS = [dict(k=16, cutoff=64, max_zlevels=8, chunk=2048),
              dict(k=256, cutoff=256, max_zlevels=2, chunk=4096),
              dict(k=1000, cutoff=100, max_zlevels=0, chunk=16384),
              dict(k=512, cutoff=256, max_zlevels=8, chunk=32768, tile=8192),
              dict(k=1024, cutoff=256, max_zlevels=8, chunk=32768, tile=8192),
              dict(k=1024, cutoff=2048, max_zlevels=8, chunk=16384, tile=4096)]


@pytest.mark.parametrize("cfg", TRACE_CFGS)
def test_fused_trace_parity(cfg):
    """level by level, every subproblem's moments, statistics bits, kind and
    histogram agree with the oracle when the statistics come from the scatter
    (z-score maps, range maps, both; tiles of 2048, 4096 and 8192 keys, the
    last with a u32 payload at k = 1024 staged in two windows)"""
    for name in ["uniform", "normal", "zipf", "gmm", "dup_heavy"]:
        n = 200_003
        x, idx = synth.make(name, n)
        say(f"case fused trace {name} {cfg}")
        tk, tp = to_dev(x, idx)
        rec, hist = zs.zsort_stable_traced(tk, tp, dict(cfg, flags=FUSED))
        st = zs.zsort_get_last_stats()
        k, p = from_dev(tk), from_dev(tp, np.uint32)
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
        assert st["device_error"] == 0, st
        assert sum(st["mkeys_per_level"][1:]) == 0, st["mkeys_per_level"]


@pytest.mark.parametrize("tile,k,pw", [(t, k, pw) for t in (2048, 4096, 8192)
                                        for k in (256, 512, 1024) for pw in (0, 4, 8)])
def test_fused_sorts_vs_oracle(tile, k, pw):
    """every scatter instance that fuses (bucket counts, payload widths,
    tiles), several work items and a ragged last tile: the oracle's output,
    and the unfused call's recursion without its moments passes below level 0"""
    n = 3 * 32768 + 12_345
    x, pay = synth.make("lognormal" if k != 512 else "dup_heavy", n, payload_bytes=pw)
    cfg = dict(k=k, cutoff=256, max_zlevels=8, chunk=32768, tile=tile)
    say(f"case fused sort {cfg} pw={pw}")
    (fk, fp, fst), (uk, up, ust) = sort_pair(x, pay if pw else None, cfg)
    ok, op, _ = oracle.sort(x, pay, k=k, cutoff=256, max_zlevels=8)
    assert np.array_equal(fk, ok) and np.array_equal(uk, ok)
    if pw:
        assert np.array_equal(fp, op) and np.array_equal(up, op)
    check_fused_stats(fst, ust, n)


@pytest.mark.parametrize("name", ["zipf", "gmm", "normal", "partial", "descending"])
def test_fused_workloads_vs_oracle(name):
    """one million keys of each distribution family at the default k = 1024"""
    n = 10**6 + 3
    x, idx = synth.make(name, n, payload_bytes=4)
    cfg = dict(k=1024, cutoff=2048, max_zlevels=8, chunk=16384)
    say(f"case fused workload {name}")
    (fk, fp, fst), (_, _, ust) = sort_pair(x, idx, cfg)
    ok, oi, _ = oracle.sort(x, idx, k=1024, cutoff=2048, max_zlevels=8)
    assert np.array_equal(fk, ok) and np.array_equal(fp, oi)
    check_fused_stats(fst, ust, n)


def test_fused_segmented_vs_oracle():
    """many arrays in one call: each array's children fused, every segment the
    oracle's"""
    keys, off, idx = synth.segments(300, 91, median=20_000, hi=120_000)
    cfg = dict(k=512, cutoff=512, max_zlevels=8, chunk=16384, tile=8192, flags=FUSED)
    say(f"case fused segmented n={keys.size}")
    tk, tp = to_dev(keys, idx)
    zs.zsort_stable_segmented(tk, torch.from_numpy(off).to(DEV), tp, cfg)
    torch.cuda.synchronize()
    st = zs.zsort_get_last_stats()
    assert st["device_error"] == 0, st
    assert sum(st["mkeys_per_level"][1:]) == 0
    ok, oi = oracle.sort_segmented(keys, off, idx, k=512, cutoff=512, max_zlevels=8)
    assert np.array_equal(from_dev(tk), ok) and np.array_equal(from_dev(tp, np.uint32), oi)


def test_fused_graph_replays_match_eager():
    """the cached graph with the flag: the first call captures, the second
    replays; both equal the eager fused call and the oracle"""
    n = 500_001
    x, idx = synth.make("lognormal", n, payload_bytes=4)
    cfg = dict(k=256, cutoff=1024, max_zlevels=8, chunk=32768, tile=8192)
    base_k, base_p = to_dev(x, idx)
    ek, ep = base_k.clone(), base_p.clone()
    zs.zsort_stable_ex(ek, ep, dict(cfg, flags=FUSED))
    torch.cuda.synchronize()
    for rep in range(3):
        say(f"case fused graph replay {rep}")
        gk, gp = base_k.clone(), base_p.clone()
        zs.zsort_stable_ex(gk, gp, dict(cfg, flags=FUSED | zs.ZSORT_FLAG_GRAPH))
        torch.cuda.synchronize()
        assert zs.zsort_get_last_stats()["device_error"] == 0
        assert torch.equal(gk, ek) and torch.equal(gp, ep)
    ok, oi, _ = oracle.sort(x, idx, k=256, cutoff=1024, max_zlevels=8)
    assert np.array_equal(from_dev(ek), ok) and np.array_equal(from_dev(ep, np.uint32), oi)


def test_fused_learned_and_u128_match_unfused():
    """the learned first pass keeps its own statistics (its children are fused
    from the next level on), and the 128-bit form: outputs equal the unfused
    calls'"""
    n = 2_000_003
    x, idx = synth.make("gmm", n, payload_bytes=4)
    cfg = dict(k=512, cutoff=2048, max_zlevels=8, chunk=32768, tile=8192)
    outs = []
    for flags in (FUSED, 0):
        say(f"case fused learned flags={flags}")
        tk, tp = to_dev(x, idx)
        rep = zs.zsort_stable_learned(tk, tp, dict(cfg, flags=flags))
        torch.cuda.synchronize()
        assert rep["used_learned"] == 1, rep
        assert zs.zsort_get_last_stats()["device_error"] == 0
        outs.append((tk, tp))
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])
    ok, oi, _ = oracle.sort(x, idx, k=512, cutoff=2048, max_zlevels=8)
    assert np.array_equal(from_dev(outs[0][0]), ok)
    keys, idx = synth.make128("prefix", 300_007)
    outs = []
    for flags in (FUSED, 0):
        say(f"case fused u128 flags={flags}")
        tk = torch.from_numpy(keys.reshape(-1).view(np.int64)).to(DEV)
        tp = torch.from_numpy(idx.view(np.int32)).to(DEV)
        rep = zs.zsort_stable_u128(tk, tp, dict(cfg, flags=flags), report=True)
        torch.cuda.synchronize()
        assert rep["device_error"] == 0, rep
        outs.append((tk, tp))
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])
    # the 128-bit order: high word, then low word; stable
    order = np.lexsort((np.arange(keys.shape[0]), keys[:, 0], keys[:, 1]))
    assert np.array_equal(from_dev(outs[0][0]).reshape(-1, 2), keys[order])
    assert np.array_equal(from_dev(outs[0][1], np.uint32), idx[order])
