"""GPU tests at the full sizes of the benchmark's workloads, in the
configurations the benchmark runs (its recorded configuration per workload
and for the learned form; the library's autotuner for the batched form, as
bench.py does).

A stable sort has one correct output, which three properties pin without a
reference sort: non-decreasing keys, an index payload that is a permutation
carrying each key, and increasing indices inside every run of equal keys
(Section III: stability).  At 10^8 keys they are checked on the device.  The
single array of 2^20 keys is compared with the CPU oracle bit for bit.
"""
import numpy as np
import pytest

import bench
import oracle
import synth
from tests.invariants import (check_segmented_stable_sorted_device,
                              check_stable_sorted128_device, check_stable_sorted_device)

torch = pytest.importorskip("torch")
zs = pytest.importorskip("paper_2605_14419_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)


def dev(keys, pay):
    tk = torch.from_numpy(keys.view(np.int64)).to(DEV)
    v = pay.view(np.int32) if pay.dtype.itemsize == 4 else pay.view(np.int64)
    return tk, torch.from_numpy(v).to(DEV)


def test_single_array_2p20_vs_oracle():
    """2^20 uniform keys + u32 index: the whole sort against the oracle, in
    the tuned configuration and in the defaults."""
    keys, idx = synth.make("uniform_2p20", 2**20, payload_bytes=4)
    base_k, base_p = dev(keys, idx)
    tuned = zs.zsort_autotune(base_k, base_p)
    for cfg in (tuned, None):
        say(f"case 2^20 uniform cfg={cfg}")
        tk, tp = base_k.clone(), base_p.clone()
        zs.zsort_stable_ex(tk, tp, cfg)
        torch.cuda.synchronize()
        st = zs.zsort_get_last_stats()
        assert st["device_error"] == 0, st
        c = tuned if cfg is not None else dict(k=1024, cutoff=2048, max_zlevels=8)
        ok, oi, _ = oracle.sort(keys, idx, k=c["k"], cutoff=c["cutoff"],
                                max_zlevels=c["max_zlevels"])
        assert np.array_equal(tk.cpu().numpy().view(np.uint64), ok)
        assert np.array_equal(tp.cpu().numpy().view(np.uint32), oi)


@pytest.mark.parametrize("name,pw", [("zipf", 8), ("lognormal", 8), ("uniform_1e8", 4),
                                     ("gmm", 4)])
def test_1e8_invariants_on_device(name, pw):
    """10^8 keys of the scale workloads (Zipf(1.2) and lognormal with a u64
    index, uniform and the mixture with a u32 index), tuned configuration."""
    n = 10**8
    keys, idx = synth.make(name, n, payload_bytes=pw)
    base_k, base_p = dev(keys, idx)
    del keys, idx
    cfg = bench.TUNED[name]
    say(f"case 1e8 {name} pw={pw} cfg={cfg}")
    tk, tp = base_k.clone(), base_p.clone()
    zs.zsort_stable_ex(tk, tp, cfg)
    torch.cuda.synchronize()
    st = zs.zsort_get_last_stats()
    assert st["device_error"] == 0, st
    check_stable_sorted_device(base_k, tk, tp)


def test_4096_segments_full_size_graph_on_device():
    """The batched workload at full size (4096 arrays, ~1.35e8 keys, lengths
    clamped to [100, 10^6]) through the cached graph: every segment sorted,
    stable and a permutation of its own keys; graph and per-call runs agree."""
    keys, off, idx = synth.segments(4096, synth.seed_for(3, 0))
    say(f"case segments 4096 n={keys.size}")
    base_k, base_p = dev(keys, idx)
    toff = torch.from_numpy(off).to(DEV)
    del keys, idx
    cfg = zs.zsort_autotune(base_k, base_p, toff)
    gcfg = dict(cfg, flags=zs.ZSORT_FLAG_GRAPH)
    gk, gp = base_k.clone(), base_p.clone()
    for rep in range(2):   # first call captures the graph, the second replays it
        gk.copy_(base_k)
        gp.copy_(base_p)
        torch.cuda.synchronize()
        zs.zsort_stable_segmented(gk, toff, gp, gcfg)
        torch.cuda.synchronize()
        st = zs.zsort_get_last_stats()
        assert st["device_error"] == 0, st
        check_segmented_stable_sorted_device(base_k, gk, gp, toff)
    ek, ep = base_k.clone(), base_p.clone()
    zs.zsort_stable_segmented(ek, toff, ep, cfg)
    torch.cuda.synchronize()
    assert torch.equal(ek, gk) and torch.equal(ep, gp)


def test_learned_1e8_invariants_on_device():
    """The learned-map form on 10^8 mixture keys with 4096 first-pass clusters
    (the model fitted inside the call): sorted, stable, a permutation; the
    learned map was used and its order check passed."""
    n = 10**8
    keys, idx = synth.make("gmm", n, payload_bytes=4)
    base_k, base_p = dev(keys, idx)
    del keys, idx
    cfg = bench.TUNED["learned"]
    say(f"case learned 1e8 cfg={cfg}")
    tk, tp = base_k.clone(), base_p.clone()
    rep = zs.zsort_stable_learned(tk, tp, cfg, dict(flags=zs.ZSORT_LEARNED_ZSCORE_DIAG))
    torch.cuda.synchronize()
    assert rep["used_learned"] == 1 and rep["fallback"] == 0, rep
    assert rep["imbalance_learned"] < rep["imbalance_zscore"], rep
    st = zs.zsort_get_last_stats()
    assert st["device_error"] == 0, st
    check_stable_sorted_device(base_k, tk, tp)


@pytest.mark.parametrize("name", ["uuid", "prefix", "zext"])
def test_u128_1e8_invariants_on_device(name):
    """128-bit keys at 10^8 with the u32 index, in the benchmark's
    configuration: sorted, a permutation carrying its key, stable."""
    n = 10**8
    keys, idx = synth.make128(name, n)
    say(f"case u128 1e8 {name}")
    base_k = torch.from_numpy(keys.reshape(-1).view(np.int64)).to(DEV)
    tp = torch.from_numpy(idx.view(np.int32)).to(DEV)
    del keys, idx
    tk = base_k.clone()
    rep = zs.zsort_stable_u128(tk, tp, bench.TUNED["uniform_1e8"], report=True)
    torch.cuda.synchronize()
    assert rep["device_error"] == 0, rep
    check_stable_sorted128_device(base_k.view(-1, 2), tk.view(-1, 2), tp)
    del base_k, tk, tp
    torch.cuda.empty_cache()


def test_fused_statistics_1e8_invariants_on_device():
    """The fused child statistics (opt-in) at 10^8 lognormal keys with a u64
    index in the benchmark's configuration: sorted, a permutation carrying its
    key, stable, and no moments pass below level 0."""
    n = 10**8
    keys, idx = synth.make("lognormal", n, payload_bytes=8)
    base_k, base_p = dev(keys, idx)
    del keys, idx
    cfg = dict(bench.TUNED["lognormal"], flags=zs.ZSORT_FLAG_FUSED_STATS)
    say(f"case fused 1e8 cfg={cfg}")
    tk, tp = base_k.clone(), base_p.clone()
    zs.zsort_stable_ex(tk, tp, cfg)
    torch.cuda.synchronize()
    st = zs.zsort_get_last_stats()
    assert st["device_error"] == 0, st
    assert st["levels"] >= 2 and sum(st["mkeys_per_level"][1:]) == 0, st["mkeys_per_level"]
    check_stable_sorted_device(base_k, tk, tp)
