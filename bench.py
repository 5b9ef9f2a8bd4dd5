#!/usr/bin/env python3
"""Throughput of the stable z-score distribution sort on one MI355X.

A step is one complete stable sort (every level of the recursion and the
local sorts) of one 10^8-key synthetic array that is already resident in HBM.
The K timed steps each sort their own copy of the input, so nothing is
sorted twice and no copy runs inside the timed region.

Prints one JSON line.  `value` is GKeys/s of the plain z-score path on the
primary workload; `roofline` describes the kernel with the largest device
time (HIP events recorded by the library on the launch stream);
`cpu_baseline` times the CPU oracle on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GKeys/s + % HBM peak, stable 1e8 u64+idx: z-score vs learned-CDF vs batched"
HBM_PEAK_GBS = 8000.0
STAGES = ("moments", "finalize", "hist", "scatter", "local", "local_hard")
# Each workload runs in the configuration the library's autotuner picked for
# it most often (its picks differ between runs by less than the run-to-run
# spread); --autotune times the candidates again instead.  The profiles kept
# beside the code were taken in these configurations.
TUNED = {
    "lognormal": dict(k=256, cutoff=4096, max_zlevels=8, chunk=32768, tile=8192),
    "zipf": dict(k=1024, cutoff=4096, max_zlevels=8, chunk=32768, tile=8192),
    "uniform_1e8": dict(k=512, cutoff=2048, max_zlevels=8, chunk=32768, tile=8192),
    "gmm": dict(k=256, cutoff=4096, max_zlevels=8, chunk=32768, tile=8192),
    # the learned map's later levels sort its first-pass clusters: measured
    # 5.08 ms per sort with the fit at k 512 / cutoff 2048, 5.35 at the
    # z-score line's k 256 / cutoff 4096
    "learned": dict(k=512, cutoff=2048, max_zlevels=8, chunk=32768, tile=8192),
}
PRIMARY = dict(workload="lognormal", n=10**8, payload_bytes=8,
               desc="plain z-score path, 1e8 u64 keys floor(exp(N(40, 2.5^2))) clamped, "
                    "u64 index payload")
EXTRAS = {
    "zipf": dict(workload="zipf", n=10**8, payload_bytes=8,
                 desc="plain z-score path, 1e8 u64 keys Zipf(1.2) over 1e6 values, u64 index"),
    "uniform_u32": dict(workload="uniform_1e8", n=10**8, payload_bytes=4,
                        desc="plain z-score path, 1e8 uniform u64 keys, u32 index"),
    "gmm_zscore": dict(workload="gmm", n=10**8, payload_bytes=4,
                       desc="plain z-score path on the 4-component mixture, 1e8 keys, u32 index"),
}
DEFAULT_CFG = dict(k=1024, cutoff=2048, max_zlevels=8, chunk=16384, tile=2048)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of the stable scatter's source text (its shared-memory layout and
    the kernel), the kernel whose counters the roofline's traffic comes from:
    a profile taken with other scatter code is not matched."""
    with open(os.path.join(ROOT, "paper_2605_14419_amd", "csrc", "zsort_kernels.hip")) as fh:
        src = fh.read()
    a = src.index("struct ScatSmem")
    b = src.index("// local sort of the leaf groups", a)
    return hashlib.sha256(src[a:b].encode()).hexdigest()[:16]


def stage_bytes(stats: dict, pw: int) -> dict:
    """Algorithmic HBM bytes per step of each kernel kind."""
    kp = 8 + pw
    mk = sum(stats["mkeys_per_level"])
    dk = sum(stats["keys_per_level"])
    return {"moments": 8.0 * mk, "finalize": 0.0, "hist": 8.0 * dk, "scatter": 2.0 * kp * dk,
            "local": 2.0 * kp * stats["local_keys"], "local_hard": 0.0}


def to_device(keys_np, pay_np, dev):
    import torch
    tk = torch.from_numpy(keys_np.view(np.int64)).to(dev)
    tp = None
    if pay_np is not None:
        v = pay_np.view(np.int32) if pay_np.dtype.itemsize == 4 else pay_np.view(np.int64)
        tp = torch.from_numpy(v).to(dev)
    return tk, tp


def verify_on_device(k_in, k_out, p_out):
    """sorted (unsigned), payload is a permutation carrying its key, stable"""
    from tests.invariants import check_stable_sorted_device
    check_stable_sorted_device(k_in, k_out, p_out)


def run_workload(spec, steps, warmup, cfg, dev, profile=True, autotune=False):
    import synth
    import torch
    import paper_2605_14419_amd as zs

    t0 = time.time()
    keys, pay = synth.make(spec["workload"], spec["n"], payload_bytes=spec["payload_bytes"])
    log(f"[bench] {spec['workload']} n={spec['n']} generated in {time.time() - t0:.1f}s")
    base_k, base_p = to_device(keys, pay, dev)
    del pay
    if cfg is None and not autotune:
        cfg = TUNED.get(spec["workload"])
    if cfg is None:  # the library's autotuner picks k / tile / chunk / cutoff
        cfg = zs.zsort_autotune(base_k, base_p)
        log(f"[bench] tuned {cfg}")
    ins = [(base_k.clone(), None if base_p is None else base_p.clone()) for _ in range(steps)]
    # untimed steps: the warmup, with every kernel kind timed (per-stage
    # times); the timed steps then bracket only the dominant kind with events,
    # since every event recorded between kernels costs a few microseconds
    nwarm = max(warmup, 1 if profile else 0)
    if profile:
        zs.zsort_profile_begin()
    for _ in range(nwarm):
        k = base_k.clone()
        p = None if base_p is None else base_p.clone()
        zs.zsort_stable_ex(k, p, cfg)
    torch.cuda.synchronize()
    kt_all = None
    if profile:
        kt_all = zs.zsort_profile_end()
        kt_all = {s: (v[0] / nwarm, v[1] / nwarm) for s, v in kt_all.items()}
        dom = max(STAGES, key=lambda s: kt_all[s][0])
        zs.zsort_profile_begin(stages=[dom])
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    ev0.record()
    for i in range(steps):
        evs[i].record()
        zs.zsort_stable_ex(ins[i][0], ins[i][1], cfg)
    evs[steps].record()
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    per_step = sorted(evs[i].elapsed_time(evs[i + 1]) for i in range(steps))
    med = per_step[steps // 2] if steps % 2 else 0.5 * (per_step[steps // 2 - 1] + per_step[steps // 2])
    kt = zs.zsort_profile_end() if profile else None
    stats = zs.zsort_get_last_stats()
    stats["ms_per_step_median"] = med
    assert stats["device_error"] == 0, stats
    verify_on_device(base_k, ins[-1][0], ins[-1][1])
    stats["kernel_ms_per_step"] = kt_all
    log(f"[bench] {spec['workload']}: {ms:.3f} ms/step, levels {stats['levels']}, verified")
    del ins
    torch.cuda.empty_cache()
    return keys, ms, stats, kt, cfg


def run_alpha(dev, n=10**7, alphas=(0.2, 0.4, 0.6, 0.8, 1.0, 1.2), steps=3):
    """The paper's sensitivity to k = alpha * sqrt(n) (its heuristics
    paragraph finds alpha = 0.6 best on a CPU), here on the GPU: uniform u64
    keys + u32 index at n = 10^7 (k up to 3795 clusters per pass, so 2048-key
    tiles), k held for every level as the method holds it."""
    import synth
    import torch
    import paper_2605_14419_amd as zs
    keys, pay = synth.make("uniform", n, payload_bytes=4)
    base_k, base_p = to_device(keys, pay, dev)
    rows = []
    for a in alphas:
        k = int(round(a * n ** 0.5))
        cfg = dict(k=k, cutoff=2048, max_zlevels=8, chunk=16384, tile=2048)
        tk, tp = base_k.clone(), base_p.clone()
        zs.zsort_stable_ex(tk, tp, cfg)
        ins = [(base_k.clone(), base_p.clone()) for _ in range(steps)]
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for i in range(steps):
            zs.zsort_stable_ex(ins[i][0], ins[i][1], cfg)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        st = zs.zsort_get_last_stats()
        assert st["device_error"] == 0, st
        verify_on_device(base_k, ins[-1][0], ins[-1][1])
        rows.append({"alpha": a, "k": k, "ms_per_step": round(ms, 4),
                     "gkeys_per_s": round(n / (ms * 1e-3) / 1e9, 3), "levels": st["levels"]})
        del ins
    log("[bench] alpha sweep: " + ", ".join(f"{r['alpha']}: {r['ms_per_step']:.3f} ms" for r in rows))
    return {"workload": f"{n} uniform u64 keys, u32 index; k = alpha*sqrt(n), cutoff 2048, "
                        "chunk 16384, 2048-key tiles", "rows": rows}


def run_batched(steps, warmup, dev, nseg=4096):
    """Batched form: nseg arrays in one segmented call replayed as a cached
    hipGraph, against a loop of plain single-array calls (one per segment)."""
    import synth
    import torch
    import paper_2605_14419_amd as zs

    keys, off, idx = synth.segments(nseg, synth.seed_for(3, 0))
    n = keys.size
    log(f"[bench] batched: {nseg} arrays, {n} keys")
    base_k, base_p = to_device(keys, idx, dev)
    toff = torch.from_numpy(off).to(dev)
    cfg = zs.zsort_autotune(base_k, base_p, toff)
    gcfg = dict(cfg, flags=zs.ZSORT_FLAG_GRAPH)
    bufs = [(base_k.clone(), base_p.clone()) for _ in range(steps)]
    for k, p in bufs:  # capture one graph per buffer pair (not timed)
        zs.zsort_stable_segmented(k, toff, p, gcfg)
    for _ in range(warmup):
        zs.zsort_stable_segmented(bufs[0][0], toff, bufs[0][1], gcfg)
    for k, p in bufs:
        k.copy_(base_k)
        p.copy_(base_p)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    for k, p in bufs:
        zs.zsort_stable_segmented(k, toff, p, gcfg)
    ev1.record()
    torch.cuda.synchronize()
    g_ms = ev0.elapsed_time(ev1) / steps
    st = zs.zsort_get_last_stats()
    assert st["device_error"] == 0, st
    gk = bufs[-1][0].cpu().numpy().view(np.uint64)
    # the loop of plain calls on views of each segment (same tuned config, paced)
    lk, lp = base_k.clone(), base_p.clone()
    offs = off.tolist()
    torch.cuda.synchronize()
    t0 = time.time()
    ev0.record()
    for i in range(nseg):
        a, b = offs[i], offs[i + 1]
        if b - a > 1:
            zs.zsort_stable_ex(lk[a:b], lp[a:b], cfg)
    ev1.record()
    torch.cuda.synchronize()
    l_ms = ev0.elapsed_time(ev1)
    log(f"[bench] batched graph {g_ms:.3f} ms/step, loop {l_ms:.1f} ms "
        f"(host {1e3 * (time.time() - t0):.1f} ms)")
    assert np.array_equal(lk.cpu().numpy().view(np.uint64), gk), "loop and graph keys disagree"
    assert torch.equal(lp, bufs[-1][1]), "loop and graph payloads disagree"
    # every segment sorted, stable and a permutation of its own keys
    from tests.invariants import check_segmented_stable_sorted_device
    check_segmented_stable_sorted_device(base_k, bufs[-1][0], bufs[-1][1], toff)
    del bufs
    torch.cuda.empty_cache()
    return {"workload": f"{nseg} arrays, lognormal lengths (median 2e4, [100, 1e6]), "
                        f"{n} u64 keys from per-array normals, u32 index payload",
            "n": n, "config": cfg,
            "graph_ms_per_step": round(g_ms, 4), "graph_gkeys_per_s": round(n / g_ms / 1e6, 3),
            "loop_ms_per_step": round(l_ms, 3), "loop_gkeys_per_s": round(n / l_ms / 1e6, 4),
            "speedup_vs_loop": round(l_ms / g_ms, 2)}


def run_counting(dev, n=10**7, steps=5):
    """Counting-sort termination for small key ranges (count_range = k): the
    recursion's depth and the time per sort with and without it, on keys of a
    restricted range, on narrow clusters among uniform keys, and on the
    duplicate-heavy and Zipf families."""
    import synth
    import torch
    import paper_2605_14419_amd as zs

    cfg = dict(k=256, cutoff=2048, max_zlevels=8, chunk=32768, tile=8192)
    rows = []
    for name in ("small_range", "clustered_ranges", "dup_heavy", "zipf"):
        keys, pay = synth.make(name, n, payload_bytes=4)
        base_k, base_p = to_device(keys, pay, dev)
        row = {"workload": name}
        for cr in (0, cfg["k"]):
            c = dict(cfg, count_range=cr)
            k, p = base_k.clone(), base_p.clone()
            zs.zsort_stable_ex(k, p, c)     # warm-up (workspace)
            ins = [(base_k.clone(), base_p.clone()) for _ in range(steps)]
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for a, b in ins:
                zs.zsort_stable_ex(a, b, c)
            e1.record()
            torch.cuda.synchronize()
            st = zs.zsort_get_last_stats()
            assert st["device_error"] == 0, st
            verify_on_device(base_k, ins[-1][0], ins[-1][1])
            tag = "with" if cr else "without"
            row[f"levels_{tag}"] = st["levels"]
            row[f"ms_{tag}"] = round(e0.elapsed_time(e1) / steps, 4)
            if cr:
                row["counted_subproblems"] = st["counted"]
            del ins
        rows.append(row)
        del base_k, base_p
        torch.cuda.empty_cache()
    log("[bench] counting: " + ", ".join(
        f"{r['workload']}: {r['levels_without']}->{r['levels_with']} levels, "
        f"{r['ms_without']:.3f}->{r['ms_with']:.3f} ms" for r in rows))
    return {"workload": f"{n} u64 keys + u32 index per family; count_range = k = {cfg['k']}",
            "config": cfg, "rows": rows}


def run_u128(dev, n=10**8, steps=4):
    """128-bit keys + u32 index at 10^8: time, GKeys/s and the levels of the
    high-word and low-word stages, beside the 64-bit path on the same words
    (uniform for random identifiers; for zero high words the low words
    themselves, lognormal)."""
    import synth
    import torch
    import paper_2605_14419_amd as zs

    cfg = TUNED["uniform_1e8"]
    rows = []
    for name in ("uuid", "prefix", "zext"):
        keys, idx = synth.make128(name, n)
        base_k = torch.from_numpy(keys.reshape(-1).view(np.int64)).to(dev)
        base_p = torch.from_numpy(idx.view(np.int32)).to(dev)
        del keys, idx
        k, p = base_k.clone(), base_p.clone()
        rep = zs.zsort_stable_u128(k, p, cfg, report=True)    # warm-up + the levels
        assert rep["device_error"] == 0, rep
        from tests.invariants import check_stable_sorted128_device
        check_stable_sorted128_device(base_k.view(-1, 2), k.view(-1, 2), p)
        del k, p
        ins = [(base_k.clone(), base_p.clone()) for _ in range(steps)]
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for a, b in ins:
            zs.zsort_stable_u128(a, b, cfg)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        row = {"workload": name, "ms_per_step": round(ms, 4),
               "gkeys_per_s": round(n / ms / 1e6, 3), "levels_high": rep["levels_high"],
               "levels_low": rep["levels_low"], "runs": rep["runs"],
               "short_runs": rep["short_runs"], "run_keys": rep["run_keys"]}
        # the 64-bit path on the same words: the high words (random ones for
        # identifiers) or, with zero high words, the low words
        w = base_k.view(-1, 2)[:, 1 if name != "zext" else 0].contiguous()
        ins64 = [(w.clone(), base_p.clone()) for _ in range(steps)]
        zs.zsort_stable_ex(w.clone(), base_p.clone(), cfg)
        torch.cuda.synchronize()
        e0.record()
        for a, b in ins64:
            zs.zsort_stable_ex(a, b, cfg)
        e1.record()
        torch.cuda.synchronize()
        st = zs.zsort_get_last_stats()
        row["u64_same_words_ms"] = round(e0.elapsed_time(e1) / steps, 4)
        row["u64_same_words_levels"] = st["levels"]
        rows.append(row)
        del ins, ins64, base_k, base_p, w
        torch.cuda.empty_cache()
    log("[bench] u128: " + ", ".join(
        f"{r['workload']}: {r['ms_per_step']:.3f} ms, levels {r['levels_high']}+{r['levels_low']} "
        f"(64-bit words: {r['u64_same_words_levels']} levels, {r['u64_same_words_ms']:.3f} ms)"
        for r in rows))
    return {"workload": f"{n} 128-bit keys + u32 index (uuid: both words uniform; prefix: 1000 "
                        "high words; zext: high word 0, low word lognormal)",
            "config": cfg, "rows": rows}


def run_learned(steps, warmup, dev, n=10**8):
    """Learned first-pass map on the 4-component mixture (narrow heavy
    component mid-range), against the z-score map: whole-sort time with the
    model fitted inside every call, time with a fitted model reused, and the
    first-pass imbalance (largest cluster / mean) of both maps at 4096
    clusters."""
    import synth
    import torch
    import paper_2605_14419_amd as zs

    keys, pay = synth.make("gmm", n, payload_bytes=4)
    base_k, base_p = to_device(keys, pay, dev)
    del keys, pay
    cfg = TUNED["learned"]   # each line in its own recorded configuration
    par = torch.empty(zs.MLP_PARAMS_BYTES, dtype=torch.uint8, device=dev)
    k, p = base_k.clone(), base_p.clone()
    diag = zs.zsort_stable_learned(k, p, cfg, dict(flags=zs.ZSORT_LEARNED_ZSCORE_DIAG),
                                   params_out=par)
    verify_on_device(base_k, k, p)
    del k, p
    reuse = dict(params=par, smin=diag["smin_out"], smax=diag["smax_out"])

    def timed(lcfg):
        ins = [(base_k.clone(), base_p.clone()) for _ in range(steps)]
        for _ in range(warmup):
            zs.zsort_stable_learned(base_k.clone(), base_p.clone(), cfg, lcfg)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record()
        reps = [zs.zsort_stable_learned(ins[i][0], ins[i][1], cfg, lcfg) for i in range(steps)]
        ev1.record()
        torch.cuda.synchronize()
        verify_on_device(base_k, ins[-1][0], ins[-1][1])
        del ins
        torch.cuda.empty_cache()
        return ev0.elapsed_time(ev1) / steps, reps

    ms_fit, reps = timed(None)
    ms_train, reps_t = timed(dict(steps=16))   # the initialisation refined by 16 Adam steps
    ms_reuse, reps2 = timed(reuse)
    st = zs.zsort_get_last_stats()
    ms_512, reps3 = timed(dict(reuse, buckets=512))
    log(f"[bench] learned: {ms_fit:.3f} ms/step fitted per call, {ms_reuse:.3f} reused; imbalance "
        f"{diag['imbalance_learned']:.2f} vs z-score {diag['imbalance_zscore']:.1f}")
    return {"workload": f"{n} u64 keys, 4-component mixture (narrow heavy component mid-range), "
                        "u32 index payload, 4096 first-pass clusters",
            "config": cfg,
            "ms_per_step": round(ms_fit, 4), "gkeys_per_s": round(n / ms_fit / 1e6, 3),
            "ms_per_step_model_reused": round(ms_reuse, 4),
            "gkeys_per_s_model_reused": round(n / ms_reuse / 1e6, 3),
            "ms_per_step_model_reused_512_clusters": round(ms_512, 4),
            "gkeys_per_s_model_reused_512_clusters": round(n / ms_512 / 1e6, 3),
            "fit_ms": round(sum(r["train_ms"] for r in reps) / len(reps), 4),
            "first_pass_ms": round(sum(r["first_pass_ms"] for r in reps2) / len(reps2), 4),
            "imbalance_learned": round(diag["imbalance_learned"], 3),
            "imbalance_zscore": round(diag["imbalance_zscore"], 3),
            "used_learned": sum(r["used_learned"] for r in reps + reps_t + reps2 + reps3),
            "fallbacks": sum(r["fallback"] for r in reps + reps_t + reps2 + reps3),
            "adam_steps": reps[0]["steps"],
            "ms_per_step_with_16_adam_steps": round(ms_train, 4),
            "fit_ms_with_16_adam_steps": round(sum(r["train_ms"] for r in reps_t) / len(reps_t), 4),
            "trained_kept_of_16_step_fits": f"{sum(r['trained'] for r in reps_t)}/{len(reps_t)}",
            "sample_max_cluster_init_vs_trained": [reps_t[0]["sample_max_init"],
                                                   reps_t[0]["sample_max_trained"]],
            "levels": st["levels"], "calls": len(reps) + len(reps_t) + len(reps2) + len(reps3)}


def roofline(kt, stats, pw, steps, traffic_file, cfg):
    per_step = stage_bytes(stats, pw)
    dom = max(STAGES, key=lambda s: kt[s][0])
    tot_ms, launches = kt[dom]
    bytes_per_launch = per_step[dom] * steps / launches
    avg_ms = tot_ms / launches
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    traffic = None
    if os.path.exists(traffic_file):
        with open(traffic_file) as fh:
            tr = json.load(fh)
        if tr.get("kernel_hash") == kernel_source_hash():
            for ent in tr.get("entries", []):
                if ent.get("stage") == dom and all(ent.get("config", {}).get(x) == cfg.get(x)
                                                   for x in ("k", "tile", "chunk", "cutoff")):
                    traffic = ent.get("bytes_per_launch")
    return {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "algorithmic_bytes_per_launch": bytes_per_launch, "avg_launch_ms": avg_ms,
            "launches": launches}


# kernel -> stage; the local stage launches up to three kernels (wave and
# block jobs, one wave per group up to 1024 keys, block jobs above 2048 keys):
# the first counts the launches
STAGE_OF_KERNEL = (("k_moments", "moments"), ("k_finalize", "finalize"), ("k_hist", "hist"),
                   ("k_scatter", "scatter"), ("k_local_hard", "local_hard"),
                   ("k_local_mid", "local"), ("k_local_big", "local"), ("k_local", "local"))
SECOND_KERNELS = ("k_local_mid", "k_local_big")


def _stage_of(name):
    for pat, st in STAGE_OF_KERNEL:
        if pat + "<" in name or pat + "(" in name:
            return st
    return None


def _is_second(name):
    return any(p + "<" in name or p + "(" in name for p in SECOND_KERNELS)


def _csv(dirname, suffix):
    import csv
    import glob
    files = sorted(glob.glob(os.path.join(dirname, "**", "*" + suffix), recursive=True))
    if not files:
        raise SystemExit(f"no *{suffix} under {dirname}")
    with open(files[0]) as fh:
        return list(csv.DictReader(fh))


def summarize_profiles(d, workload, cfg):
    """Turns the csv output of three rocprofv3 runs of this script (kernel
    trace + stats; FETCH_SIZE; WRITE_SIZE, both with --copy-probe) into the
    text summaries kept beside the code.  `d` holds kt/, fetch/, write/ and
    commands.txt (one "kt: ...", "fetch: ...", "write: ..." line each)."""
    cmds = {}
    with open(os.path.join(d, "commands.txt")) as fh:
        for ln in fh:
            if ":" in ln:
                a, b = ln.split(":", 1)
                cmds[a.strip()] = b.strip()
    out_dir = os.path.join(ROOT, "profiles")
    os.makedirs(out_dir, exist_ok=True)
    # kernel time
    rows = _csv(os.path.join(d, "kt"), "_kernel_stats.csv")
    lines = [f"# Kernel time, {workload}", "", "Command (from the repository root):", "",
             "    " + cmds.get("kt", "?"), "",
             "| kernel | stage | calls | total ms | avg us | % |", "|---|---|---|---|---|---|"]
    per_stage = {}
    for r in rows:
        st = _stage_of(r["Name"]) or "-"
        nm = r["Name"].replace("void ", "").replace("(zs::Ws, int)", "").replace("|", "/")
        lines.append(f"| `{nm[:70]}` | {st} | {r['Calls']} | {int(r['TotalDurationNs']) / 1e6:.3f} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {r['Percentage']} |")
        if st != "-":
            a = per_stage.setdefault(st, [0, 0])
            a[0] += int(r["TotalDurationNs"])
            if not _is_second(r["Name"]):
                a[1] += int(r["Calls"])
    lines += ["", "Per stage (all template instances; the local stage's calls count its first "
              "kernel):", "", "| stage | calls | total ms | avg us |",
              "|---|---|---|---|"]
    for st, (ns, c) in sorted(per_stage.items(), key=lambda x: -x[1][0]):
        lines.append(f"| {st} | {c} | {ns / 1e6:.3f} | {ns / c / 1e3:.1f} |")
    tag = f"{workload}_k{cfg['k']}_c{cfg['cutoff']}_ch{cfg['chunk']}_t{cfg['tile']}"
    with open(os.path.join(out_dir, f"kernels_{tag}.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    # HBM traffic, calibrated on the copy probe (1 GiB read + 1 GiB written per copy)
    def counter(sub, cname):
        per = {}
        probe = []
        for r in _csv(os.path.join(d, sub), "_counter_collection.csv"):
            if r["Counter_Name"] != cname:
                continue
            kib = float(r["Counter_Value"])
            if "copyBuffer" in r["Kernel_Name"] and len(probe) < 3:
                probe.append(kib)   # the probe's three copies run before anything else
            st = _stage_of(r["Kernel_Name"])
            if st:
                a = per.setdefault(st, [0.0, 0])
                a[0] += kib
                if not _is_second(r["Kernel_Name"]):
                    a[1] += 1
        return per, probe
    fetch, fprobe = counter("fetch", "FETCH_SIZE")
    write, wprobe = counter("write", "WRITE_SIZE")
    gib_kib = float(1 << 20)
    ff = gib_kib / (sum(fprobe) / len(fprobe))
    wf = gib_kib / (sum(wprobe) / len(wprobe))
    lines = [f"# HBM traffic per launch, {workload}", "",
             "Commands (from the repository root):", "", "    " + cmds.get("fetch", "?"),
             "    " + cmds.get("write", "?"), "",
             f"Copy probe (1 GiB read, 1 GiB written per copy): FETCH_SIZE reads "
             f"{sum(fprobe) / len(fprobe) / 1024:.1f} MiB -> factor {ff:.3f}; WRITE_SIZE reads "
             f"{sum(wprobe) / len(wprobe) / 1024:.1f} MiB -> factor {wf:.3f}.", "",
             "| stage | launches | fetch MB/launch (scaled) | write MB/launch (scaled) | total MB/launch "
             "| avg launch us (kernel trace) | traffic GB/s |",
             "|---|---|---|---|---|---|---|"]
    traffic = {}
    for st in STAGES:
        if st not in fetch or st not in write:
            continue
        fb = fetch[st][0] / fetch[st][1] * 1024 * ff
        wb = write[st][0] / write[st][1] * 1024 * wf
        traffic[st] = fb + wb
        us = per_stage[st][0] / per_stage[st][1] / 1e3 if st in per_stage else 0.0
        gbs = (fb + wb) / (us * 1e-6) / 1e9 if us > 0 else 0.0
        lines.append(f"| {st} | {fetch[st][1]} | {fb / 1e6:.1f} | {wb / 1e6:.1f} | {(fb + wb) / 1e6:.1f} "
                     f"| {us:.1f} | {gbs:.0f} |")
    with open(os.path.join(out_dir, f"traffic_{tag}.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    dom = max(per_stage, key=lambda s: per_stage[s][0])
    # one entry per configuration (the autotuner's pick can differ between
    # runs); entries taken with other kernel sources are dropped
    jpath = os.path.join(out_dir, f"traffic_{workload}.json")
    entries = []
    if os.path.exists(jpath):
        with open(jpath) as fh:
            old = json.load(fh)
        if old.get("kernel_hash") == kernel_source_hash():
            entries = [e for e in old.get("entries", []) if e.get("config") != cfg]
    entries.append({"stage": dom, "config": cfg, "summary": f"traffic_{tag}.md",
                    "bytes_per_launch": round(traffic.get(dom, 0.0)),
                    "per_stage_bytes_per_launch": {k: round(v) for k, v in traffic.items()},
                    "fetch_factor": ff, "write_factor": wf})
    with open(jpath, "w") as fh:
        json.dump({"kernel_hash": kernel_source_hash(), "entries": entries}, fh, indent=1)
    print(f"wrote kernels_{tag}.md, traffic_{tag}.md, traffic_{workload}.json (dominant {dom})")


def summarize_trace(d, label):
    """Kernel time only, from one rocprofv3 kernel-trace run of this script
    (`d` holds kt/ and commands.txt with a "kt: ..." line): the summary of an
    extra line (learned map, batched graph, 128-bit keys), whose kernels are
    not all distribution stages."""
    cmds = {}
    with open(os.path.join(d, "commands.txt")) as fh:
        for ln in fh:
            if ":" in ln:
                a, b = ln.split(":", 1)
                cmds[a.strip()] = b.strip()
    rows = _csv(os.path.join(d, "kt"), "_kernel_stats.csv")
    lines = [f"# Kernel time, {label}", "", "Command (from the repository root):", "",
             "    " + cmds.get("kt", "?"), "",
             "| kernel | stage | calls | total ms | avg us | % |", "|---|---|---|---|---|---|"]
    for r in rows:
        st = _stage_of(r["Name"]) or "-"
        nm = r["Name"].replace("void ", "").replace("(zs::Ws, int)", "").replace("|", "/")
        lines.append(f"| `{nm[:70]}` | {st} | {r['Calls']} | {int(r['TotalDurationNs']) / 1e6:.3f} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {r['Percentage']} |")
    out = os.path.join(ROOT, "profiles", f"kernels_{label}.md")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(f"wrote {os.path.relpath(out, ROOT)}")


def summarize_counters(d, label):
    """Hardware counters per distribution stage, from rocprofv3 --pmc runs of
    this script (`d` holds p1/, p2/, ... and commands.txt with one "pN: ..."
    line per pass): totals over every launch of the stage, and the ratios
    that say where its time goes."""
    cmds = []
    with open(os.path.join(d, "commands.txt")) as fh:
        cmds = [ln.strip() for ln in fh if ln.strip()]
    agg = {}
    for sub in sorted(os.listdir(d)):
        if not os.path.isdir(os.path.join(d, sub)):
            continue
        for r in _csv(os.path.join(d, sub), "_counter_collection.csv"):
            st = _stage_of(r["Kernel_Name"])
            if st:
                a = agg.setdefault(st, {})
                a[r["Counter_Name"]] = a.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    names = sorted({c for a in agg.values() for c in a})
    lines = [f"# Hardware counters, {label}", "", "Commands (from the repository root):", ""]
    lines += ["    " + c.split(":", 1)[1].strip() for c in cmds]
    lines += ["", "Totals over every launch of each stage (all profiled sorts):", "",
              "| stage | " + " | ".join(names) + " |", "|---|" + "---|" * len(names)]
    for st in STAGES:
        if st in agg:
            lines.append(f"| {st} | " + " | ".join(f"{agg[st].get(c, 0):.3g}" for c in names) + " |")
    def ratio(a, x, y):
        return a[x] / a[y] if a.get(y) and x in a else float("nan")
    lines += ["", "Ratios: waves waiting (SQ_WAIT_ANY / SQ_WAVE_CYCLES), VALU instructions "
              "per wave cycle, LDS bank-conflict cycles per LDS-active cycle, share of 64-byte "
              "write requests, share of 128-byte read requests.", "",
              "| stage | waiting | VALU / wave cycle | LDS conflict / active | 64 B writes | 128 B reads |",
              "|---|---|---|---|---|---|"]
    for st in STAGES:
        if st not in agg:
            continue
        a = agg[st]
        lines.append(f"| {st} | {ratio(a, 'SQ_WAIT_ANY', 'SQ_WAVE_CYCLES'):.2f} | "
                     f"{ratio(a, 'SQ_INSTS_VALU', 'SQ_WAVE_CYCLES'):.3f} | "
                     f"{ratio(a, 'SQ_LDS_BANK_CONFLICT', 'SQ_ACTIVE_INST_LDS'):.2f} | "
                     f"{ratio(a, 'TCC_EA0_WRREQ_64B_sum', 'TCC_EA0_WRREQ_sum'):.2f} | "
                     f"{ratio(a, 'TCC_EA0_RDREQ_128B_sum', 'TCC_EA0_RDREQ_sum'):.2f} |")
    out = os.path.join(ROOT, "profiles", f"counters_{label}.md")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(f"wrote {os.path.relpath(out, ROOT)}")


def measured_copy_gbs(dev, reps=5):
    """Achievable HBM bandwidth on this GPU: a 1 GiB device-to-device copy
    (1 GiB read + 1 GiB written), median of `reps`, in GB/s of read + write."""
    import torch
    src = torch.empty(1 << 27, dtype=torch.int64, device=dev).fill_(3)
    dst = torch.empty_like(src)
    dst.copy_(src)
    times = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    del src, dst
    torch.cuda.empty_cache()
    t = sorted(times)[reps // 2]
    return round(2 * (1 << 30) / (t * 1e-3) / 1e9, 1)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_library_reference(keys, budget_s=3.0):
    """numpy's stable argsort (a library sort, not the method) on the same
    sample, single-threaded: context for the oracle's number."""
    ns = min(keys.size, 10**7)
    sample = np.ascontiguousarray(keys[:ns])
    reps, t0 = 0, time.time()
    while True:
        order = np.argsort(sample, kind="stable")
        sample[order]
        reps += 1
        el = time.time() - t0
        if el >= budget_s or reps >= 10:
            break
    return {"value": round(ns * reps / el / 1e9, 5), "unit": "GKeys/s", "cores": 1,
            "kind": "numpy argsort(kind='stable') + gather",
            "sample": f"first {ns} keys of the same array, {reps} rep(s)"}


def cpu_baseline(keys, cfg, budget_s):
    """The oracle as it stands, single-threaded, on the first 10^7 keys of the
    workload: with Algorithm 1's own settings (k = floor(sqrt(n)) clusters per
    pass, insertion sort at <= 96 keys) as the baseline, and with the GPU's
    configuration beside it (half the budget each)."""
    import oracle
    ns = min(keys.size, 10**7)
    sample = np.ascontiguousarray(keys[:ns])
    idx = np.arange(ns, dtype=np.uint32)

    def timed(par):
        reps, t0 = 0, time.time()
        while True:
            oracle.sort(sample, idx, k=par["k"], cutoff=par["cutoff"],
                        max_zlevels=par["max_zlevels"])
            reps += 1
            el = time.time() - t0
            if el >= budget_s / 2 or reps >= 20:
                return round(ns * reps / el / 1e9, 5), reps, el

    paper = oracle.paper_params(ns)
    v, reps, el = timed(paper)
    vg, repg, elg = timed(cfg)
    return {"value": v, "unit": "GKeys/s", "cores": 1, "kind": "oracle",
            "settings": f"Algorithm 1: k = floor(sqrt(n)) = {paper['k']} clusters per pass, "
                        f"insertion sort at <= {paper['cutoff']} keys",
            "cpu_model": cpu_model(),
            "sample": f"first {ns} keys of the same array, u32 index payload, {reps} rep(s), "
                      f"{el:.1f}s single-threaded",
            "gpu_config": {"value": vg, "unit": "GKeys/s",
                           "settings": f"the GPU's configuration: k {cfg['k']}, cutoff "
                                       f"{cfg['cutoff']}, max_zlevels {cfg['max_zlevels']}",
                           "sample": f"the same sample, {repg} rep(s), {elg:.1f}s"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--extras", default=",".join(list(EXTRAS) + ["learned", "batched", "alpha",
                                                                "counting", "u128"]),
                    help="comma list, or 'none'")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--n", type=int, default=PRIMARY["n"])
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device-to-device copy (counter calibration)")
    ap.add_argument("--config", default=None,
                    help="fixed configuration for the primary workload instead of the "
                         "autotuner's, e.g. k=256,cutoff=2048,chunk=32768,tile=4096")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("DIR", "LABEL"),
                    help="write profiles/counters_LABEL.md from rocprofv3 --pmc runs in DIR")
    ap.add_argument("--summarize-trace", nargs=2, metavar=("DIR", "LABEL"),
                    help="write profiles/kernels_LABEL.md from one kernel-trace run in DIR")
    ap.add_argument("--summarize-profiles", metavar="DIR",
                    help="write profiles/ summaries from rocprofv3 csv output and exit")
    ap.add_argument("--autotune", action="store_true",
                    help="time the autotuner's candidates instead of the recorded configurations")
    ap.add_argument("--workload", default="primary",
                    help="workload of the main line: primary (lognormal + u64 index) or one of "
                         + ", ".join(EXTRAS) + " (profiling runs)")
    args = ap.parse_args()
    if args.summarize_trace:
        summarize_trace(*args.summarize_trace)
        return
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters)
        return
    if args.summarize_profiles:
        if not args.config:
            raise SystemExit("--summarize-profiles needs the --config the profiled runs used")
        pc = dict(DEFAULT_CFG)
        for kv in args.config.split(","):
            a, b = kv.split("=")
            pc[a.strip()] = int(b)
        wl = PRIMARY if args.workload == "primary" else EXTRAS[args.workload]
        summarize_profiles(args.summarize_profiles, wl["workload"], pc)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE "
              f"{world}); the multi-GPU sharding is a design note, not built.", flush=True)
        sys.exit(2)

    import torch
    import paper_2605_14419_amd as zs
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    zs.lib()  # fails loudly if the HIP library is missing
    dev = torch.device("cuda:0")
    spec = dict(PRIMARY if args.workload == "primary" else EXTRAS[args.workload])
    if args.workload == "primary":
        spec["n"] = args.n

    if args.copy_probe:
        src = torch.empty(1 << 27, dtype=torch.int64, device=dev).fill_(7)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("[bench] copy probe: 3 x 1 GiB device-to-device copies")
    copy_gbs = measured_copy_gbs(dev)
    log(f"[bench] measured copy bandwidth {copy_gbs} GB/s (read + write)")
    fixed = None
    if args.config:
        fixed = dict(DEFAULT_CFG)
        for kv in args.config.split(","):
            a, b = kv.split("=")
            fixed[a.strip()] = int(b)
    keys, ms, stats, kt, cfg = run_workload(spec, args.steps, args.warmup, fixed, dev,
                                            autotune=args.autotune)
    pw = spec["payload_bytes"]
    n = spec["n"]
    value = n / (ms * 1e-3) / 1e9
    model = stats["model_bytes"]
    rl = roofline(kt, stats, pw, args.steps,
                  os.path.join(ROOT, "profiles", f"traffic_{spec['workload']}.json"), cfg)
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "GKeys/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": spec["desc"], "n": n, "payload_bytes": pw, **cfg},
        "hbm_frac_effective": round(model / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "hbm_frac_sort_equivalent": round(2 * (8 + pw) * n / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "model_bytes_per_step": model,
        "ms_per_step_median": round(stats["ms_per_step_median"], 4),
        "hbm": {"peak_gbs": HBM_PEAK_GBS, "measured_copy_gbs": copy_gbs,
                "effective_frac_of_copy": round(model / (ms * 1e-3) / 1e9 / copy_gbs, 4)},
        "levels": stats["levels"],
        "keys_per_level": stats.get("keys_per_level"),
        "kernel_ms_per_step": {s: round(stats["kernel_ms_per_step"][s][0], 4) for s in STAGES},
        "kernel_ms_per_step_from": "untimed warmup steps with every kernel kind timed",
        "roofline": rl,
    }
    extras = {}
    if args.extras and args.extras != "none":
        for name in args.extras.split(","):
            if name == "batched":
                extras[name] = run_batched(max(3, args.steps // 2), 1, dev)
                continue
            if name == "alpha":
                extras[name] = run_alpha(dev)
                continue
            if name == "counting":
                extras[name] = run_counting(dev)
                continue
            if name == "u128":
                extras[name] = run_u128(dev)
                continue
            if name == "learned":
                extras[name] = run_learned(max(3, args.steps // 2), 1, dev)
                if "gmm_zscore" in extras:
                    z = extras["gmm_zscore"]["ms_per_step"]
                    extras[name]["zscore_ms_per_step_same_keys"] = z
                    extras[name]["speedup_vs_zscore_model_reused"] = round(
                        z / extras[name]["ms_per_step_model_reused"], 3)
                continue
            es = EXTRAS[name]
            esteps = max(3, args.steps // 2)
            ek, ems, est, ekt, ecfg = run_workload(es, esteps, 1, None, dev, autotune=args.autotune)
            del ek
            epw = es["payload_bytes"]
            extras[name] = {
                "workload": es["desc"], "gkeys_per_s": round(es["n"] / (ems * 1e-3) / 1e9, 3),
                "ms_per_step": round(ems, 4),
                "hbm_frac_effective": round(est["model_bytes"] / (ems * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "hbm_frac_sort_equivalent": round(2 * (8 + epw) * es["n"] / (ems * 1e-3) / 1e9
                                                  / HBM_PEAK_GBS, 4),
                "levels": est["levels"], "config": ecfg,
                "kernel_ms_per_step": {s: round(est["kernel_ms_per_step"][s][0], 4)
                                       for s in STAGES},
                "roofline": roofline(ekt, est, epw, esteps,
                                     os.path.join(ROOT, "profiles",
                                                  f"traffic_{es['workload']}.json"), ecfg),
            }
    out["extras"] = extras
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(keys, cfg, args.cpu_budget)
        out["cpu_library_reference"] = cpu_library_reference(keys)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
