"""GPU tests of the batched (segmented) form, its hipGraph mode and the
autotuner, against the CPU oracle.

Graph replays are checked one by one, with eager work and synchronisations
of the program's own between them, and each replay's output is compared with
the eager (non-graph) result and with the oracle.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
zs = pytest.importorskip("paper_2605_14419_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)


def dev_arrays(keys, pay):
    tk = torch.from_numpy(keys.view(np.int64)).to(DEV)
    tp = torch.from_numpy(pay.view(np.int32)).to(DEV)
    return tk, tp


def host(tk, tp):
    return tk.cpu().numpy().view(np.uint64), tp.cpu().numpy().view(np.uint32)


@pytest.fixture(scope="module")
def batch():
    keys, off, idx = synth.segments(600, 4242, median=2e4, hi=200_000)
    cfg = dict(k=1024, cutoff=2048, max_zlevels=8, chunk=16384, tile=2048)
    ok, oi = oracle.sort_segmented(keys, off, idx, k=1024, cutoff=2048, max_zlevels=8)
    return keys, off, idx, cfg, ok, oi


def test_graph_replays_match_eager_and_oracle(batch):
    keys, off, idx, cfg, ok, oi = batch
    say(f"case graph n={keys.size} segments={off.size - 1}")
    pristine_k, pristine_p = dev_arrays(keys, idx)
    toff = torch.from_numpy(off).to(DEV)
    # eager reference on its own buffers
    ek, ep = pristine_k.clone(), pristine_p.clone()
    zs.zsort_stable_segmented(ek, toff, ep, cfg)
    torch.cuda.synchronize()
    eager = host(ek, ep)
    assert np.array_equal(eager[0], ok) and np.array_equal(eager[1], oi)
    gcfg = dict(cfg, flags=zs.ZSORT_FLAG_GRAPH)
    gk, gp = pristine_k.clone(), pristine_p.clone()
    for rep in range(4):
        gk.copy_(pristine_k)
        gp.copy_(pristine_p)
        torch.cuda.synchronize()
        zs.zsort_stable_segmented(gk, toff, gp, gcfg)   # first call captures, later replay
        torch.cuda.synchronize()
        st = zs.zsort_get_last_stats()
        assert st["device_error"] == 0, st
        got = host(gk, gp)
        assert np.array_equal(got[0], eager[0]) and np.array_equal(got[1], eager[1]), rep
        # unrelated eager work of the program between replays
        xk, xp = pristine_k.clone(), pristine_p.clone()
        zs.zsort_stable_segmented(xk, toff, xp, cfg)
        (xk.float() * 2).sum().item()
        torch.cuda.synchronize()


def test_graph_single_array_replays():
    x, idx = synth.make("normal", 2_000_003)
    say("case graph single")
    base_k, base_p = dev_arrays(x, idx)
    ok, oi, _ = oracle.sort(x, idx, k=512, cutoff=2048, max_zlevels=8)
    cfg = dict(k=512, cutoff=2048, max_zlevels=8, chunk=32768, tile=4096,
               flags=zs.ZSORT_FLAG_GRAPH)
    tk, tp = base_k.clone(), base_p.clone()
    for rep in range(3):
        tk.copy_(base_k)
        tp.copy_(base_p)
        torch.cuda.synchronize()
        zs.zsort_stable_ex(tk, tp, cfg)
        torch.cuda.synchronize()
        gk, gp = host(tk, tp)
        assert np.array_equal(gk, ok) and np.array_equal(gp, oi), rep


def test_autotune_picks_valid_config_and_sorts(tmp_path, batch):
    keys, off, idx, cfg, ok, oi = batch
    say("case autotune")
    tk, tp = dev_arrays(keys, idx)
    toff = torch.from_numpy(off).to(DEV)
    path = str(tmp_path / "tune.txt")
    best = zs.zsort_autotune(tk, tp, toff, cache_path=path)
    assert best["k"] in (256, 512, 1024) and best["tile"] in (2048, 4096, 8192)
    assert best["cutoff"] in (1024, 2048)
    assert np.array_equal(host(tk, tp)[0], keys)         # input untouched
    lines = [ln for ln in open(path) if not ln.startswith("#")]
    assert len(lines) >= 1
    zs.zsort_stable_segmented(tk, toff, tp, None)         # uses the tuned entry
    torch.cuda.synchronize()
    got = host(tk, tp)
    assert np.array_equal(got[0], ok) and np.array_equal(got[1], oi)
    again = zs.zsort_autotune(tk, tp, toff, cache_path=path)   # known class: no re-timing
    assert again == best


def test_segmented_edge_shapes():
    """empty segments, single keys, segments at exactly the cutoff and one
    larger than a chunk, all in one call"""
    rng = np.random.default_rng(5)
    lens = [0, 1, 2, 0, 2048, 2049, 16384 * 3 + 7, 0, 1, 5000, 0]
    off = np.zeros(len(lens) + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    n = int(off[-1])
    keys = rng.integers(0, 2**64, size=n, dtype=np.uint64, endpoint=False)
    keys[off[4]:off[5]] = keys[off[4]]                    # one all-equal segment
    idx = np.arange(n, dtype=np.uint32)
    say("case segmented edges")
    for cfg in [dict(k=1024, cutoff=2048), dict(k=256, cutoff=64, chunk=2048),
                dict(k=256, cutoff=2048, flags=zs.ZSORT_FLAG_GRAPH)]:
        tk, tp = dev_arrays(keys, idx)
        zs.zsort_stable_segmented(tk, torch.from_numpy(off).to(DEV), tp, cfg)
        torch.cuda.synchronize()
        got = host(tk, tp)
        ok, oi = oracle.sort_segmented(keys, off, idx, k=cfg["k"], cutoff=cfg["cutoff"],
                                       max_zlevels=8)
        assert np.array_equal(got[0], ok) and np.array_equal(got[1], oi), cfg
