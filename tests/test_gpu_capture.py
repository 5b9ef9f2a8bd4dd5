"""The boundary's memory rules on the GPU: a caller capturing zsort_stable_*
into a graph of its own, the caller-owned workspace that makes that possible
at a new shape, and the out-of-memory path.

Each graph is replayed several times with eager work of the program's own and
synchronisations between the replays; every replay's output is compared with
an eager call's and with the CPU oracle.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
zs = pytest.importorskip("paper_2605_14419_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
CFG = dict(k=512, cutoff=1024, max_zlevels=8, chunk=32768, tile=8192)


def say(*a):
    print(*a, flush=True)


def dev(keys, idx):
    return (torch.from_numpy(keys.view(np.int64)).to(DEV),
            torch.from_numpy(idx.view(np.int32)).to(DEV))


def capture(fn, stream):
    g = torch.cuda.CUDAGraph()
    err = None
    with torch.cuda.graph(g, stream=stream, capture_error_mode="thread_local"):
        try:
            fn()
        except zs.ZsortError as e:   # end the capture normally, report afterwards
            err = e
    return g, err


def test_capture_without_workspace_at_a_new_shape_is_refused():
    keys, idx = synth.make("normal", 200_000)
    tk, tp = dev(keys, idx)
    s = torch.cuda.Stream()
    say("case capture refused")
    g, err = capture(lambda: zs.zsort_stable_ex(tk, tp, CFG, stream=s), s)
    assert err is not None and err.code == zs.ZSORT_ECAPTURE
    torch.cuda.synchronize()
    # nothing ran: the keys are untouched
    assert np.array_equal(tk.cpu().numpy().view(np.uint64), keys)


@pytest.mark.parametrize("n,segmented", [(300_001, False), (2**20, False), (250_000, True)])
def test_caller_workspace_makes_capture_work_and_replays_match(n, segmented):
    keys, idx = synth.make("lognormal", n)
    off = None
    if segmented:
        cut = np.sort(np.random.default_rng(3).choice(np.arange(1, n), size=40, replace=False))
        off = np.concatenate([[0], cut, [n]]).astype(np.int64)
        idx = np.concatenate([np.arange(off[i + 1] - off[i], dtype=np.uint32)
                              for i in range(off.size - 1)])
    base_k, base_p = dev(keys, idx)
    toff = None if off is None else torch.from_numpy(off).to(DEV)
    s = torch.cuda.Stream()
    nseg = 0 if off is None else off.size - 1
    need = zs.zsort_workspace_bytes(n, 4, nseg, CFG)
    assert need > 0
    ws = torch.empty(need + 4096, dtype=torch.uint8, device=DEV)
    ws_ptr = ws.data_ptr()
    aligned = ws[(256 - ws_ptr % 256) % 256:]
    zs.zsort_set_workspace(aligned, stream=s)
    say(f"case capture n={n} segmented={segmented} ws={need}")
    try:
        tk, tp = base_k.clone(), base_p.clone()

        def call():
            if segmented:
                zs.zsort_stable_segmented(tk, toff, tp, CFG, stream=s)
            else:
                zs.zsort_stable_ex(tk, tp, CFG, stream=s)

        g, err = capture(call, s)
        assert err is None, err
        # eager reference on other buffers, default stream (its own workspace)
        ek, ep = base_k.clone(), base_p.clone()
        if segmented:
            zs.zsort_stable_segmented(ek, toff, ep, CFG)
            ok, oi = oracle.sort_segmented(keys, off, idx, k=CFG["k"], cutoff=CFG["cutoff"],
                                           max_zlevels=8)
        else:
            zs.zsort_stable_ex(ek, ep, CFG)
            ok, oi, _ = oracle.sort(keys, idx, k=CFG["k"], cutoff=CFG["cutoff"], max_zlevels=8)
        torch.cuda.synchronize()
        assert np.array_equal(ek.cpu().numpy().view(np.uint64), ok)
        assert np.array_equal(ep.cpu().numpy().view(np.uint32), oi)
        junk = torch.randint(0, 2**62, (1 << 20,), device=DEV)
        for rep in range(4):
            tk.copy_(base_k)
            tp.copy_(base_p)
            junk.add_(rep)                      # the program's own work between replays
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(tk, ek) and torch.equal(tp, ep), f"replay {rep}"
        # an eager call on the captured stream (same workspace) still agrees
        tk.copy_(base_k)
        tp.copy_(base_p)
        call()
        torch.cuda.synchronize()
        assert torch.equal(tk, ek) and torch.equal(tp, ep)
    finally:
        torch.cuda.synchronize()
        zs.zsort_set_workspace(None, stream=s)


def test_small_caller_workspace_gives_enomem_and_never_allocates():
    keys, idx = synth.make("uniform", 500_000)
    tk, tp = dev(keys, idx)
    s = torch.cuda.Stream()
    small = torch.empty(zs.zsort_workspace_bytes(10_000, 4, 0, CFG), dtype=torch.uint8,
                        device=DEV)
    zs.zsort_set_workspace(small, stream=s)
    say("case small workspace")
    try:
        with pytest.raises(zs.ZsortError) as ei:
            zs.zsort_stable_ex(tk, tp, CFG, stream=s)
        assert ei.value.code == zs.ZSORT_ENOMEM
        torch.cuda.synchronize()
        assert np.array_equal(tk.cpu().numpy().view(np.uint64), keys)
        # a shape that fits runs in it
        k2, p2 = tk[:9000].clone(), tp[:9000].clone()
        zs.zsort_stable_ex(k2, p2, CFG, stream=s)
        torch.cuda.synchronize()
        ok, oi, _ = oracle.sort(keys[:9000], idx[:9000], k=CFG["k"], cutoff=CFG["cutoff"],
                                max_zlevels=8)
        assert np.array_equal(k2.cpu().numpy().view(np.uint64), ok)
        assert np.array_equal(p2.cpu().numpy().view(np.uint32), oi)
    finally:
        torch.cuda.synchronize()
        zs.zsort_set_workspace(None, stream=s)


def test_allocation_failure_gives_enomem_then_recovers():
    keys, idx = synth.make("uniform", 400_000)
    tk, tp = dev(keys, idx)
    s = torch.cuda.Stream()
    say("case alloc limit")
    zs.zsort_set_alloc_limit(1 << 20)
    try:
        with pytest.raises(zs.ZsortError) as ei:
            zs.zsort_stable_ex(tk, tp, CFG, stream=s)
        assert ei.value.code == zs.ZSORT_ENOMEM
    finally:
        zs.zsort_set_alloc_limit(0)
    torch.cuda.synchronize()
    assert np.array_equal(tk.cpu().numpy().view(np.uint64), keys)
    zs.zsort_stable_ex(tk, tp, CFG, stream=s)
    torch.cuda.synchronize()
    ok, oi, _ = oracle.sort(keys, idx, k=CFG["k"], cutoff=CFG["cutoff"], max_zlevels=8)
    assert np.array_equal(tk.cpu().numpy().view(np.uint64), ok)
    assert np.array_equal(tp.cpu().numpy().view(np.uint32), oi)
