"""The allocation-free entry point (zsort_stable_noalloc) against the
allocating one (zsort_stable_ex), through the C-ABI: two calls in a row on the
shared per-GPU scratch array, the second with a smaller input, each bit for bit
equal to zsort_stable_ex's output; sizes beyond the array are refused without
touching the data."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
zs = pytest.importorskip("paper_2605_14419_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)


def dev(keys, pay):
    v = pay.view(np.int32) if pay.dtype.itemsize == 4 else pay.view(np.int64)
    return (torch.from_numpy(keys.view(np.int64)).to(DEV), torch.from_numpy(v).to(DEV))


@pytest.mark.parametrize("cfg,pw", [(None, 4),
                                    (dict(k=512, cutoff=1024, chunk=32768, tile=8192), 4),
                                    (dict(k=256, cutoff=4096, chunk=32768, tile=8192), 8),
                                    (dict(k=512, cutoff=1024, chunk=32768, tile=8192,
                                          flags=4), 4)])
def test_noalloc_matches_allocating_entry_point_twice(cfg, pw):
    runs = [("lognormal", 2**21 - 5 if pw == 8 else 3 * 10**6 + 7), ("dup_heavy", 100_003)]
    for name, n in runs:   # the second call is smaller than the first
        keys, idx = synth.make(name, n, payload_bytes=pw)
        need = zs.zsort_workspace_bytes(n, pw, 0, cfg)
        assert 0 < need <= zs.NOALLOC_SCRATCH_BYTES, (n, need)
        base_k, base_p = dev(keys, idx)
        say(f"case noalloc {name} n={n} pw={pw} cfg={cfg}")
        ak, ap = base_k.clone(), base_p.clone()
        zs.zsort_stable_noalloc(ak, ap, cfg)
        ek, ep = base_k.clone(), base_p.clone()
        zs.zsort_stable_ex(ek, ep, cfg)
        torch.cuda.synchronize()
        assert zs.zsort_get_last_stats()["device_error"] == 0
        assert torch.equal(ak, ek), (name, n)
        assert torch.equal(ap, ep), (name, n)


def test_noalloc_refuses_problems_beyond_its_array():
    n = 6 * 10**6
    keys, idx = synth.make("uniform", n, payload_bytes=8)
    assert zs.zsort_workspace_bytes(n, 8, 0, None) > zs.NOALLOC_SCRATCH_BYTES
    tk, tp = dev(keys, idx)
    say("case noalloc too large")
    with pytest.raises(zs.ZsortError) as ei:
        zs.zsort_stable_noalloc(tk, tp)
    assert ei.value.code == zs.ZSORT_ETOOLARGE
    torch.cuda.synchronize()
    assert np.array_equal(tk.cpu().numpy().view(np.uint64), keys)


def test_noalloc_signed_keys_and_tiny_inputs():
    for n in (0, 1, 2, 5000):
        keys, idx = synth.make("normal", max(n, 1), payload_bytes=4)
        keys, idx = keys[:n], idx[:n]
        base_k, base_p = dev(keys, idx)
        for flags in (0, zs.ZSORT_FLAG_SIGNED):
            say(f"case noalloc small n={n} flags={flags}")
            c = dict(k=1024, cutoff=2048, chunk=16384, tile=2048, flags=flags)
            ak, ap = base_k.clone(), base_p.clone()
            zs.zsort_stable_noalloc(ak, ap, c)
            ek, ep = base_k.clone(), base_p.clone()
            zs.zsort_stable_ex(ek, ep, c)
            torch.cuda.synchronize()
            assert torch.equal(ak, ek) and torch.equal(ap, ep)
