"""128-bit keys on the GPU (zsort_stable_u128) against the oracle's
definition (the stable sort by the 128-bit key), bit for bit, and the number
of distribution levels against the 64-bit path on the same words."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
zs = pytest.importorskip("paper_2605_14419_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
CFG = dict(k=512, cutoff=2048, max_zlevels=8, chunk=16384, tile=2048)


def say(*a):
    print(*a, flush=True)


def run128(keys2, idx, cfg, report=True):
    tk = torch.from_numpy(np.ascontiguousarray(keys2).reshape(-1).view(np.int64)).to(DEV)
    tp = None if idx is None else torch.from_numpy(idx.view(np.int32)).to(DEV)
    rep = zs.zsort_stable_u128(tk, tp, cfg, report=report)
    torch.cuda.synchronize()
    k = tk.cpu().numpy().view(np.uint64).reshape(-1, 2)
    p = None if tp is None else tp.cpu().numpy().view(np.uint32)
    return k, p, rep


@pytest.mark.parametrize("name", list(synth.WORKLOADS128))
@pytest.mark.parametrize("cfg", [CFG, dict(k=256, cutoff=4096, max_zlevels=8, chunk=32768,
                                           tile=8192)])
def test_u128_families_vs_oracle(name, cfg):
    n = 300_001
    keys, idx = synth.make128(name, n)
    say(f"case u128 {name} {cfg}")
    k, p, rep = run128(keys, idx, cfg)
    assert rep["device_error"] == 0, rep
    ok, op = oracle.sort128(keys, idx)
    assert np.array_equal(k, ok) and np.array_equal(p, op)
    # without a payload the high words carry the low words themselves
    k2, _, rep2 = run128(keys, None, cfg)
    assert rep2["device_error"] == 0 and np.array_equal(k2, ok)
    if name == "narrow":
        assert rep["short_runs"] > 0
    if name == "prefix":   # 1000 runs of ~300 keys: listed, then sorted as leaves
        assert rep["runs"] - rep["short_runs"] == 1000
    if name == "uuid":
        assert rep["run_keys"] < 10 and rep["levels_low"] == 0


@pytest.mark.parametrize("name", ["uuid", "dup", "prefix"])
def test_u128_signed(name):
    n = 100_003
    keys, idx = synth.make128(name, n)
    say(f"case u128 signed {name}")
    k, p, rep = run128(keys, idx, dict(CFG, flags=zs.ZSORT_FLAG_SIGNED))
    ok, op = oracle.sort128(keys, idx, signed=True)
    assert np.array_equal(k, ok) and np.array_equal(p, op)


@pytest.mark.parametrize("n", [0, 1, 2, 3, 65, 2049, 16385, 70_001])
def test_u128_edge_sizes_and_no_payload(n):
    keys, idx = synth.make128("narrow", max(n, 1))
    keys, idx = keys[:n], idx[:n]
    say(f"case u128 small n={n}")
    k, p, _ = run128(keys, idx, CFG)
    ok, op = oracle.sort128(keys, idx)
    assert np.array_equal(k, ok) and np.array_equal(p, op)
    k2, _, _ = run128(keys, None, CFG, report=False)
    assert np.array_equal(k2, ok)


def test_u128_pass_count_equals_64bit_on_the_same_words():
    """Zero high words: the low-word stage sorts the whole array as one run
    and takes exactly the levels the 64-bit path takes on those words."""
    n = 1_000_003
    keys, idx = synth.make128("zext", n)
    say("case u128 pass count")
    k, p, rep = run128(keys, idx, CFG)
    assert rep["runs"] == 1 and rep["run_keys"] == n
    t64 = torch.from_numpy(np.ascontiguousarray(keys[:, 0]).view(np.int64)).to(DEV)
    p64 = torch.from_numpy(idx.view(np.int32)).to(DEV)
    zs.zsort_stable_ex(t64, p64, CFG)
    torch.cuda.synchronize()
    st = zs.zsort_get_last_stats()
    assert rep["levels_low"] == st["levels"]
    assert np.array_equal(k[:, 0], t64.cpu().numpy().view(np.uint64))
    assert np.array_equal(p, p64.cpu().numpy().view(np.uint32))
