"""The C-ABI library loads and exports every function include/zsort.h
declares; host-only entry points behave (no GPU needed)."""
import ctypes
import os
import re

import pytest

import paper_2605_14419_amd as zs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "zsort.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(zsort_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_expected_entry_points():
    names = declared_functions()
    for need in ["zsort_stable", "zsort_stable_segmented", "zsort_stable_p64", "zsort_stable_ex",
                 "zsort_workspace_bytes", "zsort_get_last_stats", "zsort_strerror"]:
        assert need in names
    assert set(names) == set(zs.EXPORTED)


def declared_arity():
    src = open(os.path.join(ROOT, "include", "zsort.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    out = {}
    for m in re.finditer(r"\b(zsort_\w+)\s*\(([^;{]*?)\)\s*;", src, flags=re.S):
        args = m.group(2).strip()
        out[m.group(1)] = 0 if args in ("", "void") else args.count(",") + 1
    return out


def test_binding_argument_counts_match_the_header():
    L = zs.lib()
    ar = declared_arity()
    assert set(ar) == set(declared_functions())
    for name, n in ar.items():
        at = getattr(L, name).argtypes
        if at is not None:
            assert len(at) == n, (name, len(at), n)


def test_library_exports_every_declared_symbol():
    L = zs.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
        assert ctypes.cast(getattr(L, name), ctypes.c_void_p).value


def test_host_only_entry_points():
    c = zs.zsort_default_config()
    assert (c.k, c.cutoff, c.max_zlevels, c.chunk) == (1024, 2048, 8, 16384)
    assert zs.strerror(0) == "ok" and zs.strerror(-1) == "invalid argument"
    b = zs.zsort_workspace_bytes(10**8, 4, 0)
    # the alternate buffer (12 B/key) dominates; lists, look-back words and
    # cluster starts add a few bytes per key
    assert 12 * 10**8 <= b <= 20 * 10**8
    assert zs.zsort_workspace_bytes(10**8, 3, 0) == 0        # bad payload width
    assert zs.zsort_workspace_bytes(100, 4, 0, dict(k=8)) == 0  # k below 16
    assert zs.zsort_workspace_bytes(100, 4, 0, dict(cutoff=8192)) == 0


def test_entry_points_reject_bad_arguments_without_touching_the_gpu():
    L = zs.lib()
    # bad payload width, null keys, n above the limit: rejected before any HIP call
    assert L.zsort_stable_ex(None, None, 3, 10, None, None) == zs.ZSORT_EINVAL
    assert L.zsort_stable_ex(None, None, 0, 10, None, None) == zs.ZSORT_EINVAL
    assert L.zsort_stable_ex(ctypes.c_void_p(16), None, 4, 10, None, None) == zs.ZSORT_EINVAL
    assert L.zsort_stable_ex(ctypes.c_void_p(16), None, 0, 2**31, None, None) == zs.ZSORT_EINVAL
    # profiling of no kernel kind, or of kinds that do not exist
    assert L.zsort_profile_begin_stages(None, 0) == zs.ZSORT_EINVAL
    assert L.zsort_profile_begin_stages(None, 1 << len(zs.STAGES)) == zs.ZSORT_EINVAL
    # n <= 1 is a no-op
    assert L.zsort_stable_ex(None, None, 0, 1, None, None) == zs.ZSORT_OK
    bad = zs.zsort_default_config(k=5000)
    assert L.zsort_stable_ex(ctypes.c_void_p(16), None, 0, 10, ctypes.byref(bad), None) \
        == zs.ZSORT_EINVAL
    assert L.zsort_stable_segmented(ctypes.c_void_p(16), None, 0, 10, None, 3, None, None) \
        == zs.ZSORT_EINVAL
    # 128-bit keys: null or misaligned (not 16-byte) keys, n above the limit
    assert L.zsort_stable_u128(None, None, 10, None, None, None) == zs.ZSORT_EINVAL
    assert L.zsort_stable_u128(ctypes.c_void_p(24), None, 10, None, None, None) == zs.ZSORT_EINVAL
    assert L.zsort_stable_u128(ctypes.c_void_p(32), None, 2**31, None, None, None) \
        == zs.ZSORT_EINVAL


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(zs, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(zs, "_lib", None)
    with pytest.raises(RuntimeError):
        zs.lib()


def test_workspace_bytes_follows_tile_and_set_workspace_checks_arguments():
    # 8192-key tiles need per-tile prefix rows and tile lists: more bytes
    n = 10**7
    b2 = zs.zsort_workspace_bytes(n, 4, 0, dict(k=512, chunk=32768, tile=2048))
    b8 = zs.zsort_workspace_bytes(n, 4, 0, dict(k=512, chunk=32768, tile=8192))
    assert b8 > b2 > 0
    L = zs.lib()
    # misaligned, too small, or NULL with a size: rejected before any HIP call
    assert L.zsort_set_workspace(ctypes.c_void_p(4096 + 8), 1 << 20, None) == zs.ZSORT_EINVAL
    assert L.zsort_set_workspace(ctypes.c_void_p(4096), 64, None) == zs.ZSORT_EINVAL
    assert L.zsort_set_workspace(None, 1 << 20, None) == zs.ZSORT_EINVAL
    assert L.zsort_set_alloc_limit(0) == zs.ZSORT_OK


def test_scan_row_tags_are_distinct_and_nonzero_between_clears():
    """The histogram pass's scan-row words carry tag(epoch, level) =
    1 + (64 epoch + level) mod kTagMod; rows are cleared (tag 0) at least once
    every kClearEvery epochs.  Between two clears every (epoch, level) pair
    must have its own tag, never 0, at any epoch offset, including across the
    32-bit wrap of the epoch counter."""
    import re
    import numpy as np
    src = open(os.path.join(ROOT, "paper_2605_14419_amd", "csrc", "zsort_internal.h")).read()
    mod = eval(re.search(r"kTagMod\s*=\s*([^;]+);", src).group(1).replace("u", ""))
    every = int(re.search(r"kClearEvery\s*=\s*(\d+)u", src).group(1))
    kern = open(os.path.join(ROOT, "paper_2605_14419_amd", "csrc", "zsort_kernels.hip")).read()
    assert "return 1u + (uint32_t)(((uint64_t)epoch * 64u + (uint32_t)L) % kTagMod);" in kern
    # the epoch counter's wrap to 0 forces a clear as well
    assert "ep == 0u ||" in kern
    levels = 40
    for e0 in [0, 1, 12345, 2**22, 2**32 - every]:
        ep = (np.arange(e0, e0 + every, dtype=np.uint64) % np.uint64(2**32))
        t = 1 + (ep[:, None] * np.uint64(64) + np.arange(levels, dtype=np.uint64)[None, :]) % np.uint64(mod)
        t = t.reshape(-1)
        assert t.min() >= 1 and t.max() < 2**22
        assert np.unique(t).size == t.size, e0


def test_count_range_must_not_exceed_k():
    L = zs.lib()
    bad = zs.zsort_default_config(k=256, count_range=257)
    assert L.zsort_stable_ex(ctypes.c_void_p(16), None, 0, 10, ctypes.byref(bad), None) \
        == zs.ZSORT_EINVAL
    neg = zs.zsort_default_config(count_range=-1)
    assert L.zsort_stable_ex(ctypes.c_void_p(16), None, 0, 10, ctypes.byref(neg), None) \
        == zs.ZSORT_EINVAL


def test_flag_constants_match_the_header():
    src = open(os.path.join(ROOT, "include", "zsort.h")).read()
    defs = dict(re.findall(r"^#define\s+(ZSORT_FLAG_\w+)\s+(\d+)", src, flags=re.M))
    assert set(defs) == {"ZSORT_FLAG_GRAPH", "ZSORT_FLAG_SIGNED", "ZSORT_FLAG_FUSED_STATS"}
    for name, v in defs.items():
        assert getattr(zs, name) == int(v), name


def test_fused_statistics_workspace():
    """the fused layout adds the child-of-cluster array and the accumulators
    (k <= 1024 only; larger k ignores the flag)"""
    n = 10**7
    for k in (256, 1024):
        plain = zs.zsort_workspace_bytes(n, 4, 0, dict(k=k))
        fused = zs.zsort_workspace_bytes(n, 4, 0, dict(k=k, flags=zs.ZSORT_FLAG_FUSED_STATS))
        assert plain < fused <= plain + plain // 4, (k, plain, fused)
    big = dict(k=4096, cutoff=2048, chunk=32768)
    assert (zs.zsort_workspace_bytes(n, 4, 0, big) ==
            zs.zsort_workspace_bytes(n, 4, 0, dict(big, flags=zs.ZSORT_FLAG_FUSED_STATS)))
