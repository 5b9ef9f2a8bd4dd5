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


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(zs, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(zs, "_lib", None)
    with pytest.raises(RuntimeError):
        zs.lib()
