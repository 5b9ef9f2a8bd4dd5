"""ctypes wrapper of the CPU oracle (zsort_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
benchmark's CPU-baseline leg.  The product path never imports this package.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "zsort_oracle.c")
_LIB = os.path.join(_HERE, "libzsort_oracle.so")

GCC_CMD = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-o", _LIB, _SRC, "-lm"]


def build() -> str:
    """Compile the oracle (always recompiles)."""
    subprocess.run(GCC_CMD, check=True)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        P, U64, I64, I32, D = (ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int64,
                               ctypes.c_int, ctypes.c_double)
        L.zo_u256_to_double.argtypes = [P]
        L.zo_u256_to_double.restype = D
        L.zo_moments.argtypes = [P, U64, P]
        L.zo_zstats.argtypes = [U64, P, P, I32, I32, D, U64, P]
        L.zo_zstats.restype = I32
        L.zo_zbucket.argtypes = [U64, U64, D, D, D, I32]
        L.zo_zbucket.restype = I32
        L.zo_rshift.argtypes = [U64, I32]
        L.zo_rshift.restype = I32
        L.zo_rbucket.argtypes = [U64, U64, I32]
        L.zo_rbucket.restype = I32
        L.zo_mean_est.argtypes = [I32, D, D, D, D]
        L.zo_mean_est.restype = D
        L.zo_sort.argtypes = [P, P, I32, U64, P, P, I64, P, I64, P]
        L.zo_sort.restype = I32
        L.zo_level0.argtypes = [P, P, I32, U64, P, P, P, I64]
        L.zo_level0.restype = I32
        L.zo_sort_segmented.argtypes = [P, P, I32, U64, P, I64, P]
        L.zo_sort_segmented.restype = I32
        L.zo_brute_stable_sort.argtypes = [P, P, I32, U64]
        L.zo_brute_stable_sort.restype = I32
        L.zo_seg_rec_size.restype = I32
        L.zo_sort128.argtypes = [P, P, U64, I32]
        L.zo_sort128.restype = I32
        L.zo_mlp_norm.argtypes = [U64, U64, U64]
        L.zo_mlp_norm.restype = D
        L.zo_mlp_forward.argtypes = [P, D]
        L.zo_mlp_forward.restype = ctypes.c_float
        L.zo_mlp_bucket.argtypes = [P, U64, U64, U64, I32]
        L.zo_mlp_bucket.restype = I32
        L.zo_mlp_thresholds.argtypes = [P, U64, U64, I32, P]
        L.zo_mlp_thresholds.restype = I32
        L.zo_mlp_init.argtypes = [P, U64, U64, U64, P]
        L.zo_mlp_loss_grad.argtypes = [P, P, P, U64, P]
        L.zo_mlp_loss_grad.restype = D
        L.zo_mlp_train.argtypes = [P, P, P, U64, ctypes.c_uint32, ctypes.c_uint32, D, P]
        L.zo_mlp_train.restype = D
        assert L.zo_seg_rec_size() == SEG_REC.itemsize
        _lib = L
    return _lib


class Params(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("cutoff", ctypes.c_int32),
                ("max_zlevels", ctypes.c_int32), ("counting_range", ctypes.c_int32)]


SEG_REC = np.dtype([
    ("depth", np.int32), ("kind", np.int32), ("start", np.uint64), ("count", np.uint64),
    ("o", np.uint64), ("M", np.uint64), ("s1", np.uint64, 2), ("s2", np.uint64, 4),
    ("m", np.float64), ("sigma", np.float64), ("zmin", np.float64), ("A", np.float64),
    ("B", np.float64), ("shift", np.int32), ("nonempty", np.int32), ("hist_off", np.int64),
])

KIND_IDENT, KIND_ZMAP, KIND_RMAP, KIND_COUNT = 1, 2, 3, 4


def paper_params(n: int, alpha: float = 1.0, max_zlevels: int = 16) -> dict:
    """Algorithm 1's settings: clusters = alpha*sqrt(n) (alpha = 1 in the
    listing, 0.6 best in the sensitivity table), insertion sort at <= 96."""
    return dict(k=max(2, int(math.floor(alpha * math.sqrt(max(n, 1))))), cutoff=96,
                max_zlevels=max_zlevels, counting_range=0)


def _params(k, cutoff, max_zlevels, counting_range=0):
    return Params(int(k), int(cutoff), int(max_zlevels), int(counting_range))


def _ptr(a):
    return None if a is None else a.ctypes.data


def _pw(payload):
    if payload is None:
        return 0
    if payload.dtype.itemsize not in (4, 8):
        raise ValueError("payload must be 4 or 8 bytes wide")
    return payload.dtype.itemsize


def u256_to_double(v: int) -> float:
    w = np.array([(v >> (64 * i)) & (2**64 - 1) for i in range(4)], dtype=np.uint64)
    return lib().zo_u256_to_double(w.ctypes.data)


def moments(x: np.ndarray):
    """(min, max, S1, S2) with S1, S2 about the minimum, as Python ints."""
    x = np.ascontiguousarray(x, dtype=np.uint64)
    out = np.zeros(8, dtype=np.uint64)
    lib().zo_moments(x.ctypes.data, x.size, out.ctypes.data)
    o = [int(v) for v in out]
    s1 = o[2] | (o[3] << 64)
    s2 = sum(v << (64 * i) for i, v in enumerate(o[4:8]))
    return o[0], o[1], s1, s2


def zstats(c: int, s1: int, s2: int, k: int, is_root: bool = True, e: float = 0.0,
           o_rel: int = 0):
    """(ok, m, var, sigma, zmin, A, B)"""
    s1w = np.array([s1 & (2**64 - 1), s1 >> 64], dtype=np.uint64)
    s2w = np.array([(s2 >> (64 * i)) & (2**64 - 1) for i in range(4)], dtype=np.uint64)
    out = np.zeros(6, dtype=np.float64)
    ok = lib().zo_zstats(c, s1w.ctypes.data, s2w.ctypes.data, k, int(is_root), e, o_rel,
                         out.ctypes.data)
    return (bool(ok),) + tuple(float(v) for v in out)


def zbucket(x: int, o: int, m: float, A: float, B: float, k: int) -> int:
    return lib().zo_zbucket(x, o, m, A, B, k)


def rshift(R: int, k: int) -> int:
    return lib().zo_rshift(R, k)


def rbucket(x: int, o: int, shift: int) -> int:
    return lib().zo_rbucket(x, o, shift)


def mean_est(j: int, scale: float, zmin: float, sigma: float, m: float) -> float:
    return lib().zo_mean_est(j, scale, zmin, sigma, m)


def sort(keys: np.ndarray, payload=None, k=1024, cutoff=96, max_zlevels=8,
         counting_range=0, trace=False, trace_cap=1 << 16, hist_cap=1 << 22):
    """Returns (keys, payload, info) sorted copies; with trace=True also
    (records, histograms)."""
    x = np.array(keys, dtype=np.uint64, copy=True)
    p = None if payload is None else np.array(payload, copy=True)
    pw = _pw(p)
    prm = _params(k, cutoff, max_zlevels, counting_range)
    info = np.zeros(3, dtype=np.int64)
    if trace:
        tr = np.zeros(trace_cap, dtype=SEG_REC)
        hist = np.zeros(hist_cap, dtype=np.uint32)
        rc = lib().zo_sort(x.ctypes.data, _ptr(p), pw, x.size, ctypes.byref(prm),
                           tr.ctypes.data, trace_cap, hist.ctypes.data, hist_cap,
                           info.ctypes.data)
    else:
        rc = lib().zo_sort(x.ctypes.data, _ptr(p), pw, x.size, ctypes.byref(prm),
                           None, 0, None, 0, info.ctypes.data)
    if rc:
        raise ValueError("oracle rejected the arguments")
    if trace:
        nrec = int(min(info[0], trace_cap))
        return x, p, info, tr[:nrec], hist[: int(info[1])]
    return x, p, info


def level0(keys: np.ndarray, payload=None, k=1024, cutoff=96, max_zlevels=8):
    """One distribution pass of the root: (cluster array keys, payload,
    root record, histogram[k])."""
    x = np.array(keys, dtype=np.uint64, copy=True)
    p = None if payload is None else np.array(payload, copy=True)
    prm = _params(k, cutoff, max_zlevels)
    tr = np.zeros(1, dtype=SEG_REC)
    hist = np.zeros(k, dtype=np.uint32)
    rc = lib().zo_level0(x.ctypes.data, _ptr(p), _pw(p), x.size, ctypes.byref(prm),
                         tr.ctypes.data, hist.ctypes.data, k)
    if rc:
        raise ValueError("oracle rejected the arguments")
    return x, p, tr[0], hist


def sort_segmented(keys, offsets, payload=None, k=1024, cutoff=96, max_zlevels=8):
    x = np.array(keys, dtype=np.uint64, copy=True)
    p = None if payload is None else np.array(payload, copy=True)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    prm = _params(k, cutoff, max_zlevels)
    rc = lib().zo_sort_segmented(x.ctypes.data, _ptr(p), _pw(p), x.size, off.ctypes.data,
                                 off.size - 1, ctypes.byref(prm))
    if rc:
        raise ValueError("oracle rejected the arguments")
    return x, p


def sort128(keys2, payload=None, signed=False):
    """Stable sort of 128-bit keys (an (n, 2) u64 array, low word first) with
    an optional u32 payload: the definition, written out (merge sort)."""
    k = np.array(keys2, dtype=np.uint64, copy=True).reshape(-1, 2)
    k = np.ascontiguousarray(k)
    p = None if payload is None else np.array(payload, dtype=np.uint32, copy=True)
    rc = lib().zo_sort128(k.ctypes.data, _ptr(p), k.shape[0], 1 if signed else 0)
    if rc:
        raise MemoryError("zo_sort128")
    return k, p


def brute_stable_sort(keys, payload=None):
    x = np.array(keys, dtype=np.uint64, copy=True)
    p = None if payload is None else np.array(payload, copy=True)
    rc = lib().zo_brute_stable_sort(x.ctypes.data, _ptr(p), _pw(p), x.size)
    if rc:
        raise ValueError("bad arguments")
    return x, p


# ---------------------------------------------------------------------------
# learned partition: monotone MLP CDF (1 -> 32 -> 32 -> 1), 1153 parameters
# ---------------------------------------------------------------------------
MLP_NP = 1153
MLP_H = 32
W1, B1, W2, B2, W3, B3 = 0, 32, 64, 1088, 1120, 1152


def _par(p):
    """parameters as the oracle takes them: 1153 doubles, W1 and b1 binary64,
    the rest rounded to binary32"""
    p = np.array(p, dtype=np.float64).reshape(-1)
    assert p.size == MLP_NP
    p[W2:] = p[W2:].astype(np.float32)
    return p


def mlp_norm(x: int, smin: int, smax: int) -> float:
    return lib().zo_mlp_norm(x, smin, smax)


def mlp_forward(p, u: float) -> float:
    p = _par(p)
    return float(lib().zo_mlp_forward(p.ctypes.data, u))


def mlp_bucket(p, x: int, smin: int, smax: int, B: int) -> int:
    p = _par(p)
    return int(lib().zo_mlp_bucket(p.ctypes.data, x, smin, smax, B))


def mlp_buckets(p, xs, smin, smax, B):
    p = _par(p)
    f = lib().zo_mlp_bucket
    return np.array([f(p.ctypes.data, int(x), smin, smax, B) for x in xs], dtype=np.int64)


def mlp_thresholds(p, smin: int, smax: int, B: int):
    p = _par(p)
    out = np.zeros(B - 1, dtype=np.uint64)
    nt = lib().zo_mlp_thresholds(p.ctypes.data, smin, smax, B, out.ctypes.data)
    return int(nt), out


def mlp_init(sorted_sample, smin: int, smax: int):
    s = np.ascontiguousarray(sorted_sample, dtype=np.uint64)
    p = np.zeros(MLP_NP, dtype=np.float64)
    lib().zo_mlp_init(s.ctypes.data, s.size, smin, smax, p.ctypes.data)
    return p


def mlp_loss_grad(p, u, y):
    p = _par(p)
    u = np.ascontiguousarray(u, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    g = np.zeros(MLP_NP, dtype=np.float64)
    loss = lib().zo_mlp_loss_grad(p.ctypes.data, u.ctypes.data, y.ctypes.data, u.size,
                                  g.ctypes.data)
    return float(loss), g


def mlp_train(p, u, y, steps, batches, lr):
    """Adam training as the learned form defines it; returns (params, loss of
    the first step's minibatch, loss of the last step's)."""
    p = _par(p)
    u = np.ascontiguousarray(u, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    first = ctypes.c_double(0.0)
    last = lib().zo_mlp_train(p.ctypes.data, u.ctypes.data, y.ctypes.data, u.size, batches, steps,
                              lr, ctypes.byref(first))
    return p, float(first.value), float(last)


def mlp_targets(sorted_sample):
    """mid-rank empirical CDF of a sorted sample: (rank_lt + rank_le) / (2m)"""
    s = np.asarray(sorted_sample, dtype=np.uint64)
    lo = np.searchsorted(s, s, side="left")
    hi = np.searchsorted(s, s, side="right")
    return (lo + hi) / (2.0 * s.size)
