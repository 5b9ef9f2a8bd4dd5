"""Python binding of the zSort C-ABI (include/zsort.h).

Argument marshalling only: every step of the sort runs in the HIP kernels of
the in-tree library ``_lib/libzsort.so``.  PyTorch supplies device memory and
streams.  There is no fallback: if the library has not been built the first
call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libzsort.so")

ZSORT_OK, ZSORT_EINVAL, ZSORT_ENOMEM, ZSORT_EHIP, ZSORT_ECAPTURE, ZSORT_EUNSUPPORTED, \
    ZSORT_EDEVICE, ZSORT_ETOOLARGE = 0, -1, -2, -3, -4, -5, -6, -7
NOALLOC_SCRATCH_BYTES = 64 << 20
MAX_LEVELS = 40

EXPORTED = [
    "zsort_default_config", "zsort_stable", "zsort_stable_p64", "zsort_stable_ex",
    "zsort_stable_segmented", "zsort_workspace_bytes", "zsort_get_last_stats",
    "zsort_debug_level0", "zsort_stable_traced", "zsort_release", "zsort_last_hip_error",
    "zsort_strerror", "zsort_profile_begin", "zsort_profile_begin_stages", "zsort_profile_end",
    "zsort_autotune", "zsort_set_workspace", "zsort_set_alloc_limit", "zsort_stable_noalloc",
    "zsort_stable_u128",
    "zsort_default_learned_config", "zsort_stable_learned", "zsort_learned_sample",
    "zsort_mlp_forward", "zsort_mlp_thresholds", "zsort_mlp_init", "zsort_mlp_grad",
    "zsort_mlp_train",
]
ZSORT_FLAG_GRAPH = 1
ZSORT_FLAG_SIGNED = 2
ZSORT_FLAG_FUSED_STATS = 4
ZSORT_MLP_PARAMS = 1153
MLP_PARAMS_BYTES = 4872   # sizeof(zsort_mlp_params): 64 binary64, 1089 binary32, padding
ZSORT_LEARNED_DIRECT = 1
ZSORT_LEARNED_ZSCORE_DIAG = 2
ZSORT_LEARNED_VERIFY = 4
STAGES = ("moments", "finalize", "hist", "scatter", "local", "local_hard")


class ZsortConfig(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("cutoff", ctypes.c_int32),
                ("max_zlevels", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("tile", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("count_range", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class ZsortStats(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("device_error", ctypes.c_int32),
                ("identical", ctypes.c_uint32), ("range_mapped", ctypes.c_uint32),
                ("leaf_groups", ctypes.c_uint32), ("payload_bytes", ctypes.c_int32),
                ("n", ctypes.c_uint64),
                ("keys_per_level", ctypes.c_uint64 * MAX_LEVELS),
                ("mkeys_per_level", ctypes.c_uint64 * MAX_LEVELS),
                ("segs_per_level", ctypes.c_uint32 * MAX_LEVELS),
                ("local_keys", ctypes.c_uint64),
                ("model_bytes", ctypes.c_double),
                ("counted", ctypes.c_uint32), ("fallback_groups", ctypes.c_uint32)]


class ZsortU128Report(ctypes.Structure):
    _fields_ = [("levels_high", ctypes.c_int32), ("levels_low", ctypes.c_int32),
                ("runs", ctypes.c_uint64), ("short_runs", ctypes.c_uint64),
                ("run_keys", ctypes.c_uint64), ("device_error", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class ZsortLearnedConfig(ctypes.Structure):
    _fields_ = [("buckets", ctypes.c_int32), ("sample_stride", ctypes.c_int32),
                ("steps", ctypes.c_int32), ("batches", ctypes.c_int32),
                ("lr", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("params", ctypes.c_void_p), ("smin", ctypes.c_uint64),
                ("smax", ctypes.c_uint64)]


class ZsortLearnedReport(ctypes.Structure):
    _fields_ = [("used_learned", ctypes.c_int32), ("fallback", ctypes.c_int32),
                ("thresholds", ctypes.c_int32), ("steps", ctypes.c_int32),
                ("trained", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("sample_max_init", ctypes.c_uint32), ("sample_max_trained", ctypes.c_uint32),
                ("sample_keys", ctypes.c_uint64), ("max_cluster_learned", ctypes.c_uint64),
                ("max_cluster_zscore", ctypes.c_uint64), ("imbalance_learned", ctypes.c_double),
                ("imbalance_zscore", ctypes.c_double), ("loss_first", ctypes.c_double),
                ("loss_last", ctypes.c_double), ("train_ms", ctypes.c_double),
                ("first_pass_ms", ctypes.c_double), ("counts", ctypes.c_void_p),
                ("params_out", ctypes.c_void_p), ("smin_out", ctypes.c_uint64),
                ("smax_out", ctypes.c_uint64)]


class ZsortKernelTimes(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 6), ("launches", ctypes.c_uint64 * 6)]


TRACE_REC = np.dtype([
    ("depth", np.int32), ("kind", np.int32), ("start", np.uint64), ("count", np.uint64),
    ("o", np.uint64), ("M", np.uint64), ("s1", np.uint64, 2), ("s2", np.uint64, 4),
    ("m", np.float64), ("sigma", np.float64), ("zmin", np.float64), ("A", np.float64),
    ("B", np.float64), ("shift", np.int32), ("nonempty", np.int32), ("hist_off", np.int64),
])


class ZsortError(RuntimeError):
    def __init__(self, fn, code):
        super().__init__(f"{fn} failed: {code} ({strerror(code)}), hip error {last_hip_error()}")
        self.code = code


_lib = None


def lib():
    """The loaded library; raises if it was never built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"zsort HIP library not built: {LIB_PATH} is missing "
                               "(run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        P, Z, I = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int
        L.zsort_default_config.argtypes = [P]
        L.zsort_stable.argtypes = [P, P, Z, P]
        L.zsort_stable_p64.argtypes = [P, P, Z, P]
        L.zsort_stable_ex.argtypes = [P, P, I, Z, P, P]
        L.zsort_stable_noalloc.argtypes = [P, P, I, Z, P, P]
        L.zsort_stable_u128.argtypes = [P, P, Z, P, P, P]
        L.zsort_stable_segmented.argtypes = [P, P, I, Z, P, ctypes.c_int32, P, P]
        L.zsort_workspace_bytes.argtypes = [Z, I, ctypes.c_int32, P]
        L.zsort_set_workspace.argtypes = [P, Z, P]
        L.zsort_set_alloc_limit.argtypes = [Z]
        L.zsort_workspace_bytes.restype = Z
        L.zsort_get_last_stats.argtypes = [P, P]
        L.zsort_debug_level0.argtypes = [P, P, I, Z, P, P, P, P]
        L.zsort_stable_traced.argtypes = [P, P, I, Z, P, P, ctypes.c_int64, P, ctypes.c_int64,
                                          P, P]
        L.zsort_autotune.argtypes = [P, P, I, Z, P, ctypes.c_int32, ctypes.c_char_p, P, P]
        L.zsort_profile_begin.argtypes = [P]
        L.zsort_profile_begin_stages.argtypes = [P, ctypes.c_uint32]
        L.zsort_profile_end.argtypes = [P, P]
        U64 = ctypes.c_uint64
        L.zsort_default_learned_config.argtypes = [P]
        L.zsort_stable_learned.argtypes = [P, P, I, Z, P, P, P, P]
        L.zsort_learned_sample.argtypes = [P, Z, ctypes.c_int32, U64, P, P]
        L.zsort_mlp_forward.argtypes = [P, P, Z, U64, U64, ctypes.c_int32, P, P, P]
        L.zsort_mlp_thresholds.argtypes = [P, U64, U64, ctypes.c_int32, P, P, P]
        L.zsort_mlp_init.argtypes = [P, Z, P, P]
        L.zsort_mlp_grad.argtypes = [P, P, Z, P, P]
        L.zsort_mlp_train.argtypes = [P, P, Z, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                      P, P]
        L.zsort_strerror.argtypes = [I]
        L.zsort_strerror.restype = ctypes.c_char_p
        _lib = L
    return _lib


def strerror(code: int) -> str:
    return lib().zsort_strerror(int(code)).decode()


def last_hip_error() -> int:
    return int(lib().zsort_last_hip_error())


def _check(fn, rc):
    if rc != ZSORT_OK:
        raise ZsortError(fn, rc)


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


def _keys_ptr(keys):
    import torch
    if not keys.is_cuda or keys.dtype not in (torch.int64, torch.uint64) or not keys.is_contiguous():
        raise ValueError("keys must be a contiguous int64/uint64 CUDA tensor (read as u64)")
    return ctypes.c_void_p(keys.data_ptr())


def _pay(payload, n):
    import torch
    if payload is None:
        return None, 0
    if not payload.is_cuda or not payload.is_contiguous() or payload.numel() != n:
        raise ValueError("payload must be a contiguous CUDA tensor with one element per key")
    if payload.dtype in (torch.int32, torch.uint32):
        return ctypes.c_void_p(payload.data_ptr()), 4
    if payload.dtype in (torch.int64, torch.uint64):
        return ctypes.c_void_p(payload.data_ptr()), 8
    raise ValueError("payload dtype must be 4 or 8 bytes wide")


def zsort_default_config(**overrides) -> ZsortConfig:
    c = ZsortConfig()
    _check("zsort_default_config", lib().zsort_default_config(ctypes.byref(c)))
    for k, v in overrides.items():
        setattr(c, k, int(v))
    return c


def _cfg(cfg):
    if cfg is None:
        return None
    if isinstance(cfg, dict):
        cfg = zsort_default_config(**cfg)
    return ctypes.byref(cfg)


def zsort_stable(keys, payload=None, stream=None):
    """u32 payload (or None)."""
    p, pw = _pay(payload, keys.numel())
    if pw not in (0, 4):
        raise ValueError("zsort_stable takes a 4-byte payload")
    _check("zsort_stable", lib().zsort_stable(_keys_ptr(keys), p, keys.numel(), _stream(stream)))


def zsort_stable_p64(keys, payload=None, stream=None):
    """u64 payload (or None)."""
    p, pw = _pay(payload, keys.numel())
    if pw not in (0, 8):
        raise ValueError("zsort_stable_p64 takes an 8-byte payload")
    _check("zsort_stable_p64", lib().zsort_stable_p64(_keys_ptr(keys), p, keys.numel(),
                                                      _stream(stream)))


def zsort_stable_ex(keys, payload=None, cfg=None, stream=None):
    p, pw = _pay(payload, keys.numel())
    _check("zsort_stable_ex", lib().zsort_stable_ex(_keys_ptr(keys), p, pw, keys.numel(),
                                                    _cfg(cfg), _stream(stream)))


def zsort_stable_noalloc(keys, payload=None, cfg=None, stream=None):
    """zsort_stable_ex without any allocation: runs in the library's fixed
    per-GPU scratch array (problems up to NOALLOC_SCRATCH_BYTES of workspace)."""
    p, pw = _pay(payload, keys.numel())
    _check("zsort_stable_noalloc", lib().zsort_stable_noalloc(
        _keys_ptr(keys), p, pw, keys.numel(), _cfg(cfg), _stream(stream)))


def zsort_stable_u128(keys, payload=None, cfg=None, report=False, stream=None):
    """128-bit keys: `keys` holds 2n u64 words (low word first per key, int64
    or uint64 tensor of 2n elements); payload u32 or None.  Returns the report
    as a dict when report=True (synchronous)."""
    if keys.numel() % 2:
        raise ValueError("128-bit keys need an even number of 64-bit words")
    n = keys.numel() // 2
    p, pw = _pay(payload, n)
    if pw not in (0, 4):
        raise ValueError("zsort_stable_u128 takes a 4-byte payload")
    rep = ZsortU128Report() if report else None
    _check("zsort_stable_u128", lib().zsort_stable_u128(
        _keys_ptr(keys), p, n, _cfg(cfg), ctypes.byref(rep) if rep is not None else None,
        _stream(stream)))
    if rep is None:
        return None
    return {f: getattr(rep, f) for f, _ in ZsortU128Report._fields_ if f != "reserved"}


def zsort_stable_segmented(keys, seg_offsets, payload=None, cfg=None, stream=None):
    import torch
    if (not seg_offsets.is_cuda or seg_offsets.dtype != torch.int64
            or not seg_offsets.is_contiguous()):
        raise ValueError("seg_offsets must be a contiguous int64 CUDA tensor")
    p, pw = _pay(payload, keys.numel())
    _check("zsort_stable_segmented", lib().zsort_stable_segmented(
        _keys_ptr(keys), p, pw, keys.numel(), ctypes.c_void_p(seg_offsets.data_ptr()),
        seg_offsets.numel() - 1, _cfg(cfg), _stream(stream)))


def zsort_workspace_bytes(n, payload_bytes=4, num_segments=0, cfg=None) -> int:
    return int(lib().zsort_workspace_bytes(n, payload_bytes, num_segments, _cfg(cfg)))


def zsort_set_workspace(buf=None, stream=None):
    """Hand the library caller-owned device memory (a CUDA tensor, kept alive
    by the caller) as the workspace of `stream`; None returns the stream to
    library-allocated memory."""
    if buf is None:
        _check("zsort_set_workspace", lib().zsort_set_workspace(None, 0, _stream(stream)))
        return
    if not buf.is_cuda or not buf.is_contiguous():
        raise ValueError("workspace must be a contiguous CUDA tensor")
    nbytes = buf.numel() * buf.element_size()
    _check("zsort_set_workspace", lib().zsort_set_workspace(
        ctypes.c_void_p(buf.data_ptr()), nbytes, _stream(stream)))


def zsort_set_alloc_limit(max_bytes: int):
    """Every device allocation above max_bytes fails as out of memory (0: no limit)."""
    _check("zsort_set_alloc_limit", lib().zsort_set_alloc_limit(int(max_bytes)))


def zsort_get_last_stats(stream=None) -> dict:
    s = ZsortStats()
    _check("zsort_get_last_stats", lib().zsort_get_last_stats(_stream(stream), ctypes.byref(s)))
    L = s.levels
    return dict(levels=L, device_error=s.device_error, identical=s.identical,
                range_mapped=s.range_mapped, leaf_groups=s.leaf_groups, n=s.n,
                payload_bytes=s.payload_bytes,
                keys_per_level=list(s.keys_per_level[:L]),
                mkeys_per_level=list(s.mkeys_per_level[:L]),
                segs_per_level=list(s.segs_per_level[:L]), local_keys=s.local_keys,
                model_bytes=s.model_bytes, counted=s.counted,
                fallback_groups=s.fallback_groups)


def zsort_debug_level0(keys, payload=None, cfg=None, stream=None):
    """One distribution pass of the root; returns (cluster keys, cluster payload)."""
    import torch
    p, pw = _pay(payload, keys.numel())
    ok = torch.empty_like(keys)
    op = torch.empty_like(payload) if payload is not None else None
    _check("zsort_debug_level0", lib().zsort_debug_level0(
        _keys_ptr(keys), p, pw, keys.numel(), _cfg(cfg), ctypes.c_void_p(ok.data_ptr()),
        ctypes.c_void_p(op.data_ptr()) if op is not None else None, _stream(stream)))
    return ok, op


def zsort_stable_traced(keys, payload=None, cfg=None, trace_cap=1 << 16, hist_cap=1 << 22,
                        stream=None):
    """Sort and return (records, histograms) of every subproblem above the cutoff."""
    p, pw = _pay(payload, keys.numel())
    rec = np.zeros(trace_cap, dtype=TRACE_REC)
    hist = np.zeros(hist_cap, dtype=np.uint32)
    counts = np.zeros(2, dtype=np.int64)
    rc = lib().zsort_stable_traced(_keys_ptr(keys), p, pw, keys.numel(), _cfg(cfg),
                                   rec.ctypes.data, trace_cap, hist.ctypes.data, hist_cap,
                                   counts.ctypes.data, _stream(stream))
    _check("zsort_stable_traced", rc)
    return rec[: min(int(counts[0]), trace_cap)], hist[: int(counts[1])]


def zsort_autotune(keys, payload=None, seg_offsets=None, cache_path=None, stream=None) -> dict:
    """Tunes k / tile / chunk / cutoff for arrays shaped like `keys` (left
    unchanged) and returns the chosen configuration as a dict."""
    p, pw = _pay(payload, keys.numel())
    best = ZsortConfig()
    off = None if seg_offsets is None else ctypes.c_void_p(seg_offsets.data_ptr())
    nseg = 0 if seg_offsets is None else seg_offsets.numel() - 1
    _check("zsort_autotune", lib().zsort_autotune(
        _keys_ptr(keys), p, pw, keys.numel(), off, nseg,
        None if cache_path is None else cache_path.encode(), ctypes.byref(best), _stream(stream)))
    return {f: getattr(best, f) for f in ("k", "cutoff", "max_zlevels", "chunk", "tile")}


def zsort_profile_begin(stream=None, stages=None):
    """Times every kernel kind, or only those named in `stages` (see STAGES)."""
    if stages is None:
        _check("zsort_profile_begin", lib().zsort_profile_begin(_stream(stream)))
        return
    mask = 0
    for name in stages:
        mask |= 1 << STAGES.index(name)
    _check("zsort_profile_begin_stages", lib().zsort_profile_begin_stages(_stream(stream), mask))


def zsort_profile_end(stream=None) -> dict:
    """{stage: (total ms, launches)} for every kernel kind of a level."""
    t = ZsortKernelTimes()
    _check("zsort_profile_end", lib().zsort_profile_end(_stream(stream), ctypes.byref(t)))
    return {name: (t.ms[i], int(t.launches[i])) for i, name in enumerate(STAGES)}


def zsort_release():
    _check("zsort_release", lib().zsort_release())


def _dptr(t, dtype, n=None, name="tensor"):
    if not t.is_cuda or not t.is_contiguous() or t.dtype != dtype or (n is not None and t.numel() != n):
        raise ValueError(f"{name} must be a contiguous {dtype} CUDA tensor"
                         + ("" if n is None else f" of {n} elements"))
    return ctypes.c_void_p(t.data_ptr())


def mlp_pack(flat) -> np.ndarray:
    """1153 parameter values (W1, b1, W2, b2, W3, b3) -> the bytes of a
    zsort_mlp_params (W1, b1 binary64; the rest rounded to binary32)."""
    flat = np.asarray(flat, dtype=np.float64).reshape(-1)
    if flat.size != ZSORT_MLP_PARAMS:
        raise ValueError("expected 1153 parameters")
    buf = flat[:64].astype("<f8").tobytes() + flat[64:].astype("<f4").tobytes() + bytes(4)
    return np.frombuffer(buf, dtype=np.uint8).copy()


def mlp_unpack(buf) -> np.ndarray:
    """bytes of a zsort_mlp_params -> the 1153 parameter values as float64"""
    b = np.asarray(buf, dtype=np.uint8).reshape(-1)
    if b.size != MLP_PARAMS_BYTES:
        raise ValueError("expected the bytes of one zsort_mlp_params")
    return np.concatenate([b[:512].view("<f8"), b[512:512 + 4 * 1089].view("<f4").astype(np.float64)])


def _pptr(params):
    import torch
    return _dptr(params, torch.uint8, MLP_PARAMS_BYTES, "params (zsort_mlp_params bytes)")


def zsort_default_learned_config(**overrides) -> ZsortLearnedConfig:
    c = ZsortLearnedConfig()
    _check("zsort_default_learned_config", lib().zsort_default_learned_config(ctypes.byref(c)))
    for k, v in overrides.items():
        if k == "params":
            c.params = _pptr(v).value
        elif k == "lr":
            c.lr = float(v)
        else:
            setattr(c, k, int(v))
    return c


def zsort_stable_learned(keys, payload=None, cfg=None, lcfg=None, counts=False, params_out=None,
                         stream=None):
    """Sort with the learned first-pass map; returns the report as a dict
    (with the first-pass cluster sizes under "counts" when counts=True; the
    parameters used are copied into params_out, a device uint8 tensor of
    MLP_PARAMS_BYTES, when given)."""
    p, pw = _pay(payload, keys.numel())
    if isinstance(lcfg, dict):
        lcfg = zsort_default_learned_config(**lcfg)
    rep = ZsortLearnedReport()
    buckets = lcfg.buckets if lcfg is not None else 4096
    cbuf = np.zeros(buckets, dtype=np.uint32) if counts else None
    if cbuf is not None:
        rep.counts = cbuf.ctypes.data
    if params_out is not None:
        rep.params_out = _pptr(params_out).value
    _check("zsort_stable_learned", lib().zsort_stable_learned(
        _keys_ptr(keys), p, pw, keys.numel(), _cfg(cfg),
        None if lcfg is None else ctypes.byref(lcfg), ctypes.byref(rep), _stream(stream)))
    out = {f: getattr(rep, f) for f, _ in ZsortLearnedReport._fields_
           if f not in ("counts", "reserved", "params_out")}
    if cbuf is not None:
        out["counts"] = cbuf
    return out


def zsort_learned_sample(keys, stride=100, seed=0x5A17, stream=None):
    import torch
    m = keys.numel() // stride
    out = torch.empty(max(m, 1), dtype=keys.dtype, device=keys.device)
    _check("zsort_learned_sample", lib().zsort_learned_sample(
        _keys_ptr(keys), keys.numel(), stride, seed, ctypes.c_void_p(out.data_ptr()),
        _stream(stream)))
    return out[:m]


def zsort_mlp_forward(params, keys, smin, smax, buckets=4096, stream=None):
    """(f, cluster) of every key under the MLP with the given parameters."""
    import torch
    q = keys.numel()
    f = torch.empty(max(q, 1), dtype=torch.float32, device=keys.device)
    c = torch.empty(max(q, 1), dtype=torch.int32, device=keys.device)
    _check("zsort_mlp_forward", lib().zsort_mlp_forward(
        _pptr(params), _keys_ptr(keys), q, smin, smax,
        buckets, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(c.data_ptr()), _stream(stream)))
    return f[:q], c[:q]


def zsort_mlp_thresholds(params, smin, smax, buckets=4096, stream=None):
    """(nt, thresholds[buckets - 1]) as a host array of u64."""
    import torch
    thr = torch.empty(buckets - 1, dtype=torch.int64, device=params.device)
    nt = ctypes.c_int32(0)
    _check("zsort_mlp_thresholds", lib().zsort_mlp_thresholds(
        _pptr(params), smin, smax, buckets,
        ctypes.c_void_p(thr.data_ptr()), ctypes.byref(nt), _stream(stream)))
    return int(nt.value), thr.cpu().numpy().view(np.uint64)


def zsort_mlp_init(sorted_sample, stream=None):
    import torch
    par = torch.empty(MLP_PARAMS_BYTES, dtype=torch.uint8, device=sorted_sample.device)
    _check("zsort_mlp_init", lib().zsort_mlp_init(
        _keys_ptr(sorted_sample), sorted_sample.numel(), ctypes.c_void_p(par.data_ptr()),
        _stream(stream)))
    return par


def zsort_mlp_grad(params, sorted_sample, stream=None):
    """(loss, gradient[1153]) over the whole sorted sample, float64 host values."""
    import torch
    g = torch.empty(ZSORT_MLP_PARAMS + 1, dtype=torch.float64, device=params.device)
    _check("zsort_mlp_grad", lib().zsort_mlp_grad(
        _pptr(params), _keys_ptr(sorted_sample),
        sorted_sample.numel(), ctypes.c_void_p(g.data_ptr()), _stream(stream)))
    gh = g.cpu().numpy()
    return float(gh[-1]), gh[:-1]


def zsort_mlp_train(params, sorted_sample, steps, batches=64, lr=1e-3, stream=None):
    """Trains params (in place); returns (first, last) minibatch loss."""
    import torch
    losses = np.zeros(2, dtype=np.float64)
    _check("zsort_mlp_train", lib().zsort_mlp_train(
        _pptr(params), _keys_ptr(sorted_sample),
        sorted_sample.numel(), steps, batches, lr, losses.ctypes.data, _stream(stream)))
    return float(losses[0]), float(losses[1])


def sort(keys, payload=None, cfg=None, stream=None):
    """In-place stable sort of keys (u64 bits in an int64/uint64 tensor) with an
    optional 4- or 8-byte payload."""
    zsort_stable_ex(keys, payload, cfg, stream)
    return keys, payload
