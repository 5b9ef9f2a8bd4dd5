"""Seeded generators for the synthetic workloads.

The paper draws 64-bit integers with a Mersenne Twister from five families
(uniform, normal, power-law skewed, nearly sorted, high-duplicate;
Section IV-C, Experimental Results) with unstated seeds and parameters.  These
generators stand in for them with numpy's PCG64 and fixed, stated parameters.
Keys are unsigned 64-bit; the payload is the original index (u32 or u64).

seed = SEED_BASE + 100 * workload_index + variant
"""
from __future__ import annotations

import math

import numpy as np

SEED_BASE = 20260514
U64_MAX = np.iinfo(np.uint64).max
TWO64 = 2.0 ** 64


def seed_for(workload: int, variant: int = 0) -> int:
    return SEED_BASE + 100 * workload + variant


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _float_to_u64(x: np.ndarray) -> np.ndarray:
    """round-to-nearest, clamped to [0, 2^64 - 1]"""
    x = np.rint(x)
    hi = x >= TWO64
    x = np.clip(x, 0.0, TWO64 - 2048.0)  # largest double below 2^64
    out = x.astype(np.uint64)
    out[hi] = U64_MAX
    return out


def uniform(n: int, seed: int) -> np.ndarray:
    """i.i.d. uniform over [0, 2^64) (raw 64-bit draws)."""
    return _rng(seed).integers(0, 2**64, size=n, dtype=np.uint64, endpoint=False)


def normal(n: int, seed: int, mean: float = 2.0**62, sd: float = 2.0**52) -> np.ndarray:
    """round(N(mean, sd)) clamped to the u64 range."""
    return _float_to_u64(_rng(seed).normal(mean, sd, size=n))


def dup_heavy(n: int, seed: int, distinct: int = 1000) -> np.ndarray:
    """`distinct` distinct uniform u64 values, keys drawn uniformly among them."""
    rng = _rng(seed)
    vals = np.unique(rng.integers(0, 2**64, size=distinct, dtype=np.uint64, endpoint=False))
    while vals.size < distinct:  # redraw collisions
        extra = rng.integers(0, 2**64, size=distinct - vals.size, dtype=np.uint64, endpoint=False)
        vals = np.unique(np.concatenate([vals, extra]))
    vals = rng.permutation(vals)
    return vals[rng.integers(0, distinct, size=n)]


def partial(n: int, seed: int, swap_frac: float = 0.01) -> np.ndarray:
    """uniform keys sorted ascending, then n*swap_frac swaps of two random positions."""
    rng = _rng(seed)
    x = np.sort(rng.integers(0, 2**64, size=n, dtype=np.uint64, endpoint=False))
    m = int(n * swap_frac)
    if n >= 2 and m:
        i = rng.integers(0, n, size=m)
        j = rng.integers(0, n, size=m)
        for a, b in zip(i.tolist(), j.tolist()):  # sequential swaps, in draw order
            x[a], x[b] = x[b], x[a]
    return x


def descending(n: int, seed: int) -> np.ndarray:
    """uniform keys sorted descending."""
    x = np.sort(_rng(seed).integers(0, 2**64, size=n, dtype=np.uint64, endpoint=False))
    return x[::-1].copy()


def lognormal(n: int, seed: int, mu: float = 40.0, sigma: float = 2.5) -> np.ndarray:
    """floor(exp(N(mu, sigma^2))), values >= 2^64 become 2^64 - 1."""
    x = np.floor(np.exp(_rng(seed).normal(mu, sigma, size=n)))
    hi = x >= TWO64
    x = np.minimum(x, TWO64 - 2048.0)
    out = x.astype(np.uint64)
    out[hi] = U64_MAX
    return out


def zipf(n: int, seed: int, s: float = 1.2, distinct: int = 10**6) -> np.ndarray:
    """Zipf(s) over `distinct` distinct uniform u64 values: rank r with
    probability proportional to r^-s."""
    rng = _rng(seed)
    vals = np.unique(rng.integers(0, 2**64, size=distinct, dtype=np.uint64, endpoint=False))
    while vals.size < distinct:
        extra = rng.integers(0, 2**64, size=distinct - vals.size, dtype=np.uint64, endpoint=False)
        vals = np.unique(np.concatenate([vals, extra]))
    vals = rng.permutation(vals)
    w = np.arange(1, distinct + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    u = rng.random(size=n)
    r = np.minimum(np.searchsorted(cdf, u, side="right"), distinct - 1)
    return vals[r]


GMM_WEIGHTS = (0.4, 0.3, 0.2, 0.1)
GMM_LOG2_SDS = (40.0, 40.0 + 16.0 / 3.0, 40.0 + 32.0 / 3.0, 56.0)


def gmm(n: int, seed: int, perm=(2, 0, 1, 3)) -> np.ndarray:
    """4-component Gaussian mixture: weights 0.4/0.3/0.2/0.1, standard
    deviations 2^40 .. 2^56 spaced evenly in log2, component c centred at
    (2*perm[c] + 1)/8 * 2^63.  The default perm puts the narrowest, heaviest
    component in the middle of the range."""
    rng = _rng(seed)
    comp = rng.choice(4, size=n, p=np.asarray(GMM_WEIGHTS))
    means = np.array([(2 * perm[c] + 1) / 8.0 * 2.0**63 for c in range(4)])
    sds = np.array([2.0**e for e in GMM_LOG2_SDS])
    z = rng.standard_normal(size=n)
    return _float_to_u64(means[comp] + sds[comp] * z)


def segments(nseg: int, seed: int, median: float = 2e4, sigma_ln: float = 1.0,
             lo: int = 100, hi: int = 10**6):
    """Batched workload: nseg arrays with lognormal lengths (median `median`,
    clamped to [lo, hi]); each array's keys are round(N(mu_s, sd_s)) clamped,
    mu_s ~ U[0, 2^63), sd_s = 2^U(30, 58).  Returns (keys, offsets[nseg+1],
    per-segment index payload u32)."""
    rng = _rng(seed)
    lens = np.clip(np.rint(np.exp(rng.normal(math.log(median), sigma_ln, size=nseg))), lo, hi)
    lens = lens.astype(np.int64)
    off = np.zeros(nseg + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    n = int(off[-1])
    mus = rng.random(size=nseg) * 2.0**63
    sds = 2.0 ** rng.uniform(30.0, 58.0, size=nseg)
    seg_of = np.repeat(np.arange(nseg), lens)
    z = rng.standard_normal(size=n)
    keys = _float_to_u64(mus[seg_of] + sds[seg_of] * z)
    idx = (np.arange(n, dtype=np.int64) - off[seg_of]).astype(np.uint32)
    return keys, off, idx


def wide_range_arrays(seed: int):
    """Arrays whose keys span 2^52 .. 2^64 (ranges wider than a 52-bit offset
    next to a 12-bit position), each short enough to be one leaf at cutoff
    4096: uniform over [b, b + 2^w) for w in {53, 56, 60, 64} at lengths
    around one wave's and one workgroup's share, a few distinct values spread
    over 2^58 (repeats of ~40 and of ~400 per value), and three keys spanning
    2^63.  Returns (keys, offsets[m+1]) of the m arrays laid end to end."""
    rng = _rng(seed)
    spec = [(3000, 56, 0), (2000, 64, 0), (400, 60, 0), (400, 64, 0), (700, 53, 0),
            (600, 55, 0), (4096, 64, 0), (513, 58, 0), (2000, 58, 50), (2000, 58, 5),
            (450, 58, 12), (3, 63, 0)]
    arrays = []
    for n, w, distinct in spec:
        span = 1 << w
        base = int(rng.integers(0, 2**64 - span + 1, dtype=np.uint64)) if w < 64 else 0
        if distinct:
            vals = rng.integers(0, span, size=distinct, dtype=np.uint64)
            x = vals[rng.integers(0, distinct, size=n)]
        elif w == 64:
            x = rng.integers(0, 2**64 - 1, size=n, dtype=np.uint64, endpoint=True)
        else:
            x = rng.integers(0, span, size=n, dtype=np.uint64)
        arrays.append((np.uint64(base) + x).astype(np.uint64))
    off = np.zeros(len(arrays) + 1, dtype=np.int64)
    np.cumsum([a.size for a in arrays], out=off[1:])
    return np.concatenate(arrays), off


def small_range(n: int, seed: int, span: int = 200) -> np.ndarray:
    """Restricted range: keys uniform over [b, b + span) for a random base b
    (the high-duplicate family of the paper draws from a restricted range)."""
    rng = _rng(seed)
    base = int(rng.integers(0, 2**64 - span, dtype=np.uint64))
    return (np.uint64(base) + rng.integers(0, span, size=n, dtype=np.uint64)).astype(np.uint64)


def clustered_ranges(n: int, seed: int, clusters: int = 20, span: int = 150) -> np.ndarray:
    """Half the keys uniform over [0, 2^64), half in `clusters` narrow ranges
    of `span` values at random places (small ranges show up below the root)."""
    rng = _rng(seed)
    out = rng.integers(0, 2**64, size=n, dtype=np.uint64, endpoint=False)
    bases = rng.integers(0, 2**64 - span, size=clusters, dtype=np.uint64)
    pick = rng.random(n) < 0.5
    m = int(pick.sum())
    out[pick] = bases[rng.integers(0, clusters, size=m)] + rng.integers(0, span, size=m,
                                                                           dtype=np.uint64)
    return out


# name -> (workload index, variant, generator)
WORKLOADS = {
    "uniform_2p20": (0, 0, uniform),
    "uniform": (1, 0, uniform),
    "normal": (1, 1, normal),
    "dup_heavy": (1, 2, dup_heavy),
    "partial": (1, 3, partial),
    "descending": (1, 4, descending),
    "lognormal": (2, 0, lognormal),
    "zipf": (2, 1, zipf),
    "gmm": (4, 0, gmm),
    "gmm_identity": (4, 1, lambda n, s: gmm(n, s, perm=(0, 1, 2, 3))),
    "uniform_1e8": (5, 0, uniform),
    "small_range": (6, 0, small_range),
    "clustered_ranges": (6, 1, clustered_ranges),
}


def make(name: str, n: int, payload_bytes: int = 4):
    """keys (u64) and index payload (u32, u64, or None for 0 bytes)."""
    wi, var, fn = WORKLOADS[name]
    keys = fn(n, seed_for(wi, var))
    if payload_bytes == 0:
        pay = None
    elif payload_bytes == 4:
        pay = np.arange(n, dtype=np.uint32)
    elif payload_bytes == 8:
        pay = np.arange(n, dtype=np.uint64)
    else:
        raise ValueError("payload_bytes must be 0, 4 or 8")
    return keys, pay


# ---------------------------------------------------------------------------
# 128-bit keys: (n, 2) u64 arrays, low word first
# ---------------------------------------------------------------------------
WORKLOADS128 = {"uuid": 0, "prefix": 1, "narrow": 2, "zext": 3, "dup": 4}


def make128(name: str, n: int):
    """keys (n, 2) u64 [lo, hi] and the u32 index payload.
    uuid   -- both words i.i.d. uniform (random 128-bit identifiers)
    prefix -- high word from 1000 distinct uniform values, low word uniform
              (runs of equal high words of ~n/1000 keys)
    narrow -- high word from n/20 distinct values (runs of ~20 keys)
    zext   -- high word 0, low word lognormal as the 64-bit lognormal family
              (one run: the whole array)
    dup    -- 500 distinct (high, low) pairs, keys uniform among them"""
    seed = seed_for(7, WORKLOADS128[name])
    rng = _rng(seed)
    k = np.empty((n, 2), dtype=np.uint64)
    if name == "uuid":
        k[:, 0] = rng.integers(0, 2**64, size=n, dtype=np.uint64, endpoint=False)
        k[:, 1] = rng.integers(0, 2**64, size=n, dtype=np.uint64, endpoint=False)
    elif name in ("prefix", "narrow"):
        d = 1000 if name == "prefix" else max(1, n // 20)
        vals = rng.integers(0, 2**64, size=d, dtype=np.uint64, endpoint=False)
        k[:, 1] = vals[rng.integers(0, d, size=n)]
        k[:, 0] = rng.integers(0, 2**64, size=n, dtype=np.uint64, endpoint=False)
    elif name == "zext":
        k[:, 1] = 0
        k[:, 0] = lognormal(n, seed)
    elif name == "dup":
        vals = rng.integers(0, 2**64, size=(500, 2), dtype=np.uint64, endpoint=False)
        k[:] = vals[rng.integers(0, 500, size=n)]
    else:
        raise KeyError(name)
    return k, np.arange(n, dtype=np.uint32)
