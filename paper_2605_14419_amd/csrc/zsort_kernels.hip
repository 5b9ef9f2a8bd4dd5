// zsort_kernels.hip -- HIP kernels (gfx950) of the breadth-first zSort.
//
// Method: "zSort: Stable Distribution Sort using Z-Score Partitioning",
// Section III (z-score standardisation, shift by |z_min|, scale, the mapping
// function of Eq. (1) with the clip of the cluster definition, duplicate
// handling, the recursive phase with the estimated mean) and Algorithm 1.
//
// Exactness conventions (identical to the reading used by the tests):
//   * moments are exact integers (32-bit digit sums accumulated in 64-bit
//     words, combined into 256-bit integers at finalize);
//   * the statistics are binary64, round-to-nearest-even, in one fixed order,
//     compiled with -ffp-contract=off; the map uses one explicit fma;
//   * a segment is rebased to its exact minimum before any conversion.
#include <hip/hip_runtime.h>
#include <math.h>
#include "zsort_internal.h"
#include "zsort_mlp.h"

namespace zs {

// ---------------------------------------------------------------------------
// wave / block primitives
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t lane() { return threadIdx.x & (kWave - 1); }
__device__ __forceinline__ uint32_t wave() { return threadIdx.x / kWave; }

// number of set bits of m below this lane
__device__ __forceinline__ uint32_t below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// lanes of `active` whose digit equals this lane's digit (BITS-bit digits)
template <int BITS>
__device__ __forceinline__ uint64_t match_digit(uint32_t d, uint64_t active) {
  uint64_t m = active;
#pragma unroll
  for (int i = 0; i < BITS; ++i) {
    const bool bit = (d >> i) & 1u;
    const uint64_t b = __ballot(bit);
    m &= bit ? b : ~b;
  }
  return m;
}

// Inclusive sum over the wave by DPP moves (all 64 lanes active): shifts by
// 1, 2, 4, 8 inside each row of 16 lanes (lanes before the row start read
// 0), then the last lane of row 0 is added to row 1 and that of row 2 to
// row 3 (row_bcast:15), and the last lane of row 1 to rows 2 and 3
// (row_bcast:31).
__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false);  // row_shr:1
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, false);  // row_shr:2
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false);  // row_shr:4
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, false);  // row_shr:8
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);  // row_bcast:15
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);  // row_bcast:31
  return v;
}

// 64-bit value of the DPP source lane (CTRL, ROWS as above), `idv` where the
// lane has no source
template <int CTRL, int ROWS>
__device__ __forceinline__ uint64_t dpp64(uint64_t idv, uint64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)idv, (int)(uint32_t)v,
                                                             CTRL, ROWS, 0xF, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)(idv >> 32),
                                                             (int)(uint32_t)(v >> 32), CTRL, ROWS,
                                                             0xF, false);
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
  return ((uint64_t)hi << 32) | lo;
}

// minimum and maximum over the wave (all 64 lanes active), the same DPP
// pattern as wave_incl_sum; the last lane holds the result, read by all
__device__ __forceinline__ void wave_minmax_u64(uint64_t& mn, uint64_t& mx) {
  uint64_t a, b;
#define ZS_MM_STEP(CTRL, ROWS)                        \
  a = dpp64<CTRL, ROWS>(~0ull, mn);                   \
  b = dpp64<CTRL, ROWS>(0ull, mx);                    \
  mn = a < mn ? a : mn;                               \
  mx = b > mx ? b : mx;
  ZS_MM_STEP(0x111, 0xF)
  ZS_MM_STEP(0x112, 0xF)
  ZS_MM_STEP(0x114, 0xF)
  ZS_MM_STEP(0x118, 0xF)
  ZS_MM_STEP(0x142, 0xA)
  ZS_MM_STEP(0x143, 0xC)
#undef ZS_MM_STEP
  mn = readlane64(mn, kWave - 1);
  mx = readlane64(mx, kWave - 1);
}

// the ten moment words of every lane reduced over the wave (sums of the
// first eight, min and max of the last two), the result in every lane
__device__ __forceinline__ void wave_reduce_moments(uint64_t (&v)[10]) {
#define ZS_RM_STEP(CTRL, ROWS)                                      \
  {                                                                 \
    _Pragma("unroll") for (int j = 0; j < 8; ++j) v[j] += dpp64<CTRL, ROWS>(0ull, v[j]); \
    const uint64_t a = dpp64<CTRL, ROWS>(~0ull, v[8]);             \
    const uint64_t b = dpp64<CTRL, ROWS>(0ull, v[9]);              \
    v[8] = a < v[8] ? a : v[8];                                     \
    v[9] = b > v[9] ? b : v[9];                                     \
  }
  ZS_RM_STEP(0x111, 0xF)
  ZS_RM_STEP(0x112, 0xF)
  ZS_RM_STEP(0x114, 0xF)
  ZS_RM_STEP(0x118, 0xF)
  ZS_RM_STEP(0x142, 0xA)
  ZS_RM_STEP(0x143, 0xC)
#undef ZS_RM_STEP
#pragma unroll
  for (int j = 0; j < 10; ++j) v[j] = readlane64(v[j], kWave - 1);
}

__device__ __forceinline__ int wave_incl_max(int v) {
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    int t = __shfl_up(v, o);
    if (lane() >= (uint32_t)o) v = max(v, t);
  }
  return v;
}

// exclusive block sum of one value per thread (NT threads); `sh` holds
// NT / kWave words
template <int NT = kBlock>
__device__ __forceinline__ uint32_t block_excl_sum(uint32_t v, uint32_t* sh, uint32_t* total) {
  uint32_t inc = wave_incl_sum(v);
  if (lane() == kWave - 1) sh[wave()] = inc;
  __syncthreads();
  uint32_t base = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < NT / kWave; ++i) {
    uint32_t s = sh[i];
    base += (i < (int)wave()) ? s : 0u;
    tot += s;
  }
  __syncthreads();
  if (total) *total = tot;
  return base + inc - v;
}

// in-place exclusive sum over a[0, N) in LDS; returns the total
template <int NT = kBlock>
__device__ uint32_t block_scan_lds(uint32_t* a, int N, uint32_t* sh) {
  const int ipt = (N + NT - 1) / NT;
  const int b0 = threadIdx.x * ipt;
  uint32_t s = 0;
  for (int i = 0; i < ipt; ++i) {
    int j = b0 + i;
    if (j < N) s += a[j];
  }
  uint32_t tot;
  uint32_t base = block_excl_sum<NT>(s, sh, &tot);
  for (int i = 0; i < ipt; ++i) {
    int j = b0 + i;
    if (j < N) {
      uint32_t t = a[j];
      a[j] = base;
      base += t;
    }
  }
  __syncthreads();
  return tot;
}

// in-place exclusive max over a[0, N) in LDS (identity -1)
// NA exclusive scans of N-element LDS arrays in one pass (two barriers for
// all of them); tot receives each array's total
template <int NA>
__device__ void block_scan_multi(uint32_t* const (&a)[NA], int N, uint32_t (*sh)[kWaves],
                                 uint32_t (&tot)[NA]) {
  const int ipt = (N + kBlock - 1) / kBlock;
  const int b0 = threadIdx.x * ipt;
  uint32_t s[NA], inc[NA];
#pragma unroll
  for (int q = 0; q < NA; ++q) {
    s[q] = 0;
    for (int i = 0; i < ipt; ++i)
      if (b0 + i < N) s[q] += a[q][b0 + i];
    inc[q] = wave_incl_sum(s[q]);
    if (lane() == kWave - 1) sh[q][wave()] = inc[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NA; ++q) {
    uint32_t base = 0, t = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      const uint32_t v = sh[q][w];
      base += (w < (int)wave()) ? v : 0u;
      t += v;
    }
    tot[q] = t;
    base += inc[q] - s[q];
    for (int i = 0; i < ipt; ++i) {
      if (b0 + i < N) {
        const uint32_t x = a[q][b0 + i];
        a[q][b0 + i] = base;
        base += x;
      }
    }
  }
  __syncthreads();
}

// three exclusive sums of one value per thread at once
template <int NA>
__device__ __forceinline__ void block_excl_sums(const uint32_t (&v)[NA], uint32_t (*sh)[kWaves],
                                                uint32_t (&ex)[NA], uint32_t (&tot)[NA]) {
  uint32_t inc[NA];
#pragma unroll
  for (int q = 0; q < NA; ++q) {
    inc[q] = wave_incl_sum(v[q]);
    if (lane() == kWave - 1) sh[q][wave()] = inc[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NA; ++q) {
    uint32_t base = 0, t = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      const uint32_t x = sh[q][w];
      base += (w < (int)wave()) ? x : 0u;
      t += x;
    }
    ex[q] = base + inc[q] - v[q];
    tot[q] = t;
  }
  __syncthreads();
}

__device__ void block_excl_max_lds(int* a, int N, int* sh) {
  const int ipt = (N + kBlock - 1) / kBlock;
  const int b0 = threadIdx.x * ipt;
  int s = -1;
  for (int i = 0; i < ipt; ++i) {
    int j = b0 + i;
    if (j < N) s = max(s, a[j]);
  }
  int inc = wave_incl_max(s);
  if (lane() == kWave - 1) sh[wave()] = inc;
  __syncthreads();
  int base = -1;
  for (int i = 0; i < (int)wave(); ++i) base = max(base, sh[i]);
  int ex = __shfl_up(inc, 1);
  if (lane() == 0) ex = -1;
  base = max(base, ex);
  __syncthreads();
  for (int i = 0; i < ipt; ++i) {
    int j = b0 + i;
    if (j < N) {
      int t = a[j];
      a[j] = base;
      base = max(base, t);
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// exact 256-bit unsigned arithmetic on eight 32-bit limbs (device side)
// ---------------------------------------------------------------------------
struct W8 {
  uint32_t d[8];
};

__device__ __forceinline__ W8 w8_zero() {
  W8 r;
#pragma unroll
  for (int i = 0; i < 8; ++i) r.d[i] = 0;
  return r;
}

// r += v * 2^(32*pos) for a 64-bit v.  Every loop below runs its full
// length with constant limb indices, so the numbers stay in registers.
__device__ __forceinline__ void w8_add64_at(W8& r, uint64_t v, int pos) {
  uint64_t carry = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    uint64_t add = carry;
    if (i == pos) add += (uint32_t)v;
    if (i == pos + 1) add += (uint32_t)(v >> 32);
    const uint64_t s = (uint64_t)r.d[i] + add;
    r.d[i] = (uint32_t)s;
    carry = s >> 32;
  }
}

__device__ __forceinline__ W8 w8_add(const W8& a, const W8& b) {
  W8 r;
  uint64_t c = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    uint64_t s = (uint64_t)a.d[i] + b.d[i] + c;
    r.d[i] = (uint32_t)s;
    c = s >> 32;
  }
  return r;
}

// a - b for a >= b
__device__ __forceinline__ W8 w8_sub(const W8& a, const W8& b) {
  W8 r;
  int64_t br = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    int64_t s = (int64_t)a.d[i] - (int64_t)b.d[i] - br;
    br = s < 0 ? 1 : 0;
    r.d[i] = (uint32_t)(s + (br << 32));
  }
  return r;
}

// full product of two numbers given as limb arrays (results must fit)
__device__ __forceinline__ W8 w8_mul(const W8& a, const W8& b) {
  W8 r = w8_zero();
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    uint64_t carry = 0;
#pragma unroll
    for (int j = 0; i + j < 8; ++j) {
      uint64_t t = (uint64_t)a.d[i] * b.d[j] + r.d[i + j] + carry;
      r.d[i + j] = (uint32_t)t;
      carry = t >> 32;
    }
  }
  return r;
}

__device__ __forceinline__ W8 w8_from64(uint64_t v) {
  W8 r = w8_zero();
  r.d[0] = (uint32_t)v;
  r.d[1] = (uint32_t)(v >> 32);
  return r;
}

// round-to-nearest-even conversion: the 64 bits below the leading one, with
// every lower bit folded into a sticky bit, then an exact power-of-two scale.
// Written with constant limb indices only, so the number stays in registers.
__device__ __forceinline__ double w8_to_double(const W8& a) {
  int top = -1;
#pragma unroll
  for (int i = 0; i < 8; ++i) top = a.d[i] ? i : top;
  if (top < 0) return 0.0;
  if (top <= 1) return __ull2double_rn(((uint64_t)a.d[1] << 32) | a.d[0]);
  uint32_t l2 = 0, l1 = 0, l0 = 0;
  bool sticky = false;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    l2 = (i == top) ? a.d[i] : l2;
    l1 = (i == top - 1) ? a.d[i] : l1;
    l0 = (i == top - 2) ? a.d[i] : l0;
    sticky = sticky || (i < top - 2 && a.d[i] != 0u);
  }
  // window = l2:l1:l0 (96 bits), leading one at bit 64 + (31 - clz(l2))
  const int lz = __clz(l2);                 // 0..31
  const uint64_t hi = ((uint64_t)l2 << 32) | l1;
  uint64_t w;
  if (lz == 0) {
    w = hi;
    sticky = sticky || (l0 != 0u);
  } else {
    w = (hi << lz) | ((uint64_t)l0 >> (32 - lz));
    sticky = sticky || ((l0 << lz) != 0u);
  }
  if (sticky) w |= 1u;
  const int s = 32 * (top - 2) + (32 - lz);  // bits below the 64-bit window
  return ldexp(__ull2double_rn(w), s);
}

// ---------------------------------------------------------------------------
// the map (Eq. (1) with the clip), range map of the progress guard
// ---------------------------------------------------------------------------
struct MapP {
  uint64_t o;
  double m, A, B;
  int k;
  int kind;
  int shift;
};

__device__ __forceinline__ MapP map_of(const Seg& s, int k) {
  MapP p;
  p.o = s.o; p.m = s.m; p.A = s.A; p.B = s.B; p.k = k; p.kind = s.kind; p.shift = s.shift;
  // a counting pass is the exact range map with every key value a cluster
  if (s.kind == KIND_COUNT) { p.kind = KIND_RMAP; p.shift = 0; }
  return p;
}

__device__ __forceinline__ uint32_t bucket_of(uint64_t x, const MapP& p) {
  if (p.kind == KIND_RMAP) return (uint32_t)((x - p.o) >> p.shift);
  const double xr = __ull2double_rn(x - p.o);
  const double t = __fma_rn(xr - p.m, p.A, p.B);
  const double f = floor(t);
  if (!(f >= 0.0)) return 0u;
  if (f >= (double)(p.k - 1)) return (uint32_t)(p.k - 1);
  return (uint32_t)f;
}

// ---------------------------------------------------------------------------
// payload access
// ---------------------------------------------------------------------------
template <int PW> struct PayT { using T = uint32_t; };
template <> struct PayT<8> { using T = uint64_t; };

template <int PW>
__device__ __forceinline__ typename PayT<PW>::T pay_load(const void* p, uint64_t i) {
  if constexpr (PW == 0) return 0;
  else return ((const typename PayT<PW>::T*)p)[i];
}
template <int PW>
__device__ __forceinline__ void pay_store(void* p, uint64_t i, typename PayT<PW>::T v) {
  if constexpr (PW != 0) ((typename PayT<PW>::T*)p)[i] = v;
}

// ---------------------------------------------------------------------------
// Visit keys x[beg, end) with the whole workgroup: 16-byte loads of key
// pairs, UNROLL pairs in flight per thread, plus the unaligned head/tail key.
// Order of visits is unspecified (only order-free reductions use this).
// ---------------------------------------------------------------------------
template <int UNROLL, typename F>
__device__ __forceinline__ void for_each_key(const uint64_t* __restrict__ x, uint64_t beg,
                                             uint64_t end, F&& f) {
  const uint64_t mis = ((uintptr_t)x >> 3) & 1u;  // index i is 16-byte aligned iff (i+mis) even
  const uint64_t a0 = beg + ((beg + mis) & 1u);
  const uint64_t a1 = end - ((end + mis) & 1u);
  const int t = threadIdx.x;
  if (t == 0 && beg < a0 && beg < end) f(beg, x[beg]);
  if (t == 1 && a1 >= a0 && a1 < end) f(a1, x[a1]);
  if (a1 <= a0) return;
  const ulonglong2* __restrict__ xp = reinterpret_cast<const ulonglong2*>(x + a0);
  const uint64_t np = (a1 - a0) >> 1;
  // two register sets: the next group of key pairs is loaded before the
  // current one is visited, so that every wave keeps loads in flight
  const uint64_t step = (uint64_t)kBlock * UNROLL;
  ulonglong2 va[UNROLL], vb[UNROLL];
  auto load = [&](ulonglong2 (&v)[UNROLL], uint64_t p) {
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
      const uint64_t q = p + (uint64_t)u * kBlock;
      if (q < np) v[u] = xp[q];
    }
  };
  auto visit = [&](const ulonglong2 (&v)[UNROLL], uint64_t p) {
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
      const uint64_t q = p + (uint64_t)u * kBlock;
      if (q < np) { f(a0 + 2 * q, v[u].x); f(a0 + 2 * q + 1, v[u].y); }
    }
  };
  uint64_t p = t;
  if (p < np) load(va, p);
  while (p < np) {
    if (p + step < np) load(vb, p + step);
    visit(va, p);
    p += step;
    if (p >= np) break;
    if (p + step < np) load(va, p + step);
    visit(vb, p);
    p += step;
  }
}

// a capacity or wait limit was hit earlier in this call: later kernels stop
__device__ __forceinline__ bool call_failed(const Ctl* c) {
  return __hip_atomic_load(&c->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
}

// ---------------------------------------------------------------------------
// scan rows shared between the workgroups of a level: words tag(22) |
// value(40), stored and loaded at device scope.  No fence orders a row
// before the arrival count that announces it (a device-scope fence writes
// back and invalidates a whole L2); instead a reader that finds an older tag
// waits for the word itself, which at most takes the store's flight time.
// ---------------------------------------------------------------------------
constexpr uint64_t kValMask = (1ull << 40) - 1;
constexpr uint32_t kSpinLimit = 1u << 20;

__device__ __forceinline__ uint32_t level_tag(uint32_t epoch, int L) {
  return 1u + (uint32_t)(((uint64_t)epoch * 64u + (uint32_t)L) % kTagMod);
}
__device__ __forceinline__ void row_put(uint64_t* p, uint32_t tag, uint64_t v) {
  __hip_atomic_store(p, ((uint64_t)tag << 42) | (v & kValMask), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t row_peek(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// the value of a word already loaded as w, once it carries `tag`
__device__ __forceinline__ uint32_t row_value(const uint64_t* p, uint64_t w, uint32_t tag, Ctl* c) {
  uint32_t spins = 0;
  while ((uint32_t)(w >> 42) != tag) {
    if (++spins > kSpinLimit || ((spins & 255u) == 0u && call_failed(c))) {
      atomicOr(&c->error, ERR_SPIN);
      return 0u;
    }
    __builtin_amdgcn_s_sleep(1);
    w = row_peek(p);
  }
  return (uint32_t)(w & kValMask);
}

// arrival counters of a new segment of nch chunks: one per scan unit, one for
// the segment (the level's hist pass counts on them starting at zero)
__device__ __forceinline__ void clear_arrivals(uint32_t* arr, uint32_t nch) {
  if (nch > 1)
    for (uint32_t i = 0, e = scan_units(nch); i <= e; ++i) arr[i] = 0u;
}



// ---------------------------------------------------------------------------
// reset + level-0 set-up
// ---------------------------------------------------------------------------
__device__ void seg_clear_acc(Seg& s) {
  s.kind = KIND_PENDING;
  s.shift = 0;
  s.o = s.M = 0;
  s.m = s.sigma = s.zmin = s.A = s.B = 0.0;
}

// a child (index idx of the level being made) whose statistics its parent's
// scatter accumulates
__device__ void seg_fuse_init(const Ws& ws, Seg& s, uint32_t idx) {
  uint64_t* f = ws.facc + (uint64_t)idx * 10;
  for (int j = 0; j < 8; ++j) f[j] = 0ull;
  f[8] = ~0ull;
  f[9] = 0ull;
  s.flags |= F_FUSED;
}

__global__ void k_reset(Ws ws) {
  Ctl* c = ws.ctl;
  const int t = threadIdx.x;
  if (t < kMaxLevels) {
    c->tick[t] = 0;
    c->hdone[t] = 0;
    c->lvl_keys[t] = 0;
    c->lvl_mkeys[t] = 0;
    c->lvl_fkeys[t] = 0;
    c->lvl_segs[t] = 0;
  }
  if (t == 0) {
    const uint32_t ep = c->epoch + 1u;
    c->epoch = ep;
    // a new layout of the rows, the end of the window in which tags are
    // distinct, or the wrap of the epoch counter (tags before and after it
    // are not distinct): the set-up kernel of this call clears the rows
    const bool clr = ws.force_clear != 0u || ep == 0u ||
                     (uint32_t)(ep - c->clear_epoch) >= kClearEvery;
    c->clear_rows = clr ? 1u : 0u;
    if (clr) c->clear_epoch = ep;
    for (int s = 0; s < 2; ++s) {
      c->nseg[s] = 0; c->nwork[s] = 0; c->nleaf[s] = 0; c->nleafw[s] = 0; c->nleafm[s] = 0;
      c->nleafx[s] = 0; c->nhard[s] = 0;
      c->nstatus[s] = 0; c->ntile[s] = 0;
    }
    c->error = 0;
    c->ntrace = 0;
    c->ntrace_hist = 0;
    c->n_ident = c->n_rmap = c->n_leafgroups = 0;
    c->n_count = 0;
    c->n_hard = 0;
    c->max_level = 0;
    c->local_keys = 0;
  }
}

// appends a sort job for keys [start, start+count) living in buffer `src`
// of level-slot S: groups of <= wave_job_cap(pw) keys go to the wave list
__device__ bool push_leaf(Ws& ws, int S, uint64_t start, uint32_t count, uint32_t flags,
                          uint32_t src) {
  Ctl* c = ws.ctl;
  const bool small = !(flags & LF_COPY) && count <= (uint32_t)wave_job_cap(ws.p.pw);
  const bool mid = !(flags & LF_COPY) && !small && count <= (uint32_t)kMidCap;
  uint32_t* ctr = small ? &c->nleafw[S] : (mid ? &c->nleafm[S] : &c->nleaf[S]);
  const uint32_t li = atomicAdd(ctr, 1u);
  if (li >= ws.leaf_cap) {
    atomicOr(&c->error, ERR_LEAFCAP);
    return false;
  }
  Leaf& lf = small ? ws.leavesw[S][li] : (mid ? ws.leavesm[S][li] : ws.leaves[S][li]);
  lf.start = (uint32_t)start;
  lf.count = count;
  lf.flags = flags;
  lf.src = src;
  return true;
}

// 8192-key tiles: scatter items per work item (1 with smaller tiles)
__device__ __forceinline__ uint32_t tiles_per_item(const Ws& ws) {
  return ws.p.tile == 8192 ? (uint32_t)((uint32_t)ws.p.chunk >> 13) : 1u;
}

// tile u of segment si: (segment << 32) | (chunk << 3) | tile in the chunk
__device__ __forceinline__ uint64_t tile_entry(uint32_t si, uint32_t u, uint32_t nsub) {
  return ((uint64_t)si << 32) | ((u / nsub) << 3) | (u % nsub);
}

__device__ void make_root_seg(Ws& ws, uint32_t slot_seg, uint64_t start, uint64_t count,
                              uint32_t first_work, uint32_t nch, uint32_t status_base) {
  Seg& s = ws.segs[0][slot_seg];
  s.start = start;
  s.count = count;
  s.o_parent = 0;
  s.e = 0.0;
  s.depth = 0;
  s.flags = F_ROOT | (ws.p.max_zlevels == 0 ? F_RMAP : 0u);
  s.first_work = first_work;
  s.nchunks = nch;
  s.status_base = status_base;
  s.parent = -1;
  seg_clear_acc(s);
}

// tile list of the single root segment [0, n) (8192-key tiles only)
__device__ void init_root_tiles(Ws& ws, uint64_t n) {
  const uint32_t nsub = tiles_per_item(ws);
  if (nsub == 1) return;
  const uint32_t ntl = (uint32_t)((n + 8191) >> 13);
  if (blockIdx.x == 0 && threadIdx.x == 0) ws.ctl->ntile[0] = ntl;
  for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < ntl; u += gridDim.x * blockDim.x)
    ws.tiles[0][u] = tile_entry(0u, u, nsub);
}

// arrival counters of the single root segment (rows from 0)
__device__ void init_root_arrivals(Ws& ws, uint32_t nch) {
  if (nch <= 1) return;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i <= scan_units(nch);
       i += gridDim.x * blockDim.x)
    ws.arrive[0][i] = 0u;
}

// the scan rows, zeroed by the whole grid when k_reset asked for it (no row
// is read before the histogram pass, which runs after this kernel)
__device__ void clear_rows_if_due(const Ws& ws) {
  if (__hip_atomic_load(&ws.ctl->clear_rows, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u)
    return;
  const uint64_t np = ws.status_words >> 1;
  ulonglong2* p = reinterpret_cast<ulonglong2*>(ws.status);
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np; i += stride)
    p[i] = make_ulonglong2(0ull, 0ull);
  if (blockIdx.x == 0 && threadIdx.x == 0 && (ws.status_words & 1u))
    ws.status[ws.status_words - 1] = 0ull;
}

__global__ void k_clear_rows(Ws ws) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ws.status_words; i += stride)
    ws.status[i] = 0ull;
}

// one array [0, n): root segment (n > cutoff) or a single leaf
__global__ void k_init_single(Ws ws, uint64_t n) {
  clear_rows_if_due(ws);
  Ctl* c = ws.ctl;
  const uint64_t ch = (uint64_t)ws.p.chunk;
  if (n <= (uint64_t)ws.p.cutoff) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      push_leaf(ws, 0, 0, (uint32_t)n, 0u, 0u);
      c->n_leafgroups = 1;
    }
    return;
  }
  const uint32_t nch = (uint32_t)((n + ch - 1) / ch);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    make_root_seg(ws, 0, 0, n, 0, nch, 0);
    c->nseg[0] = 1;
    c->nwork[0] = nch;
    c->nstatus[0] = status_rows(nch);
  }
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nch; i += gridDim.x * blockDim.x)
    ws.work[0][i] = (uint64_t)i;  // segment 0, chunk i
  init_root_arrivals(ws, nch);
  init_root_tiles(ws, n);
}

// empties the lists of one slot (a level that runs no moments pass)
__global__ void k_reset_lists(Ws ws, int slot) {
  Ctl* c = ws.ctl;
  if (threadIdx.x == 0) {
    c->nseg[slot] = 0; c->nwork[slot] = 0; c->nleaf[slot] = 0; c->nleafw[slot] = 0; c->nleafm[slot] = 0;
    c->nleafx[slot] = 0;
    c->nhard[slot] = 0; c->nstatus[slot] = 0; c->ntile[slot] = 0;
  }
}

// one array [0, n), n > cutoff, whose first pass uses the learned map
__global__ void k_init_learned(Ws ws, uint64_t n) {
  clear_rows_if_due(ws);
  Ctl* c = ws.ctl;
  const uint64_t ch = (uint64_t)ws.p.chunk;
  const uint32_t nch = (uint32_t)((n + ch - 1) / ch);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    make_root_seg(ws, 0, 0, n, 0, nch, 0);
    Seg& s = ws.segs[0][0];
    s.flags = 0;
    s.kind = KIND_LMAP;
    s.o = 0;
    s.M = ~0ull;
    // window: every threshold, or with two stages every sub-th one
    const uint32_t nt = ws.lm.res->nt, sub = ws.lm.sub;
    s.lm_base = sub ? sub - 1 : 0;
    s.lm_cnt = sub ? nt / sub : nt;
    s.shift = sub ? (int32_t)sub : 1;
    c->nseg[0] = 1;
    c->nwork[0] = nch;
    c->nstatus[0] = status_rows(nch);
  }
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nch; i += gridDim.x * blockDim.x)
    ws.work[0][i] = (uint64_t)i;
  init_root_arrivals(ws, nch);
  init_root_tiles(ws, n);
}

// independent arrays [off[i], off[i+1]); offsets were validated by k_check_offsets
__global__ void k_check_offsets(Ws ws, const int64_t* off, int32_t nseg, uint64_t n) {
  clear_rows_if_due(ws);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i <= nseg; i += gridDim.x * blockDim.x) {
    bool bad = false;
    if (i == 0 && off[0] != 0) bad = true;
    if (i == nseg && (uint64_t)off[nseg] != n) bad = true;
    if (i < nseg && off[i + 1] < off[i]) bad = true;
    if (bad) atomicOr(&ws.ctl->error, 0x100u);
  }
}

// independent subproblem [a, a + len) of level 0 (one array of a batch, or
// one run of equal high words of 128-bit keys): a leaf, or a root segment
// with its work items and tiles
__device__ void init_root(Ws& ws, uint64_t a, uint64_t len) {
  Ctl* c = ws.ctl;
  const uint64_t ch = (uint64_t)ws.p.chunk;
  if (len <= 1) return;
  if (len <= (uint64_t)ws.p.cutoff) {
    push_leaf(ws, 0, a, (uint32_t)len, 0u, 0u);
    atomicAdd(&c->n_leafgroups, 1u);
    return;
  }
  const uint32_t nch = (uint32_t)((len + ch - 1) / ch);
  uint32_t si = atomicAdd(&c->nseg[0], 1u);
  uint32_t wi = atomicAdd(&c->nwork[0], nch);
  uint32_t sb = nch > 1 ? atomicAdd(&c->nstatus[0], status_rows(nch)) : 0u;
  if (si >= ws.seg_cap || wi + nch > ws.work_cap || sb + status_rows(nch) > ws.status_cap) {
    atomicOr(&c->error, ERR_SEGCAP);
    return;
  }
  make_root_seg(ws, si, a, len, wi, nch, sb);
  clear_arrivals(ws.arrive[0] + sb, nch);
  for (uint32_t j = 0; j < nch; ++j) ws.work[0][wi + j] = ((uint64_t)si << 32) | j;
  const uint32_t nsub = tiles_per_item(ws);
  if (nsub > 1) {
    const uint32_t ntl = (uint32_t)((len + 8191) >> 13);
    const uint32_t ti = atomicAdd(&c->ntile[0], ntl);
    if (ti + ntl > ws.tile_cap) {
      atomicOr(&c->error, ERR_WORKCAP);
      return;
    }
    for (uint32_t u = 0; u < ntl; ++u) ws.tiles[0][ti + u] = tile_entry(si, u, nsub);
  }
}

__global__ void k_init_segments(Ws ws, const int64_t* off, int32_t nseg) {
  Ctl* c = ws.ctl;
  if (__hip_atomic_load(&c->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nseg; i += gridDim.x * blockDim.x)
    init_root(ws, (uint64_t)off[i], (uint64_t)(off[i + 1] - off[i]));
}

// subproblems given as (start, length) pairs, *nruns of them (device count):
// a workgroup per run, whose thread 0 makes the segment (or the leaf) and
// whose threads then write its work items and tiles (a run may be the whole
// array: thousands of entries)
__global__ void k_init_runs(Ws ws, const uint32_t* runs, const uint32_t* nruns) {
  clear_rows_if_due(ws);
  Ctl* c = ws.ctl;
  __shared__ uint32_t sh[5];   // segment, first work item, chunks, first tile, tiles
  const uint32_t nr = *nruns;
  const uint64_t ch = (uint64_t)ws.p.chunk;
  const uint32_t nsub = tiles_per_item(ws);
  const int t = threadIdx.x;
  for (uint32_t i = blockIdx.x; i < nr; i += gridDim.x) {
    const uint64_t a = runs[2 * i], len = runs[2 * i + 1];
    if (t == 0) {
      sh[2] = 0u;   // nothing to write unless a segment is made
      if (len > (uint64_t)ws.p.cutoff) {
        const uint32_t nch = (uint32_t)((len + ch - 1) / ch);
        const uint32_t ntl = nsub > 1 ? (uint32_t)((len + 8191) >> 13) : 0u;
        const uint32_t si = atomicAdd(&c->nseg[0], 1u);
        const uint32_t wi = atomicAdd(&c->nwork[0], nch);
        const uint32_t sb = nch > 1 ? atomicAdd(&c->nstatus[0], status_rows(nch)) : 0u;
        const uint32_t ti = ntl ? atomicAdd(&c->ntile[0], ntl) : 0u;
        if (si >= ws.seg_cap || wi + nch > ws.work_cap || sb + status_rows(nch) > ws.status_cap) {
          atomicOr(&c->error, ERR_SEGCAP);
        } else if (ntl && ti + ntl > ws.tile_cap) {
          atomicOr(&c->error, ERR_WORKCAP);
        } else {
          make_root_seg(ws, si, a, len, wi, nch, sb);
          clear_arrivals(ws.arrive[0] + sb, nch);
          sh[0] = si; sh[1] = wi; sh[2] = nch; sh[3] = ti; sh[4] = ntl;
        }
      } else if (len > 1) {
        push_leaf(ws, 0, a, (uint32_t)len, 0u, 0u);
        atomicAdd(&c->n_leafgroups, 1u);
      }
    }
    __syncthreads();
    const uint32_t nch = sh[2];
    if (nch) {
      const uint64_t segw = (uint64_t)sh[0] << 32;
      for (uint32_t j = t; j < nch; j += blockDim.x) ws.work[0][sh[1] + j] = segw | j;
      for (uint32_t u = t; u < sh[4]; u += blockDim.x) ws.tiles[0][sh[3] + u] = tile_entry(sh[0], u, nsub);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// finalize: exact moments -> statistics of the map (one thread per segment)
// ---------------------------------------------------------------------------
__device__ void trace_ident(Ws& ws, const Seg& s) {
  if (!ws.trace) return;
  uint32_t i = atomicAdd(&ws.ctl->ntrace, 1u);
  if (i >= ws.trace_cap) return;
  TraceRec& r = ws.trace[i];
  r.depth = s.depth; r.kind = KIND_IDENT; r.start = s.start; r.count = s.count;
  r.o = s.o; r.M = s.M;
  r.s1[0] = s.s1[0]; r.s1[1] = s.s1[1];
  for (int j = 0; j < 4; ++j) r.s2[j] = s.s2[j];
  r.m = r.sigma = r.zmin = r.A = r.B = 0.0;
  r.shift = 0; r.nonempty = 0; r.hist_off = -1;
}

// statistics of the call that finalize() counts; the caller adds them to the
// control block once per wave (one atomic per segment on one address would
// queue up behind each other)
struct FinStat {
  uint64_t mkeys = 0, fkeys = 0;
  uint32_t ident = 0, rmap = 0, count = 0;
};

// acc: the segment's 32-bit digit sums a0..a5 (of x^2), b0, b1 (of x), then min, max
__device__ void finalize(Ws& ws, Seg& s, int L, const uint64_t (&acc)[10], FinStat& fs) {
  const uint64_t cnt = s.count;
  const uint64_t o = acc[8];
  const uint64_t M = acc[9];
  s.o = o;
  s.M = M;
  if (s.flags & F_FUSED) fs.fkeys += cnt;
  else fs.mkeys += cnt;   // (keys the moments pass read)

  // raw sums: S1' = b0 + b1*2^32 ; S2' = a0 + a1*2^32 + a2*2^33 + a3*2^65 + a4*2^64 + a5*2^96
  W8 s1r = w8_zero();
  w8_add64_at(s1r, acc[6], 0);
  w8_add64_at(s1r, acc[7], 1);
  W8 s2r = w8_zero();
  w8_add64_at(s2r, acc[0], 0);
  w8_add64_at(s2r, acc[1], 1);
  w8_add64_at(s2r, acc[2] << 1, 1);          // a2 < 2^64 / 2 (sum of 32-bit digits over < 2^31 keys)
  w8_add64_at(s2r, acc[3] << 1, 2);
  w8_add64_at(s2r, acc[4], 2);
  w8_add64_at(s2r, acc[5], 3);
  // rebase to the minimum: S1 = S1' - c*o ; S2 = S2' + c*o^2 - 2*o*S1'
  const W8 wc = w8_from64(cnt), wo = w8_from64(o);
  const W8 co = w8_mul(wc, wo);
  const W8 s1 = w8_sub(s1r, co);
  const W8 co2 = w8_mul(co, wo);
  W8 two_o_s1 = w8_mul(w8_from64(o), s1r);
  two_o_s1 = w8_add(two_o_s1, two_o_s1);
  const W8 s2 = w8_sub(w8_add(s2r, co2), two_o_s1);
  s.s1[0] = ((uint64_t)s1.d[1] << 32) | s1.d[0];
  s.s1[1] = ((uint64_t)s1.d[3] << 32) | s1.d[2];
  for (int j = 0; j < 4; ++j) s.s2[j] = ((uint64_t)s2.d[2 * j + 1] << 32) | s2.d[2 * j];

  if (o == M) {  // all keys identical: solved, input order kept
    s.kind = KIND_IDENT;
    ++fs.ident;
    trace_ident(ws, s);
    if (L & 1) {  // keys sit in the alternate buffer: copy them home, in parallel pieces
      for (uint64_t a = 0; a < s.count; a += (uint64_t)kCopyChunk)
        if (!push_leaf(ws, L & 1, s.start + a, (uint32_t)min((uint64_t)kCopyChunk, s.count - a),
                       LF_COPY, 1u))
          break;
    }
    return;
  }

  const int k = ws.p.k;
  if (ws.p.count_range > 0 && M - o < (uint64_t)ws.p.count_range) {
    // a small key range (the counting-sort heuristic of Section III): one
    // stable counting pass on x - o finishes the subproblem (count_range <= k,
    // so every value has a cluster of its own)
    s.m = s.sigma = s.zmin = s.A = s.B = 0.0;
    s.shift = 0;
    s.kind = KIND_COUNT;
    ++fs.count;
    return;
  }
  bool rmap = (s.flags & F_RMAP) != 0;
  double m = 0, sigma = 0, zmin = 0, A = 0, B = 0;
  if (!rmap) {
    // D = c*S2 - S1^2 (c^2 times the population variance about the exact mean)
    const W8 D = w8_sub(w8_mul(wc, s2), w8_mul(s1, s1));
    const double nn = (double)cnt;
    const double a = w8_to_double(s1);
    const double mu = a / nn;
    m = (s.flags & F_ROOT) ? mu : s.e - __ull2double_rn(o - s.o_parent);
    const double Dd = w8_to_double(D);
    double v1 = Dd / nn;
    v1 = v1 / nn;
    const double dm = mu - m;
    const double dm2 = dm * dm;
    const double var = v1 + dm2;
    sigma = sqrt(var);
    zmin = fabs((0.0 - m) / sigma);
    const double scale = (double)k / 4.0;
    A = scale / sigma;
    B = zmin * scale;
    const bool ok = (var > 0.0) && isfinite(var) && isfinite(m) && isfinite(A) && isfinite(B);
    if (!ok) rmap = true;
  }
  s.m = m; s.sigma = sigma; s.zmin = zmin; s.A = A; s.B = B;
  if (rmap) {
    const uint64_t R = M - o;
    const int bl = 64 - __clzll((long long)R);
    s.shift = bl > ws.p.lb ? bl - ws.p.lb : 0;
    s.kind = KIND_RMAP;
    s.flags |= F_RMAP;
    ++fs.rmap;
  } else {
    s.shift = 0;
    s.kind = KIND_ZMAP;
  }
}

// ---------------------------------------------------------------------------
// moments: exact digit sums per chunk -> segment accumulators; the last chunk
// of a segment runs finalize
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_moments(Ws ws, int L) {
  Ctl* c = ws.ctl;
  const int S = L & 1, N = S ^ 1;
  if (call_failed(c)) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    // the segment lists of level L + 1 start empty
    c->nseg[N] = 0; c->nwork[N] = 0; c->nstatus[N] = 0; c->ntile[N] = 0;
    // and so do this level's leaf lists (level 0's may already hold the
    // set-up's jobs).  They are emptied here rather than a level earlier, so
    // that the local sorts of level L - 2, which read this slot's lists, may
    // still be running beside level L - 1.
    if (L >= 1) {
      c->nleaf[S] = 0; c->nleafw[S] = 0; c->nleafm[S] = 0; c->nleafx[S] = 0; c->nhard[S] = 0;
    }
  }
  const uint32_t nw = min(c->nwork[S], ws.work_cap);
  const uint64_t* __restrict__ x = ws.keys[S];
  const uint64_t ch = (uint64_t)ws.p.chunk;
  __shared__ uint64_t red[kWaves][10];

  for (uint32_t w = blockIdx.x; w < nw; w += gridDim.x) {
    const uint64_t item = ws.work[S][w];
    const uint32_t si = (uint32_t)(item >> 32), ci = (uint32_t)item;
    Seg& sg = ws.segs[S][si];
    if (sg.flags & F_FUSED) continue;   // its parent's scatter took its statistics
    const uint64_t beg = sg.start + (uint64_t)ci * ch;
    const uint64_t end = min(beg + ch, sg.start + sg.count);
    uint64_t a0 = 0, a1 = 0, a2 = 0, a3 = 0, a4 = 0, a5 = 0, b0 = 0, b1 = 0;
    uint64_t mn = ~0ull, mx = 0;
    for_each_key<4>(x, beg, end, [&](uint64_t, uint64_t v) {
      const uint32_t xl = (uint32_t)v, xh = (uint32_t)(v >> 32);
      const uint64_t ll = (uint64_t)xl * xl, lh = (uint64_t)xl * xh, hh = (uint64_t)xh * xh;
      a0 += (uint32_t)ll; a1 += ll >> 32;
      a2 += (uint32_t)lh; a3 += lh >> 32;
      a4 += (uint32_t)hh; a5 += hh >> 32;
      b0 += xl; b1 += xh;
      mn = v < mn ? v : mn;
      mx = v > mx ? v : mx;
    });
    uint64_t vals[10] = {a0, a1, a2, a3, a4, a5, b0, b1, mn, mx};
    (void)sg;
    wave_reduce_moments(vals);
    if (lane() == 0)
      for (int j = 0; j < 10; ++j) red[wave()][j] = vals[j];
    __syncthreads();
    if (threadIdx.x < 10) {  // this chunk's partial moments, reduced later per segment
      const int j = threadIdx.x;
      uint64_t v = red[0][j];
      for (int wv = 1; wv < kWaves; ++wv) {
        const uint64_t q = red[wv][j];
        v = j < 8 ? v + q : (j == 8 ? (q < v ? q : v) : (q > v ? q : v));
      }
      ws.part[(uint64_t)w * 10 + j] = v;
    }
    __syncthreads();
  }
}

// finalize: one workgroup per segment sums the partial moments of its chunks
// (exact, order-free integer sums), then one thread derives the statistics
constexpr int kFinThreads = kBlock;  // workgroup of the finalize kernel
constexpr uint32_t kFinBig = 256;   // segments with more chunks are summed by a whole workgroup
constexpr uint32_t kFinLane = 4;    // segments with at most this many chunks: one lane each

// sums of partials [q0, q1) with stride `step`, two chunks in flight per lane
__device__ __forceinline__ void sum_partials(const uint64_t* part, uint32_t q0, uint32_t q1,
                                             uint32_t step, uint64_t (&v)[10]) {
  uint32_t q = q0;
  for (; q + step < q1; q += 2 * step) {
    uint64_t t[2][10];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int j = 0; j < 10; ++j) t[u][j] = part[(uint64_t)(q + u * step) * 10 + j];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] += t[u][j];
      v[8] = t[u][8] < v[8] ? t[u][8] : v[8];
      v[9] = t[u][9] > v[9] ? t[u][9] : v[9];
    }
  }
  for (; q < q1; q += step) {
    const uint64_t* pr = part + (uint64_t)q * 10;
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] += pr[j];
    v[8] = pr[8] < v[8] ? pr[8] : v[8];
    v[9] = pr[9] > v[9] ? pr[9] : v[9];
  }
}


__global__ void __launch_bounds__(kFinThreads) k_finalize(Ws ws, int L) {
  Ctl* c = ws.ctl;
  if (call_failed(c)) return;
  const int S = L & 1;
  const uint32_t ns = min(c->nseg[S], ws.seg_cap);
  constexpr int NWV = kFinThreads / kWave;
  __shared__ uint64_t red[NWV][10];
  const uint32_t ln = lane(), wv = wave();
  FinStat fs;
  // segments of many chunks: a whole workgroup each
  for (uint32_t i = blockIdx.x; i < ns; i += gridDim.x) {
    Seg& sg = ws.segs[S][i];
    if (sg.nchunks < kFinBig || (sg.flags & F_FUSED)) continue;
    uint64_t v[10] = {0, 0, 0, 0, 0, 0, 0, 0, ~0ull, 0};
    sum_partials(ws.part + (uint64_t)sg.first_work * 10, threadIdx.x, sg.nchunks, kFinThreads, v);
    wave_reduce_moments(v);
    if (ln == 0)
      for (int j = 0; j < 10; ++j) red[wv][j] = v[j];
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int q = 1; q < NWV; ++q) {
        for (int j = 0; j < 8; ++j) v[j] += red[q][j];
        v[8] = red[q][8] < v[8] ? red[q][8] : v[8];
        v[9] = red[q][9] > v[9] ? red[q][9] : v[9];
      }
      finalize(ws, sg, L, v, fs);
    }
    __syncthreads();
  }
  // middle sizes: one wave each, whose lanes sum the chunk partials and
  // whose lane 0 computes the statistics (waves of a workgroup work on
  // different segments)
  const uint32_t nwv = gridDim.x * NWV;
  for (uint32_t i = blockIdx.x * NWV + wv; i < ns; i += nwv) {
    Seg& sg = ws.segs[S][i];
    if ((sg.flags & F_FUSED) || sg.nchunks >= kFinBig || sg.nchunks <= kFinLane) continue;
    uint64_t v[10] = {0, 0, 0, 0, 0, 0, 0, 0, ~0ull, 0};
    sum_partials(ws.part + (uint64_t)sg.first_work * 10, ln, sg.nchunks, kWave, v);
    wave_reduce_moments(v);
    if (ln == 0) finalize(ws, sg, L, v, fs);
  }
  // the many small segments of the deeper levels: one lane each, which sums
  // its few partials itself (the statistics are serial work of one lane in
  // any case, so 64 of them run side by side); so do the segments whose
  // statistics their parent's scatter accumulated
  const uint32_t nln = nwv * kWave;
  for (uint32_t i = (blockIdx.x * NWV + wv) * kWave + ln; i < ns; i += nln) {
    Seg& sg = ws.segs[S][i];
    const bool fused = (sg.flags & F_FUSED) != 0;
    if (!fused && sg.nchunks > kFinLane) continue;
    uint64_t v[10] = {0, 0, 0, 0, 0, 0, 0, 0, ~0ull, 0};
    if (fused) {
#pragma unroll
      for (int j = 0; j < 10; ++j) v[j] = ws.facc[(uint64_t)i * 10 + j];
    } else {
      sum_partials(ws.part + (uint64_t)sg.first_work * 10, 0u, sg.nchunks, 1u, v);
    }
    finalize(ws, sg, L, v, fs);
  }
  // statistics of the wave's segments
  uint64_t mk = fs.mkeys, fk = fs.fkeys;
  uint32_t id = fs.ident, rm = fs.rmap, ct = fs.count;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    mk += __shfl_xor(mk, d);
    fk += __shfl_xor(fk, d);
    id += __shfl_xor(id, d);
    rm += __shfl_xor(rm, d);
    ct += __shfl_xor(ct, d);
  }
  if (ln == 0) {
    if (mk) atomicAdd((unsigned long long*)&c->lvl_mkeys[L], (unsigned long long)mk);
    if (fk) atomicAdd((unsigned long long*)&c->lvl_fkeys[L], (unsigned long long)fk);
    if (id) atomicAdd(&c->n_ident, id);
    if (ct) atomicAdd(&c->n_count, ct);
    if (rm) atomicAdd(&c->n_rmap, rm);
  }
}

// ---------------------------------------------------------------------------
// hist: per-chunk LDS histogram, the scan over the chunks of a segment
// (reduce, then scan: the last arrivals do it), and the exclusive scan +
// classification of the segment's clusters
// ---------------------------------------------------------------------------
template <int KMAX>
struct alignas(16) HistSmem {   // t0, t1 double as KMAX 64-bit words (learned thresholds)
  uint32_t h[KMAX];       // histogram, later totals (8192-key tiles: 16-bit counts of
                          // tiles 0 and 1 of the work item until the totals are formed)
  uint32_t hq[KMAX <= 1024 ? KMAX : 1];   // 16-bit counts of tiles 2 and 3
  uint32_t hq2[KMAX <= 1024 ? 2 : 1][KMAX <= 1024 ? KMAX : 1];  // tiles 4, 5 and 6, 7
  uint32_t bst[KMAX];     // exclusive starts
  uint32_t t0[KMAX];      // scratch arrays for classification
  uint32_t t1[KMAX];
  uint32_t t2[KMAX];
  uint32_t sh[kWaves + 2];
  uint32_t shm[5][kWaves];  // wave totals of the multi-array scans
  uint32_t w;
  uint32_t last;          // this workgroup arrived last at a scan unit / segment
  uint32_t base_seg, base_work, base_status, base_leaf, base_tile, base_mid, base_wide;
  // statistics of this workgroup's segments, added to the control block at
  // the end of the kernel
  unsigned long long st_keys;
  uint32_t st_segs, st_groups;
};

// Which leaf groups of a distributed segment may span 2^51 keys or more, in
// whole clusters: a group of clusters b0..b1 counts b1 - b0 + 1 clusters,
// plus x0 more if it holds the clipped first cluster and x1 if it holds the
// clipped last one (those reach the segment's extremes), and is wide when the
// count reaches nwide.  Computed once per segment from the map: an interior
// cluster spans 1/A keys (z-map), 2^shift (range map), 1 (counting pass).
// Only routes groups between local sorts; rounding here changes no result.
struct WideRule {
  uint32_t nwide, x0, x1;
};
__device__ WideRule wide_rule(const Seg& s, int k) {
  WideRule w{0xFFFFFFFFu, 0u, 0u};
  const double full = __ull2double_rn(s.M - s.o);
  if (!(full >= 0x1p51) || s.kind == KIND_COUNT) return w;
  auto clusters = [](double x) {   // a width in whole clusters, clamped
    return !(x < 0x1p31) ? 0x80000000u : (x > 0.0 ? (uint32_t)x : 0u);
  };
  if (s.kind == KIND_RMAP) {
    w.nwide = s.shift >= 51 ? 1u : (1u << min(51 - s.shift, 31));
  } else if (s.kind == KIND_ZMAP && s.A > 0.0) {
    w.nwide = max(clusters(0x1p51 * s.A), 1u);
    w.x0 = clusters((s.m + (1.0 - s.B) / s.A) * s.A);
    w.x1 = clusters((full - (s.m + ((double)(k - 1) - s.B) / s.A)) * s.A);
  } else {
    w.nwide = 1u;   // a learned map: any group of such a segment may be wide
  }
  return w;
}

// the cluster holding position p of a distributed segment: the last one
// starting at or before p (a non-empty one when p < the segment's count)
template <int KMAX>
__device__ __forceinline__ int cluster_at(const HistSmem<KMAX>& sm, int k, uint32_t p) {
  int lo = 0, hi = k - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (sm.bst[mid] <= p) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <int KMAX, bool FUSE>
__device__ void classify(Ws& ws, HistSmem<KMAX>& sm, Seg& sg, uint32_t si, int L) {
  Ctl* c = ws.ctl;
  const int k = ws.p.k;
  const uint32_t cutoff = (uint32_t)ws.p.cutoff;
  const uint32_t ch = (uint32_t)ws.p.chunk;   // (n + ch - 1 < 2^32: 32-bit divisions)
  const int S = L & 1, N = S ^ 1;
  const int t = threadIdx.x;
  // the parent's fields in registers: stores to the children's records and
  // the leaf lists would otherwise make the compiler load them again
  const uint64_t sg_start = sg.start, sg_count = sg.count, sg_o = sg.o;
  const double sg_m = sg.m, sg_sigma = sg.sigma, sg_zmin = sg.zmin;
  const int32_t sg_kind = sg.kind;
  // a counting pass: every cluster holds one key value and is final
  const bool counted = sg_kind == KIND_COUNT;

  // exclusive cluster starts, and per child: index, chunk offset, scan row
  // offset, tile offset -- five scans in one pass
  for (int b = t; b < k; b += kBlock) {
    const uint32_t n = sm.h[b];
    const bool child = !counted && n > cutoff;
    const uint32_t nch = child ? (n + ch - 1) / ch : 0u;
    sm.bst[b] = n;
    sm.t0[b] = child ? 1u : 0u;
    sm.t1[b] = nch;
    sm.t2[b] = status_rows(nch);
    if constexpr (KMAX <= 1024) sm.hq[b] = child ? (n + 8191u) >> 13 : 0u;  // 8192-key tiles
  }
  __syncthreads();
  const uint32_t nsub = tiles_per_item(ws);
  uint32_t nchild, nwork, nstat, ntiles = 0;
  if constexpr (KMAX <= 1024) {
    uint32_t* const arr[5] = {sm.bst, sm.t0, sm.t1, sm.t2, sm.hq};
    uint32_t tot[5];
    block_scan_multi<5>(arr, k, sm.shm, tot);
    nchild = tot[1], nwork = tot[2], nstat = tot[3];
    if (nsub > 1) ntiles = tot[4];
  } else {
    uint32_t* const arr[4] = {sm.bst, sm.t0, sm.t1, sm.t2};
    uint32_t tot[4];
    block_scan_multi<4>(arr, k, sm.shm, tot);
    nchild = tot[1], nwork = tot[2], nstat = tot[3];
  }
  uint32_t* gb = ws.bstart + (uint64_t)si * (uint64_t)k;
  for (int b = t; b < k; b += kBlock) gb[b] = sm.bst[b];
  // fused statistics: the children of a z-score or range-map segment
  const bool fuse_children = FUSE && sg_kind != KIND_LMAP;
  // the four list allocations in one atomic instruction (four lanes): the
  // counters are shared by every workgroup of the level, so each round trip
  // is a long one
  if (t < 4) {
    uint32_t* ctr = t == 0 ? &c->nseg[N] : (t == 1 ? &c->nwork[N] : (t == 2 ? &c->nstatus[N] : &c->ntile[N]));
    const uint32_t v = t == 0 ? nchild : (t == 1 ? nwork : (t == 2 ? nstat : ntiles));
    const uint32_t r = v ? atomicAdd(ctr, v) : 0u;
    uint32_t* out = t == 0 ? &sm.base_seg : (t == 1 ? &sm.base_work : (t == 2 ? &sm.base_status : &sm.base_tile));
    *out = r;
  }
  __syncthreads();
  if (t == 0 && nchild) {
    atomicMax(&c->max_level, (uint32_t)(L + 1));
    if (sm.base_seg + nchild > ws.seg_cap) atomicOr(&c->error, ERR_SEGCAP);
    if (sm.base_work + nwork > ws.work_cap) atomicOr(&c->error, ERR_WORKCAP);
    if (sm.base_status + nstat > ws.status_cap) atomicOr(&c->error, ERR_STATUSCAP);
    if (sm.base_tile + ntiles > ws.tile_cap && ntiles) atomicOr(&c->error, ERR_WORKCAP);
  }
  const bool fits = sm.base_seg + nchild <= ws.seg_cap && sm.base_work + nwork <= ws.work_cap &&
                    sm.base_status + nstat <= ws.status_cap &&
                    (ntiles == 0 || sm.base_tile + ntiles <= ws.tile_cap);
  const double scale = (double)k / 4.0;
  const bool parent_r = sg_kind == KIND_RMAP;
  const bool parent_l = sg_kind == KIND_LMAP;  // children take their exact mean
  if (fits) {
    for (int b = t; b < k; b += kBlock) {
      const uint32_t n = sm.h[b];
      if (n <= cutoff || counted) continue;
      const uint32_t idx = sm.base_seg + sm.t0[b];
      Seg& cs = ws.segs[N][idx];
      const bool crm = !(parent_l && ws.lm.sub) &&
                       (parent_r || (L + 1 >= ws.p.max_zlevels) || (uint64_t)n == sg_count);
      cs.start = sg_start + sm.bst[b];
      cs.count = n;
      cs.o_parent = sg_o;
      double e = 0.0;
      if (!crm && !parent_l) {  // estimated mean of cluster b, parent's frame
        double q = ((double)b + 0.5) / scale;
        q = q - sg_zmin;
        q = q * sg_sigma;
        e = q + sg_m;
      }
      cs.e = e;
      cs.depth = L + 1;
      cs.flags = crm ? F_RMAP : (parent_l ? F_ROOT : 0u);
      cs.nchunks = (n + ch - 1) / ch;
      cs.first_work = sm.base_work + sm.t1[b];
      cs.status_base = sm.base_status + sm.t2[b];
      clear_arrivals(ws.arrive[N] + sm.base_status + sm.t2[b], (n + ch - 1) / ch);
      cs.parent = (int32_t)si;
      seg_clear_acc(cs);
      if (fuse_children) seg_fuse_init(ws, cs, idx);
      if (parent_l && ws.lm.sub) {
        // first stage of a two-stage learned map: the child is learned too,
        // with the sub - 1 thresholds after root threshold b
        const uint32_t sub = ws.lm.sub, nt = ws.lm.res->nt, base = (uint32_t)b * sub;
        cs.flags = 0;
        cs.kind = KIND_LMAP;
        cs.M = ~0ull;
        cs.lm_base = base;
        cs.lm_cnt = nt > base ? min(nt - base, sub - 1) : 0u;
        cs.shift = 1;
      }
    }
    // work items of the children, in chunk order; t0 now maps child -> bucket
    if (fuse_children)
      for (int b = t; b < k; b += kBlock)
        ws.child_of[(uint64_t)si * (uint64_t)k + b] =
            (!counted && sm.h[b] > cutoff) ? sm.base_seg + sm.t0[b] : ~0u;
    __syncthreads();
    // child list: position by child index
    for (int b = t; b < k; b += kBlock)
      if (!counted && sm.h[b] > cutoff) sm.t2[sm.t0[b]] = (uint32_t)b;  // t2 reused: child -> bucket
    __syncthreads();
    // work items and (8192-key tiles) scatter tiles, child by child in
    // chunk order: a wave per child, its lanes over the child's entries
    // (cheaper than a search per entry, a chain of dependent LDS reads)
    // (first the children's offsets by child index, in t0 and t1, so that a
    // wave finds a child's ranges with one round of independent LDS reads)
    constexpr int CPT = (KMAX + kBlock - 1) / kBlock;
    uint32_t ow[CPT], ou[CPT];
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
      const uint32_t cc = t + q * kBlock;
      ow[q] = 0;
      ou[q] = 0;
      if (cc < nchild) {
        const uint32_t b = sm.t2[cc];
        ow[q] = sm.t1[b];
        if constexpr (KMAX <= 1024) ou[q] = sm.hq[b];
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
      const uint32_t cc = t + q * kBlock;
      if (cc < nchild) {
        sm.t0[cc] = ow[q];
        sm.t1[cc] = ou[q];
      }
    }
    __syncthreads();
    // a child of at most kBlock entries is written by one thread, a larger
    // one by a wave (a thread per child keeps every store independent)
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
      const uint32_t cc = t + q * kBlock;
      if (cc < nchild) {
        const bool last = cc + 1 == nchild;
        const uint32_t w0 = sm.t0[cc], w1 = last ? nwork : sm.t0[cc + 1];
        const uint32_t u0 = sm.t1[cc], u1 = last ? ntiles : sm.t1[cc + 1];
        if ((w1 - w0) + (u1 - u0) <= (uint32_t)kBlock) {
          const uint64_t segw = (uint64_t)(sm.base_seg + cc) << 32;
          uint64_t* wp = ws.work[N] + sm.base_work + w0;
          for (uint32_t j = 0; j < w1 - w0; ++j) wp[j] = segw | j;
          if (nsub > 1) {
            uint64_t* tp = ws.tiles[N] + sm.base_tile + u0;
            uint32_t ci = 0, sub = 0;
            for (uint32_t j = 0; j < u1 - u0; ++j) {
              tp[j] = segw | (ci << 3) | sub;   // tile_entry of tile j of the child
              if (++sub == nsub) { sub = 0; ++ci; }
            }
          }
        }
      }
    }
    for (uint32_t cc = wave(); cc < nchild; cc += kWaves) {
      const bool last = cc + 1 == nchild;
      const uint32_t w0 = sm.t0[cc], w1 = last ? nwork : sm.t0[cc + 1];
      const uint32_t u0 = sm.t1[cc], u1 = last ? ntiles : sm.t1[cc + 1];
      if ((w1 - w0) + (u1 - u0) <= (uint32_t)kBlock) continue;
      const uint64_t segw = (uint64_t)(sm.base_seg + cc) << 32;
      for (uint32_t j = lane(); j < w1 - w0; j += kWave) ws.work[N][sm.base_work + w0 + j] = segw | j;
      if (nsub > 1)
        for (uint32_t j = lane(); j < u1 - u0; j += kWave)
          ws.tiles[N][sm.base_tile + u0 + j] = tile_entry(sm.base_seg + cc, j, nsub);
    }
  }
  __syncthreads();

  if (counted) {
    // the segment is sorted once this level's scatter has run; from the
    // alternate buffer it is copied home in pieces
    if (N == 1)
      for (uint64_t a = (uint64_t)t * kCopyChunk; a < sg_count; a += (uint64_t)kBlock * kCopyChunk)
        if (!push_leaf(ws, S, sg_start + a, (uint32_t)min((uint64_t)kCopyChunk, sg_count - a),
                       LF_COPY, 1u))
          break;
    __syncthreads();
  } else {
    // leaf groups: consecutive leaf clusters of one run (no child cluster in
    // between) whose starts fall in one window [w*kWindow, (w+1)*kWindow) form
    // one group of < 2*kWindow keys; a leaf larger than kWindow is a group of
    // its own.  Clusters are ordered (max of one < min of the next), so sorting
    // a group as a whole equals sorting each cluster.
    int* prev = (int*)sm.t0;
    for (int b = t; b < k; b += kBlock) prev[b] = sm.h[b] ? b : -1;
    __syncthreads();
    block_excl_max_lds(prev, k, (int*)sm.sh);
    for (int b = t; b < k; b += kBlock) {
      const uint32_t n = sm.h[b];
      uint32_t boundary = 0;
      if (n > cutoff) boundary = 1;
      else if (n > 0) {
        const int pb = prev[b];
        if (pb < 0 || sm.h[pb] > cutoff || sm.h[pb] > (uint32_t)kWindow || n > (uint32_t)kWindow ||
            sm.bst[pb] / (uint32_t)kWindow != sm.bst[b] / (uint32_t)kWindow)
          boundary = 2;
      }
      sm.t1[b] = boundary;
    }
    __syncthreads();
    for (int b = t; b < k; b += kBlock) sm.t2[b] = sm.t1[b] ? 1u : 0u;
    __syncthreads();
    const uint32_t nb = block_scan_lds(sm.t2, k, sm.sh);
    // compacted boundaries in cluster order: start position, top bit = group start
    uint32_t* bpos = sm.t0;
    for (int b = t; b < k; b += kBlock)
      if (sm.t1[b]) bpos[sm.t2[b]] = sm.bst[b] | (sm.t1[b] == 2 ? 0x80000000u : 0u);
    __syncthreads();
    const uint32_t wcap = (uint32_t)wave_job_cap(ws.p.pw);
    // A wave-sized group whose keys may span 2^51 or more goes to the wide
    // list: the fast local sort's words cannot hold such a range next to the
    // position, and the fallback kernel's first loop takes these groups
    // without a failed attempt first (only a segment that wide can have them).
    const WideRule wr = wide_rule(sg, k);
    auto is_wide = [&](uint32_t p0, uint32_t p1) {
      if (wr.nwide == 0xFFFFFFFFu || p1 - p0 > (uint32_t)kWaveCap) return false;
      const int b0 = cluster_at(sm, k, p0), b1 = cluster_at(sm, k, p1 - 1);
      const uint64_t nc = (uint64_t)(b1 - b0 + 1) + (b0 == 0 ? wr.x0 : 0u) +
                          (b1 == k - 1 ? wr.x1 : 0u);
      return nc >= wr.nwide;
    };
    uint32_t my_small = 0, my_mid = 0, my_big = 0, my_wide = 0;
    for (uint32_t i = t; i < nb; i += kBlock) {
      if (!(bpos[i] >> 31)) continue;
      const uint32_t p0 = bpos[i] & 0x7FFFFFFFu;
      const uint32_t p1 = (i + 1 < nb) ? (bpos[i + 1] & 0x7FFFFFFFu) : (uint32_t)sg_count;
      if (is_wide(p0, p1)) ++my_wide;
      else if (p1 - p0 <= wcap) ++my_small;
      else if (p1 - p0 <= (uint32_t)kMidCap) ++my_mid;
      else ++my_big;
    }
    const uint32_t mine[4] = {my_small, my_mid, my_big, my_wide};
    uint32_t offs[4], tots[4];
    block_excl_sums<4>(mine, sm.shm, offs, tots);
    const uint32_t off_small = offs[0], off_mid = offs[1], off_big = offs[2], off_wide = offs[3];
    const uint32_t nsmall = tots[0], nmid = tots[1], nbig = tots[2], nwide = tots[3];
    // the four leaf lists, likewise in one atomic instruction
    if (t < 4) {
      uint32_t* ctr = t == 0 ? &c->nleafw[S]
                    : (t == 1 ? &c->nleafm[S] : (t == 2 ? &c->nleaf[S] : &c->nleafx[S]));
      const uint32_t v = t == 0 ? nsmall : (t == 1 ? nmid : (t == 2 ? nbig : nwide));
      const uint32_t r = v ? atomicAdd(ctr, v) : 0u;
      // (base_status is reused as the big-list base)
      uint32_t* out = t == 0 ? &sm.base_leaf
                    : (t == 1 ? &sm.base_mid : (t == 2 ? &sm.base_status : &sm.base_wide));
      *out = r;
    }
    if (t == 0) sm.st_groups += nsmall + nmid + nbig + nwide;
    __syncthreads();
    const bool fits = sm.base_leaf + nsmall <= ws.leaf_cap && sm.base_mid + nmid <= ws.leaf_cap &&
                      sm.base_status + nbig <= ws.leaf_cap && sm.base_wide + nwide <= ws.leaf_cap;
    if (t == 0 && !fits) atomicOr(&c->error, ERR_LEAFCAP);
    if (fits) {
      uint32_t os = sm.base_leaf + off_small, om = sm.base_mid + off_mid, ob = sm.base_status + off_big;
      uint32_t ox = sm.base_wide + off_wide;
      for (uint32_t i = t; i < nb; i += kBlock) {
        if (!(bpos[i] >> 31)) continue;
        const uint32_t p0 = bpos[i] & 0x7FFFFFFFu;
        const uint32_t p1 = (i + 1 < nb) ? (bpos[i + 1] & 0x7FFFFFFFu) : (uint32_t)sg_count;
        const bool wide = is_wide(p0, p1);
        const bool small = !wide && p1 - p0 <= wcap;
        const bool mid = !wide && !small && p1 - p0 <= (uint32_t)kMidCap;
        Leaf& lf = wide ? ws.leavesx[S][ox++]
                 : (small ? ws.leavesw[S][os++] : (mid ? ws.leavesm[S][om++] : ws.leaves[S][ob++]));
        lf.start = (uint32_t)(sg_start + p0);
        lf.count = p1 - p0;
        lf.flags = 0;
        lf.src = (uint32_t)N;  // written by this level's scatter
      }
    }
    __syncthreads();
  }

  // largest final cluster of the learned map (with two stages, root
  // clusters that are not split again count whole)
  if (parent_l) {
    uint32_t mc = 0;
    for (int b = t; b < k; b += kBlock) {
      const uint32_t n = sm.h[b];
      if (!ws.lm.sub || n <= cutoff) mc = n > mc ? n : mc;
    }
    if (mc) atomicMax((unsigned long long*)&ws.lm.res->maxc, (unsigned long long)mc);
  }

  // statistics and trace
  if (t == 0) {
    sm.st_keys += sg_count;
    sm.st_segs += 1u;
  }
  if (ws.trace) {
    uint32_t ne = 0;
    for (int b = t; b < k; b += kBlock) ne += sm.h[b] ? 1u : 0u;
    uint32_t nonempty;
    block_excl_sum(ne, sm.sh, &nonempty);
    if (t == 0) {
      uint32_t i = atomicAdd(&c->ntrace, 1u);
      uint32_t ho = atomicAdd(&c->ntrace_hist, (uint32_t)k);
      sm.w = (i < ws.trace_cap) ? i : 0xFFFFFFFFu;
      sm.base_leaf = (ho + (uint32_t)k <= ws.trace_hist_cap) ? ho : 0xFFFFFFFFu;
      if (i < ws.trace_cap) {
        TraceRec& r = ws.trace[i];
        r.depth = sg.depth; r.kind = counted ? kTraceCount : sg.kind;
        r.start = sg.start; r.count = sg.count;
        r.o = sg.o; r.M = sg.M;
        r.s1[0] = sg.s1[0]; r.s1[1] = sg.s1[1];
        for (int j = 0; j < 4; ++j) r.s2[j] = sg.s2[j];
        r.m = sg.m; r.sigma = sg.sigma; r.zmin = sg.zmin; r.A = sg.A; r.B = sg.B;
        r.shift = sg.shift; r.nonempty = (int32_t)nonempty;
        r.hist_off = (sm.base_leaf != 0xFFFFFFFFu) ? (int64_t)sm.base_leaf : -1;
      }
    }
    __syncthreads();
    if (sm.base_leaf != 0xFFFFFFFFu)
      for (int b = t; b < k; b += kBlock) ws.trace_hist[sm.base_leaf + b] = sm.h[b];
  }
  __syncthreads();
}

// one key of cluster b at offset `off` in its work item.  With 8192-key
// scatter tiles (nsub > 1) the count goes to the key's tile: two tiles share
// a word, 16 bits each (a tile holds at most 8192 keys, so the halves never
// carry into each other).
template <int KMAX>
__device__ __forceinline__ void hist_add(HistSmem<KMAX>& sm, uint32_t b, uint64_t off,
                                         uint32_t nsub) {
  if (KMAX > 1024 || nsub == 1) {
    atomicAdd(&sm.h[b], 1u);
  } else {
    const uint32_t tile = (uint32_t)(off >> 13), wd = tile >> 1;
    uint32_t* a = wd == 0 ? &sm.h[b] : (wd == 1 ? &sm.hq[b] : &sm.hq2[(wd - 2) & 1][b]);
    atomicAdd(a, (tile & 1u) ? 0x10000u : 1u);
  }
}

// LM: 0 plain; the learned passes (every segment has KIND_LMAP): 1 with
// thresholds, 2 with the MLP evaluated per key; 3 plain, and the children's
// statistics are left to the scatter.  Separate instances, so that the
// per-key MLP (or the fusion) does not raise the register count of the others.
template <int KMAX, int LM>
__global__ void __launch_bounds__(kBlock) k_hist(Ws ws, int L) {
  __shared__ HistSmem<KMAX> sm;
  Ctl* c = ws.ctl;
  if (call_failed(c)) return;
  const int S = L & 1;
  const uint32_t nw = min(c->nwork[S], ws.work_cap);
  const int k = ws.p.k;
  const uint64_t ch = (uint64_t)ws.p.chunk;
  const uint64_t* __restrict__ x = ws.keys[S];
  const int t = threadIdx.x;
  // tiles of the scatter per work item, each with its own starts (8192-key
  // tiles only, at most 8)
  const uint32_t nsub = tiles_per_item(ws);
  if (t == 0) {
    sm.st_keys = 0;
    sm.st_segs = 0;
    sm.st_groups = 0;
  }

  // items by ticket (the last arrivals at a scan unit or segment do more
  // work, so a fixed share per workgroup would be uneven), last item first:
  // the moments pass reads the items in order and the scatter takes them in
  // order, so each starts on keys the pass before it read last, some of which
  // are still in the memory-side cache
  while (true) {
    if (t == 0) sm.w = atomicAdd(&c->tick[L], 1u);
    __syncthreads();
    const uint32_t tk = sm.w;
    __syncthreads();
    if (tk >= nw) break;
    const uint32_t w = nw - 1u - tk;
    const uint64_t item = ws.work[S][w];
    const uint32_t si = (uint32_t)(item >> 32), ci = (uint32_t)item;
    Seg& sg = ws.segs[S][si];
    if (sg.kind == KIND_IDENT) continue;
    const MapP mp = map_of(sg, k);
    const uint64_t beg = sg.start + (uint64_t)ci * ch;
    const uint64_t end = min(beg + ch, sg.start + sg.count);
    for (int b = t; b < k; b += kBlock) {
      sm.h[b] = 0;
      if constexpr (KMAX <= 1024) {
        sm.hq[b] = 0;
        if (nsub > 4) sm.hq2[0][b] = sm.hq2[1][b] = 0;
      }
    }
    __syncthreads();
    if constexpr (LM == 1 || LM == 2) {
      // learned map: cluster = number of the segment's window thresholds
      // <= key (binary search in LDS), or the MLP evaluated per key; the ids
      // go to the scatter pass
      const uint32_t nt = min(sg.lm_cnt, (uint32_t)(k - 1));
      const uint64_t* __restrict__ wthr = ws.lm.thr + sg.lm_base;
      const uint32_t stride = (uint32_t)sg.shift;
      uint64_t* thr = reinterpret_cast<uint64_t*>(sm.t0);  // t0, t1: KMAX words
      if constexpr (LM == 1)
        for (uint32_t q = t; q < nt; q += kBlock) thr[q] = wthr[(uint64_t)q * stride];
      __syncthreads();
      const uint32_t top = top_pow2(nt);
      const uint64_t smin = ws.lm.res->smin, smax = ws.lm.res->smax;
      uint16_t* __restrict__ ids = ws.lm.ids;
      for_each_key<4>(x, beg, end, [&](uint64_t i, uint64_t v) {
        uint32_t b;
        if constexpr (LM == 2) b = mlp_cluster(*ws.lm.par, v, smin, smax, k);
        else b = thr_cluster(thr, nt, top, v);
        hist_add(sm, b, i - beg, nsub);
        ids[i] = (uint16_t)b;
      });
    } else {
      for_each_key<4>(x, beg, end, [&](uint64_t i, uint64_t v) {
        hist_add(sm, bucket_of(v, mp), i - beg, nsub);
      });
    }
    __syncthreads();
    if (KMAX <= 1024 && nsub > 1) {
      // per-tile counts -> the totals, and for every later tile of the item
      // each cluster's count before it (the scatter's start inside the item)
      for (int b = t; b < k; b += kBlock) {
        const uint32_t v0 = sm.h[b], v1 = sm.hq[b];
        const uint32_t v2 = nsub > 4 ? sm.hq2[0][b] : 0u, v3 = nsub > 4 ? sm.hq2[1][b] : 0u;
        const uint32_t cnt[8] = {v0 & 0xFFFFu, v0 >> 16, v1 & 0xFFFFu, v1 >> 16,
                                 v2 & 0xFFFFu, v2 >> 16, v3 & 0xFFFFu, v3 >> 16};
        uint32_t run = cnt[0];
#pragma unroll
        for (uint32_t q = 1; q < 8; ++q) {
          if (q < nsub) {
            const uint64_t p = beg + ((uint64_t)q << 13);
            if (p < end) ws.subpre[(p >> 13) * (uint64_t)k + b] = (uint16_t)run;
            run += cnt[q];
          }
        }
        sm.h[b] = run;
      }
      __syncthreads();
    }
    // Across the chunks of a segment: reduce, then scan -- nothing waits.
    // The chunk's counts go to its row; the last chunk of a scan unit to
    // arrive turns the unit's rows into running sums within the unit and
    // keeps the unit's totals in the unit's row; the last unit of the segment
    // to arrive turns the unit totals into exclusive prefixes and has the
    // segment's totals, which it classifies.  A chunk's exclusive start is
    // then its unit's prefix plus the row before it in its unit.
    const uint32_t nch = sg.nchunks;
    bool seg_done = nch == 1;
    if (nch > 1) {
      const uint32_t tag = level_tag(c->epoch, L);
      const uint32_t u = scan_unit(nch), nun = scan_units(nch);
      const uint32_t un = ci / u, r0 = un * u, r1 = min(r0 + u, nch);
      uint64_t* rows = ws.status + (uint64_t)sg.status_base * (uint64_t)k;
      uint32_t* arr = ws.arrive[S] + sg.status_base;
      for (int b = t; b < k; b += kBlock) row_put(rows + (uint64_t)ci * k + b, tag, sm.h[b]);
      __syncthreads();
      if (t == 0) sm.last = atomicAdd(&arr[un], 1u) == r1 - r0 - 1u ? 1u : 0u;
      __syncthreads();
      if (sm.last) {
        constexpr uint32_t B = 16;  // rows in flight per thread
        for (int b = t; b < k; b += kBlock) {
          uint32_t run = 0;
          for (uint32_t r = r0; r < r1; r += B) {
            uint64_t v[B];
#pragma unroll
            for (uint32_t j = 0; j < B; ++j)
              v[j] = r + j < r1 ? row_peek(rows + (uint64_t)(r + j) * k + b) : 0ull;
#pragma unroll
            for (uint32_t j = 0; j < B; ++j) {
              if (r + j < r1) {
                uint64_t* p = rows + (uint64_t)(r + j) * k + b;
                run += row_value(p, v[j], tag, c);
                row_put(p, tag, run);
              }
            }
          }
          if (nun == 1) sm.h[b] = run;
          else row_put(rows + (uint64_t)(nch + un) * k + b, tag, run);
        }
        if (nun == 1) {
          seg_done = true;
        } else {
          __syncthreads();
          if (t == 0) sm.last = atomicAdd(&arr[nun], 1u) == nun - 1u ? 1u : 0u;
          __syncthreads();
          if (sm.last) {
            for (int b = t; b < k; b += kBlock) {
              uint32_t run = 0;
              for (uint32_t q = 0; q < nun; q += B) {
                uint64_t v[B];
#pragma unroll
                for (uint32_t j = 0; j < B; ++j)
                  v[j] = q + j < nun ? row_peek(rows + (uint64_t)(nch + q + j) * k + b) : 0ull;
#pragma unroll
                for (uint32_t j = 0; j < B; ++j) {
                  if (q + j < nun) {
                    uint64_t* p = rows + (uint64_t)(nch + q + j) * k + b;
                    const uint32_t x = row_value(p, v[j], tag, c);
                    row_put(p, tag, run);
                    run += x;
                  }
                }
              }
              sm.h[b] = run;  // totals of the segment
            }
            seg_done = true;
          }
        }
      }
    }
    __syncthreads();
    if (seg_done) classify<KMAX, LM == 3>(ws, sm, sg, si, L);
    __syncthreads();
  }
  if (t == 0) {
    if (sm.st_keys) atomicAdd((unsigned long long*)&c->lvl_keys[L], sm.st_keys);
    if (sm.st_segs) atomicAdd(&c->lvl_segs[L], sm.st_segs);
    if (sm.st_groups) atomicAdd(&c->n_leafgroups, sm.st_groups);
    // the host paces the levels by the next level's segment count and
    // whether this level has leaf jobs: the last workgroup to finish stores
    // both straight into the host's pinned memory.  (Every list allocation of
    // a workgroup returned before its barrier, so the counts read after this
    // atomic are final.)
    if (ws.h_pace && atomicAdd(&c->hdone[L], 1u) == gridDim.x - 1u) {
      const int S = L & 1;
      const uint32_t ns = __hip_atomic_load(&c->nseg[S ^ 1], __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
      const uint32_t nl = __hip_atomic_load(&c->nleaf[S], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) |
                          __hip_atomic_load(&c->nleafw[S], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) |
                          __hip_atomic_load(&c->nleafm[S], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) |
                          __hip_atomic_load(&c->nleafx[S], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const bool failed = call_failed(c);
      __hip_atomic_store(&ws.h_pace[L + 1], pace_word(ws.pace_token, failed ? 0u : ns, nl != 0),
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
}

// ---------------------------------------------------------------------------
// scatter: stable, key + payload, through an LDS-staged tile
// ---------------------------------------------------------------------------

// Fused statistics of the children (Section III: the statistics of a
// subproblem, the sums of Algorithm 1's mean and variance loops): once a
// window of the tile is staged in cluster order, each cluster's keys in it
// are summed like the moments pass sums a chunk (32-bit digit sums of x and
// x^2, min, max) and added to its child's accumulators with device atomics
// -- exact integer sums, so the order of the additions is free.  tpc threads
// share a cluster (as many as the workgroup has per cluster, a power of two),
// so a tile dominated by one cluster serialises on that cluster's threads;
// cst holds each cluster's start in the tile (tn: the tile's key count),
// stage the window [p0, p0 + pn) of the tile.
template <int KMAX, int SB>
__device__ __forceinline__ void fused_stats(const Ws& ws, const uint32_t* cof,
                                            const uint16_t* cst, const uint64_t* stage, int k,
                                            uint32_t tn, uint32_t p0, uint32_t pn, int t) {
  uint32_t tpc = 1;
  while (tpc * 2u * (uint32_t)k <= (uint32_t)SB) tpc <<= 1;
  const uint32_t sub = (uint32_t)t % tpc, per = (uint32_t)SB / tpc;
  for (uint32_t bb = 0; bb < (uint32_t)k; bb += per) {   // (the same trip count in every lane)
    const uint32_t b = bb + (uint32_t)t / tpc;
    uint64_t v[10] = {0, 0, 0, 0, 0, 0, 0, 0, ~0ull, 0};
    uint32_t cid = ~0u, r0 = 0, r1 = 0;
    if (b < (uint32_t)k) {
      cid = cof[b];
      const uint32_t s0 = cst[b], s1 = b + 1 < (uint32_t)k ? cst[b + 1] : tn;
      r0 = max(s0, p0);
      r1 = min(s1, p0 + pn);
      if (cid != ~0u)
        for (uint32_t p = r0 + sub; p < r1; p += tpc) {
          const uint64_t x = stage[p - p0];
          const uint32_t xl = (uint32_t)x, xh = (uint32_t)(x >> 32);
          const uint64_t ll = (uint64_t)xl * xl, lh = (uint64_t)xl * xh, hh = (uint64_t)xh * xh;
          v[0] += (uint32_t)ll; v[1] += ll >> 32;
          v[2] += (uint32_t)lh; v[3] += lh >> 32;
          v[4] += (uint32_t)hh; v[5] += hh >> 32;
          v[6] += xl; v[7] += xh;
          v[8] = x < v[8] ? x : v[8];
          v[9] = x > v[9] ? x : v[9];
        }
    }
    for (uint32_t o = 1; o < tpc; o <<= 1) {
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] += __shfl_xor(v[j], (int)o);
      const uint64_t a = __shfl_xor(v[8], (int)o), z = __shfl_xor(v[9], (int)o);
      v[8] = a < v[8] ? a : v[8];
      v[9] = z > v[9] ? z : v[9];
    }
    if (sub == 0 && cid < ws.seg_cap && r1 > r0) {
      uint64_t* f = ws.facc + (uint64_t)cid * 10;
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (v[j]) atomicAdd((unsigned long long*)&f[j], (unsigned long long)v[j]);
      atomicMin((unsigned long long*)&f[8], (unsigned long long)v[8]);
      atomicMax((unsigned long long*)&f[9], (unsigned long long)v[9]);
    }
  }
}
template <int KMAX, int PW, int ROUNDS, int SB>
struct ScatSmem {
  static constexpr int NWV = SB / kWave;           // waves of the workgroup
  static constexpr int T = SB * ROUNDS;            // keys per tile (held in registers)
  static constexpr int kFixed = NWV * KMAX * 2 + KMAX * 8;
  static constexpr int kPerKey = 12 + (PW == 4 ? 4 : 0);
  // keys per staging window: the whole tile if it fits in LDS, else halves
  static constexpr int SW = kFixed + T * kPerKey <= 160 * 1024 ? T : T / 2;
  uint16_t cnt[NWV][KMAX];      // per-wave counts -> per-wave start of the cluster in the tile
  uint32_t tst[KMAX];           // tile exclusive starts -> destination minus tile position
  uint32_t gbase[KMAX];         // running destination of each cluster (n < 2^31)
  uint64_t stage[SW];           // keys in cluster order (then 8-byte payloads)
  uint32_t sdst[SW];            // destination of each staged element (~0u: none)
  uint32_t spay4[PW == 4 ? SW : 1];  // 4-byte payloads, staged with their keys
};

// A tile of T keys is ranked in registers; its keys then leave in cluster
// order through LDS windows of SW keys (the whole tile where it fits), so
// each cluster's run per tile is T / k keys long.
// (a workgroup of 1024 threads is one per CU: its register budget is 128)
// FUSE: the instance that also accumulates the children's statistics (a
// separate instance, so that the plain scatter keeps its registers)
template <int KMAX, int KBITS, int PW, int ROUNDS, int SB, bool FUSE = false>
__global__ void __launch_bounds__(SB, (SB >= 1024 ? 1 : (ROUNDS <= 8 ? 4 : 2))) k_scatter(Ws ws, int L) {
  using P = typename PayT<PW>::T;
  using Sm = ScatSmem<KMAX, PW, ROUNDS, SB>;
  constexpr int NWV = Sm::NWV;
  constexpr int T = Sm::T;
  constexpr int SW = Sm::SW;
  constexpr int NWIN = T / SW;
  static_assert(NWIN * SW == T, "tile must be a whole number of windows");
  static_assert(T <= 8192, "positions are packed in 13 bits");
  static_assert(sizeof(Sm) <= 160 * 1024, "LDS of one workgroup");
  __shared__ Sm sm;
  Ctl* c = ws.ctl;
  if (call_failed(c)) return;
  const int S = L & 1, N = S ^ 1;
  const uint32_t nw = min(c->nwork[S], ws.work_cap);
  const int k = ws.p.k;
  const uint64_t ch = (uint64_t)ws.p.chunk;
  // (no __restrict__ on the inputs: a restrict-qualified read-only pointer
  // lets the compiler re-load a tile's keys from memory in the staging phase
  // instead of keeping them in registers)
  const uint64_t* xin = ws.keys[S];
  uint64_t* __restrict__ xout = ws.keys[N];
  const void* pin = ws.pay[S];
  void* pout = ws.pay[N];
  const int t = threadIdx.x;
  const uint32_t wv = wave(), ln = lane();

  // XCD-aware order: consecutive work items go to workgroups of one XCD
  const uint32_t G = gridDim.x;
  const uint32_t per_xcd = G / 8u;
  const uint32_t g = blockIdx.x;
  const uint32_t slot = (per_xcd * 8u == G) ? ((g % 8u) * per_xcd + g / 8u) : g;

  // With 8192-key tiles every tile of a work item is an item of its own (the
  // histogram pass left each cluster's count before it), so neighbouring
  // workgroups write neighbouring runs of each cluster at the same time;
  // otherwise a workgroup takes a work item's tiles in order.
  // (a level whose segments were made by a pass with other tiles has no
  // tile list: then the work items are taken whole)
  const uint32_t ntl = min(c->ntile[S], ws.tile_cap);
  const uint32_t nsub = ntl > 0 ? tiles_per_item(ws) : 1u;
  const uint64_t span = ch / nsub;
  const uint32_t nwt = nsub > 1 ? ntl : nw;
  const uint32_t ns = min(c->nseg[S], ws.seg_cap);

  for (uint32_t w0 = 0; w0 < nwt; w0 += G) {
    const uint32_t wt = w0 + slot;
    if (wt >= nwt) continue;
    uint32_t si, ci, sub = 0;
    if (nsub > 1) {
      const uint64_t e = ws.tiles[S][wt];
      si = (uint32_t)(e >> 32);
      ci = (uint32_t)e >> 3;
      sub = (uint32_t)e & 7u;
    } else {
      const uint64_t item = ws.work[S][wt];
      si = (uint32_t)(item >> 32);
      ci = (uint32_t)item;
    }
    if (si >= ns) continue;
    const Seg& sg = ws.segs[S][si];
    if (sg.kind == KIND_IDENT) continue;
    const MapP mp = map_of(sg, k);
    const bool lmap = sg.kind == KIND_LMAP;
    const uint64_t cbeg = sg.start + (uint64_t)ci * ch;
    const uint64_t beg = cbeg + (uint64_t)sub * span;
    const uint64_t end = min(beg + span, sg.start + sg.count);
    if (beg >= end) continue;
    const uint32_t* gb = ws.bstart + (uint64_t)si * (uint64_t)k;
    // fused statistics: this segment's classification named each cluster's
    // child (z-score and range-map segments only)
    const uint32_t* cof = (FUSE && !lmap) ? ws.child_of + (uint64_t)si * (uint64_t)k : nullptr;
    // start of each cluster: the segment's exclusive start, the prefix of
    // the chunk's scan unit, the running count within the unit before the
    // chunk, and (8192-key tiles) the count before the tile within the chunk
    const uint32_t nch = sg.nchunks;
    const uint32_t su = nch > 1 ? scan_unit(nch) : 1u;
    const uint64_t* rows = ws.status + (uint64_t)sg.status_base * (uint64_t)k;
    const uint64_t* rp = (ci % su) ? rows + (uint64_t)(ci - 1) * (uint64_t)k : nullptr;
    const uint64_t* up = (ci / su) ? rows + (uint64_t)(nch + ci / su) * (uint64_t)k : nullptr;
    const uint16_t* spp = sub > 0 ? ws.subpre + (beg >> 13) * (uint64_t)k : nullptr;
    // (all four loads are issued before any is used: one memory latency)
    const uint64_t seg0 = sg.start;
    for (int b = t; b < k; b += SB) {
      uint64_t vr = 0, vu = 0;
      uint32_t vs = 0;
      if (rp) vr = rp[b];
      if (up) vu = up[b];
      if (spp) vs = spp[b];
      const uint32_t g = gb[b];
      sm.gbase[b] = (uint32_t)(seg0 + g + (vr & kValMask) + (vu & kValMask) + vs);
    }
    // segment bounds in registers (a reference into global memory would be
    // re-read after every store the compiler cannot prove apart from it)
    const uint64_t seg_start = sg.start;
    const uint64_t seg_end = sg.start + sg.count;
    // Peers (lanes of a wave with the same cluster) by one LDS OR per key
    // into a per-wave mask slot of the cluster, read back and cleared --
    // OR is order-free, so the mask is exact; the slots live in the key
    // stage, unused until staging.  Without room for them: one ballot per
    // cluster-index bit.
    constexpr bool kPeerLds = NWV * KMAX <= SW;
    uint64_t* const peer = reinterpret_cast<uint64_t*>(sm.stage) + (kPeerLds ? wv * KMAX : 0);
    for (uint64_t tb = beg; tb < end; tb += T) {
      const uint32_t tn = (uint32_t)min((uint64_t)T, end - tb);
      // this wave's counters and peer slots (only this wave touches them
      // until the barrier)
      for (int b = ln; b < k; b += kWave) {
        sm.cnt[wv][b] = 0;
        if constexpr (kPeerLds) peer[b] = 0ull;
      }
      uint64_t key[ROUNDS];
      P pay[ROUNDS];
      uint32_t bk[ROUNDS];
#pragma unroll
      for (int r = 0; r < ROUNDS; ++r) {
        const uint32_t i = wv * (kWave * ROUNDS) + r * kWave + ln;
        const bool valid = i < tn;
        key[r] = valid ? xin[tb + i] : 0ull;
        bk[r] = (lmap && valid) ? (uint32_t)ws.lm.ids[tb + i] : 0u;  // learned map: ids of hist
      }
      // rank of each key among the wave's keys of its cluster
#pragma unroll
      for (int r = 0; r < ROUNDS; ++r) {
        const uint32_t i = wv * (kWave * ROUNDS) + r * kWave + ln;
        const bool valid = i < tn;
        const uint32_t b = valid ? (lmap ? bk[r] : bucket_of(key[r], mp)) : 0u;
        uint64_t m;
        if constexpr (kPeerLds) {
          if (valid) atomicOr((unsigned long long*)&peer[b], 1ull << ln);
          __builtin_amdgcn_wave_barrier();
          m = valid ? peer[b] : 0ull;
          __builtin_amdgcn_wave_barrier();
          if (valid) peer[b] = 0ull;
          __builtin_amdgcn_wave_barrier();
        } else {
          m = match_digit<KBITS>(b, __ballot(valid));
        }
        const uint32_t before = below(m);
        uint32_t base = 0;
        if (valid) base = sm.cnt[wv][b];
        if (valid && before == 0) sm.cnt[wv][b] = (uint16_t)(base + (uint32_t)__popcll(m));
        bk[r] = ((base + before) << 12) | b;   // rank within this wave's run (< 2^13), cluster
      }
      // the payloads load while the tile's cluster starts are worked out
      // (not during the ranking, whose registers they would crowd: the
      // empty asm hides the pointer, so the loads cannot be hoisted)
      const void* pin_late = pin;
      asm volatile("" : "+s"(pin_late));
#pragma unroll
      for (int r = 0; r < ROUNDS; ++r) {
        const uint32_t i = wv * (kWave * ROUNDS) + r * kWave + ln;
        pay[r] = i < tn ? pay_load<PW>(pin_late, tb + i) : (P)0;
      }
      __syncthreads();
      // per cluster: exclusive prefix over waves, tile count
      for (int b = t; b < k; b += SB) {
        uint32_t run = 0;
#pragma unroll
        for (int q = 0; q < NWV; ++q) {
          const uint32_t v = sm.cnt[q][b];
          sm.cnt[q][b] = (uint16_t)run;
          run += v;
        }
        sm.tst[b] = run;
      }
      __syncthreads();
      // (the scan's scratch lives in the key stage, which is free until staging)
      block_scan_lds<SB>(sm.tst, k, reinterpret_cast<uint32_t*>(sm.stage));
      // per cluster: start of each wave's run in the tile, destination minus
      // tile position, and the running destination advanced past this tile
      constexpr int KPT = (KMAX + SB - 1) / SB;
      uint32_t st0[KPT], stn[KPT];
#pragma unroll
      for (int j = 0; j < KPT; ++j) {
        const int b = t + j * SB;
        st0[j] = b < k ? sm.tst[b] : 0u;
        stn[j] = b + 1 < k ? sm.tst[b + 1] : tn;
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < KPT; ++j) {
        const int b = t + j * SB;
        if (b < k) {
#pragma unroll
          for (int q = 0; q < NWV; ++q) sm.cnt[q][b] = (uint16_t)(sm.cnt[q][b] + st0[j]);
          const uint32_t gbv = sm.gbase[b];
          sm.tst[b] = gbv - st0[j];
          sm.gbase[b] = gbv + (stn[j] - st0[j]);
        }
      }
      __syncthreads();
      // position of each key in the tile's cluster order
#pragma unroll
      for (int r = 0; r < ROUNDS; ++r) {
        const uint32_t b = bk[r] & 0xFFFu;
        const uint32_t pos = min((uint32_t)sm.cnt[wv][b] + (bk[r] >> 12), (uint32_t)T - 1);
        bk[r] = (pos << 12) | b;
      }
      // window by window: stage the keys with their destinations, write
      // them, then the same for the payloads
      const uint32_t dend = (uint32_t)seg_end;
#pragma unroll 1
      for (int wi = 0; wi < NWIN; ++wi) {
        const uint32_t p0 = (uint32_t)(wi * SW);
        if (p0 >= tn) break;
        const uint32_t pn = min((uint32_t)SW, tn - p0);
        if (wi > 0) __syncthreads();   // the previous window has left the stage
#pragma unroll
        for (int r = 0; r < ROUNDS; ++r) {
          const uint32_t i = wv * (kWave * ROUNDS) + r * kWave + ln;
          const uint32_t q = (bk[r] >> 12) - p0;
          if (i < tn && q < (uint32_t)SW) {
            const uint32_t b = bk[r] & 0xFFFu;
            const uint64_t dst = (uint64_t)(uint32_t)((bk[r] >> 12) + sm.tst[b]);
            sm.stage[q] = key[r];
            if constexpr (PW == 4) sm.spay4[q] = (uint32_t)pay[r];
            // never outside the segment when the counts are right
            const bool ok = dst >= seg_start && dst < seg_end;
            if (!ok) atomicOr(&c->error, ERR_SCATTER);
            sm.sdst[q] = ok ? (uint32_t)dst : ~0u;
          }
        }
        __syncthreads();
        // every destination lies inside the segment (an unset or rejected
        // entry, ~0u, never does), so a write can never leave the array
        for (uint32_t p = t; p < pn; p += SB) {
          const uint32_t d = sm.sdst[p];
          if (d < dend) {
            xout[d] = sm.stage[p];
            if constexpr (PW == 4) reinterpret_cast<uint32_t*>(pout)[d] = sm.spay4[p];
          }
        }
        if constexpr (FUSE)
          if (cof) fused_stats<KMAX, SB>(ws, cof, sm.cnt[0], sm.stage, k, tn, p0, pn, t);
        if constexpr (PW == 8) {   // 8-byte payloads: second round through the key stage
          using P2 = typename PayT<PW>::T;
          P2* spay = reinterpret_cast<P2*>(sm.stage);
          __syncthreads();
#pragma unroll
          for (int r = 0; r < ROUNDS; ++r) {
            const uint32_t i = wv * (kWave * ROUNDS) + r * kWave + ln;
            const uint32_t q = (bk[r] >> 12) - p0;
            if (i < tn && q < (uint32_t)SW) spay[q] = pay[r];
          }
          __syncthreads();
          for (uint32_t p = t; p < pn; p += SB) {
            const uint32_t d = sm.sdst[p];
            if (d < dend) pay_store<PW>(pout, d, spay[p]);
          }
        }
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// local sort of the leaf groups.  A "team" sorts one group: a single wave for
// groups of <= kWaveCap keys (four groups per workgroup at a time), the whole
// workgroup for larger ones (<= kLocalCap).
//
// Main path, when the group's range fits in 51 bits: each key becomes the
// unique word ((x - min) << 12) | position, so any correct sort of the words
// is the stable sort of the keys.  Each thread sorts 16 words in registers
// (bitonic network), then runs of 16 are merged pairwise in LDS (merge path)
// until one run remains; the payload is gathered by position at the end.
// Fallback (wider ranges): stable LSD radix on x - min, 8-bit digits, as many
// passes as the range needs.
// ---------------------------------------------------------------------------
constexpr int kLocPer = 16;  // keys per thread
__device__ __forceinline__ uint32_t lpad(uint32_t i) { return i + (i >> 4); }

__device__ __forceinline__ void cswap(uint64_t& a, uint64_t& b) {
  const bool lt = a < b;
  const uint64_t lo = lt ? a : b, hi = lt ? b : a;
  a = lo;
  b = hi;
}

template <int N>
__device__ __forceinline__ void bitonic_regs(uint64_t (&v)[N]) {
#pragma unroll
  for (int size = 2; size <= N; size <<= 1)
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1)
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const int j = i ^ stride;
        if (j > i) {
          if ((i & size) == 0) cswap(v[i], v[j]);
          else cswap(v[j], v[i]);
        }
      }
}

// barrier of a team of TW waves (TW == 1: LDS traffic of one wave drains in order)
template <int TW>
__device__ __forceinline__ void team_sync() {
  if constexpr (TW == 1) {
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_wave_barrier();
  } else {
    __syncthreads();
  }
}

template <int PW>
struct LocSmem {
  uint64_t k[kLocalCap + kLocalCap / 16];   // packed words (padded) / radix staging
  typename PayT<PW>::T pay[PW ? kLocalCap : 1];
  // radix counters (rows 0 .. kWaves-1) and totals (the other rows); the
  // bucket sort's 16-bit counters span the whole array
  uint32_t cnt[2 * kWaves][256];
  uint64_t rmin[kWaves], rmax[kWaves];
  uint32_t sh[kWaves + 2];
};

// team-wide exclusive sum over a[0, 256)
template <int TW>
__device__ __forceinline__ void team_scan256(uint32_t* a, uint32_t* sh, uint32_t tid) {
  if constexpr (TW == kWaves) {
    block_scan_lds(a, 256, sh);
  } else {
    // one wave: 4 entries per lane
    uint32_t v0 = a[4 * tid], v1 = a[4 * tid + 1], v2 = a[4 * tid + 2], v3 = a[4 * tid + 3];
    const uint32_t s = v0 + v1 + v2 + v3;
    const uint32_t inc = wave_incl_sum(s);
    uint32_t base = inc - s;
    a[4 * tid] = base; base += v0;
    a[4 * tid + 1] = base; base += v1;
    a[4 * tid + 2] = base; base += v2;
    a[4 * tid + 3] = base;
    team_sync<1>();
  }
}

constexpr int kBucketMax = 128;

constexpr int pow2_ceil(int v) { return v <= 1 ? 1 : 2 * pow2_ceil((v + 1) / 2); }

__device__ __forceinline__ uint32_t c16_get(const uint32_t* c, uint32_t b) {
  return (c[b >> 1] >> ((b & 1u) * 16u)) & 0xFFFFu;
}

// Turns the nb 16-bit bucket counters (two per word) into exclusive starts;
// returns false, leaving the counters as they are, if some bucket holds more
// than kBucketMax keys (unless limit is false).  Each thread owns
// ceil(nb / TT) consecutive counters.
template <int TW>
__device__ __forceinline__ bool bucket_starts(uint32_t* cnt, uint32_t nb, uint32_t* sh,
                                              uint32_t tid, bool limit = true) {
  constexpr uint32_t TT = TW * kWave;
  const uint32_t tw = tid / kWave, ln = tid & (kWave - 1);
  const uint32_t per = (nb + TT - 1) / TT;
  const uint32_t b0 = tid * per;
  uint32_t tsum = 0, tmax = 0;
  for (uint32_t j = 0; j < per; ++j) {
    const uint32_t b = b0 + j;
    if (b < nb) {
      const uint32_t v = c16_get(cnt, b);
      tsum += v;
      tmax = v > tmax ? v : tmax;
    }
  }
  uint32_t base;
  uint32_t big = __ballot(limit && tmax > (uint32_t)kBucketMax) != 0ull ? 1u : 0u;
  if constexpr (TW == 1) {
    base = wave_incl_sum(tsum) - tsum;
  } else {
    if (ln == 0) sh[tw] = big;
    team_sync<TW>();
    for (int q = 0; q < TW; ++q) big |= sh[q];
    team_sync<TW>();
    uint32_t total;
    base = block_excl_sum<TW * kWave>(tsum, sh, &total);
  }
  if (big) {
    team_sync<TW>();
    return false;
  }
  if (per >= 2) {
    for (uint32_t j = 0; j < per; j += 2) {
      const uint32_t b = b0 + j;
      if (b < nb) {
        const uint32_t v0 = c16_get(cnt, b), v1 = c16_get(cnt, b + 1);
        cnt[b >> 1] = base | ((base + v0) << 16);
        base += v0 + v1;
      }
    }
  }
  team_sync<TW>();
  if (per < 2) {  // thread tid owns bucket tid; even and odd neighbours share a word
    const uint32_t b = b0;
    const uint32_t mine = (b < nb) ? base : 0u;
    const uint32_t other = __shfl_xor(mine, 1);
    team_sync<TW>();
    if (b < nb && (b & 1u) == 0u) cnt[b >> 1] = mine | (other << 16);
    team_sync<TW>();
  }
  return true;
}

// The fallback sort of a group whose range needs more than 51 bits (bits, of
// smallest key mn), which the packed words (x - min) << 12 | position cannot
// hold: as many buckets as it takes for the offset inside a bucket to fit 52
// bits, words (offset << 12) | position, and each slot's bucket found among
// the bucket ends (the words do not hold it).  The payloads are in pb by
// position already.  The keys are read from src twice (counts, words), both
// before the barrier after which anything is stored, so a group may be
// sorted in place.  Returns false, having stored nothing in dst, if the ncnt
// 16-bit counters cannot hold the buckets or some bucket holds more than
// kBucketMax keys.
template <int PW, int TW>
__device__ bool wide_bucket_sort(uint64_t* kb, const typename PayT<PW>::T* pb, uint32_t* cnt,
                                 uint32_t ncnt, uint32_t* sh, const uint64_t* src, uint64_t* dst,
                                 void* pdst, uint64_t start, uint32_t n, uint32_t tid,
                                 uint64_t mn, int bits) {
  constexpr uint32_t TT = TW * kWave;
  uint32_t nb = 64;
  int d = 6;
  while (nb < n || (bits - d > 52 && nb < ncnt)) {
    nb <<= 1;
    ++d;
  }
  if (bits - d > 52 || nb > ncnt) return false;
  const int shb = bits - d;
  const uint64_t in_bucket = (1ull << shb) - 1ull;
  for (uint32_t i = tid; i < nb / 2; i += TT) cnt[i] = 0;
  team_sync<TW>();
  for (uint32_t i = tid; i < n; i += TT) {
    const uint32_t b = (uint32_t)((src[start + i] - mn) >> shb);
    atomicAdd(&cnt[b >> 1], 1u << ((b & 1u) * 16u));
  }
  team_sync<TW>();
  if (!bucket_starts<TW>(cnt, nb, sh, tid)) return false;
  for (uint32_t i = tid; i < n; i += TT) {
    const uint64_t dlt = src[start + i] - mn;
    const uint32_t b = (uint32_t)(dlt >> shb);
    const uint32_t sft = (b & 1u) * 16u;
    const uint32_t old = atomicAdd(&cnt[b >> 1], 1u << sft);
    const uint32_t pos = min((old >> sft) & 0xFFFFu, n - 1);
    kb[pos] = ((dlt & in_bucket) << 12) | i;
  }
  team_sync<TW>();
  // bucket b now spans [end(b-1), end(b)); slots in order, so the keys and
  // payloads are stored nearly sequentially
  for (uint32_t i = tid; i < n; i += TT) {
    const uint64_t v = kb[i];
    uint32_t lo = 0, hi = nb - 1;
    while (lo < hi) {
      const uint32_t mid = (lo + hi) >> 1;
      if (c16_get(cnt, mid) > i) hi = mid;
      else lo = mid + 1;
    }
    const uint32_t e = c16_get(cnt, lo);
    const uint32_t s0 = lo ? c16_get(cnt, lo - 1) : 0u;
    uint32_t rank = 0;
    for (uint32_t j = s0; j < e; ++j) rank += kb[j] < v ? 1u : 0u;
    const uint32_t p = min(s0 + rank, n - 1);
    dst[start + p] = mn + ((uint64_t)lo << shb) + (v >> 12);
    if constexpr (PW != 0) pay_store<PW>(pdst, start + p, pb[v & 4095u]);
  }
  team_sync<TW>();
  return true;
}


// One wave's sort of a group held in its registers (key i = r * 64 + lane),
// for any key range: as many buckets as the group has keys and as it takes
// for the offset inside a bucket to fit 52 bits (at most ncnt 16-bit
// counters), words (offset << 12) | position placed in bucket order with
// each slot's bucket beside them in bkt, and each slot's key rebuilt from
// its bucket and offset.  Nothing is read from memory but LDS (the payloads
// go to pb by position), so the group may be sorted in place.  Returns
// false, having stored nothing, if the counters cannot hold the buckets or
// some bucket holds more than kBucketMax keys.
template <int PW, int R>
__device__ bool wide_wave_sort(uint64_t* kb, uint16_t* bkt, typename PayT<PW>::T* pb,
                               uint32_t* cnt, uint32_t ncnt, uint64_t* dst, void* pdst,
                               uint64_t start, uint32_t n, uint32_t ln, const uint64_t (&key)[R],
                               const typename PayT<PW>::T (&pay)[R]) {
  uint64_t mn = ~0ull, mx = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (r * kWave + ln < n) {
      mn = key[r] < mn ? key[r] : mn;
      mx = key[r] > mx ? key[r] : mx;
    }
  }
  wave_minmax_u64(mn, mx);
  const uint64_t range = mx - mn;
  const int bits = range ? 64 - __clzll((long long)range) : 0;
  uint32_t nb = 64;
  int d = 6;
  while (nb < n || (bits - d > 52 && nb < ncnt)) {
    nb <<= 1;
    ++d;
  }
  if (bits - d > 52 || nb > ncnt) return false;
  const int shb = bits > d ? bits - d : 0;
  const uint64_t in_bucket = (1ull << shb) - 1ull;
  for (uint32_t i = ln; i < nb / 2; i += kWave) cnt[i] = 0;
  team_sync<1>();
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (r * kWave + ln < n) {
      const uint32_t b = (uint32_t)((key[r] - mn) >> shb);
      atomicAdd(&cnt[b >> 1], 1u << ((b & 1u) * 16u));
    }
  }
  team_sync<1>();
  if (!bucket_starts<1>(cnt, nb, nullptr, ln)) return false;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint32_t i = r * kWave + ln;
    if (i < n) {
      const uint64_t dlt = key[r] - mn;
      const uint32_t b = (uint32_t)(dlt >> shb);
      const uint32_t sft = (b & 1u) * 16u;
      const uint32_t old = atomicAdd(&cnt[b >> 1], 1u << sft);
      const uint32_t pos = min((old >> sft) & 0xFFFFu, n - 1);
      kb[pos] = ((dlt & in_bucket) << 12) | i;
      bkt[pos] = (uint16_t)b;
      if constexpr (PW != 0) pb[i] = pay[r];
    }
  }
  team_sync<1>();
  // bucket b spans [end(b-1), end(b)); slots in order, so the keys and
  // payloads are stored nearly sequentially
  for (uint32_t i = ln; i < n; i += kWave) {
    const uint64_t v = kb[i];
    const uint32_t b = bkt[i];
    const uint32_t e = c16_get(cnt, b);
    const uint32_t s0 = b ? c16_get(cnt, b - 1) : 0u;
    uint32_t rank = 0;
    for (uint32_t j = s0; j < e; ++j) rank += kb[j] < v ? 1u : 0u;
    const uint32_t p = min(s0 + rank, n - 1);
    dst[start + p] = mn + ((uint64_t)b << shb) + (v >> 12);
    if constexpr (PW != 0) pay_store<PW>(pdst, start + p, pb[v & 4095u]);
  }
  team_sync<1>();
  return true;
}

// Sorts keys[start, start+n) of `src` into dst (and the payload alongside).
// TW waves cooperate; tid = thread index inside the team; kb/pb = the team's
// LDS key and payload areas (TW*1024 words + padding), cnt/tot = [TW][256]
// and [256] counters, red = 2*TW words; from cnt on, ncnt 16-bit counters
// for the bucket sort of wide ranges.
template <int PW, int TW>
__device__ void team_sort(uint64_t* kb, typename PayT<PW>::T* pb, uint32_t (*cnt)[256],
                          uint32_t* tot, uint64_t* rmin, uint64_t* rmax, uint32_t* sh,
                          const uint64_t* __restrict__ src, const void* psrc,
                          uint64_t* __restrict__ dst, void* pdst, uint64_t start, uint32_t n,
                          uint32_t tid, uint32_t ncnt) {
  using P = typename PayT<PW>::T;
  constexpr uint32_t TT = TW * kWave;  // team threads
  const uint32_t tw = tid / kWave, ln = tid & (kWave - 1);

  // blocked layout: thread tid holds positions 16*tid .. 16*tid+15
  uint64_t key[kLocPer];
  uint64_t mn = ~0ull, mx = 0;
#pragma unroll
  for (int r = 0; r < kLocPer; ++r) {
    const uint32_t i = tid * kLocPer + r;
    key[r] = i < n ? src[start + i] : 0ull;
    if (i < n) { mn = key[r] < mn ? key[r] : mn; mx = key[r] > mx ? key[r] : mx; }
  }
  if constexpr (PW != 0)
    for (uint32_t i = tid; i < n; i += TT) pb[i] = pay_load<PW>(psrc, start + i);
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    const uint64_t a = __shfl_xor(mn, o), b = __shfl_xor(mx, o);
    mn = a < mn ? a : mn;
    mx = b > mx ? b : mx;
  }
  if constexpr (TW > 1) {
    if (ln == 0) { rmin[tw] = mn; rmax[tw] = mx; }
    team_sync<TW>();
    mn = rmin[0]; mx = rmax[0];
    for (int q = 1; q < TW; ++q) {
      mn = rmin[q] < mn ? rmin[q] : mn;
      mx = rmax[q] > mx ? rmax[q] : mx;
    }
  }
  const uint64_t range = mx - mn;
  const int bits = range ? 64 - __clzll((long long)range) : 0;

  if (bits <= 51) {
#pragma unroll
    for (int r = 0; r < kLocPer; ++r) {
      const uint32_t i = tid * kLocPer + r;
      key[r] = i < n ? (((key[r] - mn) << 12) | i) : ~0ull;
    }
    bitonic_regs<kLocPer>(key);
    uint32_t npad = kLocPer;
    while (npad < n) npad <<= 1;
    const bool active = tid * kLocPer < npad;
    if (active)
#pragma unroll
      for (int r = 0; r < kLocPer; ++r) kb[lpad(tid * kLocPer + r)] = key[r];
    team_sync<TW>();
    for (uint32_t w = kLocPer; w < npad; w <<= 1) {
      if (active) {
        const uint32_t o0 = tid * kLocPer;
        const uint32_t base = o0 & ~(2 * w - 1);
        const uint32_t diag = o0 - base;
        const uint32_t aB = base, bB = base + w;
        int lo = (int)diag - (int)w;
        lo = lo < 0 ? 0 : lo;
        int hi = (int)(diag < w ? diag : w);
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (kb[lpad(aB + mid)] < kb[lpad(bB + diag - 1 - mid)]) lo = mid + 1;
          else hi = mid;
        }
        uint32_t ai = aB + lo, bi = bB + (diag - lo);
        const uint32_t aE = bB, bE = bB + w;
        uint64_t a = ai < aE ? kb[lpad(ai)] : ~0ull;
        uint64_t b = bi < bE ? kb[lpad(bi)] : ~0ull;
#pragma unroll
        for (int r = 0; r < kLocPer; ++r) {
          const bool ta = a < b;
          key[r] = ta ? a : b;
          const uint32_t ni = (ta ? ai : bi) + 1;
          const uint32_t lim = ta ? aE : bE;
          const uint64_t v = ni < lim ? kb[lpad(ni)] : ~0ull;
          ai = ta ? ni : ai;
          bi = ta ? bi : ni;
          a = ta ? v : a;
          b = ta ? b : v;
        }
      }
      team_sync<TW>();
      if (active)
#pragma unroll
        for (int r = 0; r < kLocPer; ++r) kb[lpad(tid * kLocPer + r)] = key[r];
      team_sync<TW>();
    }
    for (uint32_t i = tid; i < n; i += TT) {
      const uint64_t v = kb[lpad(i)];
      dst[start + i] = (v >> 12) + mn;
      if constexpr (PW != 0) pay_store<PW>(pdst, start + i, pb[v & 4095u]);
    }
    team_sync<TW>();
    return;
  }

  // wide range: buckets on the top bits where they take the group, else a
  // stable LSD radix.  Wave-blocked layout: position
  // tw*1024 + r*64 + ln, so ranks follow positions wave by wave, round by round.
  if (wide_bucket_sort<PW, TW>(kb, pb, &cnt[0][0], ncnt, sh, src, dst, pdst, start, n, tid, mn,
                               bits))
    return;
  P pay[kLocPer];
#pragma unroll
  for (int r = 0; r < kLocPer; ++r) {
    const uint32_t i = tw * (kWave * kLocPer) + r * kWave + ln;
    const bool valid = i < n;
    key[r] = valid ? src[start + i] : 0ull;
    pay[r] = valid ? pay_load<PW>(psrc, start + i) : (P)0;
  }
  team_sync<TW>();
  const int passes = (bits + 7) / 8;
  for (int ps = 0; ps < passes; ++ps) {
    const int sh8 = ps * 8;
    for (int b = ln; b < 256; b += kWave) cnt[tw][b] = 0;
    team_sync<TW>();
    uint32_t dg[kLocPer], rk[kLocPer];
#pragma unroll
    for (int r = 0; r < kLocPer; ++r) {
      const uint32_t i = tw * (kWave * kLocPer) + r * kWave + ln;
      const bool valid = i < n;
      const uint32_t d = valid ? (uint32_t)(((key[r] - mn) >> sh8) & 255u) : 0u;
      const uint64_t act = __ballot(valid);
      const uint64_t m = match_digit<8>(d, act);
      const uint32_t before = below(m);
      uint32_t base = 0;
      if (valid) base = cnt[tw][d];
      if (valid && before == 0) cnt[tw][d] = base + (uint32_t)__popcll(m);
      dg[r] = d;
      rk[r] = base + before;
    }
    team_sync<TW>();
    for (uint32_t b = tid; b < 256; b += TT) {
      uint32_t run = 0;
#pragma unroll
      for (int q = 0; q < TW; ++q) {
        const uint32_t v = cnt[q][b];
        cnt[q][b] = run;
        run += v;
      }
      tot[b] = run;
    }
    team_sync<TW>();
    team_scan256<TW>(tot, sh, tid);
#pragma unroll
    for (int r = 0; r < kLocPer; ++r) {
      const uint32_t i = tw * (kWave * kLocPer) + r * kWave + ln;
      if (i < n) {
        const uint32_t pos = min(tot[dg[r]] + cnt[tw][dg[r]] + rk[r], TT * kLocPer - 1);
        kb[pos] = key[r];
        if constexpr (PW != 0) pb[pos] = pay[r];
      }
    }
    team_sync<TW>();
#pragma unroll
    for (int r = 0; r < kLocPer; ++r) {
      const uint32_t i = tw * (kWave * kLocPer) + r * kWave + ln;
      if (i < n) {
        key[r] = kb[i];
        if constexpr (PW != 0) pay[r] = pb[i];
      }
    }
    team_sync<TW>();
  }
#pragma unroll
  for (int r = 0; r < kLocPer; ++r) {
    const uint32_t i = tw * (kWave * kLocPer) + r * kWave + ln;
    if (i < n) {
      dst[start + i] = key[r];
      if constexpr (PW != 0) pay_store<PW>(pdst, start + i, pay[r]);
    }
  }
  team_sync<TW>();
}


// ---------------------------------------------------------------------------
// fast local sort: one counting pass on the top bits of x - min (about one
// bucket per key), then each key's place inside its bucket from the number
// of smaller words there.  Works on
// the unique words ((x - min) << 12) | position, so the result is the stable
// sort.  Returns false, before writing anything, if the group's range needs
// more than 51 bits or some bucket holds more than kBucketMax keys; such
// groups go to the fallback kernel (whose bucket sort takes the wide ones).
// ---------------------------------------------------------------------------
template <int PW>
struct FastSmem {
  // block jobs use all of it; wave jobs a quarter each
  static constexpr int KW = kBlockCap > kWaves * wave_job_cap(PW) ? kBlockCap : kWaves * wave_job_cap(PW);
  static constexpr int CW = kBlockCap / 2 > kWaves * pow2_ceil(wave_job_cap(PW)) / 2
                                ? kBlockCap / 2 : kWaves * pow2_ceil(wave_job_cap(PW)) / 2;
  uint64_t k[KW];                               // words in bucket order
  typename PayT<PW>::T pay[PW ? KW : 1];        // payload by input position
  uint32_t cnt[CW];                             // 16-bit bucket counters, two per word
  uint64_t rmin[kWaves], rmax[kWaves];
  uint32_t sh[kWaves + 2];
};

// a team's group into registers: key i = r * TT + tid of the group
template <int PW, int TT, int R>
__device__ __forceinline__ void group_load(const uint64_t* __restrict__ src, const void* psrc,
                                           uint64_t start, uint32_t n, uint32_t tid,
                                           uint64_t (&key)[R], typename PayT<PW>::T (&pay)[R]) {
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint32_t i = r * TT + tid;
    const bool valid = i < n;
    key[r] = valid ? src[start + i] : 0ull;
    pay[r] = (PW != 0 && valid) ? pay_load<PW>(psrc, start + i) : (typename PayT<PW>::T)0;
  }
}

// Sorts a group held in registers (see group_load); returns false when the
// bucket pass cannot take it (range above 51 bits, or a bucket above
// kBucketMax keys) -- the group is then left to the fallback sort.
template <int PW, int TW, int R>
__device__ bool fast_sort_regs(uint64_t* kb, typename PayT<PW>::T* pb, uint32_t* cnt,
                               uint64_t* rmin, uint64_t* rmax, uint32_t* sh,
                               const uint64_t* __restrict__ src, const void* psrc,
                               uint64_t* __restrict__ dst, void* pdst, uint64_t start, uint32_t n,
                               uint32_t tid, const uint64_t (&key)[R],
                               const typename PayT<PW>::T (&pay)[R]) {
  constexpr uint32_t TT = TW * kWave;  // n <= TT * R
  const uint32_t tw = tid / kWave, ln = tid & (kWave - 1);
  uint64_t mn = ~0ull, mx = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint32_t i = r * TT + tid;
    if (i < n) {
      mn = key[r] < mn ? key[r] : mn;
      mx = key[r] > mx ? key[r] : mx;
      if constexpr (PW != 0) pb[i] = pay[r];
    }
  }
  wave_minmax_u64(mn, mx);
  if constexpr (TW > 1) {
    if (ln == 0) { rmin[tw] = mn; rmax[tw] = mx; }
    team_sync<TW>();
    mn = rmin[0]; mx = rmax[0];
#pragma unroll
    for (int q = 1; q < TW; ++q) {
      mn = rmin[q] < mn ? rmin[q] : mn;
      mx = rmax[q] > mx ? rmax[q] : mx;
    }
  }
  const uint64_t range = mx - mn;
  const int bits = range ? 64 - __clzll((long long)range) : 0;
  if (bits == 0) {  // all keys equal: input order is the stable order
    if (src != dst)
      for (uint32_t i = tid; i < n; i += TT) {
        dst[start + i] = src[start + i];
        if constexpr (PW != 0) pay_store<PW>(pdst, start + i, pay_load<PW>(psrc, start + i));
      }
    team_sync<TW>();
    return true;
  }
  if (bits > 51) {
    team_sync<TW>();
    return false;
  }
  uint32_t nb = 64;
  while (nb < n) nb <<= 1;
  int d = 6;
  while ((1u << d) < nb) ++d;
  const int shb = bits > d ? bits - d : 0;
  for (uint32_t i = tid; i < nb / 2; i += TT) cnt[i] = 0;
  team_sync<TW>();
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint32_t i = r * TT + tid;
    if (i < n) {
      const uint32_t b = (uint32_t)((key[r] - mn) >> shb);
      atomicAdd(&cnt[b >> 1], 1u << ((b & 1u) * 16u));
    }
  }
  team_sync<TW>();
  // a bucket above kBucketMax keys: a one-wave group takes it if every such
  // bucket holds one key value (a run of duplicates, Section III's duplicate
  // handling), placed in input order; otherwise the group is left to the
  // fallback sort
  bool runs = false;
  if (!bucket_starts<TW>(cnt, nb, sh, tid)) {
    if constexpr (TW != 1) return false;
    runs = true;
    bucket_starts<TW>(cnt, nb, sh, tid, false);
  }
  // place the words
  if (!runs) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t i = r * TT + tid;
      if (i < n) {
        const uint64_t dlt = key[r] - mn;
        const uint32_t b = (uint32_t)(dlt >> shb);
        const uint32_t sft = (b & 1u) * 16u;
        const uint32_t old = atomicAdd(&cnt[b >> 1], 1u << sft);
        const uint32_t pos = min((old >> sft) & 0xFFFFu, (uint32_t)(TT * R) - 1);
        kb[pos] = (dlt << 12) | i;
      }
    }
  } else if constexpr (TW == 1) {
    // stable placement: round by round (positions in order), the lanes of a
    // bucket in lane order after the bucket's earlier rounds; the lowest lane
    // of each bucket advances its counter for all of them
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t i = r * TT + tid;
      const bool valid = i < n;
      const uint64_t dlt = key[r] - mn;
      const uint32_t b = valid ? (uint32_t)(dlt >> shb) : 0u;
      uint64_t peers = __ballot(valid);
      for (int q = 0; (1u << q) < nb; ++q) {
        const bool bit = ((b >> q) & 1u) != 0;
        const uint64_t m = __ballot(valid && bit);
        peers &= bit ? m : ~m;
      }
      const uint32_t lead = valid ? (uint32_t)__ffsll((unsigned long long)peers) - 1u : 0u;
      const uint32_t sft = (b & 1u) * 16u;
      uint32_t old = 0;
      if (valid && tid == lead) old = atomicAdd(&cnt[b >> 1], (uint32_t)__popcll(peers) << sft);
      old = __shfl(old, (int)lead);
      if (valid) {
        const uint32_t below = (uint32_t)__popcll(peers & ((1ull << tid) - 1ull));
        const uint32_t pos = min(((old >> sft) & 0xFFFFu) + below, (uint32_t)(TT * R) - 1);
        kb[pos] = (dlt << 12) | i;
      }
    }
  }
  team_sync<TW>();
  if (runs) {
    // every bucket above kBucketMax keys must hold one key value
    bool mixed = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t i = r * TT + tid;
      if (i < n) {
        const uint64_t v = kb[i];
        const uint32_t b = (uint32_t)((v >> 12) >> shb);
        const uint32_t e = c16_get(cnt, b);
        const uint32_t s0 = b ? c16_get(cnt, b - 1) : 0u;
        if (e - s0 > (uint32_t)kBucketMax && (v >> 12) != (kb[s0] >> 12)) mixed = true;
      }
    }
    if (__ballot(mixed) != 0ull) {
      team_sync<TW>();
      return false;
    }
  }
  // Bucket b now spans [end(b-1), end(b)).  A word's place in the output is
  // its bucket's start plus the number of smaller words in the bucket (the
  // words are unique); in a run of one key value, placed in input order, its
  // slot.  Keys and payloads go straight to their places (a permutation
  // inside each bucket: nearly sequential).
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint32_t i = r * TT + tid;
    if (i < n) {
      const uint64_t v = kb[i];
      const uint32_t b = (uint32_t)((v >> 12) >> shb);
      const uint32_t e = c16_get(cnt, b);
      const uint32_t s0 = b ? c16_get(cnt, b - 1) : 0u;
      uint32_t p = i;
      if (!runs || e - s0 <= (uint32_t)kBucketMax) {
        uint32_t rank = 0;
        for (uint32_t j = s0; j < e; ++j) rank += kb[j] < v ? 1u : 0u;
        p = min(s0 + rank, n - 1);
      }
      dst[start + p] = (v >> 12) + mn;
      if constexpr (PW != 0) pay_store<PW>(pdst, start + p, pb[v & 4095u]);
    }
  }
  team_sync<TW>();
  return true;
}

template <int PW, int TW, int R>
__device__ bool fast_sort(uint64_t* kb, typename PayT<PW>::T* pb, uint32_t* cnt, uint64_t* rmin,
                          uint64_t* rmax, uint32_t* sh, const uint64_t* __restrict__ src,
                          const void* psrc, uint64_t* __restrict__ dst, void* pdst,
                          uint64_t start, uint32_t n, uint32_t tid) {
  uint64_t key[R];
  typename PayT<PW>::T pay[R];
  group_load<PW, TW * kWave, R>(src, psrc, start, n, tid, key, pay);
  return fast_sort_regs<PW, TW, R>(kb, pb, cnt, rmin, rmax, sh, src, psrc, dst, pdst, start, n, tid,
                                   key, pay);
}

__device__ void push_hard(Ws& ws, int S, const Leaf& lf) {
  atomicAdd(&ws.ctl->n_hard, 1u);
  const uint32_t h = atomicAdd(&ws.ctl->nhard[S], 1u);
  if (h < ws.leaf_cap) ws.hard[S][h] = lf;
  else atomicOr(&ws.ctl->error, ERR_LEAFCAP);
}

template <int PW>
__global__ void __launch_bounds__(kBlock) k_local_hard(Ws ws, int L) {
  using Sm = LocSmem<PW>;
  __shared__ Sm sm;
  Ctl* c = ws.ctl;
  if (call_failed(c)) return;
  const int S = L & 1;
  const uint32_t nh = min(c->nhard[S], ws.leaf_cap);
  uint64_t* __restrict__ dst = ws.keys[0];
  void* pdst = ws.pay[0];
  const uint32_t wv = wave(), ln = lane();
  const int t = threadIdx.x;
  // groups of > kWaveCap keys: the whole workgroup
  for (uint32_t g = blockIdx.x; g < nh; g += gridDim.x) {
    const Leaf lf = ws.hard[S][g];
    if (lf.count <= (uint32_t)kWaveCap) continue;
    team_sort<PW, kWaves>(sm.k, sm.pay, sm.cnt, sm.cnt[kWaves], sm.rmin, sm.rmax, sm.sh,
                          ws.keys[lf.src], ws.pay[lf.src], dst, pdst, lf.start, lf.count,
                          (uint32_t)t, 2 * kWaves * 256 * 2);
  }
  __syncthreads();
  // groups of <= kWaveCap keys: one wave each
  constexpr uint32_t kWaveWords = kWaveCap + kWaveCap / 16;
  uint64_t* kb = sm.k + wv * kWaveWords;
  typename PayT<PW>::T* pb = sm.pay + (PW ? wv * kWaveCap : 0);
  for (uint32_t g = blockIdx.x * kWaves + wv; g < nh; g += gridDim.x * kWaves) {
    const Leaf lf = ws.hard[S][g];
    if (lf.count > (uint32_t)kWaveCap) continue;
    team_sort<PW, 1>(kb, pb, &sm.cnt[wv], sm.cnt[kWaves + wv], nullptr, nullptr, nullptr,
                     ws.keys[lf.src], ws.pay[lf.src], dst, pdst, lf.start, lf.count, ln, 256 * 2);
  }
}

template <int PW>
__device__ __forceinline__ void local_body(Ws ws, int L);

// the local sort's kernel: with payloads of up to 4 bytes a wave job holds 10
// keys per lane, and the register budget is pinned to four waves per SIMD
template <int PW>
__global__ void __launch_bounds__(kBlock, 4) k_local(Ws ws, int L) {
  local_body<PW>(ws, L);
}
template <>
__global__ void __launch_bounds__(kBlock) k_local<8>(Ws ws, int L) {
  local_body<8>(ws, L);
}

template <int PW>
__device__ __forceinline__ void local_body(Ws ws, int L) {
  using Sm = FastSmem<PW>;
  __shared__ Sm sm;
  Ctl* c = ws.ctl;
  if (call_failed(c)) return;
  const int S = L & 1;
  const uint32_t nl = min(c->nleaf[S], ws.leaf_cap);
  const uint32_t nlw = min(c->nleafw[S], ws.leaf_cap);
  uint64_t* __restrict__ dst = ws.keys[0];
  void* pdst = ws.pay[0];
  const uint32_t wv = wave(), ln = lane();
  const int t = threadIdx.x;
  uint64_t moved = 0;  // keys this thread accounted for (statistics only)

  // block jobs: copies of all-identical segments and groups of > kMidCap keys
  for (uint32_t g = blockIdx.x; g < nl; g += gridDim.x) {
    const Leaf lf = ws.leaves[S][g];
    const uint64_t* __restrict__ src = ws.keys[lf.src];
    const void* psrc = ws.pay[lf.src];
    const uint32_t n = lf.count;
    if (t == 0 && (lf.src != 0 || (!(lf.flags & LF_COPY) && n > 1))) moved += n;
    if ((lf.flags & LF_COPY) || n <= 1) {
      if (lf.src != 0)
        for (uint32_t i = t; i < n; i += kBlock) {
          dst[lf.start + i] = src[lf.start + i];
          if constexpr (PW != 0) pay_store<PW>(pdst, lf.start + i, pay_load<PW>(psrc, lf.start + i));
        }
      continue;
    }
    if (n > (uint32_t)kBlockCap) {  // k_local_big's (above its cap: never made; the fallback)
      if (n > (uint32_t)kBigCap && t == 0) push_hard(ws, S, lf);
      continue;
    }
    const bool ok = fast_sort<PW, kWaves, kBlockCap / kBlock>(
        sm.k, sm.pay, sm.cnt, sm.rmin, sm.rmax, sm.sh, src, psrc, dst, pdst, lf.start, n,
        (uint32_t)t);
    if (!ok && t == 0) push_hard(ws, S, lf);
  }
  __syncthreads();
  // wave jobs: groups of <= wave_job_cap(PW) keys, one wave each
  constexpr int WCAP = wave_job_cap(PW);
  uint64_t* kb = sm.k + wv * WCAP;
  typename PayT<PW>::T* pb = sm.pay + (PW ? wv * WCAP : 0);
  uint32_t* cb = sm.cnt + wv * (pow2_ceil(WCAP) / 2);
  // the next group's keys and payloads are loaded while this one is sorted
  constexpr int RW = WCAP / kWave;
  using P = typename PayT<PW>::T;
  const uint32_t gs = gridDim.x * kWaves;
  uint32_t g = blockIdx.x * kWaves + wv;
  // (and the descriptor of the group after it, so that the next group's
  // loads need not wait for their descriptor)
  Leaf lf{}, nf{};
  uint64_t key[RW];
  P pay[RW];
  if (g < nlw) {
    lf = ws.leavesw[S][g];
    group_load<PW, kWave, RW>(ws.keys[lf.src], ws.pay[lf.src], lf.start, lf.count, ln, key, pay);
  }
  if (g + gs < nlw) nf = ws.leavesw[S][g + gs];
  for (; g < nlw; g += gs) {
    const uint32_t gn = g + gs;
    Leaf nnf{};
    if (gn + gs < nlw) nnf = ws.leavesw[S][gn + gs];
    uint64_t nkey[RW];
    P npay[RW];
    if (gn < nlw)
      group_load<PW, kWave, RW>(ws.keys[nf.src], ws.pay[nf.src], nf.start, nf.count, ln, nkey,
                                npay);
    const uint64_t* __restrict__ src = ws.keys[lf.src];
    const void* psrc = ws.pay[lf.src];
    const uint32_t n = lf.count;
    if (ln == 0 && (lf.src != 0 || n > 1)) moved += n;
    if (n <= 1) {
      if (lf.src != 0 && ln == 0 && n == 1) {
        dst[lf.start] = key[0];
        if constexpr (PW != 0) pay_store<PW>(pdst, lf.start, pay[0]);
      }
    } else {
      const bool ok = fast_sort_regs<PW, 1, RW>(kb, pb, cb, nullptr, nullptr, nullptr, src, psrc,
                                                dst, pdst, lf.start, n, ln, key, pay);
      if (!ok && ln == 0) push_hard(ws, S, lf);
    }
    lf = nf;
    nf = nnf;
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      key[r] = nkey[r];
      pay[r] = npay[r];
    }
  }
  // one statistics atomic per workgroup
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) moved += __shfl_xor(moved, o);
  __syncthreads();
  if (ln == 0) sm.rmin[wv] = moved;
  __syncthreads();
  if (t == 0) {
    uint64_t tot = 0;
    for (int q = 0; q < kWaves; ++q) tot += sm.rmin[q];
    if (tot) atomicAdd((unsigned long long*)&c->local_keys, (unsigned long long)tot);
  }
}

// Groups of wave_job_cap(PW) < n <= kMidCap keys: one wave each (a workgroup
// of one wave, 16 keys per lane), which costs far less per key than a whole
// workgroup on a group of barely more than a wave job.
template <int PW>
struct MidSmem {
  uint64_t k[kMidCap];
  typename PayT<PW>::T pay[PW ? kMidCap : 1];
  uint32_t cnt[kMidCap / 2];
};

template <int PW>
__global__ void __launch_bounds__(kWave) k_local_mid(Ws ws, int L) {
  __shared__ MidSmem<PW> sm;
  Ctl* c = ws.ctl;
  if (call_failed(c)) return;
  const int S = L & 1;
  const uint32_t nl = min(c->nleafm[S], ws.leaf_cap);
  uint64_t* __restrict__ dst = ws.keys[0];
  void* pdst = ws.pay[0];
  const uint32_t ln = lane();
  uint64_t moved = 0;
  for (uint32_t g = blockIdx.x; g < nl; g += gridDim.x) {
    const Leaf lf = ws.leavesm[S][g];
    const uint32_t n = lf.count;
    if (n > (uint32_t)kMidCap) continue;   // (never: the list holds n <= kMidCap)
    moved += n;
    const bool ok = fast_sort<PW, 1, kMidCap / kWave>(sm.k, sm.pay, sm.cnt, nullptr, nullptr,
                                                      nullptr, ws.keys[lf.src], ws.pay[lf.src],
                                                      dst, pdst, lf.start, n, ln);
    if (!ok && ln == 0) push_hard(ws, S, lf);
  }
  // Wave jobs whose keys may span 2^51 or more (so the classification says):
  // the fast sort if the range turns out to fit it, else the sort for any
  // range, the next group's keys loaded meanwhile; a group neither takes
  // goes to the fallback kernel.  A group has at most kWaveCap keys: the
  // second half of the key area holds the slots' buckets.
  {
    using P = typename PayT<PW>::T;
    constexpr int RX = kWaveCap / kWave;
    static_assert(2 * kWaveCap <= kMidCap, "bucket ids beside the words");
    uint16_t* bkt = reinterpret_cast<uint16_t*>(sm.k + kWaveCap);
    const uint32_t nx = min(c->nleafx[S], ws.leaf_cap);
    uint32_t gx = blockIdx.x;
    Leaf xf{};
    uint64_t xkey[RX];
    P xpay[RX];
    if (gx < nx) {
      xf = ws.leavesx[S][gx];
      group_load<PW, kWave, RX>(ws.keys[xf.src], ws.pay[xf.src], xf.start, xf.count, ln, xkey, xpay);
    }
    for (; gx < nx; gx += gridDim.x) {
      const uint32_t gn = gx + gridDim.x;
      Leaf nf{};
      uint64_t nkey[RX];
      P npay[RX];
      if (gn < nx) {
        nf = ws.leavesx[S][gn];
        group_load<PW, kWave, RX>(ws.keys[nf.src], ws.pay[nf.src], nf.start, nf.count, ln, nkey,
                                  npay);
      }
      moved += xf.count;
      const bool ok =
          fast_sort_regs<PW, 1, RX>(sm.k, sm.pay, sm.cnt, nullptr, nullptr, nullptr,
                                    ws.keys[xf.src], ws.pay[xf.src], dst, pdst, xf.start, xf.count,
                                    ln, xkey, xpay) ||
          wide_wave_sort<PW, RX>(sm.k, bkt, sm.pay, sm.cnt, kMidCap, dst, pdst, xf.start, xf.count,
                                 ln, xkey, xpay);
      if (!ok && ln == 0) push_hard(ws, S, xf);
      xf = nf;
#pragma unroll
      for (int r = 0; r < RX; ++r) {
        xkey[r] = nkey[r];
        xpay[r] = npay[r];
      }
    }
  }
  if (ln == 0 && moved) atomicAdd((unsigned long long*)&c->local_keys, (unsigned long long)moved);
}

// Block jobs of kBlockCap < n <= kBigCap keys (cutoffs above kBlockCap): a
// workgroup of 512 threads with 8 keys each, in a kernel of its own so that
// the main kernel's LDS (and with it its occupancy) stays sized for
// kBlockCap.  The main kernel counts these groups in its statistics.
constexpr int kBigThreads = 512;
constexpr int kBigWaves = kBigThreads / kWave;
template <int PW>
struct BigSmem {
  uint64_t k[kBigCap];
  typename PayT<PW>::T pay[PW ? kBigCap : 1];
  uint32_t cnt[kBigCap / 2];
  uint64_t rmin[kBigWaves], rmax[kBigWaves];
  uint32_t sh[kBigWaves + 2];
};

template <int PW>
__global__ void __launch_bounds__(kBigThreads) k_local_big(Ws ws, int L) {
  __shared__ BigSmem<PW> sm;
  Ctl* c = ws.ctl;
  if (call_failed(c)) return;
  const int S = L & 1;
  const uint32_t nl = min(c->nleaf[S], ws.leaf_cap);
  uint64_t* __restrict__ dst = ws.keys[0];
  void* pdst = ws.pay[0];
  const int t = threadIdx.x;
  for (uint32_t g = blockIdx.x; g < nl; g += gridDim.x) {
    const Leaf lf = ws.leaves[S][g];
    const uint32_t n = lf.count;
    if ((lf.flags & LF_COPY) || n <= (uint32_t)kBlockCap || n > (uint32_t)kBigCap) continue;
    const bool ok = fast_sort<PW, kBigWaves, kBigCap / kBigThreads>(
        sm.k, sm.pay, sm.cnt, sm.rmin, sm.rmax, sm.sh, ws.keys[lf.src], ws.pay[lf.src], dst, pdst,
        lf.start, n, (uint32_t)t);
    if (!ok && t == 0) push_hard(ws, S, lf);
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <int KMAX, int KBITS, int PW, int ROUNDS, int SB>
static const void* stage_fn(int stage) {
  switch (stage) {
    case STAGE_MOMENTS: return (const void*)k_moments;
    case STAGE_FINALIZE: return (const void*)k_finalize;
    case STAGE_HIST: return (const void*)k_hist<KMAX, 0>;
    case STAGE_SCATTER: return (const void*)k_scatter<KMAX, KBITS, PW, ROUNDS, SB>;
    case STAGE_LOCAL: return (const void*)k_local<PW>;
    default: return (const void*)k_local_hard<PW>;
  }
}

// resident workgroups of a kernel on the whole device (at most 16 per CU)
static int resident_grid(const void* fn, int threads) {
  int nb = 0, dev = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, threads, 0) != hipSuccess || nb < 1)
    nb = 1;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus < 1)
    cus = 1;
  return (nb < 16 ? nb : 16) * cus;
}
// one-wave workgroups of k_local_mid
template <int PW>
static int mid_grid() {
  static int g = 0;
  if (g == 0) g = resident_grid((const void*)k_local_mid<PW>, kWave);
  return g;
}
template <int PW>
static int big_grid() {
  static int g = 0;
  if (g == 0) g = resident_grid((const void*)k_local_big<PW>, kBigThreads);
  return g;
}

template <int KMAX, int KBITS, int PW, int ROUNDS, int SB>
static void launch_stage_t(const Ws& ws, int L, int stage, int grid, hipStream_t st) {
  switch (stage) {
    case STAGE_MOMENTS:
      hipLaunchKernelGGL(k_moments, dim3(grid), dim3(kBlock), 0, st, ws, L);
      break;
    case STAGE_FINALIZE:
      hipLaunchKernelGGL(k_finalize, dim3(grid), dim3(kFinThreads), 0, st, ws, L);
      break;
    case STAGE_HIST:
      if (ws.lm.ids && ws.lm.direct)
        hipLaunchKernelGGL((k_hist<KMAX, 2>), dim3(grid), dim3(kBlock), 0, st, ws, L);
      else if (ws.lm.ids)
        hipLaunchKernelGGL((k_hist<KMAX, 1>), dim3(grid), dim3(kBlock), 0, st, ws, L);
      else if (KMAX <= 1024 && ws.p.fuse)
        hipLaunchKernelGGL((k_hist<KMAX, (KMAX <= 1024 ? 3 : 0)>), dim3(grid), dim3(kBlock), 0, st,
                           ws, L);
      else
        hipLaunchKernelGGL((k_hist<KMAX, 0>), dim3(grid), dim3(kBlock), 0, st, ws, L);
      break;
    case STAGE_SCATTER:
      if constexpr (KMAX <= 1024) {
        if (ws.p.fuse) {
          hipLaunchKernelGGL((k_scatter<KMAX, KBITS, PW, ROUNDS, SB, true>), dim3(grid), dim3(SB), 0,
                             st, ws, L);
          break;
        }
      }
      hipLaunchKernelGGL((k_scatter<KMAX, KBITS, PW, ROUNDS, SB>), dim3(grid), dim3(SB), 0, st, ws,
                         L);
      break;
    case STAGE_LOCAL:
      hipLaunchKernelGGL((k_local<PW>), dim3(grid), dim3(kBlock), 0, st, ws, L);
      hipLaunchKernelGGL((k_local_mid<PW>), dim3(mid_grid<PW>()), dim3(kWave), 0, st, ws, L);
      if (ws.p.cutoff > kBlockCap)  // groups above kBlockCap exist only then
        hipLaunchKernelGGL((k_local_big<PW>), dim3(big_grid<PW>()), dim3(kBigThreads), 0, st, ws, L);
      break;
    default:
      hipLaunchKernelGGL((k_local_hard<PW>), dim3(grid), dim3(kBlock), 0, st, ws, L);
      break;
  }
}

}  // namespace zs

// entry points used by the host planner (zsort_api.cpp)
namespace zs {

// Workspace of zsort_stable_noalloc: a fixed array in device memory, one per
// GPU.  In host code its name is only a stand-in; the device address is
// looked up once per device (with that device current) and kept.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

hipError_t scratch_address(int dev, void** out) {
  static void* addr[256] = {};
  if (dev < 0 || dev >= 256) return hipErrorInvalidDevice;
  if (!addr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = p;
  }
  *out = addr[dev];
  return hipSuccess;
}

// signed keys: two's complement order is the unsigned order of x ^ 2^63
__global__ void __launch_bounds__(kBlock) k_flip(uint64_t* __restrict__ x, uint64_t n) {
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride)
    x[i] ^= 0x8000000000000000ull;
}

hipError_t launch_flip(uint64_t* keys, uint64_t n, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_flip, dim3(grid), dim3(kBlock), 0, st, keys, n);
  return hipGetLastError();
}

hipError_t launch_reset(const Ws& ws, hipStream_t st) {
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, st, ws);
  return hipGetLastError();
}

// *flag = 1 if some keys[i] > keys[i + 1]
__global__ void k_check_sorted(const uint64_t* __restrict__ x, uint64_t n, uint32_t* flag) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  bool bad = false;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i + 1 < n; i += stride)
    bad |= x[i] > x[i + 1];
  if (__any(bad) && lane() == 0) atomicOr(flag, 1u);
}

hipError_t launch_check_sorted(const uint64_t* keys, uint64_t n, uint32_t* flag, int grid,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_check_sorted, dim3(grid), dim3(kBlock), 0, st, keys, n, flag);
  return hipGetLastError();
}

hipError_t launch_clear_rows(const Ws& ws, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_clear_rows, dim3(grid), dim3(kBlock), 0, st, ws);
  return hipGetLastError();
}

hipError_t launch_init_single(const Ws& ws, uint64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_init_single, dim3(64), dim3(kBlock), 0, st, ws, n);
  return hipGetLastError();
}

hipError_t launch_reset_lists(const Ws& ws, int slot, hipStream_t st) {
  hipLaunchKernelGGL(k_reset_lists, dim3(1), dim3(64), 0, st, ws, slot);
  return hipGetLastError();
}

hipError_t launch_init_learned(const Ws& ws, uint64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_init_learned, dim3(64), dim3(kBlock), 0, st, ws, n);
  return hipGetLastError();
}

hipError_t launch_init_runs(const Ws& ws, const uint32_t* runs, const uint32_t* nruns, int grid,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_init_runs, dim3(grid), dim3(kBlock), 0, st, ws, runs, nruns);
  return hipGetLastError();
}

hipError_t launch_init_segments(const Ws& ws, const int64_t* off, int32_t nseg, uint64_t n,
                                hipStream_t st) {
  const int blocks = (nseg + kBlock) / kBlock + 1;
  hipLaunchKernelGGL(k_check_offsets, dim3(blocks), dim3(kBlock), 0, st, ws, off, nseg, n);
  hipLaunchKernelGGL(k_init_segments, dim3(blocks), dim3(kBlock), 0, st, ws, off, nseg);
  return hipGetLastError();
}

// (k, payload bytes, tile) -> template instance (clusters, their bits, payload
// bytes, keys per thread, threads of the scatter's workgroup).  Tiles of 2048
// and 4096 keys take 256 threads (8 and 16 keys each); 8192-key tiles take
// 1024 threads of 8 keys: twice the waves per compute unit of the 4096-key
// tile at the same registers per thread, and twice its run of each cluster
// per tile.  KMAX 4096 only with 2048-key tiles.
#define ZS_TILES(CALL, KM, KB, PWV)                                         \
  do {                                                                      \
    if (ws_tile == 8192) CALL(KM, KB, PWV, 8, 1024);                        \
    else if (ws_tile == 4096) CALL(KM, KB, PWV, 16, 256);                   \
    else CALL(KM, KB, PWV, 8, 256);                                         \
  } while (0)
#define ZS_PAYLOADS(CALL, KM, KB)                                           \
  do {                                                                      \
    if (pw == 0) ZS_TILES(CALL, KM, KB, 0);                                 \
    else if (pw == 4) ZS_TILES(CALL, KM, KB, 4);                            \
    else ZS_TILES(CALL, KM, KB, 8);                                         \
  } while (0)
#define ZS_DISPATCH(CALL)                                                   \
  do {                                                                      \
    if (k <= 256) ZS_PAYLOADS(CALL, 256, 8);                                \
    else if (k <= 512) ZS_PAYLOADS(CALL, 512, 9);                           \
    else if (k <= 1024) ZS_PAYLOADS(CALL, 1024, 10);                        \
    else if (pw == 0) CALL(4096, 12, 0, 8, 256);                            \
    else if (pw == 4) CALL(4096, 12, 4, 8, 256);                            \
    else CALL(4096, 12, 8, 8, 256);                                         \
  } while (0)

hipError_t launch_stage(const Ws& ws, int L, int stage, int grid, hipStream_t st) {
  const int k = ws.p.k;
  const int pw = ws.p.pw;
  const int ws_tile = ws.p.tile;
#define ZS_LAUNCH(KM, KB, PWV, R, SB) launch_stage_t<KM, KB, PWV, R, SB>(ws, L, stage, grid, st)
  ZS_DISPATCH(ZS_LAUNCH);
#undef ZS_LAUNCH
  return hipGetLastError();
}

// resident workgroups per compute unit of a stage's kernel (at least 1)
int stage_blocks_per_cu(int k, int pw, int ws_tile, int stage) {
  const void* fn = nullptr;
  int threads = kBlock;
#define ZS_FN(KM, KB, PWV, R, SB) \
  fn = stage_fn<KM, KB, PWV, R, SB>(stage), threads = stage == STAGE_SCATTER ? SB : kBlock
  ZS_DISPATCH(ZS_FN);
#undef ZS_FN
  if (!fn) return 1;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, threads, 0) != hipSuccess || nb < 1)
    return 1;
  return nb;
}
#undef ZS_DISPATCH
#undef ZS_PAYLOADS
#undef ZS_TILES

}  // namespace zs
