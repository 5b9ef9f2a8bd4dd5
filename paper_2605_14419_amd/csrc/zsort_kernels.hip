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

__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t v) {
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    uint32_t t = __shfl_up(v, o);
    if (lane() >= (uint32_t)o) v += t;
  }
  return v;
}

__device__ __forceinline__ int wave_incl_max(int v) {
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    int t = __shfl_up(v, o);
    if (lane() >= (uint32_t)o) v = max(v, t);
  }
  return v;
}

// exclusive block sum of one value per thread; `sh` holds kWaves words
__device__ __forceinline__ uint32_t block_excl_sum(uint32_t v, uint32_t* sh, uint32_t* total) {
  uint32_t inc = wave_incl_sum(v);
  if (lane() == kWave - 1) sh[wave()] = inc;
  __syncthreads();
  uint32_t base = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kWaves; ++i) {
    uint32_t s = sh[i];
    base += (i < (int)wave()) ? s : 0u;
    tot += s;
  }
  __syncthreads();
  if (total) *total = tot;
  return base + inc - v;
}

// in-place exclusive sum over a[0, N) in LDS; returns the total
__device__ uint32_t block_scan_lds(uint32_t* a, int N, uint32_t* sh) {
  const int ipt = (N + kBlock - 1) / kBlock;
  const int b0 = threadIdx.x * ipt;
  uint32_t s = 0;
  for (int i = 0; i < ipt; ++i) {
    int j = b0 + i;
    if (j < N) s += a[j];
  }
  uint32_t tot;
  uint32_t base = block_excl_sum(s, sh, &tot);
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

// r += v * 2^(32*pos) for a 64-bit v
__device__ __forceinline__ void w8_add64_at(W8& r, uint64_t v, int pos) {
  uint64_t carry = 0;
  for (int i = pos; i < 8; ++i) {
    uint64_t add = carry;
    if (i == pos) add += (uint32_t)v;
    if (i == pos + 1) add += (uint32_t)(v >> 32);
    uint64_t s = (uint64_t)r.d[i] + add;
    r.d[i] = (uint32_t)s;
    carry = s >> 32;
    if (i > pos + 1 && carry == 0) break;
  }
}

__device__ __forceinline__ W8 w8_add(const W8& a, const W8& b) {
  W8 r;
  uint64_t c = 0;
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
  for (int i = 0; i < 8; ++i) {
    if (a.d[i] == 0) continue;
    uint64_t carry = 0;
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
// every lower bit folded into a sticky bit, then an exact power-of-two scale
__device__ double w8_to_double(const W8& a) {
  int top = -1;
  for (int i = 7; i >= 0; --i)
    if (a.d[i]) { top = i; break; }
  if (top < 0) return 0.0;
  const int bitlen = top * 32 + (32 - __clz(a.d[top]));
  if (bitlen <= 64) {
    uint64_t v = ((uint64_t)a.d[1] << 32) | a.d[0];
    return __ull2double_rn(v);
  }
  const int s = bitlen - 64;  // keep bits [s, s+64)
  uint64_t w = 0;
  for (int k = 0; k < 64; ++k) {
    int bit = s + k;
    uint32_t v = (a.d[bit >> 5] >> (bit & 31)) & 1u;
    w |= (uint64_t)v << k;
  }
  bool sticky = false;
  for (int bit = 0; bit < s; ++bit)
    if ((a.d[bit >> 5] >> (bit & 31)) & 1u) { sticky = true; break; }
  if (sticky) w |= 1;
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
// look-back status words: tag(22) | flag(2) | value(40)
// ---------------------------------------------------------------------------
constexpr uint64_t kValMask = (1ull << 40) - 1;
constexpr uint32_t FL_AGG = 1u, FL_INC = 2u;
constexpr uint32_t kSpinLimit = 1u << 20;

// a capacity or wait limit was hit earlier in this call: later kernels stop
__device__ __forceinline__ bool call_failed(const Ctl* c) {
  return __hip_atomic_load(&c->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
}

__device__ __forceinline__ uint32_t level_tag(uint32_t epoch, int L) {
  return (epoch * 64u + (uint32_t)L) & 0x3FFFFFu;
}
__device__ __forceinline__ void st_publish(uint64_t* p, uint32_t tag, uint32_t flag, uint64_t v) {
  uint64_t w = ((uint64_t)tag << 42) | ((uint64_t)flag << 40) | (v & kValMask);
  __hip_atomic_store(p, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// reset + level-0 set-up
// ---------------------------------------------------------------------------
__device__ void seg_clear_acc(Seg& s) {
  for (int i = 0; i < 8; ++i) s.acc[i] = 0;
  s.amin = ~0ull;
  s.amax = 0;
  s.done = 0;
  s.kind = KIND_PENDING;
  s.shift = 0;
  s.o = s.M = 0;
  s.m = s.sigma = s.zmin = s.A = s.B = 0.0;
}

__global__ void k_reset(Ws ws) {
  Ctl* c = ws.ctl;
  const int t = threadIdx.x;
  if (t < kMaxLevels) {
    c->tick[t] = 0;
    c->lvl_keys[t] = 0;
    c->lvl_mkeys[t] = 0;
    c->lvl_segs[t] = 0;
  }
  if (t == 0) {
    c->epoch = c->epoch + 1u;
    for (int s = 0; s < 2; ++s) { c->nseg[s] = 0; c->nwork[s] = 0; c->nleaf[s] = 0; c->nstatus[s] = 0; }
    c->error = 0;
    c->ntrace = 0;
    c->ntrace_hist = 0;
    c->n_ident = c->n_rmap = c->n_leafgroups = 0;
    c->max_level = 0;
  }
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

// one array [0, n): root segment (n > cutoff) or a single leaf
__global__ void k_init_single(Ws ws, uint64_t n) {
  Ctl* c = ws.ctl;
  const uint64_t ch = (uint64_t)ws.p.chunk;
  if (n <= (uint64_t)ws.p.cutoff) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      Leaf& lf = ws.leaves[0][0];
      lf.start = 0; lf.count = (uint32_t)n; lf.flags = 0; lf.src = 0;
      c->nleaf[0] = 1;
      c->n_leafgroups = 1;
    }
    return;
  }
  const uint32_t nch = (uint32_t)((n + ch - 1) / ch);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    make_root_seg(ws, 0, 0, n, 0, nch, 0);
    c->nseg[0] = 1;
    c->nwork[0] = nch;
    c->nstatus[0] = nch > 1 ? nch : 0;
  }
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nch; i += gridDim.x * blockDim.x)
    ws.work[0][i] = (uint64_t)i;  // segment 0, chunk i
}

// independent arrays [off[i], off[i+1]); offsets were validated by k_check_offsets
__global__ void k_check_offsets(Ws ws, const int64_t* off, int32_t nseg, uint64_t n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i <= nseg; i += gridDim.x * blockDim.x) {
    bool bad = false;
    if (i == 0 && off[0] != 0) bad = true;
    if (i == nseg && (uint64_t)off[nseg] != n) bad = true;
    if (i < nseg && off[i + 1] < off[i]) bad = true;
    if (bad) atomicOr(&ws.ctl->error, 0x100u);
  }
}

__global__ void k_init_segments(Ws ws, const int64_t* off, int32_t nseg) {
  Ctl* c = ws.ctl;
  if (__hip_atomic_load(&c->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  const uint64_t ch = (uint64_t)ws.p.chunk;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nseg; i += gridDim.x * blockDim.x) {
    const uint64_t a = (uint64_t)off[i], len = (uint64_t)(off[i + 1] - off[i]);
    if (len <= 1) continue;
    if (len <= (uint64_t)ws.p.cutoff) {
      uint32_t li = atomicAdd(&c->nleaf[0], 1u);
      if (li >= ws.leaf_cap) { atomicOr(&c->error, ERR_LEAFCAP); continue; }
      Leaf& lf = ws.leaves[0][li];
      lf.start = a; lf.count = (uint32_t)len; lf.flags = 0; lf.src = 0;
      atomicAdd(&c->n_leafgroups, 1u);
      continue;
    }
    const uint32_t nch = (uint32_t)((len + ch - 1) / ch);
    uint32_t si = atomicAdd(&c->nseg[0], 1u);
    uint32_t wi = atomicAdd(&c->nwork[0], nch);
    uint32_t sb = nch > 1 ? atomicAdd(&c->nstatus[0], nch) : 0u;
    if (si >= ws.seg_cap || wi + nch > ws.work_cap || sb + (nch > 1 ? nch : 0) > ws.status_cap) {
      atomicOr(&c->error, ERR_SEGCAP);
      continue;
    }
    make_root_seg(ws, si, a, len, wi, nch, sb);
    for (uint32_t j = 0; j < nch; ++j) ws.work[0][wi + j] = ((uint64_t)si << 32) | j;
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

__device__ __noinline__ void finalize(Ws& ws, Seg& s, int L) {
  Ctl* c = ws.ctl;
  const uint64_t cnt = s.count;
  uint64_t acc[8];
  for (int i = 0; i < 8; ++i)
    acc[i] = __hip_atomic_load(&s.acc[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const uint64_t o = __hip_atomic_load(&s.amin, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const uint64_t M = __hip_atomic_load(&s.amax, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  s.o = o;
  s.M = M;
  atomicAdd((unsigned long long*)&c->lvl_mkeys[L], (unsigned long long)cnt);

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
    atomicAdd(&c->n_ident, 1u);
    trace_ident(ws, s);
    if (L & 1) {  // keys sit in the alternate buffer: copy them home
      uint32_t li = atomicAdd(&c->nleaf[L & 1], 1u);
      if (li >= ws.leaf_cap) { atomicOr(&c->error, ERR_LEAFCAP); return; }
      Leaf& lf = ws.leaves[L & 1][li];
      lf.start = s.start; lf.count = (uint32_t)s.count; lf.flags = LF_COPY; lf.src = 1;
    }
    return;
  }

  const int k = ws.p.k;
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
    atomicAdd(&c->n_rmap, 1u);
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
  if (blockIdx.x == 0 && threadIdx.x == 0) {  // lists of level L+1 start empty
    c->nseg[N] = 0; c->nwork[N] = 0; c->nleaf[N] = 0; c->nstatus[N] = 0;
  }
  const uint32_t nw = min(c->nwork[S], ws.work_cap);
  const uint64_t* __restrict__ x = ws.keys[S];
  const uint64_t ch = (uint64_t)ws.p.chunk;
  __shared__ uint64_t red[kWaves][10];
  __shared__ int last;

  for (uint32_t w = blockIdx.x; w < nw; w += gridDim.x) {
    const uint64_t item = ws.work[S][w];
    const uint32_t si = (uint32_t)(item >> 32), ci = (uint32_t)item;
    Seg& sg = ws.segs[S][si];
    const uint64_t beg = sg.start + (uint64_t)ci * ch;
    const uint64_t end = min(beg + ch, sg.start + sg.count);
    uint64_t a0 = 0, a1 = 0, a2 = 0, a3 = 0, a4 = 0, a5 = 0, b0 = 0, b1 = 0;
    uint64_t mn = ~0ull, mx = 0;
    for (uint64_t i = beg + threadIdx.x; i < end; i += kBlock) {
      const uint64_t v = x[i];
      const uint32_t xl = (uint32_t)v, xh = (uint32_t)(v >> 32);
      const uint64_t ll = (uint64_t)xl * xl, lh = (uint64_t)xl * xh, hh = (uint64_t)xh * xh;
      a0 += (uint32_t)ll; a1 += ll >> 32;
      a2 += (uint32_t)lh; a3 += lh >> 32;
      a4 += (uint32_t)hh; a5 += hh >> 32;
      b0 += xl; b1 += xh;
      mn = v < mn ? v : mn;
      mx = v > mx ? v : mx;
    }
    uint64_t vals[10] = {a0, a1, a2, a3, a4, a5, b0, b1, mn, mx};
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
#pragma unroll
      for (int j = 0; j < 8; ++j) vals[j] += __shfl_xor(vals[j], o);
      uint64_t tmn = __shfl_xor(vals[8], o), tmx = __shfl_xor(vals[9], o);
      vals[8] = tmn < vals[8] ? tmn : vals[8];
      vals[9] = tmx > vals[9] ? tmx : vals[9];
    }
    if (lane() == 0)
      for (int j = 0; j < 10; ++j) red[wave()][j] = vals[j];
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int wv = 1; wv < kWaves; ++wv) {
        for (int j = 0; j < 8; ++j) vals[j] += red[wv][j];
        vals[8] = red[wv][8] < vals[8] ? red[wv][8] : vals[8];
        vals[9] = red[wv][9] > vals[9] ? red[wv][9] : vals[9];
      }
      for (int j = 0; j < 8; ++j)
        if (vals[j]) atomicAdd((unsigned long long*)&sg.acc[j], (unsigned long long)vals[j]);
      atomicMin((unsigned long long*)&sg.amin, (unsigned long long)vals[8]);
      atomicMax((unsigned long long*)&sg.amax, (unsigned long long)vals[9]);
      __threadfence();
      const uint32_t old = atomicAdd(&sg.done, 1u);
      last = (old == sg.nchunks - 1) ? 1 : 0;
    }
    __syncthreads();
    if (last && threadIdx.x == 0) {
      __threadfence();
      finalize(ws, sg, L);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// hist: per-chunk LDS histogram, decoupled look-back over the chunks of a
// segment, and in the last chunk the exclusive scan + classification
// ---------------------------------------------------------------------------
template <int KMAX>
struct HistSmem {
  uint32_t h[KMAX];       // histogram, later totals
  uint32_t bst[KMAX];     // exclusive starts
  uint32_t t0[KMAX];      // scratch arrays for classification
  uint32_t t1[KMAX];
  uint32_t t2[KMAX];
  uint32_t sh[kWaves + 2];
  uint32_t w;
  uint32_t base_seg, base_work, base_status, base_leaf;
};

template <int KMAX>
__device__ void classify(Ws& ws, HistSmem<KMAX>& sm, Seg& sg, uint32_t si, int L) {
  Ctl* c = ws.ctl;
  const int k = ws.p.k;
  const uint32_t cutoff = (uint32_t)ws.p.cutoff;
  const uint64_t ch = (uint64_t)ws.p.chunk;
  const int S = L & 1, N = S ^ 1;
  const int t = threadIdx.x;

  // exclusive cluster starts
  for (int b = t; b < k; b += kBlock) sm.bst[b] = sm.h[b];
  __syncthreads();
  block_scan_lds(sm.bst, k, sm.sh);
  uint32_t* gb = ws.bstart + (uint64_t)si * (uint64_t)k;
  for (int b = t; b < k; b += kBlock) gb[b] = sm.bst[b];

  // children: index, chunk offset, look-back slot offset
  for (int b = t; b < k; b += kBlock) {
    const uint32_t n = sm.h[b];
    const bool child = n > cutoff;
    const uint32_t nch = child ? (uint32_t)((n + ch - 1) / ch) : 0u;
    sm.t0[b] = child ? 1u : 0u;
    sm.t1[b] = nch;
    sm.t2[b] = nch > 1 ? nch : 0u;
  }
  __syncthreads();
  const uint32_t nchild = block_scan_lds(sm.t0, k, sm.sh);
  const uint32_t nwork = block_scan_lds(sm.t1, k, sm.sh);
  const uint32_t nstat = block_scan_lds(sm.t2, k, sm.sh);
  if (t == 0) {
    sm.base_seg = nchild ? atomicAdd(&c->nseg[N], nchild) : 0u;
    sm.base_work = nwork ? atomicAdd(&c->nwork[N], nwork) : 0u;
    sm.base_status = nstat ? atomicAdd(&c->nstatus[N], nstat) : 0u;
    if (nchild) {
      atomicMax(&c->max_level, (uint32_t)(L + 1));
      if (sm.base_seg + nchild > ws.seg_cap) atomicOr(&c->error, ERR_SEGCAP);
      if (sm.base_work + nwork > ws.work_cap) atomicOr(&c->error, ERR_WORKCAP);
      if (sm.base_status + nstat > ws.status_cap) atomicOr(&c->error, ERR_STATUSCAP);
    }
  }
  __syncthreads();
  const bool fits = sm.base_seg + nchild <= ws.seg_cap && sm.base_work + nwork <= ws.work_cap &&
                    sm.base_status + nstat <= ws.status_cap;
  const double scale = (double)k / 4.0;
  const bool parent_r = sg.kind == KIND_RMAP;
  if (fits) {
    for (int b = t; b < k; b += kBlock) {
      const uint32_t n = sm.h[b];
      if (n <= cutoff) continue;
      const uint32_t idx = sm.base_seg + sm.t0[b];
      Seg& cs = ws.segs[N][idx];
      const bool crm = parent_r || (L + 1 >= ws.p.max_zlevels) || (uint64_t)n == sg.count;
      cs.start = sg.start + sm.bst[b];
      cs.count = n;
      cs.o_parent = sg.o;
      double e = 0.0;
      if (!crm) {  // estimated mean of cluster b, parent's frame
        double q = ((double)b + 0.5) / scale;
        q = q - sg.zmin;
        q = q * sg.sigma;
        e = q + sg.m;
      }
      cs.e = e;
      cs.depth = L + 1;
      cs.flags = crm ? F_RMAP : 0u;
      cs.nchunks = (uint32_t)((n + ch - 1) / ch);
      cs.first_work = sm.base_work + sm.t1[b];
      cs.status_base = sm.base_status + sm.t2[b];
      cs.parent = (int32_t)si;
      seg_clear_acc(cs);
    }
    // work items of the children, in chunk order; t0 now maps child -> bucket
    __syncthreads();
    // child list: position by child index
    for (int b = t; b < k; b += kBlock)
      if (sm.h[b] > cutoff) sm.t2[sm.t0[b]] = (uint32_t)b;  // t2 reused: child -> bucket
    __syncthreads();
    for (uint32_t j = t; j < nwork; j += kBlock) {
      // find the child whose chunk range holds j (binary search on t1 over children)
      uint32_t lo = 0, hi = nchild;  // invariant: t1[bucket(lo)] <= j
      while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (sm.t1[sm.t2[mid]] <= j) lo = mid; else hi = mid;
      }
      const uint32_t b = sm.t2[lo];
      ws.work[N][sm.base_work + j] = ((uint64_t)(sm.base_seg + lo) << 32) | (j - sm.t1[b]);
    }
  }
  __syncthreads();

  // leaf groups: a group is the leaf clusters of one run (no child between)
  // whose starts share one window [w*cutoff, (w+1)*cutoff); < 2*cutoff keys
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
      if (pb < 0 || sm.h[pb] > cutoff || sm.bst[pb] / cutoff != sm.bst[b] / cutoff) boundary = 2;
    }
    sm.t1[b] = boundary;
  }
  __syncthreads();
  for (int b = t; b < k; b += kBlock) sm.t2[b] = sm.t1[b] ? 1u : 0u;
  __syncthreads();
  const uint32_t nb = block_scan_lds(sm.t2, k, sm.sh);
  // compacted boundaries: position and kind, reuse t0 (positions) and h? keep
  // h intact for the trace: encode kind in the top bit of the position
  uint32_t* bpos = sm.t0;
  for (int b = t; b < k; b += kBlock)
    if (sm.t1[b]) bpos[sm.t2[b]] = sm.bst[b] | (sm.t1[b] == 2 ? 0x80000000u : 0u);
  __syncthreads();
  // count leaf groups
  uint32_t mine = 0;
  for (uint32_t i = t; i < nb; i += kBlock) mine += (bpos[i] >> 31);
  uint32_t ngroups;
  uint32_t myoff = block_excl_sum(mine, sm.sh, &ngroups);
  if (t == 0) {
    sm.base_leaf = ngroups ? atomicAdd(&c->nleaf[S], ngroups) : 0u;
    if (ngroups) atomicAdd(&c->n_leafgroups, ngroups);
    if (sm.base_leaf + ngroups > ws.leaf_cap) atomicOr(&c->error, ERR_LEAFCAP);
  }
  __syncthreads();
  if (sm.base_leaf + ngroups <= ws.leaf_cap) {
    uint32_t o = sm.base_leaf + myoff;
    for (uint32_t i = t; i < nb; i += kBlock) {
      if (!(bpos[i] >> 31)) continue;
      const uint32_t p0 = bpos[i] & 0x7FFFFFFFu;
      const uint32_t p1 = (i + 1 < nb) ? (bpos[i + 1] & 0x7FFFFFFFu) : (uint32_t)sg.count;
      Leaf& lf = ws.leaves[S][o++];
      lf.start = sg.start + p0;
      lf.count = p1 - p0;
      lf.flags = 0;
      lf.src = (uint32_t)N;  // written by this level's scatter
    }
  }

  // statistics and trace
  if (t == 0) {
    atomicAdd((unsigned long long*)&c->lvl_keys[L], (unsigned long long)sg.count);
    atomicAdd(&c->lvl_segs[L], 1u);
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
        r.depth = sg.depth; r.kind = sg.kind; r.start = sg.start; r.count = sg.count;
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

template <int KMAX>
__global__ void __launch_bounds__(kBlock) k_hist(Ws ws, int L) {
  __shared__ HistSmem<KMAX> sm;
  Ctl* c = ws.ctl;
  if (call_failed(c)) return;
  const int S = L & 1;
  const uint32_t nw = min(c->nwork[S], ws.work_cap);
  const int k = ws.p.k;
  const uint64_t ch = (uint64_t)ws.p.chunk;
  const uint64_t* __restrict__ x = ws.keys[S];
  const uint32_t tag = level_tag(c->epoch, L);
  const int t = threadIdx.x;

  while (true) {
    if (t == 0) sm.w = atomicAdd(&c->tick[L], 1u);
    __syncthreads();
    const uint32_t w = sm.w;
    __syncthreads();
    if (w >= nw) break;
    const uint64_t item = ws.work[S][w];
    const uint32_t si = (uint32_t)(item >> 32), ci = (uint32_t)item;
    Seg& sg = ws.segs[S][si];
    if (sg.kind == KIND_IDENT) continue;
    const MapP mp = map_of(sg, k);
    const uint64_t beg = sg.start + (uint64_t)ci * ch;
    const uint64_t end = min(beg + ch, sg.start + sg.count);
    for (int b = t; b < k; b += kBlock) sm.h[b] = 0;
    __syncthreads();
    for (uint64_t i = beg + t; i < end; i += kBlock) atomicAdd(&sm.h[bucket_of(x[i], mp)], 1u);
    __syncthreads();
    const uint32_t nch = sg.nchunks;
    if (nch > 1) {
      uint64_t* st0 = ws.status + (uint64_t)sg.status_base * (uint64_t)k;
      uint64_t* st = st0 + (uint64_t)ci * (uint64_t)k;
      if (ci == 0) {
        for (int b = t; b < k; b += kBlock) st_publish(st + b, tag, FL_INC, sm.h[b]);
      } else {
        const bool lastc = ci == nch - 1;
        if (!lastc)
          for (int b = t; b < k; b += kBlock) st_publish(st + b, tag, FL_AGG, sm.h[b]);
        for (int b = t; b < k; b += kBlock) {
          uint64_t excl = 0;
          int j = (int)ci - 1;
          uint32_t spins = 0;
          while (true) {
            const uint64_t wv = __hip_atomic_load(st0 + (uint64_t)j * (uint64_t)k + b,
                                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t wt = (uint32_t)(wv >> 42), wf = (uint32_t)(wv >> 40) & 3u;
            if (wt != tag || wf == 0) {
              if (++spins > kSpinLimit) { atomicOr(&c->error, ERR_SPIN); break; }
              __builtin_amdgcn_s_sleep(1);
              continue;
            }
            excl += wv & kValMask;
            if (wf == FL_INC) break;
            --j;
          }
          const uint64_t inc = excl + sm.h[b];
          if (!lastc) st_publish(st + b, tag, FL_INC, inc);
          else sm.h[b] = (uint32_t)inc;  // totals of the segment
        }
      }
    }
    __syncthreads();
    if (ci == nch - 1) classify<KMAX>(ws, sm, sg, si, L);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// scatter: stable, key + payload, through an LDS-staged tile
// ---------------------------------------------------------------------------
template <int KMAX, int PW, int ROUNDS>
struct ScatSmem {
  static constexpr int T = kBlock * ROUNDS;
  uint32_t cnt[kWaves][KMAX];   // per-wave counts -> per-wave exclusive prefix
  uint32_t tst[KMAX];           // tile exclusive starts
  uint64_t gbase[KMAX];         // running destination of each cluster
  uint64_t skey[T];
  typename PayT<PW>::T spay[PW ? T : 1];
  uint16_t sbk[T];
  uint32_t sh[kWaves + 2];
};

template <int KMAX, int KBITS, int PW, int ROUNDS>
__global__ void __launch_bounds__(kBlock) k_scatter(Ws ws, int L) {
  using P = typename PayT<PW>::T;
  using Sm = ScatSmem<KMAX, PW, ROUNDS>;
  constexpr int T = Sm::T;
  __shared__ Sm sm;
  Ctl* c = ws.ctl;
  if (call_failed(c)) return;
  const int S = L & 1, N = S ^ 1;
  const uint32_t nw = min(c->nwork[S], ws.work_cap);
  const int k = ws.p.k;
  const uint64_t ch = (uint64_t)ws.p.chunk;
  const uint64_t* __restrict__ xin = ws.keys[S];
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

  for (uint32_t w0 = 0; w0 < nw; w0 += G) {
    const uint32_t w = w0 + slot;
    if (w >= nw) continue;
    const uint64_t item = ws.work[S][w];
    const uint32_t si = (uint32_t)(item >> 32), ci = (uint32_t)item;
    const Seg& sg = ws.segs[S][si];
    if (sg.kind == KIND_IDENT) continue;
    const MapP mp = map_of(sg, k);
    const uint64_t beg = sg.start + (uint64_t)ci * ch;
    const uint64_t end = min(beg + ch, sg.start + sg.count);
    const uint32_t* gb = ws.bstart + (uint64_t)si * (uint64_t)k;
    const uint64_t* stp = (ci > 0) ? ws.status + (uint64_t)(sg.status_base + ci - 1) * (uint64_t)k : nullptr;
    for (int b = t; b < k; b += kBlock) {
      uint64_t base = sg.start + gb[b];
      if (stp) base += stp[b] & kValMask;
      sm.gbase[b] = base;
    }
    for (uint64_t tb = beg; tb < end; tb += T) {
      const uint32_t tn = (uint32_t)min((uint64_t)T, end - tb);
      for (int b = ln; b < k; b += kWave) sm.cnt[wv][b] = 0;
      __syncthreads();
      uint64_t key[ROUNDS];
      P pay[ROUNDS];
      uint32_t bk[ROUNDS], rk[ROUNDS];
#pragma unroll
      for (int r = 0; r < ROUNDS; ++r) {
        const uint32_t i = wv * (kWave * ROUNDS) + r * kWave + ln;
        const bool valid = i < tn;
        key[r] = valid ? xin[tb + i] : 0ull;
        pay[r] = valid ? pay_load<PW>(pin, tb + i) : (P)0;
      }
#pragma unroll
      for (int r = 0; r < ROUNDS; ++r) {
        const uint32_t i = wv * (kWave * ROUNDS) + r * kWave + ln;
        const bool valid = i < tn;
        const uint32_t b = valid ? bucket_of(key[r], mp) : 0u;
        const uint64_t act = __ballot(valid);
        const uint64_t m = match_digit<KBITS>(b, act);
        const uint32_t before = below(m);
        uint32_t base = 0;
        if (valid) base = sm.cnt[wv][b];
        if (valid && before == 0) sm.cnt[wv][b] = base + (uint32_t)__popcll(m);
        bk[r] = b;
        rk[r] = base + before;
      }
      __syncthreads();
      // per cluster: exclusive prefix over waves, tile count
      for (int b = t; b < k; b += kBlock) {
        uint32_t run = 0;
#pragma unroll
        for (int q = 0; q < kWaves; ++q) {
          const uint32_t v = sm.cnt[q][b];
          sm.cnt[q][b] = run;
          run += v;
        }
        sm.tst[b] = run;
      }
      __syncthreads();
      block_scan_lds(sm.tst, k, sm.sh);
      // stage in cluster order
#pragma unroll
      for (int r = 0; r < ROUNDS; ++r) {
        const uint32_t i = wv * (kWave * ROUNDS) + r * kWave + ln;
        if (i < tn) {
          const uint32_t b = bk[r];
          const uint32_t pos = min(sm.tst[b] + sm.cnt[wv][b] + rk[r], (uint32_t)T - 1);
          sm.skey[pos] = key[r];
          if constexpr (PW != 0) sm.spay[pos] = pay[r];
          sm.sbk[pos] = (uint16_t)b;
        }
      }
      __syncthreads();
      const uint64_t seg_end = sg.start + sg.count;
      for (uint32_t p = t; p < tn; p += kBlock) {
        const uint32_t b = sm.sbk[p];
        const uint64_t dst = sm.gbase[b] + (p - sm.tst[b]);
        if (dst < sg.start || dst >= seg_end) {  // never taken when the counts are right
          atomicOr(&c->error, ERR_SCATTER);
          continue;
        }
        xout[dst] = sm.skey[p];
        if constexpr (PW != 0) pay_store<PW>(pout, dst, sm.spay[p]);
      }
      __syncthreads();
      // advance the running destinations by this tile's counts
      for (int b = t; b < k; b += kBlock) {
        const uint32_t nxt = (b + 1 < k) ? sm.tst[b + 1] : tn;
        sm.gbase[b] += nxt - sm.tst[b];
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// local sort: one workgroup per leaf group (< 2*cutoff <= 4096 keys), stable
// LSD radix on the key's offset from the group minimum, 8-bit digits, only
// as many passes as the group's range needs
// ---------------------------------------------------------------------------
template <int PW>
struct LocSmem {
  static constexpr int R = kLocalCap / kBlock;  // rounds per wave (16)
  uint32_t cnt[kWaves][256];
  uint32_t tot[256];
  uint64_t skey[kLocalCap];
  typename PayT<PW>::T spay[PW ? kLocalCap : 1];
  uint64_t rmin[kWaves], rmax[kWaves];
  uint32_t sh[kWaves + 2];
};

template <int PW>
__global__ void __launch_bounds__(kBlock) k_local(Ws ws, int L) {
  using P = typename PayT<PW>::T;
  using Sm = LocSmem<PW>;
  constexpr int R = Sm::R;
  __shared__ Sm sm;
  Ctl* c = ws.ctl;
  if (call_failed(c)) return;
  const int S = L & 1;
  const uint32_t nl = min(c->nleaf[S], ws.leaf_cap);
  uint64_t* __restrict__ dst = ws.keys[0];
  void* pdst = ws.pay[0];
  const uint32_t wv = wave(), ln = lane();
  const int t = threadIdx.x;

  for (uint32_t g = blockIdx.x; g < nl; g += gridDim.x) {
    const Leaf lf = ws.leaves[S][g];
    const uint64_t* __restrict__ src = ws.keys[lf.src];
    const void* psrc = ws.pay[lf.src];
    const uint32_t n = lf.count;
    if ((lf.flags & LF_COPY) || n <= 1 || n > (uint32_t)kLocalCap) {
      if (lf.src != 0)
        for (uint32_t i = t; i < n; i += kBlock) {
          dst[lf.start + i] = src[lf.start + i];
          if constexpr (PW != 0) pay_store<PW>(pdst, lf.start + i, pay_load<PW>(psrc, lf.start + i));
        }
      if (!(lf.flags & LF_COPY) && n > (uint32_t)kLocalCap && t == 0)
        atomicOr(&c->error, ERR_LEAFCAP);
      continue;
    }
    uint64_t key[R];
    P pay[R];
    uint64_t mn = ~0ull, mx = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t i = wv * (kWave * R) + r * kWave + ln;
      const bool valid = i < n;
      key[r] = valid ? src[lf.start + i] : 0ull;
      pay[r] = valid ? pay_load<PW>(psrc, lf.start + i) : (P)0;
      if (valid) { mn = key[r] < mn ? key[r] : mn; mx = key[r] > mx ? key[r] : mx; }
    }
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
      uint64_t a = __shfl_xor(mn, o), b = __shfl_xor(mx, o);
      mn = a < mn ? a : mn;
      mx = b > mx ? b : mx;
    }
    if (ln == 0) { sm.rmin[wv] = mn; sm.rmax[wv] = mx; }
    __syncthreads();
    mn = sm.rmin[0]; mx = sm.rmax[0];
    for (int q = 1; q < kWaves; ++q) {
      mn = sm.rmin[q] < mn ? sm.rmin[q] : mn;
      mx = sm.rmax[q] > mx ? sm.rmax[q] : mx;
    }
    __syncthreads();
    const uint64_t range = mx - mn;
    const int bits = range ? 64 - __clzll((long long)range) : 0;
    const int passes = (bits + 7) / 8;
    for (int ps = 0; ps < passes; ++ps) {
      const int sh = ps * 8;
      for (int b = ln; b < 256; b += kWave) sm.cnt[wv][b] = 0;
      __syncthreads();
      uint32_t dg[R], rk[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const uint32_t i = wv * (kWave * R) + r * kWave + ln;
        const bool valid = i < n;
        const uint32_t d = valid ? (uint32_t)(((key[r] - mn) >> sh) & 255u) : 0u;
        const uint64_t act = __ballot(valid);
        const uint64_t m = match_digit<8>(d, act);
        const uint32_t before = below(m);
        uint32_t base = 0;
        if (valid) base = sm.cnt[wv][d];
        if (valid && before == 0) sm.cnt[wv][d] = base + (uint32_t)__popcll(m);
        dg[r] = d;
        rk[r] = base + before;
      }
      __syncthreads();
      {
        const int b = t;  // 256 digits, one per thread
        uint32_t run = 0;
#pragma unroll
        for (int q = 0; q < kWaves; ++q) {
          const uint32_t v = sm.cnt[q][b];
          sm.cnt[q][b] = run;
          run += v;
        }
        sm.tot[b] = run;
      }
      __syncthreads();
      block_scan_lds(sm.tot, 256, sm.sh);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const uint32_t i = wv * (kWave * R) + r * kWave + ln;
        if (i < n) {
          const uint32_t pos = min(sm.tot[dg[r]] + sm.cnt[wv][dg[r]] + rk[r], (uint32_t)kLocalCap - 1);
          sm.skey[pos] = key[r];
          if constexpr (PW != 0) sm.spay[pos] = pay[r];
        }
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const uint32_t i = wv * (kWave * R) + r * kWave + ln;
        if (i < n) {
          key[r] = sm.skey[i];
          if constexpr (PW != 0) pay[r] = sm.spay[i];
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t i = wv * (kWave * R) + r * kWave + ln;
      if (i < n) {
        dst[lf.start + i] = key[r];
        if constexpr (PW != 0) pay_store<PW>(pdst, lf.start + i, pay[r]);
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
struct Grids {
  int moments, hist, scatter, local;
};

template <int KMAX, int KBITS, int PW, int ROUNDS>
static hipError_t launch_levels_t(const Ws& ws, int levels, const Grids& g, bool with_local,
                                  hipStream_t st) {
  for (int L = 0; L < levels; ++L) {
    hipLaunchKernelGGL(k_moments, dim3(g.moments), dim3(kBlock), 0, st, ws, L);
    hipLaunchKernelGGL((k_hist<KMAX>), dim3(g.hist), dim3(kBlock), 0, st, ws, L);
    hipLaunchKernelGGL((k_scatter<KMAX, KBITS, PW, ROUNDS>), dim3(g.scatter), dim3(kBlock), 0, st, ws, L);
    if (with_local) hipLaunchKernelGGL((k_local<PW>), dim3(g.local), dim3(kBlock), 0, st, ws, L);
  }
  return hipGetLastError();
}

}  // namespace zs

// entry points used by the host planner (zsort_api.cpp)
namespace zs {

hipError_t launch_reset(const Ws& ws, hipStream_t st) {
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, st, ws);
  return hipGetLastError();
}

hipError_t launch_init_single(const Ws& ws, uint64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_init_single, dim3(64), dim3(kBlock), 0, st, ws, n);
  return hipGetLastError();
}

hipError_t launch_init_segments(const Ws& ws, const int64_t* off, int32_t nseg, uint64_t n,
                                hipStream_t st) {
  const int blocks = (nseg + kBlock) / kBlock + 1;
  hipLaunchKernelGGL(k_check_offsets, dim3(blocks), dim3(kBlock), 0, st, ws, off, nseg, n);
  hipLaunchKernelGGL(k_init_segments, dim3(blocks), dim3(kBlock), 0, st, ws, off, nseg);
  return hipGetLastError();
}

hipError_t launch_levels(const Ws& ws, int levels, int grid, bool with_local, hipStream_t st) {
  Grids g{grid, grid, grid, grid};
  const int k = ws.p.k;
  const int pw = ws.p.pw;
#define ZS_DISPATCH(KM, KB)                                                                \
  if (k <= KM) {                                                                           \
    if (pw == 0) return launch_levels_t<KM, KB, 0, 8>(ws, levels, g, with_local, st);     \
    if (pw == 4) return launch_levels_t<KM, KB, 4, 8>(ws, levels, g, with_local, st);     \
    return launch_levels_t<KM, KB, 8, 8>(ws, levels, g, with_local, st);                   \
  }
  ZS_DISPATCH(1024, 10)
  ZS_DISPATCH(4096, 12)
#undef ZS_DISPATCH
  return hipErrorInvalidValue;
}

}  // namespace zs
