// zsort_learned.hip -- HIP kernels (gfx950) of the learned partition map
// that can replace the z-score map of zSort's first distribution pass.
//
// zSort's first pass needs a non-decreasing map from keys to clusters
// (Section III; Eq. (1) is one such map, built from the mean and the
// standard deviation).  Here the map is a monotone MLP fitted to the
// empirical CDF of a 1 % key sample:
//   sample   -- one key from each stride of `stride` keys, at an offset drawn
//               by SplitMix64 (Steele, Lea, Flood, OOPSLA 2014) from a seed;
//   targets  -- the sample is sorted by the plain path; key i's target is its
//               mid-rank (#{< x} + #{<= x}) / (2m), its input the normalised key;
//   init     -- the sorted sample is cut into 28 blocks of equal count, the
//               blocks with the widest internal gaps are cut again at the
//               gap; each piece becomes one ramp of the first layer,
//               weighed by its share of the sample: the sample CDF, linear
//               inside a piece and flat across the gaps between pieces;
//   training -- Adam (Kingma, Ba, ICLR 2015) on the mean squared error over
//               fixed minibatches, weights projected onto >= 0 after each
//               step; the gradient of a step is reduced in one fixed order
//               (per-workgroup partial sums, then the partials in workgroup
//               order), so training is deterministic; the trained
//               parameters are kept only if they do not enlarge the largest
//               cluster of the sample;
//   compile  -- for b = 1..nt the threshold t_b, the least key whose cluster
//               is >= b, by bisection over the 64-bit keys; the first pass
//               then finds a key's cluster by binary search in LDS;
//   check    -- max(cluster j) <= min(every later cluster) is verified on
//               the device (sorted thresholds imply it; with per-key
//               inference the first pass's output is scanned); the caller
//               falls back to the z-score map when it fails.
#include <hip/hip_runtime.h>
#include <math.h>

#include "zsort_internal.h"
#include "zsort_mlp.h"

namespace zs {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// ---------------------------------------------------------------------------
// sample: out[i] = x[i * stride + (splitmix64(seed + (i + 1) * gamma) mod stride)]
// for i < m = floor(n / stride), so every read stays below m * stride <= n
// ---------------------------------------------------------------------------
__global__ void k_lsample(const uint64_t* __restrict__ x, uint64_t m, uint32_t stride,
                          uint64_t seed, uint64_t* __restrict__ out) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < m;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t z = splitmix64(seed + (i + 1) * kGamma);
    out[i] = x[i * stride + z % stride];
  }
}

// ---------------------------------------------------------------------------
// targets and inputs from the sorted sample s[0, m)
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t lower_bound_u64(const uint64_t* s, uint64_t m, uint64_t v) {
  uint64_t lo = 0, hi = m;
  while (lo < hi) {
    const uint64_t mid = (lo + hi) >> 1;
    if (s[mid] < v) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ uint64_t upper_bound_u64(const uint64_t* s, uint64_t m, uint64_t v) {
  uint64_t lo = 0, hi = m;
  while (lo < hi) {
    const uint64_t mid = (lo + hi) >> 1;
    if (s[mid] <= v) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__global__ void k_lprep(const uint64_t* __restrict__ s, uint64_t m, double* __restrict__ U,
                        float* __restrict__ Y, LRes* res) {
  const uint64_t smin = s[0], smax = s[m - 1];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    res->smin = smin;
    res->smax = smax;
  }
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < m;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t v = s[i];
    const uint64_t lt = lower_bound_u64(s, m, v), le = upper_bound_u64(s, m, v);
    Y[i] = __double2float_rn(__ddiv_rn((double)(lt + le), 2.0 * (double)m));
    U[i] = mlp_norm(v, smin, smax);
  }
}

// caller-given normalisation range
__global__ void k_lset_range(LRes* res, uint64_t smin, uint64_t smax) {
  if (threadIdx.x == 0) {
    res->smin = smin;
    res->smax = smax;
  }
}

// Initialisation from the sorted sample (one workgroup of kBlock threads).
// The sample is cut into kNBlk blocks of equal count; a block whose largest
// gap between consecutive keys covers more than half of its key range is
// cut there (at most kNSplit blocks, largest gap-to-range ratio first, ties
// to the lower block).  Piece r of consecutive keys [a, b] becomes ramp r of
// the first layer (0 at u[a], 1 at u[b]; a step when u[a] == u[b]), passed
// through by the second layer and weighed by its share (b - a + 1) / m in
// the output: the sample CDF, linear inside a piece, flat between pieces.
constexpr int kNBlk = 28, kNSplit = 4;
static_assert(kNBlk == sizeof(LRes::iscore) / sizeof(double), "block count");

__device__ __forceinline__ void init_block_range(uint64_t i, uint64_t m, uint64_t& a, uint64_t& b) {
  a = (i * m) / kNBlk;
  b = ((i + 1) * m) / kNBlk;
}

// one workgroup per sample block: the block's largest gap (first position
// on ties) relative to its key range
__global__ void __launch_bounds__(kBlock) k_linit_gaps(const uint64_t* __restrict__ s, uint64_t m,
                                                       LRes* res) {
  __shared__ double rv[kWaves];
  __shared__ uint64_t rj[kWaves];
  const int t = threadIdx.x, i = blockIdx.x;
  const uint64_t smin = s[0], smax = s[m - 1];
  uint64_t a, b;
  init_block_range((uint64_t)i, m, a, b);
  double span = 0.0;
  if (b - a >= 2) span = __dsub_rn(mlp_norm(s[b - 1], smin, smax), mlp_norm(s[a], smin, smax));
  if (!(span > 0.0)) {
    if (t == 0) {
      res->iscore[i] = 0.0;
      res->icut[i] = 0;
    }
    return;
  }
  double best = -1.0;
  uint64_t bj = 0;
  for (uint64_t j = a + t; j + 1 < b; j += kBlock) {
    const double g = __dsub_rn(mlp_norm(s[j + 1], smin, smax), mlp_norm(s[j], smin, smax));
    if (g > best) {
      best = g;
      bj = j;
    }
  }
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    const double ov = __shfl_xor(best, o);
    const uint64_t oj = __shfl_xor(bj, o);
    if (ov > best || (ov == best && oj < bj)) {
      best = ov;
      bj = oj;
    }
  }
  if ((t & (kWave - 1)) == 0) {
    rv[t / kWave] = best;
    rj[t / kWave] = bj;
  }
  __syncthreads();
  if (t == 0) {
    for (int w = 1; w < kWaves; ++w)
      if (rv[w] > best || (rv[w] == best && rj[w] < bj)) {
        best = rv[w];
        bj = rj[w];
      }
    res->iscore[i] = __ddiv_rn(best, span);
    res->icut[i] = bj;
  }
}

// the pieces and the parameters (one workgroup)
__global__ void k_linit(const uint64_t* __restrict__ s, uint64_t m, const LRes* res,
                        MlpP* __restrict__ par) {
  const int t = threadIdx.x;
  uint32_t* z = reinterpret_cast<uint32_t*>(par);
  for (uint32_t i = t; i < sizeof(MlpP) / 4; i += blockDim.x) z[i] = 0u;
  __syncthreads();
  if (t != 0) return;
  const uint64_t smin = s[0], smax = s[m - 1];
  bool split[kNBlk];
  for (int i = 0; i < kNBlk; ++i) split[i] = false;
  for (int k = 0; k < kNSplit; ++k) {
    int bi = -1;
    for (int i = 0; i < kNBlk; ++i)
      if (!split[i] && res->iscore[i] > 0.5 && (bi < 0 || res->iscore[i] > res->iscore[bi])) bi = i;
    if (bi < 0) break;
    split[bi] = true;
  }
  int r = 0;
  for (int i = 0; i < kNBlk; ++i) {
    uint64_t a, b;
    init_block_range((uint64_t)i, m, a, b);
    if (a == b) continue;
    const int np = split[i] ? 2 : 1;
    for (int q = 0; q < np; ++q, ++r) {
      const uint64_t pa = (split[i] && q == 1) ? res->icut[i] + 1 : a;
      const uint64_t pb = (split[i] && q == 0) ? res->icut[i] : b - 1;
      const double ua = mlp_norm(s[pa], smin, smax), ub = mlp_norm(s[pb], smin, smax);
      const double w = ub > ua ? __ddiv_rn(1.0, __dsub_rn(ub, ua)) : 4503599627370496.0;  // 2^52
      par->w1[r] = w;
      par->b1[r] = __dmul_rn(-ua, w);
      par->w2[r * kH + r] = 1.0f;
      par->w3[r] = __double2float_rn(__ddiv_rn(__ull2double_rn(pb - pa + 1), __ull2double_rn(m)));
    }
  }
}

// Adam state reset: first and second moments, running powers of the decays
__global__ void k_ladam_reset(double* __restrict__ adam, LRes* res) {
  for (int i = threadIdx.x; i < 2 * kNP; i += blockDim.x) adam[i] = 0.0;
  if (threadIdx.x == 0) {
    res->ticket = 0;
    res->steps_done = 0;
    res->loss_first = res->loss_last = 0.0;
    res->fail = 0;
    res->maxc = 0;
    res->trained = 0;
    res->smax_init = res->smax_trained = 0;
  }
}

// ---------------------------------------------------------------------------
// gradient of one training step over minibatch j = step mod nb (samples
// i = j, j + nb, ...): each workgroup writes the sums over its 256 samples
// ---------------------------------------------------------------------------
constexpr int kTB = 256;          // samples per workgroup
constexpr int kRow = kTB + 1;     // padded row of the reduction matrix
constexpr int kPartW = kNP + 1;   // partial record: gradient, then loss

struct TrainSmem {
  MlpP par;
  float rows[2 * kH + 2][kRow];   // one column per sample of the workgroup
};

constexpr double kBeta1 = 0.9, kBeta2 = 0.999, kAdamEps = 1e-8;

__device__ __forceinline__ bool is_weight(int i) {
  return (i >= kW1 && i < kB1) || (i >= kW2 && i < kB2) || (i >= kW3 && i < kB3);
}

__global__ void __launch_bounds__(kTB) k_ltrain(const double* __restrict__ U,
                                                const float* __restrict__ Y, uint64_t m,
                                                uint32_t nb, uint32_t step,
                                                const MlpP* __restrict__ par,
                                                float* __restrict__ part) {
  __shared__ TrainSmem sm;
  const int t = threadIdx.x;
  const uint32_t j = step % nb;
  const uint64_t cnt = m > j ? (m - j + nb - 1) / nb : 0;
  mlp_load(sm.par, par);
  __syncthreads();
  const MlpP& p = sm.par;

  const uint64_t q = (uint64_t)blockIdx.x * kTB + t;
  const bool valid = q < cnt;
  const double u = valid ? U[j + q * nb] : 0.0;
  const float y = valid ? Y[j + q * nb] : 0.0f;

  // forward, keeping what the backward pass needs: h1 goes to LDS (row i,
  // column t) for the reduction, h2 stays in registers
  float h2[kH];
  uint32_t m1 = 0, m2 = 0;
  {
    float h1[kH];
#pragma unroll
    for (int i = 0; i < kH; ++i) {
      double a = __dmul_rn(p.w1[i], u);
      a = __dadd_rn(a, p.b1[i]);
      m1 |= (a > 0.0 && a < 1.0) ? (1u << i) : 0u;
      h1[i] = clamp01(__double2float_rn(a));
      sm.rows[i][t] = h1[i];
    }
#pragma unroll
    for (int jj = 0; jj < kH; ++jj) {
      float acc = p.b2[jj];
#pragma unroll
      for (int i = 0; i < kH; ++i) acc = __fadd_rn(acc, __fmul_rn(p.w2[jj * kH + i], h1[i]));
      m2 |= (acc > 0.0f && acc < 1.0f) ? (1u << jj) : 0u;
      h2[jj] = clamp01(acc);
    }
  }
  float f = p.b3;
#pragma unroll
  for (int jj = 0; jj < kH; ++jj) f = __fadd_rn(f, __fmul_rn(p.w3[jj], h2[jj]));
  const float r = f - y;
  const float fc = (float)(cnt ? cnt : 1);
  const float e = valid ? 2.0f * r / fc : 0.0f;       // d(loss)/d(f) of this sample
  const float lc = valid ? r * r / fc : 0.0f;

  // backward: d2 = e * W3 on live units of layer 2 (to LDS rows 32..63),
  // d1 = W2^T d2 on live units of layer 1 (registers)
#pragma unroll
  for (int jj = 0; jj < kH; ++jj) sm.rows[kH + jj][t] = ((m2 >> jj) & 1u) ? e * p.w3[jj] : 0.0f;
  float d1[kH];
#pragma unroll
  for (int i = 0; i < kH; ++i) d1[i] = 0.0f;
#pragma unroll 1
  for (int jj = 0; jj < kH; ++jj) {
    const float d2j = sm.rows[kH + jj][t];
#pragma unroll
    for (int i = 0; i < kH; ++i) d1[i] = __fadd_rn(d1[i], __fmul_rn(d2j, p.w2[jj * kH + i]));
  }
#pragma unroll
  for (int i = 0; i < kH; ++i) d1[i] = ((m1 >> i) & 1u) ? d1[i] : 0.0f;

  float* out = part + (uint64_t)blockIdx.x * kPartW;
  // phase A: rows 0..31 = h1, rows 32..63 = d2 -> W2 (outer products), b2
  __syncthreads();
  for (int ent = t; ent < kH * kH; ent += kTB) {
    const int jj = ent / kH, i = ent % kH;
    float acc = 0.0f;
    for (int s = 0; s < kTB; ++s) acc = __fadd_rn(acc, __fmul_rn(sm.rows[kH + jj][s], sm.rows[i][s]));
    out[kW2 + ent] = acc;
  }
  if (t < kH) {
    float acc = 0.0f;
    for (int s = 0; s < kTB; ++s) acc = __fadd_rn(acc, sm.rows[kH + t][s]);
    out[kB2 + t] = acc;
  }
  __syncthreads();
  // phase B: rows 0..31 = e * h2 (W3), rows 32..63 = d1 (b1), row 64 = e (b3), row 65 = loss
  // phase C reuses rows 0..31 for d1 * u (W1)
#pragma unroll
  for (int i = 0; i < kH; ++i) {
    sm.rows[i][t] = e * h2[i];
    sm.rows[kH + i][t] = d1[i];
  }
  sm.rows[2 * kH][t] = e;
  sm.rows[2 * kH + 1][t] = lc;
  __syncthreads();
  if (t < 2 * kH + 2) {
    float acc = 0.0f;
    for (int s = 0; s < kTB; ++s) acc = __fadd_rn(acc, sm.rows[t][s]);
    const int dst = t < kH ? kW3 + t : (t < 2 * kH ? kB1 + (t - kH) : (t == 2 * kH ? kB3 : kNP));
    out[dst] = acc;
  }
  __syncthreads();
  const float uf = __double2float_rn(u);
#pragma unroll
  for (int i = 0; i < kH; ++i) sm.rows[i][t] = d1[i] * uf;
  __syncthreads();
  if (t < kH) {
    float acc = 0.0f;
    for (int s = 0; s < kTB; ++s) acc = __fadd_rn(acc, sm.rows[t][s]);
    out[kW1 + t] = acc;
  }

}

// Sums the partials of the G workgroups of a step in workgroup order (one
// thread per parameter, binary64), then mode 0: Adam step with projection
// (b1p, b2p: beta1^(step+1), beta2^(step+1), by repeated products on the
// host); mode 1: the gradient and the loss into gout.
__global__ void __launch_bounds__(64) k_lreduce(const float* __restrict__ part, uint32_t G,
                                                MlpP* par, double* adam, LRes* res, double lr,
                                                double b1p, double b2p, uint32_t step, int mode,
                                                double* gout) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  if (i >= kPartW) return;
  double g = 0.0;
  uint32_t b = 0;
  for (; b + 8 <= G; b += 8) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[(uint64_t)(b + u) * kPartW + i];
#pragma unroll
    for (int u = 0; u < 8; ++u) g = __dadd_rn(g, (double)v[u]);
  }
  for (; b < G; ++b) g = __dadd_rn(g, (double)part[(uint64_t)b * kPartW + i]);
  if (mode == 1) {
    gout[i] = g;
    return;
  }
  if (i == kNP) {  // the batch loss (before this step's update)
    if (step == 0) res->loss_first = g;
    res->loss_last = g;
    res->steps_done = res->steps_done + 1;
    return;
  }
  double m1v = adam[i], m2v = adam[kNP + i];
  m1v = __dadd_rn(__dmul_rn(kBeta1, m1v), __dmul_rn(1.0 - kBeta1, g));
  m2v = __dadd_rn(__dmul_rn(kBeta2, m2v), __dmul_rn(1.0 - kBeta2, __dmul_rn(g, g)));
  adam[i] = m1v;
  adam[kNP + i] = m2v;
  const double mh = __ddiv_rn(m1v, 1.0 - b1p);
  const double vh = __ddiv_rn(m2v, 1.0 - b2p);
  // parameter i: binary64 in the first layer, binary32 after it
  double* pd = i < kB1 ? &par->w1[i] : (i < kW2 ? &par->b1[i - kB1] : nullptr);
  float* pf = i < kW2 ? nullptr
                      : (i < kB2 ? &par->w2[i - kW2]
                                 : (i < kW3 ? &par->b2[i - kB2]
                                            : (i < kB3 ? &par->w3[i - kW3] : &par->b3)));
  const double cur = pd ? *pd : (double)*pf;
  double pn = __dsub_rn(cur, __ddiv_rn(__dmul_rn(lr, mh), __dadd_rn(sqrt(vh), kAdamEps)));
  if (is_weight(i) && !(pn > 0.0)) pn = 0.0;   // projection onto W >= 0
  if (pd) *pd = pn;
  else *pf = __double2float_rn(pn);
}

// ---------------------------------------------------------------------------
// thresholds: t_b = min{x : cluster(x) >= b}, b = 1..nt, nt = cluster(2^64 - 1).
// A 65-way search by one wave per threshold: its 64 lanes evaluate 64 points
// that cut [lo, hi] into 65 parts, and the first point whose cluster is >= b
// bounds the next interval -- about 11 rounds instead of 64 bisection steps,
// with a wave per threshold so that the LDS reads of the weights overlap
// across many waves.  For a non-decreasing map the least such key is unique,
// so any exact search finds the same t_b.
// ---------------------------------------------------------------------------
constexpr int kTLanes = kWave;
constexpr uint64_t kTParts = kTLanes + 1;

__device__ __forceinline__ uint64_t tpoint(uint64_t lo, uint64_t d, uint32_t j) {
  // lo + floor(d * j / 65) without 128-bit arithmetic (j <= 64)
  const uint64_t q = d / kTParts, r = d % kTParts;
  return lo + q * j + (r * j) / kTParts;
}

__global__ void __launch_bounds__(256) k_lthresh(const MlpP* __restrict__ par, int B, LRes* res,
                                                 uint64_t* __restrict__ thr) {
  __shared__ MlpP sp;
  mlp_load(sp, par);
  __syncthreads();
  const uint64_t smin = res->smin, smax = res->smax;
  const uint32_t nt = mlp_cluster(sp, ~0ull, smin, smax, B);
  if (blockIdx.x == 0 && threadIdx.x == 0) res->nt = nt;
  const uint32_t j = (threadIdx.x & (kWave - 1)) + 1;   // point j of 1..64
  const uint32_t wid = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const uint32_t nwaves = gridDim.x * blockDim.x / kWave;
  for (uint32_t b = wid + 1; b < (uint32_t)B; b += nwaves) {   // this wave's threshold
    if (b > nt) {
      if (j == 1) thr[b - 1] = 0;
      continue;
    }
    uint64_t lo = 0, hi = ~0ull;                  // the answer lies in [lo, hi]
    while (lo < hi) {
      const uint64_t d = hi - lo;
      const uint64_t p = tpoint(lo, d, j);
      const uint64_t mask = __ballot(mlp_cluster(sp, p, smin, smax, B) >= b);
      if (mask) {
        const uint32_t js = (uint32_t)__ffsll((unsigned long long)mask);   // first point (1-based)
        const uint64_t nhi = tpoint(lo, d, js);
        if (js > 1) lo = tpoint(lo, d, js - 1) + 1;
        hi = nhi;
      } else {
        lo = tpoint(lo, d, kTLanes) + 1;
      }
    }
    if (j == 1) thr[b - 1] = lo;
  }
}

// per-key inference (tests and the direct mode's reference): f and the cluster
__global__ void __launch_bounds__(256) k_lforward(const MlpP* __restrict__ par,
                                                  const uint64_t* __restrict__ x, uint64_t q,
                                                  const LRes* res, int B, float* __restrict__ fout,
                                                  uint32_t* __restrict__ cout) {
  __shared__ MlpP sp;
  mlp_load(sp, par);
  __syncthreads();
  const uint64_t smin = res->smin, smax = res->smax;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < q;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const float f = mlp_forward(sp, mlp_norm(x[i], smin, smax));
    if (fout) fout[i] = f;
    if (cout) cout[i] = mlp_cluster_of_f(f, B);
  }
}

// cluster sizes of the sample (inputs U) under parameters par, B clusters,
// by direct inference; counts must start at zero
__global__ void __launch_bounds__(kBlock) k_lhist_sample(const double* __restrict__ U, uint64_t m,
                                                         const MlpP* __restrict__ par, int B,
                                                         uint32_t* __restrict__ counts) {
  __shared__ MlpP sp;
  __shared__ uint32_t h[kKMax];
  mlp_load(sp, par);
  for (int b = threadIdx.x; b < B; b += kBlock) h[b] = 0;
  __syncthreads();
  for (uint64_t i = blockIdx.x * (uint64_t)kBlock + threadIdx.x; i < m;
       i += (uint64_t)gridDim.x * kBlock)
    atomicAdd(&h[mlp_cluster_of_f(mlp_forward(sp, U[i]), B)], 1u);
  __syncthreads();
  for (int b = threadIdx.x; b < B; b += kBlock)
    if (h[b]) atomicAdd(&counts[b], h[b]);
}

// Keeps the trained parameters only if they do not enlarge the sample's
// largest cluster (hc0: initial, hc1: trained; ties go to the lower loss on
// minibatch 0, g0/g1 holding that loss in their last word); otherwise
// restores the initial ones.  The squared error the steps minimise follows
// the CDF's values, not its slope, so a step can lower it while leaving a
// flat stretch that fills one cluster.
__global__ void __launch_bounds__(kBlock) k_lkeep(MlpP* __restrict__ par,
                                                  const MlpP* __restrict__ par0,
                                                  const double* __restrict__ g0,
                                                  const double* __restrict__ g1,
                                                  const uint32_t* __restrict__ hc0,
                                                  const uint32_t* __restrict__ hc1, int B,
                                                  LRes* res) {
  __shared__ uint32_t mx[2];
  __shared__ uint32_t keep_s;
  if (threadIdx.x < 2) mx[threadIdx.x] = 0;
  __syncthreads();
  uint32_t a = 0, b = 0;
  for (int i = threadIdx.x; i < B; i += kBlock) {
    a = hc0[i] > a ? hc0[i] : a;
    b = hc1[i] > b ? hc1[i] : b;
  }
  atomicMax(&mx[0], a);
  atomicMax(&mx[1], b);
  __syncthreads();
  const double l0 = g0[kNP], l1 = g1[kNP];
  if (threadIdx.x == 0) keep_s = (mx[1] < mx[0] || (mx[1] == mx[0] && l1 <= l0)) ? 1u : 0u;
  __syncthreads();
  const bool keep = keep_s != 0;
  if (!keep) {
    const uint32_t* s = reinterpret_cast<const uint32_t*>(par0);
    uint32_t* d = reinterpret_cast<uint32_t*>(par);
    for (uint32_t i = threadIdx.x; i < sizeof(MlpP) / 4; i += blockDim.x) d[i] = s[i];
  }
  if (threadIdx.x == 0) {
    res->loss_first = l0;
    res->loss_last = keep ? l1 : l0;
    res->trained = keep ? 1u : 0u;
    res->smax_init = mx[0];
    res->smax_trained = mx[1];
  }
}

// ---------------------------------------------------------------------------
// order checks.
// Thresholds: if t_1 <= t_2 <= ... <= t_nt, the cluster #{b : t_b <= x} is
// non-decreasing in x, so every key of cluster j lies below t_(j+1) and
// every key of a later cluster at or above it: max(C_j) <= min(C_j') for all
// j < j'.  The check is that the thresholds are sorted.
// Keys (per-key inference): y holds the first pass's output, cluster b at
// [bst[b], bst[b+1]) (the last one up to n); per-cluster minima and maxima
// are taken in chunks of the output and combined with 64-bit atomics.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_lthr_check(const uint64_t* __restrict__ thr,
                                                       LRes* res) {
  __shared__ uint32_t bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  const uint32_t nt = res->nt;
  uint32_t my = 0;
  for (uint32_t b = threadIdx.x; b + 1 < nt; b += kBlock)
    if (thr[b] > thr[b + 1]) my = 1;
  if (my) atomicOr(&bad, 1u);
  __syncthreads();
  if (threadIdx.x == 0) res->fail = bad;
}

__global__ void k_lminmax_init(uint64_t* __restrict__ bmin, uint64_t* __restrict__ bmax, int B) {
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < B; b += gridDim.x * blockDim.x) {
    bmin[b] = ~0ull;   // an empty cluster never sits below a later maximum
    bmax[b] = 0;
  }
}

constexpr uint64_t kCheckChunk = 16384;

__global__ void __launch_bounds__(kBlock) k_lminmax(const uint64_t* __restrict__ y,
                                                    const uint32_t* __restrict__ bst, uint64_t n,
                                                    int B, uint64_t* __restrict__ bmin,
                                                    uint64_t* __restrict__ bmax) {
  __shared__ uint64_t rmn[kWaves], rmx[kWaves];
  const int t = threadIdx.x;
  // cluster starts, clamped, so that a first pass that hit a device-side
  // limit (and left inconsistent starts) still reads inside the array
  auto start = [&](int b) -> uint64_t { return b < B ? min((uint64_t)bst[b], n) : n; };
  for (uint64_t c0 = blockIdx.x * kCheckChunk; c0 < n; c0 += gridDim.x * kCheckChunk) {
    const uint64_t c1 = min(c0 + kCheckChunk, n);
    // last cluster starting at or before c0
    int lo = 0, hi = B - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (start(mid) <= c0) lo = mid; else hi = mid - 1;
    }
    for (int b = lo; b < B && start(b) < c1; ++b) {
      const uint64_t a = max(c0, start(b));
      const uint64_t z = min(c1, max(start(b), start(b + 1)));
      if (a >= z) continue;   // uniform: every thread sees the same bounds
      uint64_t mn = ~0ull, mx = 0;
      for (uint64_t i = a + t; i < z; i += kBlock) {
        const uint64_t v = y[i];
        mn = v < mn ? v : mn;
        mx = v > mx ? v : mx;
      }
#pragma unroll
      for (int o = kWave / 2; o > 0; o >>= 1) {
        const uint64_t a2 = __shfl_xor(mn, o), b2 = __shfl_xor(mx, o);
        mn = a2 < mn ? a2 : mn;
        mx = b2 > mx ? b2 : mx;
      }
      if ((t & (kWave - 1)) == 0) {
        rmn[t / kWave] = mn;
        rmx[t / kWave] = mx;
      }
      __syncthreads();
      if (t == 0) {
        for (int w = 1; w < kWaves; ++w) {
          mn = rmn[w] < mn ? rmn[w] : mn;
          mx = rmx[w] > mx ? rmx[w] : mx;
        }
        atomicMin((unsigned long long*)&bmin[b], (unsigned long long)mn);
        atomicMax((unsigned long long*)&bmax[b], (unsigned long long)mx);
      }
      __syncthreads();
    }
  }
}

// one workgroup: fail iff some non-empty cluster's maximum exceeds the minimum
// of the clusters after it; also the largest cluster
__global__ void __launch_bounds__(kBlock) k_lcheck(const uint64_t* __restrict__ bmin,
                                                   const uint64_t* __restrict__ bmax,
                                                   const uint32_t* __restrict__ bst, uint64_t n,
                                                   int B, LRes* res) {
  __shared__ uint64_t seg_min[kBlock];
  __shared__ uint32_t bad;
  __shared__ unsigned long long maxc;
  const int t = threadIdx.x;
  const int per = (B + kBlock - 1) / kBlock;
  const int b0 = min(B, t * per), b1 = min(B, b0 + per);
  if (t == 0) {
    bad = 0;
    maxc = 0;
  }
  uint64_t mn = ~0ull;
  for (int b = b0; b < b1; ++b) mn = bmin[b] < mn ? bmin[b] : mn;
  seg_min[t] = mn;
  __syncthreads();
  uint64_t suffix = ~0ull;
  for (int w = t + 1; w < kBlock; ++w) suffix = seg_min[w] < suffix ? seg_min[w] : suffix;
  uint64_t mc = 0;
  uint32_t my_bad = 0;
  for (int b = b1 - 1; b >= b0; --b) {
    const uint64_t c = ((b + 1 < B) ? (uint64_t)bst[b + 1] : n) - bst[b];
    if (!c) continue;
    if (bmax[b] > suffix) my_bad = 1;
    suffix = bmin[b] < suffix ? bmin[b] : suffix;
    mc = c > mc ? c : mc;
  }
  if (my_bad) atomicOr(&bad, 1u);
  atomicMax(&maxc, (unsigned long long)mc);
  __syncthreads();
  if (t == 0) res->fail = bad;
}

// largest cluster of a first-pass histogram given as exclusive starts
__global__ void __launch_bounds__(kBlock) k_lmaxcount(const uint32_t* __restrict__ bst, uint64_t n,
                                                      int B, uint64_t* out) {
  __shared__ unsigned long long mx;
  if (threadIdx.x == 0) mx = 0;
  __syncthreads();
  unsigned long long m = 0;
  for (int b = threadIdx.x; b < B; b += kBlock) {
    const uint64_t c = ((b + 1 < B) ? (uint64_t)bst[b + 1] : n) - bst[b];
    m = c > m ? c : m;
  }
  atomicMax(&mx, m);
  __syncthreads();
  if (threadIdx.x == 0) *out = mx;
}

// cluster sizes of the learned map over all keys, thresholds searched in
// LDS (counts must start at zero; for the report's counts output)
__global__ void __launch_bounds__(kBlock) k_lfine_hist(const uint64_t* __restrict__ x, uint64_t n,
                                                       const uint64_t* __restrict__ thr,
                                                       const LRes* res, int B,
                                                       uint32_t* __restrict__ counts) {
  __shared__ uint64_t t[kKMax];
  __shared__ uint32_t h[kKMax];
  const uint32_t nt = min(res->nt, (uint32_t)(B - 1));
  for (uint32_t q = threadIdx.x; q < nt; q += kBlock) t[q] = thr[q];
  for (int b = threadIdx.x; b < B; b += kBlock) h[b] = 0;
  __syncthreads();
  const uint32_t top = top_pow2(nt);
  for (uint64_t i = blockIdx.x * (uint64_t)kBlock + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * kBlock)
    atomicAdd(&h[thr_cluster(t, nt, top, x[i])], 1u);
  __syncthreads();
  for (int b = threadIdx.x; b < B; b += kBlock)
    if (h[b]) atomicAdd(&counts[b], h[b]);
}

// cluster counts of the first pass (tests): counts[b] from the exclusive starts
__global__ void k_lcounts(const uint32_t* __restrict__ bst, uint64_t n, int B,
                          uint32_t* __restrict__ counts) {
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < B; b += gridDim.x * blockDim.x)
    counts[b] = (uint32_t)(((b + 1 < B) ? (uint64_t)bst[b + 1] : n) - bst[b]);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_lsample(const uint64_t* x, uint64_t m, uint32_t stride, uint64_t seed,
                          uint64_t* out, hipStream_t st) {
  const int blocks = (int)std::min<uint64_t>((m + 255) / 256, 4096);
  hipLaunchKernelGGL(k_lsample, dim3(std::max(blocks, 1)), dim3(256), 0, st, x, m, stride, seed,
                     out);
  return hipGetLastError();
}

hipError_t launch_lprep(const uint64_t* s, uint64_t m, double* U, float* Y, LRes* res,
                        hipStream_t st) {
  const int blocks = (int)std::min<uint64_t>((m + 255) / 256, 4096);
  hipLaunchKernelGGL(k_lprep, dim3(std::max(blocks, 1)), dim3(256), 0, st, s, m, U, Y, res);
  return hipGetLastError();
}

hipError_t launch_lset_range(LRes* res, uint64_t smin, uint64_t smax, hipStream_t st) {
  hipLaunchKernelGGL(k_lset_range, dim3(1), dim3(64), 0, st, res, smin, smax);
  return hipGetLastError();
}

hipError_t launch_linit(const uint64_t* s, uint64_t m, MlpP* par, LRes* res, hipStream_t st) {
  hipLaunchKernelGGL(k_linit_gaps, dim3(kNBlk), dim3(kBlock), 0, st, s, m, res);
  hipLaunchKernelGGL(k_linit, dim3(1), dim3(64), 0, st, s, m, (const LRes*)res, par);
  return hipGetLastError();
}

hipError_t launch_ladam_reset(double* adam, LRes* res, hipStream_t st) {
  hipLaunchKernelGGL(k_ladam_reset, dim3(1), dim3(256), 0, st, adam, res);
  return hipGetLastError();
}

// workgroups of a training step over minibatches of ceil(m / nb) samples
uint32_t ltrain_blocks(uint64_t m, uint32_t nb) {
  const uint64_t cnt = (m + nb - 1) / nb;
  return (uint32_t)std::max<uint64_t>(1, (cnt + kTB - 1) / kTB);
}

size_t lpart_floats(uint64_t m, uint32_t nb) { return (size_t)ltrain_blocks(m, nb) * kPartW; }

hipError_t launch_ltrain(const double* U, const float* Y, uint64_t m, uint32_t nb, uint32_t step,
                         MlpP* par, double* adam, float* part, LRes* res, double lr, int mode,
                         double* gout, hipStream_t st) {
  const uint32_t j = step % nb;
  const uint64_t cnt = m > j ? (m - j + nb - 1) / nb : 0;
  const uint32_t G = (uint32_t)std::max<uint64_t>(1, (cnt + kTB - 1) / kTB);
  hipLaunchKernelGGL(k_ltrain, dim3(G), dim3(kTB), 0, st, U, Y, m, nb, step, (const MlpP*)par,
                     part);
  double b1p = 1.0, b2p = 1.0;   // beta^(step + 1) by repeated products
  for (uint32_t s = 0; s <= step && mode == 0; ++s) {
    b1p = b1p * kBeta1;
    b2p = b2p * kBeta2;
  }
  hipLaunchKernelGGL(k_lreduce, dim3((kPartW + 63) / 64), dim3(64), 0, st, (const float*)part, G,
                     par, adam, res, lr, b1p, b2p, step, mode, gout);
  return hipGetLastError();
}

hipError_t launch_lthresh(const MlpP* par, int B, LRes* res, uint64_t* thr, hipStream_t st) {
  const int blocks = ((B - 1) * kTLanes + 255) / 256;   // a wave per threshold
  hipLaunchKernelGGL(k_lthresh, dim3(std::max(blocks, 1)), dim3(256), 0, st, par, B, res, thr);
  return hipGetLastError();
}

hipError_t launch_lforward(const MlpP* par, const uint64_t* x, uint64_t q, const LRes* res, int B,
                           float* fout, uint32_t* cout, hipStream_t st) {
  const int blocks = (int)std::min<uint64_t>((q + 255) / 256, 4096);
  hipLaunchKernelGGL(k_lforward, dim3(std::max(blocks, 1)), dim3(256), 0, st, par, x, q, res, B,
                     fout, cout);
  return hipGetLastError();
}

hipError_t launch_lhist_sample(const double* U, uint64_t m, const MlpP* par, int B,
                               uint32_t* counts, hipStream_t st) {
  const int blocks = (int)std::min<uint64_t>((m + kBlock * 8 - 1) / (kBlock * 8), 1024);
  hipLaunchKernelGGL(k_lhist_sample, dim3(std::max(blocks, 1)), dim3(kBlock), 0, st, U, m, par, B,
                     counts);
  return hipGetLastError();
}

hipError_t launch_lkeep(MlpP* par, const MlpP* par0, const double* g0, const double* g1,
                        const uint32_t* hc0, const uint32_t* hc1, int B, LRes* res,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_lkeep, dim3(1), dim3(kBlock), 0, st, par, par0, g0, g1, hc0, hc1, B, res);
  return hipGetLastError();
}

hipError_t launch_lcheck(const uint64_t* y, const uint32_t* bst, uint64_t n, int B, uint64_t* bmin,
                         uint64_t* bmax, LRes* res, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_lminmax_init, dim3((B + 255) / 256), dim3(256), 0, st, bmin, bmax, B);
  const uint64_t chunks = (n + kCheckChunk - 1) / kCheckChunk;
  const int blocks = (int)std::max<uint64_t>(1, std::min<uint64_t>(chunks, (uint64_t)grid));
  hipLaunchKernelGGL(k_lminmax, dim3(blocks), dim3(kBlock), 0, st, y, bst, n, B, bmin, bmax);
  hipLaunchKernelGGL(k_lcheck, dim3(1), dim3(kBlock), 0, st, bmin, bmax, bst, n, B, res);
  return hipGetLastError();
}

hipError_t launch_lthr_check(const uint64_t* thr, LRes* res, hipStream_t st) {
  hipLaunchKernelGGL(k_lthr_check, dim3(1), dim3(kBlock), 0, st, thr, res);
  return hipGetLastError();
}

hipError_t launch_lmaxcount(const uint32_t* bst, uint64_t n, int B, uint64_t* out, hipStream_t st) {
  hipLaunchKernelGGL(k_lmaxcount, dim3(1), dim3(kBlock), 0, st, bst, n, B, out);
  return hipGetLastError();
}

hipError_t launch_lfine_hist(const uint64_t* x, uint64_t n, const uint64_t* thr, const LRes* res,
                             int B, uint32_t* counts, hipStream_t st) {
  const int blocks = (int)std::min<uint64_t>((n + kBlock * 16 - 1) / (kBlock * 16), 2048);
  hipLaunchKernelGGL(k_lfine_hist, dim3(std::max(blocks, 1)), dim3(kBlock), 0, st, x, n, thr, res,
                     B, counts);
  return hipGetLastError();
}

hipError_t launch_lcounts(const uint32_t* bst, uint64_t n, int B, uint32_t* counts,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_lcounts, dim3((B + 255) / 256), dim3(256), 0, st, bst, n, B, counts);
  return hipGetLastError();
}

}  // namespace zs
