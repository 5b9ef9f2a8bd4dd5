// zsort_wide.hip -- 128-bit keys.  The z-score sort runs in two stages over
// 64-bit words: the high words of all keys are distributed first (each
// carrying its key's low word, or with a payload the payload and the key's
// position), then every run of equal high words is sorted
// by its low words -- inside such a run the key rebased to the run's minimum
// fits 64 bits, so the same distribution applies there.  These kernels move
// the words between the caller's 128-bit layout and the two stages.
#include <hip/hip_runtime.h>

#include "zsort_internal.h"

namespace zs {

constexpr int kWideBlock = 256;
constexpr uint64_t kSignBit = 0x8000000000000000ull;

// hi[i] = high word of key i (sign bit flipped for signed keys); second[i] =
// the word the high-word stage carries with it: the key's low word, or, with
// a payload, (payload[i] << 32) | i.  The run counters start at 0: nruns[0]
// runs listed for the low-word stage, nruns[1] short runs sorted at once,
// nruns[2..3] keys in runs of either kind (64-bit).
__global__ void __launch_bounds__(kWideBlock)
k_split128(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ payload, uint64_t n,
           uint32_t sgn, uint64_t* __restrict__ hi, uint64_t* __restrict__ second,
           uint32_t* nruns) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    nruns[0] = 0u;
    nruns[1] = 0u;
    *reinterpret_cast<unsigned long long*>(nruns + 2) = 0ull;
  }
  const uint64_t i = (uint64_t)blockIdx.x * kWideBlock + threadIdx.x;
  if (i >= n) return;
  const ulonglong2 k = reinterpret_cast<const ulonglong2*>(keys)[i];
  hi[i] = k.y ^ (sgn ? kSignBit : 0ull);
  second[i] = payload ? (((uint64_t)payload[i] << 32) | i) : k.x;
}

// With a payload, after the high-word stage (lo[i] = (payload << 32) |
// original position of the key now at i): lo[i] = that key's low word (a
// gather from the caller's keys) and pay[i] = its payload.  Each element is
// rewritten in place by the thread that reads it.
__global__ void __launch_bounds__(kWideBlock)
k_unpack_lo(const uint64_t* __restrict__ keys, uint64_t* lo, uint64_t n,
            uint32_t* __restrict__ pay) {
  const uint64_t i = (uint64_t)blockIdx.x * kWideBlock + threadIdx.x;
  if (i >= n) return;
  const uint64_t v = lo[i];
  lo[i] = keys[2 * (v & 0xFFFFFFFFull)];
  pay[i] = (uint32_t)(v >> 32);
}

// Runs of >= 2 equal high words: a run of at most kSmallRun keys is sorted by
// its low words right here by the thread that finds its start (a stable
// insertion sort of the low words, the payload (may be NULL) moving along;
// equal low words keep their order, which is the input order since the
// high-word stage is stable); a longer run is appended to `runs` as (start,
// length), in no particular order, for the low-word stage.  The run's end is
// found by binary search in the sorted high words.
constexpr uint64_t kSmallRun = 64;

__global__ void __launch_bounds__(kWideBlock)
k_find_runs(const uint64_t* __restrict__ hi, uint64_t n, uint64_t* __restrict__ lo,
            uint32_t* __restrict__ pay, uint32_t* __restrict__ runs, uint32_t* nruns) {
  const uint64_t i = (uint64_t)blockIdx.x * kWideBlock + threadIdx.x;
  if (i >= n) return;
  const uint64_t v = hi[i];
  if (!(i + 1 < n && hi[i + 1] == v && (i == 0 || hi[i - 1] != v))) return;
  uint64_t a = i + 1, b = n;   // first position after the run
  while (a < b) {
    const uint64_t mid = a + (b - a) / 2;
    if (hi[mid] == v) a = mid + 1;
    else b = mid;
  }
  const uint64_t len = a - i;
  atomicAdd(reinterpret_cast<unsigned long long*>(nruns + 2), (unsigned long long)len);
  if (len <= kSmallRun) {
    for (uint64_t p = i + 1; p < a; ++p) {
      const uint64_t x = lo[p];
      const uint32_t y = pay ? pay[p] : 0u;
      uint64_t q = p;
      while (q > i && lo[q - 1] > x) {
        lo[q] = lo[q - 1];
        if (pay) pay[q] = pay[q - 1];
        --q;
      }
      lo[q] = x;
      if (pay) pay[q] = y;
    }
    atomicAdd(nruns + 1, 1u);
    return;
  }
  const uint32_t j = atomicAdd(nruns, 1u);
  runs[2 * (uint64_t)j] = (uint32_t)i;
  runs[2 * (uint64_t)j + 1] = (uint32_t)len;
}

// keys[i] = (lo[i], hi[i]) (sign bit restored)
__global__ void __launch_bounds__(kWideBlock)
k_final128(uint64_t* __restrict__ keys, uint64_t n, uint32_t sgn, const uint64_t* __restrict__ hi,
           const uint64_t* __restrict__ lo) {
  const uint64_t i = (uint64_t)blockIdx.x * kWideBlock + threadIdx.x;
  if (i >= n) return;
  reinterpret_cast<ulonglong2*>(keys)[i] = make_ulonglong2(lo[i], hi[i] ^ (sgn ? kSignBit : 0ull));
}

// one thread per key (n < 2^31: at most 2^23 workgroups)
static dim3 wide_grid(uint64_t n) { return dim3((unsigned)((n + kWideBlock - 1) / kWideBlock)); }

hipError_t launch_split128(const uint64_t* keys, const uint32_t* payload, uint64_t n, int sgn,
                           uint64_t* hi, uint64_t* second, uint32_t* nruns, hipStream_t st) {
  hipLaunchKernelGGL(k_split128, wide_grid(n), dim3(kWideBlock), 0, st, keys, payload, n,
                     (uint32_t)sgn, hi, second, nruns);
  return hipGetLastError();
}

hipError_t launch_gather_runs(const uint64_t* keys, const uint64_t* hi, uint64_t n, uint64_t* lo,
                              uint32_t* payload, uint32_t* runs, uint32_t* nruns, hipStream_t st) {
  if (payload)
    hipLaunchKernelGGL(k_unpack_lo, wide_grid(n), dim3(kWideBlock), 0, st, keys, lo, n, payload);
  hipLaunchKernelGGL(k_find_runs, wide_grid(n), dim3(kWideBlock), 0, st, hi, n, lo, payload, runs,
                     nruns);
  return hipGetLastError();
}

hipError_t launch_final128(uint64_t* keys, uint64_t n, int sgn, const uint64_t* hi,
                           const uint64_t* lo, hipStream_t st) {
  hipLaunchKernelGGL(k_final128, wide_grid(n), dim3(kWideBlock), 0, st, keys, n, (uint32_t)sgn, hi,
                     lo);
  return hipGetLastError();
}

}  // namespace zs
