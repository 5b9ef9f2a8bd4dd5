// zsort_internal.h -- device data structures shared by the HIP kernels and the
// host planner of the zSort library (not part of the public C-ABI).
//
// The sort is a breadth-first version of zSort's recursion (Section III and
// Algorithm 1 of "zSort: Stable Distribution Sort using Z-Score
// Partitioning"): level L holds every subproblem ("segment") of depth L, and
// each level runs four kernels over all of its segments at once:
//   moments  -- exact integer min/max/sum/sum of squares, then finalize
//               (mean, std, Zmin, scale -> the map's A and B)
//   hist     -- per-chunk cluster histogram, the prefix across the chunks
//               of a segment (reduce, then scan, by the last workgroups to
//               arrive), and the exclusive scan + classification of the
//               clusters
//   scatter  -- stable scatter of key+payload to the other buffer
//   local    -- in-LDS stable sort of the small clusters of this level
// The recursion never returns to the host: each kernel reads its work count
// from device memory.
#pragma once
#include <stdint.h>

namespace zs {

constexpr int kWave = 64;
constexpr int kBlock = 256;            // threads per workgroup, 4 waves
constexpr int kWaves = kBlock / kWave;
constexpr int kMaxLevels = 40;
constexpr int kKMax = 4096;            // largest clusters-per-pass supported
constexpr int kLocalCap = 4096;        // largest group the fallback local sort takes
constexpr int kBlockCap = 2048;        // largest group of the fast local sort's main kernel
constexpr int kBigCap = 4096;          // largest group (= largest cutoff) of the fast local sort:
                                       // (kBlockCap, kBigCap] in a kernel of their own
constexpr int kWaveCap = 512;          // largest group one wave of the fallback sort takes
// largest group one wave of the fast local sort takes (wave jobs): 10 keys
// per lane with payloads of up to 4 bytes, 8 with 8-byte payloads (the LDS of
// a workgroup holds four such groups)
constexpr int wave_job_cap(int pw) { return pw == 8 ? 512 : 640; }
constexpr int kMidCap = 1024;          // largest block job that one wave of k_local_mid sorts
constexpr int kWindow = 256;           // leaf-group window; larger leaves sort alone
constexpr int kCopyChunk = 65536;      // keys per copy job of an all-identical segment
// device scratch of the allocation-free entry point (one array per GPU, held
// until the process ends); the largest problem it takes is the largest whose
// workspace layout fits
constexpr unsigned long long kScratchBytes = 64ull << 20;

// Cross-chunk scan of a segment of nch > 1 work items (reduce, then scan):
// the items are grouped into scan units of scan_unit(nch) consecutive items,
// a power of two near sqrt(nch), so that neither the pass over one unit's
// rows nor the pass over the unit totals is long.  A segment owns
// status_rows(nch) rows of k counts: one per item, then one per unit.
__host__ __device__ constexpr uint32_t scan_unit(uint32_t nch) {
  uint32_t u = 8;
  while (u < 256 && u * u < nch) u <<= 1;
  return u;
}
__host__ __device__ constexpr uint32_t scan_units(uint32_t nch) {
  return (nch + scan_unit(nch) - 1) / scan_unit(nch);
}
__host__ __device__ constexpr uint32_t status_rows(uint32_t nch) {
  return nch > 1 ? nch + scan_units(nch) : 0u;
}

// the kernels of a level, in launch order
enum : int { STAGE_MOMENTS = 0, STAGE_FINALIZE = 1, STAGE_HIST = 2, STAGE_SCATTER = 3,
             STAGE_LOCAL = 4, STAGE_LOCAL_HARD = 5, NSTAGES = 6 };

// segment kinds, as in the recursion records; KIND_LMAP is the learned
// partition map of the first pass (bucket ids precomputed by the hist pass)
// KIND_COUNT: a counting pass (key range below count_range): the clusters are
// the key values themselves, so each is final after the scatter
enum : int32_t { KIND_PENDING = 0, KIND_IDENT = 1, KIND_ZMAP = 2, KIND_RMAP = 3, KIND_LMAP = 4,
                 KIND_COUNT = 5 };
// kind of a counting pass in the recursion records of the public trace
constexpr int32_t kTraceCount = 4;
// segment flags
// F_FUSED: the statistics are accumulated by the parent's scatter
enum : uint32_t { F_RMAP = 1u, F_ROOT = 2u, F_FUSED = 4u };
// leaf-group flags
enum : uint32_t { LF_COPY = 1u };

struct __attribute__((aligned(16))) Seg {
  uint64_t start;        // first position in the array
  uint64_t count;        // number of keys
  uint64_t o_parent;     // parent's minimum (frame of e)
  double e;              // estimated mean in the parent's frame (z-map child)
  int32_t depth;
  uint32_t flags;
  uint32_t first_work;   // first chunk's index in the level's work list
  uint32_t nchunks;
  uint32_t status_base;  // first scan row (segments of > 1 chunk)
  uint32_t lm_base;      // learned map: first threshold of this segment's window
  int32_t parent;        // index of the parent in the previous level's list
  uint32_t lm_cnt;       // learned map: thresholds in the window (stride in `shift`)
  // results of finalize
  uint64_t o, M;
  uint64_t s1[2];        // sum (x - o)
  uint64_t s2[4];        // sum (x - o)^2
  double m, sigma, zmin, A, B;
  int32_t kind;
  int32_t shift;         // range-map shift; learned map: threshold stride of the window
};

struct __attribute__((aligned(16))) Leaf {
  uint32_t start;        // n < 2^31
  uint32_t count;
  uint32_t flags;        // LF_COPY: identical keys, copy only
  uint32_t src;          // 0: keys are in the caller's buffer, 1: in the alternate buffer
};

// Control block in device memory.  Lists alternate between two slots: the
// segments (and their work items and leaves) of level L live in slot L & 1.
struct __attribute__((aligned(64))) Ctl {
  uint32_t nseg[2];
  uint32_t nwork[2];
  uint32_t nleaf[2];             // block jobs: big leaves and copies
  uint32_t nleafw[2];            // wave jobs: groups of <= wave_job_cap(pw) keys
  uint32_t nleafm[2];            // one-wave jobs of wave_job_cap(pw) < n <= kMidCap keys
  uint32_t nleafx[2];            // wave jobs (<= kWaveCap keys) that may span 2^51 keys
  uint32_t nhard[2];             // groups the bucket pass left to the merge / radix sort
  uint32_t nstatus[2];
  uint32_t tick[kMaxLevels];     // work-item tickets of the hist pass
  uint32_t hdone[kMaxLevels];    // workgroups of the hist pass that have finished
  uint32_t ntile[2];             // 8192-key tiles: entries of the scatter's tile list
  uint32_t epoch;                // changes every call; tags the scan rows
  uint32_t clear_epoch;          // epoch at which the scan rows were last cleared
  uint32_t clear_rows;           // 1: this call's set-up kernel clears the scan rows
  uint32_t error;                // nonzero: a capacity or wait limit was hit
  uint32_t ntrace;
  uint32_t ntrace_hist;
  // statistics of the call
  uint64_t lvl_keys[kMaxLevels]; // keys distributed at each level
  uint64_t lvl_mkeys[kMaxLevels];// keys a moments pass read at each level
  uint64_t lvl_fkeys[kMaxLevels];// keys whose statistics the parent's scatter accumulated
  uint32_t lvl_segs[kMaxLevels];
  uint32_t n_ident;
  uint32_t n_rmap;
  uint32_t n_leafgroups;
  uint32_t max_level;
  uint64_t local_keys;           // keys sorted or copied by the local kernel
  uint32_t n_count;              // subproblems finished by a counting pass
  uint32_t n_hard;               // leaf groups left to the fallback sort
};

enum : uint32_t { ERR_SEGCAP = 1u, ERR_WORKCAP = 2u, ERR_LEAFCAP = 4u, ERR_STATUSCAP = 8u,
                  ERR_SPIN = 16u, ERR_SCATTER = 32u, ERR_OFFSETS = 0x100u };

// Debug trace record (written only when the trace buffer is given).
struct TraceRec {
  int32_t depth;
  int32_t kind;
  uint64_t start, count;
  uint64_t o, M;
  uint64_t s1[2];
  uint64_t s2[4];
  double m, sigma, zmin, A, B;
  int32_t shift;
  int32_t nonempty;
  int64_t hist_off;
};

// monotone MLP 1 -> 32 -> 32 -> 1 of the learned partition map.  1153
// parameters, indexed (gradients, optimizer state) in the order W1[32],
// b1[32], W2[32][32] (row = output unit), b2[32], W3[32], b3.  The first
// layer is binary64: a ramp must be placed to a fraction of its width, and
// a narrow, heavy component of the key distribution can span less than
// binary32's resolution of the normalised range.
constexpr int kH = 32;
constexpr int kNP = 1153;
constexpr int kW1 = 0, kB1 = 32, kW2 = 64, kB2 = 1088, kW3 = 1120, kB3 = 1152;
struct MlpP {
  double w1[kH], b1[kH];
  float w2[kH * kH], b2[kH], w3[kH], b3;
};

// device-side results of the learned map's set-up and check
struct LRes {
  uint64_t smin, smax;   // normalisation range: the sample's minimum and maximum
  uint32_t nt;           // number of thresholds
  uint32_t fail;         // 1: some cluster's maximum exceeds a later cluster's minimum
  uint64_t maxc;         // largest first-pass cluster of the learned map
  uint64_t maxz;         // largest cluster of the z-score map at the same count (diagnostic)
  uint32_t ticket;       // last-workgroup ticket of a training step
  uint32_t steps_done;
  double loss_first, loss_last;  // loss on minibatch 0 before training / of the kept parameters
  uint32_t trained;              // 1: the trained parameters were kept (not the initial ones)
  uint32_t pad;
  uint32_t smax_init, smax_trained;  // largest cluster of the sample under each parameter set
  double iscore[28];             // initialisation: largest gap / key range of each sample block
  uint64_t icut[28];             // and the position of that gap
};

// learned map of the first pass
// A learned segment's clusters are counted against a window of the
// thresholds: lm_cnt of them, starting at thr[lm_base], every shift-th one.
// With two stages (sub > 0) the root's window is every sub-th threshold and
// each root cluster j becomes a learned child with the sub - 1 thresholds
// after thr[j * sub - 1], so that the two passes together give the clusters
// of all thresholds.
struct LMap {
  const uint64_t* thr;   // thresholds t_1..t_nt: t_b is the least key whose cluster is >= b
  const MlpP* par;       // parameters (direct per-key inference only)
  uint16_t* ids;         // cluster id of each key, written by hist, read by scatter
  LRes* res;             // normalisation range, threshold count, largest cluster
  int32_t direct;        // 1: evaluate the MLP per key instead of searching the thresholds
  uint32_t sub;          // two stages: clusters per root cluster (0: one stage)
};

struct Params {
  int32_t k;             // clusters per pass
  int32_t lb;            // floor(log2 k), range-map bits per pass
  int32_t cutoff;        // leaf size
  int32_t max_zlevels;
  int32_t chunk;         // keys per work item
  int32_t tile;          // keys per scatter tile (2048, 4096 or 8192)
  int32_t pw;            // payload bytes: 0, 4, 8
  int32_t count_range;   // > 0: subproblems with max - min < count_range take a counting pass
  int32_t fuse;          // 1: children's statistics accumulated by their parent's scatter
};

// the word a histogram pass leaves for the host's pacing of the levels
__host__ __device__ inline uint64_t pace_word(uint32_t token, uint32_t nseg, bool leaves) {
  return ((uint64_t)(token & 0xFFFFFFu) << 40) | ((uint64_t)(leaves ? 1u : 0u) << 32) | nseg;
}
__host__ __device__ inline uint32_t pace_token_of(uint64_t w) { return (uint32_t)(w >> 40); }
__host__ __device__ inline bool pace_leaves_of(uint64_t w) { return ((w >> 32) & 1u) != 0; }

// Everything a kernel needs, by value.
struct Ws {
  uint64_t* keys[2];     // [0] caller's buffer, [1] alternate buffer
  void* pay[2];
  Seg* segs[2];
  uint64_t* work[2];     // (segment << 32) | chunk
  Leaf* leaves[2];       // block jobs
  Leaf* leavesw[2];      // wave jobs
  Leaf* leavesm[2];      // mid-size jobs (one wave, up to kMidCap keys)
  Leaf* leavesx[2];      // wave jobs of a wide key range (the fallback kernel's first loop)
  Leaf* hard[2];         // jobs for the fallback local sort
  uint64_t* status;      // scan rows [row][k], tagged words: a work item's counts,
                         // turned into its inclusive prefix within its unit; then
                         // each unit's exclusive prefix over the segment's units
  uint64_t* part;        // per work item: 8 digit sums, min, max (moments pass)
  uint32_t* bstart;      // exclusive cluster starts relative to the segment, [seg][k]
  uint32_t* child_of;    // fused statistics: each cluster's child segment (~0u: none), [seg][k]
  uint64_t* facc;        // fused statistics: per child segment of the level being made, in
                         // the order of the moments pass's partials (8 digit sums, min, max)
  uint32_t* arrive[2];   // per level slot: arrivals per scan unit, then per segment,
                         // indexed like the scan rows (zeroed when the segment is made)
  uint16_t* subpre;      // 8192-key tiles: each cluster's count in a work item before
                         // the tile that starts at key position p, row p >> 13, [row][k]
  uint64_t* tiles[2];    // 8192-key tiles: (segment << 32) | (chunk << 3) | tile, the scatter's items
  Ctl* ctl;
  TraceRec* trace;       // may be null
  uint32_t* trace_hist;
  uint32_t trace_cap, trace_hist_cap;
  uint64_t* h_pace;      // pinned host words, or null: once level L's histogram pass has made
                         // level L + 1's segments and level L's leaf jobs, its last workgroup
                         // stores pace_word(token, that segment count (0 after an error),
                         // whether there are leaf jobs) at [L + 1]
  uint32_t pace_token;   // the call's token (24 bits), so that no store of an earlier call is taken
  uint32_t seg_cap, work_cap, leaf_cap, status_cap, tile_cap;
  uint32_t force_clear;  // 1: clear the scan rows in this call (set-up of a new layout)
  uint64_t status_words; // words of the scan-row region
  Params p;
  LMap lm;
};

// Scan-row tags: within any run of kClearEvery consecutive epochs the tags
// of (epoch, level) pairs are distinct and never 0 (the value of a cleared
// word), so a word carries the current tag only if this level of this call
// wrote it.  The rows are cleared at least once per kClearEvery epochs.
constexpr uint32_t kTagMod = (1u << 22) - 1u;
constexpr uint32_t kClearEvery = 60000u;   // * 64 levels < kTagMod
static_assert((uint64_t)kClearEvery * 64u < kTagMod, "tags must not repeat between clears");

}  // namespace zs
