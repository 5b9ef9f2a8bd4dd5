/*
 * zsort.h -- C-ABI of the MI355X (gfx950) zSort library.
 *
 * The library sorts 64-bit unsigned keys, stably, carrying a 0-, 4- or 8-byte
 * payload with each key, by the z-score distribution method of
 * "zSort: Stable Distribution Sort using Z-Score Partitioning"
 * (arXiv 2605.14419): Section III (problem statement: clusters with
 * max(C_j) < min(C_j+1); stability; duplicate handling; the mapping function
 * of Eq. (1) with its clip; the estimated mean of the recursive phase) and
 * Algorithm 1 (moments, histogram, exclusive prefix, stable scatter,
 * recursion, small-cluster sort).
 *
 * Conventions shared by every entry point
 *   - Pointers named keys/payload/seg_offsets are DEVICE pointers owned by the
 *     caller.  Sorting is in place: on return (after the stream has reached
 *     the call) keys[0, n) is ascending as unsigned 64-bit integers and every
 *     payload element sits beside the key it came with; keys that compare
 *     equal keep their input order (the stable order, which makes the output
 *     unique).
 *   - `stream` is a hipStream_t (NULL = the default stream).  Work is enqueued
 *     on it and the call returns without waiting for the device, except that
 *     a call whose problem size needs more workspace than the stream has
 *     allocates it (hipMalloc, which synchronises the device).  While the
 *     stream is being captured into a hipGraph a call never allocates: it
 *     runs in the workspace the stream has (a new problem size is laid out
 *     inside it) or returns ZSORT_ECAPTURE.  zsort_set_workspace hands the
 *     library caller-owned memory instead, so that a caller can capture any
 *     shape that fits it.
 *   - Limits: 1 <= n <= 2^31 - 1 keys per call (n <= 1 is a no-op that
 *     returns ZSORT_OK).  Buffers must not overlap.
 *   - Errors are returned as negative status codes; nothing throws across the
 *     ABI and no caller memory is freed.  Capacity overruns detected on the
 *     device are reported by zsort_get_last_stats (field device_error).
 *   - Calls on one stream are serialised; calls on different streams use
 *     different workspaces and may run concurrently.
 */
#ifndef ZSORT_H
#define ZSORT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ZSORT_OK = 0,
  ZSORT_EINVAL = -1,        /* bad argument (null pointer, size, config) */
  ZSORT_ENOMEM = -2,        /* device allocation failed */
  ZSORT_EHIP = -3,          /* a HIP runtime call failed (see zsort_last_hip_error) */
  ZSORT_ECAPTURE = -4,      /* the call would allocate while its stream is being captured */
  ZSORT_EUNSUPPORTED = -5,  /* configuration not built into this library */
  ZSORT_EDEVICE = -6,       /* a device-side limit was hit (only from synchronous calls) */
  ZSORT_ETOOLARGE = -7      /* the problem does not fit the fixed scratch buffer */
};

/*
 * The operation every sorting entry point performs (the paper's Section III,
 * problem statement and stability; Algorithm 1): the unique stable order of
 * the keys, computed by recursive distribution -- exact moments of each
 * subproblem (Algorithm 1's sum/minimum and variance loops), the z-score map
 * of Eq. (1) with the clip of the cluster definition, histogram, exclusive
 * prefix and stable scatter into one array separated by offsets (Algorithm
 * 1's distribution loops), recursion with the estimated mean of the
 * recursive phase for clusters above the cutoff, identical-key subproblems
 * finished at once (duplicate handling, Section III), and small clusters
 * sorted locally (Algorithm 1's insertion-sort step, here an in-LDS sort).
 */

/*
 * Tuning of the distribution.  k and cutoff change the recursion tree (and
 * therefore the intermediate arrays) but never the output.
 *   k            clusters per distribution pass, 16..4096.  The paper uses
 *                k = sqrt(n) held constant across levels (Section III, choice
 *                of k); here k is a constant "buckets per pass".  Default 1024.
 *   cutoff       clusters of at most this many keys are finished by the local
 *                (in-LDS) stable sort, 1..4096 (the paper's insertion-sort
 *                threshold is 96).  Default 2048.
 *   max_zlevels  depth at which the z-score map gives way to the exact range
 *                map, 0..16 (0 = range map everywhere).  Default 8.
 *   chunk        keys per work item of a pass, a multiple of 2048 in
 *                [2048, 2^20] (and of tile).  Default 16384.
 *   tile         keys a workgroup ranks per step of the stable scatter:
 *                2048, 4096 (256 threads) or 8192 (1024 threads); above 2048
 *                needs k <= 1024 and chunk a multiple of tile; 8192 needs
 *                chunk <= 65536.  Default 2048.
 *   flags        ZSORT_FLAG_GRAPH: run the whole sort as one cached hipGraph
 *                (every level of the recursion is launched; kernels of empty
 *                levels exit at once).  The graph is captured on a private
 *                stream at the first call with a given set of buffers, shape
 *                and configuration, and replayed on `stream` afterwards.
 *                Without the flag the library launches level by level,
 *                waiting for each level's histogram pass to learn whether
 *                the level has local sorts and whether another level follows
 *                (host-side pacing; the call returns once the last level is
 *                known).  A level's local sorts may run on a second stream of
 *                the library's beside the next level; `stream` waits for
 *                them, so work queued on it after the call sees the result.
 *                ZSORT_FLAG_SIGNED: the keys are two's-complement int64 and
 *                are ordered as signed numbers (the sign bit is flipped in
 *                place before the sort and back after it: two more passes
 *                over the keys).  zsort_stable_ex and zsort_stable_segmented
 *                only; the debug, traced and learned entry points return
 *                ZSORT_EUNSUPPORTED for it.
 *                ZSORT_FLAG_FUSED_STATS: the statistics of a subproblem made
 *                by a distribution pass (its exact min, max, sums of x and
 *                x^2: Section III, the variance loop of Algorithm 1) are
 *                accumulated while that pass scatters its keys, instead of in
 *                a pass of their own over them at the next level.  Applies
 *                with k <= 1024 (else ignored); output-neutral (the sums are
 *                exact integers in either order).  Off by default: it saves
 *                the 8 B/key re-read but its digit arithmetic and per-tile
 *                accumulator updates cost more than that read (about 2x the
 *                sort time on 10^8 lognormal keys, 10x on Zipf keys, whose
 *                tiles are dominated by one cluster).
 *   count_range  0 (default: off) or 1..k: a subproblem whose keys span less
 *                than count_range (max - min < count_range) is finished by one
 *                stable counting pass on x - min (the counting-sort heuristic
 *                for small ranges in Section III), in which every key value
 *                is a cluster of its own, instead of further distribution
 *                levels.  Output-neutral.
 */
#define ZSORT_FLAG_GRAPH 1
#define ZSORT_FLAG_SIGNED 2
#define ZSORT_FLAG_FUSED_STATS 4
typedef struct zsort_config {
  int32_t k;
  int32_t cutoff;
  int32_t max_zlevels;
  int32_t chunk;
  int32_t tile;
  int32_t flags;
  int32_t count_range;
  int32_t reserved;
} zsort_config;

/* Fills cfg with the defaults above (k, the cutoff and the recursion depth
 * are the parameters of Algorithm 1 and of the choice of k in Section III).
 * Returns ZSORT_OK or ZSORT_EINVAL (null). */
int zsort_default_config(zsort_config* cfg);

/*
 * Autotuner (an extension; the paper chooses k by the sensitivity study of
 * Section III's choice of k and its table of alpha values): times candidate
 * configurations (k in {256, 512, 1024}; (tile, chunk) in {(2048, 16384),
 * (4096, 32768), (8192, 8192), (8192, 32768)}; cutoff in {1024, 2048, 4096}),
 * then the three fastest of them with max_zlevels 1 and 2 as well (z-score maps on
 * the first one or two levels, range maps below; a mixture of clusters sorts
 * in fewer levels so) on a scratch copy of keys/payload (device buffers, left unchanged;
 * seg_offsets may be NULL for a single array) and remembers the fastest that
 * ran within the device's limits (device_error 0) for the shape class (n
 * rounded up to a power of two, payload width, single or segmented).
 * Later calls of that class with cfg == NULL use it.  If the class is already
 * known no timing is done.  cache_path (may be NULL) names a text file of
 * tuned entries that is read first and rewritten afterwards.  best (host, may
 * be NULL) receives the chosen configuration.  Synchronous; allocates scratch
 * memory for the copies.  The winner's output is checked to be sorted before
 * it is remembered (single arrays); ZSORT_EDEVICE if no candidate passes.
 */
int zsort_autotune(const uint64_t* keys, const void* payload, int payload_bytes, size_t n,
                   const int64_t* seg_offsets, int32_t num_segments, const char* cache_path,
                   zsort_config* best, void* stream);

/*
 * Stable sort of keys[0, n) with an optional u32 payload (payload may be
 * NULL); Algorithm 1 with the mapping of Eq. (1), Section III.  The tuned
 * configuration of the shape class (zsort_autotune), else the defaults.
 * keys: n u64, ascending unsigned on return; payload: n u32 moved with their
 * keys.  Errors: ZSORT_EINVAL (null keys with n > 1, n >= 2^31),
 * ZSORT_ENOMEM / ZSORT_EHIP / ZSORT_ECAPTURE as above.
 */
int zsort_stable(uint64_t* keys, uint32_t* payload, size_t n, void* stream);

/* As zsort_stable with a u64 payload (may be NULL): Algorithm 1, Eq. (1). */
int zsort_stable_p64(uint64_t* keys, uint64_t* payload, size_t n, void* stream);

/*
 * For callers that cannot allocate (code under hipGraph capture, tight serving
 * loops, harnesses that forbid hipMalloc): zsort_stable_ex that allocates
 * nothing, neither device nor pinned host memory nor events.  Its workspace
 * is a fixed array of ZSORT_NOALLOC_SCRATCH_BYTES (64 MiB) in device memory,
 * one per GPU, held from the library's load until the process ends; the
 * largest problem it takes is the largest whose zsort_workspace_bytes (with
 * num_segments 0 and the same cfg) is at most that, e.g. 2^21 keys with any
 * payload at the default configuration, about 3.5 * 10^6 with a 4-byte one.
 * Larger problems return ZSORT_ETOOLARGE without touching the data.  Every
 * call on a GPU shares that GPU's array and leaves its contents behind: calls
 * that overlap on one GPU (different streams, or host threads) race and must
 * be serialised by the caller.  The output equals zsort_stable_ex's with the
 * same arguments.  ZSORT_FLAG_GRAPH returns ZSORT_EUNSUPPORTED (it captures
 * on a stream of its own); every level of the recursion is launched, as in
 * graph mode.  zsort_get_last_stats does not report these calls.
 */
#define ZSORT_NOALLOC_SCRATCH_BYTES (64ull << 20)
int zsort_stable_noalloc(uint64_t* keys, void* payload, int payload_bytes, size_t n,
                         const zsort_config* cfg, void* stream);

/*
 * General form of zsort_stable (Algorithm 1, Eq. (1), Section III):
 * payload_bytes is 0 (payload ignored, may be NULL), 4 or 8; cfg may be NULL
 * (tuned entry of the shape class, else the defaults); ZSORT_EINVAL for a
 * configuration outside the ranges above.
 */
int zsort_stable_ex(uint64_t* keys, void* payload, int payload_bytes, size_t n,
                    const zsort_config* cfg, void* stream);

/*
 * Batched form (an extension: Algorithm 1 applied to each of many arrays,
 * whose recursions run level by level together): num_segments independent
 * arrays laid end to end in keys[0, n);
 * segment i is [seg_offsets[i], seg_offsets[i+1]).  seg_offsets is a DEVICE
 * array of num_segments + 1 int64 with seg_offsets[0] = 0,
 * seg_offsets[num_segments] = n and non-decreasing entries (empty segments
 * allowed).  Each segment is sorted on its own, stably.  The offsets are
 * checked on the device; if they are malformed nothing is moved and
 * zsort_get_last_stats reports device_error bit 0x100.  payload_bytes is
 * 0, 4 or 8; cfg may be NULL.  All segments go through one set of launches
 * (the recursion levels of every segment run together).
 */
int zsort_stable_segmented(uint64_t* keys, void* payload, int payload_bytes, size_t n,
                           const int64_t* seg_offsets, int32_t num_segments,
                           const zsort_config* cfg, void* stream);

/*
 * 128-bit keys (an extension named by the paper's motivation, Section I: the
 * number of distribution passes does not grow with the key width, unlike a
 * radix sort's).  keys: DEVICE array of n keys of 16 bytes (16-byte aligned),
 * each the two u64 words of an unsigned 128-bit integer, low word first;
 * sorted in place, stably, with an optional u32 payload (may be NULL).  Two
 * z-score stages over 64-bit words: the high words of all keys are sorted
 * (Algorithm 1, Eq. (1)), each carrying its key's low word (or, with a
 * payload, the payload and the key's position); then every run of equal high
 * words is sorted by its low words -- inside such a run the key rebased to
 * the run's minimum fits 64 bits.  Runs of at most 64 keys are sorted at
 * once by an insertion sort; longer ones by the same distribution as a batch
 * of subproblems.  ZSORT_FLAG_SIGNED orders the keys as two's-complement
 * int128; ZSORT_FLAG_GRAPH returns ZSORT_EUNSUPPORTED; a misaligned keys
 * pointer ZSORT_EINVAL.  The stream keeps buffers of 16 bytes per key for the
 * stages (plus the workspace of the 64-bit sort with an 8-byte payload).  The
 * payload is rewritten in the caller's array between the stages: after an
 * error in the second stage (a return code, or device_error in the report)
 * the keys may be partly sorted and the payload no longer matches them.  report (host, may be NULL) makes the call
 * synchronous and receives the recursion depth of each stage and the runs.
 */
typedef struct zsort_u128_report {
  int32_t levels_high;   /* recursion levels of the high-word stage */
  int32_t levels_low;    /* of the low-word stage (0: no run longer than 64 keys) */
  uint64_t runs;         /* runs of >= 2 equal high words */
  uint64_t short_runs;   /* of which <= 64 keys, sorted by insertion */
  uint64_t run_keys;     /* keys in all runs */
  int32_t device_error;  /* as zsort_stats.device_error, either stage */
  int32_t reserved;
} zsort_u128_report;
int zsort_stable_u128(uint64_t* keys, uint32_t* payload, size_t n, const zsort_config* cfg,
                      zsort_u128_report* report, void* stream);

/* Device bytes of workspace a call of this shape needs (0 if invalid): the
 * ping-pong partner of keys and payload (Algorithm 1's second array), the
 * recursion's lists and the histogram rows.  cfg NULL: the configuration such
 * a call would use (the tuned entry of the shape class, else the defaults).
 * Host-only; no device is touched. */
size_t zsort_workspace_bytes(size_t n, int payload_bytes, int32_t num_segments,
                             const zsort_config* cfg);

/*
 * Caller-owned workspace for the calls on `stream` (the memory of Algorithm
 * 1's second array and of the recursion's lists).  d_ws is DEVICE memory of
 * `bytes` bytes, 256-byte aligned and at least a control block in size; it
 * stays owned by the caller, who keeps it alive and unused by anything else
 * until another zsort_set_workspace on that stream (or zsort_release).  From
 * then on no call on the stream allocates: a problem whose
 * zsort_workspace_bytes exceeds `bytes` returns ZSORT_ENOMEM, so a caller can
 * capture zsort_stable_* into a graph of its own at any size that fits.
 * d_ws NULL with bytes 0 returns the stream to library-allocated memory.  The
 * library's own buffer of the stream, if any, is freed (synchronises the
 * device).  Enqueues a clear of the control block on `stream`.  Errors:
 * ZSORT_EINVAL (misaligned or too small, or NULL with bytes > 0),
 * ZSORT_ECAPTURE (the stream is being captured).  The learned form keeps its
 * own buffers (and is not capturable).
 */
int zsort_set_workspace(void* d_ws, size_t bytes, void* stream);

/*
 * Allocation limit for tests of the out-of-memory path: every device
 * allocation the library would make that is larger than max_bytes fails as
 * if the device were out of memory (the call returns ZSORT_ENOMEM).  0 (the
 * default) removes the limit.  Host-only.
 */
int zsort_set_alloc_limit(size_t max_bytes);

/*
 * Statistics of the last call on `stream` (synchronises that stream): the
 * recursion of Algorithm 1 as it ran, level by level (Section III's depth
 * analysis counts these levels).
 *   levels            number of recursion levels that held work
 *   device_error      0, or bits: 1 segment list, 2 work list, 4 leaf list,
 *                     8 scan rows full, 16 scan-row wait limit,
 *                     32 a scatter destination outside its segment (never
 *                     with consistent counts), 0x100 malformed segment offsets
 *   keys_per_level    keys distributed at each level
 *   segs_per_level    subproblems distributed at each level
 *   mkeys_per_level   keys a moments pass read at each level (with
 *                     ZSORT_FLAG_FUSED_STATS the statistics of a distribution
 *                     pass's subproblems come from that pass's scatter, and
 *                     their keys are not read again for them)
 *   local_keys        keys the local kernel sorted or copied into place
 *   fallback_groups   leaf groups left to the fallback sort (key range above 51
 *                     bits that the wide path could not take, or a bucket of
 *                     more than 128 keys that is not a run of one key value)
 *   model_bytes       algorithmic HBM bytes of the executed pass structure:
 *                     8 B per key of a moments pass, 8 B per key of a
 *                     histogram pass, 2(8+P) B per key of a scatter pass and
 *                     2(8+P) B per local-sorted or copied key (P = payload
 *                     bytes)
 */
#define ZSORT_MAX_LEVELS 40
typedef struct zsort_stats {
  int32_t levels;
  int32_t device_error;
  uint32_t identical;
  uint32_t range_mapped;
  uint32_t leaf_groups;
  int32_t payload_bytes;
  uint64_t n;
  uint64_t keys_per_level[ZSORT_MAX_LEVELS];
  uint64_t mkeys_per_level[ZSORT_MAX_LEVELS];
  uint32_t segs_per_level[ZSORT_MAX_LEVELS];
  uint64_t local_keys;
  double model_bytes;
  uint32_t counted;     /* subproblems finished by a counting pass (count_range) */
  uint32_t fallback_groups;  /* leaf groups the local sorts left to the fallback sort */
} zsort_stats;

int zsort_get_last_stats(void* stream, zsort_stats* out /* host */);

/*
 * Parity/debug entry: one distribution pass of the root (Algorithm 1 up to the
 * scatter, Eq. (1); moments, statistics,
 * histogram, scan, stable scatter), without recursion.  The resulting cluster
 * array (Algorithm 1's single array separated by offsets) is copied to
 * out_keys / out_payload (device, n elements; out_payload may be NULL when
 * payload_bytes is 0).  keys/payload are left unchanged.  Requires
 * n > cfg->cutoff.  Synchronous.
 */
int zsort_debug_level0(const uint64_t* keys, const void* payload, int payload_bytes, size_t n,
                       const zsort_config* cfg, uint64_t* out_keys, void* out_payload,
                       void* stream);

/*
 * Record of one subproblem larger than the cutoff, for level-by-level parity:
 * depth, kind (1 identical keys, 2 z-score map, 3 range map, 4 counting pass), position and
 * size, exact moments about the minimum (S1: 2 limbs, S2: 4 limbs,
 * little-endian), the binary64 statistics of the map, the range-map shift,
 * the number of non-empty clusters and the offset of its k cluster counts in
 * the histogram output (-1 if not stored).
 */
typedef struct zsort_trace_rec {
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
} zsort_trace_rec;

/*
 * zsort_stable_ex that also records every subproblem (the recursion of
 * Section III's recursive phase, one record per call of zsortRec) (host buffers; records
 * in no particular order).  counts[0] = records produced (may exceed
 * trace_cap), counts[1] = histogram words stored.  Synchronous; returns
 * ZSORT_EDEVICE if a device-side limit was hit.
 */
int zsort_stable_traced(uint64_t* keys, void* payload, int payload_bytes, size_t n,
                        const zsort_config* cfg, zsort_trace_rec* trace, int64_t trace_cap,
                        uint32_t* hist, int64_t hist_cap, int64_t counts[2], void* stream);

/*
 * Per-kernel device time (measurement; not part of the method).  Between
 * zsort_profile_begin(stream) and
 * zsort_profile_end(stream, out) every kernel the library launches on
 * `stream` is bracketed by a pair of hipEvents recorded on that same stream;
 * _end synchronises the stream and sums the elapsed times per kernel kind:
 * index 0 moments, 1 finalize (statistics of the map), 2 histogram (with
 * cross-chunk scan and classification), 3 stable scatter, 4 local sort (bucket
 * pass), 5 local sort fallback (merge / radix).  launches[i] counts the
 * launches, including those of levels that found no work.
 */
typedef struct zsort_kernel_times {
  double ms[6];
  uint64_t launches[6];
} zsort_kernel_times;

int zsort_profile_begin(void* stream);
int zsort_profile_end(void* stream, zsort_kernel_times* out /* host */);

/*
 * As zsort_profile_begin, but only the kernel kinds whose bit is set in
 * stage_mask (bit i = index i above) are bracketed by events; the others run
 * as without profiling, and their entries of zsort_kernel_times stay zero.
 * Recording an event between kernels costs a few microseconds, so timing one
 * kind disturbs the rest of the call less.  ZSORT_EINVAL for an empty mask
 * or bits above 5.
 */
int zsort_profile_begin_stages(void* stream, uint32_t stage_mask);

/*
 * Learned partition map for the first distribution pass (an extension: the
 * paper's map is Eq. (1); Section III only asks of a map that clusters come
 * out ordered, max(C_j) <= min(C_j+1), which makes the concatenation of the
 * sorted clusters sorted).
 *
 * A monotone MLP f: [0, 1] -> R, 1 -> 32 -> 32 -> 1, with non-negative
 * weights and clamp(., 0, 1) activations, approximates the CDF of a 1 %
 * strided key sample.  Key x goes to cluster
 *   min(B - 1, floor(B * clamp(f(u(x)), 0, 1))),
 *   u(x) = 0 if x <= smin, 1 if x >= smax, else (x - smin) / (smax - smin),
 * smin / smax the sample's extremes.  The first layer (weights, product
 * and sum) is binary64, its pre-activation rounded once to binary32; the
 * rest is binary32 with separately rounded products and sums in index order.
 * The 1153 parameters (W1[32], b1[32], W2[32][32], b2[32], W3[32], b3, in
 * this order wherever they are indexed, e.g. gradients) are held in a
 * zsort_mlp_params: binary64 W1 and b1 place a ramp to a small fraction of
 * its width even where a narrow, heavy component of the keys spans less than
 * binary32's resolution of the normalised range.
 *
 * zsort_stable_learned: (1) samples one key per sample_stride (offset from
 * SplitMix64 of seed), sorts the sample with the plain path, fits the MLP
 * (initialisation from the sample: 28 equal-count blocks, the 4 with the
 * widest internal gaps cut at the gap, one first-layer ramp per piece
 * weighed by its share of the sample, i.e. the sample CDF linear inside a
 * piece and flat across gaps; then `steps` Adam steps on the squared error to
 * the keys' mid-ranks, weights projected onto >= 0, deterministic gradient
 * reduction; the trained parameters are kept only if the sample's largest
 * cluster under them is not larger than under the initial ones), and
 * compiles it into
 * thresholds t_b = min{x : cluster(x) >= b} by bisection over the 64-bit
 * keys; (2) runs the first pass with B clusters
 * (cluster = number of thresholds <= key, found by binary search in LDS;
 * or, with ZSORT_LEARNED_DIRECT, the MLP evaluated per key); (3) checks on
 * the device that every non-empty cluster's maximum is <= the minimum of
 * every later cluster -- with thresholds by checking that they are sorted
 * (which implies it), with per-key inference (or ZSORT_LEARNED_VERIFY) by
 * taking every cluster's minimum and maximum from the first pass's output;
 * (4) if the check passes, finishes with the z-score
 * recursion (children take their exact mean); otherwise sorts the caller's
 * keys, which the first pass left untouched, with the plain z-score path.
 * The output is the same stable sort in every case.
 *
 * The call is synchronous (it waits for the check).  cfg as for
 * zsort_stable_ex (ZSORT_FLAG_GRAPH and ZSORT_FLAG_SIGNED are not supported); lcfg may be NULL
 * (defaults); report (host) may be NULL.  Arrays too small for a first pass
 * (n <= cutoff) or for a sample of 64 keys take the plain path
 * (report->used_learned = 0, report->fallback = 0).
 */
#define ZSORT_MLP_PARAMS 1153
typedef struct zsort_mlp_params {
  double w1[32], b1[32];           /* first layer, binary64 */
  float w2[32 * 32], b2[32];       /* second layer, w2[j * 32 + i]: input i -> unit j */
  float w3[32], b3;                /* output */
} zsort_mlp_params;
#define ZSORT_LEARNED_DIRECT 1u       /* per-key MLP inference in the first pass */
#define ZSORT_LEARNED_ZSCORE_DIAG 2u  /* also count the z-score map's clusters at B */
#define ZSORT_LEARNED_VERIFY 4u       /* scan the first pass's output in the order check */
typedef struct zsort_learned_config {
  int32_t buckets;        /* B: clusters of the first pass, 16..4096; default 4096 */
  int32_t sample_stride;  /* one key per stride is sampled; default 100 (1 %) */
  int32_t steps;          /* Adam steps, 0 = initialisation only (default: on the
                             mixture shapes no step count lowered the sample's
                             largest cluster, so the initialisation was kept anyway) */
  int32_t batches;        /* step t uses samples i with i mod batches == t mod batches; default 64 */
  double lr;              /* Adam step size (beta1 0.9, beta2 0.999, eps 1e-8); default 1e-4 */
  uint64_t seed;          /* sample offsets */
  uint32_t flags;         /* ZSORT_LEARNED_* */
  uint32_t reserved;
  const zsort_mlp_params* params;  /* DEVICE, or NULL to fit on a sample; when given, no
                                      sample is drawn and smin/smax below are used */
  uint64_t smin, smax;    /* normalisation range with params (smin <= smax) */
} zsort_learned_config;

typedef struct zsort_learned_report {
  int32_t used_learned;          /* 1: the learned map sorted the first pass */
  int32_t fallback;              /* 1: the order check failed; the z-score path ran */
  int32_t thresholds;            /* nt (-1 with ZSORT_LEARNED_DIRECT) */
  int32_t steps;                 /* Adam steps run */
  int32_t trained;               /* 1: the trained parameters were kept, 0: the initial ones */
  int32_t reserved;
  uint32_t sample_max_init;      /* largest cluster of the sample, initial parameters */
  uint32_t sample_max_trained;   /* the same after training */
  uint64_t sample_keys;          /* m = n / sample_stride (0 with given params) */
  uint64_t max_cluster_learned;  /* largest first-pass cluster of the learned map */
  uint64_t max_cluster_zscore;   /* the same for the z-score map (ZSORT_LEARNED_ZSCORE_DIAG) */
  double imbalance_learned;      /* max_cluster_learned / (n / B) */
  double imbalance_zscore;       /* max_cluster_zscore / (n / B), 0 if not measured */
  double loss_first, loss_last;  /* loss on minibatch 0 before training and of the kept
                                    parameters */
  double train_ms;               /* device time: sample, sample sort, fit, thresholds */
  double first_pass_ms;          /* device time: learned first pass and order check */
  uint32_t* counts;              /* HOST, B words, or NULL: cluster sizes of the learned first
                                    pass (set by the caller; left in place) */
  zsort_mlp_params* params_out;  /* DEVICE or NULL (set by the caller; left in place): receives
                                    the parameters the first pass used, for reuse through
                                    zsort_learned_config.params with smin_out / smax_out */
  uint64_t smin_out, smax_out;   /* their normalisation range */
} zsort_learned_report;

int zsort_default_learned_config(zsort_learned_config* lcfg);
int zsort_stable_learned(uint64_t* keys, void* payload, int payload_bytes, size_t n,
                         const zsort_config* cfg, const zsort_learned_config* lcfg,
                         zsort_learned_report* report, void* stream);

/*
 * Parity/debug entries of the learned map; all synchronous, all pointers
 * DEVICE unless noted.
 *   zsort_learned_sample  out[i] = keys[i * stride + (SplitMix64 offset)],
 *                         i < n / stride, each offset in [0, stride)
 *   zsort_mlp_forward     f(u(keys[i])) into f_out and its cluster among
 *                         `buckets` into cluster_out (either may be NULL)
 *   zsort_mlp_thresholds  thr_out[b - 1] = t_b for b = 1..nt, 0 after nt
 *                         (buckets - 1 words); *nt_out (host) = nt
 *   zsort_mlp_init        the initialisation above from a sorted sample of m
 *                         keys (range: its first and last key)
 *   zsort_mlp_grad        gradient of the mean squared error over the whole
 *                         sorted sample (targets: mid-ranks, inputs: u of
 *                         the sample's own range) into grad_out[0, 1153) and
 *                         the loss into grad_out[1153], binary64
 *   zsort_mlp_train       params (in place) after `steps` Adam steps as in
 *                         zsort_stable_learned (without its keep-the-better
 *                         rule); losses_out (host, may be NULL) = the loss
 *                         of the first and of the last step's minibatch,
 *                         each before its update
 */
int zsort_learned_sample(const uint64_t* keys, size_t n, int32_t stride, uint64_t seed,
                         uint64_t* out, void* stream);
int zsort_mlp_forward(const zsort_mlp_params* params, const uint64_t* keys, size_t q, uint64_t smin,
                      uint64_t smax, int32_t buckets, float* f_out, uint32_t* cluster_out,
                      void* stream);
int zsort_mlp_thresholds(const zsort_mlp_params* params, uint64_t smin, uint64_t smax, int32_t buckets,
                         uint64_t* thr_out, int32_t* nt_out, void* stream);
int zsort_mlp_init(const uint64_t* sorted_sample, size_t m, zsort_mlp_params* params_out,
                   void* stream);
int zsort_mlp_grad(const zsort_mlp_params* params, const uint64_t* sorted_sample, size_t m, double* grad_out,
                   void* stream);
int zsort_mlp_train(zsort_mlp_params* params, const uint64_t* sorted_sample, size_t m, int32_t steps,
                    int32_t batches, double lr, double* losses_out, void* stream);

/* Frees every workspace the library allocated (caller workspaces are left
 * alone) and drops cached graphs (synchronises the device). */
int zsort_release(void);

/* Last hipError_t seen by the library (0 if none). */
int zsort_last_hip_error(void);

/* Static description of a status code. */
const char* zsort_strerror(int status);

#ifdef __cplusplus
}
#endif
#endif /* ZSORT_H */
