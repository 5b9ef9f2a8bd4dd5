// zsort_api.cpp -- C-ABI of the zSort library: argument checks, workspace
// planning and caching (one workspace per stream), and the launch sequence of
// the breadth-first recursion.  All sorting work happens in the HIP kernels
// of zsort_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "zsort.h"
#include "zsort_internal.h"

namespace zs {
hipError_t launch_reset(const Ws& ws, hipStream_t st);
hipError_t launch_clear_rows(const Ws& ws, int grid, hipStream_t st);
hipError_t scratch_address(int dev, void** out);
hipError_t launch_init_runs(const Ws& ws, const uint32_t* runs, const uint32_t* nruns, int grid,
                            hipStream_t st);
hipError_t launch_split128(const uint64_t* keys, const uint32_t* payload, uint64_t n, int sgn,
                           uint64_t* hi, uint64_t* second, uint32_t* nruns, hipStream_t st);
hipError_t launch_gather_runs(const uint64_t* keys, const uint64_t* hi, uint64_t n, uint64_t* lo,
                              uint32_t* payload, uint32_t* runs, uint32_t* nruns, hipStream_t st);
hipError_t launch_final128(uint64_t* keys, uint64_t n, int sgn, const uint64_t* hi,
                           const uint64_t* lo, hipStream_t st);
hipError_t launch_check_sorted(const uint64_t* keys, uint64_t n, uint32_t* flag, int grid,
                               hipStream_t st);
hipError_t launch_flip(uint64_t* keys, uint64_t n, int grid, hipStream_t st);
hipError_t launch_init_single(const Ws& ws, uint64_t n, hipStream_t st);
hipError_t launch_init_segments(const Ws& ws, const int64_t* off, int32_t nseg, uint64_t n,
                                hipStream_t st);
hipError_t launch_stage(const Ws& ws, int L, int stage, int grid, hipStream_t st);
int stage_blocks_per_cu(int k, int pw, int tile, int stage);
// learned partition map (zsort_learned.hip)
hipError_t launch_init_learned(const Ws& ws, uint64_t n, hipStream_t st);
hipError_t launch_reset_lists(const Ws& ws, int slot, hipStream_t st);
hipError_t launch_lfine_hist(const uint64_t* x, uint64_t n, const uint64_t* thr, const LRes* res,
                             int B, uint32_t* counts, hipStream_t st);
hipError_t launch_lsample(const uint64_t* x, uint64_t m, uint32_t stride, uint64_t seed,
                          uint64_t* out, hipStream_t st);
hipError_t launch_lprep(const uint64_t* s, uint64_t m, double* U, float* Y, LRes* res,
                        hipStream_t st);
hipError_t launch_lset_range(LRes* res, uint64_t smin, uint64_t smax, hipStream_t st);
hipError_t launch_linit(const uint64_t* s, uint64_t m, MlpP* par, LRes* res, hipStream_t st);
hipError_t launch_lthr_check(const uint64_t* thr, LRes* res, hipStream_t st);
hipError_t launch_ladam_reset(double* adam, LRes* res, hipStream_t st);
size_t lpart_floats(uint64_t m, uint32_t nb);
hipError_t launch_ltrain(const double* U, const float* Y, uint64_t m, uint32_t nb, uint32_t step,
                         MlpP* par, double* adam, float* part, LRes* res, double lr, int mode,
                         double* gout, hipStream_t st);
hipError_t launch_lthresh(const MlpP* par, int B, LRes* res, uint64_t* thr, hipStream_t st);
hipError_t launch_lhist_sample(const double* U, uint64_t m, const MlpP* par, int B,
                               uint32_t* counts, hipStream_t st);
hipError_t launch_lkeep(MlpP* par, const MlpP* par0, const double* g0, const double* g1,
                        const uint32_t* hc0, const uint32_t* hc1, int B, LRes* res,
                        hipStream_t st);
hipError_t launch_lforward(const MlpP* par, const uint64_t* x, uint64_t q, const LRes* res, int B,
                           float* fout, uint32_t* cout, hipStream_t st);
hipError_t launch_lcheck(const uint64_t* y, const uint32_t* bst, uint64_t n, int B, uint64_t* bmin,
                         uint64_t* bmax, LRes* res, int grid, hipStream_t st);
hipError_t launch_lmaxcount(const uint32_t* bst, uint64_t n, int B, uint64_t* out, hipStream_t st);
hipError_t launch_lcounts(const uint32_t* bst, uint64_t n, int B, uint32_t* counts,
                          hipStream_t st);
}  // namespace zs

namespace {

using zs::Ws;

struct Shape {
  uint64_t n = 0;
  int pw = 0, k = 0, cutoff = 0, chunk = 0, tile = 0;
  int kfirst = 0;  // clusters of a learned first pass (0: none)
  int fuse = 0;    // fused statistics: the child-of-cluster array is laid out
  int64_t nseg = 0;
  int64_t trace_cap = 0, trace_hist_cap = 0;
  bool operator==(const Shape& o) const {
    return n == o.n && pw == o.pw && k == o.k && cutoff == o.cutoff && chunk == o.chunk &&
           tile == o.tile && kfirst == o.kfirst && fuse == o.fuse &&
           nseg == o.nseg && trace_cap == o.trace_cap && trace_hist_cap == o.trace_hist_cap;
  }
};

struct Layout {
  size_t off_ctl, off_keys, off_pay, off_segs[2], off_work[2], off_leaves[2], off_leavesw[2],
      off_leavesm[2], off_leavesx[2],
      off_hard[2],
      off_status, off_arrive[2], off_part,
      off_bstart, off_subpre, off_tiles[2], off_trace, off_thist, total;
  size_t off_child, off_facc;   // fused statistics only (has_child)
  bool has_child;
  size_t status_bytes;
  uint32_t seg_cap, work_cap, leaf_cap, status_cap, tile_cap;
};

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// smallest caller workspace accepted: the control block
size_t zs_min_workspace() { return align_up(sizeof(zs::Ctl), 256); }

Layout plan(const Shape& s) {
  Layout L{};
  const uint64_t n = s.n, ch = (uint64_t)s.chunk;
  const uint64_t seg_cap = n / ((uint64_t)s.cutoff + 1) + 1;
  const uint64_t nchunks = (n + ch - 1) / ch;
  const uint64_t work_cap = nchunks + seg_cap;
  // scan rows of one level: a segment of nch > 1 chunks holds more than
  // (nch - 1) * chunk keys, so nch < 2 * count / chunk, and it takes at most
  // 1.5 * nch rows (items + units): < 3 * count / chunk over the level
  const uint64_t status_cap = 3 * nchunks + 2;
  // leaf jobs of one level: runs (<= children + segments), windows of kWindow
  // keys, leaves above kWindow (each may also end a group), copy pieces
  const uint64_t leaf_cap = 4 * seg_cap + 4 * (n / zs::kWindow) + n / zs::kCopyChunk +
                            (uint64_t)s.nseg + 64;
  L.seg_cap = (uint32_t)seg_cap;
  L.work_cap = (uint32_t)work_cap;
  L.leaf_cap = (uint32_t)leaf_cap;
  L.status_cap = (uint32_t)status_cap;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = align_up(o, 256);
    o = at + bytes;
    return at;
  };
  L.off_ctl = take(sizeof(zs::Ctl));
  L.off_keys = take(n * 8);
  L.off_pay = take(n * (size_t)s.pw);
  for (int i = 0; i < 2; ++i) {
    L.off_segs[i] = take(seg_cap * sizeof(zs::Seg));
    L.off_work[i] = take(work_cap * 8);
    L.off_leaves[i] = take(leaf_cap * sizeof(zs::Leaf));
    L.off_leavesw[i] = take(leaf_cap * sizeof(zs::Leaf));
    L.off_leavesm[i] = take(leaf_cap * sizeof(zs::Leaf));
    L.off_leavesx[i] = take(leaf_cap * sizeof(zs::Leaf));
    L.off_hard[i] = take(leaf_cap * sizeof(zs::Leaf));
  }
  // scan rows [row][k]; a learned first pass has one root of nchunks work
  // items with kfirst clusters each
  L.status_bytes = std::max<size_t>(status_cap * (size_t)s.k,
                                    ((size_t)zs::status_rows((uint32_t)nchunks) + 1) * (size_t)s.kfirst) * 8;
  L.off_status = take(L.status_bytes);
  for (int i = 0; i < 2; ++i) L.off_arrive[i] = take(status_cap * 4);
  L.off_part = take(work_cap * 10 * 8);
  L.off_bstart = take(std::max<size_t>(seg_cap * (size_t)s.k, (size_t)s.kfirst) * 4);
  L.has_child = s.fuse != 0;
  L.off_child = L.has_child ? take(seg_cap * (size_t)s.k * 4) : 0;
  L.off_facc = L.has_child ? take(seg_cap * 10 * 8) : 0;
  // 8192-key tiles: one row of k 16-bit prefix counts per 8192 keys
  const size_t krow = std::max<size_t>((size_t)s.k, s.kfirst <= 1024 ? (size_t)s.kfirst : 0);
  L.off_subpre = take(s.tile == 8192 ? ((n >> 13) + 2) * krow * 2 : 0);
  // and the tile lists: at most one partial tile per segment
  L.tile_cap = s.tile == 8192 ? (uint32_t)((n >> 13) + seg_cap + 2) : 0u;
  for (int i = 0; i < 2; ++i) L.off_tiles[i] = take((size_t)L.tile_cap * 8);
  L.off_trace = take((size_t)s.trace_cap * sizeof(zs::TraceRec));
  L.off_thist = take((size_t)s.trace_hist_cap * 4);
  L.total = align_up(o, 256);
  return L;
}

// cached hipGraph of one whole sort: the kernels' arguments (caller's buffers,
// workspace layout, configuration) are baked into the graph
struct GraphKey {
  const void* keys;
  const void* pay;
  const void* off;
  uint64_t n;
  int32_t nseg;
  int pw, k, cutoff, maxz, chunk, tile, flags, count_range;
  bool operator<(const GraphKey& o) const {
    return std::tie(keys, pay, off, n, nseg, pw, k, cutoff, maxz, chunk, tile, flags, count_range) <
           std::tie(o.keys, o.pay, o.off, o.n, o.nseg, o.pw, o.k, o.cutoff, o.maxz, o.chunk, o.tile,
                    o.flags, o.count_range);
  }
};

struct Workspace {
  int device = -1;
  char* base = nullptr;
  size_t bytes = 0;
  bool user = false;       // base is the caller's memory (zsort_set_workspace): never freed
  bool rows_dirty = true;  // the scan-row region may hold stale words of another layout
  Shape shape;
  Layout lay{};
  bool laid_out = false;
  uint64_t calls = 0;
  // last call
  uint64_t last_n = 0;
  int last_pw = 0;
  bool has_last = false;
  // per-kernel event timing (zsort_profile_begin / _end)
  bool prof = false;
  uint32_t prof_mask = 0;  // kernel kinds that are timed (bit = stage)
  // pacing of level launches: the next level's segment count, stored by
  // the kernels with the call's token (h_pace); the learned form hands its
  // first levels' counts over by copies and events instead (h_nseg, lvl_ev)
  uint64_t* h_pace = nullptr;  // pinned, kMaxLevels + 1 words
  uint32_t pace_seq = 0;
  uint32_t* h_nseg = nullptr;  // pinned, kMaxLevels + 1 words
  hipEvent_t lvl_ev[zs::kMaxLevels] = {};
  bool lvl_ev_ok = false;
  // the local sorts of a level run on a second stream beside the next level:
  // an event after each level's scatter (the local sorts wait for it) and
  // after each level's local sorts (level L + 2 waits for those of level L)
  hipStream_t side = nullptr;
  hipEvent_t scat_ev[zs::kMaxLevels] = {};
  hipEvent_t loc_ev[zs::kMaxLevels] = {};
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<int> ev_stage;  // stage of each (start, end) pair
  // extra algorithmic bytes of the last call (learned first pass)
  double last_extra_bytes = 0.0;
  // graph mode
  hipStream_t cap_stream = nullptr;
  std::map<GraphKey, hipGraphExec_t> graphs;
};

void drop_graphs(Workspace* w) {
  for (auto& kv : w->graphs) (void)hipGraphExecDestroy(kv.second);
  w->graphs.clear();
}

hipError_t next_event(Workspace* w, hipEvent_t* ev) {
  if (w->ev_used == w->ev_pool.size()) {
    // timing only: no system-scope fence (cache write-back and invalidate)
    // when the event is recorded, which would slow the kernels around it
    hipEvent_t e;
    hipError_t r = hipEventCreateWithFlags(&e, hipEventDisableSystemFence);
    if (r != hipSuccess) return r;
    w->ev_pool.push_back(e);
  }
  *ev = w->ev_pool[w->ev_used++];
  return hipSuccess;
}

// launches one stage, bracketed by events when the stream is being profiled
hipError_t stage(Workspace* w, const Ws& ws, int L, int st_id, int grid, hipStream_t st) {
  if (!w->prof || !((w->prof_mask >> st_id) & 1u)) return zs::launch_stage(ws, L, st_id, grid, st);
  hipEvent_t a, b;
  hipError_t e = next_event(w, &a);
  if (e == hipSuccess) e = next_event(w, &b);
  if (e == hipSuccess) e = hipEventRecord(a, st);
  if (e == hipSuccess) e = zs::launch_stage(ws, L, st_id, grid, st);
  if (e == hipSuccess) e = hipEventRecord(b, st);
  if (e == hipSuccess) w->ev_stage.push_back(st_id);
  return e;
}

std::mutex g_mu;
std::unordered_map<hipStream_t, Workspace*> g_ws;
std::unordered_map<hipStream_t, Workspace*> g_ws_aux;  // sorts of the learned map's key sample
int g_last_hip = 0;
int g_cu_count = 0;

int hip_fail(hipError_t e) {
  g_last_hip = (int)e;
  if (e == hipErrorOutOfMemory) return ZSORT_ENOMEM;
  return ZSORT_EHIP;
}

bool capturing(hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess) return false;
  return cs != hipStreamCaptureStatusNone;
}

int check_cfg(const zsort_config* c) {
  if (c->k < 16 || c->k > zs::kKMax) return ZSORT_EINVAL;
  if (c->cutoff < 1 || c->cutoff > zs::kBigCap) return ZSORT_EINVAL;
  if (c->max_zlevels < 0 || c->max_zlevels > 16) return ZSORT_EINVAL;
  if (c->chunk < 2048 || c->chunk > (1 << 20) || c->chunk % 2048) return ZSORT_EINVAL;
  if (c->tile != 2048 && c->tile != 4096 && c->tile != 8192) return ZSORT_EINVAL;
  if (c->tile > 2048 && (c->k > 1024 || c->chunk % c->tile)) return ZSORT_EINVAL;
  if (c->tile == 8192 && c->chunk > 65536) return ZSORT_EINVAL;
  if (c->count_range < 0 || c->count_range > c->k) return ZSORT_EINVAL;
  return ZSORT_OK;
}

// fused statistics: asked for, and with k <= 1024 (a cluster per thread or
// more threads per cluster in the scatter's workgroup)
bool fused_on(const zsort_config& c) {
  return (c.flags & ZSORT_FLAG_FUSED_STATS) != 0 && c.k <= 1024;
}

int floor_log2(int k) {
  int lb = 0;
  while ((2 << lb) <= k) ++lb;
  return lb;
}

int levels_for(const zsort_config& c) {
  const int lb = floor_log2(c.k);
  const int L = c.max_zlevels + (64 + lb - 1) / lb + 2;
  return std::min(L, zs::kMaxLevels);
}

size_t g_alloc_limit = 0;  // zsort_set_alloc_limit: largest device allocation allowed (0: any)

hipError_t dev_alloc(void** p, size_t bytes) {
  if (g_alloc_limit && bytes > g_alloc_limit) return hipErrorOutOfMemory;
  return hipMalloc(p, bytes);
}

// Finds (or grows) the stream's workspace and lays it out for `s`.  Under
// stream capture a new layout is accepted as long as it fits the memory the
// workspace already has (nothing is allocated while a stream is captured).
// A caller's workspace (zsort_set_workspace) is never grown: a shape that
// does not fit returns ZSORT_ENOMEM.
int acquire(hipStream_t st, const Shape& s, Workspace** out, int slot = 0) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e);
  if (!g_cu_count) {
    e = hipDeviceGetAttribute(&g_cu_count, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e);
  }
  Workspace*& w = slot ? g_ws_aux[st] : g_ws[st];
  if (!w) w = new Workspace();
  if (w->device != -1 && w->device != dev) return ZSORT_EINVAL;  // stream of another device
  const Layout L = plan(s);
  const bool same = w->laid_out && w->shape == s;
  if (!same) {
    if (L.total > w->bytes) {
      if (w->user) return ZSORT_ENOMEM;
      if (capturing(st)) return ZSORT_ECAPTURE;
      drop_graphs(w);   // they name the old buffer
      if (w->base) {
        e = hipFree(w->base);
        if (e != hipSuccess) return hip_fail(e);
        w->base = nullptr;
        w->bytes = 0;
      }
      void* p = nullptr;
      e = dev_alloc(&p, L.total);
      if (e != hipSuccess) return hip_fail(e);
      w->base = (char*)p;
      w->bytes = L.total;
      e = hipMemsetAsync(w->base, 0, sizeof(zs::Ctl), st);
      if (e != hipSuccess) return hip_fail(e);
    }
    // (graphs of other shapes stay valid: a shape's layout in a given buffer
    // is always the same)
    w->rows_dirty = true;   // the row region now covers memory of the old layout
    w->device = dev;
    w->shape = s;
    w->lay = L;
    w->laid_out = true;
  }
  *out = w;
  return ZSORT_OK;
}

Ws ws_at(char* base, const Layout& L, const Shape& sh, uint64_t* keys, void* pay,
         const zsort_config& c, int pw);

Ws make_ws(Workspace* w, uint64_t* keys, void* pay, const zsort_config& c, int pw) {
  return ws_at(w->base, w->lay, w->shape, keys, pay, c, pw);
}

// kernel arguments of a workspace laid out as L at `base`
Ws ws_at(char* base, const Layout& L, const Shape& sh, uint64_t* keys, void* pay,
         const zsort_config& c, int pw) {
  Ws ws;
  std::memset(&ws, 0, sizeof ws);
  ws.keys[0] = keys;
  ws.keys[1] = (uint64_t*)(base + L.off_keys);
  ws.pay[0] = pay;
  ws.pay[1] = pw ? (void*)(base + L.off_pay) : nullptr;
  for (int i = 0; i < 2; ++i) {
    ws.segs[i] = (zs::Seg*)(base + L.off_segs[i]);
    ws.work[i] = (uint64_t*)(base + L.off_work[i]);
    ws.leaves[i] = (zs::Leaf*)(base + L.off_leaves[i]);
    ws.leavesw[i] = (zs::Leaf*)(base + L.off_leavesw[i]);
    ws.leavesm[i] = (zs::Leaf*)(base + L.off_leavesm[i]);
    ws.leavesx[i] = (zs::Leaf*)(base + L.off_leavesx[i]);
    ws.hard[i] = (zs::Leaf*)(base + L.off_hard[i]);
  }
  ws.status = (uint64_t*)(base + L.off_status);
  for (int i = 0; i < 2; ++i) ws.arrive[i] = (uint32_t*)(base + L.off_arrive[i]);
  ws.part = (uint64_t*)(base + L.off_part);
  ws.bstart = (uint32_t*)(base + L.off_bstart);
  ws.child_of = L.has_child ? (uint32_t*)(base + L.off_child) : nullptr;
  ws.facc = L.has_child ? (uint64_t*)(base + L.off_facc) : nullptr;
  ws.subpre = (uint16_t*)(base + L.off_subpre);
  for (int i = 0; i < 2; ++i) ws.tiles[i] = (uint64_t*)(base + L.off_tiles[i]);
  ws.ctl = (zs::Ctl*)(base + L.off_ctl);
  ws.trace = sh.trace_cap ? (zs::TraceRec*)(base + L.off_trace) : nullptr;
  ws.trace_hist = sh.trace_hist_cap ? (uint32_t*)(base + L.off_thist) : nullptr;
  ws.trace_cap = (uint32_t)sh.trace_cap;
  ws.trace_hist_cap = (uint32_t)sh.trace_hist_cap;
  ws.seg_cap = L.seg_cap;
  ws.work_cap = L.work_cap;
  ws.tile_cap = L.tile_cap;
  ws.leaf_cap = L.leaf_cap;
  ws.status_cap = L.status_cap;
  ws.status_words = L.status_bytes / 8;
  ws.force_clear = 0;
  ws.p.k = c.k;
  ws.p.lb = floor_log2(c.k);
  ws.p.cutoff = c.cutoff;
  ws.p.max_zlevels = c.max_zlevels;
  ws.p.chunk = c.chunk;
  ws.p.tile = c.tile;
  ws.p.pw = pw;
  ws.p.count_range = c.count_range;
  ws.p.fuse = (L.has_child && fused_on(c)) ? 1 : 0;
  return ws;
}

// grid of a stage: every compute unit filled to the kernel's occupancy
int grid_size(int k, int pw, int tile, int stage) {
  static std::mutex mu;
  static int cache[4 * 16 * 4 * 8] = {};   // (k class, payload bytes, tile class, stage)
  const int kc = k <= 256 ? 0 : (k <= 512 ? 1 : (k <= 1024 ? 2 : 3));
  const int tc = tile == 8192 ? 2 : (tile == 4096 ? 1 : 0);
  const int key = kc | (pw << 2) | (tc << 6) | (stage << 8);
  std::lock_guard<std::mutex> lk(mu);
  int per = cache[key];
  if (!per) {
    per = std::min(8, zs::stage_blocks_per_cu(k, pw, tile, stage));
    cache[key] = per;
  }
  if (stage == zs::STAGE_FINALIZE) return std::max(1, g_cu_count) * 4;
  return std::max(1, g_cu_count) * per;
}

struct Call {
  uint64_t* keys;
  void* pay;
  int pw;
  uint64_t n;
  const int64_t* off;  // segmented form
  int32_t nseg;
  zsort_config cfg;
  int64_t trace_cap, hist_cap;
  bool level0_only;
  int slot = 0;    // 1: the auxiliary workspace (sample sorts of the learned map)
  int kfirst = 0;  // clusters of a learned first pass the workspace must also hold
  // subproblems given as a device list of (start, length) pairs instead of
  // one array or a partition: *nruns of them, at most runs_cap
  const uint32_t* runs = nullptr;
  const uint32_t* nruns = nullptr;
  int64_t runs_cap = 0;
};

// pinned count buffer and per-level events, created once per workspace
bool pacing_ready(Workspace* w) {
  if (w->lvl_ev_ok) return true;
  if (!w->h_nseg) {
    void* p = nullptr;
    if (hipHostMalloc(&p, (zs::kMaxLevels + 1) * sizeof(uint32_t), hipHostMallocDefault) !=
        hipSuccess)
      return false;
    w->h_nseg = (uint32_t*)p;
  }
  if (!w->h_pace) {
    // coherent (fine-grained) memory: the device's stores reach it while the
    // kernels still run, and the host polls it
    void* p = nullptr;
    const size_t bytes = (zs::kMaxLevels + 1) * sizeof(uint64_t);
    if (hipHostMalloc(&p, bytes, hipHostMallocCoherent) != hipSuccess &&
        hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess)
      return false;
    std::memset(p, 0, (zs::kMaxLevels + 1) * sizeof(uint64_t));
    w->h_pace = (uint64_t*)p;
  }
  for (int i = 0; i < zs::kMaxLevels; ++i) {
    if (!w->lvl_ev[i] && hipEventCreateWithFlags(&w->lvl_ev[i], hipEventDisableTiming) != hipSuccess)
      return false;
    if (!w->scat_ev[i] &&
        hipEventCreateWithFlags(&w->scat_ev[i], hipEventDisableTiming | hipEventDisableSystemFence) !=
            hipSuccess)
      return false;
    if (!w->loc_ev[i] &&
        hipEventCreateWithFlags(&w->loc_ev[i], hipEventDisableTiming | hipEventDisableSystemFence) !=
            hipSuccess)
      return false;
  }
  if (!w->side && hipStreamCreateWithFlags(&w->side, hipStreamNonBlocking) != hipSuccess)
    return false;
  w->lvl_ev_ok = true;
  return true;
}

hipError_t enqueue(Workspace* w, const Ws& ws, const Call& c, hipStream_t st);

// Scan rows of a new layout are cleared before the call's kernels: at once
// on the stream, or -- while the stream is being captured -- by the set-up
// kernel of every replay of the caller's graph (k_reset is told to).
hipError_t prepare_rows(Workspace* w, Ws* ws, hipStream_t st) {
  if (!w->rows_dirty) return hipSuccess;
  if (capturing(st)) {
    ws->force_clear = 1;
    return hipSuccess;
  }
  hipError_t e = zs::launch_clear_rows(*ws, std::max(1, g_cu_count) * 4, st);
  if (e == hipSuccess) w->rows_dirty = false;
  return e;
}

int run(const Call& c, hipStream_t st, Workspace** wout) {
  Shape s;
  s.n = c.n;
  s.pw = c.pw;
  s.k = c.cfg.k;
  s.cutoff = c.cfg.cutoff;
  s.chunk = c.cfg.chunk;
  s.tile = c.cfg.tile;
  s.fuse = fused_on(c.cfg) ? 1 : 0;
  s.nseg = c.off ? c.nseg : (c.runs ? c.runs_cap : 0);
  s.trace_cap = c.trace_cap;
  s.trace_hist_cap = c.hist_cap;
  s.kfirst = c.kfirst;
  Workspace* w = nullptr;
  int rc = acquire(st, s, &w, c.slot);
  if (rc) return rc;
  Ws ws = make_ws(w, c.keys, c.pay, c.cfg, c.pw);
  hipError_t e = prepare_rows(w, &ws, st);
  if (e != hipSuccess) return hip_fail(e);
  const bool graph = (c.cfg.flags & ZSORT_FLAG_GRAPH) && !c.level0_only && !c.trace_cap &&
                     !c.runs && !capturing(st);
  if (graph) {
    GraphKey gk{c.keys, c.pay, c.off, c.n, c.off ? c.nseg : 0, c.pw, c.cfg.k, c.cfg.cutoff,
                c.cfg.max_zlevels, c.cfg.chunk, c.cfg.tile,
                c.cfg.flags & (ZSORT_FLAG_SIGNED | ZSORT_FLAG_FUSED_STATS), c.cfg.count_range};
    auto it = w->graphs.find(gk);
    hipGraphExec_t ex = nullptr;
    if (it != w->graphs.end()) {
      ex = it->second;
    } else {
      if (!w->cap_stream) {
        e = hipStreamCreateWithFlags(&w->cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(e);
      }
      const bool prof = w->prof;
      w->prof = false;
      e = hipStreamBeginCapture(w->cap_stream, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) {
        hipError_t e2 = enqueue(w, ws, c, w->cap_stream);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(w->cap_stream, &g);
        if (e == hipSuccess) e = e2;
        if (e == hipSuccess) e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
      }
      w->prof = prof;
      if (e != hipSuccess) return hip_fail(e);
      w->graphs[gk] = ex;
    }
    e = hipGraphLaunch(ex, st);
    if (e != hipSuccess) return hip_fail(e);
  } else {
    e = enqueue(w, ws, c, st);
    if (e != hipSuccess) return hip_fail(e);
  }
  w->calls++;
  w->last_n = c.n;
  w->last_pw = c.pw;
  w->has_last = true;
  w->last_extra_bytes = 0.0;
  if (wout) *wout = w;
  return ZSORT_OK;
}

hipError_t enqueue_levels(Workspace* w, const Ws& ws, const Call& c, hipStream_t st, int L0,
                          bool beside = true);

// the launch sequence of one sort on stream st (signed keys: the sign bit
// is flipped before and after, so that the unsigned sort orders them)
hipError_t enqueue(Workspace* w, const Ws& ws, const Call& c, hipStream_t st) {
  const bool sgn = (c.cfg.flags & ZSORT_FLAG_SIGNED) != 0;
  const int fgrid = std::max(1, g_cu_count) * 8;
  hipError_t e = sgn ? zs::launch_flip(c.keys, c.n, fgrid, st) : hipSuccess;
  if (e == hipSuccess) e = zs::launch_reset(ws, st);
  if (e == hipSuccess) {
    if (c.runs) e = zs::launch_init_runs(ws, c.runs, c.nruns, std::max(1, g_cu_count) * 4, st);
    else if (c.off) e = zs::launch_init_segments(ws, c.off, c.nseg, c.n, st);
    else e = zs::launch_init_single(ws, c.n, st);
  }
  if (e == hipSuccess) e = enqueue_levels(w, ws, c, st, 0);
  if (e == hipSuccess && sgn) e = zs::launch_flip(c.keys, c.n, fgrid, st);
  return e;
}

// The word level L - 1's histogram pass stores for this call (token): level
// L's segment count and whether level L - 1 has leaf jobs.  Returns
// hipSuccess, or the stream's error.  If the stream drains without the store
// (only a call that failed before that pass ends so), the count is read from
// the device and the leaf jobs are taken to exist.  The stream is queried
// only after 2 ms of waiting (a query can put a marker between the queued
// kernels, a gap of ~5 us).
hipError_t wait_pace(Workspace* w, const Ws& ws, int L, uint32_t token, hipStream_t st,
                     uint32_t* count, bool* leaves) {
  volatile uint64_t* slot = w->h_pace + L;
  auto next = std::chrono::steady_clock::now() + std::chrono::milliseconds(2);
  for (uint32_t spin = 1;; ++spin) {
    uint64_t v = __atomic_load_n(slot, __ATOMIC_ACQUIRE);
    if (zs::pace_token_of(v) == token) {
      *count = (uint32_t)v;
      *leaves = zs::pace_leaves_of(v);
      return hipSuccess;
    }
    if ((spin & 255u) == 0 && std::chrono::steady_clock::now() >= next) {
      next += std::chrono::milliseconds(1);
      const hipError_t q = hipStreamQuery(st);
      if (q == hipErrorNotReady) continue;
      if (q != hipSuccess) return q;
      v = __atomic_load_n(slot, __ATOMIC_ACQUIRE);
      if (zs::pace_token_of(v) == token) {
        *count = (uint32_t)v;
        *leaves = zs::pace_leaves_of(v);
        return hipSuccess;
      }
      *leaves = true;
      return hipMemcpy(count, &ws.ctl->nseg[L & 1], sizeof(uint32_t), hipMemcpyDeviceToHost);
    }
    __builtin_ia32_pause();
  }
}

// levels L0, L0 + 1, ... (L0 > 0: level L0 - 1 ran already; with L0 >= 2
// its segment count was copied to h_nseg[L0 - 1] before event lvl_ev[L0 - 2]);
// beside: local sorts may run beside the next level (below)
hipError_t enqueue_levels(Workspace* w, const Ws& ws, const Call& c, hipStream_t st, int L0,
                          bool beside) {
  hipError_t e = hipSuccess;
  const int levels = c.level0_only ? 1 : levels_for(c.cfg);
  // Pacing: once level L's histogram pass ends, its last workgroup stores
  // level L + 1's segment count and whether level L has leaf jobs.  The host
  // waits for that word while level L's scatter runs, then launches level
  // L's local sorts if it has leaf jobs and level L + 1 if it has segments:
  // no level after the last and no empty local stage is launched.  Under
  // stream capture every level and stage is launched (each kernel without
  // work exits at once).
  const bool paced = !c.level0_only && !capturing(st) && pacing_ready(w);
  Ws wsp = ws;
  uint32_t token = 0;
  if (paced) {
    w->pace_seq = (w->pace_seq + 1u) & 0xFFFFFFu;
    if (w->pace_seq == 0) w->pace_seq = 1;   // 0 would match the zeroed words
    token = w->pace_seq;
    wsp.h_pace = w->h_pace;
    wsp.pace_token = token;
  }
  auto locals = [&](int L, hipStream_t ls) {
    hipError_t r = stage(w, wsp, L, zs::STAGE_LOCAL, grid_size(c.cfg.k, c.pw, c.cfg.tile,
                                                               zs::STAGE_LOCAL), ls);
    if (r == hipSuccess)
      r = stage(w, wsp, L, zs::STAGE_LOCAL_HARD,
                grid_size(c.cfg.k, c.pw, c.cfg.tile, zs::STAGE_LOCAL_HARD), ls);
    return r;
  };
  // Paced, a level's local sorts run on the second stream once its scatter
  // has ended, beside the next level's read passes (moments, statistics,
  // histogram): they read only this level's leaf lists and leaf ranges, which
  // those passes do not touch (the moments pass empties the lists of its own
  // slot only).  The next level's scatter waits for them: beside it (one
  // workgroup per compute unit, most of the LDS) they cost it more than they
  // gain.  The caller's stream waits for the last of them.
  bool on_side[zs::kMaxLevels] = {};
  int last_side = -1;
  auto side_locals = [&](int L) {
    hipError_t r = hipEventRecord(w->scat_ev[L], st);
    if (r == hipSuccess) r = hipStreamWaitEvent(w->side, w->scat_ev[L], 0);
    if (r == hipSuccess) r = locals(L, w->side);
    if (r == hipSuccess) r = hipEventRecord(w->loc_ev[L], w->side);
    if (r == hipSuccess) {
      on_side[L] = true;
      last_side = L;
    }
    return r;
  };
  int pending = -1;   // the level whose local sorts wait for its histogram pass's word
  for (int L = L0; L < levels && e == hipSuccess; ++L) {
    if (pending >= 0) {
      uint32_t nseg = 0;
      bool leaves = true;
      e = wait_pace(w, ws, L, token, st, &nseg, &leaves);
      // (with no level after it, nothing would run beside them)
      if (e == hipSuccess && leaves) e = nseg && beside ? side_locals(pending) : locals(pending, st);
      pending = -1;
      if (e != hipSuccess || nseg == 0) break;
    } else if (paced && L >= 2) {   // the learned form's hand-over
      e = hipEventSynchronize(w->lvl_ev[L - 2]);
      if (e != hipSuccess || w->h_nseg[L - 1] == 0) break;
    }
    for (int sid = zs::STAGE_MOMENTS; sid <= zs::STAGE_SCATTER && e == hipSuccess; ++sid) {
      // the scatter (one workgroup per compute unit, most of the LDS) waits
      // for the previous level's local sorts; the read passes run beside them
      if (sid == zs::STAGE_SCATTER && L >= 1 && on_side[L - 1])
        e = hipStreamWaitEvent(st, w->loc_ev[L - 1], 0);
      if (e == hipSuccess) e = stage(w, wsp, L, sid, grid_size(c.cfg.k, c.pw, c.cfg.tile, sid), st);
    }
    if (e != hipSuccess || c.level0_only) continue;
    if (paced) pending = L;
    else e = locals(L, st);
  }
  if (e == hipSuccess && pending >= 0) {   // the last level launched
    uint32_t nseg = 0;
    bool leaves = true;
    e = wait_pace(w, ws, pending + 1, token, st, &nseg, &leaves);
    if (e == hipSuccess && leaves) e = locals(pending, st);
  }
  if (last_side >= 0) {
    const hipError_t j = hipStreamWaitEvent(st, w->loc_ev[last_side], 0);
    if (e == hipSuccess) e = j;
  }
  return e;
}

// ---- tuned configurations, by shape class -------------------------------
struct TuneKey {
  int ncls, pw, seg;
  bool operator<(const TuneKey& o) const {
    return std::tie(ncls, pw, seg) < std::tie(o.ncls, o.pw, o.seg);
  }
};
std::map<TuneKey, zsort_config> g_tuned;

int n_class(uint64_t n) {
  int c = 0;
  while (c < 63 && (1ull << c) < n) ++c;
  return c;
}

void tune_file_read(const char* path) {
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char line[512];
  while (std::fgets(line, sizeof line, f)) {
    TuneKey tk;
    zsort_config c;
    zsort_default_config(&c);
    if (std::sscanf(line, "%d %d %d %d %d %d %d %d", &tk.ncls, &tk.pw, &tk.seg, &c.k, &c.cutoff,
                    &c.max_zlevels, &c.chunk, &c.tile) == 8 &&
        check_cfg(&c) == ZSORT_OK)
      g_tuned[tk] = c;
  }
  std::fclose(f);
}

void tune_file_write(const char* path) {
  FILE* f = std::fopen(path, "w");
  if (!f) return;
  std::fprintf(f, "# n_class payload_bytes segmented k cutoff max_zlevels chunk tile\n");
  for (auto& kv : g_tuned)
    std::fprintf(f, "%d %d %d %d %d %d %d %d\n", kv.first.ncls, kv.first.pw, kv.first.seg,
                 kv.second.k, kv.second.cutoff, kv.second.max_zlevels, kv.second.chunk,
                 kv.second.tile);
  std::fclose(f);
}

// cfg given: validated as is; cfg NULL: the tuned entry of the class, else defaults
int resolve_cfg(const zsort_config* in, zsort_config* out, uint64_t n = 0, int pw = 0,
                int seg = 0) {
  zsort_default_config(out);
  if (in) {
    *out = *in;
  } else if (n) {
    auto it = g_tuned.find(TuneKey{n_class(n), pw, seg});
    if (it != g_tuned.end()) *out = it->second;
  }
  return check_cfg(out);
}

int common_checks(const uint64_t* keys, const void* pay, int pw, size_t n) {
  if (pw != 0 && pw != 4 && pw != 8) return ZSORT_EINVAL;
  if (n > 0x7FFFFFFFull) return ZSORT_EINVAL;
  if (n > 1 && !keys) return ZSORT_EINVAL;
  if (n > 1 && pw && !pay) return ZSORT_EINVAL;
  return ZSORT_OK;
}


// ---- learned partition map ------------------------------------------------
struct LearnedWs {
  int device = -1;
  char* base = nullptr;
  size_t bytes = 0;
  uint64_t n_cap = 0, m_cap = 0;
  size_t part_cap = 0;
  uint64_t* sample = nullptr;
  double* U = nullptr;
  float* Y = nullptr;
  zs::MlpP* par = nullptr;
  zs::MlpP* par0 = nullptr;  // initial parameters, restored if training does not help
  double* adam = nullptr;
  float* part = nullptr;
  uint64_t* thr = nullptr;
  uint16_t* ids = nullptr;
  uint64_t* bmin = nullptr;
  uint64_t* bmax = nullptr;
  zs::LRes* res = nullptr;
  double* gout = nullptr;
  double* gout1 = nullptr;
  uint32_t* counts = nullptr;
  uint32_t* hc = nullptr;  // sample cluster sizes: [0] initial, [1] trained parameters
  zs::LRes* h_res = nullptr;  // pinned, 2 records: at the order check, after the learned passes
  hipEvent_t ev[6] = {};
};
std::unordered_map<hipStream_t, LearnedWs*> g_lws;

// buffers of the learned map for n keys, m sample keys and the partial sums
// of a training step; grows (and never shrinks) per stream
int lacquire(hipStream_t st, uint64_t n, uint64_t m, size_t part_floats, LearnedWs** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e);
  LearnedWs*& w = g_lws[st];
  if (!w) w = new LearnedWs();
  if (w->device != -1 && w->device != dev) return ZSORT_EINVAL;
  w->device = dev;
  if (!w->h_res) {
    void* p = nullptr;
    e = hipHostMalloc(&p, 2 * sizeof(zs::LRes), hipHostMallocDefault);
    if (e != hipSuccess) return hip_fail(e);
    w->h_res = (zs::LRes*)p;
  }
  for (int i = 0; i < 6; ++i)
    if (!w->ev[i]) {
      e = hipEventCreate(&w->ev[i]);
      if (e != hipSuccess) return hip_fail(e);
    }
  if (w->base && n <= w->n_cap && m <= w->m_cap && part_floats <= w->part_cap) {
    *out = w;
    return ZSORT_OK;
  }
  if (capturing(st)) return ZSORT_ECAPTURE;
  n = std::max(n, w->n_cap);
  m = std::max<uint64_t>(std::max(m, w->m_cap), 1);
  part_floats = std::max<size_t>(std::max(part_floats, w->part_cap), zs::kNP + 1);
  size_t o = 0;
  auto take = [&](size_t b) {
    size_t at = align_up(o, 256);
    o = at + b;
    return at;
  };
  const size_t o_res = take(sizeof(zs::LRes)), o_par = take(sizeof(zs::MlpP)),
               o_par0 = take(sizeof(zs::MlpP)), o_adam = take(2 * zs::kNP * 8),
               o_gout = take((zs::kNP + 1) * 8), o_gout1 = take((zs::kNP + 1) * 8),
               o_thr = take(zs::kKMax * 8), o_bmin = take(zs::kKMax * 8),
               o_bmax = take(zs::kKMax * 8), o_cnt = take(zs::kKMax * 4),
               o_hc = take(2 * zs::kKMax * 4), o_smp = take(m * 8),
               o_u = take(m * 8), o_y = take(m * 4), o_part = take(part_floats * 4),
               o_ids = take(std::max<uint64_t>(n, 1) * 2);
  const size_t total = align_up(o, 256);
  if (w->base) {
    e = hipFree(w->base);
    w->base = nullptr;
    w->bytes = 0;
    if (e != hipSuccess) return hip_fail(e);
  }
  void* p = nullptr;
  e = dev_alloc(&p, total);
  if (e != hipSuccess) return hip_fail(e);
  char* b = (char*)p;
  w->base = b;
  w->bytes = total;
  w->n_cap = n;
  w->m_cap = m;
  w->part_cap = part_floats;
  w->res = (zs::LRes*)(b + o_res);
  w->par = (zs::MlpP*)(b + o_par);
  w->par0 = (zs::MlpP*)(b + o_par0);
  w->adam = (double*)(b + o_adam);
  w->gout = (double*)(b + o_gout);
  w->gout1 = (double*)(b + o_gout1);
  w->thr = (uint64_t*)(b + o_thr);
  w->bmin = (uint64_t*)(b + o_bmin);
  w->bmax = (uint64_t*)(b + o_bmax);
  w->counts = (uint32_t*)(b + o_cnt);
  w->hc = (uint32_t*)(b + o_hc);
  w->sample = (uint64_t*)(b + o_smp);
  w->U = (double*)(b + o_u);
  w->Y = (float*)(b + o_y);
  w->part = (float*)(b + o_part);
  w->ids = (uint16_t*)(b + o_ids);
  e = hipMemsetAsync(w->res, 0, sizeof(zs::LRes), st);
  if (e != hipSuccess) return hip_fail(e);
  *out = w;
  return ZSORT_OK;
}

int check_lcfg(const zsort_learned_config* L) {
  if (L->buckets < 16 || L->buckets > zs::kKMax) return ZSORT_EINVAL;
  if (L->sample_stride < 1 || L->steps < 0 || L->steps > 1000000 || L->batches < 1)
    return ZSORT_EINVAL;
  if (!(L->lr > 0.0) || !(L->lr < 1e6)) return ZSORT_EINVAL;
  if (L->params && L->smin > L->smax) return ZSORT_EINVAL;
  if (L->flags & ~(uint32_t)(ZSORT_LEARNED_DIRECT | ZSORT_LEARNED_ZSCORE_DIAG | ZSORT_LEARNED_VERIFY))
    return ZSORT_EINVAL;
  return ZSORT_OK;
}

// Ws of the learned first pass: B clusters, thresholds (or per-key MLP)
Ws first_pass_ws(const Ws& ws, const LearnedWs* lw, int B, bool direct) {
  Ws w0 = ws;
  w0.p.k = B;
  w0.p.lb = floor_log2(B);
  w0.p.fuse = 0;   // (the child-of-cluster array is laid out for the later levels' k)
  if (B > 1024) w0.p.tile = 2048;
  w0.lm.thr = lw->thr;
  w0.lm.par = lw->par;
  w0.lm.ids = lw->ids;
  w0.lm.res = lw->res;
  w0.lm.direct = direct ? 1 : 0;
  return w0;
}
}  // namespace

extern "C" {

int zsort_default_config(zsort_config* cfg) {
  if (!cfg) return ZSORT_EINVAL;
  std::memset(cfg, 0, sizeof *cfg);
  cfg->k = 1024;
  cfg->cutoff = 2048;
  cfg->max_zlevels = 8;
  cfg->chunk = 16384;
  cfg->tile = 2048;
  cfg->flags = 0;
  return ZSORT_OK;
}

int zsort_stable_ex(uint64_t* keys, void* payload, int payload_bytes, size_t n,
                    const zsort_config* cfg, void* stream) {
  int rc = common_checks(keys, payload, payload_bytes, n);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(g_mu);
  zsort_config c;
  rc = resolve_cfg(cfg, &c, n, payload_bytes, 0);
  if (rc) return rc;
  if (n <= 1) return ZSORT_OK;
  Call call{keys, payload_bytes ? payload : nullptr, payload_bytes, (uint64_t)n, nullptr, 0, c,
            0, 0, false};
  return run(call, (hipStream_t)stream, nullptr);
}

int zsort_stable(uint64_t* keys, uint32_t* payload, size_t n, void* stream) {
  return zsort_stable_ex(keys, payload, payload ? 4 : 0, n, nullptr, stream);
}

int zsort_stable_p64(uint64_t* keys, uint64_t* payload, size_t n, void* stream) {
  return zsort_stable_ex(keys, payload, payload ? 8 : 0, n, nullptr, stream);
}

int zsort_stable_noalloc(uint64_t* keys, void* payload, int payload_bytes, size_t n,
                         const zsort_config* cfg, void* stream) {
  int rc = common_checks(keys, payload, payload_bytes, n);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(g_mu);
  zsort_config c;
  rc = resolve_cfg(cfg, &c, n, payload_bytes, 0);
  if (rc) return rc;
  if (c.flags & ZSORT_FLAG_GRAPH) return ZSORT_EUNSUPPORTED;
  if (n <= 1) return ZSORT_OK;
  Shape s;
  s.n = n;
  s.pw = payload_bytes;
  s.k = c.k;
  s.cutoff = c.cutoff;
  s.chunk = c.chunk;
  s.tile = c.tile;
  s.fuse = fused_on(c) ? 1 : 0;
  const Layout L = plan(s);
  if (L.total > zs::kScratchBytes) return ZSORT_ETOOLARGE;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e);
  if (!g_cu_count) {
    e = hipDeviceGetAttribute(&g_cu_count, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e);
  }
  void* base = nullptr;
  e = zs::scratch_address(dev, &base);
  if (e != hipSuccess) return hip_fail(e);
  hipStream_t st = (hipStream_t)stream;
  Ws ws = ws_at((char*)base, L, s, keys, payload_bytes ? payload : nullptr, c, payload_bytes);
  // the array keeps the last call's contents, perhaps in another layout: the
  // set-up kernel clears the scan rows (the control block is reset by k_reset)
  ws.force_clear = 1;
  // every level is launched (no pacing: that would need pinned host memory
  // and events); kernels of levels without work exit at once
  const bool sgn = (c.flags & ZSORT_FLAG_SIGNED) != 0;
  const int fgrid = std::max(1, g_cu_count) * 8;
  e = sgn ? zs::launch_flip(keys, n, fgrid, st) : hipSuccess;
  if (e == hipSuccess) e = zs::launch_reset(ws, st);
  if (e == hipSuccess) e = zs::launch_init_single(ws, n, st);
  const int levels = levels_for(c);
  for (int lv = 0; lv < levels && e == hipSuccess; ++lv)
    for (int sid = 0; sid < zs::NSTAGES && e == hipSuccess; ++sid)
      e = zs::launch_stage(ws, lv, sid, grid_size(c.k, payload_bytes, c.tile, sid), st);
  if (e == hipSuccess && sgn) e = zs::launch_flip(keys, n, fgrid, st);
  if (e != hipSuccess) return hip_fail(e);
  return ZSORT_OK;
}

int zsort_stable_segmented(uint64_t* keys, void* payload, int payload_bytes, size_t n,
                           const int64_t* seg_offsets, int32_t num_segments,
                           const zsort_config* cfg, void* stream) {
  int rc = common_checks(keys, payload, payload_bytes, n);
  if (rc) return rc;
  if (num_segments < 0 || (num_segments > 0 && !seg_offsets)) return ZSORT_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  zsort_config c;
  rc = resolve_cfg(cfg, &c, n, payload_bytes, 1);
  if (rc) return rc;
  if (n <= 1 || num_segments == 0) return ZSORT_OK;
  Call call{keys, payload_bytes ? payload : nullptr, payload_bytes, (uint64_t)n, seg_offsets,
            num_segments, c, 0, 0, false};
  return run(call, (hipStream_t)stream, nullptr);
}

// ---- 128-bit keys ----------------------------------------------------------
}  // extern "C"
namespace {
// buffers of the two stages of a 128-bit sort, per stream (grown, never shrunk)
struct WideWs {
  char* base = nullptr;
  uint64_t n_cap = 0;
  uint64_t* hi = nullptr;
  uint64_t* lo = nullptr;   // first the word the high words carry, then the low words
  uint32_t* runs = nullptr;
  uint32_t* counters = nullptr;  // [0] runs, [2..3] keys in runs (u64)
};
std::unordered_map<hipStream_t, WideWs*> g_wide;

int wide_acquire(hipStream_t st, uint64_t n, WideWs** out) {
  WideWs*& w = g_wide[st];
  if (!w) w = new WideWs();
  if (w->base && n <= w->n_cap) {
    *out = w;
    return ZSORT_OK;
  }
  if (capturing(st)) return ZSORT_ECAPTURE;
  size_t o = 0;
  auto take = [&](size_t b) {
    size_t at = align_up(o, 256);
    o = at + b;
    return at;
  };
  const uint64_t nr = n / 65 + 1;   // runs of > 64 keys
  const size_t o_hi = take(n * 8), o_lo = take(n * 8), o_runs = take(nr * 8), o_cnt = take(16);
  if (w->base) {
    hipError_t e = hipFree(w->base);
    w->base = nullptr;
    w->n_cap = 0;
    if (e != hipSuccess) return hip_fail(e);
  }
  void* p = nullptr;
  hipError_t e = dev_alloc(&p, align_up(o, 256));
  if (e != hipSuccess) return hip_fail(e);
  char* b = (char*)p;
  w->base = b;
  w->n_cap = n;
  w->hi = (uint64_t*)(b + o_hi);
  w->lo = (uint64_t*)(b + o_lo);
  w->runs = (uint32_t*)(b + o_runs);
  w->counters = (uint32_t*)(b + o_cnt);
  *out = w;
  return ZSORT_OK;
}

// levels with work in the control block of the stream's workspace (the
// stream must have reached the call)
int ctl_levels(hipStream_t st, int32_t* levels, int32_t* err) {
  auto it = g_ws.find(st);
  if (it == g_ws.end()) return ZSORT_EINVAL;
  zs::Ctl ctl;
  hipError_t e = hipMemcpy(&ctl, it->second->base + it->second->lay.off_ctl, sizeof ctl,
                           hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e);
  int L = 0;
  for (int i = 0; i < zs::kMaxLevels; ++i)
    if (ctl.lvl_mkeys[i] || ctl.lvl_fkeys[i]) L = i + 1;
  *levels = L;
  *err |= (int32_t)ctl.error;
  return ZSORT_OK;
}
}  // namespace
extern "C" {

int zsort_stable_u128(uint64_t* keys, uint32_t* payload, size_t n, const zsort_config* cfg,
                      zsort_u128_report* report, void* stream) {
  if (report) std::memset(report, 0, sizeof *report);
  if (n > 0x7FFFFFFFull || (n > 1 && !keys) || ((uintptr_t)keys & 15u)) return ZSORT_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  zsort_config c;
  int rc = resolve_cfg(cfg, &c, n, 8, 0);   // (the high words carry 8 bytes)
  if (rc) return rc;
  if (c.flags & ZSORT_FLAG_GRAPH) return ZSORT_EUNSUPPORTED;
  if (n <= 1) return ZSORT_OK;
  const int sgn = (c.flags & ZSORT_FLAG_SIGNED) ? 1 : 0;
  c.flags &= ~ZSORT_FLAG_SIGNED;   // the high words are flipped by the split itself
  hipStream_t st = (hipStream_t)stream;
  WideWs* w = nullptr;
  rc = wide_acquire(st, n, &w);
  if (rc) return rc;
  // stage 1: the high words, each carrying its key's low word (no payload)
  // or its payload and position (so that the payload needs no gather later)
  hipError_t e = zs::launch_split128(keys, payload, n, sgn, w->hi, w->lo, w->counters, st);
  if (e != hipSuccess) return hip_fail(e);
  Call hc{w->hi, w->lo, 8, (uint64_t)n, nullptr, 0, c, 0, 0, false};
  rc = run(hc, st, nullptr);
  if (rc) return rc;
  if (report) {
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e);
    rc = ctl_levels(st, &report->levels_high, &report->device_error);
    if (rc) return rc;
  }
  // stage 2: the low words inside every run of equal high words (the key
  // rebased to the run's minimum fits 64 bits there); the payload, unpacked
  // into the caller's array, moves with them
  e = zs::launch_gather_runs(keys, w->hi, n, w->lo, payload, w->runs, w->counters, st);
  if (e != hipSuccess) return hip_fail(e);
  Call lc{w->lo, payload, payload ? 4 : 0, (uint64_t)n, nullptr, 0, c, 0, 0, false};
  lc.runs = w->runs;
  lc.nruns = w->counters;
  lc.runs_cap = (int64_t)(n / 65 + 1);
  rc = run(lc, st, nullptr);
  if (rc) return rc;
  e = zs::launch_final128(keys, n, sgn, w->hi, w->lo, st);
  if (e != hipSuccess) return hip_fail(e);
  if (report) {
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e);
    rc = ctl_levels(st, &report->levels_low, &report->device_error);
    if (rc) return rc;
    uint32_t cnt[4] = {0, 0, 0, 0};
    e = hipMemcpy(cnt, w->counters, sizeof cnt, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e);
    report->runs = (uint64_t)cnt[0] + cnt[1];
    report->short_runs = cnt[1];
    report->run_keys = (uint64_t)cnt[2] | ((uint64_t)cnt[3] << 32);
  }
  return ZSORT_OK;
}

size_t zsort_workspace_bytes(size_t n, int payload_bytes, int32_t num_segments,
                             const zsort_config* cfg) {
  if (payload_bytes != 0 && payload_bytes != 4 && payload_bytes != 8) return 0;
  if (num_segments < 0 || n > 0x7FFFFFFFull) return 0;
  std::lock_guard<std::mutex> lk(g_mu);
  zsort_config c;
  // cfg NULL: the configuration such a call would use (tuned entry or defaults)
  if (resolve_cfg(cfg, &c, n, payload_bytes, num_segments > 0 ? 1 : 0)) return 0;
  Shape s;
  s.n = n;
  s.pw = payload_bytes;
  s.k = c.k;
  s.cutoff = c.cutoff;
  s.chunk = c.chunk;
  s.tile = c.tile;
  s.fuse = fused_on(c) ? 1 : 0;
  s.nseg = num_segments > 0 ? num_segments : 0;
  return plan(s).total;
}

int zsort_set_workspace(void* d_ws, size_t bytes, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  if (d_ws && (((uintptr_t)d_ws & 255u) != 0 || bytes < zs_min_workspace())) return ZSORT_EINVAL;
  if (!d_ws && bytes) return ZSORT_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  if (capturing(st)) return ZSORT_ECAPTURE;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e);
  Workspace*& w = g_ws[st];
  if (!w) w = new Workspace();
  if (w->device != -1 && w->device != dev && w->base) return ZSORT_EINVAL;
  drop_graphs(w);
  if (w->base && !w->user) {
    e = hipFree(w->base);   // the library's own buffer (synchronises the device)
    if (e != hipSuccess) return hip_fail(e);
  }
  w->base = (char*)d_ws;
  w->bytes = d_ws ? bytes : 0;
  w->user = d_ws != nullptr;
  w->laid_out = false;
  w->rows_dirty = true;
  w->has_last = false;
  w->device = dev;
  if (d_ws) {
    e = hipMemsetAsync(d_ws, 0, sizeof(zs::Ctl), st);
    if (e != hipSuccess) return hip_fail(e);
  }
  return ZSORT_OK;
}

int zsort_set_alloc_limit(size_t max_bytes) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_alloc_limit = max_bytes;
  return ZSORT_OK;
}

int zsort_get_last_stats(void* stream, zsort_stats* out) {
  if (!out) return ZSORT_EINVAL;
  std::memset(out, 0, sizeof *out);
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_ws.find((hipStream_t)stream);
  if (it == g_ws.end() || !it->second->has_last) return ZSORT_EINVAL;
  Workspace* w = it->second;
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e);
  zs::Ctl ctl;
  e = hipMemcpy(&ctl, w->base + w->lay.off_ctl, sizeof ctl, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e);
  out->device_error = (int32_t)ctl.error;
  out->identical = ctl.n_ident;
  out->range_mapped = ctl.n_rmap;
  out->leaf_groups = ctl.n_leafgroups;
  out->payload_bytes = w->last_pw;
  out->n = w->last_n;
  int levels = 0;
  double bytes = 0;
  const double kp = 8.0 + w->last_pw;
  for (int L = 0; L < zs::kMaxLevels && L < ZSORT_MAX_LEVELS; ++L) {
    out->keys_per_level[L] = ctl.lvl_keys[L];
    out->mkeys_per_level[L] = ctl.lvl_mkeys[L];
    out->segs_per_level[L] = ctl.lvl_segs[L];
    if (ctl.lvl_mkeys[L] || ctl.lvl_fkeys[L]) levels = L + 1;
    bytes += 8.0 * (double)ctl.lvl_mkeys[L] + (8.0 + 2 * kp) * (double)ctl.lvl_keys[L];
  }
  bytes += 2 * kp * (double)ctl.local_keys + w->last_extra_bytes;
  out->local_keys = ctl.local_keys;
  out->counted = ctl.n_count;
  out->fallback_groups = ctl.n_hard;
  out->levels = levels;
  out->model_bytes = bytes;
  return ZSORT_OK;
}

int zsort_debug_level0(const uint64_t* keys, const void* payload, int payload_bytes, size_t n,
                       const zsort_config* cfg, uint64_t* out_keys, void* out_payload,
                       void* stream) {
  int rc = common_checks(keys, payload, payload_bytes, n);
  if (rc) return rc;
  zsort_config c;
  rc = resolve_cfg(cfg, &c);
  if (rc) return rc;
  if (n <= (size_t)c.cutoff || !out_keys || (payload_bytes && !out_payload)) return ZSORT_EINVAL;
  if (c.flags & ZSORT_FLAG_SIGNED) return ZSORT_EUNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_mu);
  hipStream_t st = (hipStream_t)stream;
  Call call{const_cast<uint64_t*>(keys), payload_bytes ? const_cast<void*>(payload) : nullptr,
            payload_bytes, (uint64_t)n, nullptr, 0, c, 0, 0, true};
  Workspace* w = nullptr;
  rc = run(call, st, &w);
  if (rc) return rc;
  hipError_t e = hipMemcpyAsync(out_keys, w->base + w->lay.off_keys, n * 8,
                                hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess && payload_bytes)
    e = hipMemcpyAsync(out_payload, w->base + w->lay.off_pay, n * (size_t)payload_bytes,
                       hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e);
  return ZSORT_OK;
}

int zsort_stable_traced(uint64_t* keys, void* payload, int payload_bytes, size_t n,
                        const zsort_config* cfg, zsort_trace_rec* trace, int64_t trace_cap,
                        uint32_t* hist, int64_t hist_cap, int64_t counts[2], void* stream) {
  static_assert(sizeof(zsort_trace_rec) == sizeof(zs::TraceRec), "trace record layout");
  int rc = common_checks(keys, payload, payload_bytes, n);
  if (rc) return rc;
  zsort_config c;
  rc = resolve_cfg(cfg, &c);
  if (rc) return rc;
  if (trace_cap < 0 || hist_cap < 0 || (trace_cap && !trace) || (hist_cap && !hist) || !counts)
    return ZSORT_EINVAL;
  if (trace_cap > 0xFFFFFFF || hist_cap > 0xFFFFFFFF) return ZSORT_EINVAL;
  if (c.flags & ZSORT_FLAG_SIGNED) return ZSORT_EUNSUPPORTED;
  counts[0] = counts[1] = 0;
  if (n <= 1) return ZSORT_OK;
  std::lock_guard<std::mutex> lk(g_mu);
  hipStream_t st = (hipStream_t)stream;
  Call call{keys, payload_bytes ? payload : nullptr, payload_bytes, (uint64_t)n, nullptr, 0, c,
            std::max<int64_t>(trace_cap, 1), std::max<int64_t>(hist_cap, 1), false};
  Workspace* w = nullptr;
  rc = run(call, st, &w);
  if (rc) return rc;
  hipError_t e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e);
  zs::Ctl ctl;
  e = hipMemcpy(&ctl, w->base + w->lay.off_ctl, sizeof ctl, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e);
  counts[0] = ctl.ntrace;
  counts[1] = std::min<int64_t>(ctl.ntrace_hist, hist_cap);
  const int64_t nrec = std::min<int64_t>(ctl.ntrace, trace_cap);
  if (nrec) {
    e = hipMemcpy(trace, w->base + w->lay.off_trace, (size_t)nrec * sizeof(zsort_trace_rec),
                  hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e);
  }
  if (counts[1]) {
    e = hipMemcpy(hist, w->base + w->lay.off_thist, (size_t)counts[1] * 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e);
  }
  return ctl.error ? ZSORT_EDEVICE : ZSORT_OK;
}

int zsort_autotune(const uint64_t* keys, const void* payload, int payload_bytes, size_t n,
                   const int64_t* seg_offsets, int32_t num_segments, const char* cache_path,
                   zsort_config* best, void* stream) {
  int rc = common_checks(keys, payload, payload_bytes, n);
  if (rc) return rc;
  if (num_segments < 0 || (num_segments > 0 && !seg_offsets)) return ZSORT_EINVAL;
  const int seg = seg_offsets ? 1 : 0;
  std::lock_guard<std::mutex> lk(g_mu);
  if (cache_path) tune_file_read(cache_path);
  const TuneKey key{n_class(n), payload_bytes, seg};
  auto it = g_tuned.find(key);
  if (it != g_tuned.end() || n <= 1) {
    if (best) resolve_cfg(nullptr, best, n, payload_bytes, seg);
    return ZSORT_OK;
  }
  hipStream_t st = (hipStream_t)stream;
  if (capturing(st)) return ZSORT_ECAPTURE;
  uint64_t* tk = nullptr;
  void* tp = nullptr;
  uint32_t* flag = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = dev_alloc((void**)&tk, n * 8);
  if (e == hipSuccess && payload_bytes) e = dev_alloc(&tp, n * (size_t)payload_bytes);
  if (e == hipSuccess) e = dev_alloc((void**)&flag, 256);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  zsort_config win;
  zsort_default_config(&win);
  float win_ms = 1e30f;
  constexpr int kTop = 3;
  zsort_config top[kTop];
  float top_ms[kTop] = {1e30f, 1e30f, 1e30f};
  for (zsort_config& q : top) zsort_default_config(&q);
  // the faster of two runs after a warm-up one (1e30: a device-side limit
  // was hit, the candidate is out)
  auto time_cfg = [&](const zsort_config& c) -> float {
    float t_best = 1e30f;
    for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
      e = hipMemcpyAsync(tk, keys, n * 8, hipMemcpyDeviceToDevice, st);
      if (e == hipSuccess && payload_bytes)
        e = hipMemcpyAsync(tp, payload, n * (size_t)payload_bytes, hipMemcpyDeviceToDevice, st);
      if (e == hipSuccess) e = hipEventRecord(e0, st);
      if (e != hipSuccess) break;
      Call call{tk, payload_bytes ? tp : nullptr, payload_bytes, (uint64_t)n, seg_offsets,
                num_segments, c, 0, 0, false};
      Workspace* w = nullptr;
      rc = run(call, st, &w);
      if (rc) break;
      e = hipEventRecord(e1, st);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      uint32_t derr = 0;
      if (e == hipSuccess)
        e = hipMemcpy(&derr, w->base + w->lay.off_ctl + offsetof(zs::Ctl, error), 4,
                      hipMemcpyDeviceToHost);
      if (derr) return 1e30f;
      if (rep > 0 && ms < t_best) t_best = ms;  // first run warms up
    }
    return t_best;
  };
  const int ks[3] = {256, 512, 1024};
  // (tile, chunk): one-tile work items put the runs of neighbouring tiles
  // side by side in memory at the same time; larger ones cost the histogram
  // pass less
  const int tiles[4][2] = {{2048, 16384}, {4096, 32768}, {8192, 8192}, {8192, 32768}};
  const int cuts[3] = {1024, 2048, 4096};
  for (int a = 0; a < 3 && e == hipSuccess && !rc; ++a)
    for (int b = 0; b < 4 && e == hipSuccess && !rc; ++b)
      for (int d = 0; d < 3 && e == hipSuccess && !rc; ++d) {
        zsort_config c;
        zsort_default_config(&c);
        c.k = ks[a];
        c.tile = tiles[b][0];
        c.chunk = tiles[b][1];
        c.cutoff = cuts[d];
        const float t = time_cfg(c);
        // the three fastest so far, fastest first
        int at = kTop;
        while (at > 0 && t < top_ms[at - 1]) --at;
        if (at < kTop) {
          for (int q = kTop - 1; q > at; --q) {
            top_ms[q] = top_ms[q - 1];
            top[q] = top[q - 1];
          }
          top_ms[at] = t;
          top[at] = c;
        }
      }
  win_ms = top_ms[0];
  win = top[0];
  // the three fastest with z-score maps on their first one or two levels
  // only (another k or cutoff may win once the later levels take range maps)
  for (int q = 0; q < kTop && top_ms[q] < 1e29f && e == hipSuccess && !rc; ++q)
    for (int z = 1; z <= 2 && e == hipSuccess && !rc; ++z) {
      zsort_config c = top[q];
      if (c.max_zlevels <= z) break;
      c.max_zlevels = z;
      const float t = time_cfg(c);
      if (t < win_ms) {
        win_ms = t;
        win = c;
      }
    }
  // the winner once more: its output must be sorted (single arrays) before it
  // is remembered
  uint32_t unsorted = win_ms < 1e29f ? 0u : 1u;
  if (!rc && e == hipSuccess && !unsorted && !seg_offsets) {
    e = hipMemcpyAsync(tk, keys, n * 8, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && payload_bytes)
      e = hipMemcpyAsync(tp, payload, n * (size_t)payload_bytes, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipMemsetAsync(flag, 0, 4, st);
    if (e == hipSuccess) {
      Call call{tk, payload_bytes ? tp : nullptr, payload_bytes, (uint64_t)n, nullptr, 0, win, 0, 0,
                false};
      rc = run(call, st, nullptr);
    }
    if (!rc && e == hipSuccess)
      e = zs::launch_check_sorted(tk, n, flag, std::max(1, g_cu_count) * 4, st);
    if (!rc && e == hipSuccess) e = hipMemcpyAsync(&unsorted, flag, 4, hipMemcpyDeviceToHost, st);
    if (!rc && e == hipSuccess) e = hipStreamSynchronize(st);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (tk) (void)hipFree(tk);
  if (tp) (void)hipFree(tp);
  if (flag) (void)hipFree(flag);
  if (rc) return rc;
  if (e != hipSuccess) return hip_fail(e);
  if (unsorted) return ZSORT_EDEVICE;   // no candidate ran within its limits
  g_tuned[key] = win;
  if (cache_path) tune_file_write(cache_path);
  if (best) *best = win;
  return ZSORT_OK;
}

int zsort_profile_begin(void* stream) {
  return zsort_profile_begin_stages(stream, (1u << zs::NSTAGES) - 1u);
}

int zsort_profile_begin_stages(void* stream, uint32_t stage_mask) {
  if (stage_mask == 0 || (stage_mask >> zs::NSTAGES) != 0) return ZSORT_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  Workspace*& w = g_ws[(hipStream_t)stream];
  if (!w) w = new Workspace();
  w->prof = true;
  w->prof_mask = stage_mask;
  w->ev_used = 0;
  w->ev_stage.clear();
  return ZSORT_OK;
}

int zsort_profile_end(void* stream, zsort_kernel_times* out) {
  if (!out) return ZSORT_EINVAL;
  std::memset(out, 0, sizeof *out);
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_ws.find((hipStream_t)stream);
  if (it == g_ws.end() || !it->second->prof) return ZSORT_EINVAL;
  Workspace* w = it->second;
  w->prof = false;
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e);
  for (size_t i = 0; i < w->ev_stage.size(); ++i) {
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, w->ev_pool[2 * i], w->ev_pool[2 * i + 1]);
    if (e != hipSuccess) return hip_fail(e);
    out->ms[w->ev_stage[i]] += ms;
    out->launches[w->ev_stage[i]] += 1;
  }
  w->ev_used = 0;
  w->ev_stage.clear();
  return ZSORT_OK;
}

int zsort_release(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  int rc = ZSORT_OK;
  // (work may still run on the library's own streams: the local sorts' stream)
  if (!g_ws.empty() || !g_ws_aux.empty()) {
    const hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) rc = hip_fail(e);
  }
  auto free_ws = [&](Workspace* w) {
    drop_graphs(w);
    if (w->cap_stream) (void)hipStreamDestroy(w->cap_stream);
    if (w->base && !w->user) {   // a caller's workspace is the caller's to free
      hipError_t e = hipFree(w->base);
      if (e != hipSuccess) rc = hip_fail(e);
    }
    for (hipEvent_t ev : w->ev_pool) (void)hipEventDestroy(ev);
    for (hipEvent_t ev : w->lvl_ev)
      if (ev) (void)hipEventDestroy(ev);
    for (int i = 0; i < zs::kMaxLevels; ++i) {
      if (w->scat_ev[i]) (void)hipEventDestroy(w->scat_ev[i]);
      if (w->loc_ev[i]) (void)hipEventDestroy(w->loc_ev[i]);
    }
    if (w->side) (void)hipStreamDestroy(w->side);
    if (w->h_nseg) (void)hipHostFree(w->h_nseg);
    if (w->h_pace) (void)hipHostFree(w->h_pace);
    delete w;
  };
  for (auto& kv : g_ws) free_ws(kv.second);
  g_ws.clear();
  for (auto& kv : g_ws_aux) free_ws(kv.second);
  g_ws_aux.clear();
  for (auto& kv : g_wide) {
    if (kv.second->base) {
      hipError_t e = hipFree(kv.second->base);
      if (e != hipSuccess) rc = hip_fail(e);
    }
    delete kv.second;
  }
  g_wide.clear();
  for (auto& kv : g_lws) {
    if (kv.second->base) {
      hipError_t e = hipFree(kv.second->base);
      if (e != hipSuccess) rc = hip_fail(e);
    }
    if (kv.second->h_res) (void)hipHostFree(kv.second->h_res);
    for (hipEvent_t ev : kv.second->ev)
      if (ev) (void)hipEventDestroy(ev);
    delete kv.second;
  }
  g_lws.clear();
  return rc;
}


static_assert(sizeof(zsort_mlp_params) == sizeof(zs::MlpP), "parameter layout");

int zsort_default_learned_config(zsort_learned_config* lcfg) {
  if (!lcfg) return ZSORT_EINVAL;
  std::memset(lcfg, 0, sizeof *lcfg);
  lcfg->buckets = 4096;
  lcfg->sample_stride = 100;
  lcfg->steps = 0;   // training has not lowered the largest cluster on the mixtures
  lcfg->batches = 64;
  lcfg->lr = 1e-4;
  lcfg->seed = 0x5A17ull;
  return ZSORT_OK;
}

int zsort_stable_learned(uint64_t* keys, void* payload, int payload_bytes, size_t n,
                         const zsort_config* cfg, const zsort_learned_config* lcfg,
                         zsort_learned_report* report, void* stream) {
  int rc = common_checks(keys, payload, payload_bytes, n);
  if (rc) return rc;
  zsort_learned_config L;
  zsort_default_learned_config(&L);
  if (lcfg) L = *lcfg;
  rc = check_lcfg(&L);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(g_mu);
  zsort_config c;
  rc = resolve_cfg(cfg, &c, n, payload_bytes, 0);
  if (rc) return rc;
  if (c.flags & (ZSORT_FLAG_GRAPH | ZSORT_FLAG_SIGNED)) return ZSORT_EUNSUPPORTED;
  uint32_t* host_counts = report ? report->counts : nullptr;
  zsort_mlp_params* params_out = report ? report->params_out : nullptr;
  if (report) {
    std::memset(report, 0, sizeof *report);
    report->counts = host_counts;
    report->params_out = params_out;
  }
  if (n <= 1) return ZSORT_OK;
  hipStream_t st = (hipStream_t)stream;
  if (capturing(st)) return ZSORT_ECAPTURE;
  void* pay = payload_bytes ? payload : nullptr;
  Call call{keys, pay, payload_bytes, (uint64_t)n, nullptr, 0, c, 0, 0, false};
  const int B = L.buckets;
  const uint64_t m = L.params ? 0 : (uint64_t)n / (uint64_t)L.sample_stride;
  if ((uint64_t)n <= (uint64_t)c.cutoff || (!L.params && m < 64)) {
    // too small for a first pass of its own, or for a sample: the plain path
    return run(call, st, nullptr);
  }
  const uint32_t nb = (uint32_t)L.batches;
  LearnedWs* lw = nullptr;
  rc = lacquire(st, n, m, m ? zs::lpart_floats(m, nb) : 0, &lw);
  if (rc) return rc;
  hipError_t e = hipEventRecord(lw->ev[0], st);
  // 1. the map: sample, sorted sample, targets, initialisation, training
  if (e == hipSuccess && !L.params) {
    e = zs::launch_lsample(keys, m, (uint32_t)L.sample_stride, L.seed, lw->sample, st);
    if (e == hipSuccess) {
      zsort_config cs;
      zsort_default_config(&cs);
      Call sc{lw->sample, nullptr, 0, m, nullptr, 0, cs, 0, 0, false};
      sc.slot = 1;
      rc = run(sc, st, nullptr);
      if (rc) return rc;
    }
    if (e == hipSuccess) e = zs::launch_lprep(lw->sample, m, lw->U, lw->Y, lw->res, st);
    if (e == hipSuccess) e = zs::launch_linit(lw->sample, m, lw->par, lw->res, st);
    if (e == hipSuccess) e = zs::launch_ladam_reset(lw->adam, lw->res, st);
    if (e == hipSuccess && L.steps > 0) {
      // loss on minibatch 0 before and after training; the better parameters stay
      e = hipMemcpyAsync(lw->par0, lw->par, sizeof(zs::MlpP), hipMemcpyDeviceToDevice, st);
      if (e == hipSuccess)
        e = zs::launch_ltrain(lw->U, lw->Y, m, nb, 0, lw->par, lw->adam, lw->part, lw->res, 0.0, 1,
                              lw->gout, st);
      for (int t = 0; t < L.steps && e == hipSuccess; ++t)
        e = zs::launch_ltrain(lw->U, lw->Y, m, nb, (uint32_t)t, lw->par, lw->adam, lw->part,
                              lw->res, L.lr, 0, nullptr, st);
      if (e == hipSuccess)
        e = zs::launch_ltrain(lw->U, lw->Y, m, nb, 0, lw->par, lw->adam, lw->part, lw->res, 0.0, 1,
                              lw->gout1, st);
      // the sample's largest cluster under each parameter set decides
      if (e == hipSuccess) e = hipMemsetAsync(lw->hc, 0, 2 * zs::kKMax * 4, st);
      if (e == hipSuccess) e = zs::launch_lhist_sample(lw->U, m, lw->par0, B, lw->hc, st);
      if (e == hipSuccess)
        e = zs::launch_lhist_sample(lw->U, m, lw->par, B, lw->hc + zs::kKMax, st);
      if (e == hipSuccess)
        e = zs::launch_lkeep(lw->par, lw->par0, lw->gout, lw->gout1, lw->hc, lw->hc + zs::kKMax, B,
                             lw->res, st);
    }
  } else if (e == hipSuccess) {
    e = hipMemcpyAsync(lw->par, L.params, sizeof(zs::MlpP), hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = zs::launch_ladam_reset(lw->adam, lw->res, st);
    if (e == hipSuccess) e = zs::launch_lset_range(lw->res, L.smin, L.smax, st);
  }
  const bool direct = (L.flags & ZSORT_LEARNED_DIRECT) != 0;
  if (e == hipSuccess && !direct) e = zs::launch_lthresh(lw->par, B, lw->res, lw->thr, st);
  if (e == hipSuccess && !direct) e = zs::launch_lthr_check(lw->thr, lw->res, st);
  if (e == hipSuccess) e = hipEventRecord(lw->ev[1], st);
  if (e != hipSuccess) return hip_fail(e);

  // 2. the main workspace.  More than 512 clusters (a multiple of 64) are
  //    made in two stages of the same thresholds: 64 root clusters (every
  //    (B/64)-th threshold), then B/64 sub-clusters of each, so that each
  //    scatter writes long runs; the clusters are those of one B-way pass.
  const bool two = !direct && B > 512 && B % 64 == 0;
  const int B0 = two ? 64 : B, B1 = two ? B / 64 : 0;
  Shape s;
  s.n = n;
  s.pw = payload_bytes;
  s.k = std::max(c.k, B1);
  s.cutoff = c.cutoff;
  s.chunk = c.chunk;
  s.tile = c.tile;
  s.fuse = fused_on(c) ? 1 : 0;
  s.kfirst = B;
  Workspace* w = nullptr;
  rc = acquire(st, s, &w);
  if (rc) return rc;
  if (!pacing_ready(w)) return ZSORT_EHIP;
  Ws ws = make_ws(w, keys, pay, c, payload_bytes);
  e = prepare_rows(w, &ws, st);
  if (e != hipSuccess) return hip_fail(e);
  Ws w0 = first_pass_ws(ws, lw, B0, direct);
  w0.lm.sub = (uint32_t)B1;
  const Ws w1 = first_pass_ws(ws, lw, two ? B1 : B0, false);
  const int pw = payload_bytes;
  if (L.flags & ZSORT_LEARNED_ZSCORE_DIAG) {
    // the z-score map's histogram at B clusters (moments, statistics,
    // histogram of the root; nothing moves)
    Ws wd = first_pass_ws(ws, lw, B, false);
    std::memset(&wd.lm, 0, sizeof wd.lm);
    e = zs::launch_reset(wd, st);
    if (e == hipSuccess) e = zs::launch_init_single(wd, n, st);
    for (int sid = zs::STAGE_MOMENTS; sid <= zs::STAGE_HIST && e == hipSuccess; ++sid)
      e = stage(w, wd, 0, sid, grid_size(B, pw, wd.p.tile, sid), st);
    if (e == hipSuccess) e = zs::launch_lmaxcount(wd.bstart, n, B, &lw->res->maxz, st);
    if (e != hipSuccess) return hip_fail(e);
  }
  // 3. learned first pass (hist writes the cluster ids, scatter moves key +
  //    payload to the alternate buffer); the caller's keys stay untouched
  //    until the order check has been read
  e = zs::launch_reset(w0, st);
  if (e == hipSuccess) e = zs::launch_init_learned(w0, n, st);
  if (e == hipSuccess) e = hipEventRecord(lw->ev[2], st);
  if (e == hipSuccess)
    e = stage(w, w0, 0, zs::STAGE_HIST, grid_size(B0, pw, w0.p.tile, zs::STAGE_HIST), st);
  if (e == hipSuccess)
    e = stage(w, w0, 0, zs::STAGE_SCATTER, grid_size(B0, pw, w0.p.tile, zs::STAGE_SCATTER), st);
  const bool scan = direct || (L.flags & ZSORT_LEARNED_VERIFY);
  if (e == hipSuccess && scan)  // check the output itself (root clusters)
    e = zs::launch_lcheck(ws.keys[1], ws.bstart, n, B0, lw->bmin, lw->bmax, lw->res,
                          std::max(1, g_cu_count) * 4, st);
  if (e == hipSuccess && host_counts) {
    if (two) {
      e = hipMemsetAsync(lw->counts, 0, (size_t)B * 4, st);
      if (e == hipSuccess)
        e = zs::launch_lfine_hist(ws.keys[1], n, lw->thr, lw->res, B, lw->counts, st);
    } else {
      e = zs::launch_lcounts(ws.bstart, n, B, lw->counts, st);
    }
  }
  if (e == hipSuccess && !two) e = hipEventRecord(lw->ev[3], st);
  if (e == hipSuccess && host_counts)
    e = hipMemcpyAsync(host_counts, lw->counts, (size_t)B * 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess && params_out)
    e = hipMemcpyAsync(params_out, lw->par, sizeof(zs::MlpP), hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(lw->h_res, lw->res, sizeof(zs::LRes), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipEventRecord(lw->ev[4], st);
  if (e == hipSuccess) e = hipEventSynchronize(lw->ev[4]);
  if (e != hipSuccess) return hip_fail(e);
  const zs::LRes r = *lw->h_res;
  const double kp = 8.0 + pw;
  // cluster ids (written by hist, read by scatter) of each learned pass, key check
  double extra = (two ? 8.0 : 4.0) * (double)n + (scan ? 8.0 * (double)n : 0.0);
  if (r.fail) {
    // 4a. the map broke the cluster order: the z-score path sorts the
    //     caller's keys, which the first pass left untouched
    e = enqueue(w, ws, call, st);
    extra = 4.0 * (double)n + (scan ? 8.0 * (double)n : 0.0) + (8.0 + 2.0 * kp) * (double)n;
  } else {
    // z-score levels after the learned passes: clusters hold about n / B
    // keys, so fewer clusters per pass suffice to reach the cutoff (about 4
    // times n / (B * cutoff), a power of two in [16, k])
    int k2 = 16;
    while (k2 < c.k && (double)k2 < 4.0 * (double)n / ((double)B * (double)c.cutoff)) k2 <<= 1;
    k2 = std::min(k2, c.k);
    Ws wz = ws;
    wz.p.k = k2;
    wz.p.lb = floor_log2(k2);
    Call cz = call;
    cz.cfg.k = k2;
    if (cz.cfg.tile > 2048 && k2 > 1024) cz.cfg.tile = wz.p.tile = 2048;
    // 4b. local sort of the first pass's small clusters; with two stages the
    //     second learned pass (its lists start empty: no moments pass runs
    //     for learned segments); then the z-score levels on what is left
    e = stage(w, ws, 0, zs::STAGE_LOCAL, grid_size(c.k, pw, c.tile, zs::STAGE_LOCAL), st);
    if (e == hipSuccess)
      e = stage(w, ws, 0, zs::STAGE_LOCAL_HARD, grid_size(c.k, pw, c.tile, zs::STAGE_LOCAL_HARD), st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(&w->h_nseg[1], &ws.ctl->nseg[1], sizeof(uint32_t), hipMemcpyDeviceToHost,
                         st);
    if (e == hipSuccess) e = hipEventRecord(w->lvl_ev[0], st);
    if (two) {
      if (e == hipSuccess) e = zs::launch_reset_lists(ws, 0, st);
      if (e == hipSuccess)
        e = stage(w, w1, 1, zs::STAGE_HIST, grid_size(B1, pw, w1.p.tile, zs::STAGE_HIST), st);
      if (e == hipSuccess)
        e = stage(w, w1, 1, zs::STAGE_SCATTER, grid_size(B1, pw, w1.p.tile, zs::STAGE_SCATTER), st);
      if (e == hipSuccess) e = hipEventRecord(lw->ev[3], st);
      if (e == hipSuccess && report)  // the largest cluster, complete after the second pass
        e = hipMemcpyAsync(lw->h_res + 1, lw->res, sizeof(zs::LRes), hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipEventRecord(lw->ev[5], st);
      if (e == hipSuccess)
        e = stage(w, ws, 1, zs::STAGE_LOCAL, grid_size(c.k, pw, c.tile, zs::STAGE_LOCAL), st);
      if (e == hipSuccess)
        e = stage(w, ws, 1, zs::STAGE_LOCAL_HARD,
                  grid_size(c.k, pw, c.tile, zs::STAGE_LOCAL_HARD), st);
      if (e == hipSuccess)
        e = hipMemcpyAsync(&w->h_nseg[2], &ws.ctl->nseg[0], sizeof(uint32_t),
                           hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipEventRecord(w->lvl_ev[1], st);
      if (e == hipSuccess) e = enqueue_levels(w, wz, cz, st, 2, false);
    } else {
      if (e == hipSuccess) e = enqueue_levels(w, wz, cz, st, 1, false);
    }
  }
  if (e != hipSuccess) return hip_fail(e);
  w->calls++;
  w->last_n = n;
  w->last_pw = pw;
  w->has_last = true;
  w->last_extra_bytes = extra;
  if (report) {
    uint64_t maxc = r.maxc;
    if (two && !r.fail) {
      e = hipEventSynchronize(lw->ev[5]);
      if (e != hipSuccess) return hip_fail(e);
      maxc = lw->h_res[1].maxc;
    }
    report->used_learned = r.fail ? 0 : 1;
    report->fallback = r.fail ? 1 : 0;
    report->thresholds = direct ? -1 : (int32_t)r.nt;
    report->steps = L.params ? 0 : (int32_t)r.steps_done;
    report->trained = (!L.params && L.steps > 0) ? (int32_t)r.trained : 0;
    report->smin_out = r.smin;
    report->smax_out = r.smax;
    report->sample_max_init = r.smax_init;
    report->sample_max_trained = r.smax_trained;
    report->sample_keys = m;
    report->max_cluster_learned = maxc;
    report->max_cluster_zscore = r.maxz;
    const double mean = (double)n / (double)B;
    report->imbalance_learned = (double)maxc / mean;
    report->imbalance_zscore = (L.flags & ZSORT_LEARNED_ZSCORE_DIAG) ? (double)r.maxz / mean : 0.0;
    report->loss_first = r.loss_first;
    report->loss_last = r.loss_last;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, lw->ev[0], lw->ev[1]) == hipSuccess) report->train_ms = ms;
    if (hipEventElapsedTime(&ms, lw->ev[2], lw->ev[3]) == hipSuccess) report->first_pass_ms = ms;
  }
  return ZSORT_OK;
}

int zsort_learned_sample(const uint64_t* keys, size_t n, int32_t stride, uint64_t seed,
                         uint64_t* out, void* stream) {
  if (stride < 1 || n > 0x7FFFFFFFull || (n && (!keys || !out))) return ZSORT_EINVAL;
  const uint64_t m = (uint64_t)n / (uint64_t)stride;
  if (!m) return ZSORT_OK;
  std::lock_guard<std::mutex> lk(g_mu);
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = zs::launch_lsample(keys, m, (uint32_t)stride, seed, out, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  return e == hipSuccess ? ZSORT_OK : hip_fail(e);
}

int zsort_mlp_forward(const zsort_mlp_params* params, const uint64_t* keys, size_t q, uint64_t smin,
                      uint64_t smax, int32_t buckets, float* f_out, uint32_t* cluster_out,
                      void* stream) {
  if (!params || (q && !keys) || smin > smax || buckets < 1 || buckets > zs::kKMax ||
      q > 0x7FFFFFFFull)
    return ZSORT_EINVAL;
  if (!q) return ZSORT_OK;
  std::lock_guard<std::mutex> lk(g_mu);
  hipStream_t st = (hipStream_t)stream;
  LearnedWs* lw = nullptr;
  int rc = lacquire(st, 0, 0, 0, &lw);
  if (rc) return rc;
  hipError_t e = zs::launch_lset_range(lw->res, smin, smax, st);
  if (e == hipSuccess)
    e = zs::launch_lforward((const zs::MlpP*)params, keys, q, lw->res, buckets, f_out, cluster_out,
                            st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  return e == hipSuccess ? ZSORT_OK : hip_fail(e);
}

int zsort_mlp_thresholds(const zsort_mlp_params* params, uint64_t smin, uint64_t smax, int32_t buckets,
                         uint64_t* thr_out, int32_t* nt_out, void* stream) {
  if (!params || !thr_out || !nt_out || smin > smax || buckets < 2 || buckets > zs::kKMax)
    return ZSORT_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  hipStream_t st = (hipStream_t)stream;
  LearnedWs* lw = nullptr;
  int rc = lacquire(st, 0, 0, 0, &lw);
  if (rc) return rc;
  hipError_t e = zs::launch_lset_range(lw->res, smin, smax, st);
  if (e == hipSuccess) e = zs::launch_lthresh((const zs::MlpP*)params, buckets, lw->res, thr_out, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(lw->h_res, lw->res, sizeof(zs::LRes), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e);
  *nt_out = (int32_t)lw->h_res->nt;
  return ZSORT_OK;
}

int zsort_mlp_init(const uint64_t* sorted_sample, size_t m, zsort_mlp_params* params_out,
                   void* stream) {
  if (!sorted_sample || !params_out || m < 2 || m > 0x7FFFFFFFull) return ZSORT_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  hipStream_t st = (hipStream_t)stream;
  LearnedWs* lw = nullptr;
  int rc = lacquire(st, 0, 0, 0, &lw);
  if (rc) return rc;
  hipError_t e = zs::launch_linit(sorted_sample, m, (zs::MlpP*)params_out, lw->res, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  return e == hipSuccess ? ZSORT_OK : hip_fail(e);
}

int zsort_mlp_grad(const zsort_mlp_params* params, const uint64_t* sorted_sample, size_t m, double* grad_out,
                   void* stream) {
  if (!params || !sorted_sample || !grad_out || m < 2 || m > 0x7FFFFFFFull) return ZSORT_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  hipStream_t st = (hipStream_t)stream;
  LearnedWs* lw = nullptr;
  int rc = lacquire(st, 0, m, zs::lpart_floats(m, 1), &lw);
  if (rc) return rc;
  hipError_t e = hipMemcpyAsync(lw->par, params, sizeof(zs::MlpP), hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = zs::launch_lprep(sorted_sample, m, lw->U, lw->Y, lw->res, st);
  if (e == hipSuccess) e = zs::launch_ladam_reset(lw->adam, lw->res, st);
  if (e == hipSuccess)
    e = zs::launch_ltrain(lw->U, lw->Y, m, 1, 0, lw->par, lw->adam, lw->part, lw->res, 0.0, 1,
                          grad_out, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  return e == hipSuccess ? ZSORT_OK : hip_fail(e);
}

int zsort_mlp_train(zsort_mlp_params* params, const uint64_t* sorted_sample, size_t m, int32_t steps,
                    int32_t batches, double lr, double* losses_out, void* stream) {
  if (!params || !sorted_sample || m < 2 || m > 0x7FFFFFFFull || steps < 0 || batches < 1 ||
      !(lr > 0.0))
    return ZSORT_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  hipStream_t st = (hipStream_t)stream;
  LearnedWs* lw = nullptr;
  int rc = lacquire(st, 0, m, zs::lpart_floats(m, (uint32_t)batches), &lw);
  if (rc) return rc;
  hipError_t e = hipMemcpyAsync(lw->par, params, sizeof(zs::MlpP), hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = zs::launch_lprep(sorted_sample, m, lw->U, lw->Y, lw->res, st);
  if (e == hipSuccess) e = zs::launch_ladam_reset(lw->adam, lw->res, st);
  for (int t = 0; t < steps && e == hipSuccess; ++t)
    e = zs::launch_ltrain(lw->U, lw->Y, m, (uint32_t)batches, (uint32_t)t, lw->par, lw->adam,
                          lw->part, lw->res, lr, 0, nullptr, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(params, lw->par, sizeof(zs::MlpP), hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(lw->h_res, lw->res, sizeof(zs::LRes), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e);
  if (losses_out) {
    losses_out[0] = lw->h_res->loss_first;
    losses_out[1] = lw->h_res->loss_last;
  }
  return ZSORT_OK;
}

int zsort_last_hip_error(void) { return g_last_hip; }

const char* zsort_strerror(int status) {
  switch (status) {
    case ZSORT_OK: return "ok";
    case ZSORT_EINVAL: return "invalid argument";
    case ZSORT_ENOMEM: return "device allocation failed";
    case ZSORT_EHIP: return "HIP runtime error";
    case ZSORT_ECAPTURE: return "would allocate during stream capture";
    case ZSORT_ETOOLARGE: return "problem larger than the fixed scratch buffer";
    case ZSORT_EUNSUPPORTED: return "configuration not supported";
    case ZSORT_EDEVICE: return "device-side limit hit";
    default: return "unknown status";
  }
}

}  // extern "C"
