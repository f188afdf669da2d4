// Host side of the C ABI declared in include/lsm.h: the handle, the level
// table and the order of kernel launches for each operation.
//
// State kept on the host: the batch counter r (sec. III-B: level i is full
// exactly when bit i of r is set) and one device allocation per level,
// made the first time an insertion reaches that level and kept until the
// handle is destroyed (an emptied level's contents are simply ignored).
//
// Strong guarantee: an update only reads the full levels 0 .. j-1 and
// writes scratch buffers and the empty level j = ffz(r); r is incremented
// only after every launch has been accepted, so a failure leaves the
// dictionary as it was.
#include <algorithm>
#include <chrono>
#include <new>
#include <string.h>
#include <vector>

#include "lsm.h"
#include "lsm_internal.h"

using namespace lsm;

static_assert(LSM_PROF_KERNELS == kNumKernelKinds, "profile kernel kinds out of step");
static_assert(LSM_NOALLOC_MAX_QUERIES == kFixedMaxQueries, "fixed scratch limit out of step");


// Kinds of whole-call spans in the profiler, above every kernel kind.
constexpr int kSpanUpdate = 100;
constexpr int kSpanLookup = 101;  // then count, range
constexpr int kSpanCount = 102;
constexpr int kSpanRange = 103;
static_assert(kSpanUpdate >= kNumKernelKinds, "span kinds overlap kernel kinds");

// Update launches allowed to wait on the stream ahead of the device's
// current one.  Measured at b = 2^16: with hundreds of launches queued the
// same 1024 batches took 22.3 ms of device time against 16.4 ms when the
// host stayed a few launches ahead.
constexpr int kDefaultInflight = 4;
// A pacing wait gives up after this long (the device has stopped writing
// its progress, e.g. after a fault; the call then goes ahead unpaced).
constexpr int kPaceLimitMs = 500;

struct lsm_s {
  uint32_t b = 0;
  uint32_t flags = 0;
  uint32_t key_bits = 31;
  hipStream_t stream = nullptr;
  int device = 0;
  uint64_t r = 0;

  uint32_t* lvl_kv[kMaxLevels] = {};
  uint32_t* lvl_val[kMaxLevels] = {};
  uint32_t* lvl_fence[kMaxLevels] = {};
  // Top-digit index of a level: the position of the first element of each
  // of the kTopBuckets top-digit buckets, written by the kernel that wrote the level
  // when it sorted by that digit.  digit_shift[i] is the key shift it was
  // built for, or -1 when level i was last written without one.
  uint32_t* lvl_digit[kMaxLevels] = {};
  int digit_shift[kMaxLevels];

  uint32_t* tmp_kv[2] = {};  // radix ping-pong, b elements each
  uint32_t* tmp_val[2] = {};
  // Top-digit sort: the tile-grouped batch of each slot, slots one after
  // another in one buffer (a group's bucket sort reads several of them).
  uint32_t* scat_kv[kSortSlots] = {};
  uint32_t* scat_val[kSortSlots] = {};
  uint32_t* buf_kv = nullptr;  // the sorted batch (or group) when it has to be merged
  uint32_t* buf_val = nullptr;
  // The most batches that can be sorted as one group (1, 2 or 4: every
  // batch's tiles must fit one group table, so 4 for b <= 2^17 and 2 for
  // b <= 2^18): buf and tmp[1] hold grp_cap * b.
  uint32_t grp_cap = 1;
  uint32_t* meta = nullptr;  // sort histograms, look-back words, group starts, error words
  int hist_parity = 0;       // which histogram buffer the next digit-pass sort uses

  // Pipelined insertion: batches sorted by the top-digit sort have had their
  // tiles scattered (each into its scratch slot) but not their buckets
  // sorted and merged; that second half runs in the same launch as a later
  // batch's scatter, or on its own when anything needs the levels.  Pending
  // batches form groups: a batch whose counter is a multiple of group_max
  // waits for the next group_max - 1 batches, and the group is sorted
  // together (newer first on equal keys) straight into the level its last
  // batch fills; any other batch pending alone is sorted alone.  An
  // incomplete group is sorted as aligned groups of 2 and 1.  Pending
  // batches already count in r.
  struct Pending {
    int slot = 0;
    int j = 0;        // the level the batch's insertion fills
    int lo_bit = 1;
    int passes = 0;
    uint64_t r = 0;   // the batch counter before the batch
  };
  Pending pend[kMaxGroup];
  int npend = 0;
  int group_max = 1;  // 1 (no grouping), 2 or 4; at most grp_cap
  uint32_t* fault = nullptr; // sticky device fault word (inside meta)

  uint32_t* mrg_kv[2] = {};  // cascade ping-pong
  uint32_t* mrg_val[2] = {};
  uint64_t mrg_cap = 0;
  // Top-digit indexes of the cascade's intermediate runs: the two merge
  // buffers and the sorted batch (buf_kv).
  uint32_t* mrg_digit[2] = {};
  uint32_t* buf_digit = nullptr;

  uint32_t* q_counts = nullptr;  // range pass 1 output
  uint64_t* q_status = nullptr;  // range scan look-back words
  uint32_t* q_bounds = nullptr;  // range pass 1: per-query positions in the levels
  uint64_t q_bwords = 0;         // words of q_bounds
  uint64_t q_cap = 0;
  // The device's fixed range scratch (lsm_range_async_noalloc), or nulls
  // when its address could not be looked up.
  FixedScratch fixed = {nullptr, nullptr};

  uint64_t* h_pinned = nullptr;  // read-backs (range total, key check)
  // Largest top-digit bucket of the most recent sort, written by the sort
  // kernels into mapped host memory and read without synchronising (a
  // stale value only affects which of two equivalent sort paths runs).
  uint32_t* skew_host = nullptr;
  uint32_t* skew_dev = nullptr;
  // Launch pacing: each top-digit update launch carries a sequence number
  // that its first work-group writes to mapped host memory when it starts;
  // an update call waits until the launch max_inflight before its own has
  // started (see pace()).
  uint64_t* progress_host = nullptr;
  uint64_t* progress_dev = nullptr;
  uint64_t launch_seq = 0;
  int max_inflight = kDefaultInflight;
  uint64_t pace_timeouts = 0;
  uint64_t sorts_by_path[2] = {0, 0};
  int sort_mode = LSM_SORT_AUTO;
  int fuse_max = 0;  // deepest cascade fused into the top-digit sort

  // Coalescer (batching form): user batches staged as key variables in
  // arrival order until b are collected.
  uint32_t* stage_kv = nullptr;
  uint32_t* stage_val = nullptr;
  uint32_t stage_fill = 0;

  // Merge variant per merge input level (autotuned or set).
  int merge_variant[kMaxLevels];
  float tune_us[kMaxLevels][kMergeVariants] = {};

  uint64_t merged_last = 0, merged_total = 0, sorted_total = 0;
  uint64_t device_bytes = 0;
  // Allocation-failure injection (tests): allocations left before every
  // further one fails; negative = never fail.
  int64_t fail_after = -1;

  // Profiling: events recorded on the stream between kernels, resolved on
  // lsm_profile_read.  A span is a pair of indices into `marks`.
  struct Span {
    int kind;  // KernelKind for a kernel; kSpanUpdate.. for a whole call
    uint32_t a, b;
    uint64_t items;
    double bytes;  // algorithmic bytes of a kernel launch
  };
  bool prof = false;
  std::vector<hipEvent_t> ev_pool, marks;
  std::vector<Span> spans;
  std::vector<double> update_times;
  lsm_profile_t acc = {};
};

namespace {

struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

lsm_status_t dev_alloc(lsm_t h, void** p, size_t bytes) {
  *p = nullptr;
  if (h->fail_after == 0) return LSM_ENOMEM;
  if (h->fail_after > 0) --h->fail_after;
  if (bytes == 0) bytes = 4;
  if (hipMalloc(p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return LSM_ENOMEM;
  }
  h->device_bytes += bytes;
  return LSM_OK;
}

void dev_free(lsm_t h, void* p, size_t bytes) {
  if (p != nullptr) {
    (void)hipFree(p);
    h->device_bytes -= bytes;
  }
}

inline uint64_t level_len(const lsm_t h, int i) { return static_cast<uint64_t>(h->b) << i; }

// Number of radix passes over the key-variable bits [lo_bit, key_bits + 1).
inline int sort_passes(uint32_t key_bits, int lo_bit) {
  return static_cast<int>((key_bits + 1 - lo_bit + kRadixBits - 1) / kRadixBits);
}

LevelSet occupied_levels(const lsm_t h) {
  LevelSet s;
  memset(&s, 0, sizeof(s));
  for (int i = 0; i < kMaxLevels; ++i) {
    if ((h->r >> i) & 1u) {
      s.kv[s.count] = h->lvl_kv[i];
      s.val[s.count] = h->lvl_val[i];
      s.fence[s.count] = h->lvl_fence[i];
      s.len[s.count] = static_cast<uint32_t>(level_len(h, i));
      ++s.count;
    }
  }
  return s;
}

lsm_status_t ensure_level(lsm_t h, int j) {
  if (h->lvl_kv[j] != nullptr) return LSM_OK;
  const size_t bytes = level_len(h, j) * sizeof(uint32_t);
  const size_t fbytes = fence_len(level_len(h, j)) * sizeof(uint32_t);
  void *k = nullptr, *v = nullptr, *f = nullptr, *dg = nullptr;
  lsm_status_t s = dev_alloc(h, &k, bytes);
  if (s != LSM_OK) return s;
  s = dev_alloc(h, &v, bytes);
  if (s == LSM_OK) s = dev_alloc(h, &f, fbytes);
  if (s == LSM_OK) s = dev_alloc(h, &dg, kTopBuckets * sizeof(uint32_t));
  if (s != LSM_OK) {
    dev_free(h, k, bytes);
    dev_free(h, v, bytes);
    dev_free(h, f, fbytes);
    return s;
  }
  h->lvl_kv[j] = static_cast<uint32_t*>(k);
  h->lvl_val[j] = static_cast<uint32_t*>(v);
  h->lvl_fence[j] = static_cast<uint32_t*>(f);
  h->lvl_digit[j] = static_cast<uint32_t*>(dg);
  h->digit_shift[j] = -1;
  return LSM_OK;
}

lsm_status_t ensure_merge_scratch(lsm_t h, uint64_t elems) {
  if (h->mrg_cap >= elems) return LSM_OK;
  void* p[4] = {};
  const size_t bytes = elems * sizeof(uint32_t);
  for (int i = 0; i < 4; ++i) {
    if (dev_alloc(h, &p[i], bytes) != LSM_OK) {
      for (int k = 0; k < i; ++k) dev_free(h, p[k], bytes);
      return LSM_ENOMEM;
    }
  }
  const size_t old = h->mrg_cap * sizeof(uint32_t);
  for (int i = 0; i < 2; ++i) {
    dev_free(h, h->mrg_kv[i], old);
    dev_free(h, h->mrg_val[i], old);
  }
  h->mrg_kv[0] = static_cast<uint32_t*>(p[0]);
  h->mrg_kv[1] = static_cast<uint32_t*>(p[1]);
  h->mrg_val[0] = static_cast<uint32_t*>(p[2]);
  h->mrg_val[1] = static_cast<uint32_t*>(p[3]);
  h->mrg_cap = elems;
  return LSM_OK;
}

lsm_status_t ensure_query_scratch(lsm_t h, uint32_t nq) {
  if (h->q_cap >= nq) return LSM_OK;
  uint64_t cap = h->q_cap ? h->q_cap : 4096;
  while (cap < nq) cap *= 2;
  void *c = nullptr, *s = nullptr;
  if (dev_alloc(h, &c, cap * sizeof(uint32_t)) != LSM_OK) return LSM_ENOMEM;
  const size_t sw = scan_status_words(static_cast<uint32_t>(cap < 0xFFFFFFFFull ? cap : 0xFFFFFFFFull));
  if (dev_alloc(h, &s, sw * sizeof(uint64_t)) != LSM_OK) {
    dev_free(h, c, cap * sizeof(uint32_t));
    return LSM_ENOMEM;
  }
  if (h->q_cap) {
    dev_free(h, h->q_counts, h->q_cap * sizeof(uint32_t));
    dev_free(h, h->q_status, scan_status_words(static_cast<uint32_t>(h->q_cap)) * sizeof(uint64_t));
  }
  h->q_counts = static_cast<uint32_t*>(c);
  h->q_status = static_cast<uint64_t*>(s);
  h->q_cap = cap;
  return LSM_OK;
}

// The range scratch for nq queries' positions in the levels the query will
// see (those of r after the staged elements are inserted): two words a query
// with one occupied level, one per level with several.  Grown on demand,
// before anything changes.
lsm_status_t ensure_bounds(lsm_t h, uint32_t nq) {
  const uint64_t r_after = h->r + (h->stage_fill > 0 ? 1 : 0);
  const int levels = __builtin_popcountll(r_after);
  const uint64_t words = static_cast<uint64_t>(nq) * (levels > 2 ? levels : 2);
  if (h->q_bwords >= words) return LSM_OK;
  uint64_t cap = h->q_bwords ? h->q_bwords : 8192;
  while (cap < words) cap *= 2;
  void* p = nullptr;
  if (dev_alloc(h, &p, cap * sizeof(uint32_t)) != LSM_OK) return LSM_ENOMEM;
  dev_free(h, h->q_bounds, h->q_bwords * sizeof(uint32_t));
  h->q_bounds = static_cast<uint32_t*>(p);
  h->q_bwords = cap;
  return LSM_OK;
}

void release_all(lsm_t h) {
  dev_free(h, h->stage_kv, static_cast<size_t>(h->b) * sizeof(uint32_t));
  dev_free(h, h->stage_val, static_cast<size_t>(h->b) * sizeof(uint32_t));
  const size_t bb = static_cast<size_t>(h->b) * sizeof(uint32_t);
  for (int i = 0; i < kMaxLevels; ++i) {
    dev_free(h, h->lvl_kv[i], level_len(h, i) * sizeof(uint32_t));
    dev_free(h, h->lvl_val[i], level_len(h, i) * sizeof(uint32_t));
    dev_free(h, h->lvl_fence[i], fence_len(level_len(h, i)) * sizeof(uint32_t));
    dev_free(h, h->lvl_digit[i], kTopBuckets * sizeof(uint32_t));
  }
  for (int i = 0; i < 2; ++i) {
    dev_free(h, h->tmp_kv[i], i == 1 ? h->grp_cap * bb : bb);
    dev_free(h, h->tmp_val[i], i == 1 ? h->grp_cap * bb : bb);
    dev_free(h, h->mrg_kv[i], h->mrg_cap * sizeof(uint32_t));
    dev_free(h, h->mrg_val[i], h->mrg_cap * sizeof(uint32_t));
  }
  dev_free(h, h->scat_kv[0], kSortSlots * bb);
  dev_free(h, h->scat_val[0], kSortSlots * bb);
  dev_free(h, h->buf_kv, h->grp_cap * bb);
  dev_free(h, h->buf_val, h->grp_cap * bb);
  for (int i = 0; i < 2; ++i) dev_free(h, h->mrg_digit[i], kTopBuckets * sizeof(uint32_t));
  dev_free(h, h->buf_digit, kTopBuckets * sizeof(uint32_t));
  dev_free(h, h->meta, sort_meta_words(h->b) * sizeof(uint32_t));
  if (h->q_cap) {
    dev_free(h, h->q_counts, h->q_cap * sizeof(uint32_t));
    dev_free(h, h->q_status, scan_status_words(static_cast<uint32_t>(h->q_cap)) * sizeof(uint64_t));
  }
  dev_free(h, h->q_bounds, h->q_bwords * sizeof(uint32_t));
  if (h->h_pinned) (void)hipHostFree(h->h_pinned);
  if (h->skew_host) (void)hipHostFree(h->skew_host);
  if (h->progress_host) (void)hipHostFree(h->progress_host);
}

// Two pooled events for one kernel launch (start, stop), remembered as a
// span of the given kind; returns nullptr when profiling is off.
struct Timed {
  KTimer t;
  int64_t a = -1, b = -1;
};

hipEvent_t pooled_event(lsm_t h) {
  hipEvent_t e = nullptr;
  if (!h->ev_pool.empty()) {
    e = h->ev_pool.back();
    h->ev_pool.pop_back();
  } else if (hipEventCreate(&e) != hipSuccess) {
    e = nullptr;
  }
  return e;
}

const KTimer* timer(lsm_t h, Timed& slot, int kind, uint64_t items, double bytes) {
  if (!h->prof) return nullptr;
  hipEvent_t a = pooled_event(h), b = pooled_event(h);
  if (a == nullptr || b == nullptr) {
    if (a) h->ev_pool.push_back(a);
    if (b) h->ev_pool.push_back(b);
    return nullptr;
  }
  h->marks.push_back(a);
  slot.a = static_cast<int64_t>(h->marks.size() - 1);
  h->marks.push_back(b);
  slot.b = static_cast<int64_t>(h->marks.size() - 1);
  slot.t.start = a;
  slot.t.stop = b;
  h->spans.push_back(
      {kind, static_cast<uint32_t>(slot.a), static_cast<uint32_t>(slot.b), items, bytes});
  return &slot.t;
}

// A call-level span from the start event of one launch to the stop event
// of another.
void call_span(lsm_t h, int kind, const Timed& first, const Timed& last, uint64_t items) {
  if (first.a >= 0 && last.b >= 0)
    h->spans.push_back(
        {kind, static_cast<uint32_t>(first.a), static_cast<uint32_t>(last.b), items, 0.0});
}

void release_events(lsm_t h) {
  for (hipEvent_t e : h->marks) (void)hipEventDestroy(e);
  for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
  h->marks.clear();
  h->ev_pool.clear();
  h->spans.clear();
}

// Allocations an insertion into level j = ffz(r) needs: level j itself and,
// for j >= 2, the cascade ping-pong buffers.
lsm_status_t prepare_insert(lsm_t h, int j) {
  if (j >= kMaxLevels || level_len(h, j) > (1ull << 31)) return LSM_ECAPACITY;
  lsm_status_t s = ensure_level(h, j);
  if (s != LSM_OK) return s;
  if (j >= 2) {
    s = ensure_merge_scratch(h, level_len(h, j - 1));
    if (s != LSM_OK) return s;
  }
  return LSM_OK;
}

int sort_path(lsm_t h, uint32_t tiles) {
  if (h->sort_mode == LSM_SORT_DIGIT_PASSES) return kSortLsd;
  if (h->sort_mode == LSM_SORT_TOP_DIGIT) return pick_sort_path(tiles, 0u);
  return pick_sort_path(tiles, *reinterpret_cast<volatile uint32_t*>(h->skew_host));
}
// Default depth of the fused cascade: level j is fused while a bucket of
// level j holds about 4096 elements on average (b 2^j / 256 <= 2^12).
int default_fuse_max(uint32_t b) {
  int J = 0;
  while (J < kMaxFuse && (static_cast<uint64_t>(b) << (J + 1)) <= (1ull << 20)) ++J;
  return J;
}

// Fuses the first levels of an insert's cascade into the top-digit sort.
// The sorted run stands for level `base` (0 for one batch; log2 G for a
// group of G batches, a run of that level's size); levels base..J-1 are
// merged with it in the bucket work-groups, J = min(j, fuse_max) cut short
// where a bucket would outgrow LDS and at the first level without a
// top-digit index for this key shift.  When J = j the sort writes level j
// (and its index); otherwise it writes the merge scratch buffer that the
// pairwise merge of level J then reads.
void setup_fusion(lsm_t h, SortArgs& sa, int j, int base) {
  sa.fuse.nlev = 0;
  sa.out_digit = nullptr;
  if (sa.path != kSortMsd || sort_top_shift(sa) < 1) return;
  const int shift = sort_top_shift(sa) - 1;
  if (j == base) {
    sa.out_digit = h->lvl_digit[base];
    return;
  }
  sa.out_digit = h->buf_digit;  // the sorted run, when no level is fused
  int J = j < h->fuse_max ? j : h->fuse_max;
  if (J > base + kMaxFuse) J = base + kMaxFuse;
  // Keep the fused runs of a bucket within LDS: one batch's largest bucket
  // (the previous sort's), grown 2^J times, must fit (skewed keys otherwise
  // leave one work-group ranking a huge bucket through global memory).
  const uint64_t big = *reinterpret_cast<volatile uint32_t*>(h->skew_host);
  while (J > base && (big << J) > static_cast<uint64_t>(kLocalCap)) --J;
  for (int l = base; l < J; ++l) {
    if (h->digit_shift[l] != shift) {
      J = l;
      break;
    }
  }
  const int nf = J - base;
  if (nf < 1) return;
  sa.out_digit = nullptr;
  FuseArgs& f = sa.fuse;
  f.nlev = nf;
  f.key_shift = shift;
  for (int q = 0; q < nf; ++q) {
    f.kv[q] = h->lvl_kv[base + q];
    f.val[q] = h->lvl_val[base + q];
    f.digit[q] = h->lvl_digit[base + q];
    f.len[q] = static_cast<uint32_t>(level_len(h, base + q));
  }
  f.out_len = level_len(h, J);
  if (J == j) {
    f.out_kv = h->lvl_kv[j];
    f.out_val = h->lvl_val[j];
    f.out_fence = h->lvl_fence[j];
    f.out_digit = h->lvl_digit[j];
  } else {
    f.out_kv = h->mrg_kv[(J + 1) & 1];
    f.out_val = h->mrg_val[(J + 1) & 1];
    f.out_fence = nullptr;
    f.out_digit = h->mrg_digit[(J + 1) & 1];
  }
}

// Records whether the level an insert wrote carries a top-digit index.
void note_digit_index(lsm_t h, const SortArgs& sa, int j, bool indexed) {
  h->digit_shift[j] = indexed ? sort_top_shift(sa) - 1 : -1;
}

// Merges partition their output by top-digit ranges (no split search) when
// the keys are not skewed: the latest sort's largest bucket is within a few
// times the mean bucket.  Either way the result is the same.
bool merge_by_digit(lsm_t h) {
  const uint64_t big = *reinterpret_cast<volatile uint32_t*>(h->skew_host);
  return big <= 4ull * ((h->b + kTopBuckets - 1) / kTopBuckets) + 32;
}

// Sort parameters of a batch: single-type batches sort the key variable
// without its (constant) status bit, mixed batches include it (sec. III-A
// rule 5 puts a batch's tombstone of a key before its insertion).
void sort_params(lsm_t h, int mode, SortArgs& sa) {
  sa.lo_bit = (mode == kMixed) ? 0 : 1;
  sa.passes = sort_passes(h->key_bits, sa.lo_bit);
  sa.key_limit_bits = h->key_bits;
}

// Arguments of a whole (non-pipelined) sort of the batch src for an insert
// into level j, with its fused cascade.
SortArgs sort_args(lsm_t h, const BatchSrc& src, int j, int path) {
  SortArgs sa{};
  sa.src = src;
  sort_params(h, src.mode, sa);
  sa.meta = sort_meta_carve(h->meta, h->b, h->hist_parity, 0);
  sa.tmp_kv[0] = path == kSortMsd ? h->scat_kv[0] : h->tmp_kv[0];
  sa.tmp_val[0] = path == kSortMsd ? h->scat_val[0] : h->tmp_val[0];
  sa.tmp_kv[1] = h->tmp_kv[1];
  sa.tmp_val[1] = h->tmp_val[1];
  sa.out_kv = (j == 0) ? h->lvl_kv[0] : h->buf_kv;
  sa.out_val = (j == 0) ? h->lvl_val[0] : h->buf_val;
  sa.out_fence = (j == 0) ? h->lvl_fence[0] : nullptr;
  sa.out_n = h->b;
  sa.path = path;
  sa.skew_out = h->skew_dev;
  setup_fusion(h, sa, j, 0);
  return sa;
}

// Arguments of the tile scatter of the batch src into slot `slot`; the
// launch will carry the next sequence number.
SortArgs scatter_args(lsm_t h, const BatchSrc& src, int slot) {
  SortArgs sa{};
  sa.progress = h->progress_dev;
  sa.seq = h->launch_seq + 1;
  sa.src = src;
  sort_params(h, src.mode, sa);
  sa.meta = sort_meta_carve(h->meta, h->b, h->hist_parity, slot);
  sa.tmp_kv[0] = h->scat_kv[slot];
  sa.tmp_val[0] = h->scat_val[slot];
  sa.tmp_kv[1] = h->tmp_kv[1];
  sa.tmp_val[1] = h->tmp_val[1];
  sa.out_n = h->b;
  sa.path = kSortMsd;
  sa.skew_out = h->skew_dev;
  return sa;
}

// Arguments of the bucket sort (and fused cascade) of the first G pending
// batches, a group (G = 1, 2 or 4 consecutive batches, the first one's
// counter a multiple of G), for the state of the levels they meet: every
// earlier batch's insertion has been enqueued.  *j receives the level the
// group's insertion fills (its newest batch's) and *base the level the
// sorted run stands for (log2 G: the group has that level's size).
SortArgs pending_args(lsm_t h, int G, int* j, int* base) {
  const lsm_s::Pending& p = h->pend[G - 1];  // the newest batch of the group
  SortArgs sa{};
  sa.src = BatchSrc{nullptr, nullptr, nullptr, h->b, h->b, kInsert};  // read from the slots
  sa.lo_bit = p.lo_bit;
  sa.passes = p.passes;
  sa.key_limit_bits = h->key_bits;
  sa.meta = sort_meta_carve(h->meta, h->b, h->hist_parity, p.slot);
  sa.tmp_kv[0] = h->scat_kv[0];  // every slot; batch q starts at grp_off[q]
  sa.tmp_val[0] = h->scat_val[0];
  sa.group = static_cast<uint32_t>(G);
  for (int q = 0; q < G; ++q) {
    const lsm_s::Pending& x = h->pend[G - 1 - q];  // newest first
    const SortMeta xm = sort_meta_carve(h->meta, h->b, h->hist_parity, x.slot);
    sa.grp_cnt[q] = xm.tile_cnt;
    sa.grp_n[q] = xm.bucket_n;
    sa.grp_off[q] = static_cast<uint32_t>(x.slot) * h->b;
  }
  sa.tmp_kv[1] = h->tmp_kv[1];
  sa.tmp_val[1] = h->tmp_val[1];
  *j = p.j;
  *base = G == 4 ? 2 : G == 2 ? 1 : 0;
  sa.out_kv = (p.j == *base) ? h->lvl_kv[p.j] : h->buf_kv;
  sa.out_val = (p.j == *base) ? h->lvl_val[p.j] : h->buf_val;
  sa.out_fence = (p.j == *base) ? h->lvl_fence[p.j] : nullptr;
  sa.out_n = static_cast<uint32_t>(G) * h->b;
  sa.path = kSortMsd;
  sa.skew_out = h->skew_dev;
  setup_fusion(h, sa, p.j, *base);
  return sa;
}

// Algorithmic bytes of the bucket half of a top-digit sort: the batch's key
// and value read and written, and with a fused cascade every element of the
// levels it takes over read and of the level it writes written.
double bucket_bytes(lsm_t h, const SortArgs& sa) {
  (void)h;
  return sa.fuse.nlev > 0 ? 16.0 * static_cast<double>(sa.fuse.out_len)
                          : 16.0 * static_cast<double>(sa.out_n);
}

// The cascade of Fig. 2(a): while level i is full, buffer <- merge(buffer,
// level i); the last merge writes straight into level j.  Enqueued on s,
// after the sort and after the levels the sort fused (whose output is then
// the first input).
// *indexed receives whether level j ends up with a top-digit index: written
// by the sort itself (j = 0, or every level fused), or by the last merge when
// both of its runs carried one (a run's index is the sort's, or a merge's of
// two indexed runs; level i's counts when built for the sort's key shift).
hipError_t enqueue_cascade(lsm_t h, const SortArgs& sa, int j, int base, hipStream_t s,
                           Timed* last, bool* indexed) {
  const int i0 = base + sa.fuse.nlev;
  const bool fused = sa.fuse.nlev > 0;
  const uint32_t* cur_kv = fused ? sa.fuse.out_kv : sa.out_kv;
  const uint32_t* cur_val = fused ? sa.fuse.out_val : sa.out_val;
  const uint32_t* cur_dig = fused ? sa.fuse.out_digit : sa.out_digit;
  const int shift = sort_top_shift(sa) - 1;
  const bool by_digit = merge_by_digit(h);
  if (indexed != nullptr) *indexed = (j == base) ? sa.out_digit != nullptr : (i0 == j && cur_dig);
  for (int i = i0; i < j; ++i) {
    uint32_t* o_kv = (i == j - 1) ? h->lvl_kv[j] : h->mrg_kv[i & 1];
    uint32_t* o_val = (i == j - 1) ? h->lvl_val[j] : h->mrg_val[i & 1];
    const uint32_t len = static_cast<uint32_t>(level_len(h, i));
    const bool both = cur_dig != nullptr && h->digit_shift[i] == shift;
    MergeIndex mi{cur_dig, both ? h->lvl_digit[i] : nullptr,
                  both ? ((i == j - 1) ? h->lvl_digit[j] : h->mrg_digit[i & 1]) : nullptr,
                  both && by_digit ? 1 : 0};
    Timed mt;
    const KTimer* t = (last != nullptr) ? timer(h, mt, kKMerge, 2ull * len, 16.0 * 2.0 * len) : nullptr;
    const hipError_t e = launch_merge(cur_kv, cur_val, len, h->lvl_kv[i], h->lvl_val[i], len,
                                      o_kv, o_val, (i == j - 1) ? h->lvl_fence[j] : nullptr,
                                      h->merge_variant[i], s, t, &mi);
    if (e != hipSuccess) return e;
    if (t != nullptr) *last = mt;
    cur_kv = o_kv;
    cur_val = o_val;
    cur_dig = mi.out_dig;
    if (indexed != nullptr && i == j - 1) *indexed = cur_dig != nullptr;
  }
  return hipSuccess;
}

// Sets *bad when any of n keys is >= 2^key_bits (checked mode); synchronises.
lsm_status_t check_keys(lsm_t h, const uint32_t* keys, uint32_t n, bool* bad) {
  const SortMeta m = sort_meta_carve(h->meta, h->b, 0, 0);
  if (hipMemsetAsync(m.err, 0, sizeof(uint32_t), h->stream) != hipSuccess ||
      launch_check_keys(keys, n, h->key_bits, 0, m.err, h->stream) != hipSuccess ||
      hipMemcpyAsync(h->h_pinned, m.err, sizeof(uint32_t), hipMemcpyDeviceToHost, h->stream) !=
          hipSuccess ||
      hipStreamSynchronize(h->stream) != hipSuccess)
    return LSM_EHIP;
  *bad = *reinterpret_cast<volatile uint32_t*>(h->h_pinned) != 0u;
  return LSM_OK;
}

void commit_insert(lsm_t h, int j) {
  const uint64_t merged = (j == 0) ? 0 : (2ull << j) * h->b - 2ull * h->b;
  h->r += 1;
  h->merged_last = merged;
  h->merged_total += merged;
  h->sorted_total += h->b;
}

// Enqueues the second half of the pending insertions: for each group, the
// bucket sort with its fused cascade, then the remaining merges.  A complete
// group (or a batch pending alone) is one group; an incomplete one is taken
// as aligned groups of 2 and 1, largest first.  The last group's sort runs
// in one launch with the tile scatter `next` when given.  On failure the
// batches not yet enqueued stay pending (their slots are untouched, so the
// work can be redone) and the state holds what was enqueued.
hipError_t launch_pending(lsm_t h, const SortArgs* next, Timed* first, Timed* last) {
  bool have_first = false;
  while (h->npend > 0) {
    int G = 1;
    while (2 * G <= h->npend) G *= 2;
    const SortArgs* nx = G == h->npend ? next : nullptr;
    int j = 0, base = 0;
    const SortArgs bk = pending_args(h, G, &j, &base);
    Timed ts;
    const double bytes = bucket_bytes(h, bk);
    const KTimer* t = nx != nullptr
                          ? timer(h, ts, kKSortStep, h->b, bytes + 16.0 * static_cast<double>(h->b))
                          : timer(h, ts, kKLocalSort, h->b, bytes);
    hipError_t e = nx != nullptr ? launch_sort_step(bk, *nx, h->stream, t)
                                 : launch_buckets(bk, h->stream, t);
    if (e != hipSuccess) return e;
    if (t != nullptr) {
      if (first && !have_first) *first = ts;
      have_first = true;
      if (last) *last = ts;
    }
    bool indexed = false;
    e = enqueue_cascade(h, bk, j, base, h->stream, t != nullptr ? last : nullptr, &indexed);
    if (e != hipSuccess) return e;
    note_digit_index(h, bk, j, indexed);
    for (int q = G; q < h->npend; ++q) h->pend[q - G] = h->pend[q];
    h->npend -= G;
  }
  return hipSuccess;
}

// Launch pacing.  With hundreds of update launches queued on the stream the
// device ran them markedly slower than with a few (measured in the design
// notes); so before enqueueing launch L = launch_seq + 1 the host waits until
// launch L - max_inflight has started, which it learns from the progress word
// that launch writes to mapped host memory (no runtime call).  Only top-digit
// launches count; the wait is bounded.
void pace(lsm_t h) {
  const uint64_t k = static_cast<uint64_t>(h->max_inflight > 0 ? h->max_inflight : 0);
  if (k == 0 || h->launch_seq < k) return;
  const uint64_t need = h->launch_seq + 1 - k;
  const volatile uint64_t* p = h->progress_host;
  if (*p >= need) return;
  const auto t0 = std::chrono::steady_clock::now();
  for (uint32_t spin = 1; *p < need; ++spin) {
    if ((spin & 255u) == 0 &&
        std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(kPaceLimitMs)) {
      h->pace_timeouts += 1;
      return;
    }
  }
}

// Completes the pending insertion, if any: everything that reads the levels
// calls this first.
lsm_status_t drain(lsm_t h) {
  if (h->npend == 0) return LSM_OK;
  const int slot = h->pend[h->npend - 1].slot;  // its record holds the last sort's buckets
  Timed first, last;
  if (launch_pending(h, nullptr, &first, &last) != hipSuccess) return LSM_EHIP;
  // Hand the just-sorted batch's largest bucket to the host-visible hint
  // (within a pipelined stream a later scatter hands it over, one batch
  // late), so that a caller that synchronises sees the latest sort's skew.
  // A failed launch only leaves the hint older; the insertion itself is done.
  const SortMeta m = sort_meta_carve(h->meta, h->b, h->hist_parity, slot);
  if (launch_rec_max(m.bucket_n, h->skew_dev, h->stream) != hipSuccess) (void)hipGetLastError();
  return LSM_OK;
}

// One update batch (sec. III-B insertion; deletions and mixed batches are
// insertions whose elements carry status 0 where they delete).
//
// Batches sorted by the top-digit sort are pipelined: this call scatters the
// batch's tiles and, in the same launch, sorts the buckets of the previous
// batch and merges them into that batch's level; this batch's buckets follow
// at the next update or when anything reads the levels.  The caller's arrays
// are read only by this call's launch.  Other batches (digit-pass sort) first
// complete the pending one, then are sorted and merged in this call.
lsm_status_t update_batch(lsm_t h, const uint32_t* keys, const uint32_t* vals,
                          const uint8_t* is_delete, uint32_t n, BatchMode mode) {
  if (h == nullptr) return LSM_EINVAL;
  if (n == 0) return LSM_OK;
  if (n > h->b) return LSM_EBATCH;
  if (keys == nullptr || (mode != kDelete && mode != kEncoded && vals == nullptr) ||
      (mode == kMixed && is_delete == nullptr))
    return LSM_EINVAL;
  DeviceGuard g(h->device);
  if (!g.ok) return LSM_EHIP;

  // First empty level j = ffz(r) (r counts the pending batch); the batch's
  // insertion fills it with b * 2^j elements.  Everything it needs is
  // allocated now, so the deferred half cannot fail for want of memory.
  const int j = __builtin_ctzll(~h->r);
  lsm_status_t s = prepare_insert(h, j);
  if (s != LSM_OK) return s;
  if ((h->flags & LSM_CHECKED) && mode != kEncoded) {
    bool bad = false;
    s = check_keys(h, keys, n, &bad);
    if (s != LSM_OK) return s;
    if (bad) return LSM_EKEY;
  }
  const BatchSrc src{keys, vals, is_delete, n, h->b, static_cast<int>(mode)};
  const int path = sort_path(h, sort_meta_carve(h->meta, h->b, 0, 0).num_sort_tiles);

  if (path == kSortMsd) {
    // This batch's slot: one that no pending batch holds.
    int slot = 0;
    for (bool taken = true; taken; ) {
      taken = false;
      for (int q = 0; q < h->npend; ++q) taken |= h->pend[q].slot == slot;
      if (taken) ++slot;
    }
    pace(h);
    const SortArgs sc = scatter_args(h, src, slot);
    // This batch joins the pending group when the group started at a
    // counter that is a multiple of group_max, is not complete, and this
    // batch is the next one; otherwise the pending batches' buckets run
    // beside this batch's scatter.  Only batches whose sort leaves the
    // status bit out are grouped: a stable sort of the group on the original
    // key, the newer batches first, is then what merging the batches one by
    // one gives.  (A mixed batch sorts its tombstone of a key before its
    // insertion, which a group's sort would apply across batches.)
    const uint64_t r0 = h->r;
    const int gm = h->group_max;
    const bool join = gm > 1 && h->npend > 0 && h->npend < gm &&
                      h->pend[0].r % static_cast<uint64_t>(gm) == 0 &&
                      r0 == h->pend[h->npend - 1].r + 1 && h->pend[0].lo_bit == 1 &&
                      sc.lo_bit == 1 && h->pend[0].passes == sc.passes;
    Timed first, last;
    hipError_t e;
    if (h->npend > 0 && !join) {
      e = launch_pending(h, &sc, &first, &last);
    } else {
      const KTimer* t = timer(h, first, kKMsdScatter, h->b, 16.0 * h->b);
      e = launch_scatter(sc, h->stream, t);
      last = first;
    }
    if (e != hipSuccess) return LSM_EHIP;
    h->launch_seq += 1;
    if (h->prof) call_span(h, kSpanUpdate, first, last, h->b);
    const lsm_s::Pending np{slot, j, sc.lo_bit, sc.passes, r0};
    h->pend[h->npend] = np;  // launch_pending emptied the list; a group appends
    h->npend += 1;
    h->sorts_by_path[kSortMsd] += 1;
    commit_insert(h, j);
    return LSM_OK;
  }

  s = drain(h);
  if (s != LSM_OK) return s;
  SortArgs sa = sort_args(h, src, j, path);
  Timed st[1 + kMaxPasses];
  KTimer sort_t[1 + kMaxPasses];
  bool timed = h->prof;
  const int nk = sort_kernel_count(sa);
  for (int p = 0; p < nk && timed; ++p) {
    const KTimer* t = timer(h, st[p], sort_kernel_kind(sa.path, p), h->b,
                            sort_kernel_bytes_per_elem(sa.path, p) * h->b);
    if (t == nullptr) timed = false;
    else sort_t[p] = *t;
  }
  int launched = 0;
  const hipError_t se = launch_sort(sa, h->stream, timed ? sort_t : nullptr, &launched);
  // The digit-pass sort's first kernel clears the other histogram buffer for
  // the next such sort; once it has been launched, the next one must use
  // that buffer whether or not the rest of the sort was launched.
  if (sa.path == kSortLsd && launched > 0) h->hist_parity ^= 1;
  if (se != hipSuccess) return LSM_EHIP;
  Timed last = st[nk - 1];
  bool indexed = false;
  if (enqueue_cascade(h, sa, j, 0, h->stream, timed ? &last : nullptr, &indexed) != hipSuccess)
    return LSM_EHIP;
  if (timed) call_span(h, kSpanUpdate, st[0], last, h->b);
  note_digit_index(h, sa, j, indexed);
  h->sorts_by_path[path] += 1;
  commit_insert(h, j);
  return LSM_OK;
}

// Inserts the staged batch (n elements, padded when n < b).
lsm_status_t insert_staged(lsm_t h, uint32_t n) {
  const lsm_status_t s = update_batch(h, h->stage_kv, h->stage_val, nullptr, n, kEncoded);
  if (s == LSM_OK) h->stage_fill = 0;
  return s;
}

lsm_status_t flush_staged(lsm_t h) {
  if (h->stage_fill == 0) return LSM_OK;
  return insert_staged(h, h->stage_fill);
}

// Before anything reads the levels: the staged elements are inserted and
// the pending insertion completed.
lsm_status_t settle(lsm_t h) {
  const lsm_status_t s = flush_staged(h);
  return s != LSM_OK ? s : drain(h);
}

// A batch handed to lsm_insert_batch / lsm_delete_batch / lsm_update_batch.
// Elements staged by the coalescer are older than it, so they are inserted
// first, as their own (padded) batch.  Everything the direct batch can be
// refused for (arguments, allocations for both insertions, keys in checked
// mode) is settled before the staged batch goes in.
lsm_status_t direct_update(lsm_t h, const uint32_t* keys, const uint32_t* vals,
                           const uint8_t* is_delete, uint32_t n, BatchMode mode) {
  if (h == nullptr) return LSM_EINVAL;
  if (n == 0) return LSM_OK;
  if (n > h->b) return LSM_EBATCH;
  if (keys == nullptr || (mode != kDelete && vals == nullptr) ||
      (mode == kMixed && is_delete == nullptr))
    return LSM_EINVAL;
  if (h->stage_fill > 0) {
    DeviceGuard g(h->device);
    if (!g.ok) return LSM_EHIP;
    lsm_status_t s = prepare_insert(h, __builtin_ctzll(~h->r));
    if (s == LSM_OK) s = prepare_insert(h, __builtin_ctzll(~(h->r + 1)));
    if (s != LSM_OK) return s;
    if (h->flags & LSM_CHECKED) {
      bool bad = false;
      s = check_keys(h, keys, n, &bad);
      if (s != LSM_OK) return s;
      if (bad) return LSM_EKEY;
    }
    s = flush_staged(h);
    if (s != LSM_OK) return s;
  }
  return update_batch(h, keys, vals, is_delete, n, mode);
}

}  // namespace

extern "C" {

lsm_status_t lsm_create(lsm_t* out, uint32_t b, uint32_t flags, void* stream) {
  if (out == nullptr) return LSM_EINVAL;
  *out = nullptr;
  if (b == 0 || b > (1u << 28)) return LSM_EINVAL;
  if (flags & ~(LSM_CHECKED | LSM_KEY_BITS(0x3F))) return LSM_EINVAL;
  uint32_t kb = (flags >> 8) & 0x3Fu;
  if (kb == 0) kb = 31;
  if (kb > 31) return LSM_EINVAL;

  lsm_t h = new (std::nothrow) lsm_s();
  if (h == nullptr) return LSM_ENOMEM;
  h->b = b;
  h->fuse_max = default_fuse_max(b);
  for (int i = 0; i < kMaxLevels; ++i) h->digit_shift[i] = -1;
  h->flags = flags;
  h->key_bits = kb;
  h->stream = static_cast<hipStream_t>(stream);
  if (hipGetDevice(&h->device) != hipSuccess) {
    delete h;
    return LSM_EHIP;
  }
  const size_t bb = static_cast<size_t>(b) * sizeof(uint32_t);
  {
    const uint32_t tiles = (b + kSortTile - 1) / kSortTile;
    h->grp_cap = 4u * tiles <= static_cast<uint32_t>(kMsdMaxTiles)   ? 4u
                 : 2u * tiles <= static_cast<uint32_t>(kMsdMaxTiles) ? 2u
                                                                      : 1u;
    // Pairs by default: groups of four measured no faster at b = 2^16 (their
    // buckets outgrow the rank sort and take three LDS radix passes).
    h->group_max = h->grp_cap < 2u ? 1 : 2;
  }
  void* p = nullptr;
  lsm_status_t s = LSM_OK;
  for (int i = 0; i < 2 && s == LSM_OK; ++i) {
    const size_t sz = i == 1 ? h->grp_cap * bb : bb;
    if ((s = dev_alloc(h, &p, sz)) == LSM_OK) h->tmp_kv[i] = static_cast<uint32_t*>(p);
    if (s == LSM_OK && (s = dev_alloc(h, &p, sz)) == LSM_OK) h->tmp_val[i] = static_cast<uint32_t*>(p);
  }
  if (s == LSM_OK && (s = dev_alloc(h, &p, kSortSlots * bb)) == LSM_OK)
    for (int i = 0; i < kSortSlots; ++i) h->scat_kv[i] = static_cast<uint32_t*>(p) + static_cast<size_t>(i) * b;
  if (s == LSM_OK && (s = dev_alloc(h, &p, kSortSlots * bb)) == LSM_OK)
    for (int i = 0; i < kSortSlots; ++i) h->scat_val[i] = static_cast<uint32_t*>(p) + static_cast<size_t>(i) * b;
  for (int i = 0; i < 2 && s == LSM_OK; ++i)
    if ((s = dev_alloc(h, &p, kTopBuckets * sizeof(uint32_t))) == LSM_OK)
      h->mrg_digit[i] = static_cast<uint32_t*>(p);
  if (s == LSM_OK && (s = dev_alloc(h, &p, kTopBuckets * sizeof(uint32_t))) == LSM_OK)
    h->buf_digit = static_cast<uint32_t*>(p);
  for (int i = 0; i < kMaxLevels; ++i) h->merge_variant[i] = kDefaultMergeVariant;
  if (s == LSM_OK && (s = dev_alloc(h, &p, bb)) == LSM_OK) h->stage_kv = static_cast<uint32_t*>(p);
  if (s == LSM_OK && (s = dev_alloc(h, &p, bb)) == LSM_OK) h->stage_val = static_cast<uint32_t*>(p);
  if (s == LSM_OK && (s = dev_alloc(h, &p, h->grp_cap * bb)) == LSM_OK) h->buf_kv = static_cast<uint32_t*>(p);
  if (s == LSM_OK && (s = dev_alloc(h, &p, h->grp_cap * bb)) == LSM_OK) h->buf_val = static_cast<uint32_t*>(p);
  if (s == LSM_OK && (s = dev_alloc(h, &p, sort_meta_words(b) * sizeof(uint32_t))) == LSM_OK) {
    h->meta = static_cast<uint32_t*>(p);
    h->fault = sort_meta_carve(h->meta, b, 0, 0).err + 1;
    // Both global histogram buffers start zeroed (each sort then clears
    // the buffer of the next one).
    if (hipMemset(h->meta, 0, sort_meta_words(b) * sizeof(uint32_t)) != hipSuccess) s = LSM_EHIP;
  }
  if (s == LSM_OK) {
    void* hp = nullptr;
    if (hipHostMalloc(&hp, 64, hipHostMallocDefault) != hipSuccess) s = LSM_ENOMEM;
    else h->h_pinned = static_cast<uint64_t*>(hp);
  }
  if (s == LSM_OK) {
    void* hp = nullptr;
    void* dp = nullptr;
    if (hipHostMalloc(&hp, 64, hipHostMallocMapped) != hipSuccess) {
      s = LSM_ENOMEM;
    } else {
      h->skew_host = static_cast<uint32_t*>(hp);
      *h->skew_host = 0u;
      if (hipHostGetDevicePointer(&dp, hp, 0) != hipSuccess) s = LSM_EHIP;
      else h->skew_dev = static_cast<uint32_t*>(dp);
    }
  }
  if (s == LSM_OK) {
    void* hp = nullptr;
    void* dp = nullptr;
    if (hipHostMalloc(&hp, 64, hipHostMallocMapped) != hipSuccess) {
      s = LSM_ENOMEM;
    } else {
      h->progress_host = static_cast<uint64_t*>(hp);
      *h->progress_host = 0u;
      if (hipHostGetDevicePointer(&dp, hp, 0) != hipSuccess) s = LSM_EHIP;
      else h->progress_dev = static_cast<uint64_t*>(dp);
    }
  }
  if (s != LSM_OK) {
    release_all(h);
    delete h;
    return s;
  }
  // The fixed range scratch of this device (looked up once per device); a
  // failed lookup only disables lsm_range_async_noalloc.
  if (fixed_scratch(&h->fixed) != hipSuccess) {
    (void)hipGetLastError();
    h->fixed = FixedScratch{nullptr, nullptr};
  }
  *out = h;
  return LSM_OK;
}

lsm_status_t lsm_set_stream(lsm_t h, void* stream) {
  if (h == nullptr) return LSM_EINVAL;
  h->stream = static_cast<hipStream_t>(stream);
  return LSM_OK;
}

lsm_status_t lsm_insert_batch(lsm_t h, const uint32_t* d_keys, const uint32_t* d_vals, uint32_t n) {
  return direct_update(h, d_keys, d_vals, nullptr, n, kInsert);
}

lsm_status_t lsm_delete_batch(lsm_t h, const uint32_t* d_keys, uint32_t n) {
  return direct_update(h, d_keys, nullptr, nullptr, n, kDelete);
}

lsm_status_t lsm_update_batch(lsm_t h, const uint32_t* d_keys, const uint32_t* d_vals,
                              const uint8_t* d_is_delete, uint32_t n) {
  return direct_update(h, d_keys, d_vals, d_is_delete, n, kMixed);
}

lsm_status_t lsm_lookup(lsm_t h, const uint32_t* d_keys, uint32_t nq, uint32_t* d_vals,
                        uint8_t* d_found) {
  if (h == nullptr) return LSM_EINVAL;
  if (nq == 0) return LSM_OK;
  if (d_keys == nullptr || d_vals == nullptr || d_found == nullptr) return LSM_EINVAL;
  DeviceGuard g(h->device);
  if (!g.ok) return LSM_EHIP;
  lsm_status_t fs = settle(h);
  if (fs != LSM_OK) return fs;
  const LevelSet lv = occupied_levels(h);
  Timed tl;
  const KTimer* t = timer(h, tl, kKLookup, nq, 0.0);
  if (launch_lookup(lv, d_keys, nq, d_vals, d_found, h->stream, t) != hipSuccess) return LSM_EHIP;
  if (t != nullptr) call_span(h, kSpanLookup, tl, tl, nq);
  return LSM_OK;
}

lsm_status_t lsm_count(lsm_t h, const uint32_t* d_lo, const uint32_t* d_hi, uint32_t nq,
                       uint32_t* d_counts) {
  if (h == nullptr) return LSM_EINVAL;
  if (nq == 0) return LSM_OK;
  if (d_lo == nullptr || d_hi == nullptr || d_counts == nullptr) return LSM_EINVAL;
  DeviceGuard g(h->device);
  if (!g.ok) return LSM_EHIP;
  lsm_status_t fs = settle(h);
  if (fs != LSM_OK) return fs;
  const LevelSet lv = occupied_levels(h);
  Timed tc;
  const KTimer* t = timer(h, tc, kKCount, nq, 0.0);
  if (launch_count(lv, d_lo, d_hi, nq, d_counts, nullptr, 0, nullptr, h->stream, t) != hipSuccess)
    return LSM_EHIP;
  if (t != nullptr) call_span(h, kSpanCount, tc, tc, nq);
  return LSM_OK;
}

static lsm_status_t order_query(lsm_t h, const uint32_t* d_q, uint32_t nq, uint32_t* d_keys,
                         uint32_t* d_vals, uint8_t* d_found, bool successor) {
  if (h == nullptr) return LSM_EINVAL;
  if (nq == 0) return LSM_OK;
  if (d_q == nullptr || d_keys == nullptr || d_vals == nullptr || d_found == nullptr)
    return LSM_EINVAL;
  DeviceGuard g(h->device);
  if (!g.ok) return LSM_EHIP;
  const lsm_status_t fs = settle(h);
  if (fs != LSM_OK) return fs;
  const LevelSet lv = occupied_levels(h);
  Timed to;
  const KTimer* t = timer(h, to, kKOrder, nq, 0.0);
  const hipError_t e = successor
                           ? launch_successor(lv, d_q, nq, d_keys, d_vals, d_found, h->stream, t)
                           : launch_predecessor(lv, d_q, nq, d_keys, d_vals, d_found, h->stream, t);
  return e == hipSuccess ? LSM_OK : LSM_EHIP;
}

lsm_status_t lsm_successor(lsm_t h, const uint32_t* d_q, uint32_t nq, uint32_t* d_keys,
                           uint32_t* d_vals, uint8_t* d_found) {
  return order_query(h, d_q, nq, d_keys, d_vals, d_found, true);
}

lsm_status_t lsm_predecessor(lsm_t h, const uint32_t* d_q, uint32_t nq, uint32_t* d_keys,
                             uint32_t* d_vals, uint8_t* d_found) {
  return order_query(h, d_q, nq, d_keys, d_vals, d_found, false);
}

// Multi-batch insert (sec. V-B, bulk build and its footnote): n pairs as
// ceil(n / b) consecutive insert batches of b, the last one padded.  Each
// level of the new batch count r1 = r + k that holds a new batch is built
// once: the new batches of its batch range are sorted together (read back to
// front, stable, as one batch), then merged with the old levels its range
// takes over, newest first.  Levels are produced from the largest down, so
// an old level is always read before a smaller new level overwrites it.
lsm_status_t lsm_bulk_insert(lsm_t h, const uint32_t* d_keys, const uint32_t* d_vals, uint64_t n) {
  if (h == nullptr) return LSM_EINVAL;
  if (n == 0) return LSM_OK;
  if (d_keys == nullptr || d_vals == nullptr) return LSM_EINVAL;
  if (n > 0xFFFFFFFFull) return LSM_ECAPACITY;
  DeviceGuard g(h->device);
  if (!g.ok) return LSM_EHIP;
  // Staged elements become one batch before the new ones; every allocation
  // (theirs included) is made before anything changes.
  lsm_status_t s = h->stage_fill > 0 ? prepare_insert(h, __builtin_ctzll(~h->r)) : LSM_OK;
  if (s != LSM_OK) return s;
  const uint64_t b = h->b;
  const uint64_t k = (n + b - 1) / b;
  const uint64_t r0 = h->r + (h->stage_fill > 0 ? 1 : 0), r1 = r0 + k;
  if ((r1 >> kMaxLevels) != 0) return LSM_ECAPACITY;

  struct Plan {
    int level;
    uint64_t first_new;  // first new batch in the level's range
    uint64_t end;        // end of the range (batch number)
    int old[kMaxLevels];
    int n_old;
  };
  Plan plan[kMaxLevels];
  int np = 0;
  uint64_t max_new = 0, max_level = 0;
  bool merges = false;
  for (int i = kMaxLevels - 1; i >= 0; --i) {
    if (((r1 >> i) & 1u) == 0) continue;
    const uint64_t lo = (r1 >> (i + 1)) << (i + 1), hi = lo + (1ull << i);
    if (hi <= r0) continue;  // the same range as old level i: unchanged
    if (level_len(h, i) > (1ull << 31)) return LSM_ECAPACITY;
    Plan& p = plan[np++];
    p.level = i;
    p.first_new = lo > r0 ? lo : r0;
    p.end = hi;
    p.n_old = 0;
    for (int j = 0; j < i; ++j) {
      if (((r0 >> j) & 1u) == 0) continue;
      if (((r0 >> (j + 1)) << (j + 1)) >= lo) p.old[p.n_old++] = j;  // newest first
    }
    max_new = std::max(max_new, (p.end - p.first_new) * b);
    max_level = std::max(max_level, level_len(h, i));
    merges = merges || p.n_old > 0;
  }

  if (h->flags & LSM_CHECKED) {
    const SortMeta m = sort_meta_carve(h->meta, h->b, 0, 0);
    if (hipMemsetAsync(m.err, 0, sizeof(uint32_t), h->stream) != hipSuccess ||
        launch_check_keys(d_keys, static_cast<uint32_t>(n), h->key_bits, 0, m.err, h->stream) !=
            hipSuccess ||
        hipMemcpyAsync(h->h_pinned, m.err, sizeof(uint32_t), hipMemcpyDeviceToHost, h->stream) !=
            hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess)
      return LSM_EHIP;
    if (*reinterpret_cast<volatile uint32_t*>(h->h_pinned) != 0u) return LSM_EKEY;
  }

  // Scratch: the sort's ping-pong and look-back words for the largest new
  // part; two merge buffers when a level takes over old levels.
  const size_t meta_bytes = sort_meta_words(static_cast<uint32_t>(max_new)) * sizeof(uint32_t);
  void* st[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};  // [buffer][kv, val]
  void* mg[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  void* meta = nullptr;
  auto release = [&]() {
    for (int q = 0; q < 2; ++q)
      for (int c = 0; c < 2; ++c) {
        dev_free(h, st[q][c], max_new * sizeof(uint32_t));
        dev_free(h, mg[q][c], max_level * sizeof(uint32_t));
      }
    dev_free(h, meta, meta_bytes);
  };
  for (int q = 0; q < 2 && s == LSM_OK; ++q)
    for (int c = 0; c < 2 && s == LSM_OK; ++c) {
      s = dev_alloc(h, &st[q][c], max_new * sizeof(uint32_t));
      if (s == LSM_OK && merges) s = dev_alloc(h, &mg[q][c], max_level * sizeof(uint32_t));
    }
  if (s == LSM_OK) s = dev_alloc(h, &meta, meta_bytes);
  for (int q = 0; q < np && s == LSM_OK; ++q) s = ensure_level(h, plan[q].level);
  if (s != LSM_OK) {
    release();
    return s;
  }
  s = settle(h);  // allocates nothing now
  if (s != LSM_OK || h->r != r0) {
    release();
    return s != LSM_OK ? s : LSM_EHIP;
  }
  auto u32 = [](void* p) { return static_cast<uint32_t*>(p); };
  hipError_t e = hipMemsetAsync(meta, 0, meta_bytes, h->stream);
  uint64_t merged = 0, sorted = 0;
  int parity = 0;
  for (int q = 0; q < np && e == hipSuccess; ++q) {
    const Plan& p = plan[q];
    const int i = p.level;
    const uint64_t e0 = (p.first_new - r0) * b;          // first input element
    const uint64_t len = (p.end - p.first_new) * b;      // padded length
    const uint64_t avail = n - e0 < len ? n - e0 : len;  // real elements
    SortArgs sa{};
    sa.src = BatchSrc{d_keys + e0, d_vals + e0, nullptr, static_cast<uint32_t>(avail),
                      static_cast<uint32_t>(len), static_cast<int>(kInsert)};
    sort_params(h, kInsert, sa);
    sa.meta = sort_meta_carve(u32(meta), static_cast<uint32_t>(len), parity, 0);
    sa.tmp_kv[0] = u32(st[0][0]);
    sa.tmp_val[0] = u32(st[0][1]);
    sa.tmp_kv[1] = u32(st[1][0]);
    sa.tmp_val[1] = u32(st[1][1]);
    sa.out_kv = p.n_old == 0 ? h->lvl_kv[i] : u32(mg[0][0]);
    sa.out_val = p.n_old == 0 ? h->lvl_val[i] : u32(mg[0][1]);
    sa.out_fence = p.n_old == 0 ? h->lvl_fence[i] : nullptr;
    sa.out_n = static_cast<uint32_t>(len);
    sa.path = sort_path(h, sa.meta.num_sort_tiles);
    sa.skew_out = h->skew_dev;
    Timed ts[1 + kMaxPasses];
    KTimer tt[1 + kMaxPasses];
    const int nk = sort_kernel_count(sa);
    bool timed = h->prof;
    for (int x = 0; x < nk && timed; ++x) {
      const KTimer* t = timer(h, ts[x], sort_kernel_kind(sa.path, x), len,
                              sort_kernel_bytes_per_elem(sa.path, x) * len);
      if (t == nullptr) timed = false;
      else tt[x] = *t;
    }
    int launched = 0;
    e = launch_sort(sa, h->stream, timed ? tt : nullptr, &launched);
    if (sa.path == kSortLsd && launched > 0) parity ^= 1;  // see update_batch
    sorted += len;
    const uint32_t* ak = sa.out_kv;
    const uint32_t* av = sa.out_val;
    uint64_t alen = len;
    for (int x = 0; x < p.n_old && e == hipSuccess; ++x) {
      const int j = p.old[x];
      const bool last = x == p.n_old - 1;
      uint32_t* ok = last ? h->lvl_kv[i] : u32(mg[(x + 1) & 1][0]);
      uint32_t* ov = last ? h->lvl_val[i] : u32(mg[(x + 1) & 1][1]);
      const uint64_t lj = level_len(h, j);
      Timed mt;
      e = launch_merge(ak, av, static_cast<uint32_t>(alen), h->lvl_kv[j], h->lvl_val[j],
                       static_cast<uint32_t>(lj), ok, ov, last ? h->lvl_fence[i] : nullptr,
                       h->merge_variant[j], h->stream,
                       timer(h, mt, kKMerge, alen + lj, 16.0 * (alen + lj)));
      ak = ok;
      av = ov;
      alen += lj;
      merged += alen;
    }
  }
  const hipError_t e2 = hipStreamSynchronize(h->stream);
  release();
  if (e != hipSuccess || e2 != hipSuccess) return LSM_EHIP;
  for (int q = 0; q < np; ++q) h->digit_shift[plan[q].level] = -1;
  h->r = r1;
  h->merged_last = merged;
  h->merged_total += merged;
  h->sorted_total += sorted;
  return LSM_OK;
}

// Cleanup (sec. III-E) by the bulk strategy of sec. IV-D.  Stage 1 merges
// the occupied levels from the smallest up into scratch (the accumulated,
// newer run first on equal keys), so the redistribution never writes a level
// it still reads; stages 2-5 count the valid elements per tile, scan the
// counts, and after one read-back of the total scatter the valid elements
// straight into the levels of the new batch count and pad with placebos.
lsm_status_t lsm_cleanup(lsm_t h, uint64_t* h_valid) {
  if (h == nullptr) return LSM_EINVAL;
  DeviceGuard g(h->device);
  if (!g.ok) return LSM_EHIP;
  if (h_valid != nullptr) *h_valid = 0;
  // Everything is allocated before anything changes: the staged elements'
  // level, the scratch, and every level the rebuilt dictionary can occupy
  // (r' <= r, so levels up to r's highest; they all existed already unless a
  // bulk insert or cleanup skipped some).
  lsm_status_t s = h->stage_fill > 0 ? prepare_insert(h, __builtin_ctzll(~h->r)) : LSM_OK;
  if (s != LSM_OK) return s;
  const uint64_t r_all = h->r + (h->stage_fill > 0 ? 1 : 0);
  if (r_all == 0) return drain(h);
  const uint64_t total = r_all * static_cast<uint64_t>(h->b);
  if (total > 0xFFFFFFFFull) return LSM_ECAPACITY;
  for (int i = 0; i < kMaxLevels && (r_all >> i) != 0 && s == LSM_OK; ++i) s = ensure_level(h, i);
  if (s != LSM_OK) return s;
  const uint32_t n = static_cast<uint32_t>(total);
  int occ[kMaxLevels];
  int m = 0;
  for (int i = 0; i < kMaxLevels; ++i)
    if ((r_all >> i) & 1u) occ[m++] = i;

  // Scratch: one or two merge buffers (kv + val), the tiles' offsets.
  const size_t bytes = total * sizeof(uint32_t);
  const uint32_t tiles = clean_tiles(n);
  void* tk[2] = {nullptr, nullptr};
  void* tv[2] = {nullptr, nullptr};
  void* toff = nullptr;
  const int nbuf = m >= 3 ? 2 : 1;
  auto release = [&]() {
    for (int q = 0; q < 2; ++q) {
      dev_free(h, tk[q], bytes);
      dev_free(h, tv[q], bytes);
    }
    dev_free(h, toff, (tiles + 1ull) * sizeof(uint64_t));
  };
  for (int q = 0; q < nbuf && s == LSM_OK; ++q) {
    s = dev_alloc(h, &tk[q], bytes);
    if (s == LSM_OK) s = dev_alloc(h, &tv[q], bytes);
  }
  if (s == LSM_OK) s = dev_alloc(h, &toff, (tiles + 1ull) * sizeof(uint64_t));
  if (s == LSM_OK) s = ensure_query_scratch(h, tiles);
  if (s == LSM_OK) s = settle(h);  // allocates nothing now
  if (s == LSM_OK && h->r != r_all) s = LSM_EHIP;
  if (s != LSM_OK) {
    release();
    return s;
  }
  hipError_t e = hipSuccess;
  const uint32_t* ak = h->lvl_kv[occ[0]];
  const uint32_t* av = h->lvl_val[occ[0]];
  uint64_t alen = level_len(h, occ[0]);
  if (m == 1) {
    e = hipMemcpyAsync(tk[0], ak, bytes, hipMemcpyDeviceToDevice, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(tv[0], av, bytes, hipMemcpyDeviceToDevice, h->stream);
    ak = static_cast<uint32_t*>(tk[0]);
    av = static_cast<uint32_t*>(tv[0]);
  }
  for (int k = 1; k < m && e == hipSuccess; ++k) {
    const int i = occ[k];
    const uint64_t len = level_len(h, i);
    uint32_t* ok = static_cast<uint32_t*>(tk[(k - 1) & 1]);
    uint32_t* ov = static_cast<uint32_t*>(tv[(k - 1) & 1]);
    Timed mt;
    e = launch_merge(ak, av, static_cast<uint32_t>(alen), h->lvl_kv[i], h->lvl_val[i],
                     static_cast<uint32_t>(len), ok, ov, nullptr, kDefaultMergeVariant, h->stream,
                     timer(h, mt, kKMerge, alen + len, 16.0 * (alen + len)));
    ak = ok;
    av = ov;
    alen += len;
  }
  uint64_t* tile_off = static_cast<uint64_t*>(toff);
  Timed t1, t2;
  if (e == hipSuccess)
    e = launch_clean_count(ak, n, h->q_counts, h->q_status, scan_status_words(tiles), h->stream,
                           timer(h, t1, kKClean, total, 4.0 * total));
  if (e == hipSuccess)
    e = launch_scan(h->q_counts, tiles, tile_off, h->q_status, h->fault, h->stream,
                    timer(h, t2, kKScan, tiles, 12.0 * tiles));
  if (e == hipSuccess)
    e = hipMemcpyAsync(h->h_pinned, tile_off + tiles, sizeof(uint64_t), hipMemcpyDeviceToHost,
                       h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    (void)hipStreamSynchronize(h->stream);
    release();
    return LSM_EHIP;
  }
  const uint64_t v = *reinterpret_cast<volatile uint64_t*>(h->h_pinned);
  const uint64_t r2 = (v + h->b - 1) / h->b;  // <= r_all: its levels exist
  LevelDst d{};
  for (int i = 0; i < kMaxLevels; ++i) {
    if (((r2 >> i) & 1u) == 0) continue;
    d.kv[d.count] = h->lvl_kv[i];
    d.val[d.count] = h->lvl_val[i];
    d.fence[d.count] = h->lvl_fence[i];
    d.start[d.count] = static_cast<uint64_t>(h->b) * (r2 & ((1ull << i) - 1ull));
    d.len[d.count] = level_len(h, i);
    ++d.count;
  }
  Timed t3, t4;
  e = launch_clean_scatter(ak, av, n, tile_off, d, h->stream,
                           timer(h, t3, kKClean, total, 8.0 * total + 8.0 * v));
  if (e == hipSuccess)
    e = launch_clean_pad(d, v, r2 * h->b, h->stream,
                         timer(h, t4, kKClean, r2 * h->b - v, 8.0 * (r2 * h->b - v)));
  const hipError_t e2 = hipStreamSynchronize(h->stream);
  release();
  if (e != hipSuccess || e2 != hipSuccess) return LSM_EHIP;
  for (int i = 0; i < kMaxLevels; ++i)
    if ((r2 >> i) & 1u) h->digit_shift[i] = -1;
  h->r = r2;
  h->merged_last = 0;
  if (h_valid != nullptr) *h_valid = v;
  return LSM_OK;
}

lsm_status_t lsm_range(lsm_t h, const uint32_t* d_lo, const uint32_t* d_hi, uint32_t nq,
                       uint64_t* d_offsets, uint32_t* d_keys, uint32_t* d_vals, uint64_t cap,
                       uint64_t* h_total) {
  if (h == nullptr || h_total == nullptr || d_offsets == nullptr) return LSM_EINVAL;
  if (nq > 0 && (d_lo == nullptr || d_hi == nullptr)) return LSM_EINVAL;
  if (cap > 0 && (d_keys == nullptr || d_vals == nullptr)) return LSM_EINVAL;
  DeviceGuard g(h->device);
  if (!g.ok) return LSM_EHIP;
  if (nq == 0) {
    *h_total = 0;
    return hipMemsetAsync(d_offsets, 0, sizeof(uint64_t), h->stream) == hipSuccess ? LSM_OK
                                                                                  : LSM_EHIP;
  }
  lsm_status_t s = ensure_query_scratch(h, nq);
  if (s == LSM_OK) s = ensure_bounds(h, nq);
  if (s == LSM_OK) s = settle(h);
  if (s != LSM_OK) return s;
  const LevelSet lv = occupied_levels(h);
  Timed t1, t2, t3;
  // Stage 1: per-query live counts (also clears the scan's look-back words).
  if (launch_count(lv, d_lo, d_hi, nq, h->q_counts, h->q_status, scan_status_words(nq),
                   h->q_bounds, h->stream, timer(h, t1, kKCount, nq, 0.0)) != hipSuccess)
    return LSM_EHIP;
  // Stage 2: exclusive scan into the caller's offsets.
  if (launch_scan(h->q_counts, nq, d_offsets, h->q_status, h->fault, h->stream,
                  timer(h, t2, kKScan, nq, 12.0 * nq)) != hipSuccess)
    return LSM_EHIP;
  if (hipMemcpyAsync(h->h_pinned, d_offsets + nq, sizeof(uint64_t), hipMemcpyDeviceToHost,
                     h->stream) != hipSuccess ||
      hipStreamSynchronize(h->stream) != hipSuccess)
    return LSM_EHIP;
  const uint64_t total = *reinterpret_cast<volatile uint64_t*>(h->h_pinned);
  *h_total = total;
  if (total > cap) return LSM_ECAPACITY;
  // Stage 3: each query writes its live pairs in key order at its offset.
  if (total > 0) {
    if (launch_range_emit(lv, d_lo, d_hi, nq, d_offsets, h->q_bounds, d_keys, d_vals, cap,
                          h->stream, timer(h, t3, kKRangeEmit, nq, 0.0)) != hipSuccess)
      return LSM_EHIP;
    call_span(h, kSpanRange, t1, t3, nq);
  } else {
    call_span(h, kSpanRange, t1, t2, nq);
  }
  return LSM_OK;
}

// Coalescer: packs n operations, in arrival order, into the staging batch;
// every b staged elements are inserted as one LSM batch.  is_delete[j] (or
// all_delete) makes element j a deletion.
static lsm_status_t submit(lsm_t h, const uint32_t* d_keys, const uint32_t* d_vals,
                           const uint8_t* d_is_delete, int all_delete, uint32_t n) {
  DeviceGuard g(h->device);
  if (!g.ok) return LSM_EHIP;
  if (h->flags & LSM_CHECKED) {
    // Validate the whole user batch before staging any of it.
    bool bad = false;
    const lsm_status_t s = check_keys(h, d_keys, n, &bad);
    if (s != LSM_OK) return s;
    if (bad) return LSM_EKEY;
  }
  // Every LSM batch this call fills is allocated for before anything is
  // staged, so that a failure leaves the staged elements as they were.
  const uint64_t full = (static_cast<uint64_t>(h->stage_fill) + n) / h->b;
  for (uint64_t k = 0; k < full; ++k) {
    const lsm_status_t s = prepare_insert(h, __builtin_ctzll(~(h->r + k)));
    if (s != LSM_OK) return s;
  }
  uint32_t done = 0;
  while (done < n) {
    const uint32_t take = (n - done) < (h->b - h->stage_fill) ? (n - done) : (h->b - h->stage_fill);
    if (launch_stage(d_keys + done, d_vals ? d_vals + done : nullptr,
                     d_is_delete ? d_is_delete + done : nullptr, all_delete, take, h->stage_kv,
                     h->stage_val, h->stage_fill, h->stream) != hipSuccess)
      return LSM_EHIP;
    h->stage_fill += take;
    done += take;
    if (h->stage_fill == h->b) {
      const lsm_status_t s = insert_staged(h, h->b);
      if (s != LSM_OK) return s;
    }
  }
  return LSM_OK;
}

lsm_status_t lsm_submit(lsm_t h, const uint32_t* d_keys, const uint32_t* d_vals, uint32_t n,
                        int is_delete) {
  if (h == nullptr) return LSM_EINVAL;
  if (n == 0) return LSM_OK;
  if (d_keys == nullptr || (!is_delete && d_vals == nullptr)) return LSM_EINVAL;
  return submit(h, d_keys, is_delete ? nullptr : d_vals, nullptr, is_delete ? 1 : 0, n);
}

lsm_status_t lsm_submit_mixed(lsm_t h, const uint32_t* d_keys, const uint32_t* d_vals,
                              const uint8_t* d_is_delete, uint32_t n) {
  if (h == nullptr) return LSM_EINVAL;
  if (n == 0) return LSM_OK;
  if (d_keys == nullptr || d_vals == nullptr || d_is_delete == nullptr) return LSM_EINVAL;
  return submit(h, d_keys, d_vals, d_is_delete, 0, n);
}

lsm_status_t lsm_range_async(lsm_t h, const uint32_t* d_lo, const uint32_t* d_hi, uint32_t nq,
                             uint64_t* d_offsets, uint32_t* d_keys, uint32_t* d_vals,
                             uint64_t cap) {
  if (h == nullptr || d_offsets == nullptr) return LSM_EINVAL;
  if (nq > 0 && (d_lo == nullptr || d_hi == nullptr)) return LSM_EINVAL;
  if (cap > 0 && (d_keys == nullptr || d_vals == nullptr)) return LSM_EINVAL;
  DeviceGuard g(h->device);
  if (!g.ok) return LSM_EHIP;
  if (nq == 0)
    return hipMemsetAsync(d_offsets, 0, sizeof(uint64_t), h->stream) == hipSuccess ? LSM_OK
                                                                                  : LSM_EHIP;
  lsm_status_t s = ensure_query_scratch(h, nq);
  if (s == LSM_OK) s = ensure_bounds(h, nq);
  if (s == LSM_OK) s = settle(h);
  if (s != LSM_OK) return s;
  const LevelSet lv = occupied_levels(h);
  Timed t1, t2, t3;
  if (launch_count(lv, d_lo, d_hi, nq, h->q_counts, h->q_status, scan_status_words(nq),
                   h->q_bounds, h->stream, timer(h, t1, kKCount, nq, 0.0)) != hipSuccess ||
      launch_scan(h->q_counts, nq, d_offsets, h->q_status, h->fault, h->stream,
                  timer(h, t2, kKScan, nq, 12.0 * nq)) != hipSuccess ||
      launch_range_emit(lv, d_lo, d_hi, nq, d_offsets, h->q_bounds, d_keys, d_vals, cap,
                        h->stream, timer(h, t3, kKRangeEmit, nq, 0.0)) != hipSuccess)
    return LSM_EHIP;
  return LSM_OK;
}

// lsm_range_async with the query scratch in the device's fixed array: no
// allocation of any kind.  The staged elements and the pending insertion
// are completed first, as for every query, but only when that needs no
// memory the handle does not already hold; kernel timing stays off for the
// call (it creates events).
lsm_status_t lsm_range_async_noalloc(lsm_t h, const uint32_t* d_lo, const uint32_t* d_hi,
                                     uint32_t nq, uint64_t* d_offsets, uint32_t* d_keys,
                                     uint32_t* d_vals, uint64_t cap) {
  if (h == nullptr || d_offsets == nullptr) return LSM_EINVAL;
  if (nq > 0 && (d_lo == nullptr || d_hi == nullptr)) return LSM_EINVAL;
  if (cap > 0 && (d_keys == nullptr || d_vals == nullptr)) return LSM_EINVAL;
  if (nq > kFixedMaxQueries) return LSM_ECAPACITY;
  DeviceGuard g(h->device);
  if (!g.ok) return LSM_EHIP;
  if (h->fixed.counts == nullptr) return LSM_EHIP;
  if (nq == 0) return launch_zero_u64(d_offsets, h->stream) == hipSuccess ? LSM_OK : LSM_EHIP;
  if (h->stage_fill > 0) {
    const int j = __builtin_ctzll(~h->r);
    if (j < kMaxLevels && (h->lvl_kv[j] == nullptr ||
                           (j >= 2 && h->mrg_cap < level_len(h, j - 1))))
      return LSM_ENOMEM;
  }
  const bool prof = h->prof;
  h->prof = false;
  const lsm_status_t s = settle(h);
  h->prof = prof;
  if (s != LSM_OK) return s;
  const LevelSet lv = occupied_levels(h);
  if (launch_count(lv, d_lo, d_hi, nq, h->fixed.counts, h->fixed.status, scan_status_words(nq),
                   nullptr, h->stream, nullptr) != hipSuccess ||
      launch_scan(h->fixed.counts, nq, d_offsets, h->fixed.status, h->fault, h->stream,
                  nullptr) != hipSuccess ||
      launch_range_emit(lv, d_lo, d_hi, nq, d_offsets, nullptr, d_keys, d_vals, cap, h->stream,
                        nullptr) != hipSuccess)
    return LSM_EHIP;
  return LSM_OK;
}

lsm_status_t lsm_flush(lsm_t h) {
  if (h == nullptr) return LSM_EINVAL;
  DeviceGuard g(h->device);
  if (!g.ok) return LSM_EHIP;
  return settle(h);
}

uint32_t lsm_pending(lsm_t h) { return h ? h->stage_fill : 0; }

lsm_status_t lsm_set_tuning(lsm_t h, uint32_t level, uint32_t variant) {
  if (h == nullptr || level >= static_cast<uint32_t>(kMaxLevels) ||
      variant >= static_cast<uint32_t>(kMergeVariants))
    return LSM_EINVAL;
  h->merge_variant[level] = static_cast<int>(variant);
  return LSM_OK;
}

lsm_status_t lsm_get_tuning(lsm_t h, uint32_t level, uint32_t* variant, float* us) {
  if (h == nullptr || variant == nullptr || level >= static_cast<uint32_t>(kMaxLevels))
    return LSM_EINVAL;
  *variant = static_cast<uint32_t>(h->merge_variant[level]);
  if (us != nullptr)
    for (int v = 0; v < kMergeVariants; ++v) us[v] = h->tune_us[level][v];
  return LSM_OK;
}

lsm_status_t lsm_autotune(lsm_t h, uint32_t max_level, uint32_t reps) {
  if (h == nullptr || reps == 0) return LSM_EINVAL;
  if (max_level >= static_cast<uint32_t>(kMaxLevels) || level_len(h, max_level) > (1ull << 27))
    return LSM_ECAPACITY;
  DeviceGuard g(h->device);
  if (!g.ok) return LSM_EHIP;
  const uint64_t len_max = level_len(h, max_level);
  void* buf[6] = {};
  const size_t sz[6] = {len_max * 4, len_max * 4, len_max * 4, len_max * 4, len_max * 8, len_max * 8};
  lsm_status_t s = LSM_OK;
  for (int i = 0; i < 6 && s == LSM_OK; ++i) s = dev_alloc(h, &buf[i], sz[i]);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (s == LSM_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
    s = LSM_EHIP;
  auto* ak = static_cast<uint32_t*>(buf[0]);
  auto* av = static_cast<uint32_t*>(buf[1]);
  auto* bk = static_cast<uint32_t*>(buf[2]);
  auto* bv = static_cast<uint32_t*>(buf[3]);
  auto* ok = static_cast<uint32_t*>(buf[4]);
  auto* ov = static_cast<uint32_t*>(buf[5]);
  // Merges of the sizes the cascade performs: two runs of b * 2^i each.
  for (uint32_t i = 0; i <= max_level && s == LSM_OK; ++i) {
    const uint32_t len = static_cast<uint32_t>(level_len(h, static_cast<int>(i)));
    if (launch_fill_runs(ak, av, bk, bv, len, h->stream) != hipSuccess) {
      s = LSM_EHIP;
      break;
    }
    int best = kDefaultMergeVariant;
    float best_us = 0.f;
    for (int v = 0; v < kMergeVariants && s == LSM_OK; ++v) {
      if (launch_merge(ak, av, len, bk, bv, len, ok, ov, nullptr, v, h->stream, nullptr) != hipSuccess ||
          hipEventRecord(e0, h->stream) != hipSuccess) {
        s = LSM_EHIP;
        break;
      }
      for (uint32_t k = 0; k < reps; ++k)
        if (launch_merge(ak, av, len, bk, bv, len, ok, ov, nullptr, v, h->stream, nullptr) != hipSuccess)
          s = LSM_EHIP;
      float ms = 0.f;
      if (s != LSM_OK || hipEventRecord(e1, h->stream) != hipSuccess ||
          hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        s = LSM_EHIP;
        break;
      }
      const float us = 1000.f * ms / static_cast<float>(reps);
      h->tune_us[i][v] = us;
      if (v == 0 || us < best_us) {
        best_us = us;
        best = v;
      }
    }
    if (s == LSM_OK) h->merge_variant[i] = best;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(h->stream);
  for (int i = 0; i < 6; ++i) dev_free(h, buf[i], sz[i]);
  return s;
}

lsm_status_t lsm_sync(lsm_t h) {
  if (h == nullptr) return LSM_EINVAL;
  DeviceGuard g(h->device);
  if (!g.ok) return LSM_EHIP;
  const lsm_status_t ds = drain(h);
  if (ds != LSM_OK) return ds;
  if (hipMemcpyAsync(h->h_pinned, h->fault, sizeof(uint32_t), hipMemcpyDeviceToHost, h->stream) !=
          hipSuccess ||
      hipStreamSynchronize(h->stream) != hipSuccess)
    return LSM_EHIP;
  if (*reinterpret_cast<volatile uint32_t*>(h->h_pinned) != 0u) {
    (void)hipMemsetAsync(h->fault, 0, sizeof(uint32_t), h->stream);
    (void)hipStreamSynchronize(h->stream);
    return LSM_EHIP;
  }
  return LSM_OK;
}

lsm_status_t lsm_clear(lsm_t h) {
  if (h == nullptr) return LSM_EINVAL;
  h->npend = 0;  // the half-done insertions are simply dropped
  h->r = 0;
  h->stage_fill = 0;
  h->merged_last = 0;
  return LSM_OK;
}

void lsm_struct_sizes(size_t* stats_size, size_t* profile_size) {
  if (stats_size != nullptr) *stats_size = sizeof(lsm_stats_t);
  if (profile_size != nullptr) *profile_size = sizeof(lsm_profile_t);
}

lsm_status_t lsm_profile_enable(lsm_t h, int on) {
  if (h == nullptr) return LSM_EINVAL;
  h->prof = on != 0;
  return LSM_OK;
}

lsm_status_t lsm_profile_read(lsm_t h, lsm_profile_t* out, int reset) {
  if (h == nullptr || out == nullptr) return LSM_EINVAL;
  DeviceGuard g(h->device);
  if (!g.ok || hipStreamSynchronize(h->stream) != hipSuccess) return LSM_EHIP;
  lsm_profile_t& p = h->acc;
  for (const auto& sp : h->spans) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, h->marks[sp.a], h->marks[sp.b]) != hipSuccess) continue;
    if (sp.kind < kNumKernelKinds) {
      p.launches[sp.kind] += 1;
      p.elems[sp.kind] += sp.items;
      p.kernel_ms[sp.kind] += ms;
      p.kernel_bytes[sp.kind] += sp.bytes;
      if (sp.kind == kKMerge && sp.items > 0) {
        // Size class: entry k holds outputs of 2^(k-1) + 1 .. 2^k elements.
        int k = sp.items > 1 ? 64 - __builtin_clzll(sp.items - 1) : 0;
        if (k >= LSM_PROF_SIZES) k = LSM_PROF_SIZES - 1;
        p.merge_launches_by_size[k] += 1;
        p.merge_ms_by_size[k] += ms;
        p.merge_bytes_by_size[k] += sp.bytes;
      }
    } else if (sp.kind == kSpanUpdate) {
      p.update_ms += ms;
      p.update_calls += 1;
      h->update_times.push_back(ms);
    } else {
      const int q = sp.kind - kSpanLookup;
      p.query_ms[q] += ms;
      p.query_calls[q] += 1;
      p.query_items[q] += sp.items;
    }
  }
  for (hipEvent_t e : h->marks) h->ev_pool.push_back(e);
  h->marks.clear();
  h->spans.clear();
  if (!h->update_times.empty()) {
    std::vector<double> t = h->update_times;
    std::sort(t.begin(), t.end());
    auto q = [&](double f) { return t[static_cast<size_t>(f * (t.size() - 1) + 0.5)]; };
    p.update_p50_ms = q(0.50);
    p.update_p99_ms = q(0.99);
    p.update_max_ms = t.back();
  }
  *out = p;
  if (reset) {
    h->acc = lsm_profile_t{};
    h->update_times.clear();
  }
  return LSM_OK;
}

lsm_status_t lsm_destroy(lsm_t h) {
  if (h == nullptr) return LSM_EINVAL;
  lsm_status_t s = LSM_OK;
  {
    DeviceGuard g(h->device);
    if (!g.ok || hipStreamSynchronize(h->stream) != hipSuccess) s = LSM_EHIP;
    release_events(h);
    release_all(h);
  }
  delete h;
  return s;
}

const char* lsm_strerror(lsm_status_t s) {
  switch (s) {
    case LSM_OK: return "ok";
    case LSM_EINVAL: return "invalid argument";
    case LSM_EKEY: return "key out of range";
    case LSM_EBATCH: return "batch larger than b";
    case LSM_ENOMEM: return "out of memory";
    case LSM_ECAPACITY: return "capacity exceeded";
    case LSM_EHIP: return "HIP runtime error";
  }
  return "unknown status";
}

uint64_t lsm_num_batches(lsm_t h) { return h ? h->r : 0; }

lsm_status_t lsm_fail_alloc_after(lsm_t h, int64_t n) {
  if (h == nullptr) return LSM_EINVAL;
  h->fail_after = n < 0 ? -1 : n;
  return LSM_OK;
}
uint32_t lsm_batch_size(lsm_t h) { return h ? h->b : 0; }

lsm_status_t lsm_level_view(lsm_t h, uint32_t i, const uint32_t** d_kv, const uint32_t** d_vals,
                            uint64_t* len) {
  if (h == nullptr || d_kv == nullptr || d_vals == nullptr || len == nullptr) return LSM_EINVAL;
  {
    DeviceGuard g(h->device);
    if (!g.ok) return LSM_EHIP;
    const lsm_status_t ds = drain(h);
    if (ds != LSM_OK) return ds;
  }
  if (i >= static_cast<uint32_t>(kMaxLevels) || !((h->r >> i) & 1u)) {
    *d_kv = nullptr;
    *d_vals = nullptr;
    *len = 0;
    return LSM_OK;
  }
  *d_kv = h->lvl_kv[i];
  *d_vals = h->lvl_val[i];
  *len = level_len(h, static_cast<int>(i));
  return LSM_OK;
}

lsm_status_t lsm_level_copy(lsm_t h, uint32_t i, uint32_t* d_kv_out, uint32_t* d_vals_out,
                            uint64_t* len) {
  if (h == nullptr || len == nullptr) return LSM_EINVAL;
  if (i >= static_cast<uint32_t>(kMaxLevels) || !((h->r >> i) & 1u)) {
    *len = 0;
    return LSM_OK;
  }
  if (d_kv_out == nullptr || d_vals_out == nullptr) return LSM_EINVAL;
  DeviceGuard g(h->device);
  if (!g.ok) return LSM_EHIP;
  const lsm_status_t ds = drain(h);
  if (ds != LSM_OK) return ds;
  const uint64_t n = level_len(h, static_cast<int>(i));
  *len = n;
  if (hipMemcpyAsync(d_kv_out, h->lvl_kv[i], n * sizeof(uint32_t), hipMemcpyDeviceToDevice,
                     h->stream) != hipSuccess ||
      hipMemcpyAsync(d_vals_out, h->lvl_val[i], n * sizeof(uint32_t), hipMemcpyDeviceToDevice,
                     h->stream) != hipSuccess)
    return LSM_EHIP;
  return LSM_OK;
}

lsm_status_t lsm_set_fusion(lsm_t h, int max_levels) {
  if (h == nullptr || max_levels > kMaxFuse) return LSM_EINVAL;
  h->fuse_max = max_levels < 0 ? default_fuse_max(h->b) : max_levels;
  return LSM_OK;
}

lsm_status_t lsm_set_grouping(lsm_t h, int max_batches) {
  if (h == nullptr || max_batches < 0) return LSM_EINVAL;
  int g = max_batches >= 4 ? 4 : max_batches >= 2 ? 2 : 1;
  while (g > static_cast<int>(h->grp_cap)) g /= 2;
  h->group_max = g;
  return LSM_OK;
}

lsm_status_t lsm_set_max_inflight(lsm_t h, int launches) {
  if (h == nullptr || launches < 0) return LSM_EINVAL;
  h->max_inflight = launches;
  return LSM_OK;
}

lsm_status_t lsm_set_sort_path(lsm_t h, int mode) {
  if (h == nullptr || mode < LSM_SORT_AUTO || mode > LSM_SORT_DIGIT_PASSES) return LSM_EINVAL;
  h->sort_mode = mode;
  return LSM_OK;
}

lsm_status_t lsm_get_stats(lsm_t h, lsm_stats_t* out) {
  if (h == nullptr || out == nullptr) return LSM_EINVAL;
  out->num_batches = h->r;
  out->resident_elems = h->r * h->b;
  out->merged_elems_last = h->merged_last;
  out->merged_elems_total = h->merged_total;
  out->sorted_elems_total = h->sorted_total;
  out->device_bytes = h->device_bytes;
  out->sorts_top_digit = h->sorts_by_path[kSortMsd];
  out->sorts_digit_passes = h->sorts_by_path[kSortLsd];
  return LSM_OK;
}

}  // extern "C"
