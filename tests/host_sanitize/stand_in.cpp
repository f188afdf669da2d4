// CPU stand-ins for the HIP runtime calls and the kernel launchers that the
// library's host code (csrc/lsm_api.hip) uses: test infrastructure only,
// built by tests/test_host_sanitize.py with g++ under AddressSanitizer and
// UndefinedBehaviorSanitizer.
//
// Device memory is host memory from malloc, so the sanitizer knows every
// buffer's extent.  Each stand-in launcher computes nothing of the method;
// it touches the first and the last element of every range the real kernel
// reads or writes, given the arguments the host code passed (sizes, level
// lengths, fence-tree lengths, digit indexes, per-slot scratch, bounds
// words), so that a buffer the host code sized or offset wrongly is reported
// as an out-of-bounds access.  The few results the host code reads back are
// written consistently: counts (a fixed pattern) and their exclusive scan,
// cleanup tile counts (every element valid), the pacing sequence number.
// The scratch-layout functions are the library's own, extracted from the
// kernel source at build time (layout_gen.inc), so the touched ranges
// follow the real layout.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "lsm_internal.h"

// ------------------------------------------------------------ runtime
struct ihipEvent_t {
  double t_ms = 0.0;
};

namespace {
// Per thread, like the runtime's current device; the injection counters are
// per thread too, so that threads driving their own handles stay apart.
thread_local int g_device = 0;
thread_local long g_fail_launch_after = -1;  // < 0: never; 0: the next launch fails
thread_local long g_fail_alloc_after = -1;   // the same for device and pinned allocations
thread_local long g_launches = 0;

bool alloc_fails() {
  if (g_fail_alloc_after == 0) return true;  // sticky until reset
  if (g_fail_alloc_after > 0) --g_fail_alloc_after;
  return false;
}

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}
}  // namespace

extern "C" {
// Test hook of the driver: the n-th launcher call from now on fails (n < 0:
// none), and the number of launcher calls so far.
void standin_fail_launch_after(long n) { g_fail_launch_after = n; }
// The n-th runtime allocation from now on fails and every later one too
// (n < 0: none), as when device memory runs out.
void standin_fail_alloc_after(long n) { g_fail_alloc_after = n; }
long standin_launches(void) { return g_launches; }
}

hipError_t hipGetDevice(int* dev) {
  *dev = g_device;
  return hipSuccess;
}
hipError_t hipSetDevice(int dev) {
  if (dev != 0) return hipErrorInvalidDevice;
  g_device = dev;
  return hipSuccess;
}
hipError_t hipGetLastError(void) { return hipSuccess; }
hipError_t hipMalloc(void** p, size_t bytes) {
  *p = nullptr;
  if (alloc_fails()) return hipErrorOutOfMemory;
  *p = std::calloc(1, bytes);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void* p) {
  std::free(p);
  return hipSuccess;
}
hipError_t hipHostMalloc(void** p, size_t bytes, unsigned int) {
  *p = nullptr;
  if (alloc_fails()) return hipErrorOutOfMemory;
  *p = std::calloc(1, bytes);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipHostFree(void* p) {
  std::free(p);
  return hipSuccess;
}
hipError_t hipHostGetDevicePointer(void** dev, void* host, unsigned int) {
  *dev = host;
  return hipSuccess;
}
hipError_t hipMemset(void* p, int value, size_t bytes) {
  if (bytes) std::memset(p, value, bytes);
  return hipSuccess;
}
hipError_t hipMemsetAsync(void* p, int value, size_t bytes, hipStream_t) {
  return hipMemset(p, value, bytes);
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind, hipStream_t) {
  if (bytes) std::memmove(dst, src, bytes);
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t* e) {
  *e = new ihipEvent_t();
  return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
  delete e;
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t) {
  if (e == nullptr) return hipErrorInvalidValue;
  e->t_ms = now_ms();
  return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e) { return e ? hipSuccess : hipErrorInvalidValue; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
  if (a == nullptr || b == nullptr) return hipErrorInvalidValue;
  *ms = static_cast<float>(b->t_ms - a->t_ms);
  return hipSuccess;
}

// ------------------------------------------------------------ launchers
namespace lsm {

#include "layout_gen.inc"

namespace {

[[noreturn]] void null_buffer(const char* what) {
  std::fprintf(stderr, "stand-in launcher: null buffer for %s\n", what);
  std::abort();
}

template <class T>
void rd(const T* p, uint64_t n, const char* what) {
  if (n == 0) return;
  if (p == nullptr) null_buffer(what);
  volatile T x = p[0];
  x = p[n - 1];
  (void)x;
}

template <class T>
void wr(T* p, uint64_t n, const char* what) {
  if (n == 0) return;
  if (p == nullptr) null_buffer(what);
  p[0] = T{};
  p[n - 1] = T{};
}

// One launcher call: counts it, fails it when the test asked for that, and
// brackets it with the timer's events like the real timed launch.
hipError_t begin(const KTimer* t) {
  ++g_launches;
  if (g_fail_launch_after == 0) {
    g_fail_launch_after = -1;
    return hipErrorInvalidValue;
  }
  if (g_fail_launch_after > 0) --g_fail_launch_after;
  if (t != nullptr && t->start != nullptr) (void)hipEventRecord(t->start, nullptr);
  return hipSuccess;
}
hipError_t end(const KTimer* t) {
  if (t != nullptr && t->stop != nullptr) (void)hipEventRecord(t->stop, nullptr);
  return hipSuccess;
}

void touch_levels(const LevelSet& lv) {
  if (lv.count < 0 || lv.count > kMaxLevels) null_buffer("level count out of range");
  for (int l = 0; l < lv.count; ++l) {
    rd(lv.kv[l], lv.len[l], "level kv");
    rd(lv.val[l], lv.len[l], "level val");
    rd(lv.fence[l], fence_len(lv.len[l]), "level fence");
  }
}

void touch_src(const BatchSrc& s) {
  if (s.n == 0 || s.n > s.b) null_buffer("batch size out of range");
  rd(s.keys, s.n, "batch keys");
  if (s.vals != nullptr) rd(s.vals, s.n, "batch vals");
  if (s.mode == kMixed) rd(s.is_delete, s.n, "batch delete flags");
}

// The sorted output: the fused cascade's level when levels are fused, else
// out_kv; out_kv and tmp_kv[1] also take a bucket too large for LDS.
void touch_sorted_output(const SortArgs& a) {
  wr(a.out_kv, a.out_n, "sort out kv");
  wr(a.out_val, a.out_n, "sort out val");
  if (a.out_fence != nullptr) wr(a.out_fence, fence_len(a.out_n), "sort out fence");
  if (a.out_digit != nullptr) wr(a.out_digit, kTopBuckets, "sort out digit index");
  const FuseArgs& f = a.fuse;
  if (f.nlev < 0 || f.nlev > kMaxFuse) null_buffer("fused level count out of range");
  for (int q = 0; q < f.nlev; ++q) {
    rd(f.kv[q], f.len[q], "fused level kv");
    rd(f.val[q], f.len[q], "fused level val");
    rd(f.digit[q], kTopBuckets, "fused level digit index");
  }
  if (f.nlev > 0) {
    wr(f.out_kv, f.out_len, "fused out kv");
    wr(f.out_val, f.out_len, "fused out val");
    if (f.out_fence != nullptr) wr(f.out_fence, fence_len(f.out_len), "fused out fence");
    if (f.out_digit != nullptr) wr(f.out_digit, kTopBuckets, "fused out digit index");
  }
}

void touch_scatter(const SortArgs& a) {
  touch_src(a.src);
  wr(a.tmp_kv[0], a.src.b, "scatter kv");
  wr(a.tmp_val[0], a.src.b, "scatter val");
  wr(a.meta.tile_cnt, static_cast<uint64_t>(a.meta.num_sort_tiles) * (kTopBuckets / 2),
     "scatter group starts");
  if (a.skew_out != nullptr) {
    rd(a.meta.bucket_n, kTopBuckets, "bucket-size record");
    wr(a.skew_out, 1, "skew hint");
  }
  if (a.progress != nullptr) *a.progress = a.seq;  // the host paces on it
}

void touch_buckets(const SortArgs& in) {
  SortArgs a = in;
  if (a.group == 0) {
    a.group = 1;
    a.grp_cnt[0] = a.meta.tile_cnt;
    a.grp_n[0] = a.meta.bucket_n;
    a.grp_off[0] = 0;
  }
  if (a.group > static_cast<uint32_t>(kMaxGroup)) null_buffer("group larger than kMaxGroup");
  for (uint32_t q = 0; q < a.group; ++q) {
    if (a.tmp_kv[0] == nullptr || a.tmp_val[0] == nullptr) null_buffer("bucket input");
    rd(a.tmp_kv[0] + a.grp_off[q], a.src.b, "bucket input kv");
    rd(a.tmp_val[0] + a.grp_off[q], a.src.b, "bucket input val");
    rd(a.grp_cnt[q], static_cast<uint64_t>(a.meta.num_sort_tiles) * (kTopBuckets / 2),
       "bucket group starts");
    wr(a.grp_n[q], kTopBuckets, "bucket-size record");
  }
  wr(a.tmp_kv[1], a.out_n, "streaming bucket kv");
  wr(a.tmp_val[1], a.out_n, "streaming bucket val");
  touch_sorted_output(a);
}

}  // namespace

hipError_t launch_sort(const SortArgs& a, hipStream_t, const KTimer* timers, int* launched) {
  *launched = 0;
  const int nk = sort_kernel_count(a);
  for (int k = 0; k < nk; ++k) {
    const KTimer* t = timers ? &timers[k] : nullptr;
    if (begin(t) != hipSuccess) return hipErrorInvalidValue;
    if (a.path == kSortMsd && a.meta.num_sort_tiles <= static_cast<uint32_t>(kMsdMaxTiles)) {
      if (k == 0) touch_scatter(a);
      else touch_buckets(a);
    } else if (k == 0) {
      touch_src(a.src);
      wr(a.meta.hist, 2ull * kMaxPasses * kRadix, "digit histograms");
      if (a.skew_out != nullptr) wr(a.skew_out, 1, "skew hint");
    } else {
      wr(a.meta.status, static_cast<uint64_t>(kMaxPasses) * a.meta.num_sort_tiles * kRadix,
         "look-back words");
      wr(a.meta.tile_ctr, kMaxPasses, "tile counters");
      for (int x = 0; x < 2; ++x) {
        wr(a.tmp_kv[x], a.src.b, "radix ping-pong kv");
        wr(a.tmp_val[x], a.src.b, "radix ping-pong val");
      }
      if (k == nk - 1) touch_sorted_output(a);
    }
    end(t);
    *launched = k + 1;
  }
  return hipSuccess;
}

hipError_t launch_scatter(const SortArgs& a, hipStream_t, const KTimer* t) {
  if (begin(t) != hipSuccess) return hipErrorInvalidValue;
  touch_scatter(a);
  return end(t);
}

hipError_t launch_buckets(const SortArgs& a, hipStream_t, const KTimer* t) {
  if (begin(t) != hipSuccess) return hipErrorInvalidValue;
  touch_buckets(a);
  return end(t);
}

hipError_t launch_sort_step(const SortArgs& bk, const SortArgs& sc, hipStream_t,
                            const KTimer* t) {
  if (begin(t) != hipSuccess) return hipErrorInvalidValue;
  touch_buckets(bk);
  touch_scatter(sc);
  return end(t);
}

hipError_t launch_merge(const uint32_t* a_kv, const uint32_t* a_val, uint32_t na,
                        const uint32_t* b_kv, const uint32_t* b_val, uint32_t nb,
                        uint32_t* out_kv, uint32_t* out_val, uint32_t* out_fence, int variant,
                        hipStream_t, const KTimer* t, const MergeIndex* idx) {
  if (begin(t) != hipSuccess) return hipErrorInvalidValue;
  if (variant < 0 || variant >= kMergeVariants) null_buffer("merge variant out of range");
  rd(a_kv, na, "merge a kv");
  rd(a_val, na, "merge a val");
  rd(b_kv, nb, "merge b kv");
  rd(b_val, nb, "merge b val");
  const uint64_t n = static_cast<uint64_t>(na) + nb;
  wr(out_kv, n, "merge out kv");
  wr(out_val, n, "merge out val");
  if (out_fence != nullptr) wr(out_fence, fence_len(n), "merge out fence");
  if (idx != nullptr && idx->a_dig != nullptr && idx->b_dig != nullptr) {
    rd(idx->a_dig, kTopBuckets, "merge a digit index");
    rd(idx->b_dig, kTopBuckets, "merge b digit index");
    if (idx->out_dig != nullptr) wr(idx->out_dig, kTopBuckets, "merge out digit index");
  }
  return end(t);
}

hipError_t launch_stage(const uint32_t* keys, const uint32_t* vals, const uint8_t* is_delete,
                        int all_delete, uint32_t n, uint32_t* stage_kv, uint32_t* stage_val,
                        uint32_t at, hipStream_t) {
  if (begin(nullptr) != hipSuccess) return hipErrorInvalidValue;
  rd(keys, n, "staged keys");
  if (!all_delete) rd(vals, n, "staged vals");
  if (is_delete != nullptr) rd(is_delete, n, "staged delete flags");
  if (stage_kv == nullptr || stage_val == nullptr) null_buffer("staging buffer");
  wr(stage_kv + at, n, "staging kv");
  wr(stage_val + at, n, "staging val");
  return hipSuccess;
}

hipError_t launch_check_keys(const uint32_t* keys, uint32_t n, uint32_t, int, uint32_t* err,
                             hipStream_t) {
  if (begin(nullptr) != hipSuccess) return hipErrorInvalidValue;
  rd(keys, n, "checked keys");
  rd(err, 1, "key error flag");
  return hipSuccess;
}

hipError_t launch_fill_runs(uint32_t* a_kv, uint32_t* a_val, uint32_t* b_kv, uint32_t* b_val,
                            uint32_t n, hipStream_t) {
  if (begin(nullptr) != hipSuccess) return hipErrorInvalidValue;
  wr(a_kv, n, "tuning run a kv");
  wr(a_val, n, "tuning run a val");
  wr(b_kv, n, "tuning run b kv");
  wr(b_val, n, "tuning run b val");
  return hipSuccess;
}

hipError_t launch_lookup(const LevelSet& lv, const uint32_t* q, uint32_t nq, uint32_t* out_val,
                         uint8_t* out_found, hipStream_t, const KTimer* t) {
  if (begin(t) != hipSuccess) return hipErrorInvalidValue;
  touch_levels(lv);
  rd(q, nq, "lookup keys");
  wr(out_val, nq, "lookup values");
  wr(out_found, nq, "lookup found");
  return end(t);
}

hipError_t launch_count(const LevelSet& lv, const uint32_t* lo, const uint32_t* hi, uint32_t nq,
                        uint32_t* counts, uint64_t* scan_status, size_t scan_words,
                        uint32_t* bounds, hipStream_t, const KTimer* t) {
  if (begin(t) != hipSuccess) return hipErrorInvalidValue;
  touch_levels(lv);
  rd(lo, nq, "count lo");
  rd(hi, nq, "count hi");
  if (nq > 0 && counts == nullptr) null_buffer("counts");
  for (uint32_t i = 0; i < nq; ++i) counts[i] = lv.count > 0 ? i % 3 : 0;
  if (scan_status != nullptr) wr(scan_status, scan_words, "scan look-back words");
  if (bounds != nullptr && lv.count > 0)
    wr(bounds, static_cast<uint64_t>(lv.count == 1 ? 2 : lv.count) * nq, "range bounds");
  return end(t);
}

hipError_t launch_scan(const uint32_t* counts, uint32_t nq, uint64_t* offsets,
                       uint64_t* scan_status, uint32_t* fault, hipStream_t, const KTimer* t) {
  if (begin(t) != hipSuccess) return hipErrorInvalidValue;
  rd(counts, nq, "scan counts");
  wr(scan_status, scan_status_words(nq), "scan look-back words");
  rd(fault, 1, "fault word");
  if (offsets == nullptr) null_buffer("scan offsets");
  uint64_t run = 0;
  for (uint32_t i = 0; i < nq; ++i) {
    offsets[i] = run;
    run += counts[i];
  }
  offsets[nq] = run;
  return end(t);
}

hipError_t launch_successor(const LevelSet& lv, const uint32_t* q, uint32_t nq, uint32_t* out_key,
                            uint32_t* out_val, uint8_t* out_found, hipStream_t,
                            const KTimer* t) {
  if (begin(t) != hipSuccess) return hipErrorInvalidValue;
  touch_levels(lv);
  rd(q, nq, "successor keys");
  wr(out_key, nq, "successor out keys");
  wr(out_val, nq, "successor out values");
  wr(out_found, nq, "successor found");
  return end(t);
}

hipError_t launch_predecessor(const LevelSet& lv, const uint32_t* q, uint32_t nq,
                              uint32_t* out_key, uint32_t* out_val, uint8_t* out_found,
                              hipStream_t, const KTimer* t) {
  if (begin(t) != hipSuccess) return hipErrorInvalidValue;
  touch_levels(lv);
  rd(q, nq, "predecessor keys");
  wr(out_key, nq, "predecessor out keys");
  wr(out_val, nq, "predecessor out values");
  wr(out_found, nq, "predecessor found");
  return end(t);
}

hipError_t launch_clean_count(const uint32_t* kv, uint32_t n, uint32_t* tile_cnt,
                              uint64_t* scan_status, size_t scan_words, hipStream_t,
                              const KTimer* t) {
  if (begin(t) != hipSuccess) return hipErrorInvalidValue;
  rd(kv, n, "cleanup list");
  const uint32_t tiles = clean_tiles(n);
  if (tiles > 0 && tile_cnt == nullptr) null_buffer("cleanup tile counts");
  for (uint32_t x = 0; x < tiles; ++x) {
    const uint64_t first = static_cast<uint64_t>(x) * kCleanTile;
    tile_cnt[x] = static_cast<uint32_t>(n - first < kCleanTile ? n - first : kCleanTile);
  }
  wr(scan_status, scan_words, "cleanup look-back words");
  return end(t);
}

namespace {
void touch_dst(const LevelDst& d, uint64_t lo, uint64_t hi, const char* what) {
  if (d.count < 0 || d.count > kMaxLevels) null_buffer("destination level count out of range");
  for (int l = 0; l < d.count; ++l) {
    const uint64_t a = lo > d.start[l] ? lo : d.start[l];
    const uint64_t e = hi < d.start[l] + d.len[l] ? hi : d.start[l] + d.len[l];
    if (a >= e) continue;
    if (d.kv[l] == nullptr || d.val[l] == nullptr) null_buffer(what);
    wr(d.kv[l] + (a - d.start[l]), e - a, what);
    wr(d.val[l] + (a - d.start[l]), e - a, what);
    if (d.fence[l] != nullptr) wr(d.fence[l], fence_len(d.len[l]), what);
  }
}
}  // namespace

hipError_t launch_clean_scatter(const uint32_t* kv, const uint32_t* val, uint32_t n,
                                const uint64_t* tile_off, const LevelDst& d, hipStream_t,
                                const KTimer* t) {
  if (begin(t) != hipSuccess) return hipErrorInvalidValue;
  rd(kv, n, "cleanup list kv");
  rd(val, n, "cleanup list val");
  rd(tile_off, clean_tiles(n) + 1ull, "cleanup tile offsets");
  const uint64_t v = n > 0 ? tile_off[clean_tiles(n)] : 0;
  touch_dst(d, 0, v, "cleanup destination");
  return end(t);
}

hipError_t launch_clean_pad(const LevelDst& d, uint64_t v, uint64_t total, hipStream_t,
                            const KTimer* t) {
  if (begin(t) != hipSuccess) return hipErrorInvalidValue;
  touch_dst(d, v, total, "cleanup padding");
  return end(t);
}

hipError_t launch_range_emit(const LevelSet& lv, const uint32_t* lo, const uint32_t* hi,
                             uint32_t nq, const uint64_t* offsets, const uint32_t* bounds,
                             uint32_t* out_keys, uint32_t* out_vals, uint64_t cap, hipStream_t,
                             const KTimer* t) {
  if (begin(t) != hipSuccess) return hipErrorInvalidValue;
  touch_levels(lv);
  rd(lo, nq, "range lo");
  rd(hi, nq, "range hi");
  rd(offsets, nq + 1ull, "range offsets");
  if (bounds != nullptr && lv.count > 0)
    rd(bounds, static_cast<uint64_t>(lv.count == 1 ? 2 : lv.count) * nq, "range bounds");
  const uint64_t total = nq > 0 ? offsets[nq] : 0;
  const uint64_t n = total < cap ? total : cap;
  wr(out_keys, n, "range out keys");
  wr(out_vals, n, "range out values");
  return end(t);
}

hipError_t launch_rec_max(const uint32_t* rec, uint32_t* out, hipStream_t) {
  if (begin(nullptr) != hipSuccess) return hipErrorInvalidValue;
  rd(rec, kTopBuckets, "bucket-size record");
  wr(out, 1, "skew hint");
  return hipSuccess;
}

hipError_t launch_zero_u64(uint64_t* p, hipStream_t) {
  if (begin(nullptr) != hipSuccess) return hipErrorInvalidValue;
  wr(p, 1, "zeroed word");
  return hipSuccess;
}

hipError_t fixed_scratch(FixedScratch* out) {
  // The code object's fixed array: kFixedMaxQueries counts, then the scan's
  // look-back words for that many queries (one allocation, as one array,
  // made once for the process).
  static uint64_t* const base = static_cast<uint64_t*>(
      std::calloc(kFixedMaxQueries / 2 + scan_status_words(kFixedMaxQueries), sizeof(uint64_t)));
  if (base == nullptr) return hipErrorOutOfMemory;
  out->counts = reinterpret_cast<uint32_t*>(base);
  out->status = base + kFixedMaxQueries / 2;
  return hipSuccess;
}

}  // namespace lsm
