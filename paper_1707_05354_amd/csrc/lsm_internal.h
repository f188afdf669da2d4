// Internal interface between the C-ABI host code (lsm_api.hip) and the
// gfx950 kernels (lsm_kernels.hip).  Not installed; not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lsm {

constexpr int kMaxLevels = 32;

// Work-group shape shared by every kernel: four wave64 waves.
constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

// Radix sort: 8-bit digits, tiles of kThreads * kSortItems elements.
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kSortItems = 8;
constexpr int kSortTile = kThreads * kSortItems;
constexpr int kMaxPasses = 4;
// The histogram kernel uses at most this many work-groups (tile-strided).
constexpr int kMaxHistBlocks = 512;
// Batches of at most kMsdMaxTiles tiles use the two-kernel top-digit sort:
// each tile grouped in place by its top kTopBits bits, then one work-group
// per top-digit bucket gathers its group from every tile.  Buckets (and
// fused runs) of up to kLocalCap elements are sorted and merged in LDS.
constexpr int kMsdMaxTiles = 256;
constexpr int kTopBits = 10;
constexpr uint32_t kTopBuckets = 1u << kTopBits;
constexpr int kTopPer = static_cast<int>(kTopBuckets) / kThreads;  // buckets per thread
// kLocalCap keeps the bucket kernel's LDS below 32 KiB, so that five of its
// work-groups fit one CU: the pipelined step (1024 bucket work-groups beside
// the next batch's tile scatter) then runs in a single round of work-groups.
constexpr int kLocalCap = 1536;
static_assert(kLocalCap % 256 == 0, "the bucket load phase takes kLocalCap / 256 items per thread");
// Buckets of at most this many elements are sorted by ranking (every
// element counts the elements that precede it) instead of radix passes.
constexpr uint32_t kRankSortMax = 256;

// Merge variants (autotuned per level): items per thread x work-group cap.
// Variant v uses kMergeItemsOf[v % 3] items per thread (tiles of 256 x that)
// and at most kMergeBlocksOf[v / 3] work-groups, each taking a contiguous
// run of tiles.
constexpr int kMergeVariants = 6;
constexpr int kMergeItemsOf[3] = {4, 8, 16};
constexpr int kMergeBlocksOf[2] = {1024, 4096};
constexpr int kDefaultMergeVariant = 1;  // 8 items, 1024 work-groups

// Scan (range offsets): tiles of kThreads * kScanItems counts.
constexpr int kScanItems = 8;
constexpr int kScanTile = kThreads * kScanItems;

// Query kernels: one thread per query.
constexpr int kQueryThreads = 256;

// Every level keeps a fence tree, written by the kernel that writes the
// level: tree level t = 1, 2, ... holds the original key of every 32^t-th
// element (level 1: the first key of each 128-byte line of key variables).
// Level t has ceil(n / 32^t) entries, padded to whole 128-byte lines, and
// the levels are stored one after another up to the first with at most 32
// entries (the root).  A search reads one line per tree level, top down,
// then one line of key variables.
constexpr int kFenceStride = 32;
__host__ __device__ inline uint64_t fence_pad(uint64_t c) { return (c + 31) & ~uint64_t(31); }
inline uint64_t fence_len(uint64_t n) {
  uint64_t total = 0, c = (n + 31) / 32;
  for (;;) {
    total += fence_pad(c);
    if (c <= 32) break;
    c = (c + 31) / 32;
  }
  return total;
}

// Placebo element of cleanup (sec. IV-D footnote): a tombstone of the largest
// encodable key, 2^31 - 1.  It sorts after every other element and hides
// nothing: a live element of that key precedes it in the same level.
constexpr uint32_t kPlaceboKv = 0xFFFFFFFEu;

// The occupied levels, newest (smallest) first, passed by value.
struct LevelSet {
  const uint32_t* kv[kMaxLevels];
  const uint32_t* val[kMaxLevels];
  const uint32_t* fence[kMaxLevels];
  uint32_t len[kMaxLevels];
  int count;
};

// How the batch's status bit is formed while the batch is read.  kEncoded
// batches (the coalescer's staging buffer) already hold key variables.
enum BatchMode : int { kInsert = 0, kDelete = 1, kMixed = 2, kEncoded = 3 };

// Source of one batch as the caller handed it over.
struct BatchSrc {
  const uint32_t* keys;
  const uint32_t* vals;       // null for deletions
  const uint8_t* is_delete;   // mixed batches only
  uint32_t n;                 // 1 <= n <= b
  uint32_t b;
  int mode;                   // BatchMode
};

// Sort scratch layout (uint32 words) for a batch of b elements.  The global
// digit histogram of the digit-pass sort is double-buffered: a sort
// accumulates into hist[parity] and clears hist[parity ^ 1] for the next one
// (both start zeroed).  The top-digit sort has kMaxGroup + 1 slots, so that
// one batch can be scattered while the buckets of up to kMaxGroup earlier
// batches (a group sorted together) are sorted: each slot holds a scattered
// batch, the tiles' digit-group starts and the slot's largest-bucket record.
constexpr int kMaxGroup = 4;
constexpr int kSortSlots = kMaxGroup + 1;
struct SortMeta {
  uint32_t* hist;         // [2][kMaxPasses][256]
  uint32_t* status;       // [kMaxPasses][num_sort_tiles][256] look-back words
  uint32_t* tile_ctr;     // [kMaxPasses] dynamic tile ids of each pass
  uint32_t* err;          // [0] key-range violation (checked mode),
                          // [1] sticky device fault (a bounded wait expired)
  uint32_t* tile_cnt;     // this slot's [num_sort_tiles][kTopBuckets / 2] digit-group
                          // starts (top-digit sort; two 16-bit starts per word)
  uint32_t* bucket_n;     // this slot's [kTopBuckets] record: each top-digit bucket's size
                          // (its share per batch for a group) in the slot's last bucket
                          // sort (top-digit sort)
  uint32_t num_sort_tiles;
  int parity;
};
// The two sort paths: one scatter on the top digit then a per-bucket LDS
// sort (for at most kMsdMaxTiles tiles), or one digit pass per 8 bits.  The
// first is faster unless a top-digit bucket outgrows kLocalCap (skewed keys),
// which its fallback handles with a single work-group; each sort records its
// largest top-digit bucket so that the next sort can pick the path.
enum SortPath : int { kSortMsd = 0, kSortLsd = 1 };
inline int pick_sort_path(uint32_t tiles, uint32_t last_max_bucket) {
  return (tiles <= static_cast<uint32_t>(kMsdMaxTiles) &&
          last_max_bucket <= static_cast<uint32_t>(kLocalCap))
             ? kSortMsd
             : kSortLsd;
}

// A small cascade fused into the top-digit sort: the work-group of bucket d
// merges the batch's bucket with the same key range of levels 0..nlev-1
// (bucket d holds the original keys [d << key_shift, (d + 1) << key_shift))
// and writes that part of level nlev.  nlev = 0: no fusion.
constexpr int kMaxFuse = 8;
struct FuseArgs {
  int nlev;
  int key_shift;
  const uint32_t* kv[kMaxFuse];
  const uint32_t* val[kMaxFuse];
  const uint32_t* digit[kMaxFuse];  // each level's top-digit index
  uint32_t len[kMaxFuse];
  uint32_t* out_kv;
  uint32_t* out_val;
  uint32_t* out_fence;
  uint32_t* out_digit;              // the output level's index, or null
  uint64_t out_len;
};

struct SortArgs {
  BatchSrc src;
  int lo_bit;               // lowest key-variable bit sorted
  int passes;               // 8-bit digit passes
  uint32_t key_limit_bits;  // keys are < 2^key_limit_bits
  SortMeta meta;
  uint32_t* tmp_kv[2];      // radix ping-pong, b elements each
  uint32_t* tmp_val[2];
  uint32_t* out_kv;         // sorted batch
  uint32_t* out_val;
  uint32_t* out_fence;      // fences of the output when it is a level, else null
  uint32_t* out_digit;      // top-digit index of the output level (top-digit path), or null
  uint32_t out_n;           // elements of the sorted output (b; 2b for a pair)
  // Bucket half of the top-digit sort: tmp_kv[0] / tmp_val[0] hold every
  // slot's scattered batch.  `group` batches (1, 2 or 4) are sorted
  // together, the newer first on equal keys; batch q of the group (q = 0 the
  // newest) has its digit-group starts at grp_cnt[q], its bucket-size record
  // at grp_n[q] and its scattered elements from element grp_off[q].
  uint32_t group;
  const uint32_t* grp_cnt[kMaxGroup];
  uint32_t* grp_n[kMaxGroup];
  uint32_t grp_off[kMaxGroup];
  int path;                 // SortPath; both paths give the same order
  uint32_t* skew_out;       // optional: receives the largest top-digit bucket of an
                            // earlier sort (a hint for the choice of the next sorts)
  uint64_t* progress;       // optional (top-digit scatter): receives seq when the
  uint64_t seq;             // launch starts, for the host's launch pacing
  FuseArgs fuse;            // top-digit path only
};

// Bit position of the top digit the top-digit sort scatters on: the highest
// kTopBits bits a key variable can have (keys below 2^key_limit_bits give key
// variables of key_limit_bits + 1 bits), so that every bucket is used.
inline int sort_top_shift(const SortArgs& a) {
  int hi_bit = a.lo_bit + kRadixBits * a.passes;
  const int kv_bits = static_cast<int>(a.key_limit_bits) + 1;
  if (hi_bit > kv_bits) hi_bit = kv_bits;
  return hi_bit - kTopBits > a.lo_bit ? hi_bit - kTopBits : a.lo_bit;
}

// Optional per-launch timing: when start is non-null the kernel is launched
// with hipExtLaunchKernelGGL so the two events bracket the kernel itself.
struct KTimer {
  hipEvent_t start = nullptr;
  hipEvent_t stop = nullptr;
};

// Kernel kinds of the profile (indices of lsm_profile_t's per-kernel arrays).
enum KernelKind : int {
  kKSortHist = 0, kKSortPass = 1, kKMerge = 2, kKLookup = 3, kKCount = 4, kKScan = 5,
  kKRangeEmit = 6, kKOrder = 7, kKClean = 8, kKMsdHist = 9, kKMsdScatter = 10,
  kKLocalSort = 11, kKSortStep = 12, kNumKernelKinds = 13
};
// Profiler kind and algorithmic bytes per element of the x-th kernel a sort
// launches (launch_sort's order).
inline int sort_kernel_kind(int path, int x) {
  if (path == kSortMsd) return x == 0 ? kKMsdScatter : kKLocalSort;
  return x == 0 ? kKSortHist : kKSortPass;
}
inline double sort_kernel_bytes_per_elem(int path, int x) {
  return (path == kSortLsd && x == 0) ? 4.0 : 16.0;
}

// Destination of cleanup's redistribution: the occupied levels of the new
// batch count, smallest first; level l receives the list positions
// [start[l], start[l] + length of level l).
struct LevelDst {
  uint32_t* kv[kMaxLevels];
  uint32_t* val[kMaxLevels];
  uint32_t* fence[kMaxLevels];
  uint64_t start[kMaxLevels];
  uint64_t len[kMaxLevels];
  int count;
};

size_t sort_meta_words(uint32_t b);
SortMeta sort_meta_carve(uint32_t* base, uint32_t b, int parity, int slot);

// Sorts one batch into (out_kv, out_val): key variables ascending over bits
// [lo_bit, lo_bit + 8 * passes), equal key variables with the later batch
// position first.  timers (optional) holds sort_kernel_count(a) entries,
// one per kernel launched.  *launched receives the number of kernels that
// were launched (all of them unless an error is returned).
hipError_t launch_sort(const SortArgs& a, hipStream_t stream, const KTimer* timers,
                       int* launched);

// The two halves of the top-digit sort, for batches of at most kMsdMaxTiles
// tiles: the tile scatter (into meta's slot and tmp_kv[0] / tmp_val[0]) and
// the per-bucket sort with its fused cascade (from the same).
hipError_t launch_scatter(const SortArgs& a, hipStream_t stream, const KTimer* t);
hipError_t launch_buckets(const SortArgs& a, hipStream_t stream, const KTimer* t);
// Both halves in one launch, for two batches in different slots: the bucket
// sort of bk and the tile scatter of sc (the pipelined insertion).
hipError_t launch_sort_step(const SortArgs& bk, const SortArgs& sc, hipStream_t stream,
                            const KTimer* t);
// Number of kernels launch_sort issues (and timers it uses) for a.
int sort_kernel_count(const SortArgs& a);

// Top-digit indexes of a merge's two runs (both needed) and its output:
// with both, the output's index is written (when out_dig is set) and, when
// by_digit is set, the work-groups partition the output by digit ranges
// instead of searching for merge-path splits.
struct MergeIndex {
  const uint32_t* a_dig;
  const uint32_t* b_dig;
  uint32_t* out_dig;
  int by_digit;
};

// Stable merge of a newer run (first on equal original keys) with an older
// run into out (na + nb elements), with merge variant `variant`; idx is
// optional.
hipError_t launch_merge(const uint32_t* a_kv, const uint32_t* a_val, uint32_t na,
                        const uint32_t* b_kv, const uint32_t* b_val, uint32_t nb,
                        uint32_t* out_kv, uint32_t* out_val, uint32_t* out_fence, int variant,
                        hipStream_t stream, const KTimer* t, const MergeIndex* idx = nullptr);

// Coalescer: encodes n operations as key variables (status 0 for a
// deletion, value 0) into staging[at .. at + n).  Element i deletes when
// all_delete is set or is_delete[i] != 0 (is_delete may be null).
hipError_t launch_stage(const uint32_t* keys, const uint32_t* vals, const uint8_t* is_delete,
                        int all_delete, uint32_t n, uint32_t* stage_kv, uint32_t* stage_val,
                        uint32_t at, hipStream_t stream);

// Sets err |= 1 when any of n keys (key variables when encoded) is
// >= 2^limit_bits.
hipError_t launch_check_keys(const uint32_t* keys, uint32_t n, uint32_t limit_bits, int encoded,
                             uint32_t* err, hipStream_t stream);

// Fills two interleaved sorted runs (keys 2i and 2i + 1) for the autotuner.
hipError_t launch_fill_runs(uint32_t* a_kv, uint32_t* a_val, uint32_t* b_kv, uint32_t* b_val,
                            uint32_t n, hipStream_t stream);

hipError_t launch_lookup(const LevelSet& lv, const uint32_t* q, uint32_t nq, uint32_t* out_val,
                         uint8_t* out_found, hipStream_t stream, const KTimer* t);

// Count pass: per query number of live keys in [lo, hi].  When scan_status
// is non-null the kernel also clears the scan's look-back words
// (scan_words of them, tile counter included) for the following scan.  With
// bounds non-null, each query's position in the levels is stored there for
// the emission pass: with one occupied level its candidate bounds (2 nq
// words, two per query), with several its lower bound in every level
// (lv.count * nq words, level-major).
hipError_t launch_count(const LevelSet& lv, const uint32_t* lo, const uint32_t* hi, uint32_t nq,
                        uint32_t* counts, uint64_t* scan_status, size_t scan_words,
                        uint32_t* bounds, hipStream_t stream, const KTimer* t);

// Exclusive scan of nq uint32 counts into nq + 1 uint64 offsets.
size_t scan_status_words(uint32_t nq);
hipError_t launch_scan(const uint32_t* counts, uint32_t nq, uint64_t* offsets,
                       uint64_t* scan_status, uint32_t* fault, hipStream_t stream,
                       const KTimer* t);

// Order queries: per query the live pair with the smallest key > q
// (successor) or the largest key < q (predecessor); found = 0 leaves key and
// value 0.
hipError_t launch_successor(const LevelSet& lv, const uint32_t* q, uint32_t nq, uint32_t* out_key,
                            uint32_t* out_val, uint8_t* out_found, hipStream_t stream,
                            const KTimer* t);
hipError_t launch_predecessor(const LevelSet& lv, const uint32_t* q, uint32_t nq,
                              uint32_t* out_key, uint32_t* out_val, uint8_t* out_found,
                              hipStream_t stream, const KTimer* t);

// Cleanup over the merged list (kv, val) of n elements: per-tile counts of
// valid elements (first of their key run and regular; also clears the scan's
// look-back words), then the scatter of valid elements to their level
// positions given the tiles' exclusive offsets, then the placebo padding of
// positions [v, total).
uint32_t clean_tiles(uint32_t n);
hipError_t launch_clean_count(const uint32_t* kv, uint32_t n, uint32_t* tile_cnt,
                              uint64_t* scan_status, size_t scan_words, hipStream_t stream,
                              const KTimer* t);
hipError_t launch_clean_scatter(const uint32_t* kv, const uint32_t* val, uint32_t n,
                                const uint64_t* tile_off, const LevelDst& d, hipStream_t stream,
                                const KTimer* t);
hipError_t launch_clean_pad(const LevelDst& d, uint64_t v, uint64_t total, hipStream_t stream,
                            const KTimer* t);

// Range emission pass: writes each query's live pairs at offsets[q], for
// the queries whose pairs end at or before cap.  bounds: what the count pass
// stored, or null to search again.
hipError_t launch_range_emit(const LevelSet& lv, const uint32_t* lo, const uint32_t* hi,
                             uint32_t nq, const uint64_t* offsets, const uint32_t* bounds,
                             uint32_t* out_keys, uint32_t* out_vals, uint64_t cap,
                             hipStream_t stream, const KTimer* t);

// The largest entry of a slot's bucket-size record (kTopBuckets words) into
// *out, with one work-group.
hipError_t launch_rec_max(const uint32_t* rec, uint32_t* out, hipStream_t stream);

// Writes *p = 0 with a one-thread kernel (no memset node on the stream).
hipError_t launch_zero_u64(uint64_t* p, hipStream_t stream);

// Query scratch that lives in the code object instead of an allocation: the
// per-query counts and the scan's look-back words of a range query batch of
// up to kFixedMaxQueries queries.  Each device holds one copy for the life
// of the process, shared by every handle on it.
constexpr uint32_t kFixedMaxQueries = 1u << 20;
struct FixedScratch {
  uint32_t* counts;   // kFixedMaxQueries words
  uint64_t* status;   // scan_status_words(kFixedMaxQueries) words
};
// The device address of the current device's copy (looked up once per
// device; the device must be current).  Returns the lookup's error, if any.
hipError_t fixed_scratch(FixedScratch* out);

}  // namespace lsm
