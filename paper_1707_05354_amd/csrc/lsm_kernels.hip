// gfx950 kernels of the batched LSM dictionary.
//
// Every kernel runs in work-groups of four wave64 waves.  Nothing here is a
// dense contraction, so there is no MFMA: the batch sort and the level
// merges are HBM/L2 streams, the searches are random-access.
//
//   k_sort_hist / k_sort_pass : stable LSD radix sort of one batch (the
//       "sort the batch" step of sec. III-B / Fig. 2(a)): one histogram
//       kernel, then one counting pass per 8-bit digit with decoupled
//       look-back.  The batch is read back to front, so among equal key
//       variables the later batch position comes first (the last duplicate
//       wins), and padded with copies of its last element (sec. IV-A).
//   k_msd_scatter / k_local_sort : the same stable order for batches of at
//       most 256 tiles: each tile grouped by its top digit in place, then one
//       work-group gathers and sorts each top-digit bucket in LDS.
//   Every kernel that writes a level also writes its fences (the original
//       key of every 32nd element), which the searches use first.
//   k_merge : merge of a newer run with an older run on the original key,
//       the newer element first on equal keys (sec. IV-A), merge-path
//       partitioned with a 64-ary wave search.
//   k_lookup : per-query lower bound over the occupied levels, newest first,
//       stopping at the first hit (sec. III-D, IV-B).
//   k_count / k_range_emit : per-query bounds in every occupied level and a
//       merge of the per-level candidate runs in level order, keeping the
//       first element of each key run when it is a regular element
//       (sec. III-E, IV-C, IV-D).  k_range_emit_one : the emission with one
//       occupied level, a wave copying one query's candidates at a time.
//   k_scan : single-pass exclusive scan with decoupled look-back for the
//       range output offsets (stage 2 of sec. IV-C).
//   k_successor / k_predecessor : the order queries of the sec. I-B
//       footnote, the same walk as count stopped at the first live key.
//   k_clean_count / k_clean_scatter / k_clean_pad : cleanup (sec. III-E,
//       IV-D) after the levels are merged: mark stale elements, compact the
//       valid ones straight into the new levels, pad with placebos.
#include <hip/hip_ext.h>

#include "lsm_internal.h"

#include <mutex>
#include <type_traits>

namespace lsm {
namespace {

// ------------------------------------------------------------ wave helpers
__device__ __forceinline__ uint32_t lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}
// Number of set bits of m below this lane.
__device__ __forceinline__ uint32_t count_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32),
                                   __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0u));
}
__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Inclusive scan over the wave (every lane active).  Within each row of 16
// lanes, four DPP row shifts by 1, 2, 4 and 8 (lanes shifted in from outside
// the row read 0); then each row adds the totals of the rows below it, read
// from lanes 15, 31 and 47.
template <int kCtrl>
__device__ __forceinline__ uint32_t dpp_row_shr(uint32_t x) {
  return static_cast<uint32_t>(
      __builtin_amdgcn_update_dpp(0, static_cast<int>(x), kCtrl, 0xf, 0xf, true));
}
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x, uint32_t lane) {
  x += dpp_row_shr<0x111>(x);  // row_shr:1
  x += dpp_row_shr<0x112>(x);  // row_shr:2
  x += dpp_row_shr<0x114>(x);  // row_shr:4
  x += dpp_row_shr<0x118>(x);  // row_shr:8
  const uint32_t r0 = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(x), 15));
  const uint32_t r1 = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(x), 31));
  const uint32_t r2 = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(x), 47));
  const uint32_t row = lane >> 4;
  return x + (row > 0 ? r0 : 0u) + (row > 1 ? r1 : 0u) + (row > 2 ? r2 : 0u);
}
__device__ __forceinline__ uint64_t wave_incl_scan64(uint64_t x, uint32_t lane) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint64_t y = __shfl_up(x, o, 64);
    if (lane >= static_cast<uint32_t>(o)) x += y;
  }
  return x;
}
__device__ __forceinline__ uint64_t wave_sum64(uint64_t x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// Exclusive scan over the work-group, one value per thread.  tmp holds
// kWaves words; the call contains two barriers.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t* tmp) {
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t inc = wave_incl_scan(x, lane);
  if (lane == 63) tmp[wave] = inc;
  __syncthreads();
  uint32_t pre = 0;
  for (uint32_t w = 0; w < wave; ++w) pre += tmp[w];
  __syncthreads();
  return pre + inc - x;
}

// Two exclusive scans over the work-group in one pass (the barriers of one).
// tmp holds 2 kWaves words.
__device__ __forceinline__ void block_excl_scan2(uint32_t& x, uint32_t& y, uint32_t* tmp) {
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t ix = wave_incl_scan(x, lane), iy = wave_incl_scan(y, lane);
  if (lane == 63) {
    tmp[wave] = ix;
    tmp[kWaves + wave] = iy;
  }
  __syncthreads();
  uint32_t px = 0, py = 0;
  for (uint32_t w = 0; w < wave; ++w) {
    px += tmp[w];
    py += tmp[kWaves + w];
  }
  __syncthreads();
  x = px + ix - x;
  y = py + iy - y;
}

// Writes the largest of the work-group's 256 per-thread values to *out
// (thread 0).  tmp holds kWaves words; two barriers, so the whole
// work-group must call it.
__device__ void record_max(uint32_t x, uint32_t* out, uint32_t* tmp) {
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = max(x, static_cast<uint32_t>(__shfl_xor(x, o, 64)));
  if (lane == 0) tmp[wave] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t r = tmp[0];
    for (int w = 1; w < kWaves; ++w) r = max(r, tmp[w]);
    *out = r;
  }
  __syncthreads();
}

// Device-scope relaxed atomics for the look-back words: each word carries
// its own payload, so no other memory needs ordering with it.
__device__ __forceinline__ uint32_t ld_dev(const uint32_t* p) {
  return __hip_atomic_load(const_cast<uint32_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_dev64(const uint64_t* p) {
  return __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev64(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// A pointer known to address global memory (loads through it are global,
// not flat, loads).
__device__ __forceinline__ const __attribute__((address_space(1))) uint32_t* as_global(
    const uint32_t* p) {
  return (const __attribute__((address_space(1))) uint32_t*)(p);
}


// ------------------------------------------------------------ searches
// Number of entries line[i], lo <= i < hi, that are < k (upper: <= k); the
// 128-byte line at `line` is read whole (eight 16-byte loads in flight).
// kv: the entries are key variables, compared by their original key.
__device__ __forceinline__ uint32_t line_count(const uint32_t* line, uint32_t lo, uint32_t hi,
                                               uint32_t k, bool upper, bool kv) {
  const uint4* p = reinterpret_cast<const uint4*>(line);
  uint4 v[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) v[q] = p[q];
  uint32_t c = 0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const uint32_t e[4] = {v[q].x, v[q].y, v[q].z, v[q].w};
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const uint32_t i = 4u * q + r;
      const uint32_t x = kv ? (e[r] >> 1) : e[r];
      c += (i >= lo && i < hi && (upper ? x <= k : x < k)) ? 1u : 0u;
    }
  }
  return c;
}

// Lower / upper bound of original key k in a level of n elements through its
// fence tree: the first index whose original key is >= k (upper: > k), or n.
// At every tree level, g counts the entries that qualify (< k, or <= k);
// the next level down then holds the answer among entries
// 32 (g - 1) + 1 .. 32 g - 1 (entry 32 (g - 1) qualifies by its parent,
// entry 32 g fails by its parent), all in one 128-byte line.
__device__ __forceinline__ uint32_t fenced_bound(const uint32_t* kv, const uint32_t* tree,
                                                 uint32_t n, uint32_t k, bool upper) {
  if (n == 0) return 0;
  // Offset and size of the root level.
  uint64_t off = 0, c = (static_cast<uint64_t>(n) + 31) / 32;
  int t = 1;
  while (c > 32) {
    off += fence_pad(c);
    c = (c + 31) / 32;
    ++t;
  }
  uint32_t g = line_count(tree + off, 0, static_cast<uint32_t>(c), k, upper, false);
  for (--t; t >= 1; --t) {
    if (g == 0) return 0;
    const uint64_t ct = (static_cast<uint64_t>(n) + (1ull << (5 * t)) - 1) >> (5 * t);
    off -= fence_pad(ct);
    const uint32_t base = (g - 1) * 32u;
    const uint32_t end = (base + 32u < ct) ? base + 32u : static_cast<uint32_t>(ct);
    g = base + line_count(tree + off + base, 1, end - base, k, upper, false) + 1u;
  }
  if (g == 0) return 0;
  const uint32_t base = (g - 1) * 32u;
  if (base + 32u <= n) return base + line_count(kv + base, 1, 32, k, upper, true) + 1u;
  // The last, partial line of the level: read only what exists.
  uint32_t r = base + 1u;
  for (uint32_t i = base + 1u; i < n; ++i) {
    const uint32_t x = kv[i] >> 1;
    r += (upper ? x <= k : x < k) ? 1u : 0u;
  }
  return r;
}

// Sum over the eight lanes of an octet (lanes 8o .. 8o + 7), in every lane
// of it: DPP swaps with lane ^ 1 and lane ^ 2, then the half-row mirror
// (lane i with lane 7 - i inside each group of eight).  Every lane of the
// octet must be active.
__device__ __forceinline__ uint32_t octet_sum(uint32_t x) {
  x += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0xB1, 0xf, 0xf, true));
  x += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x4E, 0xf, 0xf, true));
  x += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x141, 0xf, 0xf, true));
  return x;
}

// fenced_bound for a whole wave at once, the eight lanes of an octet
// searching the octet's eight queries together: at every tree level lane s
// of the octet reads bytes 16 s .. 16 s + 15 of each of the eight queries'
// 128-byte lines, so a load instruction of the wave reads eight whole lines
// instead of 64 scattered 16-byte pieces of 64 lines (the per-lane search
// keeps the texture addresser busy nearly all the time).  Entry counts are
// summed over the octet.  Each lane passes its own key and receives its own
// bound; every lane of the wave must call it (lanes without a query pass
// any key and ignore the result).
template <bool kUpper>
__device__ __forceinline__ uint32_t octet_bound(const uint32_t* kv, const uint32_t* tree,
                                                uint32_t n, uint32_t k) {
  const uint32_t lane = lane_id(), sub = lane & 7u, ob = lane & ~7u;
  uint32_t kq[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) kq[j] = __shfl(k, static_cast<int>(ob) + j, 64);
  if (n == 0) return 0u;
  auto qual = [](uint32_t x, uint32_t key) { return kUpper ? x <= key : x < key; };
  uint64_t off = 0, c = (static_cast<uint64_t>(n) + 31) / 32;
  int t = 1;
  while (c > 32) {
    off += fence_pad(c);
    c = (c + 31) / 32;
    ++t;
  }
  uint32_t g[8];
  {
    // The root line, the same for every query.
    const uint4 w = *reinterpret_cast<const uint4*>(tree + off + 4u * sub);
    const uint32_t e4[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      uint32_t cnt = 0;
#pragma unroll
      for (int r = 0; r < 4; ++r) cnt += (4u * sub + r < c && qual(e4[r], kq[j])) ? 1u : 0u;
      g[j] = octet_sum(cnt);
    }
  }
  for (--t; t >= 1; --t) {
    const uint64_t ct = (static_cast<uint64_t>(n) + (1ull << (5 * t)) - 1) >> (5 * t);
    off -= fence_pad(ct);
    uint4 w[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const uint32_t base = g[j] > 0 ? (g[j] - 1) * 32u : 0u;
      w[j] = *reinterpret_cast<const uint4*>(tree + off + base + 4u * sub);
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const uint32_t base = g[j] > 0 ? (g[j] - 1) * 32u : 0u;
      const uint32_t lim = (base + 32u < ct) ? 32u : static_cast<uint32_t>(ct - base);
      const uint32_t e4[4] = {w[j].x, w[j].y, w[j].z, w[j].w};
      uint32_t cnt = 0;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const uint32_t i = 4u * sub + r;
        cnt += (i >= 1u && i < lim && qual(e4[r], kq[j])) ? 1u : 0u;
      }
      const uint32_t sum = octet_sum(cnt);
      g[j] = g[j] > 0 ? base + sum + 1u : 0u;
    }
  }
  // The level's own line (the last one may be partial: read what exists).
  uint4 w[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const uint32_t i0 = (g[j] > 0 ? (g[j] - 1) * 32u : 0u) + 4u * sub;
    if (i0 + 4u <= n) {
      w[j] = *reinterpret_cast<const uint4*>(kv + i0);
    } else {
      w[j].x = i0 < n ? kv[i0] : 0u;
      w[j].y = i0 + 1u < n ? kv[i0 + 1u] : 0u;
      w[j].z = i0 + 2u < n ? kv[i0 + 2u] : 0u;
      w[j].w = 0u;
    }
  }
  uint32_t res = 0;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const uint32_t base = g[j] > 0 ? (g[j] - 1) * 32u : 0u;
    const uint32_t lim = (base + 32u <= n) ? 32u : n - base;
    const uint32_t e4[4] = {w[j].x, w[j].y, w[j].z, w[j].w};
    uint32_t cnt = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const uint32_t i = 4u * sub + r;
      cnt += (i >= 1u && i < lim && qual(e4[r] >> 1, kq[j])) ? 1u : 0u;
    }
    const uint32_t sum = octet_sum(cnt);
    const uint32_t b = g[j] > 0 ? base + sum + 1u : 0u;
    res = (sub == static_cast<uint32_t>(j)) ? b : res;
  }
  return res;
}

// Records output position o of a level of n elements in the level's fence
// tree: in tree level t when o is a multiple of 32^t.
__device__ __forceinline__ void put_fence(uint32_t* tree, uint64_t n, uint64_t o, uint32_t kv) {
  if (tree == nullptr || (o & 31u) != 0) return;
  const uint32_t key = kv >> 1;
  uint64_t off = 0, c = (n + 31) / 32, q = o >> 5;
  for (;;) {
    tree[off + q] = key;
    if (c <= 32 || (q & 31u) != 0) break;
    off += fence_pad(c);
    c = (c + 31) / 32;
    q >>= 5;
  }
}

// ------------------------------------------------------------ radix sort
constexpr uint32_t kFlagAgg = 1u << 30;  // tile aggregate published
constexpr uint32_t kFlagInc = 2u << 30;  // inclusive prefix published
constexpr uint32_t kCountMask = (1u << 30) - 1;

// Every device-side wait is bounded: after kSpinLimit polls the waiter
// records kFaultTimeout in the fault word and stops waiting; writes whose
// position could then be wrong are skipped, so a broken protocol can give
// wrong results (reported by lsm_sync) but never hangs or writes out of
// bounds.  A correct run never reaches the limit: every tile a look-back
// waits for has already started.
constexpr uint32_t kSpinLimit = 1u << 24;
constexpr uint32_t kFaultTimeout = 2u;

// One thread's kN items of the tile starting at tb (positions tile_pos).
// Element e of the batch as the sort sees it: read back to front and padded
// with copies of the caller's last element, so e = 0 .. b-n-1 are padding and
// e = b-n .. b-1 are the caller's elements n-1 .. 0.  Written so that the
// tile's loads are all in flight together.  Every load is issued unconditionally (the source index is
// clamped, so each address is in bounds; deletions read their values from the
// keys and drop them), only a mixed batch's flags sit behind a branch (on the
// batch mode, uniform), and the key variables are formed afterwards.  Items
// at or past b are invalid and read as 0.
template <int kN>
__device__ __forceinline__ void tile_items(const BatchSrc& s, uint32_t tb, uint32_t wave,
                                           uint32_t lane, uint32_t (&kv)[kN], uint32_t (&val)[kN],
                                           uint32_t (&key)[kN], bool (&valid)[kN]) {
  const uint32_t* vp = s.vals != nullptr ? s.vals : s.keys;
  uint32_t src[kN], rk[kN], rv[kN], st[kN];
#pragma unroll
  for (int i = 0; i < kN; ++i) {
    const uint32_t e = tb + wave * 64 * kN + static_cast<uint32_t>(i) * 64 + lane;
    valid[i] = e < s.b;
    const uint32_t x = s.b - 1 - e;
    src[i] = x < s.n - 1 ? x : s.n - 1;
  }
#pragma unroll
  for (int i = 0; i < kN; ++i) rk[i] = s.keys[src[i]];
#pragma unroll
  for (int i = 0; i < kN; ++i) rv[i] = vp[src[i]];
  if (s.mode == kMixed) {
#pragma unroll
    for (int i = 0; i < kN; ++i) st[i] = s.is_delete[src[i]] ? 0u : 1u;
  } else {
    const uint32_t c = s.mode == kDelete ? 0u : 1u;
#pragma unroll
    for (int i = 0; i < kN; ++i) st[i] = c;
  }
  const bool enc = s.mode == kEncoded;
#pragma unroll
  for (int i = 0; i < kN; ++i) {
    const uint32_t x = enc ? rk[i] : ((rk[i] << 1) | st[i]);
    const uint32_t v = (enc || st[i] != 0u) ? rv[i] : 0u;  // tombstones carry value 0
    kv[i] = valid[i] ? x : 0u;
    val[i] = valid[i] ? v : 0u;
    key[i] = valid[i] ? (enc ? rk[i] >> 1 : rk[i]) : 0u;
  }
}

struct SortLds {
  uint32_t kv[kSortTile];
  uint32_t val[kSortTile];
  uint32_t wcnt[kWaves][kRadix];
  uint32_t local[kRadix];
  uint32_t gbase[kRadix];
  uint32_t gstart[kRadix];
  uint32_t hist[kMaxPasses * kRadix];
  uint32_t tmp[kWaves];
  uint32_t abort;
};

// Item i of lane l of wave w holds tile position w*64*I + i*64 + l, so
// (item, lane) order is batch order.
__device__ __forceinline__ uint32_t tile_pos(uint32_t wave, int i, uint32_t lane) {
  return wave * 64 * kSortItems + static_cast<uint32_t>(i) * 64 + lane;
}

// One stable counting pass over one tile held in registers: wave64 match-any
// ranking, publication of the tile's digit counts, decoupled look-back over
// the tiles before it, and a scatter through LDS so consecutive threads
// write consecutive output addresses.
__device__ void sort_tile_pass(const uint32_t (&kv)[kSortItems], const uint32_t (&val)[kSortItems],
                               uint32_t tile, uint32_t b, int shift, uint32_t* st,
                               uint32_t* out_kv, uint32_t* out_val, uint32_t* out_fence,
                               bool coherent_out, uint32_t* fault, SortLds& L) {
  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t tbase = tile * kSortTile;
  for (uint32_t i = tid; i < kWaves * kRadix; i += kThreads) (&L.wcnt[0][0])[i] = 0u;
  if (tid == 0) L.abort = 0u;
  __syncthreads();

  uint32_t off[kSortItems];
#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
    const bool valid = tbase + tile_pos(wave, i, lane) < b;
    const uint32_t d = (kv[i] >> shift) & (kRadix - 1);
    uint64_t peers = ballot(valid);
#pragma unroll
    for (int bit = 0; bit < kRadixBits; ++bit) {
      const bool set = (d >> bit) & 1u;
      const uint64_t m = ballot(set);
      peers &= set ? m : ~m;
    }
    const uint32_t r = count_below(peers);
    uint32_t prev = 0;
    if (valid) prev = L.wcnt[wave][d];
    if (valid && r == 0) L.wcnt[wave][d] = prev + static_cast<uint32_t>(__popcll(peers));
    off[i] = prev + r;
  }
  __syncthreads();

  // Thread tid owns digit d = tid (kThreads == kRadix).
  const uint32_t d = tid;
  uint32_t tile_count = 0;
  for (uint32_t w = 0; w < kWaves; ++w) {
    const uint32_t c = L.wcnt[w][d];
    L.wcnt[w][d] = tile_count;
    tile_count += c;
  }
  if (tile == 0) st_dev(&st[d], kFlagInc | tile_count);
  else st_dev(&st[static_cast<size_t>(tile) * kRadix + d], kFlagAgg | tile_count);
  L.local[d] = block_excl_scan(tile_count, L.tmp);

  // Look back in chunks of kChunk predecessors (loads issued together).
  constexpr int kChunk = 16;
  uint32_t excl = 0;
  if (tile > 0) {
    int64_t j = static_cast<int64_t>(tile) - 1;
    uint32_t spins = 0;
    for (;;) {
      const int nchunk = j + 1 < kChunk ? static_cast<int>(j + 1) : kChunk;
      uint32_t w[kChunk];
#pragma unroll
      for (int k = 0; k < kChunk; ++k)
        w[k] = (k < nchunk) ? ld_dev(&st[static_cast<size_t>(j - k) * kRadix + d]) : 0u;
      int used = 0;
      bool done = false;
#pragma unroll
      for (int k = 0; k < kChunk; ++k) {
        if (k >= nchunk || done) break;
        const uint32_t f = w[k] & ~kCountMask;
        if (f == 0u) break;
        excl += w[k] & kCountMask;
        ++used;
        if (f == kFlagInc) done = true;
      }
      if (done) break;
      j -= used;
      if (used == 0) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins == kSpinLimit) {
          atomicOr(fault, kFaultTimeout);
          L.abort = 1u;
          break;
        }
      }
    }
    st_dev(&st[static_cast<size_t>(tile) * kRadix + d], kFlagInc | (excl + tile_count));
  }
  L.gbase[d] = L.gstart[d] + excl;
  __syncthreads();

#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
    if (tbase + tile_pos(wave, i, lane) < b) {
      const uint32_t dd = (kv[i] >> shift) & (kRadix - 1);
      const uint32_t pos = L.local[dd] + L.wcnt[wave][dd] + off[i];
      L.kv[pos] = kv[i];
      L.val[pos] = val[i];
    }
  }
  __syncthreads();
  const uint32_t tile_n = (b - tbase) < static_cast<uint32_t>(kSortTile) ? (b - tbase) : kSortTile;
  if (L.abort == 0u) {
    for (uint32_t x = tid; x < tile_n; x += kThreads) {
      const uint32_t k = L.kv[x];
      const uint32_t dd = (k >> shift) & (kRadix - 1);
      const uint32_t o = L.gbase[dd] + (x - L.local[dd]);
      if (o < b) {
        if (coherent_out) {  // read by other work-groups after a grid barrier
          st_dev(&out_kv[o], k);
          st_dev(&out_val[o], L.val[x]);
        } else {
          out_kv[o] = k;
          out_val[o] = L.val[x];
          put_fence(out_fence, b, o, k);
        }
      }
    }
  }
  __syncthreads();
}

// Digit histograms of every pass in one read of the batch, accumulated into
// hist[parity] (LDS first, then one global atomic per non-zero bucket).
// Also clears hist[parity ^ 1] for the next sort, and this sort's look-back
// words and tile counters.
__global__ __launch_bounds__(kThreads) void k_sort_hist(SortArgs a) {
  __shared__ uint32_t s_h[kMaxPasses * kRadix];
  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const SortMeta& m = a.meta;
  const size_t gthreads = static_cast<size_t>(gridDim.x) * kThreads;
  const size_t gid = static_cast<size_t>(blockIdx.x) * kThreads + tid;
  const size_t nstatus = static_cast<size_t>(a.passes) * m.num_sort_tiles * kRadix;
  for (size_t i = gid; i < nstatus; i += gthreads) m.status[i] = 0u;
  uint32_t* other = m.hist + static_cast<size_t>(m.parity ^ 1) * kMaxPasses * kRadix;
  for (size_t i = gid; i < static_cast<size_t>(kMaxPasses) * kRadix; i += gthreads) other[i] = 0u;
  if (gid < static_cast<size_t>(kMaxPasses)) m.tile_ctr[gid] = 0u;
  for (uint32_t i = tid; i < static_cast<uint32_t>(kMaxPasses * kRadix); i += kThreads) s_h[i] = 0u;
  __syncthreads();

  for (uint32_t t = blockIdx.x; t < m.num_sort_tiles; t += gridDim.x) {
    const uint32_t tb = t * kSortTile;
    uint32_t kv[kSortItems], key[kSortItems], val[kSortItems];
    bool valid[kSortItems];
    tile_items<kSortItems>(a.src, tb, wave, lane, kv, val, key, valid);  // all loads, then count
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
      if (!valid[i]) continue;
      for (int p = 0; p < a.passes; ++p)
        atomicAdd(&s_h[p * kRadix + ((kv[i] >> (a.lo_bit + kRadixBits * p)) & (kRadix - 1))], 1u);
    }
  }
  __syncthreads();
  uint32_t* mine = m.hist + static_cast<size_t>(m.parity) * kMaxPasses * kRadix;
  for (uint32_t i = tid; i < static_cast<uint32_t>(a.passes * kRadix); i += kThreads)
    if (s_h[i] != 0u) atomicAdd(&mine[i], s_h[i]);
}

// One stable counting pass of the batch sort on digit `pass`.  Tiles take
// dynamic ids in start order (so every predecessor a tile waits for has
// started); the tile a work-group most likely receives is loaded while the
// id is in flight.
__global__ __launch_bounds__(kThreads) void k_sort_pass(SortArgs a, int pass) {
  __shared__ SortLds L;
  __shared__ uint32_t s_tile;
  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const SortMeta& m = a.meta;
  const uint32_t b = a.src.b;
  if (tid == 0) s_tile = atomicAdd(&m.tile_ctr[pass], 1u);
  const uint32_t* mine = m.hist + static_cast<size_t>(m.parity) * kMaxPasses * kRadix;
  const uint32_t gtotal = mine[static_cast<size_t>(pass) * kRadix + tid];
  const uint32_t* in_kv = (pass == 0) ? nullptr : a.tmp_kv[(pass - 1) & 1];
  const uint32_t* in_val = (pass == 0) ? nullptr : a.tmp_val[(pass - 1) & 1];
  uint32_t* o_kv = (pass == a.passes - 1) ? a.out_kv : a.tmp_kv[pass & 1];
  uint32_t* o_val = (pass == a.passes - 1) ? a.out_val : a.tmp_val[pass & 1];

  uint32_t kv[kSortItems], val[kSortItems];
  auto load_tile = [&](uint32_t t) {
    const uint32_t tb = t * kSortTile;
    if (in_kv == nullptr) {
      uint32_t key[kSortItems];
      bool valid[kSortItems];
      tile_items<kSortItems>(a.src, tb, wave, lane, kv, val, key, valid);
      return;
    }
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
      const uint32_t e = tb + tile_pos(wave, i, lane);
      const uint32_t ec = e < b ? e : b - 1;  // in bounds; the item is dropped below
      kv[i] = in_kv[ec];
      val[i] = in_val[ec];
    }
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
      const bool ok = tb + tile_pos(wave, i, lane) < b;
      kv[i] = ok ? kv[i] : 0u;
      val[i] = ok ? val[i] : 0u;
    }
  };
  load_tile(blockIdx.x);
  L.gstart[tid] = block_excl_scan(gtotal, L.tmp);  // contains the barrier publishing s_tile
  const uint32_t tile = s_tile;
  if (tile != blockIdx.x) load_tile(tile);
  if (pass == 0 && tile == 0 && a.skew_out != nullptr)
    record_max(mine[static_cast<size_t>(a.passes - 1) * kRadix + tid], a.skew_out, L.tmp);
  uint32_t* st = m.status + static_cast<size_t>(pass) * m.num_sort_tiles * kRadix;
  sort_tile_pass(kv, val, tile, b, a.lo_bit + kRadixBits * pass, st, o_kv, o_val,
                 (pass == a.passes - 1) ? a.out_fence : nullptr, false, &m.err[1], L);
}

// ------------------------------------------------------------ MSD sort
// For batches of at most kMsdMaxTiles tiles the sort exchanges data across
// the device only once: each tile grouped in place by its top kTopBits-bit
// digit (with the batch's digit totals and each tile's group starts), then
// each of the kTopBuckets buckets gathered from every tile and sorted on
// its own by one work-group on the remaining bits (in LDS when it fits,
// streaming through the bucket's global range otherwise).  Two kernels
// instead of 1 + passes, and no look-back chains.

// Stable ranking of one item per lane by digit d among the valid lanes of
// the wave: returns the item's position after the entries already counted
// in wcnt[d], and adds the wave's count of d to wcnt[d].
template <int kBits>
__device__ __forceinline__ uint32_t wave_rank(uint32_t d, bool valid, uint32_t* wcnt) {
  uint64_t peers = ballot(valid);
#pragma unroll
  for (int bit = 0; bit < kBits; ++bit) {
    const bool set = (d >> bit) & 1u;
    const uint64_t m = ballot(set);
    peers &= set ? m : ~m;
  }
  const uint32_t r = count_below(peers);
  uint32_t prev = 0;
  if (valid) prev = wcnt[d];
  if (valid && r == 0) wcnt[d] = prev + static_cast<uint32_t>(__popcll(peers));
  return prev + r;
}

// Stable ranks of a wave's items among equal top digits, item i of every
// lane after item i - 1 (tile order is item-major within the wave).  The
// 10-bit digit is split into two 5-bit halves with a table of lane masks
// each: for every item, each lane ORs its lane bit into the entry of its
// high half in one table and of its low half in the other, reads both
// entries back and clears them, and the AND of the two masks is the set of
// lanes whose item has the same digit.  The six LDS operations of all items
// are issued back to back (one wave's LDS operations are applied in issue
// order, so each item sees exactly its own lanes).  Invalid items use the
// spare entry kHalf of both tables.  Then the lowest lane of each digit
// group adds the group's size to wcnt[d] with an LDS fetch-and-add, items in
// order, and its old count is broadcast to the group.  The tables are this
// wave's own, so no work-group barrier is needed; their entries are zero
// before and after.
constexpr uint32_t kHalfBits = kTopBits / 2;
constexpr uint32_t kHalf = 1u << kHalfBits;
static_assert(2 * kHalfBits == kTopBits, "the top digit splits into two equal halves");
template <int kN>
__device__ __forceinline__ void wave_rank_items(const uint32_t (&d)[kN], const bool (&valid)[kN],
                                                uint64_t* mhi, uint64_t* mlo, uint32_t* wcnt,
                                                uint32_t (&off)[kN]) {
  const uint32_t lane = lane_id();
  const uint64_t bit = 1ull << lane;
  uint64_t grp[kN];
#pragma unroll
  for (int i = 0; i < kN; ++i) {
    uint64_t* eh = &mhi[valid[i] ? (d[i] >> kHalfBits) : kHalf];
    uint64_t* el = &mlo[valid[i] ? (d[i] & (kHalf - 1)) : kHalf];
    __hip_atomic_fetch_or(eh, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __hip_atomic_fetch_or(el, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    grp[i] = *eh & *el;
    *eh = 0ull;
    *el = 0ull;
  }
  uint32_t r[kN], lead[kN], size[kN];
#pragma unroll
  for (int i = 0; i < kN; ++i) {
    r[i] = count_below(grp[i]);
    lead[i] = static_cast<uint32_t>(__builtin_ctzll(grp[i] | (1ull << 63)));
    size[i] = static_cast<uint32_t>(__popcll(grp[i]));
  }
  // Every lane issues the add (others add 0, so the leader's old count is the
  // count before this item whatever order the lanes are applied in).  The
  // counts are 16-bit halves of wcnt's words (digit d in half d & 1 of word
  // d >> 1): a wave adds at most 64 kN <= 65535 per digit, so no carry
  // crosses into the other half.
  static_assert(64 * kN <= 0xFFFF, "per-wave digit counts fit 16 bits");
  uint32_t prev[kN];
#pragma unroll
  for (int i = 0; i < kN; ++i) {
    const uint32_t dd = valid[i] ? d[i] : 0u;
    const uint32_t sh = (dd & 1u) * 16u;
    prev[i] = atomicAdd(&wcnt[dd >> 1], ((valid[i] && r[i] == 0) ? size[i] : 0u) << sh) >> sh;
  }
#pragma unroll
  for (int i = 0; i < kN; ++i)
    off[i] = (static_cast<uint32_t>(__shfl(static_cast<int>(prev[i]), static_cast<int>(lead[i]), 64)) &
              0xFFFFu) + r[i];
}

// Stable scatter of one tile on the top digit, tile-major: the tile's
// elements, grouped by digit (stable within a digit), go back to the tile's
// own range of tmp_kv[0] / tmp_val[0] with coalesced writes, and the tile
// records where each digit's group starts (two 16-bit starts per word; a
// tile holds at most kSortTile elements).  A bucket's elements are then its
// digit's group in every tile, in tile order.  Thread t owns the digits
// [kTopPer t, kTopPer t + kTopPer).  Tile 0 also hands the largest bucket
// recorded by the previous sort in this scratch slot to the host-visible
// hint and restarts the record, and first writes the launch's sequence
// number to the host-visible progress word (the launch has started, so every
// earlier launch on the stream has finished).
struct ScatterLds {
  // Per-wave digit counts, then each wave's offset inside each digit's
  // group: 16-bit halves, digit d in half d & 1 of word d >> 1.
  uint32_t wcnt[kWaves][kTopBuckets / 2];
  uint32_t kv[kSortTile];              // the tile grouped by digit
  uint32_t val[kSortTile];
  union {
    uint64_t mask[kWaves][2][kHalf + 1];  // ranking tables, zero between items
    uint32_t local[kTopBuckets];          // each digit's group start in the tile
  } u;
  uint32_t tmp[2 * kWaves];
  uint32_t rmax[kWaves];
};

__device__ void tile_scatter(const SortArgs& a, int top_shift, uint32_t tile, ScatterLds& S) {
  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const SortMeta& m = a.meta;
  const uint32_t b = a.src.b;
  const uint32_t tbase = tile * kSortTile;
  const uint32_t d0 = tid * kTopPer;
  static_assert(kTopPer == 4 && kSortTile < 65536, "four digits per thread, 16-bit starts");
  uint32_t kv[kSortItems], val[kSortItems], off[kSortItems], dg[kSortItems], key[kSortItems];
  bool valid[kSortItems];
  tile_items<kSortItems>(a.src, tbase, wave, lane, kv, val, key, valid);
  if (tile == 0 && tid == 0 && a.progress != nullptr)
    __hip_atomic_store(a.progress, a.seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  // Tile 0 hands over the largest bucket of the slot's previous bucket sort
  // (a hint for the choice of the next sorts): its loads go out now, the
  // maximum is taken after the tile's ranking.
  static_assert(kTopBuckets == 4 * kThreads, "four bucket records per thread");
  const bool hand = tile == 0 && a.skew_out != nullptr;
  uint4 rec4 = make_uint4(0u, 0u, 0u, 0u);
  if (hand) rec4 = reinterpret_cast<const uint4*>(m.bucket_n)[tid];
  // Rank the tile: each wave clears and fills its own tables.
  for (uint32_t i = lane; i < kTopBuckets / 2; i += 64) S.wcnt[wave][i] = 0u;
  for (uint32_t i = lane; i < 2 * (kHalf + 1); i += 64) (&S.u.mask[wave][0][0])[i] = 0ull;
#pragma unroll
  for (int i = 0; i < kSortItems; ++i) dg[i] = (kv[i] >> top_shift) & (kTopBuckets - 1);
  wave_rank_items(dg, valid, S.u.mask[wave][0], S.u.mask[wave][1], S.wcnt[wave], off);
  __syncthreads();  // every wave is done with its tables: S.u.local may be written
  // This thread's four digits are the halves of words d0 / 2 and d0 / 2 + 1;
  // the wave offsets inside a group are below kSortTile, so they fit too.
  uint32_t cnt[kTopPer], tsum = 0;
  uint32_t wpk[kWaves][2];
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    wpk[w][0] = S.wcnt[w][d0 / 2];
    wpk[w][1] = S.wcnt[w][d0 / 2 + 1];
  }
  uint32_t wo[kWaves][kTopPer];
#pragma unroll
  for (int q = 0; q < kTopPer; ++q) {
    uint32_t run = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      wo[w][q] = run;
      run += (wpk[w][q >> 1] >> ((q & 1) * 16)) & 0xFFFFu;
    }
    cnt[q] = run;
    tsum += run;
  }
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    S.wcnt[w][d0 / 2] = wo[w][0] | (wo[w][1] << 16);
    S.wcnt[w][d0 / 2 + 1] = wo[w][2] | (wo[w][3] << 16);
  }
  uint32_t lrun = block_excl_scan(tsum, S.tmp);
  uint32_t start[kTopPer];
#pragma unroll
  for (int q = 0; q < kTopPer; ++q) {
    start[q] = lrun;
    S.u.local[d0 + q] = lrun;
    lrun += cnt[q];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
    if (valid[i]) {
      const uint32_t dd = dg[i];
      const uint32_t wof = (S.wcnt[wave][dd >> 1] >> ((dd & 1u) * 16u)) & 0xFFFFu;
      const uint32_t pos = S.u.local[dd] + wof + off[i];
      S.kv[pos] = kv[i];
      S.val[pos] = val[i];
    }
  }
  __syncthreads();
  if (hand) {
    uint32_t x = max(max(rec4.x, rec4.y), max(rec4.z, rec4.w));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = max(x, static_cast<uint32_t>(__shfl_xor(x, o, 64)));
    if (lane == 0) S.rmax[wave] = x;
    __syncthreads();
    if (tid == 0) {
      uint32_t mx = 0;
#pragma unroll
      for (int w = 0; w < kWaves; ++w) mx = max(mx, S.rmax[w]);
      *a.skew_out = mx;
    }
  }
  // Global writes last, so that no barrier waits for them: the group starts
  // and the grouped tile.
  uint32_t* row = m.tile_cnt + static_cast<size_t>(tile) * (kTopBuckets / 2);
  row[2 * tid] = start[0] | (start[1] << 16);
  row[2 * tid + 1] = start[2] | (start[3] << 16);
  const uint32_t tile_n = (b - tbase) < static_cast<uint32_t>(kSortTile) ? (b - tbase) : kSortTile;
  for (uint32_t x = tid; x < tile_n; x += kThreads) {
    a.tmp_kv[0][tbase + x] = S.kv[x];
    a.tmp_val[0][tbase + x] = S.val[x];
  }
  (void)key;
}

__global__ __launch_bounds__(kThreads) void k_msd_scatter(SortArgs a, int top_shift) {
  __shared__ ScatterLds S;
  tile_scatter(a, top_shift, blockIdx.x, S);
}

struct alignas(16) LocalLds {
  uint32_t k[2][kLocalCap];
  uint32_t v[2][kLocalCap];
  uint32_t wcnt[kWaves][kRadix];
  uint32_t tmp[2 * kWaves + 2];  // scans; then the bucket's start and size
  uint32_t lo[kMaxFuse];      // fused cascade: start of the digit's range per level
  uint32_t rs[kMaxFuse + 2];  // run starts in the concatenated runs
  const uint32_t* run_k[kMaxFuse + 1];  // fused load: source of each run
  const uint32_t* run_v[kMaxFuse + 1];
  uint32_t run_delta[kMaxFuse + 1];
};

// One stable counting pass over n <= kLocalCap elements in LDS, from
// buffer `from` to buffer 1 - from, on the digit at `shift`.  Wave w owns
// positions [w*S, (w+1)*S) in (item, lane) order, S a multiple of 64.
__device__ void lds_pass(LocalLds& L, int from, uint32_t n, int shift) {
  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t S = ((n + kThreads - 1) / kThreads) * 64;
  const uint32_t* sk = L.k[from];
  const uint32_t* sv = L.v[from];
  uint32_t* dk = L.k[1 - from];
  uint32_t* dv = L.v[1 - from];
  for (uint32_t i = tid; i < kWaves * kRadix; i += kThreads) (&L.wcnt[0][0])[i] = 0u;
  __syncthreads();
  for (uint32_t it = 0; it < S / 64; ++it) {
    const uint32_t pos = wave * S + it * 64 + lane;
    const bool valid = pos < n;
    (void)wave_rank<kRadixBits>(valid ? (sk[pos] >> shift) & (kRadix - 1) : 0u, valid, L.wcnt[wave]);
  }
  __syncthreads();
  uint32_t tot = 0;
  for (uint32_t w = 0; w < kWaves; ++w) {
    const uint32_t c = L.wcnt[w][tid];
    L.wcnt[w][tid] = tot;
    tot += c;
  }
  const uint32_t local = block_excl_scan(tot, L.tmp);
  for (uint32_t w = 0; w < kWaves; ++w) L.wcnt[w][tid] += local;
  __syncthreads();
  for (uint32_t it = 0; it < S / 64; ++it) {
    const uint32_t pos = wave * S + it * 64 + lane;
    const bool valid = pos < n;
    const uint32_t x = valid ? sk[pos] : 0u;
    const uint32_t o = wave_rank<kRadixBits>((x >> shift) & (kRadix - 1), valid, L.wcnt[wave]);
    if (valid) {
      dk[o] = x;
      dv[o] = sv[pos];
    }
  }
  __syncthreads();
}

// Stable passes over a bucket too large for LDS.  The bucket is first
// gathered from the tile-major scatter (group table segb / segp over ntiles
// tiles) into one of two global buffers at the bucket's own range: the
// output (out_kv at s) or the second scratch buffer (tmp_kv[1] at s), chosen
// so that the passes, ping-ponging between the two, end in the output.
// Nothing else reads either range.
__device__ void local_sort_streaming(const SortArgs& a, int lo_bit, int passes, uint32_t s,
                                     uint32_t n, LocalLds& L, const uint32_t* segb,
                                     const uint32_t* segp, uint32_t ntiles) {
  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  uint32_t* bk[2] = {a.out_kv + s, a.tmp_kv[1] + s};
  uint32_t* bv[2] = {a.out_val + s, a.tmp_val[1] + s};
  const int first = passes & 1;
  for (uint32_t x = tid; x < n; x += kThreads) {
    uint32_t g = 0;
    for (uint32_t step = 1u << (31 - __builtin_clz(ntiles)); step > 0; step >>= 1) {
      const uint32_t probe = g + step;
      if (probe < ntiles && segp[probe] <= x) g = probe;
    }
    const uint32_t at = segb[g] + (x - segp[g]);
    const uint32_t k = a.tmp_kv[0][at];
    bk[first][x] = k;
    bv[first][x] = a.tmp_val[0][at];
    if (passes == 0) put_fence(a.out_fence, a.out_n, s + x, k);
  }
  if (passes == 0) return;
  __threadfence_block();
  __syncthreads();
  uint32_t* run = L.k[0];       // running output position per digit
  uint32_t* chunk_cnt = L.k[1];
  for (int p = 0; p < passes; ++p) {
    const int shift = lo_bit + kRadixBits * p;
    const int cur = first ^ (p & 1);  // the last pass writes buffer 0, the output
    const uint32_t* ik = bk[cur];
    const uint32_t* iv = bv[cur];
    uint32_t* ok = bk[cur ^ 1];
    uint32_t* ov = bv[cur ^ 1];
    run[tid] = 0u;
    __syncthreads();
    // Every pass reads this work-group's own writes.
    for (uint32_t x = tid; x < n; x += kThreads) {
      const uint32_t k = ik[x];
      atomicAdd(&run[(k >> shift) & (kRadix - 1)], 1u);
    }
    __syncthreads();
    const uint32_t c = run[tid];
    __syncthreads();
    run[tid] = block_excl_scan(c, L.tmp);
    __syncthreads();
    for (uint32_t cb = 0; cb < n; cb += kSortTile) {
      uint32_t kv[kSortItems], vv[kSortItems], off[kSortItems];
#pragma unroll
      for (int i = 0; i < kSortItems; ++i) {
        const uint32_t e = cb + tile_pos(wave, i, lane);
        kv[i] = e < n ? ik[e] : 0u;
        vv[i] = e < n ? iv[e] : 0u;
      }
      for (uint32_t i = tid; i < kWaves * kRadix; i += kThreads) (&L.wcnt[0][0])[i] = 0u;
      __syncthreads();
#pragma unroll
      for (int i = 0; i < kSortItems; ++i)
        off[i] = wave_rank<kRadixBits>((kv[i] >> shift) & (kRadix - 1), cb + tile_pos(wave, i, lane) < n,
                            L.wcnt[wave]);
      __syncthreads();
      uint32_t tot = 0;
      for (uint32_t w = 0; w < kWaves; ++w) {
        const uint32_t cc = L.wcnt[w][tid];
        L.wcnt[w][tid] = tot;
        tot += cc;
      }
      chunk_cnt[tid] = tot;
      __syncthreads();
#pragma unroll
      for (int i = 0; i < kSortItems; ++i) {
        if (cb + tile_pos(wave, i, lane) < n) {
          const uint32_t dd = (kv[i] >> shift) & (kRadix - 1);
          const uint32_t o = run[dd] + L.wcnt[wave][dd] + off[i];
          if (o < n) {
            ok[o] = kv[i];
            ov[o] = vv[i];
            if (p == passes - 1) put_fence(a.out_fence, a.out_n, s + o, kv[i]);
          }
        }
      }
      __syncthreads();
      run[tid] += chunk_cnt[tid];
      __syncthreads();
    }
  }
}

// Stable merge in LDS of a = src[0, A) (newer) and b = src[A, A + c)
// (older) into dst[0, A + c), a first on equal original keys.  Each thread
// finds the merge-path split of its share of the output by binary search,
// then merges it sequentially.  Ends with a barrier.
__device__ void lds_merge_pair(const uint32_t* sk, const uint32_t* sv, uint32_t A, uint32_t c,
                               uint32_t* dk, uint32_t* dv) {
  const uint32_t total = A + c;
  const uint32_t per = (total + kThreads - 1) / kThreads;
  const uint32_t d0 = threadIdx.x * per < total ? threadIdx.x * per : total;
  const uint32_t d1 = d0 + per < total ? d0 + per : total;
  uint32_t lo = d0 > c ? d0 - c : 0, hi = d0 < A ? d0 : A;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if ((sk[mid] >> 1) <= (sk[A + d0 - 1 - mid] >> 1)) lo = mid + 1;
    else hi = mid;
  }
  uint32_t ia = lo, ib = d0 - lo;
  for (uint32_t o = d0; o < d1; ++o) {
    const bool take_a = ia < A && (ib >= c || (sk[ia] >> 1) <= (sk[A + ib] >> 1));
    const uint32_t src = take_a ? ia : A + ib;
    dk[o] = sk[src];
    dv[o] = sv[src];
    ia += take_a ? 1u : 0u;
    ib += take_a ? 0u : 1u;
  }
  __syncthreads();
}

// Stable rank sort of the bucket's n <= kRankSortMax elements, held in
// L.k[0] / L.v[0], into L.k[1] / L.v[1].  fld[0, n8) holds each element's
// sort key (field << 8) | x, where the field is bits [lo_bit, lo_bit + 8
// passes) of its key variable (at most 24 bits: the bits below the top
// digit) and x its position; n8 = n rounded up to 8, with 0xFFFFFFFF past n.
// The keys are distinct, so the rank of element x, the number of smaller
// keys, orders by field and then by position (a stable sort, the same order
// as the radix passes over those bits).  The keys are read four at a time
// (16-byte LDS reads, eight in flight); the entries past n are above every
// element's key.  Waves without elements skip the count.
__device__ void rank_sort(LocalLds& L, const uint32_t* fld, uint32_t n) {
  static_assert(kRankSortMax <= 256u && kRankSortMax <= static_cast<uint32_t>(kThreads),
                "positions fit 8 bits; one element per thread");
  const uint32_t tid = threadIdx.x;
  if ((tid & ~63u) < n) {
    const uint32_t n8 = (n + 7u) & ~7u;
    const uint32_t cx = tid < n ? fld[tid] : 0u;
    uint32_t rank = 0;
    const uint4* f4 = reinterpret_cast<const uint4*>(fld);
    auto below = [cx](const uint4& p) {
      return (p.x < cx ? 1u : 0u) + (p.y < cx ? 1u : 0u) + (p.z < cx ? 1u : 0u) +
             (p.w < cx ? 1u : 0u);
    };
    uint32_t y = 0;
    for (; y + 32u <= n8; y += 32u) {  // eight 16-byte reads in flight
      uint4 p[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) p[u] = f4[y / 4 + u];
#pragma unroll
      for (int u = 0; u < 8; ++u) rank += below(p[u]);
    }
    for (; y < n8; y += 8u) {
      const uint4 p = f4[y / 4];
      const uint4 q = f4[y / 4 + 1];
      rank += below(p) + below(q);
    }
    if (tid < n) {
      L.k[1][rank] = L.k[0][tid];
      L.v[1][rank] = L.v[0][tid];
    }
  }
  __syncthreads();
}

// Bound of original key k in the sorted segment [lo, hi) of s (LDS or
// global): first position whose key is >= k (upper: > k).
__device__ __forceinline__ uint32_t seg_bound(const uint32_t* s, uint32_t lo, uint32_t hi,
                                              uint32_t k, bool upper) {
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    const uint32_t x = s[mid] >> 1;
    if (upper ? x <= k : x < k) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// One work-group per top-digit bucket d.  The bucket is digit d's group in
// every tile of the tile-major scatter, gathered in tile order (the batch's
// order), and is sorted on the digits below the top one: by ranking up to
// kRankSortMax elements, by LDS radix passes up to kLocalCap, else by
// streaming passes over global memory.  Without a fused cascade the sorted
// bucket is the output.
//
// With a fused cascade (a.fuse.nlev = j > 0), the work-group then merges
// its bucket with the same digit's key range of levels 0..j-1 (read from
// each level's top-digit index) and writes that part of level j, recording
// where it starts in level j's index.  Runs fitting in LDS are merged there
// pairwise, newest first, exactly as the cascade merges whole levels.  Larger
// ones are ranked with searches in global memory: runs are numbered newest
// first (the batch, then level 0, 1, ...), and an element's output rank is
// its position in its run plus, for every newer run, the elements with a key
// <= its key and, for every older run, the elements with a smaller key;
// (key, run, position) is a strict total order, so the order is again the
// cascade's.  Without fusion, the sort of a level records its buckets'
// starts as that level's top-digit index.
__device__ void bucket_sort(const SortArgs& a, int lo_bit, int passes, uint32_t d, LocalLds& L) {
  const uint32_t tid = threadIdx.x;
  const SortMeta& m = a.meta;
  const FuseArgs& f = a.fuse;
  const bool fused = f.nlev > 0;
  const int R = f.nlev + 1;  // runs: the batch, then levels 0..j-1
  // Bucket d is digit d's group in every tile of the tile-major scatter, in
  // tile order; its sorted output starts at s, the number of batch elements
  // with a smaller digit, which is the sum over the tiles of the start of
  // digit d's group.  Every load of this prologue is issued unconditionally
  // (clamped index), so each tile's group bounds and the levels' digit
  // ranges are in flight together.
  auto next_of = [](uint32_t q) { return q + 1 < kTopBuckets ? q + 1 : q; };
  // A group (consecutive batches sorted together, the newer first on equal
  // keys) has the newest batch's tiles, then the next older batch's, and so
  // on: nta group-table entries, one per thread.
  const uint32_t ntiles = m.num_sort_tiles;
  const uint32_t G = a.group;
  const uint32_t nta = G * ntiles;
  static_assert(kMsdMaxTiles <= kThreads, "one tile per thread");
  static_assert(kMaxGroup == 4, "the batch of a tile is chosen among four");
  const uint32_t bq = tid >= nta ? 0u
                    : (tid >= ntiles ? 1u : 0u) + (tid >= 2 * ntiles ? 1u : 0u) +
                          (tid >= 3 * ntiles ? 1u : 0u);  // the tile's batch in the group
  const uint32_t tt = tid < nta ? tid - bq * ntiles : 0u;  // tile in its batch
  const uint32_t* cnt_q = bq == 0 ? a.grp_cnt[0] : bq == 1 ? a.grp_cnt[1]
                        : bq == 2 ? a.grp_cnt[2] : a.grp_cnt[3];
  const uint32_t off_q = bq == 0 ? a.grp_off[0] : bq == 1 ? a.grp_off[1]
                       : bq == 2 ? a.grp_off[2] : a.grp_off[3];
  const uint32_t* row = cnt_q + static_cast<size_t>(tt) * (kTopBuckets / 2);
  const uint32_t seg_w0 = row[d >> 1];
  const uint32_t seg_w1 = row[next_of(d) >> 1];
  // The digit's range in each fused level, from the level's top-digit index:
  // uniform loads, all issued before any is used (slots past j read level
  // 0's index and are ignored).
  uint32_t dlo[kMaxFuse], dhi[kMaxFuse], dlen[kMaxFuse];
  if (fused) {
#pragma unroll
    for (int q = 0; q < kMaxFuse; ++q) {
      const uint32_t* dp = f.digit[q < f.nlev ? q : 0];
      dlo[q] = dp[d];
      dhi[q] = dp[next_of(d)];
      dlen[q] = q < f.nlev ? f.len[q] : 0u;
    }
  } else {
#pragma unroll
    for (int q = 0; q < kMaxFuse; ++q) dlo[q] = dhi[q] = dlen[q] = 0u;
  }
  // The group of digit d in tile t = tid: [start_t[d], start_t[d + 1]) of
  // the tile (the last digit's ends at the tile's size).
  const uint32_t g_st = (d & 1) ? seg_w0 >> 16 : seg_w0 & 0xFFFFu;
  const uint32_t tile_n =
      tid < nta ? min(a.src.b - tt * kSortTile, static_cast<uint32_t>(kSortTile)) : 0u;
  const uint32_t g_en = d + 1 < kTopBuckets ? (((d + 1) & 1) ? seg_w1 >> 16 : seg_w1 & 0xFFFFu)
                                            : tile_n;
  const uint32_t g_c = (tid < nta && g_en > g_st) ? g_en - g_st : 0u;
  // One pass of two scans: the group starts (their total is the bucket's
  // output start) and the group sizes (each group's first position in the
  // bucket; their total is the bucket's size).
  const uint32_t g_s0 = tid < nta ? g_st : 0u;
  uint32_t ssum = g_s0, csum = g_c;
  block_excl_scan2(ssum, csum, L.tmp);
  uint32_t* segb = &L.wcnt[0][0] + (kRankSortMax + 8);  // group sources in the batch
  uint32_t* segp = segb + kMsdMaxTiles;                  // group starts in the bucket
  static_assert(kRankSortMax + 8 + 2 * kMsdMaxTiles <= kWaves * kRadix,
                "group tables fit beside the rank-sort keys");
  if (tid < nta) {
    segb[tid] = off_q + tt * kSortTile + g_st;
    segp[tid] = csum;
  }
  if (tid == kThreads - 1) {
    L.tmp[2 * kWaves] = ssum + g_s0;
    L.tmp[2 * kWaves + 1] = csum + g_c;
  }
  if (tid == 0) {  // run 0 of the load table: the scattered batch
    L.run_k[0] = a.tmp_kv[0];
    L.run_v[0] = a.tmp_val[0];
    L.run_delta[0] = 0;
  }
  __syncthreads();
  const uint32_t s = L.tmp[2 * kWaves];
  const uint32_t n = L.tmp[2 * kWaves + 1];
  // The sort's largest bucket, for the choice of the next sorts' path and
  // fused depth (only sizes that can change those choices are recorded).
  // Bucket d's size (for a group, its share per batch) goes to the record of
  // every batch's slot with a plain store: every bucket sort writes all of
  // a record, so no atomics and no clearing are needed; the next scatter
  // into any of the slots takes the largest entry.
  if (tid < G) {
    uint32_t* rec = tid == 0 ? a.grp_n[0] : tid == 1 ? a.grp_n[1]
                  : tid == 2 ? a.grp_n[2] : a.grp_n[3];
    rec[d] = (n + G - 1) / G;
  }
  if (!fused && a.out_digit != nullptr && tid == 0) a.out_digit[d] = s;
  if (n == 0 && !fused) return;

  // Run starts in the concatenation (the batch's bucket, then each level's
  // range) and the first output position, computed by every thread (uniform
  // values); thread 0 also keeps them in LDS for the merge code below.
  uint32_t lo_q[kMaxFuse], rs_q[kMaxFuse + 2];
  rs_q[0] = 0;
  rs_q[1] = n;
  uint64_t out0 = s;
  uint32_t T = n;
#pragma unroll
  for (int q = 0; q < kMaxFuse; ++q) {
    const bool on = q < f.nlev;
    const uint32_t len = dlen[q];
    const uint32_t lo = dlo[q] < len ? dlo[q] : len;
    const uint32_t hi_d = d == kTopBuckets - 1 ? len : dhi[q];
    const uint32_t hi = hi_d < lo ? lo : (hi_d < len ? hi_d : len);
    lo_q[q] = lo;
    rs_q[q + 2] = rs_q[q + 1] + (hi - lo);
    out0 += lo;
    T += hi - lo;
    if (on && tid == 0) {
      L.lo[q] = lo;
      L.rs[q + 2] = rs_q[q + 2];
    }
  }
  if (fused && tid == 0) {
    L.rs[0] = 0;
    L.rs[1] = n;
    if (f.out_digit != nullptr) f.out_digit[d] = static_cast<uint32_t>(out0);
  }
  if (T == 0) return;

  // ---- one load phase.  The batch's bucket goes to buffer 0 (the sort's
  // input); when all runs fit in LDS, level l's range goes to its place in
  // [n, T) of buffer buf (l even) or 1 - buf (l odd), buf being the buffer
  // the sorted bucket ends in (the rank sort writes buffer 1, the radix
  // passes alternate from buffer 0): the cascade below then finds each run
  // next to the accumulated one.  Up to kLocalCap / kThreads elements per
  // thread, loads issued unconditionally (clamped position) before any is
  // stored.
  const bool rank_path = n <= kRankSortMax;
  const int buf = (rank_path || (passes & 1)) ? 1 : 0;
  const uint32_t nl = T <= static_cast<uint32_t>(kLocalCap) ? T
                      : (n <= static_cast<uint32_t>(kLocalCap) ? n : 0u);
  // The bits below the top digit: at most 32 - kTopBits, so 8 passes <= 24
  // and the rank sort's (field << 8) | position fits 32 bits.
  static_assert(32 - kTopBits <= 3 * kRadixBits, "local passes <= 3");
  const uint32_t fmask = (kRadixBits * passes >= 24) ? 0xFFFFFFu
                                                     : ((1u << (kRadixBits * passes)) - 1u);
  uint32_t* fld = &L.wcnt[0][0];  // rank-sort keys
  static_assert(kWaves * kRadix >= kRankSortMax + 8, "field scratch");
  const bool levels_in_lds = nl > n;  // fused, and all runs fit
  if (levels_in_lds) {
    // Run table: run q + 1 is level q, whose element x is source position
    // x + delta[q + 1]; run 0, the batch's bucket (written in the
    // prologue), is read through the group table instead.
    if (tid == 0) {
#pragma unroll
      for (int q = 0; q < kMaxFuse; ++q) {
        if (q < f.nlev) {
          L.run_k[q + 1] = f.kv[q];
          L.run_v[q + 1] = f.val[q];
          L.run_delta[q + 1] = lo_q[q] - rs_q[q + 1];
        }
      }
    }
    __syncthreads();
  }
  // The load phase for at most kPer items per thread (instantiated for 1,
  // 4 and 8, so that a small bucket does not search for absent items).
  auto load_phase = [&](auto per_c) {
    constexpr int kPer = decltype(per_c)::value;
    uint32_t rk[kPer], rv[kPer], run[kPer];
    // Each element's run (the number of level starts at or below it); a
    // batch element's position in the scattered batch comes from its
    // tile's group (the last group starting at or below it, by a search
    // over the group starts, the searches of a thread's elements in
    // lockstep), a level element's from the run table; loads issued before
    // any store.
    uint32_t bidx[kPer];
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const uint32_t x = tid + i * kThreads;
      const uint32_t xc = x < nl ? x : nl - 1;
      run[i] = 0;
      if (levels_in_lds) {
#pragma unroll
        for (int q = 1; q <= kMaxFuse; ++q) run[i] += (q <= f.nlev && xc >= rs_q[q]) ? 1u : 0u;
      }
      bidx[i] = 0;
    }
    // Straight-line searches and table reads for every item (positions
    // clamped, results of items past nl unused), so that the LDS reads of
    // all items are in flight together and the loads below issue back to
    // back.
    // Only items that can hold batch elements search (all kPer, or just the
    // first when the bucket fits one item per thread).
    const uint32_t xbmax = n > 0 ? n - 1 : 0u;
    auto search = [&](auto cnt_c) {
      constexpr int kS = decltype(cnt_c)::value;
      for (uint32_t step = 1u << (31 - __builtin_clz(nta)); step > 0; step >>= 1) {
#pragma unroll
        for (int i = 0; i < kS; ++i) {
          const uint32_t x = tid + i * kThreads;
          const uint32_t xb = x < xbmax ? x : xbmax;
          const uint32_t probe = bidx[i] + step;
          const uint32_t pc = probe < nta ? probe : nta - 1;
          const uint32_t v = segp[pc];
          bidx[i] = ((probe < nta) & (v <= xb)) ? probe : bidx[i];
        }
      }
    };
    if (n <= static_cast<uint32_t>(kThreads))
      search(std::integral_constant<int, 1>{});
    else
      search(std::integral_constant<int, kPer>{});
    const uint32_t* pk[kPer];
    const uint32_t* pv[kPer];
    uint32_t at[kPer];
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const uint32_t x = tid + i * kThreads;
      const uint32_t xc = x < nl ? x : nl - 1;
      const uint32_t xb = x < xbmax ? x : xbmax;
      const uint32_t r = levels_in_lds ? run[i] : 0u;
      const uint32_t gb = segb[bidx[i]], gp = segp[bidx[i]];
      pk[i] = L.run_k[r];
      pv[i] = L.run_v[r];
      at[i] = r == 0 ? gb + (xb - gp) : xc + L.run_delta[r];
    }
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      if (static_cast<uint32_t>(i) * kThreads < nl) {
        rk[i] = as_global(pk[i])[at[i]];
        rv[i] = as_global(pv[i])[at[i]];
      }
    }
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const uint32_t x = tid + i * kThreads;
      if (static_cast<uint32_t>(i) * kThreads < nl && x < nl) {
        const int to = x < n ? 0 : ((run[i] & 1u) ? buf : 1 - buf);
        L.k[to][x] = rk[i];
        L.v[to][x] = rv[i];
        if (rank_path && x < n) fld[x] = (((rk[i] >> lo_bit) & fmask) << 8) | x;
      }
    }
    if (rank_path && tid >= n && tid < ((n + 7u) & ~7u)) fld[tid] = 0xFFFFFFFFu;
  };
  if (nl > 0) {
    if (nl <= static_cast<uint32_t>(kThreads))
      load_phase(std::integral_constant<int, 1>{});
    else if (nl <= static_cast<uint32_t>(4 * kThreads))
      load_phase(std::integral_constant<int, 4>{});
    else
      load_phase(std::integral_constant<int, kLocalCap / kThreads>{});
  }
  __syncthreads();  // the loaded runs, fields and L.lo / L.rs

  // ---- sort the batch's bucket.  sorted = true when it ends in LDS buffer
  // buf, false when it was sorted in global memory (at out_k / out_v).
  uint32_t* out_k = a.out_kv + s;
  uint32_t* out_v = a.out_val + s;
  bool sorted_lds = true;
  if (n == 0) {
  } else if (rank_path) {
    rank_sort(L, fld, n);
  } else if (n <= static_cast<uint32_t>(kLocalCap)) {
    int cur = 0;
    for (int p = 0; p < passes; ++p) {
      lds_pass(L, cur, n, lo_bit + kRadixBits * p);
      cur = 1 - cur;
    }
  } else {
    sorted_lds = false;
    local_sort_streaming(a, lo_bit, passes, s, n, L, segb, segp, nta);
  }

  if (!fused) {
    if (sorted_lds) {
      for (uint32_t x = tid; x < n; x += kThreads) {
        const uint32_t k = L.k[buf][x];
        out_k[x] = k;
        out_v[x] = L.v[buf][x];
        put_fence(a.out_fence, a.out_n, s + x, k);
      }
    }
    return;
  }

  if (sorted_lds && T <= static_cast<uint32_t>(kLocalCap)) {
    // A pairwise cascade in LDS: the accumulated run (newer, [0, rs[q]))
    // and the next level's run (older, [rs[q], rs[q + 1]), loaded into the
    // same buffer) are merged into [0, rs[q + 1]) of the other buffer, which
    // holds no run still to be read there.
    int acc = buf;
    for (int q = 1; q < R; ++q) {
      const uint32_t A = L.rs[q], c = L.rs[q + 1] - L.rs[q];
      lds_merge_pair(L.k[acc], L.v[acc], A, c, L.k[1 - acc], L.v[1 - acc]);
      acc = 1 - acc;
    }
    for (uint32_t x = tid; x < T; x += kThreads) {
      const uint64_t pos = out0 + x;
      if (pos < f.out_len) {
        const uint32_t k = L.k[acc][x];
        f.out_kv[pos] = k;
        f.out_val[pos] = L.v[acc][x];
        put_fence(f.out_fence, f.out_len, pos, k);
      }
    }
    return;
  }

  // Runs too large for LDS: rank with searches in global memory.  The
  // batch's bucket is put in global scratch first (it may be in LDS).
  if (sorted_lds) {
    for (uint32_t x = tid; x < n; x += kThreads) {
      out_k[x] = L.k[buf][x];
      out_v[x] = L.v[buf][x];
    }
  }
  __threadfence_block();
  __syncthreads();
  for (uint32_t e = tid; e < T; e += kThreads) {
    int r = 0;
    while (r + 1 < R && L.rs[r + 1] <= e) ++r;
    const uint32_t p = e - L.rs[r];
    const uint32_t* rkp = r == 0 ? out_k : f.kv[r - 1] + L.lo[r - 1];
    const uint32_t* rvp = r == 0 ? out_v : f.val[r - 1] + L.lo[r - 1];
    const uint32_t x = rkp[p];
    const uint32_t key = x >> 1;
    uint32_t rank = p;
    for (int q = 0; q < R; ++q) {
      if (q == r) continue;
      const uint32_t* qk = q == 0 ? out_k : f.kv[q - 1] + L.lo[q - 1];
      rank += seg_bound(qk, 0, L.rs[q + 1] - L.rs[q], key, q < r);
    }
    const uint64_t pos = out0 + rank;
    if (pos < f.out_len) {
      f.out_kv[pos] = x;
      f.out_val[pos] = rvp[p];
      put_fence(f.out_fence, f.out_len, pos, x);
    }
  }
}

// Bucket work-group w (counted from the first bucket work-group) takes top
// digit (w % 8) * 128 + w / 8: work-groups go to the 8 XCDs in turn, so the
// work-groups with one w % 8 share an XCD, take 128 consecutive digits and
// read each tile's groups (adjacent in the tile) through that XCD's L2.
__device__ __forceinline__ uint32_t xcd_digit(uint32_t w) {
  return (w & 7u) * (kTopBuckets / 8) + (w >> 3);
}

__global__ __launch_bounds__(kThreads) void k_local_sort(SortArgs a, int lo_bit, int passes) {
  __shared__ LocalLds L;
  bucket_sort(a, lo_bit, passes, xcd_digit(blockIdx.x), L);
}

// One step of the pipelined top-digit sort: the first work-groups scatter
// the tiles of the new batch (sc) into one scratch slot while the others
// sort the buckets of the previous batch (bk) out of the other slot, with
// its fused cascade.  The two halves share no memory except what each reads
// from earlier kernels, so they need no synchronisation.
union StepLds {
  ScatterLds S;
  LocalLds L;
};
static_assert(sizeof(ScatterLds) <= sizeof(LocalLds),
              "the scatter half must not raise the step's LDS above the bucket sort's");

__global__ __launch_bounds__(kThreads) void k_sort_step(SortArgs bk, int lo_bit, int passes,
                                                        SortArgs sc, int top_shift) {
  __shared__ StepLds U;
  const uint32_t nt = sc.meta.num_sort_tiles;
  if (blockIdx.x < nt) tile_scatter(sc, top_shift, blockIdx.x, U.S);
  else bucket_sort(bk, lo_bit, passes, xcd_digit(blockIdx.x - nt), U.L);
}

// ------------------------------------------------------------ merge
// Number of elements of a (the newer run) among the first `diag` outputs of
// the merge, a first on equal original keys.  The whole wave searches: each
// round tests 64 evenly spaced candidates of the open interval and keeps the
// gap where the predicate flips, so a run of 2^26 takes five rounds.
__device__ uint32_t wave_merge_path(const uint32_t* a, uint32_t na, const uint32_t* bb,
                                    uint32_t nb, uint64_t diag) {
  const uint32_t lane = lane_id();
  uint64_t lo = diag > nb ? diag - nb : 0;
  uint64_t hi = diag < na ? diag : na;
  while (hi > lo) {
    const uint64_t len = hi - lo;
    if (len <= 64) {
      bool p = false;
      if (lane < len) {
        const uint64_t i = lo + lane;
        p = (a[i] >> 1) <= (bb[diag - 1 - i] >> 1);
      }
      return static_cast<uint32_t>(lo + __popcll(ballot(p)));
    }
    const uint64_t pos = lo + ((lane + 1) * len) / 65;
    const bool p = (a[pos] >> 1) <= (bb[diag - 1 - pos] >> 1);
    const uint32_t c = static_cast<uint32_t>(__popcll(ballot(p)));
    if (c == 0) {
      hi = lo + len / 65;
    } else if (c == 64) {
      lo = lo + (64 * len) / 65 + 1;
    } else {
      const uint64_t plo = lo + (c * len) / 65;
      const uint64_t phi = lo + ((c + 1) * len) / 65;
      lo = plo + 1;
      hi = phi;
    }
  }
  return static_cast<uint32_t>(lo);
}


// Merge-path split inside the work-group's windows, held in circular LDS
// buffers: window a is positions [a0, a0 + wa) of run a at slots
// (a0 + i) & mask, window b likewise.  Returns how many of the first dt
// outputs come from a (a first on equal original keys).
__device__ __forceinline__ uint32_t ring_merge_path(const uint32_t* sa, uint32_t a0, uint32_t wa,
                                                    const uint32_t* sb, uint32_t b0, uint32_t wb,
                                                    uint32_t dt, uint32_t mask) {
  uint32_t lo = dt > wb ? dt - wb : 0, hi = dt < wa ? dt : wa;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if ((sa[(a0 + mid) & mask] >> 1) <= (sb[(b0 + dt - 1 - mid) & mask] >> 1)) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Merge of run a (newer) with run b (older) on the original key.  Each
// work-group produces one contiguous range of the output, found one of two
// ways:
//   * digit mode (both runs carry a top-digit index): work-group w takes the
//     top digits [w per_wg, (w + 1) per_wg); each index gives the range of its
//     run holding those digits, and the output range starts at the sum of the
//     two starts (equal keys share a digit, so no tie crosses a range
//     boundary).  No search at all.  The output's own index is the sum of the
//     two indexes, digit by digit.
//   * search mode: work-group w takes output tiles [w per_wg, (w + 1) per_wg)
//     and finds the splits at the start and the end of its range with two
//     wave searches in global memory (waves 0 and 1, side by side).
// The range is then produced tile by tile, the tiles anchored at 16-byte
// aligned output positions (the first tile of a range may start inside its
// tile).  Both runs' windows live in LDS ring buffers: a tile's outputs
// consume la elements of a and n - la of b, and the next tile loads exactly
// those counts; windows never extend past the range's end, so every input
// element is read from HBM once.  A window's new elements are all loaded
// before any is stored.  Each thread merges kMergeItems consecutive outputs
// and stores them with 16-byte stores.
struct MergeArgs {
  const uint32_t* a_kv;
  const uint32_t* a_val;
  const uint32_t* b_kv;
  const uint32_t* b_val;
  uint32_t na, nb;
  uint32_t* out_kv;
  uint32_t* out_val;
  uint32_t* out_fence;     // the output level's fence tree, or null
  const uint32_t* a_dig;   // top-digit indexes of both runs, or null
  const uint32_t* b_dig;
  uint32_t* out_dig;       // receives the output's index (both runs indexed), or null
  int digit_mode;          // partition by digit ranges (needs both indexes)
  uint32_t per_wg;         // digits (digit mode) or output tiles per work-group
};

template <int kMergeItems>
__global__ __launch_bounds__(kThreads) void k_merge(MergeArgs m) {
  constexpr uint32_t kMergeTile = kThreads * kMergeItems;
  constexpr uint32_t kMask = kMergeTile - 1;
  static_assert((kMergeTile & kMask) == 0, "merge tile must be a power of two");
  static_assert(kMergeItems % 4 == 0, "16-byte stores");
  __shared__ uint32_t sa_k[kMergeTile], sa_v[kMergeTile], sb_k[kMergeTile], sb_v[kMergeTile];
  __shared__ uint32_t s_split, s_split_end;
  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t na = m.na, nb = m.nb;
  const uint64_t total = static_cast<uint64_t>(na) + nb;
  uint32_t a0, b0, a_lim, b_lim;  // the work-group consumes a[a0, a_lim), b[b0, b_lim)
  if (m.digit_mode) {
    const uint32_t q0 = blockIdx.x * m.per_wg;
    if (q0 >= kTopBuckets) return;
    const uint32_t q1 = min(q0 + m.per_wg, kTopBuckets);
    // Index entries are positions in their run; clamped so that a damaged
    // index can only give wrong output, never an access out of bounds.
    a0 = min(m.a_dig[q0], na);
    b0 = min(m.b_dig[q0], nb);
    a_lim = q1 < kTopBuckets ? min(max(m.a_dig[q1], a0), na) : na;
    b_lim = q1 < kTopBuckets ? min(max(m.b_dig[q1], b0), nb) : nb;
    if (m.out_dig != nullptr)
      for (uint32_t q = q0 + tid; q < q1; q += kThreads) m.out_dig[q] = m.a_dig[q] + m.b_dig[q];
  } else {
    if (m.out_dig != nullptr)
      for (uint32_t q = blockIdx.x * kThreads + tid; q < kTopBuckets; q += gridDim.x * kThreads)
        m.out_dig[q] = m.a_dig[q] + m.b_dig[q];
    const uint64_t tiles = (total + kMergeTile - 1) / kMergeTile;
    const uint64_t t = static_cast<uint64_t>(blockIdx.x) * m.per_wg;
    const uint64_t t_end = (t + m.per_wg < tiles) ? t + m.per_wg : tiles;
    if (t >= t_end) return;
    if (wave == 0) {
      const uint32_t sp = wave_merge_path(m.a_kv, na, m.b_kv, nb, t * kMergeTile);
      if (lane == 0) s_split = sp;
    } else if (wave == 1) {
      const uint64_t de = t_end * kMergeTile;
      const uint32_t sp = de >= total ? na : wave_merge_path(m.a_kv, na, m.b_kv, nb, de);
      if (lane == 0) s_split_end = sp;
    }
    __syncthreads();
    a0 = s_split;
    b0 = static_cast<uint32_t>(t * kMergeTile - a0);
    a_lim = s_split_end;
    b_lim = static_cast<uint32_t>((t_end * kMergeTile < total ? t_end * kMergeTile : total) - a_lim);
  }
  const uint64_t o_end = static_cast<uint64_t>(a_lim) + b_lim;
  uint32_t a_end = a0, b_end = b0;  // loaded into the rings up to here
  // New window elements [from, to) of one run into its ring: at most
  // kMergeTile, so kMergeItems per thread; loads at clamped positions first.
  auto fill = [&](const uint32_t* gk, const uint32_t* gv, uint32_t from, uint32_t to,
                  uint32_t* rk_s, uint32_t* rv_s) {
    if (from >= to) return;
    uint32_t k[kMergeItems], v[kMergeItems];
#pragma unroll
    for (int j = 0; j < kMergeItems; ++j) {
      const uint32_t x = from + tid + static_cast<uint32_t>(j) * kThreads;
      const uint32_t xc = x < to ? x : to - 1;
      k[j] = gk[xc];
      v[j] = gv[xc];
    }
#pragma unroll
    for (int j = 0; j < kMergeItems; ++j) {
      const uint32_t x = from + tid + static_cast<uint32_t>(j) * kThreads;
      if (x < to) {
        rk_s[x & kMask] = k[j];
        rv_s[x & kMask] = v[j];
      }
    }
  };
  // Tiles anchored at 16-byte aligned output positions g0; the next output
  // is always at a0 + b0.
  for (uint64_t g0 = (static_cast<uint64_t>(a0) + b0) & ~uint64_t(3); g0 < o_end; g0 += kMergeTile) {
    const uint64_t p0 = static_cast<uint64_t>(a0) + b0;  // first output of this tile's part
    const uint64_t tile_end = (g0 + kMergeTile < o_end) ? g0 + kMergeTile : o_end;
    const uint32_t n = static_cast<uint32_t>(tile_end - p0);
    const uint32_t wa = (a_lim - a0) < n ? (a_lim - a0) : n;
    const uint32_t wb = (b_lim - b0) < n ? (b_lim - b0) : n;
    fill(m.a_kv, m.a_val, a_end, a0 + wa, sa_k, sa_v);
    fill(m.b_kv, m.b_val, b_end, b0 + wb, sb_k, sb_v);
    a_end = (a0 + wa > a_end) ? a0 + wa : a_end;
    b_end = (b0 + wb > b_end) ? b0 + wb : b_end;
    __syncthreads();
    // This thread's outputs: positions p .. p + kMergeItems - 1, of which
    // those before p0 (first tile of a range only) belong to another range.
    const uint64_t p = g0 + static_cast<uint64_t>(tid) * kMergeItems;
    const uint32_t skip =
        p < p0 ? ((p0 - p) < kMergeItems ? static_cast<uint32_t>(p0 - p) : kMergeItems) : 0u;
    const uint32_t dt = p < p0 ? 0u : ((p - p0) < n ? static_cast<uint32_t>(p - p0) : n);
    uint32_t ia = ring_merge_path(sa_k, a0, wa, sb_k, b0, wb, dt, kMask);
    uint32_t ib = dt - ia;
    uint32_t rk[kMergeItems], rv[kMergeItems];
#pragma unroll
    for (int k = 0; k < kMergeItems; ++k) {
      rk[k] = 0u;
      rv[k] = 0u;
      if (static_cast<uint32_t>(k) >= skip && p + k < tile_end) {
        const uint32_t ka = ia < wa ? sa_k[(a0 + ia) & kMask] : 0u;
        const uint32_t kb = ib < wb ? sb_k[(b0 + ib) & kMask] : 0u;
        const bool take_a = ia < wa && (ib >= wb || (ka >> 1) <= (kb >> 1));
        rk[k] = take_a ? ka : kb;
        rv[k] = take_a ? sa_v[(a0 + ia) & kMask] : sb_v[(b0 + ib) & kMask];
        ia += take_a ? 1u : 0u;
        ib += take_a ? 0u : 1u;
      }
    }
    if (tid == kThreads - 1) s_split = ring_merge_path(sa_k, a0, wa, sb_k, b0, wb, n, kMask);
    if (skip == 0 && p + kMergeItems <= tile_end) {
#pragma unroll
      for (int k = 0; k < kMergeItems; k += 4) {
        *reinterpret_cast<uint4*>(m.out_kv + p + k) = make_uint4(rk[k], rk[k + 1], rk[k + 2], rk[k + 3]);
        *reinterpret_cast<uint4*>(m.out_val + p + k) = make_uint4(rv[k], rv[k + 1], rv[k + 2], rv[k + 3]);
      }
    } else {
#pragma unroll
      for (int k = 0; k < kMergeItems; ++k) {
        if (static_cast<uint32_t>(k) >= skip && p + k < tile_end) {
          m.out_kv[p + k] = rk[k];
          m.out_val[p + k] = rv[k];
        }
      }
    }
#pragma unroll
    for (int k = 0; k < kMergeItems; ++k)
      if (static_cast<uint32_t>(k) >= skip && p + k < tile_end)
        put_fence(m.out_fence, total, p + k, rk[k]);
    __syncthreads();
    const uint32_t la = s_split;
    a0 += la;
    b0 += n - la;
  }
}

// ------------------------------------------------------------ coalescer
// Step a1 for the coalescer: encodes n operations as key variables (status
// 0 for a deletion, whose value is 0) into staging[at .. at + n).  Element i
// deletes when all_delete is set or is_delete[i] != 0.
__global__ __launch_bounds__(kThreads) void k_stage(const uint32_t* keys, const uint32_t* vals,
                                                    const uint8_t* is_delete, int all_delete,
                                                    uint32_t n, uint32_t* stage_kv,
                                                    uint32_t* stage_val, uint32_t at) {
  const uint32_t i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const bool del = all_delete != 0 || (is_delete != nullptr && is_delete[i] != 0);
  stage_kv[at + i] = (keys[i] << 1) | (del ? 0u : 1u);
  stage_val[at + i] = del ? 0u : vals[i];
}

__global__ __launch_bounds__(kThreads) void k_check_keys(const uint32_t* keys, uint32_t n,
                                                         uint32_t limit_bits, int encoded,
                                                         uint32_t* err) {
  const uint32_t i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const uint32_t k = encoded ? (keys[i] >> 1) : keys[i];
  if ((k >> limit_bits) != 0u) atomicOr(err, 1u);
}

__global__ __launch_bounds__(kThreads) void k_fill_runs(uint32_t* a_kv, uint32_t* a_val,
                                                        uint32_t* b_kv, uint32_t* b_val,
                                                        uint32_t n) {
  const uint32_t i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  a_kv[i] = ((2u * i) << 1) | 1u;
  a_val[i] = i;
  b_kv[i] = ((2u * i + 1u) << 1) | 1u;
  b_val[i] = i;
}

// ------------------------------------------------------------ queries
__global__ __launch_bounds__(kQueryThreads) void k_lookup(LevelSet lv, const uint32_t* q,
                                                          uint32_t nq, uint32_t* out_val,
                                                          uint8_t* out_found) {
  // Every lane stays until the wave is done: the searches are wave-wide.
  const uint32_t i = blockIdx.x * kQueryThreads + threadIdx.x;
  const bool active = i < nq;
  const uint32_t k = active ? q[i] : 0u;
  uint32_t v = 0u;
  uint8_t f = 0;
  bool done = !active;
  for (int l = 0; l < lv.count; ++l) {
    if (ballot(!done) == 0) break;
    const uint32_t* kv = lv.kv[l];
    const uint32_t n = lv.len[l];
    const uint32_t p = octet_bound<false>(kv, lv.fence[l], n, k);
    if (!done && p < n) {
      const uint32_t x = kv[p];
      if ((x >> 1) == k) {
        if (x & 1u) {
          v = lv.val[l][p];
          f = 1;
        }
        done = true;  // the newest instance decides, tombstone or not
      }
    }
  }
  if (active) {
    out_val[i] = v;
    out_found[i] = f;
  }
}

constexpr uint32_t kNoKey = 0xFFFFFFFFu;  // above every original key (< 2^31)

// First index in (c, e) whose original key differs from k, where kv[c] has
// key k: one probe for the common run of length 1, then a galloping search,
// so long runs of one key (hot keys, padded batches) cost O(log run).
__device__ __forceinline__ uint32_t skip_run(const uint32_t* kv, uint32_t c, uint32_t e,
                                             uint32_t k) {
  uint32_t lo = c + 1;  // kv[lo - 1] has key k
  if (lo >= e || (kv[lo] >> 1) != k) return lo;
  uint32_t step = 1;
  // Invariant: kv[lo] has key k.
  while (lo + step < e && (kv[lo + step] >> 1) == k) {
    lo += step;
    step <<= 1;
  }
  uint32_t hi = (lo + step < e) ? lo + step : e;  // key(hi) > k, or hi == e
  while (hi - lo > 1) {
    const uint32_t mid = lo + ((hi - lo) >> 1);
    if ((kv[mid] >> 1) == k) lo = mid;
    else hi = mid;
  }
  return hi;
}

// The candidates of a query [k1, k2] in the first kW occupied levels run
// from lower_bound(k1) (one fence-tree descent per level) up to the first
// key above k2, which the walks find by reading on (they read every
// candidate anyway), so no second descent is made.  The cursors are kept in
// registers: level l's goes to slot l through a compare per slot, so no
// register array is indexed at run time (which would put the walk state in
// scratch memory).  A slot past the occupied levels stays at 0 of a level of
// length 0 (lv.len is zero there).
// The descents are wave-wide (octet_bound): every lane of the wave calls
// this; for k1 > k2 the walks then find no candidate (every key from the
// lower bound on is above k2).
template <int kW>
__device__ __forceinline__ void level_bounds(const LevelSet& lv, uint32_t k1,
                                             uint32_t (&cur)[kW]) {
#pragma unroll
  for (int q = 0; q < kW; ++q) cur[q] = 0u;
  for (int l = 0; l < lv.count && l < kW; ++l) {
    const uint32_t lo = octet_bound<false>(lv.kv[l], lv.fence[l], lv.len[l], k1);
#pragma unroll
    for (int q = 0; q < kW; ++q) {
      if (q == l) cur[q] = lo;
    }
  }
}

// Key of the candidate at cur in a level, or kNoKey past the level's end or
// past k2.
__device__ __forceinline__ uint32_t cand_key(const uint32_t* kv, uint32_t cur, uint32_t end,
                                             uint32_t k2) {
  if (cur >= end) return kNoKey;
  const uint32_t key = kv[cur] >> 1;
  return key <= k2 ? key : kNoKey;
}

// One level: the live keys among the candidates of [k1, k2], from p =
// lower_bound(k1) (so the candidate at p starts a key run) to the first key
// above k2 or n, whichever comes first, which goes to *e.  The first element of
// every key run is that key's newest instance, so the candidates are
// scanned in order, 16 at a time (their loads independent); a chunk that
// holds no run start lies inside one long run, which is skipped by
// galloping.
__device__ __forceinline__ uint32_t count_run_starts(const uint32_t* kv, uint32_t p, uint32_t n,
                                                     uint32_t k2, uint32_t* e) {
  uint32_t count = 0, prev = kNoKey;
  while (p < n) {
    const uint32_t m = (n - p) < 16u ? (n - p) : 16u;
    uint32_t x[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      x[i] = static_cast<uint32_t>(i) < m ? kv[p + i] : 0u;
    }
    bool any_start = false;
    uint32_t stop = m;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      if (static_cast<uint32_t>(i) < stop) {
        const uint32_t key = x[i] >> 1;
        if (key > k2) {
          stop = static_cast<uint32_t>(i);
        } else {
          const bool start = key != prev;
          if (start && (x[i] & 1u)) ++count;
          any_start |= start;
          prev = key;
        }
      }
    }
    if (stop < m) {
      p += stop;
      break;
    }
    p = any_start ? p + m : skip_run(kv, p + m - 1, n, prev);
  }
  *e = p < n ? p : n;
  return count;
}

// Walk the candidates of all occupied levels in key order.  For each
// distinct key the element met first is the newest instance (smaller levels
// are newer, and inside a level a key's run starts with its newest
// element); it counts when it is a regular element.  At most kW occupied
// levels, the walk state in registers (loops unrolled over the kW slots).
template <int kW>
__device__ __forceinline__ uint32_t range_walk(const LevelSet& lv, uint32_t (&cur)[kW],
                                               uint32_t k2) {
  uint32_t ck[kW];
#pragma unroll
  for (int l = 0; l < kW; ++l) ck[l] = cand_key(lv.kv[l], cur[l], lv.len[l], k2);
  uint32_t count = 0;
  for (;;) {
    uint32_t mk = kNoKey;
#pragma unroll
    for (int l = 0; l < kW; ++l) mk = ck[l] < mk ? ck[l] : mk;
    if (mk == kNoKey) break;
    bool newest = true;
#pragma unroll
    for (int l = 0; l < kW; ++l) {
      if (ck[l] == mk) {
        const uint32_t* kv = lv.kv[l];
        if (newest) count += kv[cur[l]] & 1u;
        newest = false;
        cur[l] = skip_run(kv, cur[l], lv.len[l], mk);
        ck[l] = cand_key(kv, cur[l], lv.len[l], k2);
      }
    }
  }
  return count;
}

// Count pass.  With one level and bounds non-null, each query's candidate
// bounds [lower_bound(lo), upper_bound(hi)) are also stored (two words per
// query) for the emission pass.
template <int kW>
__global__ __launch_bounds__(kQueryThreads) void k_count(LevelSet lv, const uint32_t* lo,
                                                         const uint32_t* hi, uint32_t nq,
                                                         uint32_t* counts, uint64_t* scan_status,
                                                         uint64_t scan_words, uint32_t* bounds) {
  const uint64_t gi = static_cast<uint64_t>(blockIdx.x) * kQueryThreads + threadIdx.x;
  if (scan_status != nullptr) {
    for (uint64_t w = gi; w < scan_words; w += static_cast<uint64_t>(gridDim.x) * kQueryThreads)
      scan_status[w] = 0ull;
  }
  // Every lane takes part in the wave-wide descents; lanes without a query
  // search the empty range [1, 0].  Several levels: with bounds non-null,
  // each query's per-level cursors (lower bounds) are stored level-major
  // (word l * nq + query) for the emission pass.
  const bool active = gi < nq;
  const uint32_t k1 = active ? lo[gi] : 1u, k2 = active ? hi[gi] : 0u;
  if constexpr (kW == 1) {
    // Both bounds by descents, so the scan reads only the candidates.
    uint32_t p = octet_bound<false>(lv.kv[0], lv.fence[0], lv.len[0], k1);
    uint32_t e = octet_bound<true>(lv.kv[0], lv.fence[0], lv.len[0], k2);
    if (!active) return;
    uint32_t c = 0;
    if (k1 <= k2) c = count_run_starts(lv.kv[0], p, e, k2, &e);
    else p = e = 0;
    if (bounds != nullptr) reinterpret_cast<uint2*>(bounds)[gi] = make_uint2(p, e);
    counts[gi] = c;
  } else {
    uint32_t cur[kW];
    level_bounds<kW>(lv, k1, cur);
    if (bounds != nullptr && active) {
#pragma unroll
      for (int q = 0; q < kW; ++q)
        if (q < lv.count) bounds[static_cast<size_t>(q) * nq + gi] = cur[q];
    }
    const uint32_t c = range_walk<kW>(lv, cur, k2);
    if (active) counts[gi] = c;
  }
}

// Resumable form of the several-level range_walk for the emission pass:
// the walk of one query keeps its cursors between calls, and each call
// emits the pairs whose output positions fall in [pos, lim), writing pair
// position x at sk[x - c0] / sv[x - c0].  Returns the next position.  The
// pairs and their order are range_walk's.
template <int kW>
struct WalkMany {
  uint32_t cur[kW], ck[kW];
  uint32_t k2;
};

// The cursors come from the count pass (cursors non-null: word l * nq + i
// for query i, read only when `use`) or from wave-wide descents (every lane
// of the wave calls it then).
template <int kW, bool kSearch>
__device__ __forceinline__ void walk_init(const LevelSet& lv, uint32_t k1, uint32_t k2,
                                          const uint32_t* cursors, uint32_t nq, uint32_t i,
                                          bool use, WalkMany<kW>& w) {
  w.k2 = k2;
  if constexpr (!kSearch) {
#pragma unroll
    for (int q = 0; q < kW; ++q)
      w.cur[q] = (use && q < lv.count) ? cursors[static_cast<size_t>(q) * nq + i] : 0u;
  } else {
    level_bounds<kW>(lv, k1, w.cur);
  }
#pragma unroll
  for (int l = 0; l < kW; ++l) w.ck[l] = cand_key(lv.kv[l], w.cur[l], lv.len[l], k2);
}

// Several levels: the k-way walk over the level runs in key order; the
// element met first for each key (smallest level first) is its newest
// instance, emitted when regular.
template <int kW>
__device__ __forceinline__ uint64_t walk_emit(const LevelSet& lv, WalkMany<kW>& w, uint64_t pos,
                                              uint64_t lim, uint64_t c0, uint32_t* sk,
                                              uint32_t* sv) {
  for (;;) {
    uint32_t mk = kNoKey;
#pragma unroll
    for (int l = 0; l < kW; ++l) mk = w.ck[l] < mk ? w.ck[l] : mk;
    if (mk == kNoKey) break;
    // The newest instance: the first level holding the key.
    uint32_t x = 0, v = 0;
    bool newest = true;
#pragma unroll
    for (int l = 0; l < kW; ++l) {
      if (newest && w.ck[l] == mk) {
        x = lv.kv[l][w.cur[l]];
        v = lv.val[l][w.cur[l]];
        newest = false;
      }
    }
    if (x & 1u) {
      if (pos >= lim) break;  // this key is emitted by a later call
      sk[pos - c0] = mk;
      sv[pos - c0] = v;
      ++pos;
    }
#pragma unroll
    for (int l = 0; l < kW; ++l) {
      if (w.ck[l] == mk) {
        w.cur[l] = skip_run(lv.kv[l], w.cur[l], lv.len[l], mk);
        w.ck[l] = cand_key(lv.kv[l], w.cur[l], lv.len[l], w.k2);
      }
    }
  }
  return pos;
}

// Stage 3 of sec. IV-C / IV-D over several levels, with coalesced writes.
// The pairs of a wave's 64 consecutive queries form one contiguous span of
// the output, which the wave produces in chunks of kEmitChunk pairs: every query emits the pairs
// that fall in the chunk into the wave's LDS buffer (its walk resumes where
// the previous chunk stopped it), then the wave copies the chunk out with
// consecutive lanes on consecutive addresses.  A query whose pairs would end
// beyond cap writes nothing (the caller sees offsets[q + 1] > cap); the other
// checks only guard against offsets corrupted by a timed-out scan.
constexpr uint32_t kEmitChunk = 512;
constexpr int kQueryWaves = kQueryThreads / 64;

template <int kW, bool kSearch>
__global__ __launch_bounds__(kQueryThreads) void k_range_emit(LevelSet lv, const uint32_t* lo,
                                                              const uint32_t* hi, uint32_t nq,
                                                              const uint64_t* offsets,
                                                              const uint32_t* cursors,
                                                              uint32_t* out_keys,
                                                              uint32_t* out_vals, uint64_t cap) {
  __shared__ uint32_t sk[kQueryWaves][kEmitChunk], sv[kQueryWaves][kEmitChunk];
  __shared__ uint32_t s_rounds[kQueryWaves];
  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t i = blockIdx.x * kQueryThreads + tid;
  const uint32_t q0 = blockIdx.x * kQueryThreads + wave * 64;
  const uint32_t qa = q0 < nq ? q0 : nq, qb = q0 + 64 < nq ? q0 + 64 : nq;
  const uint64_t base = offsets[qa], span_end = offsets[qb], all = offsets[nq];
  const bool active = i < nq;
  const uint64_t o = active ? offsets[i] : 0, e = active ? offsets[i + 1] : 0;
  const bool fits = active && e >= o && o >= base && e <= span_end && e <= all && e <= cap;
  // The writable part of the span ends where the first query that does not
  // fit begins (offsets are non-decreasing).
  uint64_t stop = (active && !fits) ? o : ~0ull;
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) {
    const uint64_t y = __shfl_xor(stop, d, 64);
    stop = y < stop ? y : stop;
  }
  const uint64_t copy_end = stop < span_end ? stop : span_end;
  const uint32_t rounds =
      copy_end > base ? static_cast<uint32_t>((copy_end - base + kEmitChunk - 1) / kEmitChunk) : 0u;
  if (lane == 0) s_rounds[wave] = rounds;
  static_assert(kW > 1, "one level: k_range_emit_one");
  WalkMany<kW> w;
  // Stored cursors (only the queries that emit read theirs), or wave-wide
  // descents by every lane.
  walk_init<kW, kSearch>(lv, fits ? lo[i] : 1u, fits ? hi[i] : 0u, cursors, nq, i, fits, w);
  __syncthreads();
  uint32_t R = 0;
#pragma unroll
  for (int x = 0; x < kQueryWaves; ++x) R = s_rounds[x] > R ? s_rounds[x] : R;
  uint64_t pos = o;
  for (uint32_t r = 0; r < R; ++r) {
    const uint64_t c0 = base + static_cast<uint64_t>(r) * kEmitChunk;
    const uint64_t c1 = c0 + kEmitChunk;
    if (fits && pos < e && pos < c1) pos = walk_emit(lv, w, pos, e < c1 ? e : c1, c0, sk[wave], sv[wave]);
    __syncthreads();
    for (uint32_t x = lane; x < kEmitChunk; x += 64) {
      const uint64_t g = c0 + x;
      if (g < copy_end) {
        out_keys[g] = sk[wave][x];
        out_vals[g] = sv[wave][x];
      }
    }
    __syncthreads();
  }
}

// Stage 3 of sec. IV-C / IV-D with one occupied level, a wave working on
// one query at a time: the 64 lanes read 64 consecutive candidates with one
// load, mark the regular run starts (a key that differs from the candidate
// before it; the first candidate, at a lower bound, always starts a run) and
// store them at the query's offset, ranked by a ballot, so every store
// instruction writes one contiguous piece of the output.  A chunk with no
// run start lies inside one long run, which is skipped by galloping.  The
// query is done once its pairs are written.
__device__ __forceinline__ void emit_run_starts(const uint32_t* kv, const uint32_t* vv, uint32_t c,
                                                uint32_t e, uint64_t w, uint64_t z, uint32_t x,
                                                uint32_t v, uint32_t lane, uint32_t* ok,
                                                uint32_t* ov) {
  uint32_t prev = kNoKey;
  for (;;) {
    const bool in = c + lane < e;
    const uint32_t key = x >> 1;
    uint32_t pk = __shfl_up(key, 1, 64);
    if (lane == 0) pk = prev;
    const bool start = in && key != pk;
    const bool keep = start && (x & 1u);
    const uint64_t km = ballot(keep);
    const uint64_t at = w + count_below(km);
    if (keep && at < z) {
      ok[at] = key;
      ov[at] = v;
    }
    w += static_cast<uint64_t>(__popcll(km));
    const uint32_t n = (e - c) < 64u ? (e - c) : 64u;
    prev = __shfl(key, static_cast<int>(n - 1), 64);
    const bool any_start = ballot(start) != 0;
    c += n;
    if (c >= e || w >= z) break;
    if (!any_start) {
      c = skip_run(kv, c - 1, e, prev);
      if (c >= e) break;
    }
    const bool in2 = c + lane < e;
    x = in2 ? kv[c + lane] : 0u;
    v = in2 ? vv[c + lane] : 0u;
  }
}

// The wave's 64 queries are taken kU at a time, their first chunks loaded
// together.  Each query's candidate bounds come from the count pass, or,
// with kSearch, are searched here (wave-wide descents; a separate
// instantiation, so that the usual form keeps its smaller register
// footprint).  A query
// whose pairs would end beyond cap writes nothing (the caller sees
// offsets[q + 1] > cap); writes stay inside [offsets[q], offsets[q + 1])
// even for offsets corrupted by a timed-out scan.
template <int kU, bool kSearch>
__global__ __launch_bounds__(kQueryThreads) void k_range_emit_one(
    LevelSet lv, const uint32_t* lo, const uint32_t* hi, uint32_t nq, const uint64_t* offsets,
    const uint32_t* bounds, uint32_t* out_keys, uint32_t* out_vals, uint64_t cap) {
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t i = blockIdx.x * kQueryThreads + threadIdx.x;
  const uint32_t* kv = lv.kv[0];
  const uint32_t* vv = lv.val[0];
  const uint32_t len = lv.len[0];
  uint32_t p = 0, e = 0;
  uint64_t o = 0, z = 0;
  bool emit = false;
  if (i < nq) {
    const uint64_t a = offsets[i], b = offsets[i + 1];
    if (b > a && b <= offsets[nq] && b <= cap) {
      o = a;
      z = b;
      emit = true;
    }
  }
  if constexpr (!kSearch) {
    if (emit) {
      const uint2 pe = reinterpret_cast<const uint2*>(bounds)[i];
      p = pe.x;
      e = pe.y;
    }
  } else {
    // Wave-wide descents: every lane searches (an empty range if it emits
    // nothing).
    const uint32_t k1 = emit ? lo[i] : 1u, k2 = emit ? hi[i] : 0u;
    p = octet_bound<false>(kv, lv.fence[0], len, k1);
    e = octet_bound<true>(kv, lv.fence[0], len, k2);
    if (!emit || k1 > k2) p = e = 0;
  }
  e = e < len ? e : len;
  p = p < e ? p : e;
  // Every lane stays to the end: the loop below is uniform over the wave.
  for (uint32_t q0 = 0; q0 < 64; q0 += kU) {
    uint32_t qp[kU], qe[kU], x[kU], v[kU];
    uint64_t qo[kU], qz[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int src = static_cast<int>(q0) + u;
      qp[u] = __shfl(p, src, 64);
      qe[u] = __shfl(e, src, 64);
      qo[u] = __shfl(o, src, 64);
      qz[u] = __shfl(z, src, 64);
      const uint32_t at = qp[u] + lane;
      const bool in = at < qe[u];
      x[u] = in ? kv[at] : 0u;
      v[u] = in ? vv[at] : 0u;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u)
      if (qp[u] < qe[u])
        emit_run_starts(kv, vv, qp[u], qe[u], qo[u], qz[u], x[u], v[u], lane, out_keys, out_vals);
  }
}

// ------------------------------------------------------------ scan
constexpr uint64_t kFlagAgg64 = 1ull << 62;
constexpr uint64_t kFlagInc64 = 2ull << 62;
constexpr uint64_t kSumMask64 = (1ull << 62) - 1;

// status[0] is the dynamic tile counter, status[1 + t] tile t's look-back
// word; all cleared beforehand by k_count.
__global__ __launch_bounds__(kThreads) void k_scan(const uint32_t* counts, uint32_t nq,
                                                   uint64_t* offsets, uint64_t* status,
                                                   uint32_t* fault) {
  __shared__ uint64_t s_w[kWaves];
  __shared__ uint32_t s_tile;
  __shared__ uint64_t s_prefix;
  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) s_tile = static_cast<uint32_t>(atomicAdd(reinterpret_cast<unsigned long long*>(status), 1ull));
  __syncthreads();
  const uint32_t tile = s_tile;
  const uint64_t base = static_cast<uint64_t>(tile) * kScanTile + static_cast<uint64_t>(tid) * kScanItems;
  uint32_t v[kScanItems];
  uint64_t tsum = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = (base + k < nq) ? counts[base + k] : 0u;
    tsum += v[k];
  }
  const uint64_t winc = wave_incl_scan64(tsum, lane);
  if (lane == 63) s_w[wave] = winc;
  __syncthreads();
  uint64_t wpre = 0, tile_total = 0;
  for (uint32_t w = 0; w < kWaves; ++w) {
    if (w < wave) wpre += s_w[w];
    tile_total += s_w[w];
  }
  const uint64_t texcl = wpre + winc - tsum;

  if (wave == 0) {
    uint64_t excl = 0;
    if (tile == 0) {
      if (lane == 0) st_dev64(&status[1], kFlagInc64 | tile_total);
    } else {
      if (lane == 0) st_dev64(&status[1 + tile], kFlagAgg64 | tile_total);
      int64_t j = static_cast<int64_t>(tile) - 1;
      uint32_t spins = 0;
      for (;;) {
        const int64_t idx = j - static_cast<int64_t>(lane);
        const uint64_t w = idx >= 0 ? ld_dev64(&status[1 + idx]) : kFlagInc64;
        const uint64_t f = w & ~kSumMask64;
        const uint64_t nr = ballot(f == 0), inc = ballot(f == kFlagInc64);
        const uint32_t first_nr = nr ? static_cast<uint32_t>(__builtin_ctzll(nr)) : 64u;
        const uint32_t first_inc = inc ? static_cast<uint32_t>(__builtin_ctzll(inc)) : 64u;
        if (first_inc < first_nr) {
          excl += wave_sum64(lane <= first_inc ? (w & kSumMask64) : 0ull);
          break;
        }
        excl += wave_sum64(lane < first_nr ? (w & kSumMask64) : 0ull);
        j -= first_nr;
        if (first_nr == 0) {
          __builtin_amdgcn_s_sleep(1);
          if (++spins == kSpinLimit) {
            if (lane == 0) atomicOr(fault, kFaultTimeout);
            break;
          }
        }
      }
      if (lane == 0) st_dev64(&status[1 + tile], kFlagInc64 | (excl + tile_total));
    }
    if (lane == 0) s_prefix = excl;
  }
  __syncthreads();
  uint64_t run = s_prefix + texcl;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < nq) offsets[base + k] = run;
    run += v[k];
  }
  const uint64_t tiles = (static_cast<uint64_t>(nq) + kScanTile - 1) / kScanTile;
  if (tile == tiles - 1 && tid == kThreads - 1) offsets[nq] = s_prefix + tile_total;
}

// ------------------------------------------------------------ order queries
constexpr uint32_t kMaxKey = 0x7FFFFFFFu;  // largest encodable original key

// Successor: walk the level runs that start at upper_bound(q) in key order
// (as range_walk does); the first key whose newest instance is a regular
// element is the answer.
__global__ __launch_bounds__(kQueryThreads) void k_successor(LevelSet lv, const uint32_t* q,
                                                             uint32_t nq, uint32_t* out_key,
                                                             uint32_t* out_val,
                                                             uint8_t* out_found) {
  const uint32_t i = blockIdx.x * kQueryThreads + threadIdx.x;
  const bool active = i < nq;
  const uint32_t k = active ? q[i] : 0u;
  uint32_t rk = 0u, rv = 0u;
  uint8_t f = 0;
  // The first descents are wave-wide: every lane makes them.
  uint32_t cur[kMaxLevels], ck[kMaxLevels];
  const int L = lv.count;
  for (int l = 0; l < L; ++l) {
    cur[l] = octet_bound<true>(lv.kv[l], lv.fence[l], lv.len[l], k);
    ck[l] = cur[l] < lv.len[l] ? (lv.kv[l][cur[l]] >> 1) : kNoKey;
  }
  if (!active) return;
  if (k < kMaxKey) {
    for (;;) {
      uint32_t mk = kNoKey;
      int mi = -1;
      for (int l = 0; l < L; ++l) {
        if (ck[l] < mk) {
          mk = ck[l];
          mi = l;
        }
      }
      if (mi < 0) break;
      if (lv.kv[mi][cur[mi]] & 1u) {
        rk = mk;
        rv = lv.val[mi][cur[mi]];
        f = 1;
        break;
      }
      for (int l = mi; l < L; ++l) {
        if (ck[l] == mk) {
          cur[l] = skip_run(lv.kv[l], cur[l], lv.len[l], mk);
          ck[l] = cur[l] < lv.len[l] ? (lv.kv[l][cur[l]] >> 1) : kNoKey;
        }
      }
    }
  }
  out_key[i] = rk;
  out_val[i] = rv;
  out_found[i] = f;
}

// Predecessor: the mirror walk, downwards from lower_bound(q).  For the
// largest remaining key, the newest instance is the first element of its run
// in the smallest level holding it; a tombstone there discards the key, and
// every level then drops its run of that key.
__global__ __launch_bounds__(kQueryThreads) void k_predecessor(LevelSet lv, const uint32_t* q,
                                                               uint32_t nq, uint32_t* out_key,
                                                               uint32_t* out_val,
                                                               uint8_t* out_found) {
  const uint32_t i = blockIdx.x * kQueryThreads + threadIdx.x;
  const bool active = i < nq;
  const uint32_t k = active ? q[i] : 0u;
  uint32_t rk = 0u, rv = 0u;
  uint8_t f = 0;
  // The first descents are wave-wide: every lane makes them.
  uint32_t e[kMaxLevels], ck[kMaxLevels];  // ck = key just below e, or kNoKey
  const int L = lv.count;
  for (int l = 0; l < L; ++l) {
    e[l] = octet_bound<false>(lv.kv[l], lv.fence[l], lv.len[l], k);
    ck[l] = e[l] > 0u ? (lv.kv[l][e[l] - 1u] >> 1) : kNoKey;
  }
  if (!active) return;
  if (k > 0u) {
    for (;;) {
      uint32_t mk = 0u;
      int mi = -1;
      for (int l = 0; l < L; ++l) {
        if (ck[l] != kNoKey && (mi < 0 || ck[l] > mk)) {
          mk = ck[l];
          mi = l;
        }
      }
      if (mi < 0) break;
      bool done = false;
      for (int l = mi; l < L; ++l) {
        if (ck[l] != mk) continue;
        // The run of mk ends at e[l] - 1, so the bound over the whole level
        // (the fence tree's layout is that of the whole level) is its start.
        const uint32_t s = fenced_bound(lv.kv[l], lv.fence[l], lv.len[l], mk, false);
        if (l == mi && (lv.kv[l][s] & 1u)) {
          rk = mk;
          rv = lv.val[l][s];
          f = 1;
          done = true;
          break;
        }
        e[l] = s;
        ck[l] = s > 0u ? (lv.kv[l][s - 1u] >> 1) : kNoKey;
      }
      if (done) break;
    }
  }
  out_key[i] = rk;
  out_val[i] = rv;
  out_found[i] = f;
}

// ------------------------------------------------------------ cleanup
// Stages 2-5 of the bulk cleanup of sec. IV-D over the merged list (stage 1
// is a chain of ordinary merges).  A tile is kThreads x kCleanItems
// consecutive elements, each thread holding kCleanItems consecutive ones.
constexpr int kCleanItems = 8;
constexpr uint32_t kCleanTile = kThreads * kCleanItems;

// Valid flags of the thread's elements [e0, e0 + kCleanItems): the first
// element of a key run, when regular (stage 2: everything else is stale).
__device__ __forceinline__ uint32_t clean_flags(const uint32_t* kv, uint32_t n, uint32_t e0,
                                                uint32_t (&x)[kCleanItems]) {
  uint32_t prev = (e0 > 0u && e0 < n) ? (kv[e0 - 1u] >> 1) : kNoKey;
  uint32_t mask = 0u;
#pragma unroll
  for (int j = 0; j < kCleanItems; ++j) {
    const uint32_t e = e0 + j;
    x[j] = e < n ? kv[e] : 0u;
    if (e < n && (x[j] & 1u) && (x[j] >> 1) != prev) mask |= 1u << j;
    prev = x[j] >> 1;
  }
  return mask;
}

__global__ __launch_bounds__(kThreads) void k_clean_count(const uint32_t* kv, uint32_t n,
                                                          uint32_t* tile_cnt,
                                                          uint64_t* scan_status,
                                                          uint64_t scan_words) {
  __shared__ uint32_t tmp[kWaves];
  const uint32_t tid = threadIdx.x;
  const uint64_t gi = static_cast<uint64_t>(blockIdx.x) * kThreads + tid;
  for (uint64_t w = gi; w < scan_words; w += static_cast<uint64_t>(gridDim.x) * kThreads)
    scan_status[w] = 0ull;
  const uint32_t e0 = blockIdx.x * kCleanTile + tid * kCleanItems;
  uint32_t x[kCleanItems];
  const uint32_t c = __popc(clean_flags(kv, n, e0, x));
  const uint32_t pre = block_excl_scan(c, tmp);
  if (tid == kThreads - 1) tile_cnt[blockIdx.x] = pre + c;
}

// Position p of the redistributed list -> (level slot, index in the level).
__device__ __forceinline__ int dst_level(const LevelDst& d, uint64_t p, int l) {
  while (l + 1 < d.count && d.start[l + 1] <= p) ++l;
  return l;
}

__device__ __forceinline__ void dst_write(const LevelDst& d, int l, uint64_t p, uint32_t x,
                                          uint32_t v) {
  const uint64_t o = p - d.start[l];
  d.kv[l][o] = x;
  d.val[l][o] = v;
  put_fence(d.fence[l], d.len[l], o, x);
}

__global__ __launch_bounds__(kThreads) void k_clean_scatter(const uint32_t* kv,
                                                            const uint32_t* val, uint32_t n,
                                                            const uint64_t* tile_off,
                                                            LevelDst d) {
  __shared__ uint32_t tmp[kWaves];
  const uint32_t tid = threadIdx.x;
  const uint32_t e0 = blockIdx.x * kCleanTile + tid * kCleanItems;
  uint32_t x[kCleanItems];
  const uint32_t mask = clean_flags(kv, n, e0, x);
  const uint32_t pre = block_excl_scan(__popc(mask), tmp);
  if (mask == 0u) return;
  uint64_t p = tile_off[blockIdx.x] + pre;
  int l = dst_level(d, p, 0);
#pragma unroll
  for (int j = 0; j < kCleanItems; ++j) {
    if (mask & (1u << j)) {
      l = dst_level(d, p, l);
      dst_write(d, l, p, x[j], val[e0 + j]);
      ++p;
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_clean_pad(LevelDst d, uint64_t v, uint64_t total) {
  const uint64_t p = v + static_cast<uint64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (p >= total) return;
  dst_write(d, dst_level(d, p, 0), p, kPlaceboKv, 0u);
}

// Writes one zero word: clears a range call's total where a memset node on
// the stream is not wanted.
__global__ void k_zero_u64(uint64_t* p) { *p = 0ull; }

inline unsigned grid_for(uint64_t n, uint64_t per) { return static_cast<unsigned>((n + per - 1) / per); }

template <typename Kernel, typename... Args>
hipError_t launch(Kernel k, unsigned grid, unsigned block, hipStream_t s, const KTimer* t,
                  Args... args) {
  if (t != nullptr && t->start != nullptr)
    hipExtLaunchKernelGGL(k, dim3(grid), dim3(block), 0, s, t->start, t->stop, 0, args...);
  else
    k<<<grid, block, 0, s>>>(args...);
  return hipGetLastError();
}

}  // namespace

// ------------------------------------------------------------ fixed scratch
// Range scratch held in the code object (the per-query counts, then the
// scan's look-back words), for callers that cannot allocate.  Every device
// that loads the library holds its own copy until the process ends.  Host
// code must never pass `scratch` itself to a kernel: on the host the name
// stands for a host-side shadow, so kernels get the address that
// hipGetSymbolAddress returns for the current device.
constexpr uint64_t kFixedStatusWords = 1 + (kFixedMaxQueries + kScanTile - 1) / kScanTile;
constexpr uint64_t kFixedWords = kFixedMaxQueries / 2 + kFixedStatusWords;
static __device__ __align__(256) uint64_t scratch[kFixedWords];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_fixed_mu;
void* g_fixed_addr[kMaxDevices] = {};
}  // namespace

hipError_t fixed_scratch(FixedScratch* out) {
  out->counts = nullptr;
  out->status = nullptr;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_fixed_mu);
  if (g_fixed_addr[dev] == nullptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (p == nullptr) return hipErrorInvalidSymbol;
    g_fixed_addr[dev] = p;
  }
  uint64_t* base = static_cast<uint64_t*>(g_fixed_addr[dev]);
  out->counts = reinterpret_cast<uint32_t*>(base);
  out->status = base + kFixedMaxQueries / 2;
  return hipSuccess;
}

hipError_t launch_zero_u64(uint64_t* p, hipStream_t stream) {
  return launch(k_zero_u64, 1, 1, stream, nullptr, p);
}

// ------------------------------------------------------------ launchers
size_t sort_meta_words(uint32_t b) {
  const size_t ns = grid_for(b, kSortTile);
  return static_cast<size_t>(2) * kMaxPasses * kRadix + static_cast<size_t>(kMaxPasses) * ns * kRadix +
         kMaxPasses + 4 + kSortSlots * (ns * (kTopBuckets / 2) + kTopBuckets);
}

SortMeta sort_meta_carve(uint32_t* base, uint32_t b, int parity, int slot) {
  SortMeta m;
  const size_t ns = grid_for(b, kSortTile);
  m.num_sort_tiles = static_cast<uint32_t>(ns);
  m.hist = base;
  m.status = m.hist + static_cast<size_t>(2) * kMaxPasses * kRadix;
  m.tile_ctr = m.status + static_cast<size_t>(kMaxPasses) * ns * kRadix;
  m.err = m.tile_ctr + kMaxPasses;
  // Per slot: the group starts, then the bucket-size record (both 16-byte
  // aligned).
  uint32_t* slot_base =
      m.err + 4 + static_cast<size_t>(slot) * (ns * (kTopBuckets / 2) + kTopBuckets);
  m.tile_cnt = slot_base;
  m.bucket_n = slot_base + ns * (kTopBuckets / 2);
  m.parity = parity;
  return m;
}

int sort_kernel_count(const SortArgs& a) {
  if (a.path == kSortMsd) return 2;
  return 1 + a.passes;
}

// The number of 8-bit passes that sort a top-digit bucket: the key-variable
// bits below the top digit.
static int bucket_passes(const SortArgs& a) {
  return (sort_top_shift(a) - a.lo_bit + kRadixBits - 1) / kRadixBits;
}

hipError_t launch_scatter(const SortArgs& a, hipStream_t stream, const KTimer* t) {
  return launch(k_msd_scatter, a.meta.num_sort_tiles, kThreads, stream, t, a, sort_top_shift(a));
}

// The largest entry of a slot's bucket-size record into *out (one work-group).
__global__ __launch_bounds__(kThreads) void k_rec_max(const uint32_t* rec, uint32_t* out) {
  __shared__ uint32_t s_max[kWaves];
  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint4 r = reinterpret_cast<const uint4*>(rec)[tid];
  uint32_t x = max(max(r.x, r.y), max(r.z, r.w));
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = max(x, static_cast<uint32_t>(__shfl_xor(x, o, 64)));
  if (lane == 0) s_max[wave] = x;
  __syncthreads();
  if (tid == 0) {
    uint32_t mx = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) mx = max(mx, s_max[w]);
    *out = mx;
  }
}

hipError_t launch_rec_max(const uint32_t* rec, uint32_t* out, hipStream_t stream) {
  return launch(k_rec_max, 1, kThreads, stream, nullptr, rec, out);
}

// Arguments without a group (group == 0) sort the one batch of their slot,
// scattered from element 0 of tmp_kv[0].
SortArgs grouped(SortArgs a) {
  if (a.group == 0) {
    a.group = 1;
    a.grp_cnt[0] = a.meta.tile_cnt;
    a.grp_n[0] = a.meta.bucket_n;
    a.grp_off[0] = 0;
  }
  return a;
}

hipError_t launch_buckets(const SortArgs& a, hipStream_t stream, const KTimer* t) {
  return launch(k_local_sort, kTopBuckets, kThreads, stream, t, grouped(a), a.lo_bit,
                bucket_passes(a));
}

hipError_t launch_sort_step(const SortArgs& bk, const SortArgs& sc, hipStream_t stream,
                            const KTimer* t) {
  return launch(k_sort_step, sc.meta.num_sort_tiles + kTopBuckets, kThreads, stream, t,
                grouped(bk), bk.lo_bit, bucket_passes(bk), sc, sort_top_shift(sc));
}

hipError_t launch_sort(const SortArgs& a, hipStream_t stream, const KTimer* timers,
                       int* launched) {
  const uint32_t tiles = a.meta.num_sort_tiles;
  *launched = 0;
  if (a.path == kSortMsd && tiles <= static_cast<uint32_t>(kMsdMaxTiles)) {
    // Top digit: the highest 8 bits a key variable of this handle can have.
    hipError_t e = launch_scatter(a, stream, timers ? &timers[0] : nullptr);
    if (e != hipSuccess) return e;
    *launched = 1;
    e = launch_buckets(a, stream, timers ? &timers[1] : nullptr);
    if (e == hipSuccess) *launched = 2;
    return e;
  }
  const uint32_t hist_grid = tiles < static_cast<uint32_t>(kMaxHistBlocks) ? tiles : kMaxHistBlocks;
  hipError_t e = launch(k_sort_hist, hist_grid, kThreads, stream, timers ? &timers[0] : nullptr, a);
  if (e != hipSuccess) return e;
  *launched = 1;
  for (int p = 0; p < a.passes; ++p) {
    e = launch(k_sort_pass, tiles, kThreads, stream, timers ? &timers[1 + p] : nullptr, a, p);
    if (e != hipSuccess) return e;
    *launched += 1;
  }
  return hipSuccess;
}

template <int kItems>
hipError_t launch_merge_items(MergeArgs m, uint32_t max_blocks, hipStream_t stream,
                              const KTimer* t) {
  const uint64_t total = static_cast<uint64_t>(m.na) + m.nb;
  const uint64_t tile = static_cast<uint64_t>(kThreads) * kItems;
  const uint64_t tiles = (total + tile - 1) / tile;
  if (m.digit_mode) {
    // Work-groups over the digits: at most one per digit, and no more than
    // output tiles (a small merge takes a few work-groups of many digits).
    const uint64_t groups = tiles < kTopBuckets ? (tiles > 0 ? tiles : 1) : kTopBuckets;
    m.per_wg = static_cast<uint32_t>((kTopBuckets + groups - 1) / groups);
    return launch(k_merge<kItems>, grid_for(kTopBuckets, m.per_wg), kThreads, stream, t, m);
  }
  m.per_wg = static_cast<uint32_t>((tiles + max_blocks - 1) / max_blocks);
  return launch(k_merge<kItems>, grid_for(tiles, m.per_wg), kThreads, stream, t, m);
}

hipError_t launch_merge(const uint32_t* a_kv, const uint32_t* a_val, uint32_t na,
                        const uint32_t* b_kv, const uint32_t* b_val, uint32_t nb,
                        uint32_t* out_kv, uint32_t* out_val, uint32_t* out_fence, int variant,
                        hipStream_t stream, const KTimer* t, const MergeIndex* idx) {
  const uint64_t total = static_cast<uint64_t>(na) + nb;
  if (total == 0) return hipSuccess;
  if (variant < 0 || variant >= kMergeVariants) variant = kDefaultMergeVariant;
  MergeArgs m{};
  m.a_kv = a_kv;
  m.a_val = a_val;
  m.b_kv = b_kv;
  m.b_val = b_val;
  m.na = na;
  m.nb = nb;
  m.out_kv = out_kv;
  m.out_val = out_val;
  m.out_fence = out_fence;
  if (idx != nullptr && idx->a_dig != nullptr && idx->b_dig != nullptr) {
    m.a_dig = idx->a_dig;
    m.b_dig = idx->b_dig;
    m.out_dig = idx->out_dig;
    m.digit_mode = idx->by_digit;
  }
  const uint32_t blocks = static_cast<uint32_t>(kMergeBlocksOf[variant / 3]);
  switch (kMergeItemsOf[variant % 3]) {
    case 4: return launch_merge_items<4>(m, blocks, stream, t);
    case 16: return launch_merge_items<16>(m, blocks, stream, t);
    default: return launch_merge_items<8>(m, blocks, stream, t);
  }
}

hipError_t launch_stage(const uint32_t* keys, const uint32_t* vals, const uint8_t* is_delete,
                        int all_delete, uint32_t n, uint32_t* stage_kv, uint32_t* stage_val,
                        uint32_t at, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  return launch(k_stage, grid_for(n, kThreads), kThreads, stream, nullptr, keys, vals, is_delete,
                all_delete, n, stage_kv, stage_val, at);
}

hipError_t launch_check_keys(const uint32_t* keys, uint32_t n, uint32_t limit_bits, int encoded,
                             uint32_t* err, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  return launch(k_check_keys, grid_for(n, kThreads), kThreads, stream, nullptr, keys, n,
                limit_bits, encoded, err);
}

hipError_t launch_fill_runs(uint32_t* a_kv, uint32_t* a_val, uint32_t* b_kv, uint32_t* b_val,
                            uint32_t n, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  return launch(k_fill_runs, grid_for(n, kThreads), kThreads, stream, nullptr, a_kv, a_val, b_kv,
                b_val, n);
}

hipError_t launch_lookup(const LevelSet& lv, const uint32_t* q, uint32_t nq, uint32_t* out_val,
                         uint8_t* out_found, hipStream_t stream, const KTimer* t) {
  if (nq == 0) return hipSuccess;
  return launch(k_lookup, grid_for(nq, kQueryThreads), kQueryThreads, stream, t, lv, q, nq,
                out_val, out_found);
}

hipError_t launch_count(const LevelSet& lv, const uint32_t* lo, const uint32_t* hi, uint32_t nq,
                        uint32_t* counts, uint64_t* scan_status, size_t scan_words,
                        uint32_t* bounds, hipStream_t stream, const KTimer* t) {
  if (nq == 0) return hipSuccess;
  auto k = lv.count <= 1 ? k_count<1> : lv.count <= 8 ? k_count<8> : lv.count <= 16 ? k_count<16>
                                                                           : k_count<kMaxLevels>;
  return launch(k, grid_for(nq, kQueryThreads), kQueryThreads, stream, t, lv, lo, hi, nq,
                counts, scan_status, static_cast<uint64_t>(scan_words), bounds);
}

size_t scan_status_words(uint32_t nq) { return 1 + grid_for(nq, kScanTile); }

hipError_t launch_scan(const uint32_t* counts, uint32_t nq, uint64_t* offsets,
                       uint64_t* scan_status, uint32_t* fault, hipStream_t stream,
                       const KTimer* t) {
  if (nq == 0) return hipSuccess;
  return launch(k_scan, grid_for(nq, kScanTile), kThreads, stream, t, counts, nq, offsets,
                scan_status, fault);
}

hipError_t launch_successor(const LevelSet& lv, const uint32_t* q, uint32_t nq, uint32_t* out_key,
                            uint32_t* out_val, uint8_t* out_found, hipStream_t stream,
                            const KTimer* t) {
  if (nq == 0) return hipSuccess;
  return launch(k_successor, grid_for(nq, kQueryThreads), kQueryThreads, stream, t, lv, q, nq,
                out_key, out_val, out_found);
}

hipError_t launch_predecessor(const LevelSet& lv, const uint32_t* q, uint32_t nq,
                              uint32_t* out_key, uint32_t* out_val, uint8_t* out_found,
                              hipStream_t stream, const KTimer* t) {
  if (nq == 0) return hipSuccess;
  return launch(k_predecessor, grid_for(nq, kQueryThreads), kQueryThreads, stream, t, lv, q, nq,
                out_key, out_val, out_found);
}

uint32_t clean_tiles(uint32_t n) { return grid_for(n, kCleanTile); }

hipError_t launch_clean_count(const uint32_t* kv, uint32_t n, uint32_t* tile_cnt,
                              uint64_t* scan_status, size_t scan_words, hipStream_t stream,
                              const KTimer* t) {
  if (n == 0) return hipSuccess;
  return launch(k_clean_count, clean_tiles(n), kThreads, stream, t, kv, n, tile_cnt, scan_status,
                static_cast<uint64_t>(scan_words));
}

hipError_t launch_clean_scatter(const uint32_t* kv, const uint32_t* val, uint32_t n,
                                const uint64_t* tile_off, const LevelDst& d, hipStream_t stream,
                                const KTimer* t) {
  if (n == 0 || d.count == 0) return hipSuccess;
  return launch(k_clean_scatter, clean_tiles(n), kThreads, stream, t, kv, val, n, tile_off, d);
}

hipError_t launch_clean_pad(const LevelDst& d, uint64_t v, uint64_t total, hipStream_t stream,
                            const KTimer* t) {
  if (total <= v || d.count == 0) return hipSuccess;
  return launch(k_clean_pad, grid_for(total - v, kThreads), kThreads, stream, t, d, v, total);
}

hipError_t launch_range_emit(const LevelSet& lv, const uint32_t* lo, const uint32_t* hi,
                             uint32_t nq, const uint64_t* offsets, const uint32_t* bounds,
                             uint32_t* out_keys, uint32_t* out_vals, uint64_t cap,
                             hipStream_t stream, const KTimer* t) {
  if (nq == 0) return hipSuccess;
  if (lv.count <= 1)
    return launch(bounds != nullptr ? k_range_emit_one<4, false> : k_range_emit_one<4, true>,
                  grid_for(nq, kQueryThreads), kQueryThreads, stream, t, lv, lo, hi, nq, offsets,
                  bounds, out_keys, out_vals, cap);
  // Emission from stored cursors and emission that searches (no scratch)
  // are separate instantiations, so that the first keeps a smaller register
  // footprint.
  auto k = bounds != nullptr
               ? (lv.count <= 8 ? k_range_emit<8, false> : lv.count <= 16 ? k_range_emit<16, false>
                                                                          : k_range_emit<kMaxLevels, false>)
               : (lv.count <= 8 ? k_range_emit<8, true> : lv.count <= 16 ? k_range_emit<16, true>
                                                                         : k_range_emit<kMaxLevels, true>);
  return launch(k, grid_for(nq, kQueryThreads), kQueryThreads, stream, t, lv, lo, hi, nq, offsets,
                bounds, out_keys, out_vals, cap);
}

}  // namespace lsm
