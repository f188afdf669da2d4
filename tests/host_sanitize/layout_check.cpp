// Checks the sort-scratch carving of the library (sort_meta_words and
// sort_meta_carve, copied out of the kernel source at build time) on the
// CPU: for batch sizes across tile edges, past the top-digit sort's 256
// tiles up to 2^20 (the carving is linear in the tile count), both
// histogram parities and every slot, the regions (digit histograms,
// look-back words, tile counters, error words, each slot's digit-group
// starts and bucket-size record) lie inside the allocation, do not overlap
// (the shared regions coincide across slots and parities, the per-slot ones
// are disjoint), and the per-slot regions start on 16-byte boundaries (the
// kernels read them with 16-byte loads).  Exit status 0 when all hold.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <vector>

#include "lsm_internal.h"

namespace lsm {
#include "layout_gen.inc"
}  // namespace lsm

namespace {

struct Region {
  uint64_t at, len;
  const char* what;
};

int g_fail = 0;
void fail(const char* msg, uint32_t b, const char* a, const char* c) {
  if (g_fail++ < 20) std::fprintf(stderr, "b %u: %s (%s, %s)\n", b, msg, a, c);
}

}  // namespace

int main() {
  using namespace lsm;
  const uint32_t sizes[] = {1, 2, 100, 2047, 2048, 2049, 4096, 65535, 65536, 65537, 1u << 17,
                            (1u << 17) + 1, 1u << 18, (1u << 19) - 1, 1u << 19, (1u << 19) + 1,
                            1u << 20};
  for (uint32_t b : sizes) {
    const size_t words = sort_meta_words(b);
    std::vector<uint32_t> mem(words + 4);  // + 4: base aligned to 16 bytes below
    uint32_t* base = mem.data();
    while (reinterpret_cast<uintptr_t>(base) % 16 != 0) ++base;
    std::vector<Region> all;
    SortMeta first{};
    for (int parity = 0; parity < 2; ++parity) {
      for (int slot = 0; slot < kSortSlots; ++slot) {
        const SortMeta m = sort_meta_carve(base, b, parity, slot);
        const uint64_t ns = m.num_sort_tiles;
        if (ns != (b + kSortTile - 1) / static_cast<uint64_t>(kSortTile))
          fail("tile count", b, "num_sort_tiles", "");
        if (parity == 0 && slot == 0) {
          first = m;
          all.push_back({static_cast<uint64_t>(m.hist - base), 2ull * kMaxPasses * kRadix, "hist"});
          all.push_back({static_cast<uint64_t>(m.status - base), kMaxPasses * ns * kRadix, "status"});
          all.push_back({static_cast<uint64_t>(m.tile_ctr - base), kMaxPasses, "tile_ctr"});
          all.push_back({static_cast<uint64_t>(m.err - base), 2, "err"});
        } else if (m.hist != first.hist || m.status != first.status ||
                   m.tile_ctr != first.tile_ctr || m.err != first.err) {
          fail("shared regions differ between slots or parities", b, "", "");
        }
        if (m.parity != parity) fail("parity not kept", b, "", "");
        if (parity == 0) {
          all.push_back({static_cast<uint64_t>(m.tile_cnt - base), ns * (kTopBuckets / 2),
                         "tile_cnt"});
          all.push_back({static_cast<uint64_t>(m.bucket_n - base), kTopBuckets, "bucket_n"});
          if (reinterpret_cast<uintptr_t>(m.tile_cnt) % 16 != 0)
            fail("group starts not 16-byte aligned", b, "tile_cnt", "");
          if (reinterpret_cast<uintptr_t>(m.bucket_n) % 16 != 0)
            fail("bucket record not 16-byte aligned", b, "bucket_n", "");
        } else {
          const SortMeta m0 = sort_meta_carve(base, b, 0, slot);
          if (m.tile_cnt != m0.tile_cnt || m.bucket_n != m0.bucket_n)
            fail("slot regions depend on the parity", b, "", "");
        }
      }
    }
    for (size_t i = 0; i < all.size(); ++i) {
      if (all[i].at + all[i].len > words) fail("region past the allocation", b, all[i].what, "");
      for (size_t j = i + 1; j < all.size(); ++j) {
        const bool apart = all[i].at + all[i].len <= all[j].at || all[j].at + all[j].len <= all[i].at;
        if (!apart) fail("regions overlap", b, all[i].what, all[j].what);
      }
    }
  }
  if (g_fail) {
    std::fprintf(stderr, "%d checks failed\n", g_fail);
    return 1;
  }
  std::printf("sort scratch layout: ok\n");
  return 0;
}
