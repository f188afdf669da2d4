// Drives the library's host code through its C ABI with the CPU stand-ins of
// stand_in.cpp (test infrastructure only; see tests/test_host_sanitize.py).
//
// Seeded random streams call every entry point for several batch sizes:
// direct insert, delete and mixed batches (full and partial), the coalescer
// (single-type and mixed submissions, flushes), every query form (lookup,
// count, range with too small and sufficient capacity, asynchronous and
// allocation-free ranges, successor, predecessor), cleanup, bulk insertion,
// the tuning and profiling calls, level views and copies, clear and
// destroy.  Allocation failures (the library's injection hook) and launch
// failures (the stand-in's) are injected at random points: a failed call
// must return LSM_ENOMEM or LSM_EHIP and leave r unchanged, and the next
// call must succeed.  Argument errors must return their documented status.
// The kernels are stand-ins, so no answer is checked here; what is checked
// is the host code's memory safety and status handling, under the
// sanitizers.  Exit status 0 when every check holds.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <thread>
#include <vector>

#include "lsm.h"

extern "C" void standin_fail_launch_after(long n);
extern "C" void standin_fail_alloc_after(long n);

namespace {

thread_local uint64_t g_state = 0x853C49E6748FEA9Bull;
uint64_t next_u64() {  // splitmix64
  uint64_t z = (g_state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
uint32_t below(uint32_t n) { return static_cast<uint32_t>(next_u64() % n); }

thread_local int g_fail = 0;
// Set in the threaded run: lsm_range_async_noalloc is left out there, since
// its calls share one scratch array per device (documented) and would race.
thread_local bool g_threaded = false;
thread_local long g_enomem = 0, g_ehip = 0;  // failed calls seen, by status
void check(bool ok, const char* what, int line) {
  if (!ok && g_fail++ < 20) std::fprintf(stderr, "check failed (line %d): %s\n", line, what);
}
#define CHECK(c) check((c), #c, __LINE__)

// A device buffer of exactly n elements (stand-in device memory is host
// memory, so the sanitizer sees its extent).
template <class T>
struct Buf {
  T* p = nullptr;
  size_t n = 0;
  explicit Buf(size_t count) : n(count) {
    void* v = nullptr;
    if (hipMalloc(&v, (count ? count : 1) * sizeof(T)) != hipSuccess) std::abort();
    p = static_cast<T*>(v);
  }
  ~Buf() { (void)hipFree(p); }
  Buf(const Buf&) = delete;
  Buf& operator=(const Buf&) = delete;
};

void fill_keys(Buf<uint32_t>& k, uint32_t n, uint32_t domain) {
  for (uint32_t i = 0; i < n; ++i) k.p[i] = below(domain);
}

// One operation of the random stream; returns its status.
lsm_status_t random_op(lsm_t h, uint32_t b, uint32_t domain, int op) {
  const uint32_t n = below(3) == 0 ? 1 + below(b) : b;
  switch (op) {
    case 0: case 1: case 2: {
      Buf<uint32_t> k(n), v(n);
      fill_keys(k, n, domain);
      return lsm_insert_batch(h, k.p, v.p, n);
    }
    case 3: {
      Buf<uint32_t> k(n);
      fill_keys(k, n, domain);
      return lsm_delete_batch(h, k.p, n);
    }
    case 4: {
      Buf<uint32_t> k(n), v(n);
      Buf<uint8_t> d(n);
      fill_keys(k, n, domain);
      for (uint32_t i = 0; i < n; ++i) d.p[i] = static_cast<uint8_t>(below(2));
      return lsm_update_batch(h, k.p, v.p, d.p, n);
    }
    case 5: {
      const uint32_t m = 1 + below(3 * b);
      Buf<uint32_t> k(m), v(m);
      fill_keys(k, m, domain);
      const int del = below(4) == 0;
      return lsm_submit(h, k.p, del ? nullptr : v.p, m, del);
    }
    case 6: {
      const uint32_t m = 1 + below(2 * b);
      Buf<uint32_t> k(m), v(m);
      Buf<uint8_t> d(m);
      fill_keys(k, m, domain);
      for (uint32_t i = 0; i < m; ++i) d.p[i] = static_cast<uint8_t>(below(2));
      return lsm_submit_mixed(h, k.p, v.p, d.p, m);
    }
    case 7:
      return lsm_flush(h);
    case 8: {
      const uint32_t nq = 1 + below(300);
      Buf<uint32_t> q(nq), v(nq);
      Buf<uint8_t> f(nq);
      fill_keys(q, nq, domain);
      return lsm_lookup(h, q.p, nq, v.p, f.p);
    }
    case 9: {
      const uint32_t nq = 1 + below(300);
      Buf<uint32_t> lo(nq), hi(nq), c(nq);
      fill_keys(lo, nq, domain);
      fill_keys(hi, nq, domain);
      return lsm_count(h, lo.p, hi.p, nq, c.p);
    }
    case 10: {
      const uint32_t nq = 1 + below(300);
      Buf<uint32_t> lo(nq), hi(nq);
      Buf<uint64_t> off(nq + 1);
      fill_keys(lo, nq, domain);
      fill_keys(hi, nq, domain);
      uint64_t total = 0;
      lsm_status_t s = lsm_range(h, lo.p, hi.p, nq, off.p, nullptr, nullptr, 0, &total);
      if (s == LSM_ECAPACITY || (s == LSM_OK && total == 0)) {
        Buf<uint32_t> ok(total), ov(total);
        s = lsm_range(h, lo.p, hi.p, nq, off.p, ok.p, ov.p, total, &total);
      }
      return s;
    }
    case 11: {
      const uint32_t nq = 1 + below(300);
      Buf<uint32_t> lo(nq), hi(nq), ok(4 * nq), ov(4 * nq);
      Buf<uint64_t> off(nq + 1);
      fill_keys(lo, nq, domain);
      fill_keys(hi, nq, domain);
      lsm_status_t s;
      if (below(2) || g_threaded) {
        s = lsm_range_async(h, lo.p, hi.p, nq, off.p, ok.p, ov.p, 4 * nq);
      } else {
        const uint32_t staged = lsm_pending(h);
        s = lsm_range_async_noalloc(h, lo.p, hi.p, nq, off.p, ok.p, ov.p, 4 * nq);
        if (s == LSM_ENOMEM && staged > 0 && lsm_pending(h) == staged) {
          // Documented refusal: inserting the staged elements first would
          // need memory.  The caller flushes (which may allocate) and retries.
          s = lsm_flush(h);
          if (s == LSM_OK) s = lsm_range_async_noalloc(h, lo.p, hi.p, nq, off.p, ok.p, ov.p, 4 * nq);
        }
      }
      if (s == LSM_OK) s = lsm_sync(h);
      return s;
    }
    case 12: {
      const uint32_t nq = 1 + below(300);
      Buf<uint32_t> q(nq), k(nq), v(nq);
      Buf<uint8_t> f(nq);
      fill_keys(q, nq, domain);
      return below(2) ? lsm_successor(h, q.p, nq, k.p, v.p, f.p)
                      : lsm_predecessor(h, q.p, nq, k.p, v.p, f.p);
    }
    case 13: {
      uint64_t valid = 0;
      return lsm_cleanup(h, &valid);
    }
    case 14: {
      const uint64_t m = 1 + below(5 * b);
      Buf<uint32_t> k(m), v(m);
      fill_keys(k, static_cast<uint32_t>(m), domain);
      return lsm_bulk_insert(h, k.p, v.p, m);
    }
    default: {
      // Tuning calls between operations (none changes any result).
      lsm_status_t s = lsm_set_grouping(h, static_cast<int>(below(6)));
      if (s == LSM_OK) s = lsm_set_sort_path(h, static_cast<int>(below(3)));
      if (s == LSM_OK) s = lsm_set_fusion(h, static_cast<int>(below(10)) - 1);
      if (s == LSM_OK) s = lsm_set_max_inflight(h, static_cast<int>(below(9)));
      return s;
    }
  }
}

void look_at_levels(lsm_t h) {
  const uint64_t r = lsm_num_batches(h);
  for (uint32_t i = 0; i < 40; ++i) {
    const uint32_t* kv = nullptr;
    const uint32_t* vals = nullptr;
    uint64_t len = 0;
    const lsm_status_t s = lsm_level_view(h, i, &kv, &vals, &len);
    const bool full = i < 64 && ((r >> i) & 1u);
    if (!full) continue;
    CHECK(s == LSM_OK && len == (static_cast<uint64_t>(lsm_batch_size(h)) << i));
    Buf<uint32_t> ck(len), cv(len);
    uint64_t len2 = 0;
    CHECK(lsm_level_copy(h, i, ck.p, cv.p, &len2) == LSM_OK && len2 == len);
  }
}

void run(uint32_t b, uint32_t flags, uint32_t domain, int steps) {
  lsm_t h = nullptr;
  CHECK(lsm_create(&h, b, flags, nullptr) == LSM_OK && h != nullptr);
  if (h == nullptr) return;
  CHECK(lsm_batch_size(h) == b);
  CHECK(lsm_profile_enable(h, static_cast<int>(below(2))) == LSM_OK);
  for (int s = 0; s < steps; ++s) {
    const int op = static_cast<int>(below(16));
    const uint64_t r0 = lsm_num_batches(h);
    const uint32_t staged0 = lsm_pending(h);
    const int inject = static_cast<int>(below(8));
    if (inject == 0) CHECK(lsm_fail_alloc_after(h, below(4)) == LSM_OK);
    if (inject == 1) standin_fail_launch_after(static_cast<long>(below(4)));
    const lsm_status_t st = random_op(h, b, domain, op);
    CHECK(lsm_fail_alloc_after(h, -1) == LSM_OK);
    standin_fail_launch_after(-1);
    if (st != LSM_OK) {
      if (!(st == LSM_ENOMEM || st == LSM_EHIP) || inject > 1)
        std::fprintf(stderr, "b %u step %d op %d: status %d without an injected failure (%d)\n",
                     b, s, op, static_cast<int>(st), inject);
      CHECK(st == LSM_ENOMEM || st == LSM_EHIP);
      g_enomem += st == LSM_ENOMEM;
      g_ehip += st == LSM_EHIP;
      CHECK(inject <= 1);
      // A failed update leaves r as it was, except for the batch of
      // elements that were staged before it: every update, bulk insertion
      // and cleanup first inserts those (a step of its own, which may have
      // succeeded before the failure).
      if (op <= 4 || op == 13 || op == 14) {
        const uint64_t r = lsm_num_batches(h);
        const bool ok = (r == r0) || (staged0 > 0 && r == r0 + 1);
        if (!ok)
          std::fprintf(stderr, "op %d status %d: r %llu -> %llu, staged %u\n", op,
                       static_cast<int>(st), static_cast<unsigned long long>(r0),
                       static_cast<unsigned long long>(r), staged0);
        CHECK(ok);
      }
      CHECK(lsm_flush(h) == LSM_OK);
      CHECK(lsm_sync(h) == LSM_OK);
    }
    if (s % 16 == 15) look_at_levels(h);
    if (s % 64 == 63) {
      lsm_stats_t stats;
      CHECK(lsm_get_stats(h, &stats) == LSM_OK && stats.num_batches == lsm_num_batches(h));
      lsm_profile_t prof;
      CHECK(lsm_profile_read(h, &prof, static_cast<int>(below(2))) == LSM_OK);
    }
  }
  // Autotuning of the first levels, explicit tuning and its errors.
  CHECK(lsm_autotune(h, 2, 1) == LSM_OK);
  uint32_t variant = 99;
  float us[6] = {0};
  CHECK(lsm_get_tuning(h, 1, &variant, us) == LSM_OK && variant < 6);
  CHECK(lsm_set_tuning(h, 1, 6) == LSM_EINVAL);
  CHECK(lsm_set_tuning(h, 40, 0) == LSM_EINVAL);
  CHECK(lsm_set_grouping(h, -1) == LSM_EINVAL);
  CHECK(lsm_autotune(h, 0, 0) == LSM_EINVAL);
  CHECK(lsm_clear(h) == LSM_OK && lsm_num_batches(h) == 0);
  // Argument errors leave everything as it was.
  {
    Buf<uint32_t> k(b + 1), v(b + 1);
    Buf<uint64_t> off(2);
    uint64_t total = 0;
    CHECK(lsm_insert_batch(h, k.p, v.p, b + 1) == LSM_EBATCH);
    CHECK(lsm_insert_batch(h, nullptr, v.p, 1) == LSM_EINVAL);
    CHECK(lsm_insert_batch(h, k.p, nullptr, 1) == LSM_EINVAL);
    CHECK(lsm_update_batch(h, k.p, v.p, nullptr, 1) == LSM_EINVAL);
    CHECK(lsm_insert_batch(h, k.p, v.p, 0) == LSM_OK);
    CHECK(lsm_lookup(h, nullptr, 1, v.p, nullptr) == LSM_EINVAL);
    CHECK(lsm_range(h, k.p, k.p, 1, off.p, nullptr, nullptr, 0, nullptr) == LSM_EINVAL);
    CHECK(lsm_range(h, k.p, k.p, 0, off.p, nullptr, nullptr, 0, &total) == LSM_OK && total == 0);
    CHECK(lsm_range_async_noalloc(h, k.p, k.p, LSM_NOALLOC_MAX_QUERIES + 1, off.p, k.p, v.p, 1) ==
          LSM_ECAPACITY);
    CHECK(lsm_num_batches(h) == 0);
    const uint32_t* kv = nullptr;
    const uint32_t* vals = nullptr;
    uint64_t len = 0;
    CHECK(lsm_level_view(h, 0, &kv, &vals, &len) == LSM_OK && len == 0);
  }
  CHECK(lsm_destroy(h) == LSM_OK);
}

}  // namespace

int main(int argc, char** argv) {
  // Optional arguments: a seed, then "large" for the benchmark's batch size
  // (1500 operations at b = 2^16, reaching level 10, and b = 2^18; for runs
  // by hand) or "threads" (handles driven from four threads at once).
  if (argc > 1) g_state = std::strtoull(argv[1], nullptr, 0);
  if (argc > 2 && std::strcmp(argv[2], "large") == 0) {
    run(65536, 0, 1u << 31, 1500);
    run(1u << 18, LSM_CHECKED, 1u << 31, 300);
    if (g_fail) return 1;
    std::printf("host sanitize check: ok (%ld calls failed with LSM_ENOMEM, %ld with LSM_EHIP)\n",
                g_enomem, g_ehip);
    return 0;
  }
  if (argc > 2 && std::strcmp(argv[2], "threads") == 0) {
    // Four threads, each driving handles of its own (the header makes calls
    // on different handles independent, the allocation-free range apart):
    // built with ThreadSanitizer, any state the host code shared between
    // handles would be reported.
    const uint64_t seed = g_state;
    std::atomic<int> fails{0};
    std::atomic<long> failed_calls{0};
    std::vector<std::thread> th;
    for (int t = 0; t < 4; ++t)
      th.emplace_back([t, seed, &fails, &failed_calls] {
        g_state = seed + 7919u * static_cast<uint64_t>(t + 1);
        g_threaded = true;
        run(t == 0 ? 1u : 100u * static_cast<uint32_t>(t), t == 2 ? LSM_CHECKED : 0u,
            t == 0 ? 5u : 1u << 20, 150);
        run(2048 + static_cast<uint32_t>(t), 0, 1u << 31, 60);
        fails += g_fail;
        failed_calls += g_enomem + g_ehip;
      });
    for (auto& x : th) x.join();
    if (fails.load() != 0) return 1;
    std::printf("host sanitize check, threads: ok (%ld calls failed)\n", failed_calls.load());
    return 0;
  }
  lsm_t h = nullptr;
  CHECK(lsm_create(&h, 0, 0, nullptr) == LSM_EINVAL && h == nullptr);
  CHECK(lsm_create(&h, (1u << 28) + 1, 0, nullptr) == LSM_EINVAL);
  CHECK(lsm_create(&h, 64, LSM_KEY_BITS(40), nullptr) == LSM_EINVAL);
  CHECK(lsm_create(nullptr, 64, 0, nullptr) == LSM_EINVAL);
  CHECK(lsm_destroy(nullptr) == LSM_EINVAL || lsm_destroy(nullptr) == LSM_OK);
  CHECK(lsm_num_batches(nullptr) == 0 && lsm_batch_size(nullptr) == 0);
  CHECK(lsm_strerror(LSM_ENOMEM) != nullptr);
  run(1, 0, 5, 300);
  run(7, LSM_CHECKED, 50, 300);
  run(100, 0, 1u << 20, 300);
  run(2048, LSM_KEY_BITS(20), 4000, 200);
  run(5000, 0, 1u << 31, 160);
  run(3 * 2048 + 5, LSM_CHECKED | LSM_KEY_BITS(24), 9000, 120);
  // Running out of memory while the handle is created, at every allocation
  // in turn: LSM_ENOMEM, no handle, nothing leaked.
  bool created = false;
  for (long k = 0; k < 64 && !created; ++k) {
    lsm_t g = nullptr;
    standin_fail_alloc_after(k);
    const lsm_status_t s = lsm_create(&g, 3000, LSM_CHECKED, nullptr);
    standin_fail_alloc_after(-1);
    if (s == LSM_OK) {
      created = true;
      CHECK(lsm_destroy(g) == LSM_OK);
    } else {
      CHECK(s == LSM_ENOMEM && g == nullptr);
    }
  }
  CHECK(created);
  if (g_fail) {
    std::fprintf(stderr, "%d checks failed\n", g_fail);
    return 1;
  }
  std::printf("host sanitize check: ok (%ld calls failed with LSM_ENOMEM, %ld with LSM_EHIP)\n",
              g_enomem, g_ehip);
  return 0;
}
