// Sanitizer run of the CPU oracle (test infrastructure only; built and run by
// tests/test_oracle_sanitize.py with AddressSanitizer and
// UndefinedBehaviorSanitizer, host code only).
//
// Seeded random streams of insert, delete, mixed and coalesced batches
// (partial batches and tiny key domains included), with cleanups at random
// points, drive both oracles through their C entry points; every entry point
// is called.  After each step the dictionary the cascade layout encodes is
// compared with the map oracle: scanning the occupied levels from the
// smallest (newest) up, the first element met for a key decides it (a
// regular element is live, a tombstone deletes it), which is the query rule
// of the paper's lookups (sec. III-D); counts, ranges and order queries of the
// map are checked against brute force over its items.  Exit status 0 when
// every check holds; a sanitizer report aborts the run.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <vector>

extern "C" {
void* om_create();
void om_destroy(void* h);
void om_insert(void* h, const uint32_t* keys, const uint32_t* vals, uint64_t n);
void om_delete(void* h, const uint32_t* keys, uint64_t n);
void om_mixed(void* h, const uint32_t* keys, const uint32_t* vals, const uint8_t* is_delete,
              uint64_t n);
void om_lookup(void* h, const uint32_t* q, uint64_t nq, uint32_t* vals, uint8_t* found);
void om_count(void* h, const uint32_t* lo, const uint32_t* hi, uint64_t nq, uint32_t* out);
uint64_t om_range(void* h, const uint32_t* lo, const uint32_t* hi, uint64_t nq,
                  uint64_t* offsets, uint32_t* out_keys, uint32_t* out_vals, uint64_t cap);
void om_successor(void* h, const uint32_t* q, uint64_t nq, uint32_t* keys, uint32_t* vals,
                  uint8_t* found);
void om_predecessor(void* h, const uint32_t* q, uint64_t nq, uint32_t* keys, uint32_t* vals,
                    uint8_t* found);
uint64_t om_size(void* h);
void om_items(void* h, uint32_t* keys, uint32_t* vals);
void* oc_create(uint32_t b);
void oc_destroy(void* h);
int oc_insert(void* h, const uint32_t* keys, const uint32_t* vals, const uint8_t* status,
              uint32_t n);
int oc_insert_ordered(void* h, const uint32_t* keys, const uint32_t* vals, const uint8_t* status,
                      uint32_t n);
uint64_t oc_cleanup(void* h);
uint64_t oc_num_batches(void* h);
uint64_t oc_merged_last(void* h);
uint64_t oc_merged_total(void* h);
uint64_t oc_level_size(void* h, uint32_t i);
void oc_level(void* h, uint32_t i, uint32_t* kv, uint32_t* vals);
}

namespace {

uint64_t g_state = 0x9E3779B97F4A7C15ull;
uint64_t next_u64() {  // splitmix64
  uint64_t z = (g_state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
uint32_t below(uint32_t n) { return static_cast<uint32_t>(next_u64() % n); }

int g_fail = 0;
void check(bool ok, const char* what, uint64_t step) {
  if (!ok && g_fail++ < 10) std::fprintf(stderr, "check failed: %s (step %llu)\n", what,
                                         static_cast<unsigned long long>(step));
}

// The dictionary the cascade layout encodes: levels from the smallest up,
// the first element met for a key decides it.
std::map<uint32_t, uint32_t> decode(void* c) {
  std::map<uint32_t, uint32_t> live;
  std::map<uint32_t, bool> seen;
  const uint64_t r = oc_num_batches(c);
  for (uint32_t i = 0; i < 64 && (r >> i) != 0; ++i) {
    if (((r >> i) & 1u) == 0) continue;
    const uint64_t n = oc_level_size(c, i);
    std::vector<uint32_t> kv(n), v(n);
    oc_level(c, i, kv.data(), v.data());
    for (uint64_t x = 0; x < n; ++x) {
      const uint32_t key = kv[x] >> 1;
      if (seen.count(key)) continue;
      seen[key] = true;
      if (kv[x] & 1u) live[key] = v[x];
    }
  }
  return live;
}

void compare(void* m, void* c, uint32_t domain, uint64_t step) {
  const uint64_t n = om_size(m);
  std::vector<uint32_t> ik(n), iv(n);
  om_items(m, ik.data(), iv.data());
  const std::map<uint32_t, uint32_t> live = decode(c);
  check(live.size() == n, "live count", step);
  uint64_t x = 0;
  for (const auto& kv : live) {
    if (x >= n) break;
    check(kv.first == ik[x] && kv.second == iv[x], "live pair", step);
    ++x;
  }
  // Queries of the map against brute force over its items.
  const uint32_t nq = 64;
  std::vector<uint32_t> q(nq), lo(nq), hi(nq), val(nq), cnt(nq), sk(nq), sv(nq), pk(nq), pv(nq);
  std::vector<uint8_t> f(nq), sf(nq), pf(nq);
  for (uint32_t i = 0; i < nq; ++i) {
    q[i] = below(domain + 2);
    lo[i] = below(domain + 2);
    hi[i] = i % 9 == 0 ? lo[i] - 1 : lo[i] + below(domain / 4 + 2);  // some empty ranges
  }
  om_lookup(m, q.data(), nq, val.data(), f.data());
  om_count(m, lo.data(), hi.data(), nq, cnt.data());
  std::vector<uint64_t> off(nq + 1);
  const uint64_t total = om_range(m, lo.data(), hi.data(), nq, off.data(), nullptr, nullptr, 0);
  std::vector<uint32_t> rk(total + 1), rv(total + 1);
  check(om_range(m, lo.data(), hi.data(), nq, off.data(), rk.data(), rv.data(), total) == total,
        "range total", step);
  om_successor(m, q.data(), nq, sk.data(), sv.data(), sf.data());
  om_predecessor(m, q.data(), nq, pk.data(), pv.data(), pf.data());
  for (uint32_t i = 0; i < nq; ++i) {
    const auto it = live.find(q[i]);
    check((it != live.end()) == (f[i] != 0), "lookup found", step);
    if (it != live.end()) check(val[i] == it->second, "lookup value", step);
    uint32_t c2 = 0;
    if (lo[i] <= hi[i])
      for (auto jt = live.lower_bound(lo[i]); jt != live.end() && jt->first <= hi[i]; ++jt) {
        const uint64_t at = off[i] + c2;
        check(at < off[i + 1] && rk[at] == jt->first && rv[at] == jt->second, "range pair", step);
        ++c2;
      }
    check(cnt[i] == c2 && off[i + 1] - off[i] == c2, "count", step);
    const auto up = live.upper_bound(q[i]);
    check((up != live.end()) == (sf[i] != 0), "successor found", step);
    if (up != live.end()) check(sk[i] == up->first && sv[i] == up->second, "successor", step);
    const auto lb = live.lower_bound(q[i]);
    const bool has_pred = lb != live.begin();
    check(has_pred == (pf[i] != 0), "predecessor found", step);
    if (has_pred) {
      auto pt = lb;
      --pt;
      check(pk[i] == pt->first && pv[i] == pt->second, "predecessor", step);
    }
  }
}

void run(uint32_t b, uint32_t domain, uint32_t steps) {
  void* m = om_create();
  void* c = oc_create(b);
  uint64_t merged = 0;
  for (uint32_t s = 0; s < steps; ++s) {
    const uint32_t n = below(4) == 0 ? 1 + below(b) : b;  // partial batches now and then
    std::vector<uint32_t> k(n), v(n);
    std::vector<uint8_t> st(n), del(n);
    for (uint32_t i = 0; i < n; ++i) {
      k[i] = below(domain);
      v[i] = static_cast<uint32_t>(next_u64());
      del[i] = below(3) == 0 ? 1 : 0;
      st[i] = del[i] ? 0 : 1;
    }
    const uint32_t kind = below(5);
    if (kind == 0) {
      om_insert(m, k.data(), v.data(), n);
      check(oc_insert(c, k.data(), v.data(), nullptr, n) == 0, "insert", s);
    } else if (kind == 1) {
      om_delete(m, k.data(), n);
      std::vector<uint8_t> zero(n, 0);
      check(oc_insert(c, k.data(), nullptr, zero.data(), n) == 0, "delete", s);
    } else if (kind == 2) {
      om_mixed(m, k.data(), v.data(), del.data(), n);
      check(oc_insert(c, k.data(), v.data(), st.data(), n) == 0, "mixed", s);
    } else {
      // A coalesced batch: the same operations one at a time on the map.
      for (uint32_t i = 0; i < n; ++i) {
        if (del[i]) om_delete(m, &k[i], 1);
        else om_insert(m, &k[i], &v[i], 1);
      }
      std::vector<uint32_t> vz(v);
      for (uint32_t i = 0; i < n; ++i) if (del[i]) vz[i] = 0;
      check(oc_insert_ordered(c, k.data(), vz.data(), st.data(), n) == 0, "ordered", s);
    }
    merged += oc_merged_last(c);
    check(oc_merged_total(c) == merged, "merge total", s);
    if (below(7) == 0) check(oc_cleanup(c) == om_size(m), "cleanup size", s);
    compare(m, c, domain, s);
  }
  // Rejected batch sizes change nothing.
  const uint64_t r = oc_num_batches(c);
  std::vector<uint32_t> big(b + 1, 1);
  check(oc_insert(c, big.data(), big.data(), nullptr, b + 1) != 0, "oversized batch", steps);
  check(oc_insert(c, big.data(), big.data(), nullptr, 0) != 0, "empty batch", steps);
  check(oc_num_batches(c) == r, "rejected batches", steps);
  oc_destroy(c);
  om_destroy(m);
}

}  // namespace

int main() {
  run(1, 7, 200);
  run(5, 40, 160);
  run(64, 300, 120);
  run(100, 1u << 20, 60);
  run(1000, 2500, 40);
  if (g_fail) {
    std::fprintf(stderr, "%d checks failed\n", g_fail);
    return 1;
  }
  std::printf("oracle sanitize check: ok\n");
  return 0;
}
