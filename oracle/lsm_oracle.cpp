// CPU oracle for the GPU LSM dictionary (Ashkiani et al., "GPU LSM: A Dynamic
// Dictionary Data Structure for the GPU").
//
// TEST INFRASTRUCTURE ONLY. Nothing in the product library links, loads or
// calls this file; only the tests, the smoke check and the benchmark's CPU
// baseline do. It shares no code, header or constant with the HIP path.
//
// Two independent oracles live here:
//
//  * MapOracle: the dictionary of section I-B written out with std::map and
//    applied one operation at a time, batches in call order. Its answers are
//    the plain definition of every query result.
//
//  * CascadeOracle: the level layout, computed by taking the insertion
//    algorithm's steps in the paper's order (Fig. 2(a) / Fig. 3): sort the
//    batch on the whole key variable, then, while level i is full, merge the
//    buffer with level i on the original key (newer run first on ties) and
//    empty level i; finally place the buffer in the first empty level and
//    increment the batch counter.  std::sort and std::merge are the library
//    primitives used as steps.
//
// Readings taken where the paper is silent or ambiguous (each is also listed
// in the design notes):
//   - duplicates inside one batch: the LAST one in batch order wins (sec.
//     III-A rule 3 leaves the choice open); for the layout this means equal
//     key variables inside a batch are ordered by descending batch position;
//   - a partial batch of n < b elements is padded with copies of its last
//     element (sec. IV-A names "the last one" as an example);
//   - tombstones carry value 0 (the paper gives them no value);
//   - status bit: 1 = regular element, 0 = tombstone (sec. IV-A, IV-B);
//   - merge ties: the element of the newer run comes first (sec. IV-A prose;
//     Fig. 3 passes the older level as the first merge argument, which the
//     prose overrides);
//   - count and range bounds are inclusive; k1 > k2 gives 0 / empty;
//   - a mixed batch applies its inserts in batch order and then its deletes
//     (sec. III-A rule 5: inserted and deleted in one batch means deleted);
//   - a coalesced batch (several single-type user batches packed in arrival
//     order into one batch of b) must instead behave like its user batches
//     applied one after another: it is sorted on the original key alone, the
//     later position first, so the newest operation on a key wins whatever
//     its type (oc_insert_ordered);
//   - successor(k) is the pair with the smallest key strictly greater than k
//     and predecessor(k) the pair with the largest key strictly smaller than
//     k (the order queries the footnote of sec. I-B names); none: not found;
//   - cleanup's placebo elements (sec. IV-D footnote) are tombstones of the
//     largest encodable key, 2^31 - 1, i.e. key variable 0xFFFFFFFE with
//     value 0 (the footnote's 2^32 - 1 would carry the regular status bit);
//     the redistributed list fills the occupied levels of the new batch count
//     from the smallest level up, so smaller keys land in smaller levels.
//
// Build: g++ -O2 -std=c++17 -shared -fPIC lsm_oracle.cpp -o liblsm_oracle.so
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <map>
#include <vector>

namespace {

// ---------------------------------------------------------------- MapOracle
struct MapOracle {
  std::map<uint32_t, uint32_t> m;
};

// ------------------------------------------------------------ CascadeOracle
struct Elem {
  uint32_t kv;   // key variable: (original key << 1) | status
  uint32_t val;  // value (0 for tombstones)
};

struct CascadeOracle {
  uint32_t b = 0;
  uint64_t r = 0;                          // number of resident batches
  std::vector<std::vector<Elem>> level;    // level i holds b * 2^i or nothing
  uint64_t merged_elems_last = 0;          // merge output elements, last insert
  uint64_t merged_elems_total = 0;
};

inline uint32_t orig_key(const Elem& e) { return e.kv >> 1; }

}  // namespace

extern "C" {

// ---------------------------------------------------------------- MapOracle
void* om_create() { return new MapOracle(); }
void om_destroy(void* h) { delete static_cast<MapOracle*>(h); }

// INSERT(k, v) for each pair in batch order: S <- (S - {<k,*>}) u {<k,v>}
// (sec. I-B).  A later duplicate in the batch overwrites an earlier one.
void om_insert(void* h, const uint32_t* keys, const uint32_t* vals, uint64_t n) {
  auto& m = static_cast<MapOracle*>(h)->m;
  for (uint64_t j = 0; j < n; ++j) m[keys[j]] = vals[j];
}

// DELETE(k) for each key: S <- S - {<k,*>} (sec. I-B). Idempotent.
void om_delete(void* h, const uint32_t* keys, uint64_t n) {
  auto& m = static_cast<MapOracle*>(h)->m;
  for (uint64_t j = 0; j < n; ++j) m.erase(keys[j]);
}

// Mixed batch (sec. III-A rules 2 and 5): inserts in batch order, then deletes.
void om_mixed(void* h, const uint32_t* keys, const uint32_t* vals,
              const uint8_t* is_delete, uint64_t n) {
  auto& m = static_cast<MapOracle*>(h)->m;
  for (uint64_t j = 0; j < n; ++j)
    if (!is_delete[j]) m[keys[j]] = vals[j];
  for (uint64_t j = 0; j < n; ++j)
    if (is_delete[j]) m.erase(keys[j]);
}

// LOOKUP(k): the pair with key k, or "not found" (sec. I-B).
void om_lookup(void* h, const uint32_t* q, uint64_t nq, uint32_t* vals,
               uint8_t* found) {
  auto& m = static_cast<MapOracle*>(h)->m;
  for (uint64_t i = 0; i < nq; ++i) {
    auto it = m.find(q[i]);
    if (it == m.end()) {
      vals[i] = 0;
      found[i] = 0;
    } else {
      vals[i] = it->second;
      found[i] = 1;
    }
  }
}

// COUNT(k1, k2): number of pairs with k1 <= k <= k2 (sec. I-B).
void om_count(void* h, const uint32_t* lo, const uint32_t* hi, uint64_t nq,
              uint32_t* counts) {
  auto& m = static_cast<MapOracle*>(h)->m;
  for (uint64_t i = 0; i < nq; ++i) {
    uint32_t c = 0;
    if (lo[i] <= hi[i]) {
      for (auto it = m.lower_bound(lo[i]); it != m.end() && it->first <= hi[i]; ++it) ++c;
    }
    counts[i] = c;
  }
}

// RANGE(k1, k2): all pairs with k1 <= k <= k2 (sec. I-B), per query in
// ascending key order, queries concatenated; offsets[nq+1] is the exclusive
// scan of the per-query sizes (sec. IV-D output form).  Returns the total;
// keys/vals are written only when total <= cap.
uint64_t om_range(void* h, const uint32_t* lo, const uint32_t* hi, uint64_t nq,
                  uint64_t* offsets, uint32_t* out_keys, uint32_t* out_vals,
                  uint64_t cap) {
  auto& m = static_cast<MapOracle*>(h)->m;
  uint64_t total = 0;
  for (uint64_t i = 0; i < nq; ++i) {
    offsets[i] = total;
    if (lo[i] > hi[i]) continue;
    for (auto it = m.lower_bound(lo[i]); it != m.end() && it->first <= hi[i]; ++it) ++total;
  }
  offsets[nq] = total;
  if (total > cap) return total;
  uint64_t w = 0;
  for (uint64_t i = 0; i < nq; ++i) {
    if (lo[i] > hi[i]) continue;
    for (auto it = m.lower_bound(lo[i]); it != m.end() && it->first <= hi[i]; ++it) {
      out_keys[w] = it->first;
      out_vals[w] = it->second;
      ++w;
    }
  }
  return total;
}

// Order queries (footnote of sec. I-B): successor = smallest key > k,
// predecessor = largest key < k.  found = 0 leaves key and value 0.
void om_successor(void* h, const uint32_t* q, uint64_t nq, uint32_t* keys, uint32_t* vals,
                  uint8_t* found) {
  const auto& m = static_cast<MapOracle*>(h)->m;
  for (uint64_t i = 0; i < nq; ++i) {
    auto it = m.upper_bound(q[i]);
    const bool f = it != m.end();
    found[i] = f ? 1 : 0;
    keys[i] = f ? it->first : 0u;
    vals[i] = f ? it->second : 0u;
  }
}

void om_predecessor(void* h, const uint32_t* q, uint64_t nq, uint32_t* keys, uint32_t* vals,
                    uint8_t* found) {
  const auto& m = static_cast<MapOracle*>(h)->m;
  for (uint64_t i = 0; i < nq; ++i) {
    auto it = m.lower_bound(q[i]);
    const bool f = it != m.begin();
    if (f) --it;
    found[i] = f ? 1 : 0;
    keys[i] = f ? it->first : 0u;
    vals[i] = f ? it->second : 0u;
  }
}

uint64_t om_size(void* h) { return static_cast<MapOracle*>(h)->m.size(); }

// All live pairs in ascending key order.
void om_items(void* h, uint32_t* keys, uint32_t* vals) {
  auto& m = static_cast<MapOracle*>(h)->m;
  uint64_t w = 0;
  for (auto& kv : m) {
    keys[w] = kv.first;
    vals[w] = kv.second;
    ++w;
  }
}

// ------------------------------------------------------------ CascadeOracle
void* oc_create(uint32_t b) {
  auto* c = new CascadeOracle();
  c->b = b;
  return c;
}
void oc_destroy(void* h) { delete static_cast<CascadeOracle*>(h); }

// INSERT(batch) of Fig. 2(a) / Fig. 3, for a batch of n <= b elements.
// status[j] = 1 for a regular element, 0 for a tombstone (DELETE(batch) is
// INSERT(tombed(batch)), sec. III-C); status == nullptr means all regular.
// vals == nullptr means all values are 0.  Returns 0, or -1 if n == 0 or
// n > b (nothing is changed then).
static int insert_impl(void* h, const uint32_t* keys, const uint32_t* vals,
                       const uint8_t* status, uint32_t n, bool status_in_sort) {
  auto* c = static_cast<CascadeOracle*>(h);
  const uint32_t b = c->b;
  if (n == 0 || n > b) return -1;

  // Build the batch of key variables (sec. IV-A), padded to b with copies of
  // the last element.  pos is the position in the padded batch.
  struct Tagged {
    Elem e;
    uint32_t pos;
  };
  std::vector<Tagged> batch(b);
  for (uint32_t p = 0; p < b; ++p) {
    uint32_t src = p < n ? p : n - 1;
    uint32_t s = status ? (status[src] ? 1u : 0u) : 1u;
    uint32_t v = (s && vals) ? vals[src] : 0u;
    batch[p].e.kv = (keys[src] << 1) | s;
    batch[p].e.val = v;
    batch[p].pos = p;
  }
  // buffer <- sort(input): radix order on the whole key variable, status bit
  // included (tombstone before regular element of the same key); equal key
  // variables ordered so the later batch position comes first.
  std::sort(batch.begin(), batch.end(), [status_in_sort](const Tagged& x, const Tagged& y) {
    const uint32_t kx = status_in_sort ? x.e.kv : (x.e.kv >> 1);
    const uint32_t ky = status_in_sort ? y.e.kv : (y.e.kv >> 1);
    if (kx != ky) return kx < ky;
    return x.pos > y.pos;
  });
  std::vector<Elem> buffer(b);
  for (uint32_t p = 0; p < b; ++p) buffer[p] = batch[p].e;

  // while level i is full: buffer <- merge(buffer, level i); empty level i.
  c->merged_elems_last = 0;
  uint32_t i = 0;
  while ((c->r >> i) & 1u) {
    std::vector<Elem> out(buffer.size() + c->level[i].size());
    // std::merge takes from the first range on ties, so the newer run
    // (the buffer) goes first; the comparison ignores the status bit.
    std::merge(buffer.begin(), buffer.end(), c->level[i].begin(), c->level[i].end(),
               out.begin(),
               [](const Elem& x, const Elem& y) { return orig_key(x) < orig_key(y); });
    buffer.swap(out);
    c->level[i].clear();
    c->merged_elems_last += buffer.size();
    ++i;
  }
  if (c->level.size() <= i) c->level.resize(i + 1);
  c->level[i].swap(buffer);
  c->r += 1;
  c->merged_elems_total += c->merged_elems_last;
  return 0;
}

int oc_insert(void* h, const uint32_t* keys, const uint32_t* vals, const uint8_t* status,
              uint32_t n) {
  return insert_impl(h, keys, vals, status, n, true);
}

// A coalesced batch (see the readings above): identical to oc_insert except
// that the batch sort ignores the status bit.
int oc_insert_ordered(void* h, const uint32_t* keys, const uint32_t* vals, const uint8_t* status,
                      uint32_t n) {
  return insert_impl(h, keys, vals, status, n, false);
}

// CLEANUP (sec. III-E), by the bulk strategy of sec. IV-D: (1) merge the
// occupied levels from the smallest to the largest, the accumulated newer
// run first on equal original keys; (2) mark every element that is not the
// first of its key run, and every tombstone, as stale; (3) compact the
// valid elements, order kept; (4) pad with fewer than b placebos up to a
// multiple of b; (5) slice the list into the levels of the new batch count.
// Returns the number of valid elements.
uint64_t oc_cleanup(void* h) {
  auto* c = static_cast<CascadeOracle*>(h);
  const uint64_t b = c->b;
  std::vector<Elem> acc;
  for (size_t i = 0; i < c->level.size(); ++i) {
    if (((c->r >> i) & 1u) == 0) continue;
    std::vector<Elem> out(acc.size() + c->level[i].size());
    std::merge(acc.begin(), acc.end(), c->level[i].begin(), c->level[i].end(), out.begin(),
               [](const Elem& x, const Elem& y) { return orig_key(x) < orig_key(y); });
    acc.swap(out);
  }
  std::vector<Elem> valid;
  for (size_t p = 0; p < acc.size(); ++p) {
    const bool first = p == 0 || orig_key(acc[p - 1]) != orig_key(acc[p]);
    if (first && (acc[p].kv & 1u)) valid.push_back(acc[p]);
  }
  const uint64_t v = valid.size();
  const uint64_t r2 = (v + b - 1) / b;
  valid.resize(r2 * b, Elem{0xFFFFFFFEu, 0u});
  c->level.assign(64, std::vector<Elem>());
  uint64_t off = 0;
  for (int i = 0; i < 64 && (r2 >> i) != 0; ++i) {
    if (((r2 >> i) & 1u) == 0) continue;
    const uint64_t len = b << i;
    c->level[i].assign(valid.begin() + off, valid.begin() + off + len);
    off += len;
  }
  c->r = r2;
  c->merged_elems_last = 0;
  return v;
}

uint64_t oc_num_batches(void* h) { return static_cast<CascadeOracle*>(h)->r; }
uint64_t oc_merged_last(void* h) { return static_cast<CascadeOracle*>(h)->merged_elems_last; }
uint64_t oc_merged_total(void* h) { return static_cast<CascadeOracle*>(h)->merged_elems_total; }

// Number of elements held by level i (0 when empty).
uint64_t oc_level_size(void* h, uint32_t i) {
  auto* c = static_cast<CascadeOracle*>(h);
  return i < c->level.size() ? c->level[i].size() : 0;
}

// Copy level i out as separate key-variable and value arrays.
void oc_level(void* h, uint32_t i, uint32_t* kv, uint32_t* vals) {
  auto* c = static_cast<CascadeOracle*>(h);
  if (i >= c->level.size()) return;
  const auto& L = c->level[i];
  for (size_t p = 0; p < L.size(); ++p) {
    kv[p] = L[p].kv;
    vals[p] = L[p].val;
  }
}

}  // extern "C"
