"""Plant plausible mistakes in a copy of the oracle (on the CPU) and check
that the pins in test_oracle_pins.py catch every one of them."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "lsm_oracle.cpp")

# (name, text in the oracle, planted replacement)
MUTATIONS = [
    ("merge_ties_to_older",
     "std::merge(buffer.begin(), buffer.end(), c->level[i].begin(), c->level[i].end(),",
     "std::merge(c->level[i].begin(), c->level[i].end(), buffer.begin(), buffer.end(),"),
    ("batch_duplicates_first_wins", "return x.pos > y.pos;", "return x.pos < y.pos;"),
    ("pad_with_first_element", "uint32_t src = p < n ? p : n - 1;", "uint32_t src = p < n ? p : 0;"),
    ("status_polarity", "(status[src] ? 1u : 0u)", "(status[src] ? 0u : 1u)"),
    ("tombstone_keeps_value", "uint32_t v = (s && vals) ? vals[src] : 0u;",
     "uint32_t v = vals ? vals[src] : 0u;"),
    ("level_not_emptied", "    c->level[i].clear();\n", "\n"),
    ("cascade_stops_early", "while ((c->r >> i) & 1u) {", "while (i < 1 && ((c->r >> i) & 1u)) {"),
    ("count_upper_bound_exclusive",
     "for (auto it = m.lower_bound(lo[i]); it != m.end() && it->first <= hi[i]; ++it) ++c;",
     "for (auto it = m.lower_bound(lo[i]); it != m.end() && it->first < hi[i]; ++it) ++c;"),
    ("insert_keeps_old_value", "  for (uint64_t j = 0; j < n; ++j) m[keys[j]] = vals[j];\n}",
     "  for (uint64_t j = 0; j < n; ++j) m.emplace(keys[j], vals[j]);\n}"),
    ("mixed_deletes_first", "    if (!is_delete[j]) m[keys[j]] = vals[j];\n  for (uint64_t j = 0; j < n; ++j)\n    if (is_delete[j]) m.erase(keys[j]);",
     "    if (is_delete[j]) m.erase(keys[j]);\n  for (uint64_t j = 0; j < n; ++j)\n    if (!is_delete[j]) m[keys[j]] = vals[j];"),
    ("ordered_batch_sorts_on_status",
     "    const uint32_t kx = status_in_sort ? x.e.kv : (x.e.kv >> 1);",
     "    const uint32_t kx = x.e.kv;"),
    ("cleanup_keeps_last_of_run",
     "const bool first = p == 0 || orig_key(acc[p - 1]) != orig_key(acc[p]);",
     "const bool first = p + 1 == acc.size() || orig_key(acc[p + 1]) != orig_key(acc[p]);"),
    ("cleanup_merges_older_first",
     "std::merge(acc.begin(), acc.end(), c->level[i].begin(), c->level[i].end(), out.begin(),",
     "std::merge(c->level[i].begin(), c->level[i].end(), acc.begin(), acc.end(), out.begin(),"),
    ("cleanup_placebo_regular", "valid.resize(r2 * b, Elem{0xFFFFFFFEu, 0u});",
     "valid.resize(r2 * b, Elem{0xFFFFFFFFu, 0u});"),
    ("cleanup_keeps_tombstones", "if (first && (acc[p].kv & 1u)) valid.push_back(acc[p]);",
     "if (first) valid.push_back(acc[p]);"),
    ("cleanup_large_keys_in_small_levels",
     "c->level[i].assign(valid.begin() + off, valid.begin() + off + len);",
     "c->level[i].assign(valid.end() - off - len, valid.end() - off);"),
    ("successor_not_strict", "auto it = m.upper_bound(q[i]);", "auto it = m.lower_bound(q[i]);"),
    ("predecessor_off_by_one", "    const bool f = it != m.begin();\n    if (f) --it;",
     "    const bool f = it != m.end();"),
    ("lookup_miss_value", "      vals[i] = 0;\n      found[i] = 0;", "      vals[i] = 1;\n      found[i] = 0;"),
]


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_planted_mistake(name, old, new, tmp_path):
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation anchor not found: " + name
    mutated = tmp_path / "mut.cpp"
    mutated.write_text(src.replace(old, new))
    lib = tmp_path / "libmut.so"
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", str(mutated), "-o", str(lib)])
    env = dict(os.environ, LSM_ORACLE_LIB=str(lib))
    res = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                          os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert res.returncode != 0, "pins did not catch planted mistake " + name
