// Host check of the library's id -> slot map (snn_host.h) against
// std::unordered_map under a long random sequence of puts, overwrites and
// erases (with many ids that collide in the table); prints "ok" or the first
// disagreement.
#include <cstdio>
#include <random>
#include <unordered_map>

#include "snn_host.h"

int main() {
  snn::IdMap m;
  std::unordered_map<uint32_t, uint32_t> ref;
  std::mt19937_64 rng(7);
  for (int step = 0; step < 400000; ++step) {
    // a small id range forces long probe runs and wrap-around at the table end
    const uint32_t id = (step & 1) ? (uint32_t)(rng() % 3000) : (uint32_t)(rng() % 3000) * 65536u;
    const int op = (int)(rng() % 3);
    if (op == 0 || op == 1) {
      const uint32_t v = (uint32_t)rng();
      m.put(id, v);
      ref[id] = v;
    } else {
      const bool a = m.erase(id), b = ref.erase(id) > 0;
      if (a != b) { printf("erase %u: %d vs %d\n", id, a, b); return 1; }
    }
    if (m.size() != ref.size()) { printf("size %zu vs %zu at %d\n", m.size(), ref.size(), step); return 1; }
    if (step % 997 == 0) {
      for (auto &kv : ref) {
        const uint32_t *f = m.find(kv.first);
        if (!f || *f != kv.second) { printf("find %u\n", kv.first); return 1; }
      }
      size_t n = 0;
      bool bad = false;
      m.for_each([&](uint32_t k, uint32_t v) { ++n; auto it = ref.find(k); bad |= it == ref.end() || it->second != v; });
      if (bad || n != ref.size()) { printf("for_each\n"); return 1; }
    }
  }
  printf("ok\n");
  return 0;
}
