// Host check of the library's free-slot pool (snn_host.h) against a plain
// model (per-block sets of free slots and stale flags) under a long random
// sequence of inserts, deletes and compactions, with and without array
// containers: every slot handed out is free (or fresh) and never handed out
// twice, and each choice follows the pool's order -- a stale block's free slot
// while one exists; then, with array containers, a fresh slot; then the clean
// block with the most free slots (without array containers, freed slots
// before fresh ones). Prints "ok" or the first disagreement.
#include <cstdio>
#include <random>
#include <set>
#include <vector>

#include "snn_host.h"

int main() {
  const uint32_t cap = 16 * 1024;
  const uint32_t nblk = cap >> 10;
  std::mt19937_64 rng(11);
  for (int arrays = 0; arrays < 2; ++arrays) {
    snn::SlotPool pool;
    pool.init(cap);
    uint32_t next_fresh = 0;
    std::vector<std::set<uint32_t>> freeb(nblk);
    std::vector<uint8_t> stale(nblk, 0);
    std::vector<uint8_t> used(cap, 0);  // slot holds a document
    std::vector<uint32_t> held;        // slots holding documents
    size_t nfree = 0;
    for (int step = 0; step < 300000; ++step) {
      const int op = (int)(rng() % 100);
      if (op < 55 && (nfree > 0 || next_fresh < cap)) {
        // what the order allows
        bool any_stale_free = false;
        for (uint32_t b = 0; b < nblk; ++b) any_stale_free |= stale[b] && !freeb[b].empty();
        size_t best = 0;
        for (uint32_t b = 0; b < nblk; ++b)
          if (!stale[b]) best = std::max(best, freeb[b].size());
        const uint32_t nf0 = next_fresh;
        const uint32_t s = pool.take(next_fresh, cap, arrays != 0);
        const uint32_t b = s >> 10;
        const bool fresh = s == nf0 && next_fresh == nf0 + 1;
        if (fresh) {
          if (any_stale_free || (!arrays && best > 0)) { printf("fresh slot %u taken too early\n", s); return 1; }
        } else {
          if (next_fresh != nf0 || !freeb[b].count(s)) { printf("slot %u was not free\n", s); return 1; }
          if (any_stale_free && !stale[b]) { printf("clean block %u before a stale one\n", b); return 1; }
          if (!any_stale_free) {
            if (arrays && nf0 < cap) { printf("free slot %u before a fresh one\n", s); return 1; }
            if (freeb[b].size() != best) { printf("block %u has %zu free, best %zu\n", b, freeb[b].size(), best); return 1; }
          }
          freeb[b].erase(s);
          --nfree;
        }
        if (used[s]) { printf("slot %u handed out twice\n", s); return 1; }
        used[s] = 1;
        stale[b] = 1;
        held.push_back(s);
      } else if (op < 95 && !held.empty()) {
        const size_t i = rng() % held.size();
        const uint32_t s = held[i];
        held[i] = held.back();
        held.pop_back();
        used[s] = 0;
        freeb[s >> 10].insert(s);
        ++nfree;
        pool.release(s);
      } else if (op >= 99) {
        pool.clear_stale();
        std::fill(stale.begin(), stale.end(), (uint8_t)0);
      }
      if (pool.size() != nfree) { printf("size %zu vs %zu at %d\n", pool.size(), nfree, step); return 1; }
      for (uint32_t b = 0; b < nblk; b += 5)
        if (pool.is_stale(b) != (stale[b] != 0)) { printf("stale flag of block %u at %d\n", b, step); return 1; }
    }
  }
  printf("ok\n");
  return 0;
}
