// Randomised check of the render server's device-memory arena (host-only
// logic): blocks never overlap, stay inside the arena, are aligned, and after
// every block is released the arena is one free range again.  Prints "ok".
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <vector>

#include "../../paper_2404_16221_amd/csrc/arena.hpp"

int main() {
  const size_t size = 1u << 24;
  xl::Arena a;
  a.reset(size);
  std::mt19937_64 rng(2404);
  std::map<size_t, size_t> live;  // offset -> bytes
  size_t live_bytes = 0;
  for (int step = 0; step < 200000; ++step) {
    const bool grow = live.empty() || (rng() % 100) < 55;
    if (grow) {
      const size_t want = 1 + rng() % (size / 64);
      size_t off;
      if (a.alloc(want, &off)) {
        const size_t b = xl::Arena::round(want);
        if (off % xl::Arena::kAlign || off + b > size) { std::printf("bad block\n"); return 1; }
        auto nx = live.lower_bound(off);
        if (nx != live.end() && off + b > nx->first) { std::printf("overlap next\n"); return 1; }
        if (nx != live.begin()) {
          auto pv = std::prev(nx);
          if (pv->first + pv->second > off) { std::printf("overlap prev\n"); return 1; }
        }
        live[off] = b;
        live_bytes += b;
      }
    } else {
      auto it = live.begin();
      std::advance(it, rng() % live.size());
      // release either the whole block or its tail, as the server does
      if (rng() % 4 == 0 && it->second > 2 * xl::Arena::kAlign) {
        const size_t keep = xl::Arena::round(it->second / 2);
        a.release(it->first + keep, it->second - keep);
        live_bytes -= it->second - keep;
        it->second = keep;
      } else {
        a.release(it->first, it->second);
        live_bytes -= it->second;
        live.erase(it);
      }
    }
    if (a.used() != live_bytes) { std::printf("used %zu != %zu\n", a.used(), live_bytes); return 1; }
  }
  for (auto& kv : live) a.release(kv.first, kv.second);
  size_t off;
  if (a.used() != 0 || !a.alloc(size, &off) || off != 0) { std::printf("not coalesced\n"); return 1; }
  std::printf("ok\n");
  return 0;
}
