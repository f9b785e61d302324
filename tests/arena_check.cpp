// Randomised check of the server's first-fit arena (hp_arena.h) against a
// unit-by-unit occupancy model: blocks never overlap, stay aligned and in
// range, the in-use count matches, and a drained arena is one free block.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "hp_arena.h"

#define CHECK(c)                                                        \
  do {                                                                  \
    if (!(c)) {                                                         \
      std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
      return 1;                                                         \
    }                                                                   \
  } while (0)

int main() {
  using hp::Arena;
  const size_t units = 4096;
  Arena a(units * Arena::kAlign + 100);   // the ragged tail is not usable
  CHECK(a.size() == units * Arena::kAlign);
  CHECK(a.free_blocks() == 1 && a.largest_free() == a.size());
  std::vector<int> owner(units, -1);
  std::vector<std::pair<size_t, size_t>> live;  // (offset, rounded bytes)
  std::mt19937_64 rng(12345);
  size_t used = 0;
  for (int step = 0; step < 200000; ++step) {
    const bool do_alloc = live.empty() || (rng() % 100) < 55;
    if (do_alloc) {
      const size_t bytes = (rng() % 4 == 0) ? rng() % (64 * Arena::kAlign) : rng() % (4 * Arena::kAlign);
      const size_t need = Arena::round(bytes ? bytes : 1);
      const size_t at = a.alloc(bytes);
      if (at == Arena::kFail) {
        // first fit failed: no run of free units is long enough
        size_t run = 0, best = 0;
        for (size_t u = 0; u < units; ++u) {
          run = owner[u] < 0 ? run + 1 : 0;
          best = run > best ? run : best;
        }
        CHECK(best * Arena::kAlign < need);
        continue;
      }
      CHECK(at % Arena::kAlign == 0);
      CHECK(at + need <= a.size());
      for (size_t u = at / Arena::kAlign; u < (at + need) / Arena::kAlign; ++u) {
        CHECK(owner[u] < 0);
        owner[u] = step;
      }
      live.push_back({at, need});
      used += need;
    } else {
      const size_t i = rng() % live.size();
      const auto blk = live[i];
      live[i] = live.back();
      live.pop_back();
      CHECK(a.release(blk.first));
      CHECK(!a.release(blk.first));    // a second release is refused
      for (size_t u = blk.first / Arena::kAlign; u < (blk.first + blk.second) / Arena::kAlign; ++u) owner[u] = -1;
      used -= blk.second;
    }
    CHECK(a.in_use() == used);
    CHECK(a.live_blocks() == live.size());
  }
  for (const auto &blk : live) CHECK(a.release(blk.first));
  CHECK(a.in_use() == 0);
  CHECK(a.free_blocks() == 1 && a.largest_free() == a.size());
  CHECK(a.alloc(a.size()) == 0);
  CHECK(a.alloc(1) == Arena::kFail);
  std::printf("arena ok\n");
  return 0;
}
