// Randomised check of the server's arena allocator against a byte map:
// blocks never overlap, stay in range and aligned, accounting is exact, and
// after everything is released the arena is one free block again.
#include <cstdio>
#include <random>
#include <vector>

#include "arena.h"

int main() {
  using fdwt::Arena;
  const size_t size = (size_t)1 << 20;
  Arena a;
  a.reset(size);
  std::vector<int> owner(size / 256, -1);
  struct Blk { size_t off, bytes; };
  std::vector<Blk> live;
  std::mt19937_64 rng(12345);
  size_t used = 0;
  for (int it = 0; it < 200000; ++it) {
    const bool do_alloc = live.empty() || (rng() % 100) < 55;
    if (do_alloc) {
      const size_t bytes = 1 + rng() % (size / 16);
      const size_t off = a.alloc(bytes);
      const size_t r = fdwt::arena_round(bytes);
      if (off == fdwt::kNone) {
        if (a.largest_free() >= r) { std::printf("refused although a block fits\n"); return 1; }
        continue;
      }
      if (off % 256 || off + r > size) { std::printf("bad block\n"); return 1; }
      for (size_t u = off / 256; u < (off + r) / 256; ++u) {
        if (owner[u] != -1) { std::printf("overlap at %zu\n", u); return 1; }
        owner[u] = it;
      }
      live.push_back({off, bytes});
      used += r;
    } else {
      const size_t k = rng() % live.size();
      const Blk b = live[k];
      live[k] = live.back();
      live.pop_back();
      const size_t r = fdwt::arena_round(b.bytes);
      for (size_t u = b.off / 256; u < (b.off + r) / 256; ++u) owner[u] = -1;
      a.release(b.off, b.bytes);
      used -= r;
    }
    if (a.used() != used) { std::printf("accounting %zu vs %zu\n", a.used(), used); return 1; }
  }
  for (const Blk& b : live) a.release(b.off, b.bytes);
  if (a.used() != 0 || a.free_blocks() != 1 || a.largest_free() != size) {
    std::printf("not coalesced: %zu blocks\n", a.free_blocks());
    return 1;
  }
  std::printf("ok peak=%zu\n", a.peak());
  return 0;
}
