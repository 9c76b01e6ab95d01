// arena_check.cpp -- randomized self-check of gx::Arena, built with g++ by
// the host tests: allocations never overlap and stay inside the arena, and
// once everything is released the free space is one block again.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "arena.h"

int main(int argc, char** argv) {
  const uint64_t cap = 1ull << 30;
  const unsigned seed = argc > 1 ? (unsigned)std::atoi(argv[1]) : 1u;
  std::mt19937_64 rng(seed);
  gx::Arena a(cap);
  struct Blk { uint64_t off, size; };
  std::vector<Blk> live;
  std::vector<uint8_t> owner(cap / 256, 0);
  for (int it = 0; it < 200000; ++it) {
    const bool do_alloc = live.empty() || (rng() % 100) < 55;
    if (do_alloc) {
      const uint64_t size = 1 + rng() % (8u << 20);
      uint64_t off;
      if (!a.alloc(size, &off)) continue;
      const uint64_t g = (size + 255) / 256;
      if (off % 256 || off + g * 256 > cap) { std::printf("out of range\n"); return 1; }
      for (uint64_t k = off / 256; k < off / 256 + g; ++k) {
        if (owner[k]) { std::printf("overlap at granule %llu\n", (unsigned long long)k); return 1; }
        owner[k] = 1;
      }
      live.push_back({off, size});
    } else {
      const size_t i = rng() % live.size();
      const Blk b = live[i];
      live[i] = live.back();
      live.pop_back();
      for (uint64_t k = b.off / 256; k < b.off / 256 + (b.size + 255) / 256; ++k) owner[k] = 0;
      a.release(b.off, b.size);
    }
  }
  for (const Blk& b : live) a.release(b.off, b.size);
  uint64_t off;
  if (!a.alloc(cap, &off) || off != 0) { std::printf("not coalesced\n"); return 1; }
  std::printf("ok\n");
  return 0;
}
