// Randomised check of the server's first-fit arena against a brute-force
// occupancy map (one flag per 256-byte unit).  Exit status 0 = all checks
// passed; prints the first violation otherwise.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "arena.h"

namespace {

struct Live {
  size_t off, bytes;
};

int fail(const char* what, long step) {
  std::printf("violation at step %ld: %s\n", step, what);
  return 1;
}

}  // namespace

int main() {
  const size_t U = lr::Arena::ALIGN;
  for (unsigned seed = 1; seed <= 20; ++seed) {
    std::mt19937_64 rng(seed);
    const size_t units = 64 + rng() % 512;
    lr::Arena a(units * U + (rng() % U));  // capacity is rounded down to whole units
    if (a.capacity() != units * U) return fail("capacity rounding", -1);
    std::vector<char> used(units, 0);
    std::vector<Live> live;
    for (long step = 0; step < 4000; ++step) {
      const bool do_alloc = live.empty() || (rng() % 100) < 55;
      if (do_alloc) {
        const size_t bytes = 1 + rng() % (units * U / 6);
        const size_t need = (bytes + U - 1) / U;
        // brute force: lowest start of `need` free units
        long first = -1;
        for (size_t s = 0; s + need <= units && first < 0; ++s) {
          size_t j = 0;
          while (j < need && !used[s + j]) ++j;
          if (j == need) first = (long)s;
        }
        if (a.fits(bytes) != (first >= 0)) return fail("fits() disagrees", step);
        size_t off = 0;
        const bool ok = a.alloc(bytes, &off);
        if (ok != (first >= 0)) return fail("alloc() success disagrees", step);
        if (!ok) continue;
        if (off % U) return fail("misaligned offset", step);
        if (off / U != (size_t)first) return fail("not the lowest fitting range", step);
        for (size_t j = 0; j < need; ++j) {
          if (used[off / U + j]) return fail("overlap", step);
          used[off / U + j] = 1;
        }
        live.push_back({off, bytes});
      } else {
        const size_t i = rng() % live.size();
        const Live l = live[i];
        live[i] = live.back();
        live.pop_back();
        a.release(l.off, l.bytes);
        for (size_t j = 0; j < (l.bytes + U - 1) / U; ++j) used[l.off / U + j] = 0;
      }
      size_t nused = 0, runs = 0;
      for (size_t s = 0; s < units; ++s) {
        nused += used[s];
        if (!used[s] && (s == 0 || used[s - 1])) ++runs;
      }
      if (a.used() != nused * U) return fail("used() disagrees", step);
      if (a.free_ranges() != runs) return fail("free ranges not coalesced", step);
    }
    for (const Live& l : live) a.release(l.off, l.bytes);
    if (a.used() != 0 || a.free_ranges() != 1) return fail("not empty at the end", -1);
  }
  std::printf("arena ok\n");
  return 0;
}
