// Host-only checks of the shot server's arena allocator (fd_arena.h) against a
// brute-force model: a byte-granular occupancy map and a first-fit scan over it.
#include <stdio.h>
#include <stdlib.h>

#include <random>
#include <vector>

#include "fd_arena.h"

static int fails = 0;
#define CHECK(c)                                                     \
  do {                                                               \
    if (!(c)) {                                                      \
      fprintf(stderr, "FAIL %s:%d: %s\n", __FILE__, __LINE__, #c);   \
      ++fails;                                                       \
    }                                                                \
  } while (0)

// first fit over an occupancy map: lowest offset of a run of n free units
static bool model_first_fit(const std::vector<char>& used, size_t n, size_t* off) {
  size_t run = 0;
  for (size_t i = 0; i < used.size(); ++i) {
    run = used[i] ? 0 : run + 1;
    if (run == n) {
      *off = i + 1 - n;
      return true;
    }
  }
  return false;
}

// the holes must be exactly the maximal free runs of the model
static void check_holes(const fd::Arena& a, const std::vector<char>& used) {
  std::vector<std::pair<size_t, size_t>> runs;
  for (size_t i = 0; i < used.size();) {
    if (used[i]) { ++i; continue; }
    size_t j = i;
    while (j < used.size() && !used[j]) ++j;
    runs.push_back({i, j - i});
    i = j;
  }
  CHECK(runs.size() == a.holes().size());
  size_t k = 0;
  for (const auto& h : a.holes()) {
    if (k < runs.size()) CHECK(h.first == runs[k].first && h.second == runs[k].second);
    ++k;
  }
}

int main() {
  {  // fixed sequence: first fit, exact fit, merges on both sides
    fd::Arena a(100);
    size_t o1, o2, o3, o4;
    CHECK(a.alloc(30, &o1) && o1 == 0);
    CHECK(a.alloc(30, &o2) && o2 == 30);
    CHECK(a.alloc(30, &o3) && o3 == 60);
    CHECK(!a.alloc(11, &o4));             // only 10 left
    CHECK(a.alloc(10, &o4) && o4 == 90);  // exact fit of the tail
    CHECK(a.holes().empty());
    a.release(o2, 30);                    // hole in the middle
    size_t o5;
    CHECK(a.alloc(20, &o5) && o5 == 30);  // first fit takes it
    CHECK(a.holes().size() == 1 && a.holes().begin()->first == 50);
    a.release(o1, 30);                    // [0,30) and [50,60): two holes
    CHECK(a.holes().size() == 2);
    a.release(o5, 20);                    // merges with both neighbours: [0,60)
    CHECK(a.holes().size() == 1 && a.holes().begin()->second == 60);
    a.release(o3, 30);
    a.release(o4, 10);
    CHECK(a.holes().size() == 1 && a.holes().begin()->first == 0 &&
          a.holes().begin()->second == 100);
    size_t z = 12345;
    CHECK(!a.alloc(0, &z) && z == 12345);  // zero bytes: refused, offset untouched
    fd::Arena empty(0);
    CHECK(!empty.alloc(1, &z) && empty.holes().empty());
  }
  {  // random stress against the model
    const size_t size = 4096;
    std::mt19937_64 rng(7);
    for (int trial = 0; trial < 20; ++trial) {
      fd::Arena a(size);
      std::vector<char> used(size, 0);
      std::vector<std::pair<size_t, size_t>> live;
      for (int op = 0; op < 4000; ++op) {
        const bool do_alloc = live.empty() || (rng() % 100) < 55;
        if (do_alloc) {
          // sizes from 1 to 600 units, small ones more likely
          const size_t n = 1 + (rng() % 600) * (rng() % 600) / 600;
          size_t want = 0, got = 0;
          const bool m = model_first_fit(used, n, &want);
          const bool ok = a.alloc(n, &got);
          CHECK(m == ok);
          if (ok && m) {
            CHECK(got == want);
            for (size_t i = got; i < got + n; ++i) {
              CHECK(!used[i]);  // never overlaps a live block
              used[i] = 1;
            }
            live.push_back({got, n});
          }
        } else {
          const size_t k = rng() % live.size();
          a.release(live[k].first, live[k].second);
          for (size_t i = live[k].first; i < live[k].first + live[k].second; ++i) used[i] = 0;
          live[k] = live.back();
          live.pop_back();
        }
        if (op % 97 == 0) check_holes(a, used);
        if (fails) break;
      }
      for (const auto& b : live) a.release(b.first, b.second);
      CHECK(a.holes().size() == 1 && a.holes().begin()->first == 0 &&
            a.holes().begin()->second == size);
      if (fails) break;
    }
  }
  if (fails) {
    printf("%d failures\n", fails);
    return 1;
  }
  printf("ok\n");
  return 0;
}
