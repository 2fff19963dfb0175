// Host-only checks of the shot server's buddy allocator (fd_arena.h) and bounded
// stream pool (fd_stream_pool.h) against brute-force models.
//
// Buddy: a unit-granular occupancy map; the free blocks must always be exactly the
// maximal free aligned blocks within the roots, and each allocation must be the
// lowest sub-block of the lowest-offset free block of the smallest order that
// holds the request.
// Pool: simulated streams with completion times; every acquire is checked against
// the stated policy (reuse, lazy creation up to the bound, release of the older half
// of the completed streams, else a wait for the oldest).
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <map>
#include <random>
#include <set>
#include <vector>

#include "fd_arena.h"
#include "fd_stream_pool.h"

static int fails = 0;
#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      fprintf(stderr, "FAIL %s:%d: %s\n", __FILE__, __LINE__, #c); \
      ++fails;                                                     \
    }                                                              \
  } while (0)

// ---------------------------------------------------------------- buddy model
struct BuddyModel {
  size_t units;
  std::map<size_t, int> roots;  // unit offset -> order
  std::vector<char> used;
  explicit BuddyModel(size_t u) : units(u), used(u, 0) {
    size_t at = 0, left = u;
    while (left) {
      int o = 0;
      while (((size_t)2 << o) <= left) ++o;
      roots[at] = o;
      at += (size_t)1 << o;
      left -= (size_t)1 << o;
    }
  }
  bool all_free(size_t at, int o) const {
    for (size_t i = at; i < at + ((size_t)1 << o); ++i)
      if (used[i]) return false;
    return true;
  }
  // maximal free aligned blocks: per order, offsets (units)
  std::vector<std::set<size_t>> canonical(int max_order) const {
    std::vector<std::set<size_t>> out(max_order + 1);
    for (const auto& r : roots) collect(r.first, r.second, out);
    return out;
  }
  void collect(size_t at, int o, std::vector<std::set<size_t>>& out) const {
    if (all_free(at, o)) {
      out[o].insert(at);
      return;
    }
    if (o == 0) return;
    collect(at, o - 1, out);
    collect(at + ((size_t)1 << (o - 1)), o - 1, out);
  }
};

static void check_buddy_state(const fd::BuddyArena& b, const BuddyModel& m) {
  const auto& fb = b.free_blocks();
  const auto canon = m.canonical((int)fb.size() - 1);
  for (size_t o = 0; o < fb.size(); ++o) {
    std::set<size_t> got;
    for (size_t off : fb[o]) got.insert(off / b.unit());
    CHECK(got == canon[o]);
  }
}

static void test_buddy() {
  const size_t unit = 256;
  {  // fixed sequence on a 16-unit arena
    fd::BuddyArena b(16 * unit, unit);
    size_t a, c, d, e;
    CHECK(b.alloc(1, &a) && a == 0);               // splits 16 -> 8 -> 4 -> 2 -> 1
    CHECK(b.alloc(unit + 1, &c) && c == 2 * unit);  // 2 units
    CHECK(b.alloc(unit, &d) && d == unit);          // the buddy of the first block
    CHECK(b.alloc(8 * unit, &e) && e == 8 * unit);
    size_t f;
    CHECK(!b.alloc(5 * unit, &f));                  // needs an 8-unit block: none left
    b.release(a, 1);
    b.release(d, unit);
    b.release(c, unit + 1);                         // 0..3 merge with 4..7 into 0..7
    CHECK(b.free_blocks()[3].count(0) == 1);
    b.release(e, 8 * unit);
    CHECK(b.free_blocks()[4].size() == 1 && *b.free_blocks()[4].begin() == 0);
  }
  {  // non-power-of-two arenas: several roots that never merge with one another
    fd::BuddyArena b(13 * unit + 100, unit);        // roots 8, 4, 1 units
    CHECK(b.roots().size() == 3);
    size_t o;
    CHECK(b.alloc(8 * unit, &o) && o == 0);
    CHECK(!b.alloc(5 * unit, &o));
    CHECK(b.alloc(4 * unit, &o) && o == 8 * unit);
    CHECK(b.alloc(unit, &o) && o == 12 * unit);
    CHECK(!b.alloc(1, &o));
    fd::BuddyArena z(100, unit);                    // below one unit: nothing to hand out
    CHECK(!z.alloc(1, &o));
  }
  // random sequences against the model
  std::mt19937_64 rng(7);
  for (int trial = 0; trial < 40; ++trial) {
    const size_t units = 1 + rng() % 300;
    fd::BuddyArena b(units * unit + rng() % unit, unit);
    BuddyModel m(units);
    std::vector<std::pair<size_t, size_t>> live;  // (offset bytes, request bytes)
    for (int step = 0; step < 400; ++step) {
      if (live.empty() || rng() % 3) {
        const size_t n = 1 + rng() % (unit * (1 + rng() % 40));
        const int want = b.order_for(n);
        // model: lowest offset among free canonical blocks of the smallest order >= want
        const auto canon = m.canonical((int)b.free_blocks().size() - 1 + 1);
        bool exp_ok = false;
        size_t exp_off = 0;
        for (int o = want; o < (int)canon.size() && !exp_ok; ++o)
          if (!canon[o].empty()) {
            exp_ok = true;
            exp_off = *canon[o].begin();
          }
        size_t off = 0;
        const bool ok = b.alloc(n, &off);
        CHECK(ok == exp_ok);
        if (ok) {
          CHECK(off / unit == exp_off && off % unit == 0);
          const size_t len = (size_t)1 << want;
          CHECK(off / unit + len <= units);
          for (size_t i = off / unit; i < off / unit + len; ++i) {
            CHECK(!m.used[i]);
            m.used[i] = 1;
          }
          live.push_back({off, n});
        }
      } else {
        const size_t k = rng() % live.size();
        const auto blk = live[k];
        live.erase(live.begin() + k);
        b.release(blk.first, blk.second);
        const size_t len = (size_t)1 << b.order_for(blk.second);
        for (size_t i = blk.first / unit; i < blk.first / unit + len; ++i) m.used[i] = 0;
      }
      check_buddy_state(b, m);
    }
    for (const auto& blk : live) b.release(blk.first, blk.second);
    std::fill(m.used.begin(), m.used.end(), 0);
    check_buddy_state(b, m);  // everything merged back into the roots
    size_t nfree = 0;
    for (const auto& s : b.free_blocks()) nfree += s.size();
    CHECK(nfree == b.roots().size());
  }
}

// ---------------------------------------------------------------- pool model
struct FakeStreams {
  struct State {
    int created = 0, destroyed = 0, syncs = 0;
    long now = 0;
    std::map<int, long> done_at;  // stream -> time its work completes
  };
  using Stream = int;
  State* st;
  int fail_after = -1;
  bool create(Stream* s) {
    if (fail_after >= 0 && st->created >= fail_after) return false;
    *s = st->created++;
    st->done_at[*s] = 0;
    return true;
  }
  bool done(Stream s) { return st->done_at[s] <= st->now; }
  void sync(Stream s) {
    ++st->syncs;
    if (st->done_at[s] > st->now) st->now = st->done_at[s];  // waiting advances time
  }
  void destroy(Stream) { ++st->destroyed; }
};

static void test_pool() {
  std::mt19937_64 rng(11);
  for (int trial = 0; trial < 200; ++trial) {
    FakeStreams::State st;
    const int bound = 1 + (int)(rng() % 6);
    {
      fd::StreamPool<FakeStreams> pool(FakeStreams{&st}, bound);
      for (int step = 0; step < 300; ++step) {
        st.now += (long)(rng() % 5);
        // model of the next acquire, from the pool's state before it
        std::vector<int> act(pool.active_streams().begin(), pool.active_streams().end());
        const int idle = pool.idle();
        std::vector<int> completed;
        for (int s : act)
          if (st.done_at[s] <= st.now) completed.push_back(s);
        int s = -1;
        bool created = false;
        int synced = 0;
        const int syncs_before = st.syncs;
        CHECK(pool.acquire(&s, &created, &synced));
        if (idle > 0) {
          CHECK(!created && synced == 0);  // reuse
        } else if ((int)act.size() < bound) {
          CHECK(created && synced == 0);  // lazy creation
          CHECK(s == st.created - 1);
        } else if (completed.empty()) {
          CHECK(!created && synced == 1 && s == act[0]);  // wait for the oldest
        } else {
          const int half = ((int)completed.size() + 1) / 2;
          CHECK(!created && synced == half && s == completed[0]);
          // the released ones are the older half of the completed ones
          for (int i = 0; i < half; ++i)
            CHECK(std::find(pool.active_streams().begin(), pool.active_streams().end(),
                            completed[i]) == pool.active_streams().end() ||
                  completed[i] == s);
          for (size_t i = half; i < completed.size(); ++i)
            CHECK(std::find(pool.active_streams().begin(), pool.active_streams().end(),
                            completed[i]) != pool.active_streams().end());
        }
        // only a wait for the oldest stream synchronises; completed ones are released
        CHECK(st.syncs - syncs_before ==
              (idle == 0 && (int)act.size() >= bound && completed.empty() ? 1 : 0));
        CHECK(pool.active() <= bound && pool.live() <= bound);
        CHECK(pool.active_streams().back() == s);
        st.done_at[s] = st.now + (long)(rng() % 20);  // new work on it
      }
      CHECK(st.created <= bound);
    }
    CHECK(st.destroyed == st.created);  // the pool destroys what it made
  }
  {  // creation failure is reported, nothing is handed out
    FakeStreams::State st;
    FakeStreams ops{&st};
    ops.fail_after = 0;
    fd::StreamPool<FakeStreams> pool(ops, 3);
    int s = -1;
    CHECK(!pool.acquire(&s));
    CHECK(pool.live() == 0);
  }
}

int main() {
  test_buddy();
  test_pool();
  if (fails) {
    fprintf(stderr, "%d failure(s)\n", fails);
    return 1;
  }
  printf("ok\n");
  return 0;
}
