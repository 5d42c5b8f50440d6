// Host-only checks of the serving engine's FIFO ring allocator: randomized
// alloc/release sequences against an explicit model of the live blocks, plus
// hand-made wrap and out-of-order cases.  Exit status 0 and "OK" on success.
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <vector>

#include "../../paper_1512_06637_amd/csrc/gv_arena.h"

using gv::RingAlloc;

#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      std::fprintf(stderr, "FAIL line %d: %s\n", __LINE__, #c);  \
      std::exit(1);                                                \
    }                                                              \
  } while (0)

static void no_overlap(const std::map<size_t, size_t>& live, size_t off, size_t len, size_t cap) {
  CHECK(off % RingAlloc::kAlign == 0);
  CHECK(off + len <= cap);
  for (auto& kv : live) CHECK(off + len <= kv.first || kv.first + kv.second <= off);
}

int main() {
  const size_t A = RingAlloc::kAlign;
  // hand-made cases
  {
    RingAlloc r(10 * A);
    CHECK(r.capacity() == 10 * A);
    CHECK(r.alloc(0) == RingAlloc::npos);
    CHECK(r.alloc(11 * A) == RingAlloc::npos);
    size_t a = r.alloc(4 * A), b = r.alloc(4 * A);
    CHECK(a == 0 && b == 4 * A);
    CHECK(r.alloc(3 * A) == RingAlloc::npos);  // 2 A left at the end, nothing before a
    CHECK(r.release(b));                        // b is younger than a: space stays held
    CHECK(r.in_use() == 8 * A);
    CHECK(r.alloc(3 * A) == RingAlloc::npos);
    CHECK(r.release(a));  // both gone: ring empties and restarts at 0
    CHECK(r.in_use() == 0 && r.blocks() == 0);
    CHECK(r.alloc(10 * A) == 0);
    CHECK(r.release(0));
    // wrap: a [0,4) b [4,8); release a; c needs 3 A: [8,10) too short -> pad, c at 0
    a = r.alloc(4 * A);
    b = r.alloc(4 * A);
    CHECK(r.release(a));
    size_t c = r.alloc(3 * A);
    CHECK(c == 0);
    CHECK(r.in_use() == 4 * A + 2 * A + 3 * A);
    CHECK(r.alloc(2 * A) == RingAlloc::npos);  // [3, 4) only
    CHECK(r.alloc(1) == 3 * A);                // rounds up to one unit
    CHECK(!r.release(5 * A));                  // not a block start
    CHECK(r.release(b));                       // b and the pad go
    CHECK(r.in_use() == 4 * A);
    CHECK(r.alloc(6 * A) == 4 * A);
  }
  // randomized against a model
  std::mt19937_64 rng(1512066370ull);
  for (int trial = 0; trial < 200; ++trial) {
    const size_t cap = (1 + rng() % 64) * A;
    RingAlloc r(cap);
    std::map<size_t, size_t> live;  // off -> rounded len
    std::vector<size_t> order;      // allocation order of live blocks
    size_t fails = 0, allocs = 0;
    for (int step = 0; step < 4000; ++step) {
      if (live.empty() || rng() % 3 != 0) {
        size_t len = 1 + rng() % (cap / 2 + 1);
        size_t off = r.alloc(len);
        if (off == RingAlloc::npos) {
          ++fails;
          CHECK(!live.empty());  // an empty ring always fits len <= cap
          continue;
        }
        ++allocs;
        size_t rl = RingAlloc::round_up(len);
        no_overlap(live, off, rl, cap);
        live[off] = rl;
        order.push_back(off);
      } else {
        size_t k = rng() % order.size();
        size_t off = order[k];
        order.erase(order.begin() + k);
        CHECK(r.release(off));
        CHECK(!r.release(off));  // twice: no
        live.erase(off);
      }
      size_t sum = 0;
      for (auto& kv : live) sum += kv.second;
      CHECK(r.in_use() >= sum && r.in_use() <= cap);
      if (live.empty()) CHECK(r.in_use() == 0 && r.blocks() == 0);
    }
    CHECK(allocs > 0);
    (void)fails;
  }
  std::printf("OK\n");
  return 0;
}
