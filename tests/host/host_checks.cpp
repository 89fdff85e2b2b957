// Host-only parts of the library built alone with AddressSanitizer and
// UndefinedBehaviorSanitizer (tests/test_host_sanitizers.py): the Daubechies
// spectral factorisation, the work-item block scheduler and the serving
// arena's free list, each checked against a brute-force model on random
// inputs. Prints "host checks ok" and exits 0 on success.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "host/arena.hpp"
#include "host/daubechies.hpp"
#include "host/schedule.hpp"

namespace {

int failures = 0;

void check(bool ok, const char* what, long a = 0, long b = 0) {
  if (!ok) {
    std::fprintf(stderr, "FAIL: %s (%ld, %ld)\n", what, a, b);
    ++failures;
  }
}

struct Item { int x, y, z, w; };

// Daubechies filters: sum h = sqrt 2, even-shift orthonormality, N vanishing
// moments of the high-pass g_k = (-1)^k h_{2N-1-k}.
void daubechies() {
  for (int N = 1; N <= 8; ++N) {
    double h[16] = {};
    check(pr::host::daubechies_filter(N, h), "factorisation converges", N);
    double s = 0;
    for (int k = 0; k < 2 * N; ++k) s += h[k];
    check(std::fabs(s - std::sqrt(2.0)) < 1e-13, "sum h = sqrt 2", N);
    for (int m = 0; m < N; ++m) {
      double c = 0;
      for (int k = 0; k + 2 * m < 2 * N; ++k) c += h[k] * h[k + 2 * m];
      check(std::fabs(c - (m == 0 ? 1.0 : 0.0)) < 1e-13, "orthonormal shifts", N, m);
    }
    for (int p = 0; p < N; ++p) {
      double mom = 0;
      for (int k = 0; k < 2 * N; ++k) mom += ((k & 1) ? -1.0 : 1.0) * h[2 * N - 1 - k] * std::pow(double(k), p);
      check(std::fabs(mom) < 1e-9 * std::pow(2.0 * N, p), "vanishing moments", N, p);
    }
  }
  double h[16];
  check(!pr::host::daubechies_filter(0, h) && !pr::host::daubechies_filter(9, h), "orders outside 1..8 refused");
}

// Scheduler: every item exactly once, block ranges contiguous and ordered,
// .w the item index; with few items per block the LPT bound holds.
void schedule() {
  std::mt19937_64 rng(7);
  for (int trial = 0; trial < 300; ++trial) {
    const int G = 1 + static_cast<int>(rng() % 64);
    const int n = static_cast<int>(rng() % (20 * G + 1));
    std::vector<Item> items(n);
    int64_t pos = 0;
    for (int i = 0; i < n; ++i) {
      const int len = static_cast<int>(rng() % 9000);
      items[i] = Item{static_cast<int>(rng() % 1000), static_cast<int>(pos), static_cast<int>(pos + len), -1};
      pos += len;
    }
    const int64_t overhead = static_cast<int64_t>(rng() % 500);
    std::vector<Item> sched;
    std::vector<int32_t> off;
    pr::lpt_schedule(items, G, overhead, sched, off);
    check(static_cast<int>(sched.size()) == n, "every item scheduled", n, static_cast<long>(sched.size()));
    check(static_cast<int>(off.size()) == G + 1 && off[0] == 0 && off[G] == n, "block offsets", G);
    std::vector<int> seen(n, 0);
    int64_t maxload = 0, total = 0, maxcost = 0;
    for (int b = 0; b < G && static_cast<int>(off.size()) == G + 1; ++b) {
      check(off[b] <= off[b + 1], "offsets ordered", b);
      int64_t load = 0;
      for (int k = off[b]; k < off[b + 1]; ++k) {
        const Item e = sched[k];
        check(e.w >= 0 && e.w < n, "entry index in range", e.w);
        if (e.w < 0 || e.w >= n) continue;
        ++seen[e.w];
        const Item& o = items[e.w];
        check(e.x == o.x && e.y == o.y && e.z == o.z, "entry copies its item", e.w);
        const int64_t c = (o.z - o.y) + overhead;
        load += c;
        maxcost = c > maxcost ? c : maxcost;
      }
      total += load;
      maxload = load > maxload ? load : maxload;
    }
    for (int i = 0; i < n; ++i) check(seen[i] == 1, "each item once", i, seen[i]);
    if (n < 8 * G && n > 0) check(maxload <= total / G + maxcost, "LPT bound", maxload, total / G + maxcost);
  }
  std::vector<Item> none, sched;
  std::vector<int32_t> off;
  pr::lpt_schedule(none, 0, 0, sched, off);
  check(sched.empty() && off.size() == 1, "no blocks");
}

// Arena: random alloc/release against a byte map; blocks never overlap, stay
// inside the arena, first fit is the lowest offset, and a fully released
// arena is one block again.
void arena() {
  std::mt19937_64 rng(11);
  for (int trial = 0; trial < 50; ++trial) {
    const size_t size = 1 + rng() % 5000;
    pr::ArenaFreeList fl;
    fl.reset(size);
    std::vector<int> owner(size, -1);
    struct Live { size_t off, len; };
    std::vector<Live> live;
    for (int step = 0; step < 400; ++step) {
      if (live.empty() || rng() % 3) {
        const size_t len = 1 + rng() % (size / 4 + 1);
        size_t off = 0;
        // the model: lowest offset with len free bytes
        size_t want = size;
        for (size_t a = 0; a + len <= size; ++a) {
          bool ok = true;
          for (size_t q = a; q < a + len; ++q)
            if (owner[q] >= 0) { ok = false; a = q; break; }
          if (ok) { want = a; break; }
        }
        const bool got = fl.alloc(len, &off);
        check(got == (want < size), "alloc succeeds exactly when a run fits", static_cast<long>(len));
        if (!got) continue;
        check(off == want, "first fit", static_cast<long>(off), static_cast<long>(want));
        check(off + len <= size, "inside the arena", static_cast<long>(off + len));
        for (size_t q = off; q < off + len && q < size; ++q) {
          check(owner[q] < 0, "no overlap", static_cast<long>(q));
          owner[q] = static_cast<int>(live.size());
        }
        live.push_back(Live{off, len});
      } else {
        const size_t k = rng() % live.size();
        const Live l = live[k];
        fl.release(l.off, l.len);
        for (size_t q = l.off; q < l.off + l.len; ++q) owner[q] = -1;
        live.erase(live.begin() + static_cast<long>(k));
        for (size_t q = 0; q < size; ++q)
          if (owner[q] > static_cast<int>(k)) --owner[q];
      }
      size_t free_model = 0;
      for (size_t q = 0; q < size; ++q) free_model += owner[q] < 0;
      check(fl.free_bytes() == free_model, "free bytes", static_cast<long>(fl.free_bytes()), static_cast<long>(free_model));
      // free blocks are maximal: no two adjacent
      size_t prev_end = static_cast<size_t>(-1);
      for (const auto& kv : fl.blocks()) {
        check(kv.first != prev_end, "adjacent free blocks merged", static_cast<long>(kv.first));
        prev_end = kv.first + kv.second;
      }
    }
    for (const Live& l : live) fl.release(l.off, l.len);
    check(fl.blocks().size() == 1 && fl.largest() == size, "fully released arena is one block");
  }
  pr::ArenaFreeList fl;
  fl.reset(100);
  size_t off = 0;
  check(!fl.alloc(0, &off), "zero-byte request refused");
  check(!fl.alloc(101, &off), "oversize request refused");
}

}  // namespace

int main() {
  daubechies();
  schedule();
  arena();
  if (failures) {
    std::fprintf(stderr, "%d host check(s) failed\n", failures);
    return 1;
  }
  std::printf("host checks ok\n");
  return 0;
}
