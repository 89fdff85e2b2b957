// Block schedule of gridding/degridding work items (host, plain C++; also
// built alone with sanitizers by the CPU tests).
//
// Items are (tile, begin, end, .) records. With at least 8 items per block,
// block b takes items b, b + G, b + 2G, ... (blocks running together read
// neighbouring parts of the visibility arrays); with fewer, longest first
// (cost: visibilities plus a per-item overhead, ties by index) each item goes
// to the block with the least load so far (ties to the lower block). The
// schedule is fixed at plan time, so every launch sums in the same order.
// Each scheduled entry carries its item's index in .w; block b's entries are
// sched[off[b]] .. sched[off[b + 1] - 1].
#pragma once

#include <algorithm>
#include <cstdint>
#include <functional>
#include <queue>
#include <utility>
#include <vector>

namespace pr {

template <class Item>
void lpt_schedule(const std::vector<Item>& items, int G, int64_t overhead, std::vector<Item>& sched,
                  std::vector<int32_t>& off) {
  auto entry = [&](int64_t i) {
    Item e = items[static_cast<size_t>(i)];
    e.w = static_cast<int>(i);
    return e;
  };
  const int64_t n = static_cast<int64_t>(items.size());
  sched.clear();
  off.assign(static_cast<size_t>(G > 0 ? G : 0) + 1, 0);
  if (G <= 0) return;
  if (n >= 8 * static_cast<int64_t>(G)) {
    for (int b = 0; b < G; ++b) {
      for (int64_t i = b; i < n; i += G) sched.push_back(entry(i));
      off[b + 1] = static_cast<int32_t>(sched.size());
    }
    return;
  }
  std::vector<int32_t> order(static_cast<size_t>(n));
  for (int64_t i = 0; i < n; ++i) order[static_cast<size_t>(i)] = static_cast<int32_t>(i);
  auto cost = [&](int32_t i) { return static_cast<int64_t>(items[i].z - items[i].y) + overhead; };
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return cost(a) > cost(b); });
  using Load = std::pair<int64_t, int>;
  std::priority_queue<Load, std::vector<Load>, std::greater<Load>> heap;
  for (int b = 0; b < G; ++b) heap.push(Load(0, b));
  std::vector<std::vector<int32_t>> per(static_cast<size_t>(G));
  for (int32_t i : order) {
    Load l = heap.top();
    heap.pop();
    per[static_cast<size_t>(l.second)].push_back(i);
    heap.push(Load(l.first + cost(i), l.second));
  }
  for (int b = 0; b < G; ++b) {
    for (int32_t i : per[static_cast<size_t>(b)]) sched.push_back(entry(i));
    off[static_cast<size_t>(b) + 1] = static_cast<int32_t>(sched.size());
  }
}

}  // namespace pr
