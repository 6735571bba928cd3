// Host check of the persistent apply's work plan (cpm::plan_pipe): for random
// work lists, costs and grid sizes, every work item is taken by exactly one
// workgroup, each workgroup only takes items of its own XCD's eighth of the
// list, and the reordered list is a permutation of the input that keeps each
// item inside its eighth. Exit status 0 when all cases pass.
#include <cstdio>
#include <random>
#include <vector>

#include "../../paper_2110_06322_amd/csrc/common.h"

using cpm::PipeSpan;
using cpm::WorkItem;

int main() {
  std::mt19937 rng(12345);
  int bad = 0;
  for (int trial = 0; trial < 300; ++trial) {
    // both regimes: cost-balanced lists and long lists walked with a stride
    const int n = trial < 150 ? (int)(rng() % 3000) : (int)(rng() % 20000);
    const int grid = 8 * (1 + (int)(rng() % 80));
    std::vector<WorkItem> w(n);
    std::vector<int32_t> cost(n);
    for (int i = 0; i < n; ++i) {
      w[i] = WorkItem{(int32_t)(rng() % 3), i};
      cost[i] = (int32_t)(rng() % 900);
    }
    std::vector<PipeSpan> plan;
    cpm::plan_pipe(w, cost, n ? grid : 0, plan);
    if (n == 0) {
      if (!plan.empty()) ++bad;
      continue;
    }
    if ((int)plan.size() != grid || (int)w.size() != n) {
      ++bad;
      continue;
    }
    std::vector<int> taken(n, 0);
    for (int b = 0; b < grid; ++b) {
      const PipeSpan& s = plan[b];
      const int x = b & 7;
      const int lo = (int)((int64_t)n * x / 8), hi = (int)((int64_t)n * (x + 1) / 8);
      if (s.step <= 0 || (s.first < s.end && (s.first < lo || s.end > hi))) {
        ++bad;
        break;
      }
      for (int p = s.first; p < s.end; p += s.step) taken[p]++;
    }
    for (int i = 0; i < n; ++i)
      if (taken[i] != 1) {
        ++bad;
        break;
      }
    std::vector<int> count(n, 0);
    for (const WorkItem& it : w)
      if (it.idx >= 0 && it.idx < n) count[it.idx]++;
    for (int i = 0; i < n; ++i)
      if (count[i] != 1) {
        ++bad;
        break;
      }
    for (int x = 0; x < 8; ++x) {
      const int lo = (int)((int64_t)n * x / 8), hi = (int)((int64_t)n * (x + 1) / 8);
      bool ok = true;
      for (int p = lo; p < hi && ok; ++p) ok = w[p].idx >= lo && w[p].idx < hi;
      if (!ok) {
        ++bad;
        break;
      }
    }
  }
  std::printf("plan_pipe cases failed: %d\n", bad);
  return bad != 0;
}
