// Admission decision of the serving loop (plain C++, no device code): which
// queued requests join the next group, given their memory bounds, the
// reserved memory and the budget.
//
// Rules:
//   - requests are considered in arrival order; a request whose bound is not
//     known yet stops the scan;
//   - a request fits if reserved + bound <= budget; fitting requests join the
//     group (at most max_batch, at most `slots`);
//   - a request whose bound exceeds exact_above (at most the budget: a large
//     request's upper bound can reserve several times what it uses) is sized
//     exactly first ("probe"), and only when it is at the head of the queue
//     and the group is empty: at most one exactly planned request waits at
//     any time, so the memory its plan holds cannot keep a second such
//     request out forever;
//   - an exactly planned request runs alone;
//   - later requests may pass the oldest request that does not fit, but each
//     pass is counted on it, and after max_bypass passes nothing is admitted
//     behind it until it fits: as running requests finish and are released,
//     it is admitted.
#pragma once

#include <stdint.h>

#include <cstddef>
#include <vector>

namespace mgsrv {

struct QItem {
  int64_t bound;  // bytes to reserve (< 0: not known yet)
  bool pre;       // sized exactly and planned: bound is exact, runs alone
  int skipped;    // later requests admitted ahead of it
};

struct Decision {
  std::vector<size_t> admit;  // queue positions, in order
  long probe = -1;            // queue position to size exactly (0 or -1)
};

inline Decision admit_pass(std::vector<QItem>& q, int64_t reserved, int64_t budget, int slots,
                           int max_batch, int max_bypass, int64_t exact_above = -1) {
  Decision d;
  if (exact_above < 0 || exact_above > budget) exact_above = budget;
  const size_t none = (size_t)-1;
  size_t blocker = none;
  for (size_t i = 0; i < q.size(); ++i) {
    if ((int)d.admit.size() >= max_batch || slots <= 0) break;
    QItem& r = q[i];
    if (r.bound < 0) break;
    const bool oversized = r.bound > exact_above && !r.pre;
    if (oversized && i == 0 && d.admit.empty()) {
      d.probe = 0;
      break;
    }
    const bool fits = !oversized && !(r.pre && !d.admit.empty()) && reserved + r.bound <= budget;
    if (fits) {
      if (blocker != none) q[blocker].skipped++;
      d.admit.push_back(i);
      reserved += r.bound;
      --slots;
      if (r.pre) break;
      continue;
    }
    if (blocker == none) blocker = i;
    if (q[blocker].skipped >= max_bypass) break;
  }
  return d;
}

}  // namespace mgsrv
