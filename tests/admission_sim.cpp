// Host simulation of the serving loop's admission (the rule the server runs,
// from the package's admission.h) against a fake executor: requests arrive,
// get memory bounds, oversized ones are sized exactly ("probe"), groups run
// on a fixed number of streams for a simulated time, finished requests are
// released at once.  Prints one line per scenario:
//   <name> completed rejected deadlock max_c_over_budget max_wait_passes
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <random>
#include <vector>

#include "admission.h"

struct Req {
  double arrival;
  int64_t bound, exact_c, plan;  // bytes
  double service;                // seconds on the device
  bool pre = false, done = false, rejected = false;
  int skipped = 0;
  int64_t held = 0;
};

struct Group {
  std::vector<int> ids;
  double end;
  int64_t plan;
  bool probe;
};

static void run(const char* name, std::vector<Req> R, int64_t budget, int streams, int max_batch,
                int max_bypass, int slots_max, int64_t exact_above = -1) {
  std::deque<int> q;
  std::vector<Group> running;
  int64_t reserved = 0, c_held = 0, c_max = 0;
  int nrun = 0, completed = 0, rejected = 0;
  size_t next = 0;
  double t = 0;
  int passes_waiting_max = 0;
  std::vector<int> passes_waiting(R.size(), 0);
  bool deadlock = false;
  for (int guard = 0; guard < 10000000; ++guard) {
    // finish groups that end by t
    for (size_t g = 0; g < running.size();) {
      if (running[g].end <= t) {
        Group G = running[g];
        running.erase(running.begin() + g);
        if (G.probe) {
          Req& r = R[G.ids[0]];
          if (r.exact_c + r.plan > budget) {
            r.rejected = true;
            ++rejected;
            q.erase(std::find(q.begin(), q.end(), G.ids[0]));
          } else {
            r.pre = true;
            r.bound = r.exact_c;
            reserved += r.plan;
          }
        } else {
          reserved -= G.plan;
          nrun -= (int)G.ids.size();
          for (int id : G.ids) {  // released at once
            reserved -= R[id].held;
            c_held -= R[id].exact_c;
            R[id].done = true;
            ++completed;
          }
        }
      } else {
        ++g;
      }
    }
    while (next < R.size() && R[next].arrival <= t) q.push_back((int)next++);
    // one admission pass per free stream
    bool launched = false;
    while ((int)running.size() < streams && !q.empty()) {
      std::vector<mgsrv::QItem> items;
      for (int id : q) items.push_back({R[id].bound, R[id].pre, R[id].skipped});
      mgsrv::Decision d = mgsrv::admit_pass(items, reserved, budget, slots_max - nrun, max_batch,
                                            max_bypass, exact_above);
      for (size_t i = 0; i < items.size(); ++i) R[q[i]].skipped = items[i].skipped;
      if (d.probe >= 0) {
        running.push_back({{q[0]}, t + 0.001, 0, true});
        launched = true;
        break;  // the probe holds its stream; the queue head stays
      }
      if (d.admit.empty()) break;
      Group G{{}, t, 0, false};
      double svc = 0;
      for (size_t i : d.admit) {
        Req& r = R[q[i]];
        G.ids.push_back(q[i]);
        if (!r.pre) G.plan += r.plan;
        else reserved -= r.plan, G.plan += r.plan;  // its plan moves to the group
        reserved += r.exact_c;
        r.held = r.exact_c;
        c_held += r.exact_c;
        svc += r.service;
      }
      reserved += G.plan;
      G.end = t + svc;
      nrun += (int)G.ids.size();
      std::deque<int> rest;
      for (size_t i = 0, k = 0; i < q.size(); ++i) {
        if (k < d.admit.size() && d.admit[k] == i) ++k;
        else rest.push_back(q[i]);
      }
      q.swap(rest);
      running.push_back(G);
      launched = true;
      c_max = std::max(c_max, c_held);
    }
    for (int id : q) passes_waiting_max = std::max(passes_waiting_max, ++passes_waiting[id]);
    // advance to the next event
    double tn = 1e300;
    for (auto& G : running) tn = std::min(tn, G.end);
    if (next < R.size()) tn = std::min(tn, R[next].arrival);
    if (tn == 1e300) {
      if (!q.empty()) deadlock = true;
      break;
    }
    if (!launched || tn > t) t = std::max(t, tn);
  }
  std::printf("%s %d %d %d %lld %d\n", name, completed, rejected, deadlock ? 1 : 0,
              (long long)(c_max - budget), passes_waiting_max);
}

int main() {
  const int64_t GB = 1000000000LL;
  std::mt19937_64 rng(12345);
  std::uniform_real_distribution<double> U(0.0, 1.0);
  // 1. the serving mix: many small requests and a few whose bounds exceed
  //    the budget but whose exact sizes fit; plans of the big ones hold 10 GB
  {
    std::vector<Req> R;
    double t = 0;
    for (int i = 0; i < 400; ++i) {
      t += -std::log(1.0 - U(rng)) / 20.0;
      Req r{};
      r.arrival = t;
      if (i % 25 == 3 || i % 25 == 4) {
        r.exact_c = (int64_t)(118 * GB + U(rng) * 4 * GB);
        r.bound = 3 * r.exact_c;
        r.plan = 10 * GB;
        r.service = 0.6;
      } else {
        r.exact_c = (int64_t)(U(rng) * 2 * GB);
        r.bound = 2 * r.exact_c + 1;
        r.plan = GB / 10;
        r.service = 0.01;
      }
      R.push_back(r);
    }
    run("mix", R, 140 * GB, 2, 32, 8, 64);
    // the same under a budget that holds two big requests exactly, with
    // every request whose bound exceeds a quarter of it sized exactly first
    run("mix_quarter", R, 280 * GB, 2, 32, 8, 64, 70 * GB);
  }
  // 2. two oversized requests back to back, each fitting only alone
  {
    std::vector<Req> R;
    for (int i = 0; i < 6; ++i) {
      Req r{};
      r.arrival = 0.0;
      r.exact_c = 125 * GB;
      r.bound = 400 * GB;
      r.plan = 10 * GB;
      r.service = 0.5;
      R.push_back(r);
    }
    run("oversized_pair", R, 140 * GB, 2, 32, 8, 64);
  }
  // 3. a request too large even exactly is rejected; the rest complete
  {
    std::vector<Req> R;
    for (int i = 0; i < 30; ++i) {
      Req r{};
      r.arrival = 0.001 * i;
      r.exact_c = (i == 7) ? 150 * GB : GB;
      r.bound = (i == 7) ? 300 * GB : 2 * GB;
      r.plan = GB / 10;
      r.service = 0.01;
      R.push_back(r);
    }
    run("reject_one", R, 140 * GB, 3, 4, 8, 64);
  }
  // 4. a large request under a steady stream of small ones: bypass is bounded
  {
    std::vector<Req> R;
    for (int i = 0; i < 2000; ++i) {
      Req r{};
      r.arrival = 0.0005 * i;
      r.exact_c = (i == 10) ? 100 * GB : GB;
      r.bound = (i == 10) ? 100 * GB : GB;
      r.plan = GB / 100;
      r.service = 0.02;
      R.push_back(r);
    }
    run("starvation", R, 120 * GB, 2, 8, 8, 64);
  }
  return 0;
}
