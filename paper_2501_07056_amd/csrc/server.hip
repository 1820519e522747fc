// Serving loop: products C = A * B of registered, device-resident operands
// are submitted as requests; a scheduler thread bounds each request's memory
// from the setup phase's per-row count (Section 3.1: row i of C has at most
// min(ip_i, columns) entries), admits requests while the bound fits the free
// budget and a slot is free, groups admitted requests into one batched plan
// and execution (the batch calls), and runs several such groups at once on
// separate streams.  A request whose bound exceeds a share of the budget is
// planned exactly first (precise symbolic phase, Section 2.1), reserves its
// exact size, and is rejected only if that does not fit either.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "admission.h"
#include "runtime_int.h"

using namespace mgrt;

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct SrvReq {
  int64_t id = 0;
  int32_t a = 0, b = 0;
  std::atomic<int> state{MAGNUS_REQ_QUEUED};
  std::atomic<double> t_done{0.0};
  double t_submit = 0, t_admit = 0;
  int64_t bound_bytes = -1;  // bytes reserved at admission: c_bound + plan_est
  int64_t c_bound = 0;       // C at the setup phase's nnz bound
  int64_t plan_est = 0;      // the memory its planning may use (doubled on deferral)
  int64_t held = 0;          // bytes reserved against the budget
  int64_t exact_bytes = 0, nnz = 0;
  int32_t batch_size = 0, skipped = 0;
  magnus_status_t status = MAGNUS_OK;
  void* mem = nullptr;  // C: row pointers, columns, values in one allocation
  hipStream_t mem_st = nullptr;
  magnus_csr_out_t C{};
  magnus_batch_plan_t pre = nullptr;  // exact plan of an oversized request
  int64_t pre_nnz = 0, pre_plan_bytes = 0;
  int64_t probe_wait = -1;  // reserved bytes when its exact sizing last had to wait
};

struct SrvBatch {
  magnus_batch_plan_t bp = nullptr;
  std::vector<SrvReq*> reqs;
  std::vector<int64_t> ids;  // the requests' ids (a request may be released before its group is reaped)
  int stream = 0;
  int64_t plan_bytes = 0;
  std::atomic<int> done{0};
};

// Host function enqueued after a group's launches: stamps completion.  It
// runs on a runtime thread and calls no HIP API.
void done_cb(void* p) {
  SrvBatch* B = (SrvBatch*)p;
  const double t = now_s();
  for (SrvReq* r : B->reqs) {
    r->t_done.store(t);
    r->state.store(MAGNUS_REQ_DONE);
  }
  B->done.store(1);
}

// Device memory of the server: a caching allocator over hipMalloc that
// splits and coalesces.  Memory is taken from the driver in slabs (at least
// SLAB bytes, so that small plan arrays share one), handed out best fit
// from the free spans of all slabs (a span larger than the request is
// split), and given back as a span that merges with its free neighbours in
// the same slab.  Freed memory records an event on the stream that last
// used it; a later allocation on another stream waits for it on the device
// (no host wait).  Slabs go back to the driver only when wholly free and
// hipMalloc fails, and when the server is destroyed.  (A cache of whole
// blocks reused only at up to twice their size called hipMalloc and hipFree
// hundreds of times in a serving run, seconds on the scheduler thread.)
struct DevCache {
  struct Ev {
    hipEvent_t e = nullptr;
    ~Ev() {
      if (e) (void)hipEventDestroy(e);
    }
  };
  using EvList = std::vector<std::shared_ptr<Ev>>;
  struct Slab {
    char* base;
    size_t n;
  };
  struct Span {
    size_t n;
    Slab* slab;
    EvList ev;
  };
  static constexpr size_t SLAB = (size_t)1 << 30;
  std::mutex mu;
  std::vector<std::unique_ptr<Slab>> slabs;
  std::map<char*, Span> free_;               // by address
  std::multimap<size_t, char*> by_size;      // free spans by size
  std::unordered_map<void*, std::pair<size_t, Slab*>> live;

  static size_t round(size_t n) { return (n + 255) & ~(size_t)255; }
  void erase_size(size_t n, char* p) {
    auto r = by_size.equal_range(n);
    for (auto it = r.first; it != r.second; ++it)
      if (it->second == p) {
        by_size.erase(it);
        return;
      }
  }
  static void prune(EvList& ev) {
    EvList keep;
    for (auto& e : ev)
      if (e && e->e && hipEventQuery(e->e) != hipSuccess) keep.push_back(e);
    ev.swap(keep);
  }
  void put(char* p, Span sp) {
    prune(sp.ev);
    by_size.emplace(sp.n, p);
    free_.emplace(p, std::move(sp));
  }
  // slabs wholly free go back to the driver
  void drop_free_locked() {
    for (auto it = slabs.begin(); it != slabs.end();) {
      Slab* sl = it->get();
      auto f = free_.find(sl->base);
      if (f != free_.end() && f->second.n == sl->n) {
        for (auto& e : f->second.ev)
          if (e && e->e) (void)hipEventSynchronize(e->e);
        erase_size(f->second.n, f->first);
        free_.erase(f);
        (void)hipFree(sl->base);
        it = slabs.erase(it);
      } else {
        ++it;
      }
    }
  }
  void add_slab(void* p, size_t n) {
    slabs.emplace_back(new Slab{(char*)p, n});
    put((char*)p, Span{n, slabs.back().get(), {}});
  }
  // a new slab that holds n bytes: SLAB for small requests, else n rounded
  // up to 2 MiB; when the driver refuses, the wholly free slabs go back and
  // the slab, then the exact size, is tried again
  bool grow(size_t n) {
    const size_t g = (size_t)2 << 20;
    const size_t sn = n < SLAB ? SLAB : (n + g - 1) / g * g;
    void* p = nullptr;
    if (hipMalloc(&p, sn) == hipSuccess) {
      add_slab(p, sn);
      return true;
    }
    (void)hipGetLastError();
    drop_free_locked();
    if (hipMalloc(&p, sn) == hipSuccess) {
      add_slab(p, sn);
      return true;
    }
    (void)hipGetLastError();
    if (sn != n && hipMalloc(&p, n) == hipSuccess) {
      add_slab(p, n);
      return true;
    }
    (void)hipGetLastError();
    return false;
  }
  void* alloc(size_t n, hipStream_t st) {
    n = round(n ? n : 1);
    std::lock_guard<std::mutex> lk(mu);
    auto it = by_size.lower_bound(n);
    if (it == by_size.end()) {
      if (!grow(n)) return nullptr;
      it = by_size.lower_bound(n);
      if (it == by_size.end()) return nullptr;
    }
    char* p = it->second;
    by_size.erase(it);
    auto f = free_.find(p);
    Span sp = std::move(f->second);
    free_.erase(f);
    for (auto& e : sp.ev)
      if (e && e->e && hipEventQuery(e->e) != hipSuccess) (void)hipStreamWaitEvent(st, e->e, 0);
    if (sp.n > n) put(p + n, Span{sp.n - n, sp.slab, sp.ev});
    live[p] = {n, sp.slab};
    return p;
  }
  void release(void* vp, hipStream_t st) {
    if (!vp) return;
    std::lock_guard<std::mutex> lk(mu);
    auto it = live.find(vp);
    if (it == live.end()) return;
    char* p = (char*)vp;
    Span sp{it->second.first, it->second.second, {}};
    live.erase(it);
    auto ev = std::make_shared<Ev>();
    if (hipEventCreateWithFlags(&ev->e, hipEventDisableTiming) == hipSuccess &&
        hipEventRecord(ev->e, st) == hipSuccess) {
      sp.ev.push_back(ev);
    } else {
      (void)hipStreamSynchronize(st);
    }
    // merge with the free span after it, then with the one before it, in
    // the same slab
    auto nx = free_.find(p + sp.n);
    if (nx != free_.end() && nx->second.slab == sp.slab) {
      sp.n += nx->second.n;
      sp.ev.insert(sp.ev.end(), nx->second.ev.begin(), nx->second.ev.end());
      erase_size(nx->second.n, nx->first);
      free_.erase(nx);
    }
    auto pv = free_.lower_bound(p);
    if (pv != free_.begin()) {
      --pv;
      if (pv->second.slab == sp.slab && pv->first + pv->second.n == p) {
        char* q = pv->first;
        Span m = std::move(pv->second);
        erase_size(m.n, q);
        free_.erase(pv);
        m.n += sp.n;
        m.ev.insert(m.ev.end(), sp.ev.begin(), sp.ev.end());
        put(q, std::move(m));
        return;
      }
    }
    put(p, std::move(sp));
  }
  ~DevCache() {
    std::lock_guard<std::mutex> lk(mu);
    (void)hipDeviceSynchronize();
    free_.clear();
    by_size.clear();
    live.clear();
    for (auto& sl : slabs) (void)hipFree(sl->base);
    slabs.clear();
  }
};

void* srv_alloc(size_t n, void* stream, void* ctx) {
  return ((DevCache*)ctx)->alloc(n, (hipStream_t)stream);
}
void srv_free(void* p, size_t, void* stream, void* ctx) {
  ((DevCache*)ctx)->release(p, (hipStream_t)stream);
}

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

struct magnus_server_s {
  DevCache mem;  // destroyed last
  magnus_handle_t h = nullptr;
  magnus_server_config_t cfg{};
  int64_t budget = 0;
  std::vector<magnus_csr_t> ops;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<SrvReq*> pending;
  std::unordered_map<int64_t, std::unique_ptr<SrvReq>> reqs;
  std::vector<std::unique_ptr<SrvBatch>> inflight;
  std::vector<hipStream_t> streams;
  std::vector<char> stream_busy;
  hipStream_t ctl = nullptr;
  int64_t reserved = 0;
  int running = 0;
  int64_t next_id = 1;
  bool stop = false;
  std::thread thr;
  magnus_server_stats_t stats{};
  std::deque<magnus_completion_t> completions;  // final states not yet polled
};

namespace {

int64_t val_bytes(const magnus_csr_t& X) { return X.val_type == MAGNUS_F64 ? 8 : 4; }

// Queues the final state of r for magnus_server_poll (S->mu held).
void push_completion(magnus_server_s* S, const SrvReq* r) {
  magnus_completion_t c{};
  c.request_id = r->id;
  c.state = r->state.load();
  c.status = c.state == MAGNUS_REQ_DONE ? MAGNUS_OK : r->status;
  c.nnz = c.state == MAGNUS_REQ_DONE ? r->nnz : 0;
  c.latency_ms = c.state == MAGNUS_REQ_DONE ? 1e3 * (r->t_done.load() - r->t_submit) : -1.0;
  S->completions.push_back(c);
}
int64_t col_bytes(const magnus_csr_t& X) { return X.col_type == MAGNUS_I64 ? 8 : 4; }

int64_t c_bytes(const magnus_csr_t& A, const magnus_csr_t& B, int64_t nnz) {
  return (int64_t)(a256((size_t)(A.nrows + 1) * 8) + a256((size_t)nnz * col_bytes(B)) +
                   a256((size_t)nnz * val_bytes(A)));
}

// Fail the requests of a group that never reached the device.
// Adds d to the reserved bytes (S->mu held) and keeps the peak.
void reserve(magnus_server_s* S, int64_t d) {
  S->reserved += d;
  S->stats.peak_reserved_bytes = std::max(S->stats.peak_reserved_bytes, S->reserved);
}

// A group whose planning did not fit the memory reserved for it goes back to
// the head of the queue, in order, each request with twice its planning
// estimate (a request whose bound then exceeds the exact-sizing share of the
// budget is sized exactly, alone, next).
void defer_group(magnus_server_s* S, std::vector<SrvReq*>& g, int sidx) {
  std::lock_guard<std::mutex> lk(S->mu);
  for (auto it = g.rbegin(); it != g.rend(); ++it) {
    SrvReq* r = *it;
    S->reserved -= r->held;
    r->held = 0;
    r->plan_est *= 2;
    r->bound_bytes = r->c_bound + r->plan_est;
    r->state.store(MAGNUS_REQ_QUEUED);
    S->pending.push_front(r);
  }
  S->running -= (int)g.size();
  S->stats.deferred++;
  if (sidx >= 0) S->stream_busy[sidx] = 0;
}

void fail_group(magnus_server_s* S, std::vector<SrvReq*>& g, int sidx, magnus_status_t st) {
  std::lock_guard<std::mutex> lk(S->mu);
  for (SrvReq* r : g) {
    if (r->mem) S->mem.release(r->mem, r->mem_st);
    r->mem = nullptr;
    S->reserved -= r->held;
    r->held = 0;
    r->status = st;
    r->state.store(MAGNUS_REQ_FAILED);
    S->stats.failed++;
    push_completion(S, r);
  }
  S->running -= (int)g.size();
  if (sidx >= 0) S->stream_busy[sidx] = 0;
}

// Bounds of queued requests (one batched pass on the control stream).
void compute_bounds(magnus_server_s* S, std::vector<SrvReq*>& need) {
  const int n = (int)need.size();
  std::vector<magnus_csr_t> A(n), B(n);
  for (int i = 0; i < n; ++i) {
    A[i] = S->ops[need[i]->a];
    B[i] = S->ops[need[i]->b];
  }
  std::vector<int64_t> ip(n), nb(n);
  magnus_status_t s = magnus_batch_bound(S->h, n, A.data(), B.data(), S->ctl, ip.data(), nb.data());
  std::lock_guard<std::mutex> lk(S->mu);
  for (int i = 0; i < n; ++i) {
    SrvReq* r = need[i];
    if (s != MAGNUS_OK) {
      r->status = s;
      r->state.store(MAGNUS_REQ_FAILED);
      S->stats.failed++;
      push_completion(S, r);
      continue;
    }
    // planning memory: per-row arrays, the product workspace (capped) and
    // per-chunk arrays; enforced while the group plans (plan_cap), and a
    // group that needs more is put back with twice the estimate
    const int64_t vs = val_bytes(A[i]);
    r->plan_est = 192 * (A[i].nrows + 1) +
                  std::min<int64_t>(S->cfg.workspace_cap_bytes, (2 + vs) * ip[i]) +
                  ip[i] / 64 * 48 + (1 << 20);
    r->plan_est = std::max<int64_t>(1 << 16, r->plan_est / 100 * S->cfg.plan_estimate_pct);
    r->c_bound = c_bytes(A[i], B[i], nb[i]);
    r->bound_bytes = r->c_bound + r->plan_est;
  }
  if (s != MAGNUS_OK) {
    for (auto it = S->pending.begin(); it != S->pending.end();)
      if ((*it)->state.load() == MAGNUS_REQ_FAILED) it = S->pending.erase(it);
      else ++it;
  }
}

// Exact size of a request whose bound alone exceeds the budget: it is
// planned on its own, with its planning capped at the memory not reserved,
// and keeps that plan if the plan and its exact C fit.  Returns false when it
// must wait for running groups to release memory.
bool probe_exact(magnus_server_s* S, SrvReq* r, int sidx) {
  const magnus_csr_t& A = S->ops[r->a];
  const magnus_csr_t& B = S->ops[r->b];
  int64_t room = 0;
  bool others = false;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    room = S->budget - S->reserved;
    others = S->reserved > 0;
    // after a wait, sized again only once running groups released memory
    const bool blocked = r->probe_wait > 0 && S->reserved >= r->probe_wait;
    if ((room <= 0 && others) || blocked) {
      S->stream_busy[sidx] = 0;
      r->probe_wait = S->reserved;  // > 0 here
      return false;
    }
  }
  magnus_batch_plan_t bp = nullptr;
  int64_t nnz = 0;
  magnus_plan_info_t info{};
  magnus_status_t s = MAGNUS_ERR_REJECTED;
  if (room > 0) {
    S->h->plan_cap = S->h->plan_live.load() + room;
    s = magnus_batch_plan(S->h, 1, &A, &B, nullptr, S->streams[sidx], &bp, &nnz, &info);
    S->h->plan_cap = 0;
  }
  std::lock_guard<std::mutex> lk(S->mu);
  S->stream_busy[sidx] = 0;
  // results released by the client while it planned lower the reserved
  // bytes: it waits for a release only while something else is reserved
  if (s == MAGNUS_ERR_OOM && others) {  // again once memory is released
    r->probe_wait = S->reserved > 0 ? S->reserved : -1;
    return false;
  }
  if (s == MAGNUS_ERR_OOM) s = MAGNUS_ERR_REJECTED;  // does not fit even alone
  const int64_t total = (s == MAGNUS_OK) ? c_bytes(A, B, nnz) + info.plan_bytes : 0;
  if (s == MAGNUS_OK && S->reserved + total > S->budget) {
    if (others) {  // it may fit once the running groups are done
      magnus_batch_plan_destroy(bp);
      r->probe_wait = S->reserved > 0 ? S->reserved : -1;
      return false;
    }
    s = MAGNUS_ERR_REJECTED;
  }
  if (s != MAGNUS_OK) {
    if (bp) magnus_batch_plan_destroy(bp);
    const bool rej = s == MAGNUS_ERR_REJECTED;
    r->status = s;
    r->state.store(rej ? MAGNUS_REQ_REJECTED : MAGNUS_REQ_FAILED);
    if (rej) S->stats.rejected++;
    else S->stats.failed++;
    push_completion(S, r);
    for (auto it = S->pending.begin(); it != S->pending.end(); ++it)
      if (*it == r) {
        S->pending.erase(it);
        break;
      }
    return true;
  }
  // the plan's memory is held from now on
  r->pre = bp;
  r->pre_nnz = nnz;
  r->pre_plan_bytes = info.plan_bytes;
  reserve(S, info.plan_bytes);
  r->bound_bytes = c_bytes(A, B, nnz);
  S->stats.exact_probes++;
  return true;
}

void launch_group(magnus_server_s* S, std::vector<SrvReq*> g, int sidx) {
  hipStream_t st = S->streams[sidx];
  const int n = (int)g.size();
  std::vector<magnus_csr_t> A(n), B(n);
  std::vector<magnus_csr_out_t> C(n);
  for (int i = 0; i < n; ++i) {
    A[i] = S->ops[g[i]->a];
    B[i] = S->ops[g[i]->b];
  }
  magnus_batch_plan_t bp = nullptr;
  std::vector<int64_t> nnz(n, 0);
  int64_t plan_bytes = 0;
  bool pre = (n == 1 && g[0]->pre);
  if (pre) {
    bp = g[0]->pre;
    g[0]->pre = nullptr;
    nnz[0] = g[0]->pre_nnz;
    plan_bytes = g[0]->pre_plan_bytes;  // reserved when it was planned
  } else {
    // the planning may use what was reserved for it: its allocations past
    // that fail (the plan then retries with narrower row batches), and a
    // group that still does not fit is deferred
    int64_t allowance = 0;
    for (SrvReq* r : g) allowance += r->plan_est;
    S->h->plan_cap = S->h->plan_live.load() + allowance;
    magnus_plan_info_t info{};
    magnus_status_t s =
        magnus_batch_plan(S->h, n, A.data(), B.data(), nullptr, st, &bp, nnz.data(), &info);
    S->h->plan_cap = 0;
    if (s == MAGNUS_ERR_OOM) {
      defer_group(S, g, sidx);
      return;
    }
    if (s != MAGNUS_OK) {
      fail_group(S, g, sidx, s);
      return;
    }
    plan_bytes = info.plan_bytes;
  }
  for (int i = 0; i < n; ++i) {
    SrvReq* r = g[i];
    const int64_t bytes = c_bytes(A[i], B[i], nnz[i]);
    void* p = nullptr;
    p = S->mem.alloc((size_t)bytes, st);
    if (!p) {
      // the device is short of memory although the reservation fits (its
      // memory is not only this server's): while other requests hold
      // memory the group waits for them in the queue, else it fails
      for (int k = 0; k < i; ++k) {
        S->mem.release(g[k]->mem, st);
        g[k]->mem = nullptr;
      }
      bool others = false;
      {
        std::lock_guard<std::mutex> lk(S->mu);
        int64_t mine = pre ? plan_bytes : 0;
        for (SrvReq* q : g) mine += q->held;
        others = S->reserved > mine;
      }
      if (others && pre) {
        g[0]->pre = bp;  // keeps its exact plan, which stays reserved
        std::lock_guard<std::mutex> lk(S->mu);
        S->reserved -= g[0]->held;
        g[0]->held = 0;
        g[0]->state.store(MAGNUS_REQ_QUEUED);
        S->pending.push_front(g[0]);
        S->running -= 1;
        S->stats.deferred++;
        S->stream_busy[sidx] = 0;
        return;
      }
      magnus_batch_plan_destroy(bp);
      if (others) {
        for (SrvReq* q : g) q->plan_est /= 2;  // undone by the deferral's doubling
        defer_group(S, g, sidx);
        return;
      }
      if (pre) {
        std::lock_guard<std::mutex> lk(S->mu);
        S->reserved -= plan_bytes;
      }
      fail_group(S, g, sidx, MAGNUS_ERR_OOM);
      return;
    }
    r->mem = p;
    r->mem_st = st;
    magnus_csr_out_t& O = C[i];
    O.nrows = A[i].nrows;
    O.ncols = B[i].ncols;
    O.capacity = nnz[i];
    O.rowptr_type = MAGNUS_I64;
    O.col_type = B[i].col_type;
    O.val_type = A[i].val_type;
    char* base = (char*)p;
    O.rowptr = base;
    O.col = base + a256((size_t)(A[i].nrows + 1) * 8);
    O.val = base + a256((size_t)(A[i].nrows + 1) * 8) + a256((size_t)nnz[i] * col_bytes(B[i]));
  }
  {
    // the requests' reservations become the plan and the exact C at once:
    // plan_bytes <= the planning allowance and exact <= c_bound, so the
    // change is never an increase (an exactly sized request's plan was
    // reserved when it was planned)
    std::lock_guard<std::mutex> lk(S->mu);
    int64_t delta = pre ? 0 : plan_bytes;
    for (int i = 0; i < n; ++i) {
      SrvReq* r = g[i];
      const int64_t exact = c_bytes(A[i], B[i], nnz[i]);
      delta += exact - r->held;
      r->held = exact;
      r->exact_bytes = exact;
      r->nnz = nnz[i];
      r->batch_size = n;
      r->C = C[i];
    }
    reserve(S, delta);
  }
  magnus_status_t s =
      magnus_batch_execute(S->h, bp, n, A.data(), B.data(), C.data(), MAGNUS_BATCH_EAGER, st);
  if (s != MAGNUS_OK) {
    (void)hipStreamSynchronize(st);
    magnus_batch_plan_destroy(bp);
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->reserved -= plan_bytes;
    }
    fail_group(S, g, sidx, s);
    return;
  }
  auto B_ = std::make_unique<SrvBatch>();
  B_->bp = bp;
  B_->reqs = g;
  for (SrvReq* r : g) B_->ids.push_back(r->id);
  B_->stream = sidx;
  B_->plan_bytes = plan_bytes;
  SrvBatch* raw = B_.get();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->inflight.push_back(std::move(B_));
    S->stats.batches++;
    S->stats.batched_requests += n;
  }
  if (hipLaunchHostFunc(st, done_cb, raw) != hipSuccess) {
    // no completion callback: wait here and stamp it directly
    (void)hipStreamSynchronize(st);
    done_cb(raw);
  }
}

void sched_loop(magnus_server_s* S) {
  const int window = std::max(4 * S->cfg.max_batch, 64);
  for (;;) {
    bool worked = false;
    // 1. finished groups: release their plans and streams
    std::vector<std::unique_ptr<SrvBatch>> fin;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      for (auto it = S->inflight.begin(); it != S->inflight.end();) {
        if ((*it)->done.load()) {
          fin.push_back(std::move(*it));
          it = S->inflight.erase(it);
        } else {
          ++it;
        }
      }
      for (auto& B : fin) {
        S->stream_busy[B->stream] = 0;
        S->running -= (int)B->reqs.size();
        S->reserved -= B->plan_bytes;
        S->stats.completed += (int64_t)B->reqs.size();
        for (int64_t id : B->ids) {
          auto f = S->reqs.find(id);
          if (f != S->reqs.end()) push_completion(S, f->second.get());
        }
      }
      if (S->stop && S->pending.empty() && S->inflight.empty()) break;
    }
    for (auto& B : fin) magnus_batch_plan_destroy(B->bp);
    worked |= !fin.empty();

    // 2. bounds of queued requests that have none yet
    std::vector<SrvReq*> need;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      for (SrvReq* r : S->pending) {
        if ((int)need.size() >= window) break;
        if (r->bound_bytes < 0) need.push_back(r);
      }
    }
    if (!need.empty()) {
      compute_bounds(S, need);
      worked = true;
    }

    // 3. admission into one group on an idle stream
    std::vector<SrvReq*> group;
    SrvReq* probe = nullptr;
    int sidx = -1;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      for (int i = 0; i < (int)S->streams.size(); ++i)
        if (!S->stream_busy[i]) {
          sidx = i;
          break;
        }
      if (sidx >= 0) {
        // the admission rules live in admission.h (tested on the host)
        std::vector<mgsrv::QItem> q;
        std::vector<SrvReq*> qr;
        for (SrvReq* r : S->pending) {
          if ((int)q.size() >= window) break;
          q.push_back({r->bound_bytes, r->pre != nullptr, r->skipped});
          qr.push_back(r);
        }
        mgsrv::Decision d = mgsrv::admit_pass(q, S->reserved, S->budget,
                                              S->cfg.max_inflight - S->running,
                                              S->cfg.max_batch, S->cfg.max_bypass,
                                              S->budget / 100 * S->cfg.exact_above_pct);
        for (size_t i = 0; i < q.size(); ++i) qr[i]->skipped = q[i].skipped;
        if (d.probe >= 0) probe = qr[(size_t)d.probe];
        for (size_t i : d.admit) {
          SrvReq* r = qr[i];
          r->held = r->bound_bytes;
          reserve(S, r->bound_bytes);
          r->t_admit = now_s();
          r->state.store(MAGNUS_REQ_RUNNING);
          group.push_back(r);
        }
        if (!group.empty()) {
          // admitted requests leave the queue (positions are ascending)
          size_t k = 0;
          std::deque<SrvReq*> rest;
          size_t pos = 0;
          for (SrvReq* r : S->pending) {
            if (k < d.admit.size() && d.admit[k] == pos) ++k;
            else rest.push_back(r);
            ++pos;
          }
          S->pending.swap(rest);
        }
        if (!group.empty() || probe) {
          S->stream_busy[sidx] = 1;
          S->running += (int)group.size();
        }
      }
    }
    if (probe) {
      worked = probe_exact(S, probe, sidx);
    } else if (!group.empty()) {
      launch_group(S, group, sidx);
      worked = true;
    }
    if (!worked) {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv.wait_for(lk, std::chrono::microseconds(100));
    }
  }
}

}  // namespace

extern "C" {

void magnus_server_config_default(magnus_server_config_t* c) {
  if (!c) return;
  memset(c, 0, sizeof(*c));
}

magnus_status_t magnus_server_create(int device, const magnus_options_t* opts,
                                     const magnus_server_config_t* cfg, magnus_server_t* out) {
  if (!out) return MAGNUS_ERR_INVALID_ARG;
  *out = nullptr;
  if (opts && opts->deterministic) return MAGNUS_ERR_INVALID_ARG;  // batch plans do not take it
  magnus_server_config_t c{};
  if (cfg) c = *cfg;
  if (c.memory_budget_bytes < 0 || c.workspace_cap_bytes < 0 || c.max_inflight < 0 ||
      c.max_batch < 0 || c.streams < 0 || c.max_bypass < 0 || c.plan_estimate_pct < 0 ||
      c.exact_above_pct < 0 || c.exact_above_pct > 100)
    return MAGNUS_ERR_INVALID_ARG;
  if (c.plan_estimate_pct == 0) c.plan_estimate_pct = 100;
  if (c.exact_above_pct == 0) c.exact_above_pct = 25;
  magnus_handle_t h = nullptr;
  magnus_status_t s = magnus_create(&h, device, opts);
  if (s != MAGNUS_OK) return s;
  if (hipSetDevice(device) != hipSuccess) {
    magnus_destroy(h);
    return MAGNUS_ERR_HIP;
  }
  if (c.memory_budget_bytes == 0) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
      magnus_destroy(h);
      return MAGNUS_ERR_HIP;
    }
    c.memory_budget_bytes = (int64_t)(fr / 2);
  }
  if (c.workspace_cap_bytes == 0) c.workspace_cap_bytes = c.memory_budget_bytes / 16;
  if (c.max_inflight == 0) c.max_inflight = 64;
  if (c.max_batch == 0) c.max_batch = 32;
  if (c.streams == 0) c.streams = 2;
  if (c.max_bypass == 0) c.max_bypass = 8;
  c.streams = std::min(c.streams, 8);
  // the CHUNKED workspace of any one plan stays within the per-request cap
  magnus_options_t o;
  magnus_options_default(&o);
  if (opts) o = *opts;
  if (o.max_workspace_bytes <= 0 || o.max_workspace_bytes > c.workspace_cap_bytes)
    o.max_workspace_bytes = c.workspace_cap_bytes;
  magnus_set_options(h, &o);
  magnus_server_s* S = new magnus_server_s();
  magnus_set_allocator(h, srv_alloc, srv_free, &S->mem);
  S->h = h;
  S->cfg = c;
  S->budget = c.memory_budget_bytes;
  S->streams.resize(c.streams, nullptr);
  S->stream_busy.assign(c.streams, 0);
  hipError_t e = hipStreamCreateWithFlags(&S->ctl, hipStreamNonBlocking);
  for (int i = 0; i < c.streams && e == hipSuccess; ++i)
    e = hipStreamCreateWithFlags(&S->streams[i], hipStreamNonBlocking);
  if (e != hipSuccess) {
    for (auto st : S->streams)
      if (st) (void)hipStreamDestroy(st);
    if (S->ctl) (void)hipStreamDestroy(S->ctl);
    magnus_destroy(h);
    delete S;
    return MAGNUS_ERR_HIP;
  }
  S->thr = std::thread([S, device] {
    (void)hipSetDevice(device);
    sched_loop(S);
  });
  *out = S;
  return MAGNUS_OK;
}

magnus_status_t magnus_server_destroy(magnus_server_t S) {
  if (!S) return MAGNUS_OK;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
    // queued requests are dropped; running ones finish
    for (SrvReq* r : S->pending) {
      r->status = MAGNUS_ERR_REJECTED;
      r->state.store(MAGNUS_REQ_REJECTED);
    }
    S->pending.clear();
  }
  S->cv.notify_all();
  if (S->thr.joinable()) S->thr.join();
  for (auto& kv : S->reqs) {
    SrvReq* r = kv.second.get();
    if (r->mem) S->mem.release(r->mem, r->mem_st);
    if (r->pre) magnus_batch_plan_destroy(r->pre);
  }
  for (auto st : S->streams) (void)hipStreamSynchronize(st);
  (void)hipStreamSynchronize(S->ctl);
  for (auto st : S->streams) (void)hipStreamDestroy(st);
  (void)hipStreamDestroy(S->ctl);
  magnus_destroy(S->h);
  delete S;
  return MAGNUS_OK;
}

magnus_status_t magnus_server_register(magnus_server_t S, const magnus_csr_t* X, int32_t* id) {
  if (!S || !X || !id) return MAGNUS_ERR_INVALID_ARG;
  magnus_status_t s = check_csr(X);
  if (s != MAGNUS_OK) return s;
  std::lock_guard<std::mutex> lk(S->mu);
  if (!S->ops.empty()) {
    const magnus_csr_t& F = S->ops[0];
    if (X->rowptr_type != F.rowptr_type || X->col_type != F.col_type || X->val_type != F.val_type)
      return MAGNUS_ERR_DTYPE;
  }
  if (X->nrows > INT32_MAX) return MAGNUS_ERR_INDEX_OVERFLOW;
  *id = (int32_t)S->ops.size();
  S->ops.push_back(*X);
  return MAGNUS_OK;
}

magnus_status_t magnus_server_submit(magnus_server_t S, int32_t a_id, int32_t b_id,
                                     int64_t* request_id) {
  if (!S || !request_id) return MAGNUS_ERR_INVALID_ARG;
  const double t = now_s();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) return MAGNUS_ERR_INVALID_ARG;
    if (a_id < 0 || b_id < 0 || a_id >= (int32_t)S->ops.size() || b_id >= (int32_t)S->ops.size())
      return MAGNUS_ERR_INVALID_ARG;
    if (S->ops[a_id].ncols != S->ops[b_id].nrows) return MAGNUS_ERR_SHAPE;
    auto r = std::make_unique<SrvReq>();
    r->id = S->next_id++;
    r->a = a_id;
    r->b = b_id;
    r->t_submit = t;
    *request_id = r->id;
    S->pending.push_back(r.get());
    S->reqs.emplace(r->id, std::move(r));
    S->stats.submitted++;
  }
  S->cv.notify_one();
  return MAGNUS_OK;
}

magnus_status_t magnus_server_query(magnus_server_t S, int64_t request_id,
                                    magnus_request_info_t* info) {
  if (!S || !info) return MAGNUS_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(request_id);
  if (it == S->reqs.end()) return MAGNUS_ERR_INVALID_ARG;
  SrvReq* r = it->second.get();
  memset(info, 0, sizeof(*info));
  info->state = r->state.load();
  info->batch_size = r->batch_size;
  info->nnz = r->nnz;
  info->bound_bytes = r->bound_bytes;
  info->exact_bytes = r->exact_bytes;
  info->queue_ms = r->t_admit > 0 ? 1e3 * (r->t_admit - r->t_submit) : -1.0;
  info->latency_ms = info->state == MAGNUS_REQ_DONE ? 1e3 * (r->t_done.load() - r->t_submit) : -1.0;
  info->status = r->status;
  return MAGNUS_OK;
}

magnus_status_t magnus_server_result(magnus_server_t S, int64_t request_id, magnus_csr_out_t* C) {
  if (!S || !C) return MAGNUS_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(request_id);
  if (it == S->reqs.end()) return MAGNUS_ERR_INVALID_ARG;
  SrvReq* r = it->second.get();
  const int st = r->state.load();
  if (st == MAGNUS_REQ_REJECTED) return MAGNUS_ERR_REJECTED;
  if (st == MAGNUS_REQ_FAILED) return r->status != MAGNUS_OK ? r->status : MAGNUS_ERR_INTERNAL;
  if (st != MAGNUS_REQ_DONE) return MAGNUS_ERR_NOT_READY;
  *C = r->C;
  return MAGNUS_OK;
}

magnus_status_t magnus_server_release(magnus_server_t S, int64_t request_id) {
  if (!S) return MAGNUS_ERR_INVALID_ARG;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(request_id);
    if (it == S->reqs.end()) return MAGNUS_ERR_INVALID_ARG;
    SrvReq* r = it->second.get();
    const int st = r->state.load();
    if (st == MAGNUS_REQ_QUEUED || st == MAGNUS_REQ_RUNNING) return MAGNUS_ERR_NOT_READY;
    // a finished request's group may still be in the in-flight list (its
    // plan not yet released), but nothing of the group reads C any more
    if (r->mem) S->mem.release(r->mem, r->mem_st);
    r->mem = nullptr;
    S->reserved -= r->held;
    r->held = 0;
    for (auto c = S->completions.begin(); c != S->completions.end(); ++c)
      if (c->request_id == request_id) {
        S->completions.erase(c);
        break;
      }
    S->reqs.erase(it);
  }
  S->cv.notify_one();
  return MAGNUS_OK;
}

magnus_status_t magnus_server_poll(magnus_server_t S, magnus_completion_t* out, int32_t max,
                                   int32_t* n) {
  if (!S || !n || max < 0 || (max > 0 && !out)) return MAGNUS_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(S->mu);
  int32_t k = 0;
  while (k < max && !S->completions.empty()) {
    out[k++] = S->completions.front();
    S->completions.pop_front();
  }
  *n = k;
  return MAGNUS_OK;
}

magnus_status_t magnus_server_get_stats(magnus_server_t S, magnus_server_stats_t* out) {
  if (!S || !out) return MAGNUS_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(S->mu);
  *out = S->stats;
  out->reserved_bytes = S->reserved;
  out->budget_bytes = S->budget;
  out->queued = (int64_t)S->pending.size();
  out->running = S->running;
  return MAGNUS_OK;
}

}  // extern "C"
