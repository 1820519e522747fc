// The server's device-memory allocator (DevCache in the serving source),
// compiled on the host against stand-ins for the HIP calls it makes and
// driven by a random sequence of allocations and releases of every size
// class, with a device that runs out of memory.  Checked: every block lies
// inside one slab and overlaps no other live block; the free and live spans
// tile the slabs exactly; no two adjacent free spans of one slab stay
// unmerged; everything is free at the end.  The test that builds this file
// extracts the allocator's source and includes it as DEVCACHE_SRC.

#include <cstdio>
#include <cstdlib>
#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <random>
#include <unordered_map>
#include <vector>
#include <algorithm>
// stand-ins for the HIP runtime: device addresses are numbers handed out
// from a fixed capacity, events complete at random
typedef int hipError_t; typedef void* hipStream_t; typedef int* hipEvent_t;
enum { hipSuccess = 0, hipErrorOutOfMemory = 2, hipErrorNotReady = 600 };
static size_t g_cap = (size_t)64 << 30, g_used = 0;
static std::map<char*, size_t> g_allocs;
static char* g_next = (char*)0x100000000000ull;
hipError_t hipMalloc(void** p, size_t n) { if (g_used + n > g_cap) return hipErrorOutOfMemory; *p = g_next; g_allocs[g_next] = n; g_next += (n + 4095) / 4096 * 4096 + 4096; g_used += n; return hipSuccess; }
hipError_t hipFree(void* p) { auto it = g_allocs.find((char*)p); if (it == g_allocs.end()) { printf("BAD FREE\n"); exit(1);} g_used -= it->second; g_allocs.erase(it); return hipSuccess; }
hipError_t hipGetLastError() { return 0; }
hipError_t hipEventCreateWithFlags(hipEvent_t* e, int) { *e = new int(0); return 0; }
hipError_t hipEventDestroy(hipEvent_t e) { delete e; return 0; }
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return 0; }
hipError_t hipEventQuery(hipEvent_t) { return (rand() & 1) ? hipSuccess : hipErrorNotReady; }
hipError_t hipEventSynchronize(hipEvent_t) { return 0; }
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, int) { return 0; }
hipError_t hipStreamSynchronize(hipStream_t) { return 0; }
hipError_t hipDeviceSynchronize() { return 0; }
#define hipEventDisableTiming 2
#include DEVCACHE_SRC

int main() {
  std::mt19937_64 rng(7);
  DevCache c;
  std::vector<std::pair<char*, size_t>> held;
  for (int it = 0; it < 200000; ++it) {
    if (held.empty() || (rng() % 100) < 55) {
      size_t n;
      const int k = rng() % 10;
      if (k < 6) n = 1 + rng() % (1 << 20);
      else if (k < 9) n = (size_t)(1 + rng() % 512) << 20;
      else n = (size_t)(1 + rng() % 16) << 30;
      char* p = (char*)c.alloc(n, nullptr);
      if (!p) continue;
      // inside a slab, no overlap with held blocks
      bool ok = false;
      for (auto& kv : g_allocs) if (p >= kv.first && p + n <= kv.first + kv.second) ok = true;
      if (!ok) { printf("OUTSIDE SLAB at %d\n", it); return 1; }
      for (auto& h : held) if (p < h.first + h.second && h.first < p + n) { printf("OVERLAP at %d\n", it); return 1; }
      held.push_back({p, n});
    } else {
      size_t k = rng() % held.size();
      c.release(held[k].first, nullptr);
      held[k] = held.back(); held.pop_back();
    }
    if (it % 20000 == 0) {
      // free spans + live spans tile every slab exactly
      size_t slab_tot = 0, span_tot = 0, live_tot = 0;
      for (auto& sl : c.slabs) slab_tot += sl->n;
      for (auto& kv : c.free_) span_tot += kv.second.n;
      for (auto& kv : c.live) live_tot += kv.second.first;
      if (slab_tot != span_tot + live_tot) { printf("ACCOUNTING %zu != %zu + %zu at %d\n", slab_tot, span_tot, live_tot, it); return 1; }
      if (c.by_size.size() != c.free_.size()) { printf("INDEX MISMATCH\n"); return 1; }
      // adjacent free spans in one slab must have been merged
      char* prev_end = nullptr; DevCache::Slab* prev_slab = nullptr;
      for (auto& kv : c.free_) {
        if (kv.first == prev_end && kv.second.slab == prev_slab) { printf("UNMERGED at %d\n", it); return 1; }
        prev_end = kv.first + kv.second.n; prev_slab = kv.second.slab;
      }
    }
  }
  for (auto& h : held) c.release(h.first, nullptr);
  size_t span_tot = 0, slab_tot = 0;
  for (auto& kv : c.free_) span_tot += kv.second.n;
  for (auto& sl : c.slabs) slab_tot += sl->n;
  printf("ok: slabs %zu, free spans %zu (%zu bytes of %zu), live %zu\n", c.slabs.size(), c.free_.size(), span_tot, slab_tot, c.live.size());
  return span_tot == slab_tot ? 0 : 1;
}
