// Shared device helpers for the gfx950 kernels: index access, wave-level
// scans and a register bitonic sort over one 64-lane wavefront.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define MG_WAVE 64
#define MG_INLINE __device__ __forceinline__

namespace mg {

// A dispatch counts its work-items (grid x block) in 32 bits: a launch of
// 2^32 or more work-items runs a truncated grid and reports no error.
// Launches whose grid grows with the data are cut into pieces of at most
// max_grid(block) blocks.
inline int64_t max_grid(int block) { return (int64_t)(0xFFFFFFFFull / (unsigned)block); }

// -------------------------------------------------------------------------
// Index widths: A and B share a row pointer type RP and a column type CI.
// -------------------------------------------------------------------------
template <typename T>
MG_INLINE int64_t ld64(const T* p, int64_t i) { return (int64_t)p[i]; }

MG_INLINE int lane() { return (int)__lane_id(); }

// Streaming accesses for data touched once (the reordered intermediate
// product and C): non-temporal, so they do not evict B's rows and the
// accumulators' neighbours from L2 and the memory-side cache.  This is the
// role of the non-temporal stores of the reorder in Section 3.2.
// Access classes that may take the non-temporal forms (a compile-time mask:
// the hint is instruction encoding, so it cannot be chosen at run time).
constexpr int HINT_WS_STORE = 1, HINT_WS_LOAD = 2, HINT_C_STORE = 4;
#ifndef MG_NT_MASK
#define MG_NT_MASK 1
#endif
//
// All of these take pointers into device memory (global address space).  The
// compiler cannot always see that (a pointer read back from LDS or from a
// table in memory is a generic one), and then emits flat accesses, which
// count against the wait counter that LDS accesses share: every wait for an
// LDS read would also wait for the outstanding gathers.  The casts give the
// global forms.
template <typename T>
using gmem_t = __attribute__((address_space(1))) T;
template <typename T>
MG_INLINE T ld_global(const T* p) { return *(const gmem_t<T>*)p; }
template <typename T>
MG_INLINE void st_global(T* p, T v) { *(gmem_t<T>*)p = v; }
template <int CLASS, typename T>
MG_INLINE void st_stream(T* p, T v) {
  if constexpr ((MG_NT_MASK & CLASS) != 0) __builtin_nontemporal_store(v, (gmem_t<T>*)p);
  else *(gmem_t<T>*)p = v;
}
template <int CLASS, typename T>
MG_INLINE T ld_stream(const T* p) {
  if constexpr ((MG_NT_MASK & CLASS) != 0) return __builtin_nontemporal_load((const gmem_t<T>*)p);
  else return *(const gmem_t<T>*)p;
}

// Wave-wide inclusive prefix sum (64 lanes).
template <typename T>
MG_INLINE T wave_incl_scan(T v) {
#pragma unroll
  for (int d = 1; d < MG_WAVE; d <<= 1) {
    T u = __shfl_up(v, d, MG_WAVE);
    if (lane() >= d) v += u;
  }
  return v;
}

template <typename T>
MG_INLINE T wave_sum(T v) {
#pragma unroll
  for (int d = MG_WAVE / 2; d >= 1; d >>= 1) v += __shfl_xor(v, d, MG_WAVE);
  return v;
}

template <typename T>
MG_INLINE T wave_max(T v) {
#pragma unroll
  for (int d = MG_WAVE / 2; d >= 1; d >>= 1) {
    T u = __shfl_xor(v, d, MG_WAVE);
    v = u > v ? u : v;
  }
  return v;
}

template <typename T>
MG_INLINE T wave_min(T v) {
#pragma unroll
  for (int d = MG_WAVE / 2; d >= 1; d >>= 1) {
    T u = __shfl_xor(v, d, MG_WAVE);
    v = u < v ? u : v;
  }
  return v;
}

MG_INLINE uint64_t ballot(bool p) { return __ballot(p); }
MG_INLINE int popc64(uint64_t x) { return __popcll(x); }
// lanes below this one whose predicate is set
MG_INLINE int rank_below(uint64_t mask) {
  int l = lane();
  uint64_t below = (l == 0) ? 0ull : (mask & ((~0ull) >> (64 - l)));
  return __popcll(below);
}

// Runs of equal keys over consecutive active lanes (call with every lane of
// the current exec mask holding a key).  head_lane: the first lane of this
// lane's run; len: the run's length (meaningful on the head lane).  A caller
// updates a shared counter once per run instead of once per lane: lanes of a
// wave walking a sorted B row mostly fall into the same chunk, and per-lane
// atomics on one LDS word serialise.
MG_INLINE void wave_run(uint32_t key, int& head_lane, int& len) {
  const int l = lane();
  const uint32_t prev = __shfl_up(key, 1, MG_WAVE);
  const uint64_t act = __ballot(1);
  const bool h = (l == 0) || !((act >> (l - 1)) & 1ull) || prev != key;
  const uint64_t hm = __ballot(h);
  const uint64_t upto = (l == 63) ? ~0ull : ((2ull << l) - 1ull);
  head_lane = 63 - __clzll(hm & upto);
  const uint64_t above = (l == 63) ? 0ull : (~0ull << (l + 1));
  const uint64_t stop = (hm | ~act) & above;
  const int end = stop ? (__ffsll((unsigned long long)stop) - 1) : MG_WAVE;
  len = end - l;
}

// Largest index k in [lo, hi) with pre[k] <= x (pre ascending, pre[lo] <= x).
template <typename T, typename S>
MG_INLINE int upper_index(const T* pre, int lo, int hi, S x) {
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if ((S)pre[mid] <= x) lo = mid; else hi = mid;
  }
  return lo;
}

// The same over exactly 64 nondecreasing entries with pre[0] <= x (entries
// past the live ones padded with a value above every x): six fixed steps
// with no branch, so the searches of several products interleave.
template <typename T, typename S>
MG_INLINE int upper_index64(const T* pre, S x) {
  int k = 0;
#pragma unroll
  for (int step = 32; step >= 1; step >>= 1) k = ((S)pre[k + step] <= x) ? k + step : k;
  return k;
}

// -------------------------------------------------------------------------
// Lane exchange v <- v of lane (l ^ LM) without the LDS crossbar where the
// distance allows: DPP quad permutes (1, 2), DPP row rotates (4, 8) and the
// gfx950 permlane swaps (16, 32).  The lane layouts of the rotate and swap
// forms were checked against __shfl_xor on the device.
// -------------------------------------------------------------------------
template <int LM>
MG_INLINE uint32_t xshfl32(uint32_t v) {
  if constexpr (LM == 1) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, true);
  } else if constexpr (LM == 2) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, true);
  } else if constexpr (LM == 4) {
    const uint32_t a = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x124, 0xF, 0xF, true);
    const uint32_t b = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x12C, 0xF, 0xF, true);
    return (lane() & 4) ? a : b;
  } else if constexpr (LM == 8) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x128, 0xF, 0xF, true);
  } else if constexpr (LM == 16) {
    const auto q = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    return ((lane() >> 4) & 1) ? q[0] : q[1];
  } else if constexpr (LM == 32) {
    const auto q = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return (lane() < 32) ? q[1] : q[0];
  } else {
    return __shfl_xor(v, LM, MG_WAVE);
  }
}
template <int LM, typename T>
MG_INLINE T xshfl(T v) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit values");
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, xshfl32<LM>(__builtin_bit_cast(uint32_t, v)));
  } else {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint64_t lo = xshfl32<LM>((uint32_t)u), hi = xshfl32<LM>((uint32_t)(u >> 32));
    return __builtin_bit_cast(T, lo | (hi << 32));
  }
}

constexpr int ilog2c(int x) { return x <= 1 ? 0 : 1 + ilog2c(x >> 1); }

// -------------------------------------------------------------------------
// Bitonic sort of N = 64 * E keys held in blocked layout: lane l owns
// elements l*E .. l*E+E-1 in registers k[0..E-1].  Ascending.  The network
// is generated at compile time (every stage's distance is a template
// constant), and every compare-exchange is a branch-free min/max select.
// -------------------------------------------------------------------------
template <int E, int SIZE, int STRIDE, typename K>
MG_INLINE void bitonic_stage(K (&k)[E]) {
  const int l = lane();
  if constexpr (STRIDE < E) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if ((e & STRIDE) == 0) {
        // direction of this pair: bit SIZE of the element index l*E + e
        bool up;
        if constexpr (SIZE < E) up = (e & SIZE) == 0;
        else up = ((l * E) & SIZE) == 0;
        const K x = k[e], y = k[e | STRIDE];
        const K mn = x < y ? x : y, mx = x < y ? y : x;
        k[e] = up ? mn : mx;
        k[e | STRIDE] = up ? mx : mn;
      }
    }
  } else {
    constexpr int LM = STRIDE / E;
    const bool lower = (l & LM) == 0;
    const bool up = ((l * E) & SIZE) == 0;
    const bool keep_min = (lower == up);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const K p = xshfl<LM>(k[e]);
      const K mn = p < k[e] ? p : k[e], mx = p < k[e] ? k[e] : p;
      k[e] = keep_min ? mn : mx;
    }
  }
  if constexpr (STRIDE > 1) bitonic_stage<E, SIZE, STRIDE / 2>(k);
}

template <int E, int SIZE, typename K>
MG_INLINE void bitonic_merge_from(K (&k)[E]) {
  bitonic_stage<E, SIZE, SIZE / 2>(k);
  if constexpr (SIZE < MG_WAVE * E) bitonic_merge_from<E, SIZE * 2>(k);
}

template <int E, typename K>
MG_INLINE void bitonic_sort_keys(K (&k)[E]) {
  bitonic_merge_from<E, 2>(k);
}

}  // namespace mg
