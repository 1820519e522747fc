// Shared device helpers for the gfx950 kernels: index access, wave-level
// scans and a register bitonic sort over one 64-lane wavefront.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define MG_WAVE 64
#define MG_INLINE __device__ __forceinline__

namespace mg {

// -------------------------------------------------------------------------
// Index widths: A and B share a row pointer type RP and a column type CI.
// -------------------------------------------------------------------------
template <typename T>
MG_INLINE int64_t ld64(const T* p, int64_t i) { return (int64_t)p[i]; }

MG_INLINE int lane() { return (int)__lane_id(); }

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

// Largest index k in [lo, hi) with pre[k] <= x (pre ascending, pre[lo] <= x).
template <typename T, typename S>
MG_INLINE int upper_index(const T* pre, int lo, int hi, S x) {
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if ((S)pre[mid] <= x) lo = mid; else hi = mid;
  }
  return lo;
}

// -------------------------------------------------------------------------
// Bitonic sort of N = 64 * E keys held in blocked layout: lane l owns
// elements l*E .. l*E+E-1 in registers k[0..E-1] (payload v[] follows its
// key).  Ascending.  For equal keys both partners keep their own element, so
// no payload is duplicated or lost.
// -------------------------------------------------------------------------
template <int E, typename K>
MG_INLINE void cas_local(K* k, int a, int b, bool up) {
  K x = k[a], y = k[b];
  bool sw = up ? (y < x) : (x < y);
  if (sw) { k[a] = y; k[b] = x; }
}
template <int E, typename K, typename V>
MG_INLINE void cas_local(K* k, V* v, int a, int b, bool up) {
  K x = k[a], y = k[b];
  bool sw = up ? (y < x) : (x < y);
  if (sw) {
    k[a] = y; k[b] = x;
    V t = v[a]; v[a] = v[b]; v[b] = t;
  }
}

template <int E, typename K>
MG_INLINE void bitonic_sort_keys(K (&k)[E]) {
  const int l = lane();
  constexpr int N = MG_WAVE * E;
#pragma unroll
  for (int size = 2; size <= N; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride >= 1; stride >>= 1) {
      if (stride < E) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
          if ((e & stride) == 0) {
            int x = l * E + e;
            bool up = (x & size) == 0;
            cas_local<E>(k, e, e | stride, up);
          }
        }
      } else {
        const int lm = stride / E;
        const bool lower = (l & lm) == 0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
          int x = l * E + e;
          bool up = (x & size) == 0;
          K p = __shfl_xor(k[e], lm, MG_WAVE);
          bool take = (lower == up) ? (p < k[e]) : (k[e] < p);
          if (take) k[e] = p;
        }
      }
    }
  }
}

template <int E, typename K, typename V>
MG_INLINE void bitonic_sort_pairs(K (&k)[E], V (&v)[E]) {
  const int l = lane();
  constexpr int N = MG_WAVE * E;
#pragma unroll
  for (int size = 2; size <= N; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride >= 1; stride >>= 1) {
      if (stride < E) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
          if ((e & stride) == 0) {
            int x = l * E + e;
            bool up = (x & size) == 0;
            cas_local<E>(k, v, e, e | stride, up);
          }
        }
      } else {
        const int lm = stride / E;
        const bool lower = (l & lm) == 0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
          int x = l * E + e;
          bool up = (x & size) == 0;
          K p = __shfl_xor(k[e], lm, MG_WAVE);
          V pv = __shfl_xor(v[e], lm, MG_WAVE);
          bool take = (lower == up) ? (p < k[e]) : (k[e] < p);
          if (take) { k[e] = p; v[e] = pv; }
        }
      }
    }
  }
}

}  // namespace mg
