// Seeded synthetic CSR generators shared by the GPU path's tests/bench and by
// the CPU oracle's tests.  This file holds no SpGEMM arithmetic: it only draws
// sparsity patterns and values.
//
// Random numbers come from SplitMix64 used as a counter-based generator
// (Steele, Lea, Flood, "Fast splittable pseudorandom number generators",
// OOPSLA 2014): draw(key, k) = mix(key + (k + 1) * GAMMA).  Every row / edge /
// value owns a fixed counter range, so the output does not depend on the
// number of threads that produce it.
//
// Patterns:
//   * Erdos-Renyi with exactly d distinct uniform columns per row (Floyd's
//     sampling without replacement, then sorted);
//   * the same for wide rows with many entries (d draws, sorted, duplicates
//     replaced by further draws), optionally only for the rows a mask names;
//   * R-MAT (Chakrabarti, Zhan, Faloutsos 2004) with quadrant probabilities
//     (a, b, c, d); the first choice sets the most significant bit; duplicate
//     edges merged; no noise and no vertex permutation;
//   * banded: the diagonal plus k distinct uniform columns with |i - j| <= w.
// Values: uniform in [-1, 1) (53 random bits for f64, 24 for f32) or
// integers uniform in {-4, ..., 4}.
#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

namespace {

constexpr uint64_t GAMMA = 0x9E3779B97F4A7C15ull;

inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
inline uint64_t stream_key(uint64_t seed, uint64_t stream) {
  return mix64(seed ^ mix64(stream * GAMMA + 0x632BE59BD9B4E019ull));
}
inline uint64_t draw(uint64_t key, uint64_t k) { return mix64(key + (k + 1) * GAMMA); }
// uniform integer in [0, bound) by the multiply-shift method
inline uint64_t below(uint64_t r, uint64_t bound) {
  return (uint64_t)(((__uint128_t)r * bound) >> 64);
}
inline double unit53(uint64_t r) { return (double)(r >> 11) * (1.0 / 9007199254740992.0); }

int nthreads_default() {
  unsigned h = std::thread::hardware_concurrency();
  return h ? (int)h : 1;
}

template <class F>
void parallel_for(int64_t n, int nthreads, F f) {
  if (nthreads <= 0) nthreads = nthreads_default();
  if (n < 4096 || nthreads == 1) { f(0, n); return; }
  std::vector<std::thread> ts;
  int64_t per = (n + nthreads - 1) / nthreads;
  for (int t = 0; t < nthreads; ++t) {
    int64_t lo = t * per, hi = std::min(n, lo + per);
    if (lo >= hi) break;
    ts.emplace_back([=] { f(lo, hi); });
  }
  for (auto& th : ts) th.join();
}

inline void put_idx(void* p, int width, int64_t k, int64_t v) {
  if (width == 4) ((int32_t*)p)[k] = (int32_t)v;
  else ((int64_t*)p)[k] = v;
}

// Floyd's algorithm: d distinct values in [0, m), written sorted to out.
inline void floyd_sorted(uint64_t key, uint64_t ctr0, int64_t m, int d, int64_t* out) {
  int cnt = 0;
  for (int64_t j = m - d; j < m; ++j) {
    int64_t t = (int64_t)below(draw(key, ctr0 + (uint64_t)(j - (m - d))), (uint64_t)(j + 1));
    bool seen = false;
    for (int q = 0; q < cnt; ++q) if (out[q] == t) { seen = true; break; }
    out[cnt++] = seen ? j : t;
  }
  std::sort(out, out + d);
}

enum { STREAM_ER = 1, STREAM_RMAT = 2, STREAM_BAND = 3, STREAM_VAL = 4, STREAM_ERW = 5 };

// d distinct uniform values in [0, m) (m >= 2d), sorted: draw d, sort, drop
// duplicates, top up with the next draws of the row's counter range (at most
// `budget` draws); false if the range runs out.
inline bool draw_sorted_distinct(uint64_t key, uint64_t ctr0, uint64_t budget, int64_t m, int d,
                                 std::vector<int64_t>& out) {
  out.clear();
  uint64_t used = 0;
  while ((int)out.size() < d) {
    const int need = d - (int)out.size();
    if (used + (uint64_t)need > budget) return false;
    for (int q = 0; q < need; ++q) out.push_back((int64_t)below(draw(key, ctr0 + used++), (uint64_t)m));
    std::sort(out.begin(), out.end());
    out.erase(std::unique(out.begin(), out.end()), out.end());
  }
  return true;
}

}  // namespace

extern "C" {

uint64_t wl_draw(uint64_t seed, uint64_t stream, uint64_t k) {
  return draw(stream_key(seed, stream), k);
}

// Erdos-Renyi: n rows, m columns, exactly d distinct uniform columns per row.
// rowptr: int64[n+1]; col: n*d entries of col_width (4 or 8) bytes.
int wl_er(int64_t n, int64_t m, int d, uint64_t seed, int64_t* rowptr, void* col, int col_width,
          int nthreads) {
  if (d < 0 || d > m || d > 4096) return -1;
  uint64_t key = stream_key(seed, STREAM_ER);
  for (int64_t i = 0; i <= n; ++i) rowptr[i] = i * d;
  parallel_for(n, nthreads, [&](int64_t lo, int64_t hi) {
    std::vector<int64_t> buf(d > 0 ? d : 1);
    for (int64_t i = lo; i < hi; ++i) {
      floyd_sorted(key, (uint64_t)i * (uint64_t)d, m, d, buf.data());
      for (int q = 0; q < d; ++q) put_idx(col, col_width, i * d + q, buf[q]);
    }
  });
  return 0;
}

// Wide Erdos-Renyi: rows i with mask[i] != 0 (every row when mask is null)
// hold d distinct uniform columns in [0, m), the other rows are empty; needs
// m >= 2d.  Row i draws from counters [8di, 8d(i+1)).  Returns nnz (rowptr
// int64[n+1]; col capacity = d * rows named), or -1.
int64_t wl_er_wide(int64_t n, int64_t m, int d, uint64_t seed, const uint8_t* mask,
                   int64_t* rowptr, void* col, int col_width, int nthreads) {
  if (d < 0 || m < 2 * (int64_t)d) return -1;
  const uint64_t key = stream_key(seed, STREAM_ERW);
  rowptr[0] = 0;
  for (int64_t i = 0; i < n; ++i) rowptr[i + 1] = rowptr[i] + ((!mask || mask[i]) ? d : 0);
  std::atomic<int> bad{0};
  parallel_for(n, nthreads, [&](int64_t lo, int64_t hi) {
    std::vector<int64_t> buf;
    buf.reserve(2 * (size_t)d + 1);
    for (int64_t i = lo; i < hi; ++i) {
      if (mask && !mask[i]) continue;
      const uint64_t budget = 8 * (uint64_t)d;
      if (!draw_sorted_distinct(key, (uint64_t)i * budget, budget, m, d, buf)) {
        bad = 1;
        return;
      }
      for (int q = 0; q < d; ++q) put_idx(col, col_width, rowptr[i] + q, buf[q]);
    }
  });
  return bad ? -1 : rowptr[n];
}

// Banded: n x n, each row holds the diagonal plus k distinct uniform columns j
// with |i - j| <= w, j != i (all of them when fewer than k are available).
// Returns nnz; rowptr int64[n+1]; col capacity n*(k+1).
int64_t wl_banded(int64_t n, int64_t w, int k, uint64_t seed, int64_t* rowptr, void* col,
                  int col_width, int nthreads) {
  uint64_t key = stream_key(seed, STREAM_BAND);
  std::vector<int32_t> len(n);
  for (int64_t i = 0; i < n; ++i) {
    int64_t lo = std::max<int64_t>(0, i - w), hi = std::min<int64_t>(n - 1, i + w);
    int64_t avail = hi - lo;  // excluding the diagonal
    len[i] = 1 + (int32_t)std::min<int64_t>(avail, k);
  }
  rowptr[0] = 0;
  for (int64_t i = 0; i < n; ++i) rowptr[i + 1] = rowptr[i] + len[i];
  parallel_for(n, nthreads, [&](int64_t lo_r, int64_t hi_r) {
    std::vector<int64_t> buf(k + 1);
    for (int64_t i = lo_r; i < hi_r; ++i) {
      int64_t lo = std::max<int64_t>(0, i - w), hi = std::min<int64_t>(n - 1, i + w);
      int64_t avail = hi - lo;
      int kk = (int)std::min<int64_t>(avail, k);
      floyd_sorted(key, (uint64_t)i * (uint64_t)k, avail, kk, buf.data());
      // map candidate index t in [0, avail) to a column in [lo, hi] \ {i}
      for (int q = 0; q < kk; ++q) {
        int64_t c = lo + buf[q];
        if (c >= i) c += 1;
        buf[q] = c;
      }
      buf[kk] = i;
      std::sort(buf.begin(), buf.begin() + kk + 1);
      for (int q = 0; q <= kk; ++q) put_idx(col, col_width, rowptr[i] + q, buf[q]);
    }
  });
  return rowptr[n];
}

// R-MAT with 2^scale vertices and edge_factor * 2^scale edge draws.
// Duplicates are merged when merge != 0; self loops kept.  rowptr int64[n+1]; col capacity =
// number of draws.  Returns nnz after merging.
int64_t wl_rmat(int scale, int64_t edge_factor, double a, double b, double c, uint64_t seed,
                int merge, int64_t* rowptr, void* col, int col_width, int nthreads) {
  if (scale < 0 || scale > 31) return -1;
  const int64_t n = (int64_t)1 << scale;
  const int64_t M = edge_factor * n;
  const uint64_t key = stream_key(seed, STREAM_RMAT);
  const double ab = a + b, abc = a + b + c;
  if (nthreads <= 0) nthreads = nthreads_default();
  std::vector<int64_t> er(M), ec(M);
  parallel_for(M, nthreads, [&](int64_t lo, int64_t hi) {
    for (int64_t e = lo; e < hi; ++e) {
      int64_t r = 0, cc = 0;
      for (int l = 0; l < scale; ++l) {
        double u = unit53(draw(key, (uint64_t)e * (uint64_t)scale + (uint64_t)l));
        int64_t bit = (int64_t)1 << (scale - 1 - l);
        if (u < a) {
        } else if (u < ab) {
          cc |= bit;
        } else if (u < abc) {
          r |= bit;
        } else {
          r |= bit;
          cc |= bit;
        }
      }
      er[e] = r;
      ec[e] = cc;
    }
  });
  // counting sort by row
  std::vector<int64_t> cnt(n + 1, 0);
  for (int64_t e = 0; e < M; ++e) cnt[er[e] + 1]++;
  for (int64_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
  std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1), sorted(M);
  for (int64_t e = 0; e < M; ++e) sorted[pos[er[e]]++] = ec[e];
  std::vector<int64_t>().swap(er);
  std::vector<int64_t>().swap(ec);
  std::vector<int64_t> ulen(n);
  parallel_for(n, nthreads, [&](int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i) {
      int64_t* s = sorted.data() + cnt[i];
      int64_t len = cnt[i + 1] - cnt[i];
      std::sort(s, s + len);
      ulen[i] = merge ? (int64_t)(std::unique(s, s + len) - s) : len;
    }
  });
  rowptr[0] = 0;
  for (int64_t i = 0; i < n; ++i) rowptr[i + 1] = rowptr[i] + ulen[i];
  parallel_for(n, nthreads, [&](int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i)
      for (int64_t q = 0; q < ulen[i]; ++q) put_idx(col, col_width, rowptr[i] + q, sorted[cnt[i] + q]);
  });
  return rowptr[n];
}

// Values for entries [0, nnz): kind 0 = uniform [-1,1), kind 1 = integers in
// {-4..4}.  val_width 4 (float) or 8 (double).
int wl_values(int64_t nnz, uint64_t seed, int kind, void* out, int val_width, int nthreads) {
  const uint64_t key = stream_key(seed, STREAM_VAL);
  parallel_for(nnz, nthreads, [&](int64_t lo, int64_t hi) {
    for (int64_t e = lo; e < hi; ++e) {
      uint64_t r = draw(key, (uint64_t)e);
      double v;
      if (kind == 1) {
        v = (double)((int64_t)below(r, 9) - 4);
      } else if (val_width == 4) {
        v = (double)(r >> 40) * (1.0 / 8388608.0) - 1.0;  // k * 2^-23 - 1, exact in f32
      } else {
        v = (double)(r >> 11) * (1.0 / 4503599627370496.0) - 1.0;  // k * 2^-52 - 1
      }
      if (val_width == 4) ((float*)out)[e] = (float)v;
      else ((double*)out)[e] = v;
    }
  });
  return 0;
}

}  // extern "C"
