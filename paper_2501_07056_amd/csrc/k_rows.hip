// Row-level kernels: the setup phase (per-row intermediate-product count and
// column range, row categorisation; Section 3.1) and DENSE rows (dense
// accumulator over the row's column range; Algorithm 1).  The accumulator
// kernel runs in two modes: count
// (precise symbolic phase: exact nnz per row, Section 2.1) and numeric (values
// written straight into C at the row offsets the symbolic phase produced).
#include "common.h"
#include "kernels.h"
#include "dispatch.h"

namespace mg {

// ---------------------------------------------------------------------------
// wave-private LDS: order LDS writes of this wave before other lanes read
// ---------------------------------------------------------------------------
MG_INLINE void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

// ---------------------------------------------------------------------------
// Setup: ip_i = sum over entries (i,j) of nnz(B_j); minc/maxc = smallest /
// largest column over those B rows (B rows sorted); class of the row.
// G lanes cooperate on one row; rows with more than HEAVY_ENTRIES entries of
// A are listed and set up by a workgroup each (k_rowinfo_heavy), so a few
// very long rows do not hold the whole grid.
// ---------------------------------------------------------------------------
constexpr int64_t HEAVY_ENTRIES = 1024;

// Category (Section 3.1) and class of a row from its products and range.
MG_INLINE int row_class(int64_t s, int64_t range, int force, int64_t sort_max, int64_t dense_max,
                        int64_t coarse_range, int& cat) {
  if (s == 0) {
    cat = 3;
    return CLS_EMPTY;
  }
  int want = force;
  if (want < 0) want = (s < sort_max) ? 0 : (range <= dense_max ? 1 : 2);
  if (want == 0 && s > SORT_CAP) want = (range <= dense_max) ? 1 : 2;
  if (want == 1 && range > dense_max) want = 2;
  cat = want;
  if (want == 0) {
    int lg = 0;
    while (((int64_t)1 << lg) < s) ++lg;
    return lg;
  }
  if (want == 1) return CLS_DENSE;
  return (coarse_range > 0 && range > coarse_range) ? CLS_COARSE : CLS_CHUNKED;
}
template <typename RP, typename CI, bool BATCH>
__global__ void __launch_bounds__(256) k_rowinfo(RowSrc src, int64_t n, int G, ClassParams cp,
                                                 int64_t* ip, int64_t* minc, int64_t* maxc,
                                                 int32_t* cls, DevStats* stats, int32_t* flags,
                                                 int32_t* heavy) {
  // grid-stride over groups of G lanes per row; the statistics of all rows a
  // block visits are combined in LDS and added to the global totals once per
  // block (a global atomic per block on a handful of addresses would
  // serialise in L2 across hundreds of thousands of blocks)
  __shared__ unsigned long long sh[21];
  if (threadIdx.x < 21) sh[threadIdx.x] = 0;
  __syncthreads();
  const int64_t groups_per_block = blockDim.x / G;
  const int sub = (int)(threadIdx.x % G);
  unsigned long long l_ip = 0, l_max = 0, l_rng = 0, l_ipc[4] = {0, 0, 0, 0}, l_rc[4] = {0, 0, 0, 0};
  unsigned long long l_ent[4] = {0, 0, 0, 0}, l_rcat[3] = {0, 0, 0};
  for (int64_t rb = (int64_t)blockIdx.x * groups_per_block; rb < n;
       rb += (int64_t)gridDim.x * groups_per_block) {
    const int64_t row = rb + threadIdx.x / G;
    int64_t s = 0, mn = INT64_MAX, mx = -1, nent = 0, p0 = 0, p1 = 0, mcols = 0;
    int32_t b = 0;
    int64_t sort_max = cp.sort_max, dense_max = cp.dense_max;
    const MatEnt* Mp = &src.one;
    if (row < n) {
      // a batch: the row's product from the per-row table
      if (BATCH) {
        b = src.mat_of_row[row];
        Mp = &src.tab[b];
        sort_max = Mp->sort_max;
        dense_max = Mp->dense_max;
      }
      const int64_t lrow = row - (BATCH ? Mp->row0 : 0);
      const RP* arp = (const RP*)Mp->arp;
      const CI* acol = (const CI*)Mp->acol;
      const RP* brp = (const RP*)Mp->brp;
      mcols = Mp->mcols;
      p0 = arp[lrow];
      p1 = arp[lrow + 1];
      nent = p1 - p0;
      if (!BATCH && nent > HEAVY_ENTRIES) {
        // the whole group skips this row; one lane lists it
        if (sub == 0) heavy[atomicAdd(&stats->heavy, 1ull)] = (int32_t)row;
        continue;
      }
      for (int64_t p = p0 + sub; p < p1; p += G) {
        const int64_t j = acol[p];
        s += (int64_t)brp[j + 1] - (int64_t)brp[j];
      }
    }
    for (int d = G >> 1; d >= 1; d >>= 1) s += __shfl_xor(s, d, G);
    // the column range (first and last column of every B row: two more
    // gathers per entry) only where the category depends on it; SORT rows
    // key their products on the full column (range = the columns of C)
    const bool need = row < n && s > 0 && (cp.force > 0 || s >= sort_max || s > SORT_CAP);
    if (need) {
      const CI* acol = (const CI*)Mp->acol;
      const RP* brp = (const RP*)Mp->brp;
      const CI* bcol = (const CI*)Mp->bcol;
      for (int64_t p = p0 + sub; p < p1; p += G) {
        const int64_t j = acol[p];
        const int64_t b0 = brp[j], b1 = brp[j + 1];
        if (b1 > b0) {
          const int64_t f = bcol[b0], l = bcol[b1 - 1];
          mn = f < mn ? f : mn;
          mx = l > mx ? l : mx;
        }
      }
    }
    for (int d = G >> 1; d >= 1; d >>= 1) {
      const int64_t a = __shfl_xor(mn, d, G);
      const int64_t c2 = __shfl_xor(mx, d, G);
      mn = a < mn ? a : mn;
      mx = c2 > mx ? c2 : mx;
    }
    if (!need && s > 0) {
      mn = 0;
      mx = mcols - 1;
    }
    if (row < n && sub == 0) {
      int cat;
      const int64_t range = (s > 0) ? (mx - mn + 1) : 0;
      const int c = row_class(s, range, cp.force, sort_max, dense_max, cp.coarse_range, cat);
      if (s == 0) {
        mn = 0;
        mx = -1;
      }
      if (BATCH && cat == 2 && flags[b] == 0) flags[b] = 1;  // idempotent store
      ip[row] = s;
      minc[row] = mn;
      maxc[row] = mx;
      cls[row] = c;
      l_ip += (unsigned long long)s;
      l_max = (unsigned long long)s > l_max ? (unsigned long long)s : l_max;
      l_rng = (unsigned long long)range > l_rng ? (unsigned long long)range : l_rng;
      l_ipc[cat] += (unsigned long long)s;
      l_rc[cat] += 1;
      l_ent[cat] += (unsigned long long)nent;
      if (cat < 3 && (unsigned long long)range > l_rcat[cat]) l_rcat[cat] = (unsigned long long)range;
    }
  }
  if (sub == 0) {
    atomicAdd(&sh[0], l_ip);
    atomicMax(&sh[1], l_max);
    atomicMax(&sh[2], l_rng);
    for (int k = 0; k < 4; ++k) {
      if (l_ipc[k]) atomicAdd(&sh[6 + k], l_ipc[k]);
      if (l_rc[k]) atomicAdd(&sh[10 + k], l_rc[k]);
      if (l_ent[k]) atomicAdd(&sh[14 + k], l_ent[k]);
    }
    for (int k = 0; k < 3; ++k)
      if (l_rcat[k]) atomicMax(&sh[18 + k], l_rcat[k]);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    atomicAdd(&stats->ip_total, sh[0]);
    atomicMax(&stats->max_ip, sh[1]);
    atomicMax(&stats->max_range, sh[2]);
    for (int k = 0; k < 4; ++k) {
      if (sh[6 + k]) atomicAdd(&stats->ip_cat[k], sh[6 + k]);
      if (sh[10 + k]) atomicAdd(&stats->rows_cat[k], sh[10 + k]);
      if (sh[14 + k]) atomicAdd(&stats->ent_cat[k], sh[14 + k]);
    }
    for (int k = 0; k < 3; ++k)
      if (sh[18 + k]) atomicMax(&stats->range_cat[k], sh[18 + k]);
  }
}

// Setup of the listed long rows: one workgroup per row (grid-stride over the
// list, whose length the first kernel left in stats->heavy).
template <typename RP, typename CI>
__global__ void __launch_bounds__(256) k_rowinfo_heavy(RowSrc src, ClassParams cp,
                                                       const int32_t* __restrict__ heavy,
                                                       int64_t* ip, int64_t* minc, int64_t* maxc,
                                                       int32_t* cls, DevStats* stats) {
  __shared__ int64_t sh_s[4], sh_mn[4], sh_mx[4];
  const unsigned long long nh = stats->heavy;
  const RP* arp = (const RP*)src.one.arp;
  const CI* acol = (const CI*)src.one.acol;
  const RP* brp = (const RP*)src.one.brp;
  const CI* bcol = (const CI*)src.one.bcol;
  const int w = threadIdx.x / MG_WAVE;
  for (unsigned long long h = blockIdx.x; h < nh; h += gridDim.x) {
    const int32_t row = heavy[h];
    const int64_t p0 = arp[row], p1 = arp[row + 1];
    int64_t s = 0, mn = INT64_MAX, mx = -1;
    for (int64_t p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
      const int64_t j = acol[p];
      const int64_t b0 = brp[j], b1 = brp[j + 1];
      if (b1 > b0) {
        s += b1 - b0;
        const int64_t f = bcol[b0], l = bcol[b1 - 1];
        mn = f < mn ? f : mn;
        mx = l > mx ? l : mx;
      }
    }
    s = wave_sum(s);
    mn = wave_min(mn);
    mx = wave_max(mx);
    if (lane() == 0) {
      sh_s[w] = s;
      sh_mn[w] = mn;
      sh_mx[w] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int v = 1; v < (int)(blockDim.x / MG_WAVE); ++v) {
        s += sh_s[v];
        mn = sh_mn[v] < mn ? sh_mn[v] : mn;
        mx = sh_mx[v] > mx ? sh_mx[v] : mx;
      }
      int cat;
      const int64_t range = (s > 0) ? (mx - mn + 1) : 0;
      const int c = row_class(s, range, cp.force, cp.sort_max, cp.dense_max, cp.coarse_range, cat);
      if (s == 0) {
        mn = 0;
        mx = -1;
      }
      ip[row] = s;
      minc[row] = mn;
      maxc[row] = mx;
      cls[row] = c;
      atomicAdd(&stats->ip_total, (unsigned long long)s);
      atomicMax(&stats->max_ip, (unsigned long long)s);
      atomicMax(&stats->max_range, (unsigned long long)range);
      atomicAdd(&stats->ip_cat[cat], (unsigned long long)s);
      atomicAdd(&stats->rows_cat[cat], 1ull);
      atomicAdd(&stats->ent_cat[cat], (unsigned long long)(p1 - p0));
      if (cat < 3) atomicMax(&stats->range_cat[cat], (unsigned long long)range);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// CSR validation (only on request): rowptr monotone from 0, columns in range,
// rows of B strictly ascending.
// ---------------------------------------------------------------------------
template <typename RP, typename CI>
__global__ void k_validate(const RP* rp, const CI* col, int64_t n, int64_t ncols, int64_t nnz,
                           int strict_sorted, DevStats* stats) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n) return;
  bool bad = false;
  if (i == 0 && rp[0] != 0) bad = true;
  if (i == n && (int64_t)rp[n] != nnz) bad = true;
  if (i < n) {
    const int64_t p0 = rp[i], p1 = rp[i + 1];
    if (p1 < p0 || p0 < 0 || p1 > nnz) {
      bad = true;
    } else {
      int64_t prev = -1;
      for (int64_t p = p0; p < p1; ++p) {
        const int64_t c = col[p];
        if (c < 0 || c >= ncols) { bad = true; break; }
        if (strict_sorted && c <= prev) { bad = true; break; }
        prev = c;
      }
    }
  }
  if (bad) atomicOr(&stats->err, ERR_INVALID_CSR);
}

// ---------------------------------------------------------------------------
// Stable partition of rows by class (counts per block, scan, scatter).
// ---------------------------------------------------------------------------
constexpr int CL_BS = 256;

__global__ void __launch_bounds__(CL_BS) k_class_count(const int32_t* cls, int64_t n, int32_t* cnt,
                                                        int64_t nblk) {
  __shared__ int32_t h[NCLS];
  if (threadIdx.x < NCLS) h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * CL_BS + threadIdx.x;
  if (i < n) atomicAdd(&h[cls[i]], 1);
  __syncthreads();
  if (threadIdx.x < NCLS) cnt[(int64_t)threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

__global__ void __launch_bounds__(CL_BS) k_class_scatter(const int32_t* cls, int64_t n,
                                                          const int64_t* off, int64_t nblk,
                                                          int32_t* list) {
  __shared__ int32_t wc[CL_BS / MG_WAVE][NCLS];
  const int64_t i = (int64_t)blockIdx.x * CL_BS + threadIdx.x;
  const int c = (i < n) ? cls[i] : -1;
  const int w = threadIdx.x / MG_WAVE;
  int my_rank = 0;
  for (int k = 0; k < NCLS; ++k) {
    uint64_t m = ballot(c == k);
    if (c == k) my_rank = rank_below(m);
    if (lane() == 0) wc[w][k] = popc64(m);
  }
  __syncthreads();
  if (c >= 0) {
    int before = 0;
    for (int v = 0; v < w; ++v) before += wc[v][c];
    list[off[(int64_t)c * nblk + blockIdx.x] + before + my_rank] = (int32_t)i;
  }
}

__global__ void k_class_offsets(const int64_t* off, int64_t nblk, int64_t n, int64_t* list_off) {
  const int c = threadIdx.x;
  if (c < NCLS) list_off[c] = off[(int64_t)c * nblk];
  if (c == 0) list_off[NCLS] = n;
}

size_t classify_temp_bytes(int64_t n) {
  const int64_t nblk = (n + CL_BS - 1) / CL_BS;
  const int64_t tab = (int64_t)NCLS * nblk;
  return (size_t)tab * 4 + (size_t)tab * 8 + scan_temp_bytes(tab) + 256;
}

hipError_t launch_classify(const int32_t* cls, int64_t n, int32_t* list, int64_t* list_off,
                           void* temp, hipStream_t st) {
  const int64_t nblk = (n + CL_BS - 1) / CL_BS;
  const int64_t tab = (int64_t)NCLS * nblk;
  char* t = (char*)temp;
  int32_t* cnt = (int32_t*)t;
  t += ((size_t)tab * 4 + 255) / 256 * 256;
  int64_t* off = (int64_t*)t;
  t += ((size_t)tab * 8 + 255) / 256 * 256;
  if (n > 0) {
    hipLaunchKernelGGL(k_class_count, (unsigned)nblk, CL_BS, 0, st, cls, n, cnt, nblk);
    hipError_t e = scan_excl_i32(cnt, off, tab, nullptr, nullptr, t, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_class_scatter, (unsigned)nblk, CL_BS, 0, st, cls, n, (const int64_t*)off,
                       nblk, list);
    hipLaunchKernelGGL(k_class_offsets, 1, 64, 0, st, (const int64_t*)off, nblk, n, list_off);
  } else {
    hipError_t e = hipMemsetAsync(list_off, 0, sizeof(int64_t) * (NCLS + 1), st);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// DENSE rows.  One workgroup per row; the dense accumulator covers the row's
// column range [minc, maxc] (<= 2^shift columns): values in LDS plus one
// bitmap bit per column (Algorithm 1 with the bitmap as a bit array).  The
// write-out walks the bitmap in column order.
// ---------------------------------------------------------------------------
size_t dense_rows_lds(int f64, int shift, int block) {
  const size_t L = (size_t)1 << shift;
  return L * (f64 ? 8 : 4) + (L / 32) * 4 + (size_t)block * (4 + 8 + 8) + 64;
}

template <typename V>
MG_INLINE int64_t block_excl_scan64(int64_t v, int64_t* sh_w, int64_t& total) {
  const int t = threadIdx.x, wv = t / MG_WAVE, nw = blockDim.x / MG_WAVE;
  const int64_t inc = wave_incl_scan(v);
  if (lane() == MG_WAVE - 1) sh_w[wv] = inc;
  __syncthreads();
  int64_t before = 0;
  total = 0;
  for (int k = 0; k < nw; ++k) {
    const int64_t s = sh_w[k];
    if (k < wv) before += s;
    total += s;
  }
  __syncthreads();
  return before + inc - v;
}

template <typename RP, typename CI, typename V, bool NUMERIC>
MG_INLINE void dense_row(const RowSrc& src, const int32_t* __restrict__ list,
                         const int64_t* __restrict__ minc, const int64_t* __restrict__ maxc,
                         int shift, int64_t* rownnz, const int64_t* __restrict__ crp,
                         int64_t idx) {
  extern __shared__ __align__(16) unsigned char dsm[];
  const int BS = blockDim.x;
  const int64_t L = (int64_t)1 << shift;
  V* acc = (V*)dsm;
  uint32_t* bits = (uint32_t*)(dsm + L * sizeof(V));
  int32_t* w_pre = (int32_t*)(bits + L / 32);
  int64_t* w_b0 = (int64_t*)(((uintptr_t)(w_pre + BS + 1) + 7) & ~(uintptr_t)7);
  V* w_av = (V*)(w_b0 + BS);
  __shared__ int64_t sh_w[16];

  const int t = threadIdx.x;
  const int32_t row = list[idx];
  const MatEnt& M = src.tab ? src.tab[src.mat_of_row[row]] : src.one;
  const int64_t lrow = row - M.row0;
  const RP* __restrict__ arp = (const RP*)M.arp;
  const CI* __restrict__ acol = (const CI*)M.acol;
  const V* __restrict__ aval = (const V*)M.aval;
  const RP* __restrict__ brp = (const RP*)M.brp;
  const CI* __restrict__ bcol = (const CI*)M.bcol;
  const V* __restrict__ bval = (const V*)M.bval;
  const int64_t mn = minc[row];
  const int64_t range = maxc[row] - mn + 1;
  const int64_t nwords = (range + 31) / 32;
  for (int64_t q = t; q < nwords; q += BS) bits[q] = 0u;
  if (NUMERIC)
    for (int64_t q = t; q < range; q += BS) acc[q] = (V)0;
  __syncthreads();

  const int64_t a0 = arp[lrow], a1 = arp[lrow + 1];
  for (int64_t e0 = a0; e0 < a1; e0 += BS) {
    const int64_t e = e0 + t;
    int len = 0;
    int64_t b0 = 0;
    V av = (V)0;
    if (e < a1) {
      const int64_t j = acol[e];
      b0 = brp[j];
      len = (int)((int64_t)brp[j + 1] - b0);
      if (NUMERIC) av = aval[e];
    }
    int64_t tot;
    const int64_t pre = block_excl_scan64<V>(len, sh_w, tot);
    w_pre[t] = (int32_t)pre;
    w_b0[t] = b0;
    w_av[t] = av;
    const int nvalid = (int)((a1 - e0) < BS ? (a1 - e0) : BS);
    __syncthreads();
    for (int64_t q = t; q < tot; q += BS) {
      const int k = upper_index(w_pre, 0, nvalid, (int32_t)q);
      const int64_t bi = w_b0[k] + (q - w_pre[k]);
      const int64_t lc = (int64_t)bcol[bi] - mn;
      atomicOr(&bits[lc >> 5], 1u << (lc & 31));
      if (NUMERIC) atomicAdd(&acc[lc], w_av[k] * bval[bi]);
    }
    __syncthreads();
  }

  // write-out / count: thread t owns a contiguous run of bitmap words
  const int64_t wpt = (nwords + BS - 1) / BS;
  const int64_t w0 = t * wpt, w1 = (w0 + wpt < nwords) ? (w0 + wpt) : nwords;
  int64_t cnt = 0;
  for (int64_t q = w0; q < w1; ++q) cnt += __popc(bits[q]);
  int64_t total;
  const int64_t base = block_excl_scan64<V>(cnt, sh_w, total);
  if (!NUMERIC) {
    if (t == 0) rownnz[row] = total;
    return;
  }
  CI* ccol = (CI*)M.ccol;
  V* cval = (V*)M.cval;
  int64_t pos = crp[row] - (src.tab ? crp[M.row0] : 0) + base;
  for (int64_t q = w0; q < w1; ++q) {
    uint32_t b = bits[q];
    while (b) {
      const int bit = __ffs(b) - 1;
      b &= b - 1;
      const int64_t lc = q * 32 + bit;
      st_stream<HINT_C_STORE>(&ccol[pos], (CI)(mn + lc));
      st_stream<HINT_C_STORE>(&cval[pos], acc[lc]);
      ++pos;
    }
  }
}

// One row per workgroup from the grid (work == nullptr), or persistent
// workgroups taking rows from the counter *work (holding 0) until done.
template <typename RP, typename CI, typename V, bool NUMERIC>
__global__ void __launch_bounds__(1024)
    k_dense_rows(RowSrc src, const int32_t* __restrict__ list, const int64_t* __restrict__ minc,
                 const int64_t* __restrict__ maxc, int shift, int64_t* rownnz,
                 const int64_t* __restrict__ crp) {
  dense_row<RP, CI, V, NUMERIC>(src, list, minc, maxc, shift, rownnz, crp, blockIdx.x);
}

template <typename RP, typename CI, typename V, bool NUMERIC>
__global__ void __launch_bounds__(1024)
    k_dense_rows_persistent(RowSrc src, const int32_t* __restrict__ list,
                            const int64_t* __restrict__ minc, const int64_t* __restrict__ maxc,
                            int shift, int64_t* rownnz, const int64_t* __restrict__ crp,
                            int64_t count, unsigned int* work) {
  __shared__ unsigned int sh_idx;
  for (;;) {
    __syncthreads();  // the previous row's LDS reads are done
    if (threadIdx.x == 0) sh_idx = atomicAdd(work, 1u);
    __syncthreads();
    const int64_t idx = sh_idx;
    if (idx >= count) return;
    dense_row<RP, CI, V, NUMERIC>(src, list, minc, maxc, shift, rownnz, crp, idx);
  }
}

template <typename RP, typename CI, typename V>
static hipError_t dense_rows_t(const RowSrc& src, bool numeric, const int32_t* list, int64_t count,
                               const int64_t* minc, const int64_t* maxc, int shift, int block,
                               int64_t* rownnz, const int64_t* crp, unsigned int* work,
                               hipStream_t st) {
  if (count == 0) return hipSuccess;
  const size_t lds = dense_rows_lds(sizeof(V) == 8, shift, block);
  if (work) {
    auto kp = numeric ? k_dense_rows_persistent<RP, CI, V, true>
                      : k_dense_rows_persistent<RP, CI, V, false>;
    hipError_t e =
        hipFuncSetAttribute((const void*)kp, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    int per_cu = 0, dev = 0, cus = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kp, block, lds) != hipSuccess ||
        per_cu < 1)
      per_cu = 1;
    if (hipGetDevice(&dev) == hipSuccess)
      (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int64_t grid = std::min<int64_t>((int64_t)per_cu * std::max(cus, 1), count);
    hipLaunchKernelGGL(kp, (unsigned)grid, block, lds, st, src, list, minc, maxc, shift, rownnz,
                       crp, count, work);
    return hipGetLastError();
  }
  auto k = numeric ? k_dense_rows<RP, CI, V, true> : k_dense_rows<RP, CI, V, false>;
  hipError_t e =
      hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int64_t cap = max_grid(block);  // one workgroup per row
  for (int64_t o = 0; o < count; o += cap)
    hipLaunchKernelGGL(k, (unsigned)std::min(cap, count - o), block, lds, st, src, list + o, minc,
                       maxc, shift, rownnz, crp);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// misc
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_cat_nnz(const int32_t* cls, const int64_t* rownnz, int64_t n,
                                                 DevStats* stats) {
  __shared__ unsigned long long sh[4];
  if (threadIdx.x < 4) sh[threadIdx.x] = 0;
  __syncthreads();
  unsigned long long loc[4] = {0, 0, 0, 0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int c = cls[i];
    const int cat =
        c < CLS_DENSE ? 0 : (c == CLS_DENSE ? 1 : ((c == CLS_CHUNKED || c == CLS_COARSE) ? 2 : 3));
    loc[cat] += (unsigned long long)rownnz[i];
  }
  for (int k = 0; k < 4; ++k) {
    const unsigned long long v = wave_sum(loc[k]);
    if (lane() == 0 && v) atomicAdd(&sh[k], v);
  }
  __syncthreads();
  if (threadIdx.x < 4 && sh[threadIdx.x]) atomicAdd(&stats->nnz_cat[threadIdx.x], sh[threadIdx.x]);
}
hipError_t launch_cat_nnz(const int32_t* cls, const int64_t* rownnz, int64_t n, DevStats* stats,
                          hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t want = (n + 255) / 256;
  hipLaunchKernelGGL(k_cat_nnz, (unsigned)(want < 2048 ? want : 2048), 256, 0, st, cls, rownnz, n,
                     stats);
  return hipGetLastError();
}

__global__ void k_gather_rows(const int64_t* v, const int32_t* rows, int64_t nrows, int64_t* out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nrows) out[k] = v[rows[k]];
}
hipError_t launch_gather_rows(const int64_t* v, const int32_t* rows, int64_t nrows, int64_t* out,
                              hipStream_t st) {
  if (nrows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_rows, (unsigned)((nrows + 255) / 256), 256, 0, st, v, rows, nrows,
                     out);
  return hipGetLastError();
}

// Plain streaming copy (16-byte vectors, grid-stride): the reference for the
// achievable HBM bandwidth and for scaling the memory counters.
__global__ void __launch_bounds__(256) k_stream_copy(uint4* __restrict__ dst,
                                                     const uint4* __restrict__ src, int64_t n16) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}
__global__ void k_copy_tail(unsigned char* dst, const unsigned char* src, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}
hipError_t launch_stream_copy(void* dst, const void* src, size_t bytes, hipStream_t st) {
  const int64_t n16 = (int64_t)(bytes / 16);
  if (n16 > 0) {
    const int64_t want = (n16 + 255) / 256;
    hipLaunchKernelGGL(k_stream_copy, (unsigned)(want < 256 * 64 ? want : 256 * 64), 256, 0, st,
                       (uint4*)dst, (const uint4*)src, n16);
  }
  const int64_t tail = (int64_t)(bytes - (size_t)n16 * 16);
  if (tail > 0)
    hipLaunchKernelGGL(k_copy_tail, 1, 64, 0, st, (unsigned char*)dst + n16 * 16,
                       (const unsigned char*)src + n16 * 16, tail);
  return hipGetLastError();
}
__global__ void k_fill_i64(int64_t* p, int64_t n, int64_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
hipError_t launch_fill_i64(int64_t* p, int64_t n, int64_t v, hipStream_t st) {
  const int64_t cap = max_grid(256) * 256;
  for (int64_t o = 0; o < n; o += cap) {
    const int64_t m = std::min(cap, n - o);
    hipLaunchKernelGGL(k_fill_i64, (unsigned)((m + 255) / 256), 256, 0, st, p + o, m, v);
  }
  return hipGetLastError();
}

template <typename T>
__global__ void k_write_rowptr(const int64_t* crp, int64_t n1, T* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n1) out[i] = (T)crp[i];
}
hipError_t launch_write_rowptr(const int64_t* crp, int64_t n, void* out, int out64,
                               hipStream_t st) {
  const int64_t n1 = n + 1;
  const unsigned g = (unsigned)((n1 + 255) / 256);
  if (out64) hipLaunchKernelGGL(k_write_rowptr<int64_t>, g, 256, 0, st, crp, n1, (int64_t*)out);
  else hipLaunchKernelGGL(k_write_rowptr<int32_t>, g, 256, 0, st, crp, n1, (int32_t*)out);
  return hipGetLastError();
}

static int rowinfo_lanes(int64_t n, int64_t a_nnz) {
  // lanes per row: the power of two nearest the mean row length of A, 1..64
  const int64_t avg = n ? (a_nnz + n - 1) / n : 1;
  int G = 1;
  while (G < 64 && G < avg) G <<= 1;
  return G;
}

hipError_t launch_rowinfo(const Mats& M, int64_t a_nnz, const ClassParams& cp, int64_t* ip,
                          int64_t* minc, int64_t* maxc, int32_t* cls, DevStats* stats,
                          int32_t* heavy, hipStream_t st) {
  if (M.n == 0) return hipSuccess;
  const int G = rowinfo_lanes(M.n, a_nnz);
  const int64_t want = (M.n * G + 255) / 256;
  const unsigned grid = (unsigned)(want < 4096 ? want : 4096);
  const RowSrc src = single_src(M, nullptr, nullptr);
  MG_DISPATCH2(M, {
    hipLaunchKernelGGL((k_rowinfo<RP, CI, false>), grid, 256, 0, st, src, M.n, G, cp, ip, minc,
                       maxc, cls, stats, nullptr, heavy);
    hipLaunchKernelGGL((k_rowinfo_heavy<RP, CI>), 1024, 256, 0, st, src, cp, heavy, ip, minc,
                       maxc, cls, stats);
  });
  return hipGetLastError();
}

hipError_t launch_rowinfo_batch(const Mats& T, const RowSrc& src, int64_t nrows, int64_t a_nnz,
                                const ClassParams& cp, int64_t* ip, int64_t* minc, int64_t* maxc,
                                int32_t* cls, DevStats* stats, int32_t* flags, hipStream_t st) {
  if (nrows == 0) return hipSuccess;
  const int G = rowinfo_lanes(nrows, a_nnz);
  const int64_t want = (nrows * G + 255) / 256;
  const unsigned grid = (unsigned)(want < 4096 ? want : 4096);
  MG_DISPATCH2(T, hipLaunchKernelGGL((k_rowinfo<RP, CI, true>), grid, 256, 0, st, src, nrows, G,
                                     cp, ip, minc, maxc, cls, stats, flags, nullptr));
  return hipGetLastError();
}

// Upper bound of a row's nnz in C: its intermediate-product count, and at
// most the number of columns of C (the bound of the admission estimate).  G
// lanes per row as in the setup kernel.
template <typename RP, typename CI>
__global__ void __launch_bounds__(256) k_row_bound(RowSrc src, int64_t n, int G, int64_t* ip,
                                                   int64_t* bound) {
  const int64_t groups_per_block = blockDim.x / G;
  const int sub = (int)(threadIdx.x % G);
  for (int64_t rb = (int64_t)blockIdx.x * groups_per_block; rb < n;
       rb += (int64_t)gridDim.x * groups_per_block) {
    const int64_t row = rb + threadIdx.x / G;
    int64_t s = 0, m = 0;
    if (row < n) {
      const MatEnt& M = src.tab[src.mat_of_row[row]];
      const int64_t lrow = row - M.row0;
      const RP* arp = (const RP*)M.arp;
      const CI* acol = (const CI*)M.acol;
      const RP* brp = (const RP*)M.brp;
      m = M.mcols;
      const int64_t p0 = arp[lrow], p1 = arp[lrow + 1];
      for (int64_t p = p0 + sub; p < p1; p += G) {
        const int64_t j = acol[p];
        s += (int64_t)brp[j + 1] - (int64_t)brp[j];
      }
    }
    for (int d = G >> 1; d >= 1; d >>= 1) s += __shfl_xor(s, d, G);
    if (row < n && sub == 0) {
      ip[row] = s;
      bound[row] = s < m ? s : m;
    }
  }
}

hipError_t launch_row_bound(const Mats& T, const RowSrc& src, int64_t nrows, int64_t a_nnz,
                            int64_t* ip, int64_t* bound, hipStream_t st) {
  if (nrows == 0) return hipSuccess;
  const int G = rowinfo_lanes(nrows, a_nnz);
  const int64_t want = (nrows * G + 255) / 256;
  const unsigned grid = (unsigned)(want < 4096 ? want : 4096);
  MG_DISPATCH2(T, hipLaunchKernelGGL((k_row_bound<RP, CI>), grid, 256, 0, st, src, nrows, G, ip,
                                     bound));
  return hipGetLastError();
}

__global__ void k_mat_of_row(const int64_t* row0, int64_t nmat, int64_t nrows, int32_t* out) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  // largest b with row0[b] <= r (row0 ascending, row0[0] = 0, row0[nmat] = nrows)
  int64_t lo = 0, hi = nmat;
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (row0[mid] <= r) lo = mid; else hi = mid;
  }
  out[r] = (int32_t)lo;
}
hipError_t launch_mat_of_row(const int64_t* row0, int64_t nmat, int64_t nrows, int32_t* mat_of_row,
                             hipStream_t st) {
  if (nrows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mat_of_row, (unsigned)((nrows + 255) / 256), 256, 0, st, row0, nmat, nrows,
                     mat_of_row);
  return hipGetLastError();
}

__global__ void k_drop_flagged(const int32_t* flags, const int32_t* mat_of_row, int64_t nrows,
                               int32_t* cls) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nrows && flags[mat_of_row[r]]) cls[r] = CLS_EMPTY;
}
hipError_t launch_drop_flagged(const int32_t* flags, const int32_t* mat_of_row, int64_t nrows,
                               int32_t* cls, hipStream_t st) {
  if (nrows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_drop_flagged, (unsigned)((nrows + 255) / 256), 256, 0, st, flags,
                     mat_of_row, nrows, cls);
  return hipGetLastError();
}

// Row r of the batch is row r - row0 of its product; each product's last row
// also writes the closing entry, and thread b < nmat writes the single entry
// of a product without rows.  Products planned alone (flag set) are skipped:
// their own execution writes their row pointers.
__global__ void k_write_rowptr_batch(RowSrc src, const int64_t* __restrict__ crp, int64_t nrows,
                                     int64_t nmat, const int32_t* __restrict__ flags) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nmat && src.tab[r].nrows == 0 && !flags[r]) {
    const MatEnt& E = src.tab[r];
    if (E.crp_out64) ((int64_t*)E.crp_out)[0] = 0;
    else ((int32_t*)E.crp_out)[0] = 0;
  }
  if (r >= nrows) return;
  const int32_t b = src.mat_of_row[r];
  if (flags[b]) return;
  const MatEnt& M = src.tab[b];
  const int64_t base = crp[M.row0];
  const int64_t lr = r - M.row0;
  const bool last = (lr == M.nrows - 1);
  if (M.crp_out64) {
    int64_t* o = (int64_t*)M.crp_out;
    o[lr] = crp[r] - base;
    if (last) o[lr + 1] = crp[r + 1] - base;
  } else {
    int32_t* o = (int32_t*)M.crp_out;
    o[lr] = (int32_t)(crp[r] - base);
    if (last) o[lr + 1] = (int32_t)(crp[r + 1] - base);
  }
}
hipError_t launch_write_rowptr_batch(const RowSrc& src, const int64_t* crp, int64_t nrows,
                                     int64_t nmat, const int32_t* flags, hipStream_t st) {
  const int64_t n = nrows > nmat ? nrows : nmat;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_write_rowptr_batch, (unsigned)((n + 255) / 256), 256, 0, st, src, crp,
                     nrows, nmat, flags);
  return hipGetLastError();
}
hipError_t launch_validate(const Mats& M, int64_t a_nnz, int64_t b_nnz, DevStats* stats,
                           hipStream_t st) {
  // A: columns in [0, k), rows sorted not required; B: columns in [0, m), strictly ascending
  const unsigned ga = (unsigned)((M.n + 1 + 255) / 256);
  const unsigned gb = (unsigned)((M.k + 1 + 255) / 256);
  MG_DISPATCH2(M, {
    hipLaunchKernelGGL((k_validate<RP, CI>), ga, 256, 0, st, (const RP*)M.arp, (const CI*)M.acol,
                       M.n, M.k, a_nnz, 0, stats);
    hipLaunchKernelGGL((k_validate<RP, CI>), gb, 256, 0, st, (const RP*)M.brp, (const CI*)M.bcol,
                       M.k, M.m, b_nnz, 1, stats);
  });
  return hipGetLastError();
}

hipError_t launch_dense_rows(const Mats& M, const RowSrc& src, bool numeric, const int32_t* list,
                             int64_t begin, int64_t count, const int64_t* minc,
                             const int64_t* maxc, int shift, int block, int64_t* rownnz,
                             const int64_t* crp, hipStream_t st, unsigned int* work) {
  hipError_t e = hipSuccess;
  MG_DISPATCH3(M, e = (dense_rows_t<RP, CI, V>(src, numeric, list + begin, count, minc, maxc,
                                                shift, block, rownnz, crp, work, st)));
  return e;
}

}  // namespace mg
