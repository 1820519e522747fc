// CHUNKED rows binned by runs.  A run is the part of one row of B that falls
// into one column chunk.  B's rows list ascending columns, so the products
// a_ij * B[j, chunk] of one entry (i, j) of A and one chunk are consecutive
// in B.  The reorder of Algorithm 3 (histogram of the chunks, prefix sum,
// scatter into the chunks) is applied to these runs rather than to single
// products: the reordered intermediate product of a chunk becomes the list
// of its runs (B position, A entry, product offset), and the chunk's
// accumulator (Section 3.4: dense in LDS for many products, a wavefront
// sort for few) reads the products from B through that list.  The chunk
// lengths, the accumulators and the output layout are those of the product
// reorder; only what is moved differs, which pays where runs are long (a
// power-law B, whose heavy rows hold many columns per chunk) and not where
// they hold one product each (uniform B over a wide column range).
#include <algorithm>
#include <type_traits>

#include "common.h"
#include "kernels.h"
#include "dispatch.h"

namespace mg {

namespace {

MG_INLINE void wave_sync_r() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

// product offsets of a run inside its chunk occupy the low 40 bits of the
// packed (runs, products) counters; the run count the high 24
constexpr int RUN_SHIFT = 40;
constexpr unsigned long long RUN_PMASK = (1ull << RUN_SHIFT) - 1ull;

}  // namespace

// ---------------------------------------------------------------------------
// Chunk index of B: for row j, entries [ptr[j], ptr[j+1]) hold the start
// position (in B's column array) and the chunk (column >> shift) of each of
// its runs, then one more entry whose position is the row's end, so run r's
// length is pos[r + 1] - pos[r].  One wave per row; the count pass writes
// runs + 1 per row, the fill pass writes the entries after their scan.
// ---------------------------------------------------------------------------
template <typename RP, typename CI, bool FILL>
__global__ void __launch_bounds__(256)
    k_bci(const RP* __restrict__ brp, const CI* __restrict__ bcol, int64_t nrows, int shift,
          int64_t* cnt, const int64_t* __restrict__ ptr, uint32_t* pos, uint32_t* chunk) {
  const int64_t nw = (int64_t)gridDim.x * 4;
  for (int64_t j = (int64_t)blockIdx.x * 4 + threadIdx.x / MG_WAVE; j < nrows; j += nw) {
    const int64_t p0 = brp[j], p1 = brp[j + 1];
    const int64_t base = FILL ? ptr[j] : 0;
    int64_t n = 0;
    for (int64_t pb = p0; pb < p1; pb += MG_WAVE) {
      const int64_t p = pb + lane();
      bool head = false;
      int64_t c = 0;
      if (p < p1) {
        c = (int64_t)bcol[p] >> shift;
        head = (p == p0) || (((int64_t)bcol[p - 1] >> shift) != c);
      }
      const uint64_t m = ballot(head);
      if (FILL && head) {
        const int64_t o = base + n + rank_below(m);
        pos[o] = (uint32_t)p;
        chunk[o] = (uint32_t)c;
      }
      n += popc64(m);
    }
    if (lane() == 0) {
      if (FILL) pos[base + n] = (uint32_t)p1;
      else cnt[j] = n + 1;
    }
  }
}

// Runs of the listed rows (one wave per row): their total, the largest count
// of A entries in one row, and the rows' products.
template <typename RP, typename CI>
__global__ void __launch_bounds__(256)
    k_run_count(const RP* __restrict__ arp, const CI* __restrict__ acol, const int32_t* rows,
                int64_t nrows, const int64_t* __restrict__ bptr, const int64_t* __restrict__ ip,
                unsigned long long* out) {
  // a wave per row, grid-stride; totals reduced per workgroup, then one
  // atomic each (one per row serialised on the three counters)
  __shared__ unsigned long long sh[4][3];
  const int w = threadIdx.x / MG_WAVE;
  unsigned long long runs = 0, amax = 0, prods = 0;
  for (int64_t k = (int64_t)blockIdx.x * 4 + w; k < nrows; k += (int64_t)gridDim.x * 4) {
    const int32_t r = rows[k];
    const int64_t a0 = arp[r], a1 = arp[r + 1];
    unsigned long long s = 0;
    for (int64_t e = a0 + lane(); e < a1; e += MG_WAVE) {
      const int64_t j = acol[e];
      s += (unsigned long long)(bptr[j + 1] - bptr[j] - 1);
    }
    runs += wave_sum(s);
    amax = amax > (unsigned long long)(a1 - a0) ? amax : (unsigned long long)(a1 - a0);
    prods += (unsigned long long)ip[r];
  }
  if (lane() == 0) {
    sh[w][0] = runs;
    sh[w][1] = amax;
    sh[w][2] = prods;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t0 = 0, t1 = 0, t2 = 0;
    for (int v = 0; v < 4; ++v) {
      t0 += sh[v][0];
      t1 = t1 > sh[v][1] ? t1 : sh[v][1];
      t2 += sh[v][2];
    }
    atomicAdd(&out[0], t0);
    atomicMax(&out[1], t1);
    atomicAdd(&out[2], t2);
  }
}

// ---------------------------------------------------------------------------
// Histogram (HIST) and scatter (!HIST) of the runs of CHUNKED rows, one
// workgroup per row.  The row's A entries are staged RR_BS at a time with
// the exclusive prefix of their run counts; every thread then takes runs
// striped over the window and finds its A entry by a binary search.  Per
// chunk, one 64-bit LDS counter packs (runs << 40) + products, so a single
// atomic add gives a run both its slot among the chunk's runs and its
// product offset inside the chunk, in the same order.
// ---------------------------------------------------------------------------
constexpr int RR_BS = 256;

size_t run_rows_lds(int64_t max_nb) {
  return (size_t)(RR_BS + 4) * 4 + (size_t)RR_BS * 8 + (size_t)max_nb * 24 + 256;
}

template <typename RP, typename CI, bool HIST>
__global__ void __launch_bounds__(RR_BS)
    k_run_rows(const RP* __restrict__ arp, const CI* __restrict__ acol, ChunkGeom g,
               const int64_t* __restrict__ bptr, const uint32_t* __restrict__ bpos,
               const uint32_t* __restrict__ bchunk, int64_t k0, int64_t* bin_seg,
               int64_t* bin_cnt, int32_t* bin_row, const int64_t* __restrict__ seg_beg,
               const int64_t* __restrict__ bin_start, run_t* runs) {
  extern __shared__ __align__(16) unsigned char dsm[];
  const int t = threadIdx.x;
  const int64_t k = k0 + blockIdx.x;
  const int32_t row = g.rows[k];
  const int64_t nbk = g.nb[k], bb = g.binBase[k];
  const int64_t base_chunk = g.minc[row] >> g.shift;
  unsigned long long* ctr = (unsigned long long*)dsm;   // nbk
  int64_t* sbase = (int64_t*)(ctr + nbk);                // nbk (scatter)
  int64_t* pbase = sbase + nbk;                          // nbk (scatter)
  int64_t* e_k0 = pbase + nbk;                           // RR_BS
  int32_t* e_pre = (int32_t*)(e_k0 + RR_BS);             // RR_BS
  __shared__ int32_t s_tmp[RR_BS / MG_WAVE];
  for (int64_t c = t; c < nbk; c += RR_BS) {
    ctr[c] = 0ull;
    if (!HIST) {
      sbase[c] = seg_beg[bb + c];
      pbase[c] = bin_start[bb + c];
    }
  }
  const int64_t a0 = arp[row], a1 = arp[row + 1];
  for (int64_t eb = a0; eb < a1; eb += RR_BS) {
    const int64_t e = eb + t;
    int32_t ns = 0;
    int64_t kb = 0;
    if (e < a1) {
      const int64_t j = acol[e];
      kb = bptr[j];
      ns = (int32_t)(bptr[j + 1] - kb - 1);
    }
    const int32_t inc = wave_incl_scan(ns);
    if (lane() == MG_WAVE - 1) s_tmp[t / MG_WAVE] = inc;
    __syncthreads();
    int32_t before = 0, tot = 0;
    for (int w = 0; w < RR_BS / MG_WAVE; ++w) {
      if (w < t / MG_WAVE) before += s_tmp[w];
      tot += s_tmp[w];
    }
    e_pre[t] = before + inc - ns;
    e_k0[t] = kb;
    const int nvalid = (int)((a1 - eb) < RR_BS ? (a1 - eb) : RR_BS);
    __syncthreads();
    for (int32_t q = t; q < tot; q += RR_BS) {
      const int i = upper_index(e_pre, 0, nvalid, q);
      const int64_t kk = e_k0[i] + (q - e_pre[i]);
      const uint32_t p = bpos[kk];
      const unsigned long long len = (unsigned long long)(bpos[kk + 1] - p);
      const int64_t c = (int64_t)bchunk[kk] - base_chunk;
      const unsigned long long o = atomicAdd(&ctr[c], (1ull << RUN_SHIFT) | len);
      if (!HIST) {
        const int64_t slot = sbase[c] + (int64_t)(o >> RUN_SHIFT);
        const int64_t off = pbase[c] + (int64_t)(o & RUN_PMASK);
        st_global(&runs[slot],
                  run_t{(uint32_t)off, (uint32_t)((uint64_t)off >> 32), p, (uint32_t)(eb + i)});
      }
    }
    __syncthreads();
  }
  if (HIST) {
    for (int64_t c = t; c < nbk; c += RR_BS) {
      const unsigned long long h = ctr[c];
      bin_seg[bb + c] = (int64_t)(h >> RUN_SHIFT);
      bin_cnt[bb + c] = (int64_t)(h & RUN_PMASK);
      bin_row[bb + c] = (int32_t)k;
    }
  }
}

// ---------------------------------------------------------------------------
// Dense accumulation of chunks from their runs: persistent workgroups take
// chunks from a counter.  A chunk's runs are staged BS at a time (product
// offset inside the chunk, B position, A value); threads take the window's
// products striped by BS, each finding its run by a binary search narrowed
// to the runs holding its group of 64 products, gather the B column and
// value, and add a * b into the LDS accumulator (one bitmap bit per
// column).  The write-out is that of the product reorder's dense
// accumulator: ascending columns, touched slots cleared as they are read.
// ---------------------------------------------------------------------------
// Products per thread whose loads are in flight together: numeric 12 (the
// 512-thread workgroups are held to two per CU by the LDS, so the registers
// are there; uniform 2^20 columns, chunks of 16K products: run_accum 47.3 ->
// 42.1 ms against 8, R-MAT scale 20 unchanged), count mode 4 (8: no gain).
#ifndef MG_RUN_UNROLL
#define MG_RUN_UNROLL 12
#endif
#ifndef MG_RUN_UNROLL_C
#define MG_RUN_UNROLL_C 4
#endif

// Per dense item, everything its workgroup needs before the first product:
// product start and count, run start and count, the chunk's first column,
// and the chunk.  One 48-byte record instead of a chain of dependent loads
// (item -> chunk -> row -> column base) at the start of every chunk.
constexpr int RUN_REC = 6;

// column chunk index of bin gb, and its key in the XCD order
MG_INLINE int64_t bin_chunk(const ChunkGeom& g, const int32_t* bin_row, int64_t gb) {
  const int64_t kk = bin_row[gb];
  return (g.minc[g.rows[kk]] >> g.shift) + (gb - g.binBase[kk]);
}
MG_INLINE int64_t xcd_key(int64_t c, int64_t cpx) { return (c % N_XCD) * cpx + c / N_XCD; }

// a run record's product offset, from the record or from memory (its first
// eight bytes)
MG_INLINE int64_t run_off(const run_t& r) { return (int64_t)(((uint64_t)r.y << 32) | r.x); }
MG_INLINE int64_t run_off_at(const run_t* runs, int64_t s) {
  return ld_global((const int64_t*)(runs + s));
}

// Both kernels take DK_ITEMS consecutive items per thread and aggregate the
// keys of a workgroup in LDS (when the keys fit, dk_lds): one global atomic
// per (workgroup, key) instead of one per item, which serialised on the few
// chunk counters.
constexpr int DK_BS = 1024, DK_ITEMS = 8, DK_MAXK = 4096;

__global__ void __launch_bounds__(DK_BS)
    k_dense_key_hist(ChunkGeom g, const int64_t* __restrict__ items, const int32_t* item_counts,
                     const int32_t* __restrict__ bin_row, int64_t cpx, unsigned long long* cnt) {
  __shared__ unsigned int lh[DK_MAXK];
  const int64_t nk = N_XCD * cpx, nit = item_counts[0];
  const bool lds = nk <= DK_MAXK;
  if (lds)
    for (int64_t k = threadIdx.x; k < nk; k += DK_BS) lh[k] = 0u;
  __syncthreads();
  const int64_t i0 = (int64_t)blockIdx.x * DK_BS * DK_ITEMS;
  for (int u = 0; u < DK_ITEMS; ++u) {
    const int64_t it = i0 + (int64_t)u * DK_BS + threadIdx.x;
    if (it >= nit) break;
    const int64_t key = xcd_key(bin_chunk(g, bin_row, items[it]), cpx);
    if (lds) atomicAdd(&lh[key], 1u);
    else atomicAdd(&cnt[key], 1ull);
  }
  __syncthreads();
  if (lds)
    for (int64_t k = threadIdx.x; k < nk; k += DK_BS)
      if (lh[k]) atomicAdd(&cnt[k], (unsigned long long)lh[k]);
}

__global__ void __launch_bounds__(DK_BS)
    k_run_records(ChunkGeom g, const int64_t* __restrict__ items, const int32_t* item_counts,
                  const int64_t* __restrict__ bin_start, const int64_t* __restrict__ bin_cnt,
                  const int32_t* __restrict__ bin_row, const int64_t* __restrict__ seg_beg,
                  int64_t cpx, unsigned long long* cur, int64_t* rec) {
  __shared__ unsigned int lh[DK_MAXK];
  __shared__ unsigned long long lb[DK_MAXK];
  const int64_t nk = N_XCD * cpx, nit = item_counts[0];
  const bool lds = nk <= DK_MAXK;
  const int64_t i0 = (int64_t)blockIdx.x * DK_BS * DK_ITEMS;
  int64_t key[DK_ITEMS];
  if (lds)
    for (int64_t k = threadIdx.x; k < nk; k += DK_BS) lh[k] = 0u;
  __syncthreads();
#pragma unroll
  for (int u = 0; u < DK_ITEMS; ++u) {
    const int64_t it = i0 + (int64_t)u * DK_BS + threadIdx.x;
    key[u] = it < nit ? xcd_key(bin_chunk(g, bin_row, items[it]), cpx) : -1;
    if (lds && key[u] >= 0) atomicAdd(&lh[key[u]], 1u);
  }
  __syncthreads();
  if (lds) {
    // reserve each key's range, then hand out ranks within it
    for (int64_t k = threadIdx.x; k < nk; k += DK_BS) {
      lb[k] = lh[k] ? atomicAdd(&cur[k], (unsigned long long)lh[k]) : 0ull;
      lh[k] = 0u;
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < DK_ITEMS; ++u) {
    if (key[u] < 0) continue;
    const int64_t it = i0 + (int64_t)u * DK_BS + threadIdx.x;
    const int64_t gb = items[it];
    const int64_t pos = lds ? (int64_t)(lb[key[u]] + atomicAdd(&lh[key[u]], 1u))
                            : (int64_t)atomicAdd(&cur[key[u]], 1ull);
    int64_t* r = rec + RUN_REC * pos;
    r[0] = bin_start[gb];
    r[1] = seg_beg[gb];
    r[2] = bin_cnt[gb];
    r[3] = seg_beg[gb + 1] - seg_beg[gb];
    r[4] = bin_chunk(g, bin_row, gb) << g.shift;
    r[5] = gb;
  }
}

// runs staged per window: at most 512, so that two 1024-thread workgroups
// with an f64 accumulator of 2^13 columns fit the LDS of one CU
constexpr int RUN_WIN = 512;

size_t run_dense_lds(int f64, int shift, int block) {
  const size_t L = (size_t)1 << shift, vs = f64 ? 8 : 4;
  const size_t wr = (size_t)std::min(block, RUN_WIN);
  return L * vs + (L / 32) * 4 + wr * (4 + 4 + vs) + (size_t)(block / 4 + 2) * 4 + 128;
}

template <typename CI, typename V, bool NUMERIC>
__global__ void __launch_bounds__(1024)
    k_run_dense(ChunkGeom g, const int64_t* __restrict__ rec, const int32_t* item_counts,
                const run_t* __restrict__ runs, const V* __restrict__ aval,
                const CI* __restrict__ bcol, const V* __restrict__ bval, int64_t* bin_nnz,
                const int64_t* __restrict__ bin_out, void* ccol_, int col64, V* cval,
                unsigned int* work, uint32_t* chunk_bm, const int64_t* __restrict__ xcd_start,
                int64_t cpx) {
  // count mode stores every item's column bitmap in chunk_bm (L / 32 words
  // per item); the numeric phase reads it back instead of setting bits.
  // Items (records in XCD order) are taken from this XCD's counter work[x],
  // then, when it is done, from the others' in turn.
  extern __shared__ __align__(16) unsigned char dsm[];
  constexpr int U = NUMERIC ? MG_RUN_UNROLL : MG_RUN_UNROLL_C;
  const int BS = blockDim.x;
  const int WR = BS < RUN_WIN ? BS : RUN_WIN;
  const int64_t L = (int64_t)1 << g.shift;
  V* acc = (V*)dsm;
  uint32_t* bits = (uint32_t*)(dsm + (NUMERIC ? L * sizeof(V) : 0));
  V* w_av = (V*)(bits + L / 32);
  int32_t* w_pre = (int32_t*)(w_av + (NUMERIC ? WR : 0));
  uint32_t* w_b = (uint32_t*)(w_pre + WR);
  int32_t* s_grp = (int32_t*)(w_b + WR);  // BS / 4 + 1
  __shared__ int64_t sh_w[16];
  __shared__ int64_t sh_item;
  __shared__ int64_t sh_rec[RUN_REC];
  const int t = threadIdx.x;
  const int64_t nitems = item_counts[0];
  const int64_t nwords = L / 32;
  const int SC = 16 * BS, NG = SC / MG_WAVE;
  for (int64_t q = t; q < nwords; q += BS) bits[q] = 0u;
  if (NUMERIC)
    for (int64_t q = t; q < L; q += BS) acc[q] = (V)0;
  const int64_t wpt = (nwords + BS - 1) / BS;
  const int64_t w0 = t * wpt, w1 = (w0 + wpt < nwords) ? (w0 + wpt) : nwords;
  const int wv = t / MG_WAVE, nw = BS / MG_WAVE;
  // thread 0 takes the next item and loads its record while the current
  // one is accumulated
  const int x0 = (int)(blockIdx.x % N_XCD);
  int xs = 0;  // thread 0: XCD lists tried and found done
  auto take = [&]() -> int64_t {
    while (xs < N_XCD) {
      const int x = (x0 + xs) % N_XCD;
      const int64_t lo = xcd_start[x * cpx], hi = xcd_start[(x + 1) * cpx];
      if (lo < hi) {
        const int64_t i = lo + (int64_t)atomicAdd(&work[x], 1u);
        if (i < hi) return i;
      }
      ++xs;
    }
    return nitems;
  };
  int64_t nxt = 0;
  int64_t nr[RUN_REC] = {0, 0, 0, 0, 0, 0};
  if (t == 0) {
    nxt = take();
    if (nxt < nitems)
      for (int k = 0; k < RUN_REC; ++k) nr[k] = rec[RUN_REC * nxt + k];
  }
  for (;;) {
    __syncthreads();
    if (t == 0) {
      sh_item = nxt;
      for (int k = 0; k < RUN_REC; ++k) sh_rec[k] = nr[k];
    }
    __syncthreads();
    const int64_t it = sh_item;
    if (it >= nitems) break;
    const int64_t s0 = sh_rec[0], sg0 = sh_rec[1], cnt = sh_rec[2];
    const int64_t sg1 = sg0 + sh_rec[3], colbase = sh_rec[4], gb = sh_rec[5];
    if (t == 0) {
      nxt = take();
      if (nxt < nitems)
        for (int k = 0; k < RUN_REC; ++k) nr[k] = rec[RUN_REC * nxt + k];
    }
    for (int64_t sb = sg0; sb < sg1; sb += WR) {
      const int64_t s = sb + t;
      if (t < WR && s < sg1) {
        const run_t r = ld_global(&runs[s]);
        w_pre[t] = (int32_t)(run_off(r) - s0);
        w_b[t] = r.z;
        if (NUMERIC) w_av[t] = aval[r.w];
      }
      const int nvalid = (int)((sg1 - sb) < WR ? (sg1 - sb) : WR);
      const int32_t wend = (sb + WR < sg1) ? (int32_t)(run_off_at(runs, sb + WR) - s0) : (int32_t)cnt;
      __syncthreads();
      const int32_t wstart = w_pre[0];
      for (int32_t q0 = wstart; q0 < wend; q0 += SC) {
        const int32_t q1 = (wend - q0 < SC) ? wend : q0 + SC;
        const int32_t ng = (q1 - q0 + MG_WAVE - 1) / MG_WAVE;
        for (int32_t G = t; G < ng; G += BS) s_grp[G] = upper_index(w_pre, 0, nvalid, q0 + G * MG_WAVE);
        if (t == 0) s_grp[NG] = nvalid - 1;
        __syncthreads();
        for (int32_t qb = q0 + t; qb < q1; qb += U * BS) {
          uint32_t bi[U];
          V a4[U];
          bool ok[U];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int32_t q = qb + u * BS;
            ok[u] = q < q1;
            bi[u] = 0;
            a4[u] = (V)0;
            if (ok[u]) {
              const int G = (q - q0) / MG_WAVE;
              const int klo = s_grp[G];
              const int khi = (G + 1 < ng) ? s_grp[G + 1] : s_grp[NG];
              const int i = (khi > klo) ? upper_index(w_pre, klo, khi + 1, q) : klo;
              bi[u] = w_b[i] + (uint32_t)(q - w_pre[i]);
              if (NUMERIC) a4[u] = w_av[i];
            }
          }
          uint32_t c4[U];
          V v4[U];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            c4[u] = ok[u] ? (uint32_t)((int64_t)bcol[bi[u]] - colbase) : 0u;
            if (NUMERIC) v4[u] = ok[u] ? a4[u] * bval[bi[u]] : (V)0;
          }
#pragma unroll
          for (int u = 0; u < U; ++u) {
            if (!ok[u]) continue;
            if (NUMERIC) atomicAdd(&acc[c4[u]], v4[u]);
            else atomicOr(&bits[c4[u] >> 5], 1u << (c4[u] & 31));
          }
        }
        __syncthreads();
      }
    }
    __syncthreads();
    uint32_t* gbm = chunk_bm + it * nwords;
    int64_t my = 0;
    for (int64_t w = w0; w < w1; ++w) my += __popc(NUMERIC ? gbm[w] : bits[w]);
    const int64_t inc = wave_incl_scan(my);
    if (lane() == MG_WAVE - 1) sh_w[wv] = inc;
    __syncthreads();
    int64_t before = 0, total = 0;
    for (int v = 0; v < nw; ++v) {
      if (v < wv) before += sh_w[v];
      total += sh_w[v];
    }
    if (!NUMERIC) {
      if (t == 0) bin_nnz[gb] = total;
      for (int64_t w = w0; w < w1; ++w) {
        gbm[w] = bits[w];
        bits[w] = 0u;
      }
      continue;
    }
    const int64_t obase = bin_out[gb];
    if (nwords <= WR && (nwords & 1) == 0) {
      // every word's first output (w_pre, free here) and the bitmap (bits)
      // in LDS; then each wave writes 64 columns at a time, lane l the
      // column l of the pair of words, at its word's start plus the set bits
      // below it: one store instruction covers consecutive outputs
      int32_t o = (int32_t)(before + inc - my);
      for (int64_t w = w0; w < w1; ++w) {
        const uint32_t bb = gbm[w];
        bits[w] = bb;
        w_pre[w] = o;
        o += __popc(bb);
      }
      __syncthreads();
      const int hl = lane() >> 5, bit = lane() & 31;
      for (int64_t pw = 2 * wv; pw < nwords; pw += 2 * nw) {
        const int64_t w = pw + hl;
        const uint32_t bb = bits[w];
        if ((bb >> bit) & 1u) {
          const int64_t lc = w * 32 + bit;
          const int64_t pos = obase + w_pre[w] + __popc(bb & ((1u << bit) - 1u));
          if (col64) st_stream<HINT_C_STORE>(&((int64_t*)ccol_)[pos], (int64_t)(colbase + lc));
          else st_stream<HINT_C_STORE>(&((int32_t*)ccol_)[pos], (int32_t)(colbase + lc));
          st_stream<HINT_C_STORE>(&cval[pos], acc[lc]);
          acc[lc] = (V)0;
        }
      }
      continue;
    }
    int64_t pos = obase + before + inc - my;
    for (int64_t w = w0; w < w1; ++w) {
      uint32_t bb = gbm[w];
      while (bb) {
        const int bit = __ffs(bb) - 1;
        bb &= bb - 1;
        const int64_t lc = w * 32 + bit;
        if (col64) st_stream<HINT_C_STORE>(&((int64_t*)ccol_)[pos], (int64_t)(colbase + lc));
        else st_stream<HINT_C_STORE>(&((int32_t*)ccol_)[pos], (int32_t)(colbase + lc));
        st_stream<HINT_C_STORE>(&cval[pos], acc[lc]);
        acc[lc] = (V)0;
        ++pos;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Sort accumulation of small chunks from their runs: one wave per packed
// item (<= 64 consecutive chunks of one row, < 1024 products).  The item's
// runs are taken 64 at a time (one per lane, staged in LDS); every lane
// fills its register slots x = e * 64 + lane whose product falls in these
// runs (binary search over the 64 run offsets), with key = column relative
// to the item's first chunk.  Sort, heads of equal columns, segmented sums
// from +0.0 and the write-out follow the product reorder's sort.
// ---------------------------------------------------------------------------
constexpr int RS_WAVES = 4;
// count mode: an item whose chunks span at most this many bitmap words (one
// bit per column) counts its distinct columns in a per-wave LDS bitmap.  4
// KiB per wave leaves the LDS for 32 waves per CU (8 KiB held it to 16:
// R-MAT scale 20, run_count 70.9 -> 62.4 ms; the items over four chunks of
// 2^13 columns that now take the sort cost less than that occupancy)
constexpr int RS_BM_WORDS = 1024;

template <typename CI, typename V, int E, bool NUMERIC>
MG_INLINE void run_sort_item(const ChunkGeom& g, int64_t g0, int nbg,
                             const int64_t* __restrict__ bin_start,
                             const int64_t* __restrict__ bin_cnt,
                             const int32_t* __restrict__ bin_row,
                             const int64_t* __restrict__ seg_beg,
                             const run_t* __restrict__ runs, const V* __restrict__ aval,
                             const CI* __restrict__ bcol, const V* __restrict__ bval,
                             int64_t* bin_nnz, const int64_t* __restrict__ bin_out, void* ccol_,
                             int col64, V* cval, int32_t* w_x0, uint32_t* w_b, V* w_av,
                             int32_t* s_cnt, V* s_v, uint32_t* s_bm) {
  constexpr int CAP = MG_WAVE * E;
  constexpr int IDXB = NUMERIC ? ilog2c(CAP) : 0;
  const int l = lane();
  const int64_t start = bin_start[g0];
  const int P = (int)(bin_start[g0 + nbg - 1] + bin_cnt[g0 + nbg - 1] - start);
  const int64_t sg0 = seg_beg[g0], sg1 = seg_beg[g0 + nbg];
  const int64_t kk = bin_row[g0];
  const int64_t colbase = ((g.minc[g.rows[kk]] >> g.shift) + (g0 - g.binBase[kk])) << g.shift;
  if constexpr (!NUMERIC) {
    // distinct columns per chunk from a bitmap over the item's chunks, when
    // it fits: one bit set per product instead of a sort network
    if (g.shift >= 5 && ((int64_t)nbg << (g.shift - 5)) <= RS_BM_WORDS) {
      const int wpc = 1 << (g.shift - 5);
      const int words = nbg * wpc;
      for (int w = l; w < words; w += MG_WAVE) s_bm[w] = 0u;
      for (int64_t sb = sg0; sb < sg1; sb += MG_WAVE) {
        const int64_t s = sb + l;
        // lanes past the window's runs hold a start above every product
        if (s < sg1) {
          const run_t r = ld_global(&runs[s]);
          w_x0[l] = (int32_t)(run_off(r) - start);
          w_b[l] = r.z;
        } else {
          w_x0[l] = INT32_MAX;
        }
        const int32_t xhi =
            (sb + MG_WAVE < sg1) ? (int32_t)(run_off_at(runs, sb + MG_WAVE) - start) : P;
        wave_sync_r();
        const int32_t xlo = w_x0[0];
        for (int32_t x = xlo + l; x < xhi; x += MG_WAVE) {
          const int i = upper_index64(w_x0, x);
          const uint32_t key = (uint32_t)((int64_t)bcol[w_b[i] + (uint32_t)(x - w_x0[i])] - colbase);
          atomicOr(&s_bm[key >> 5], 1u << (key & 31));
        }
        wave_sync_r();
      }
      for (int c = 0; c < nbg; ++c) {
        int n = 0;
        for (int w = l; w < wpc; w += MG_WAVE) n += __popc(s_bm[c * wpc + w]);
        n = wave_sum(n);
        if (l == 0) bin_nnz[g0 + c] = n;
      }
      return;
    }
  }
  if (!NUMERIC && l < nbg) s_cnt[l] = 0;
  uint32_t k[E];
#pragma unroll
  for (int e = 0; e < E; ++e) k[e] = 0xFFFFFFFFu;
  for (int64_t sb = sg0; sb < sg1; sb += MG_WAVE) {
    const int64_t s = sb + l;
    // lanes past the window's runs hold a start above every product
    if (s < sg1) {
      const run_t r = ld_global(&runs[s]);
      w_x0[l] = (int32_t)(run_off(r) - start);
      w_b[l] = r.z;
      if (NUMERIC) w_av[l] = aval[r.w];
    } else {
      w_x0[l] = INT32_MAX;
    }
    const int32_t xhi =
        (sb + MG_WAVE < sg1) ? (int32_t)(run_off_at(runs, sb + MG_WAVE) - start) : P;
    wave_sync_r();
    const int32_t xlo = w_x0[0];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int x = e * MG_WAVE + l;
      if (x >= xlo && x < xhi) {
        const int i = upper_index64(w_x0, x);
        const uint32_t b = w_b[i] + (uint32_t)(x - w_x0[i]);
        const uint32_t key = (uint32_t)((int64_t)bcol[b] - colbase);
        k[e] = NUMERIC ? ((key << IDXB) | (uint32_t)x) : key;
        if (NUMERIC) s_v[x] = w_av[i] * bval[b];
      }
    }
    wave_sync_r();
  }
  // lane l holds elements l*E .. l*E+E-1 after the sort (blocked layout)
  bitonic_sort_keys<E>(k);
  wave_sync_r();
  const uint32_t prevk = __shfl_up(k[E - 1], 1, MG_WAVE) >> IDXB;
  bool head[E];
  int hc = 0;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int x = l * E + e;
    const uint32_t pk = (e == 0) ? prevk : (k[e - 1] >> IDXB);
    head[e] = (x < P) && (x == 0 || (k[e] >> IDXB) != pk);
    hc += head[e] ? 1 : 0;
  }
  if (!NUMERIC) {
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (head[e]) atomicAdd(&s_cnt[k[e] >> g.shift], 1);
    wave_sync_r();
    if (l < nbg) bin_nnz[g0 + l] = s_cnt[l];
    return;
  } else {
    V v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int x = l * E + e;
      v[e] = (x < P) ? s_v[k[e] & (CAP - 1)] : (V)0;
    }
    const int hinc = wave_incl_scan(hc);
    const int hbase = hinc - hc;
    V t = (V)0;
    bool anyh = false;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if (head[e]) { t = (V)0 + v[e]; anyh = true; }
      else t = t + v[e];
    }
    V s = t;
    bool f = anyh;
#pragma unroll
    for (int d = 1; d < MG_WAVE; d <<= 1) {
      const V ps = __shfl_up(s, d, MG_WAVE);
      const int pf = __shfl_up((int)f, d, MG_WAVE);
      if (l >= d && !f) { s = ps + s; f = pf != 0; }
    }
    V carry = __shfl_up(s, 1, MG_WAVE);
    if (l == 0) carry = (V)0;
    const uint32_t nextk = __shfl_down(k[0], 1, MG_WAVE) >> IDXB;
    const int64_t obase = bin_out[g0];
    V run = carry;
    int hr = hbase;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int x = l * E + e;
      if (head[e]) { run = (V)0 + v[e]; ++hr; }
      else run = run + v[e];
      const uint32_t key = k[e] >> IDXB;
      const uint32_t nk = (e == E - 1) ? nextk : (k[e + 1] >> IDXB);
      const bool tail = (x < P) && (x == P - 1 || nk != key);
      if (tail) {
        const int64_t pos = obase + hr - 1;
        const int64_t col = colbase + (int64_t)key;
        if (col64) st_stream<HINT_C_STORE>(&((int64_t*)ccol_)[pos], (int64_t)col);
        else st_stream<HINT_C_STORE>(&((int32_t*)ccol_)[pos], (int32_t)col);
        st_stream<HINT_C_STORE>(&cval[pos], run);
      }
    }
  }
}

template <typename CI, typename V, bool NUMERIC>
__global__ void __launch_bounds__(RS_WAVES * MG_WAVE)
    k_run_sort(ChunkGeom g, const int64_t* __restrict__ items, const int32_t* item_counts,
               const int64_t* __restrict__ bin_start, const int64_t* __restrict__ bin_cnt,
               const int32_t* __restrict__ bin_row, const int64_t* __restrict__ seg_beg,
               const run_t* __restrict__ runs, const V* __restrict__ aval,
               const CI* __restrict__ bcol, const V* __restrict__ bval, int64_t* bin_nnz,
               const int64_t* __restrict__ bin_out, void* ccol_, int col64, V* cval,
               int64_t it0) {
  __shared__ int32_t s_x0[RS_WAVES][MG_WAVE];
  __shared__ uint32_t s_b[RS_WAVES][MG_WAVE];
  __shared__ V s_av[RS_WAVES][NUMERIC ? MG_WAVE : 1];
  __shared__ int32_t s_cnt[RS_WAVES][MG_WAVE];
  __shared__ V s_v[RS_WAVES][NUMERIC ? SORT_CAP : 1];
  __shared__ uint32_t s_bm[RS_WAVES][NUMERIC ? 1 : RS_BM_WORDS];
  const int w = threadIdx.x / MG_WAVE;
  const int64_t it = it0 + (int64_t)blockIdx.x * RS_WAVES + w;
  if (it >= item_counts[1]) return;
  const int64_t g0 = items[2 * it];
  const int nbg = (int)items[2 * it + 1];
  const int64_t P = bin_start[g0 + nbg - 1] + bin_cnt[g0 + nbg - 1] - bin_start[g0];
#define MG_RS(E)                                                                                  \
  run_sort_item<CI, V, E, NUMERIC>(g, g0, nbg, bin_start, bin_cnt, bin_row, seg_beg, runs,       \
                                   aval, bcol, bval, bin_nnz, bin_out, ccol_,                    \
                                   col64, cval, s_x0[w], s_b[w], s_av[w], s_cnt[w], s_v[w],  \
                                   s_bm[w])
  if (P <= 64) MG_RS(1);
  else if (P <= 128) MG_RS(2);
  else if (P <= 256) MG_RS(4);
  else if (P <= 512) MG_RS(8);
  else MG_RS(16);
#undef MG_RS
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_bci(const Mats& M, int shift, bool fill, int64_t* cnt, const int64_t* ptr,
                      uint32_t* pos, uint32_t* chunk, hipStream_t st) {
  if (M.k <= 0) return hipSuccess;
  const unsigned grid = (unsigned)std::min<int64_t>((M.k + 3) / 4, 1 << 16);
  MG_DISPATCH2(M, {
    if (fill)
      hipLaunchKernelGGL((k_bci<RP, CI, true>), grid, 256, 0, st, (const RP*)M.brp,
                         (const CI*)M.bcol, M.k, shift, cnt, ptr, pos, chunk);
    else
      hipLaunchKernelGGL((k_bci<RP, CI, false>), grid, 256, 0, st, (const RP*)M.brp,
                         (const CI*)M.bcol, M.k, shift, cnt, ptr, pos, chunk);
  });
  return hipGetLastError();
}

hipError_t launch_run_count(const Mats& M, const int32_t* rows, int64_t nrows, const int64_t* bptr,
                            const int64_t* ip, unsigned long long* out, hipStream_t st) {
  if (nrows <= 0) return hipSuccess;
  const unsigned grid = (unsigned)std::min<int64_t>((nrows + 3) / 4, 4096);
  MG_DISPATCH2(M, hipLaunchKernelGGL((k_run_count<RP, CI>), grid, 256, 0, st, (const RP*)M.arp,
                                      (const CI*)M.acol, rows, nrows, bptr, ip, out));
  return hipGetLastError();
}

hipError_t launch_run_rows(const Mats& M, const ChunkGeom& g, bool hist, const int64_t* bptr,
                           const uint32_t* bpos, const uint32_t* bchunk, int64_t max_nb,
                           int64_t* bin_seg, int64_t* bin_cnt, int32_t* bin_row,
                           const int64_t* seg_beg, const int64_t* bin_start, run_t* runs,
                           hipStream_t st) {
  if (g.nch <= 0) return hipSuccess;
  const size_t lds = run_rows_lds(max_nb);
  const int64_t cap = max_grid(RR_BS);
  for (int64_t o = 0; o < g.nch; o += cap) {
    const unsigned grid = (unsigned)std::min(cap, g.nch - o);
    MG_DISPATCH2(M, {
      auto kf = hist ? k_run_rows<RP, CI, true> : k_run_rows<RP, CI, false>;
      (void)hipFuncSetAttribute((const void*)kf, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds);
      hipLaunchKernelGGL(kf, grid, RR_BS, lds, st, (const RP*)M.arp, (const CI*)M.acol, g, bptr,
                         bpos, bchunk, o, bin_seg, bin_cnt, bin_row, seg_beg, bin_start, runs);
    });
  }
  return hipGetLastError();
}

hipError_t launch_dense_order(const ChunkGeom& g, int64_t nitems, const int64_t* dense_items,
                              const int32_t* item_counts, const int32_t* bin_row, int64_t cpx,
                              int64_t* xcd_start, int64_t* xcd_cur, void* temp, hipStream_t st) {
  const int64_t nk = N_XCD * cpx;
  hipError_t e = launch_fill_i64(xcd_start, nk + 1, 0, st);
  if (e != hipSuccess) return e;
  const int64_t per = (int64_t)DK_BS * DK_ITEMS;
  if (nitems > 0)
    hipLaunchKernelGGL(k_dense_key_hist, (unsigned)((nitems + per - 1) / per), DK_BS, 0, st, g,
                       dense_items, item_counts, bin_row, cpx, (unsigned long long*)xcd_start);
  e = scan_excl_i64(xcd_start, xcd_start, nk, xcd_start + nk, nullptr, temp, st);
  if (e != hipSuccess) return e;
  return hipMemcpyAsync(xcd_cur, xcd_start, sizeof(int64_t) * (nk + 1), hipMemcpyDeviceToDevice,
                        st);
}

hipError_t launch_run_records(const ChunkGeom& g, int64_t nitems, const int64_t* dense_items,
                              const int32_t* item_counts, const int64_t* bin_start,
                              const int64_t* bin_cnt, const int32_t* bin_row,
                              const int64_t* seg_beg, int64_t cpx, int64_t* xcd_cur,
                              int64_t* rec, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  const int64_t per = (int64_t)DK_BS * DK_ITEMS;
  hipLaunchKernelGGL(k_run_records, (unsigned)((nitems + per - 1) / per), DK_BS, 0, st, g,
                     dense_items, item_counts, bin_start, bin_cnt, bin_row, seg_beg, cpx,
                     (unsigned long long*)xcd_cur, rec);
  return hipGetLastError();
}

hipError_t launch_run_accum(const Mats& M, const ChunkGeom& g, int64_t nbins, bool numeric,
                            const int64_t* bin_start, const int64_t* bin_cnt,
                            const int32_t* bin_row, const int64_t* dense_rec,
                            const int64_t* sort_items, const int32_t* item_counts,
                            const int64_t* seg_beg, const run_t* runs, int64_t* bin_nnz,
                            const int64_t* bin_out,
                            void* ccol, int col64, void* cval, int dense_block,
                            unsigned int* work, int persistent_wgs, uint32_t* chunk_bm,
                            int64_t n_sort_items, const int64_t* xcd_start, int64_t cpx,
                            hipStream_t st) {
  if (nbins <= 0) return hipSuccess;
  // count mode keeps no values in LDS and runs RUN_COUNT_BLOCK threads per
  // workgroup
  const int db = numeric ? dense_block : RUN_COUNT_BLOCK;
  const size_t lds = run_dense_lds(M.f64, g.shift, db) -
                     (numeric ? 0 : ((size_t)1 << g.shift) * (M.f64 ? 8 : 4) +
                                        (size_t)std::min(db, RUN_WIN) * (M.f64 ? 8 : 4));
  const unsigned gd = (unsigned)std::min<int64_t>(nbins, persistent_wgs);
  // one wave per sort item: the count the host read back (the grid is not
  // sized by the bins, mostly empty waves), the bins when it is not known
  const int64_t nsi = n_sort_items >= 0 ? n_sort_items : nbins;
  const int64_t gs_all = (nsi + RS_WAVES - 1) / RS_WAVES;
  const int64_t gcap = max_grid(RS_WAVES * MG_WAVE);
#define MG_RA(CI, V)                                                                              \
  {                                                                                               \
    auto kd = numeric ? k_run_dense<CI, V, true> : k_run_dense<CI, V, false>;                     \
    (void)hipFuncSetAttribute((const void*)kd, hipFuncAttributeMaxDynamicSharedMemorySize,        \
                              (int)lds);                                                          \
    hipLaunchKernelGGL(kd, gd, db, lds, st, g, dense_rec,          item_counts, runs,             \
                       (const V*)M.aval, (const CI*)M.bcol, (const V*)M.bval, bin_nnz,     \
                       bin_out, ccol, col64, (V*)cval, work, chunk_bm, xcd_start, cpx);           \
    auto ks = numeric ? k_run_sort<CI, V, true> : k_run_sort<CI, V, false>;                       \
    for (int64_t o = 0; o < gs_all; o += gcap)                                                    \
      hipLaunchKernelGGL(ks, (unsigned)std::min(gcap, gs_all - o), RS_WAVES * MG_WAVE, 0, st, g,  \
                         sort_items, item_counts, bin_start, bin_cnt, bin_row, seg_beg, runs,     \
                         (const V*)M.aval, (const CI*)M.bcol, (const V*)M.bval,     \
                         bin_nnz, bin_out, ccol, col64, (V*)cval, o * RS_WAVES);                  \
  }
  if (M.col64) {
    if (M.f64) MG_RA(int64_t, double) else MG_RA(int64_t, float)
  } else {
    if (M.f64) MG_RA(int32_t, double) else MG_RA(int32_t, float)
  }
#undef MG_RA
  return hipGetLastError();
}

}  // namespace mg
