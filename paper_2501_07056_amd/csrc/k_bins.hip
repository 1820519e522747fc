// CHUNKED rows: reorder each row's intermediate product into column chunks
// of 2^shift columns (histogram, prefix sum, reorder; Algorithm 3), then
// accumulate every chunk on chip (Section 3.4): a dense accumulator in LDS for
// chunks with many products, a wavefront sort for small ones, several
// consecutive small chunks of a row packed into one sort (Section 4.1.1
// combines chunks so a sort is near its best size).
//
// Work units: a row's products (in the order of Eq. 1) are cut into tiles of
// `tile` products; one workgroup bins one tile.  Per (row, chunk, tile) the
// tile's count is stored in a table whose prefix sum (row-major, chunk, then
// tile) gives every tile a private, contiguous destination inside every chunk,
// so the reorder needs no global atomics and is deterministic.
#include <algorithm>
#include <type_traits>

#include "common.h"
#include "kernels.h"
#include "dispatch.h"

namespace mg {

MG_INLINE void wave_sync2() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

// ---------------------------------------------------------------------------
// geometry of CHUNKED rows
// ---------------------------------------------------------------------------
__global__ void k_chunk_geom(const int32_t* rows, const int64_t* ip, const int64_t* minc,
                             const int64_t* maxc, int64_t nch, int shift, int tile, int64_t* nb,
                             int64_t* nt, int64_t* ipr) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nch) return;
  const int32_t r = rows[k];
  const int64_t b = (maxc[r] >> shift) - (minc[r] >> shift) + 1;
  const int64_t t = (ip[r] + tile - 1) / tile;
  nb[k] = b;
  nt[k] = t;
  ipr[k] = ip[r];
}

hipError_t launch_chunk_geom(const ChunkGeom& g, hipStream_t st) {
  // ipBase doubles as the per-row ip input of its own scan (in place)
  if (g.nch <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_chunk_geom, (unsigned)((g.nch + 255) / 256), 256, 0, st, g.rows, g.ip,
                     g.minc, g.maxc, g.nch, g.shift, g.tile, g.nb, g.nt, g.ipBase);
  return hipGetLastError();
}

// first_of[s] = first CHUNKED row whose product range starts in [s*W, (s+1)*W)
// bases[s*3 + {0,1,2}] = ipBase, tileBase, binBase at that row
__global__ void k_batch_bounds(const int64_t* ipBase, const int64_t* tileBase,
                               const int64_t* binBase, int64_t nch, int64_t W, int32_t* first_of,
                               int64_t* bases) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nch) return;
  const int64_t s = ipBase[k] / W;
  if (k == 0 || ipBase[k - 1] / W != s) {
    first_of[s] = (int32_t)k;
    bases[s * 3 + 0] = ipBase[k];
    bases[s * 3 + 1] = tileBase[k];
    bases[s * 3 + 2] = binBase[k];
  }
}

hipError_t launch_batch_bounds(const ChunkGeom& g, int64_t W, int32_t* first_of, int64_t* bases,
                                hipStream_t st) {
  if (g.nch <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_bounds, (unsigned)((g.nch + 255) / 256), 256, 0, st, g.ipBase,
                     g.tileBase, g.binBase, g.nch, W, first_of, bases);
  return hipGetLastError();
}

// aoff[e] = offset of A entry e's products inside its row (exclusive scan of
// B row lengths along the row); one wave per CHUNKED row
template <typename RP, typename CI>
__global__ void __launch_bounds__(256) k_aoff(const RP* __restrict__ arp, const CI* __restrict__ acol,
                                              const RP* __restrict__ brp, const int32_t* rows,
                                              int64_t nrows, int64_t* aoff, int64_t* ent) {
  const int64_t k = (int64_t)blockIdx.x * 4 + threadIdx.x / MG_WAVE;
  if (k >= nrows) return;
  const int l = lane();
  const int32_t r = rows[k];
  const int64_t a0 = arp[r], a1 = arp[r + 1];
  if (l == 0) ent[k] = a1 - a0;
  int64_t carry = 0;
  for (int64_t e0 = a0; e0 < a1; e0 += MG_WAVE) {
    const int64_t e = e0 + l;
    int64_t len = 0;
    if (e < a1) {
      const int64_t j = acol[e];
      len = (int64_t)brp[j + 1] - (int64_t)brp[j];
    }
    const int64_t inc = wave_incl_scan(len);
    if (e < a1) aoff[e] = carry + inc - len;
    carry += __shfl(inc, MG_WAVE - 1, MG_WAVE);
  }
}

__global__ void k_tiles(const int64_t* nt, const int64_t* tileBase, int64_t k0, int64_t k1,
                        int32_t* tile_row) {
  const int64_t k = k0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= k1) return;
  const int64_t b = tileBase[k], n = nt[k];
  for (int64_t t = 0; t < n; ++t) tile_row[b + t] = (int32_t)k;
}

hipError_t launch_tiles(const int64_t* nt, const int64_t* tileBase, int64_t k0, int64_t k1,
                        int32_t* tile_row, hipStream_t st) {
  if (k1 <= k0) return hipSuccess;
  hipLaunchKernelGGL(k_tiles, (unsigned)((k1 - k0 + 255) / 256), 256, 0, st, nt, tileBase, k0, k1,
                     tile_row);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Tile expansion shared by the histogram and reorder passes: the workgroup
// walks the A entries overlapping its product range [p0, p1) in windows of
// blockDim entries; each window's entry offsets sit in LDS and every thread
// finds the owner of its product by binary search.
// ---------------------------------------------------------------------------
constexpr int BIN_BS = 256;

struct TileCtx {
  int64_t row, k, ti, p0, p1, a0, a1, e0, base_bin, nbk, ntk;
};

template <typename RP>
MG_INLINE void tile_setup(const ChunkGeom& g, const BatchArgs& b, const int32_t* tile_row,
                          const RP* arp, const int64_t* aoff, TileCtx& c,
                          const int64_t* tile_e0 = nullptr) {
  const int64_t tg = b.tile0 + blockIdx.x;
  c.k = tile_row[tg];
  c.ti = tg - g.tileBase[c.k];
  c.row = g.rows[c.k];
  c.p0 = c.ti * (int64_t)g.tile;
  const int64_t ipr = g.ip[c.row];
  c.p1 = (c.p0 + g.tile < ipr) ? (c.p0 + g.tile) : ipr;
  c.a0 = arp[c.row];
  c.a1 = arp[c.row + 1];
  c.base_bin = g.minc[c.row] >> g.shift;
  c.nbk = g.nb[c.k];
  c.ntk = g.nt[c.k];
  if (tile_e0) {
    c.e0 = tile_e0[tg];
    return;
  }
  // first entry whose products reach past p0: largest e with aoff[e] <= p0
  int64_t lo = c.a0, hi = c.a1;
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (aoff[mid] <= c.p0) lo = mid; else hi = mid;
  }
  c.e0 = lo;
}

// First A entry of every tile (largest e with aoff[e] <= the tile's first
// product), one thread per tile: the searches' latencies overlap here instead
// of stalling every reorder workgroup at its start.
template <typename RP>
__global__ void k_tile_e0(const RP* __restrict__ arp, ChunkGeom g, const int32_t* tile_row,
                          const int64_t* __restrict__ aoff, int64_t ntiles, int64_t* tile_e0) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntiles) return;
  const int64_t k = tile_row[t];
  const int64_t p0 = (t - g.tileBase[k]) * (int64_t)g.tile;
  const int32_t row = g.rows[k];
  int64_t lo = arp[row], hi = arp[row + 1];
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (aoff[mid] <= p0) lo = mid; else hi = mid;
  }
  tile_e0[t] = lo;
}

// products gathered per lane before any is used (count-only expansions)
#ifndef MG_EXPAND_UNROLL
#define MG_EXPAND_UNROLL 4
#endif

// Calls f(q, col, prod) for every product q in [0, p1 - p0) of a row's
// product range [p0, p1) (the order of Eq. 1), where col is the product's
// column and prod = a_ij * b_jk (only when WANT_VAL).  The A entries
// overlapping the range are staged in LDS in windows of BS entries (their
// product offsets relative to p0, B row starts, A values); threads take
// products striped by BS, so the B loads of a wave are contiguous.  The
// window's products are taken in super-chunks of 16*BS: first the A entry
// holding the first product of every group of 64 products is recorded (one
// binary search over the window per group), then a
// product's entry is found by a binary search between the entries of its
// group's start and the next group's start (0 steps inside long B rows, a
// few for short ones).  Four products per thread are gathered before any is
// used.  Offsets into B are 32-bit when B's row pointers are.
template <int BS, typename RP, typename CI, typename V, bool WANT_VAL, typename F,
          int U = MG_EXPAND_UNROLL>
MG_INLINE void expand_products(int64_t p0, int64_t p1, int64_t e0, int64_t a1,
                               const CI* __restrict__ acol, const V* __restrict__ aval,
                               const RP* __restrict__ brp, const CI* __restrict__ bcol,
                               const V* __restrict__ bval, const int64_t* __restrict__ aoff,
                               int32_t* w_pre, int64_t* w_b0, V* w_av, F&& f) {
  using OFF = typename std::conditional<sizeof(RP) == 4, int32_t, int64_t>::type;
  constexpr int SC = 16 * BS;            // products per super-chunk
  constexpr int NG = SC / MG_WAVE;       // groups of 64 products per super-chunk
  __shared__ int32_t s_grp[NG + 1];
  OFF* w_off = (OFF*)w_b0;
  const int t = threadIdx.x;
  // offsets relative to p0 fit 32 bits: the range spans < 2^31 products
  const int32_t span = (int32_t)(p1 - p0);
  for (int64_t eb = e0; eb < a1; eb += BS) {
    const int64_t e = eb + t;
    int64_t pre = INT32_MAX;
    OFF b0 = 0;
    V av = (V)0;
    if (e < a1) {
      pre = aoff[e] - p0;
      if (pre > INT32_MAX) pre = INT32_MAX;
      const int64_t j = acol[e];
      b0 = (OFF)brp[j];
      if (WANT_VAL) av = aval[e];
    }
    w_pre[t] = (int32_t)pre;
    w_off[t] = b0;
    if (WANT_VAL) w_av[t] = av;
    const int nvalid = (int)((a1 - eb) < BS ? (a1 - eb) : BS);
    __syncthreads();
    const int32_t wstart = w_pre[0] > 0 ? w_pre[0] : 0;
    const int64_t we = (eb + BS < a1) ? (aoff[eb + BS] - p0) : (int64_t)span;
    const int32_t wend = (int32_t)(we < span ? we : span);
    for (int32_t s0 = wstart; s0 < wend; s0 += SC) {
      const int32_t s1 = (wend - s0 < SC) ? wend : s0 + SC;
      // the entry holding each group start s0 + 64 G (entries partition the
      // products; empty entries hold none): one search per group, so a long
      // entry does not mark its groups one by one while the others wait
      {
        const int32_t ng = (s1 - s0 + MG_WAVE - 1) / MG_WAVE;
        for (int32_t G = t; G < ng; G += BS)
          s_grp[G] = upper_index(w_pre, 0, nvalid, s0 + G * MG_WAVE);
      }
      if (t == 0) s_grp[NG] = nvalid - 1;
      __syncthreads();
      const int32_t ngr = (s1 - s0 + MG_WAVE - 1) / MG_WAVE;
      for (int32_t qb = s0 + t; qb < s1; qb += U * BS) {
      OFF bi[U];
      V a4[U];
      bool ok[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int32_t q = qb + u * BS;
        ok[u] = q < s1;
        bi[u] = 0;
        a4[u] = (V)0;
        if (ok[u]) {
          const int G = (q - s0) / MG_WAVE;
          const int klo = s_grp[G];
          const int khi = (G + 1 < ngr) ? s_grp[G + 1] : s_grp[NG];
          const int k = (khi > klo) ? upper_index(w_pre, klo, khi + 1, q) : klo;
          bi[u] = w_off[k] + (OFF)(q - w_pre[k]);
          if (WANT_VAL) a4[u] = w_av[k];
        }
      }
      CI c4[U];
      V v4[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        c4[u] = ok[u] ? bcol[bi[u]] : (CI)0;
        if (WANT_VAL) v4[u] = ok[u] ? a4[u] * bval[bi[u]] : (V)0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (ok[u]) f(qb + u * BS, c4[u], WANT_VAL ? v4[u] : (V)0);
      }
      __syncthreads();
    }
    __syncthreads();
    if (wend >= span) break;
  }
}

// ---------------------------------------------------------------------------
// Histogram pass: per tile, products per chunk, added into the chunk's total
// (one global atomic per non-empty chunk of the tile); the first tile of a
// row also records the row of each of its chunks.
// ---------------------------------------------------------------------------
template <typename RP, typename CI>
__global__ void __launch_bounds__(BIN_BS)
    k_bin_hist(const RP* __restrict__ arp, const CI* __restrict__ acol, const RP* __restrict__ brp,
               const CI* __restrict__ bcol, ChunkGeom g, BatchArgs b,
               const int32_t* __restrict__ tile_row, const int64_t* __restrict__ aoff,
               const int64_t* __restrict__ tile_e0, unsigned long long* bin_cnt,
               int32_t* bin_row) {
  extern __shared__ __align__(16) unsigned char dsm[];
  int32_t* w_pre = (int32_t*)dsm;                        // BIN_BS
  int64_t* w_b0 = (int64_t*)(dsm + BIN_BS * 8);            // BIN_BS
  int32_t* hist = (int32_t*)(w_b0 + BIN_BS);               // nb
  TileCtx c;
  tile_setup<RP>(g, b, tile_row, arp, aoff, c, tile_e0);
  for (int64_t q = threadIdx.x; q < c.nbk; q += BIN_BS) hist[q] = 0;
  __syncthreads();
  expand_products<BIN_BS, RP, CI, float, false>(
      c.p0, c.p1, c.e0, c.a1, acol, (const float*)nullptr, brp, bcol, (const float*)nullptr, aoff,
      w_pre, w_b0, (float*)nullptr, [&](int32_t, CI col, float) {
        const uint32_t bin = (uint32_t)(col >> g.shift) - (uint32_t)c.base_bin;
        int hl, len;
        wave_run(bin, hl, len);
        if (lane() == hl) atomicAdd(&hist[bin], len);
      });
  __syncthreads();
  const int64_t gb = g.binBase[c.k];
  for (int64_t q = threadIdx.x; q < c.nbk; q += BIN_BS) {
    const int h = hist[q];
    if (h > 0) atomicAdd(&bin_cnt[gb + q], (unsigned long long)h);
    if (c.ti == 0) bin_row[gb + q] = (int32_t)c.k;
  }
}

// ---------------------------------------------------------------------------
// Symbolic phase of a CHUNKED row with the whole row's column bitmap in LDS
// (the symbolic phase needs only the bitmap, Section 3.5: s_denseAccum = 1).
// One workgroup per row: every product sets its column bit and counts into
// its chunk; then per chunk the distinct columns (popcount of the chunk's
// bits) and the products are written, and the row's nnz.
// ---------------------------------------------------------------------------
// LDS bitmaps of a row or coarse chunk: cleared and counted 16 bytes per
// access where the words allow it (a quarter of the LDS instructions of
// word accesses; the bitmap, not the products, dominates sparse chunks).
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
MG_INLINE void lds_clear_words(uint32_t* bits, int64_t nwords, int t, int bs) {
  u32x4_t* b4 = (u32x4_t*)bits;  // 16-byte aligned
  const int64_t n4 = nwords >> 2;
  for (int64_t q = t; q < n4; q += bs) b4[q] = u32x4_t{0u, 0u, 0u, 0u};
  for (int64_t q = (n4 << 2) + t; q < nwords; q += bs) bits[q] = 0u;
}
// this lane's share (words lane, lane + 64, ...) of the set bits of p[0, n)
MG_INLINE unsigned long long lds_popc_words(const uint32_t* p, int64_t n) {
  unsigned long long s = 0;
  if ((n & 3) == 0 && ((uintptr_t)p & 15) == 0) {
    const u32x4_t* p4 = (const u32x4_t*)p;
    for (int64_t q = lane(); q < (n >> 2); q += MG_WAVE) {
      const u32x4_t x = p4[q];
      s += __popc(x.x) + __popc(x.y) + __popc(x.z) + __popc(x.w);
    }
  } else {
    for (int64_t q = lane(); q < n; q += MG_WAVE) s += __popc(p[q]);
  }
  return s;
}

constexpr int RB_BS = 1024;

size_t row_bitmap_lds(int shift, int64_t max_nb) {
  const size_t words = ((size_t)max_nb << shift) / 32;
  // + static LDS of the expansion (group owners) and the row total
  return words * 4 + (size_t)max_nb * 4 + RB_BS * 16 + 64 + 1024;
}

template <typename RP, typename CI>
__global__ void __launch_bounds__(RB_BS)
    k_row_bitmap(const RP* __restrict__ arp, const CI* __restrict__ acol, const RP* __restrict__ brp,
                 const CI* __restrict__ bcol, ChunkGeom g, const int64_t* __restrict__ aoff,
                 int64_t* bin_nnz, int64_t* bin_cnt, int32_t* bin_row, int64_t* rownnz,
                 int64_t k0) {
  extern __shared__ __align__(16) unsigned char dsm[];
  const int64_t k = k0 + blockIdx.x;
  const int32_t row = g.rows[k];
  const int64_t nbk = g.nb[k], bb = g.binBase[k];
  const int sh = g.shift;
  const int64_t base = (g.minc[row] >> sh) << sh;
  const int64_t nwords = (nbk << sh) >> 5;
  int32_t* w_pre = (int32_t*)dsm;
  int64_t* w_b0 = (int64_t*)(dsm + RB_BS * 8);
  uint32_t* bits = (uint32_t*)(w_b0 + RB_BS);
  int32_t* cnt = (int32_t*)(bits + nwords);
  __shared__ unsigned long long tot;
  lds_clear_words(bits, nwords, threadIdx.x, RB_BS);
  for (int64_t q = threadIdx.x; q < nbk; q += RB_BS) cnt[q] = 0;
  if (threadIdx.x == 0) tot = 0;
  __syncthreads();
  const int64_t a0 = arp[row], a1 = arp[row + 1];
  expand_products<RB_BS, RP, CI, float, false>(
      0, g.ip[row], a0, a1, acol, (const float*)nullptr, brp, bcol, (const float*)nullptr, aoff,
      w_pre, w_b0, (float*)nullptr, [&](int32_t, CI col, float) {
        const uint32_t lc = (uint32_t)col - (uint32_t)base;
        atomicOr(&bits[lc >> 5], 1u << (lc & 31));
        const uint32_t bin = lc >> sh;
        int hl, len;
        wave_run(bin, hl, len);
        if (lane() == hl) atomicAdd(&cnt[bin], len);
      });
  __syncthreads();
  // one wave per chunk: popcount of the chunk's words
  const int w = threadIdx.x / MG_WAVE, nw = RB_BS / MG_WAVE;
  const int64_t wpb = ((int64_t)1 << sh) >> 5;
  for (int64_t b = w; b < nbk; b += nw) {
    unsigned long long s = lds_popc_words(bits + b * wpb, wpb);
    s = wave_sum(s);
    if (lane() == 0) {
      bin_nnz[bb + b] = (int64_t)s;
      bin_cnt[bb + b] = cnt[b];
      bin_row[bb + b] = (int32_t)k;
      atomicAdd(&tot, s);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) rownnz[row] = (int64_t)tot;
}

// ---------------------------------------------------------------------------
// Numeric reorder of a tile with chunk ranges reserved by atomics: the tile's
// products are gathered once into LDS (unsorted, with their chunk), counted
// per chunk, each chunk's range inside its bin is reserved with one atomic
// add on that bin's cursor, the products are ranked within their chunk, and
// every chunk's run is copied out contiguously.
// ---------------------------------------------------------------------------
// Exclusive scan of a[0, n) into out[0, n) (both LDS) by a workgroup of BS
// threads; tmp holds BS / 64 ints.  Ends with a barrier.
template <int BS>
MG_INLINE void block_excl_scan(const int32_t* a, int32_t* out, int64_t n, int32_t* tmp) {
  const int t = threadIdx.x;
  const int64_t per = (n + BS - 1) / BS;
  const int64_t i0 = t * per, i1 = (i0 + per < n) ? (i0 + per) : n;
  int32_t s = 0;
  for (int64_t i = i0; i < i1; ++i) s += a[i];
  const int32_t inc = wave_incl_scan(s);
  const int w = t / MG_WAVE;
  if (lane() == MG_WAVE - 1) tmp[w] = inc;
  __syncthreads();
  int32_t run = inc - s;
  for (int v = 0; v < w; ++v) run += tmp[v];
  for (int64_t i = i0; i < i1; ++i) {
    out[i] = run;
    run += a[i];
  }
  __syncthreads();
}

// Chunk-local columns go out as 16-bit words (chunks of <= 2^16 columns) or,
// for the coarse level's chunks, as 32-bit words.
// With `sorted`, the staged tile is written out in chunk order (as in the
// level-2 reorder below), so that a wave stores consecutive addresses of one
// chunk's run even where the expansion order interleaves many chunks: a
// 16-bit index per position of the chunk-ordered tile names the staged
// product to store there (2 bytes per product instead of a second copy of
// the tile, so that tiles twice as long fit and the runs per chunk double).
// The chunk-ordered reorder of 32-bit columns (the coarse level's first
// reorder, where a tile spreads over hundreds of chunks and one tile fills
// the LDS of a CU) runs `block` threads (256, 512 or 1024), so that the
// gathers of more waves are in flight; the other modes run BIN_BS.
static int scatter2_block(int lc32, int sorted, int block) {
  return (lc32 && sorted && block > 0) ? block : BIN_BS;
}

size_t bin_scatter2_lds(int f64, int tile, int64_t max_nb, int lc32, int sorted, int block) {
  const size_t vs = f64 ? 8 : 4;
  const size_t w = 4 + (lc32 ? 2 : 0);
  size_t b = (size_t)scatter2_block(lc32, sorted, block) * (8 + 8 + 8) + (size_t)max_nb * (4 + 8) + 16 + (size_t)tile * (4 + w) + 16 +
             (size_t)tile * vs + 64;
  if (sorted) b += (size_t)max_nb * 4 + 16 + (size_t)tile * 2 + 16;
  return b;
}

template <int BS, typename RP, typename CI, typename V, typename LC, bool NUMERIC, bool SORTED>
__global__ void __launch_bounds__(BS)
    k_bin_scatter2(const RP* __restrict__ arp, const CI* __restrict__ acol, const V* __restrict__ aval,
                   const RP* __restrict__ brp, const CI* __restrict__ bcol, const V* __restrict__ bval,
                   ChunkGeom g, BatchArgs b, const int32_t* __restrict__ tile_row,
                   const int64_t* __restrict__ aoff, const int64_t* __restrict__ tile_e0,
                   const int64_t* __restrict__ bin_start, unsigned long long* bin_cursor,
                   LC* ws_col, V* ws_val) {
  constexpr bool W16 = sizeof(LC) == 2;
  extern __shared__ __align__(16) unsigned char dsm[];
  int32_t* w_pre = (int32_t*)dsm;
  int64_t* w_b0 = (int64_t*)(dsm + BS * 8);
  V* w_av = (V*)(w_b0 + BS);
  TileCtx c;
  tile_setup<RP>(g, b, tile_row, arp, aoff, c, tile_e0);
  int32_t* hist = (int32_t*)((char*)w_av + BS * 8);
  int64_t* dst = (int64_t*)(((uintptr_t)(hist + c.nbk) + 15) & ~(uintptr_t)15);
  uint32_t* u_word = (uint32_t*)(dst + c.nbk);
  uint32_t* u_rank = u_word + g.tile;
  uint16_t* u_bin = (uint16_t*)(u_rank + g.tile);  // 32-bit columns: the chunk apart
  V* u_val = (V*)(((uintptr_t)(u_bin + (W16 ? 0 : g.tile)) + 15) & ~(uintptr_t)15);
  // chunk order of the tile (SORTED): each chunk's first position, and the
  // staged product at every position
  int32_t* loff = (int32_t*)(u_val + g.tile);
  uint16_t* s_idx = (uint16_t*)(((uintptr_t)(loff + c.nbk) + 15) & ~(uintptr_t)15);
  __shared__ int32_t s_tmp[BS / MG_WAVE];

  for (int64_t q = threadIdx.x; q < c.nbk; q += BS) hist[q] = 0;
  __syncthreads();
  const int64_t lmask = ((int64_t)1 << g.shift) - 1;
  // gather once; the chunk counter's old value is the product's rank inside
  // this tile's run of that chunk
  expand_products<BS, RP, CI, V, NUMERIC>(
      c.p0, c.p1, c.e0, c.a1, acol, aval, brp, bcol, bval, aoff, w_pre, w_b0, w_av,
      [&](int32_t q, CI col, V pv) {
        const uint32_t bin = (uint32_t)(col >> g.shift) - (uint32_t)c.base_bin;
        int hl, len;
        wave_run(bin, hl, len);
        int r = 0;
        if (lane() == hl) r = atomicAdd(&hist[bin], len);
        r = __shfl(r, hl, MG_WAVE);
        if (W16) {
          u_word[q] = (bin << 16) | ((uint32_t)col & (uint32_t)lmask);
        } else {
          u_word[q] = (uint32_t)((uint64_t)col & (uint64_t)lmask);
          u_bin[q] = (uint16_t)bin;
        }
        u_rank[q] = (uint32_t)(r + (lane() - hl));
        if (NUMERIC) u_val[q] = pv;
      });
  __syncthreads();
  if (SORTED) block_excl_scan<BS>(hist, loff, c.nbk, s_tmp);
  // reserve each chunk's run inside its bin with one atomic add
  const int64_t gb = g.binBase[c.k];
  for (int64_t q = threadIdx.x; q < c.nbk; q += BS) {
    const int h = hist[q];
    if (h > 0) {
      const unsigned long long r = atomicAdd(&bin_cursor[gb + q], (unsigned long long)h);
      dst[q] = bin_start[gb + q] + (int64_t)r;
    }
  }
  const int32_t nloc = (int32_t)(c.p1 - c.p0);
  if (SORTED) {
    for (int32_t q = threadIdx.x; q < nloc; q += BS) {
      const uint32_t w = u_word[q];
      const uint32_t bin = W16 ? (w >> 16) : (uint32_t)u_bin[q];
      s_idx[loff[bin] + (int32_t)u_rank[q]] = (uint16_t)q;
    }
  }
  __syncthreads();
  if (SORTED) {
    for (int32_t p = threadIdx.x; p < nloc; p += BS) {
      const int32_t q = s_idx[p];
      const uint32_t w = u_word[q];
      const uint32_t bin = W16 ? (w >> 16) : (uint32_t)u_bin[q];
      const int64_t d = dst[bin] + (p - loff[bin]);
      st_stream<HINT_WS_STORE>(&ws_col[d], W16 ? (LC)(w & 0xFFFFu) : (LC)w);
      if (NUMERIC) st_stream<HINT_WS_STORE>(&ws_val[d], u_val[q]);
    }
  } else {
    for (int32_t q = threadIdx.x; q < nloc; q += BS) {
      const uint32_t w = u_word[q];
      const uint32_t bin = W16 ? (w >> 16) : (uint32_t)u_bin[q];
      const int64_t d = dst[bin] + u_rank[q];
      st_stream<HINT_WS_STORE>(&ws_col[d], W16 ? (LC)(w & 0xFFFFu) : (LC)w);
      if (NUMERIC) st_stream<HINT_WS_STORE>(&ws_val[d], u_val[q]);
    }
  }
}

// ---------------------------------------------------------------------------
// Order-preserving reorder (deterministic mode): the products of every chunk
// land in the workspace in the order of Eq. 1, so that an accumulator adding
// them in workspace order reproduces the plain row-wise sum bit for bit.
// A row's tiles are grouped into segments of S consecutive tiles.  At plan
// time a count pass writes, per segment, its products in each chunk of its
// row into a table laid out [row][chunk][segment]; one exclusive scan of the
// table then gives every segment the products that the row's earlier
// segments put into each chunk.  In the numeric phase one workgroup per
// segment takes the segment's tiles in order: each tile is staged in LDS and
// one wave walks it in product order, giving every product the next slot of
// its chunk (a cursor per chunk, started from the scanned table).
// ---------------------------------------------------------------------------
constexpr int DS_BS = 256;

// per CHUNKED row: its segments and its table entries (segments x chunks)
__global__ void k_det_nseg(ChunkGeom g, int S, int64_t* nseg, int64_t* ntab) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= g.nch) return;
  const int64_t ns = (g.nt[k] + S - 1) / S;
  nseg[k] = ns;
  ntab[k] = ns * g.nb[k];
}

hipError_t launch_det_nseg(const ChunkGeom& g, int S, int64_t* nseg, int64_t* ntab,
                           hipStream_t st) {
  if (g.nch <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_det_nseg, (unsigned)((g.nch + 255) / 256), 256, 0, st, g, S, nseg, ntab);
  return hipGetLastError();
}

// the segment's place: its row k, index s among the row's segments, tiles
// [t0, t1) and products [p0, p1) of the row
struct DetSeg {
  int64_t k, s, ns, t0, t1, p0, p1;
};
MG_INLINE DetSeg det_seg(const ChunkGeom& g, int64_t sg, const int32_t* seg_row,
                         const int64_t* segBase, int S) {
  DetSeg d;
  d.k = seg_row[sg];
  d.s = sg - segBase[d.k];
  d.ns = segBase[d.k + 1] - segBase[d.k];
  d.t0 = d.s * S;
  d.t1 = (d.t0 + S < g.nt[d.k]) ? (d.t0 + S) : g.nt[d.k];
  const int64_t ipr = g.ip[g.rows[d.k]];
  d.p0 = d.t0 * (int64_t)g.tile;
  d.p1 = (d.t1 * (int64_t)g.tile < ipr) ? (d.t1 * (int64_t)g.tile) : ipr;
  return d;
}

size_t det_seg_hist_lds(int64_t max_nb) { return DS_BS * (8 + 8) + (size_t)max_nb * 4 + 64; }

template <typename RP, typename CI>
__global__ void __launch_bounds__(DS_BS)
    k_det_seg_hist(const RP* __restrict__ arp, const CI* __restrict__ acol,
                   const RP* __restrict__ brp, const CI* __restrict__ bcol, ChunkGeom g,
                   const int64_t* __restrict__ aoff, const int64_t* __restrict__ tile_e0,
                   const int32_t* __restrict__ seg_row, const int64_t* __restrict__ segBase,
                   const int64_t* __restrict__ tabBase, int S, int64_t sg0, int64_t* tab) {
  extern __shared__ __align__(16) unsigned char dsm[];
  int32_t* w_pre = (int32_t*)dsm;
  int64_t* w_b0 = (int64_t*)(dsm + DS_BS * 8);
  int32_t* hist = (int32_t*)(w_b0 + DS_BS);
  const DetSeg d = det_seg(g, sg0 + blockIdx.x, seg_row, segBase, S);
  const int32_t row = g.rows[d.k];
  const int64_t nbk = g.nb[d.k];
  const int sh = g.shift;
  const uint32_t base_bin = (uint32_t)(g.minc[row] >> sh);
  for (int64_t q = threadIdx.x; q < nbk; q += DS_BS) hist[q] = 0;
  __syncthreads();
  expand_products<DS_BS, RP, CI, float, false>(
      d.p0, d.p1, tile_e0[g.tileBase[d.k] + d.t0], arp[row + 1], acol, (const float*)nullptr,
      brp, bcol, (const float*)nullptr, aoff, w_pre, w_b0, (float*)nullptr,
      [&](int32_t, CI col, float) { atomicAdd(&hist[(uint32_t)(col >> sh) - base_bin], 1); });
  __syncthreads();
  const int64_t tb = tabBase[d.k];
  for (int64_t c = threadIdx.x; c < nbk; c += DS_BS) tab[tb + c * d.ns + d.s] = hist[c];
}

hipError_t launch_det_seg_hist(const Mats& M, const ChunkGeom& g, const int64_t* aoff,
                               const int64_t* tile_e0, const int32_t* seg_row,
                               const int64_t* segBase, const int64_t* tabBase, int S,
                               int64_t nsegs, int64_t max_nb, int64_t* tab, hipStream_t st) {
  if (nsegs <= 0) return hipSuccess;
  const size_t lds = det_seg_hist_lds(max_nb);
  const int64_t cap = max_grid(DS_BS);
  for (int64_t o = 0; o < nsegs; o += cap) {
    MG_DISPATCH2(M, {
      auto kf = k_det_seg_hist<RP, CI>;
      (void)hipFuncSetAttribute((const void*)kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      hipLaunchKernelGGL(kf, (unsigned)std::min(cap, nsegs - o), DS_BS, lds, st,
                         (const RP*)M.arp, (const CI*)M.acol, (const RP*)M.brp,
                         (const CI*)M.bcol, g, aoff, tile_e0, seg_row, segBase, tabBase, S, o,
                         tab);
    });
  }
  return hipGetLastError();
}

size_t bin_scatter_det_lds(int f64, int tile, int64_t max_nb) {
  const size_t vs = f64 ? 8 : 4;
  return DS_BS * (8 + 8 + 8) + (size_t)max_nb * 8 + 64 + (size_t)tile * (4 + vs + 8) + 64;
}

template <typename RP, typename CI, typename V>
__global__ void __launch_bounds__(DS_BS)
    k_bin_scatter_det(const RP* __restrict__ arp, const CI* __restrict__ acol,
                      const V* __restrict__ aval, const RP* __restrict__ brp,
                      const CI* __restrict__ bcol, const V* __restrict__ bval, ChunkGeom g,
                      const int64_t* __restrict__ aoff, const int64_t* __restrict__ tile_e0,
                      const int32_t* __restrict__ seg_row, const int64_t* __restrict__ segBase,
                      const int64_t* __restrict__ tabBase, const int64_t* __restrict__ tabS,
                      int S, int64_t sg0, const int64_t* __restrict__ bin_start,
                      uint16_t* ws_col, V* ws_val) {
  extern __shared__ __align__(16) unsigned char dsm[];
  int32_t* w_pre = (int32_t*)dsm;
  int64_t* w_b0 = (int64_t*)(dsm + DS_BS * 8);
  V* w_av = (V*)(w_b0 + DS_BS);
  const DetSeg d = det_seg(g, sg0 + blockIdx.x, seg_row, segBase, S);
  const int64_t k = d.k;
  const int32_t row = g.rows[k];
  const int64_t nbk = g.nb[k], gb = g.binBase[k], tb = g.tileBase[k], xb = tabBase[k];
  int64_t* cur = (int64_t*)((char*)w_av + DS_BS * 8);  // nbk: next free slot of each chunk
  uint32_t* u_word = (uint32_t*)(((uintptr_t)(cur + nbk) + 15) & ~(uintptr_t)15);
  V* u_val = (V*)(((uintptr_t)(u_word + g.tile) + 15) & ~(uintptr_t)15);
  int64_t* dst = (int64_t*)(u_val + g.tile);
  const int t = threadIdx.x, l = lane();
  const int64_t ipr = g.ip[row];
  const int64_t a1 = arp[row + 1];
  const uint32_t base_bin = (uint32_t)(g.minc[row] >> g.shift);
  const uint32_t lmask = (1u << g.shift) - 1u;
  // bits of a chunk index of this row
  const int nbits = (nbk > 1) ? 32 - __clz((unsigned)(nbk - 1)) : 0;
  const uint64_t below = (1ull << l) - 1ull;
  // the products the row's earlier segments put into each chunk
  for (int64_t q = t; q < nbk; q += DS_BS)
    cur[q] = bin_start[gb + q] + (tabS[xb + q * d.ns + d.s] - tabS[xb + q * d.ns]);
  for (int64_t ti = d.t0; ti < d.t1; ++ti) {
    const int64_t p0 = ti * (int64_t)g.tile;
    const int64_t p1 = (p0 + g.tile < ipr) ? (p0 + g.tile) : ipr;
    __syncthreads();  // the previous tile's copy-out has read u_word, u_val and dst
    expand_products<DS_BS, RP, CI, V, true>(
        p0, p1, tile_e0[tb + ti], a1, acol, aval, brp, bcol, bval, aoff, w_pre, w_b0, w_av,
        [&](int32_t q, CI col, V pv) {
          const uint32_t bin = (uint32_t)(col >> g.shift) - base_bin;
          u_word[q] = (bin << 16) | ((uint32_t)col & lmask);
          u_val[q] = pv;
        });
    __syncthreads();
    const int32_t nloc = (int32_t)(p1 - p0);
    if (t < MG_WAVE) {
      // one wave walks the tile in product order, 64 products at a time: a
      // product's slot is its chunk's cursor plus the number of earlier
      // products of the window in the same chunk (lanes matched bit by bit
      // of the chunk index); the lowest lane of each chunk advances the cursor
      for (int32_t w0 = 0; w0 < nloc; w0 += MG_WAVE) {
        const int32_t q = w0 + l;
        const bool ok = q < nloc;
        const uint32_t bin = ok ? (u_word[q] >> 16) : 0u;
        uint64_t m = __ballot(ok);
        for (int b = 0; b < nbits; ++b) {
          const bool bit = (bin >> b) & 1u;
          const uint64_t bb = __ballot(bit);
          m &= bit ? bb : ~bb;
        }
        const int rank = __popcll(m & below);
        int64_t base = 0;
        if (ok) {
          base = cur[bin];
          dst[q] = base + rank;
        }
        if (ok && rank == 0) cur[bin] = base + __popcll(m);
      }
    }
    __syncthreads();
    for (int32_t q = t; q < nloc; q += DS_BS) {
      const int64_t dd = dst[q];
      st_stream<HINT_WS_STORE>(&ws_col[dd], (uint16_t)(u_word[q] & 0xFFFFu));
      st_stream<HINT_WS_STORE>(&ws_val[dd], u_val[q]);
    }
  }
}

// ---------------------------------------------------------------------------
// Coarse level (Section 3.3).  Every chunk of 2^cshift columns that the first
// reorder produced becomes a "virtual row" of a second chunk geometry: its
// products sit contiguously in the first workspace with 32-bit columns local
// to the chunk, and the chunks of 2^shift columns inside it are handled like
// the chunks of an ordinary CHUNKED row.
// ---------------------------------------------------------------------------
// per coarse row k (one wave): the column base, last column and fine chunk
// count of each of its coarse chunks
__global__ void k_vrow_geom(ChunkGeom g1, int fshift, int64_t* minc2, int64_t* maxc2, int64_t* nb2,
                            int64_t k0) {
  const int64_t k = k0 + (int64_t)blockIdx.x * 4 + threadIdx.x / MG_WAVE;
  if (k >= g1.nch) return;
  const int32_t row = g1.rows[k];
  const int cs = g1.shift;
  const int64_t c0 = g1.minc[row] >> cs, mx = g1.maxc[row];
  const int64_t bb = g1.binBase[k], nbk = g1.nb[k];
  for (int64_t q = lane(); q < nbk; q += MG_WAVE) {
    const int64_t base = (c0 + q) << cs;
    const int64_t last = base + ((int64_t)1 << cs) - 1;
    const int64_t hi = last < mx ? last : mx;
    minc2[bb + q] = base;
    maxc2[bb + q] = hi;
    nb2[bb + q] = (hi >> fshift) - (base >> fshift) + 1;
  }
}

// tiles of the level-2 reorder: nt = ceil(products / tile) per listed virtual row
__global__ void k_vrow_tiles(ChunkGeom g2, int64_t k0, int64_t k1) {
  const int64_t k = k0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= k1) return;
  g2.nt[k] = (g2.ip[g2.rows[k]] + g2.tile - 1) / g2.tile;
}

// Coarse chunks of a batch split by size: those with more than SORT_CAP
// products go through the fine level (`big`), the others are sorted
// directly (`small`); pos = exclusive scan of the big flags.
__global__ void k_vrow_flags(const int64_t* cnt1, int64_t k0, int64_t n, int64_t* flags) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) flags[i] = cnt1[k0 + i] > SORT_CAP ? 1 : 0;
}
__global__ void k_vrow_split(const int64_t* cnt1, int64_t k0, int64_t n, const int64_t* pos,
                             int32_t* big, int32_t* small) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t v = k0 + i;
  if (cnt1[v] > SORT_CAP) big[pos[i]] = (int32_t)v;
  else small[i - pos[i]] = (int32_t)v;
}
// per listed virtual row: fine chunks, products
__global__ void k_vrow_gather(const int32_t* rows, int64_t n, const int64_t* vnb,
                              const int64_t* cnt1, int64_t* nb, int64_t* cnt) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  nb[k] = vnb[rows[k]];
  cnt[k] = cnt1[rows[k]];
}

// Symbolic phase of a coarse chunk: its column bitmap (2^cshift bits) in
// LDS, one workgroup per virtual row; per fine chunk the distinct columns
// and the products, and the virtual row's nnz.
constexpr int VB_BS = 1024;

size_t vrow_bitmap_lds(int cshift, int64_t max_nb2) {
  return (((size_t)1 << cshift) >> 3) + (size_t)max_nb2 * 4 + 64;
}

__global__ void __launch_bounds__(VB_BS)
    k_vrow_bitmap(ChunkGeom g2, int64_t k0, const int64_t* __restrict__ start1,
                  const uint32_t* __restrict__ ws1_col, int64_t* bin_cnt2, int64_t* bin_nnz2,
                  int32_t* bin_row2, int64_t* vnnz) {
  extern __shared__ __align__(16) unsigned char dsm[];
  const int64_t k = k0 + blockIdx.x;
  const int64_t nbk = g2.nb[k], bb = g2.binBase[k];
  const int sh = g2.shift;
  const int64_t v = g2.rows[k];
  const int64_t cnt = g2.ip[v], s0 = start1[v];
  const int t = threadIdx.x;
  if (cnt == 0) {
    for (int64_t q = t; q < nbk; q += VB_BS) {
      bin_cnt2[bb + q] = 0;
      bin_nnz2[bb + q] = 0;
      bin_row2[bb + q] = (int32_t)k;
    }
    if (t == 0) vnnz[v] = 0;
    return;
  }
  const int64_t nwords = (nbk << sh) >> 5;
  uint32_t* bits = (uint32_t*)dsm;
  int32_t* cntf = (int32_t*)(bits + nwords);
  __shared__ unsigned long long tot;
  lds_clear_words(bits, nwords, t, VB_BS);
  for (int64_t q = t; q < nbk; q += VB_BS) cntf[q] = 0;
  if (t == 0) tot = 0;
  __syncthreads();
  for (int64_t q = t; q < cnt; q += VB_BS) {
    const uint32_t lc = ld_stream<HINT_WS_LOAD>(&ws1_col[s0 + q]);
    atomicOr(&bits[lc >> 5], 1u << (lc & 31));
    const uint32_t f = lc >> sh;
    int hl, len;
    wave_run(f, hl, len);
    if (lane() == hl) atomicAdd(&cntf[f], len);
  }
  __syncthreads();
  const int w = t / MG_WAVE, nw = VB_BS / MG_WAVE;
  const int64_t wpb = ((int64_t)1 << sh) >> 5;
  for (int64_t f = w; f < nbk; f += nw) {
    unsigned long long s = lds_popc_words(bits + f * wpb, wpb);
    s = wave_sum(s);
    if (lane() == 0) {
      bin_nnz2[bb + f] = (int64_t)s;
      bin_cnt2[bb + f] = cntf[f];
      bin_row2[bb + f] = (int32_t)k;
      atomicAdd(&tot, s);
    }
  }
  __syncthreads();
  if (t == 0) vnnz[v] = (int64_t)tot;
}

// Level-2 reorder: a tile of a virtual row's products (first workspace) is
// staged in LDS with its fine chunk and its rank inside that chunk, the
// tile is permuted into chunk order in LDS (offsets from a scan of the
// tile's chunk counts), each chunk's run is reserved in its bin with one
// atomic add, and the permuted tile is written out, so that consecutive
// lanes store consecutive addresses of one chunk's run (the staging order
// interleaves the chunks: inside a coarse chunk, neighbouring products
// seldom share a fine chunk).  16-bit chunk-local columns.
// The level-2 reorder writes each tile out in fine-chunk order through a
// 16-bit index per position (as the first reorder), 1024 threads per tile
// (MG_L2_BS) unless the caller asks for 256.
#ifndef MG_L2_BS
#define MG_L2_BS 1024
#endif
size_t l2_scatter_lds(int f64, int tile, int64_t max_nb2) {
  const size_t vs = f64 ? 8 : 4;
  return (size_t)max_nb2 * (4 + 4 + 8) + 3 * 16 + (size_t)tile * (4 + 4 + vs) +
         (size_t)tile * 2 + 16 + 64;
}

template <int BS, typename V, bool NUMERIC>
__global__ void __launch_bounds__(BS)
    k_l2_scatter(ChunkGeom g2, BatchArgs b2, const int32_t* __restrict__ tile_row2,
                 const int64_t* __restrict__ start1, const uint32_t* __restrict__ ws1_col,
                 const V* __restrict__ ws1_val, const int64_t* __restrict__ bin_start2,
                 unsigned long long* bin_cursor2, uint16_t* ws2_col, V* ws2_val) {
  extern __shared__ __align__(16) unsigned char dsm[];
  __shared__ int32_t s_tmp[BS / MG_WAVE];
  const int64_t tg = b2.tile0 + blockIdx.x;
  const int64_t k = tile_row2[tg];
  const int64_t ti = tg - g2.tileBase[k];
  const int64_t v = g2.rows[k];
  const int64_t cnt = g2.ip[v];
  const int64_t p0 = ti * (int64_t)g2.tile;
  const int32_t nloc = (int32_t)((cnt - p0 < g2.tile) ? (cnt - p0) : g2.tile);
  const int64_t s0 = start1[v] + p0;
  const int64_t nbk = g2.nb[k], gb = g2.binBase[k];
  const int sh = g2.shift;
  const uint32_t lmask = (1u << sh) - 1u;
  auto al16 = [](void* p) { return (void*)(((uintptr_t)p + 15) & ~(uintptr_t)15); };
  int32_t* hist = (int32_t*)dsm;
  int32_t* loff = (int32_t*)al16(hist + nbk);
  int64_t* dst = (int64_t*)al16(loff + nbk);
  uint32_t* u_word = (uint32_t*)(dst + nbk);
  uint32_t* u_rank = u_word + g2.tile;
  V* u_val = (V*)al16(u_rank + g2.tile);
  uint16_t* s_idx = (uint16_t*)al16(u_val + g2.tile);  // staged product at each position
  for (int64_t q = threadIdx.x; q < nbk; q += BS) hist[q] = 0;
  __syncthreads();
  for (int32_t qb = threadIdx.x; qb < nloc; qb += 4 * BS) {
    uint32_t c4[4];
    V v4[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int32_t q = qb + u * BS;
      c4[u] = (q < nloc) ? ld_stream<HINT_WS_LOAD>(&ws1_col[s0 + q]) : 0u;
      v4[u] = (NUMERIC && q < nloc) ? ld_stream<HINT_WS_LOAD>(&ws1_val[s0 + q]) : (V)0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int32_t q = qb + u * BS;
      if (q < nloc) {
        const uint32_t f = c4[u] >> sh;
        int hl, len;
        wave_run(f, hl, len);
        int r = 0;
        if (lane() == hl) r = atomicAdd(&hist[f], len);
        r = __shfl(r, hl, MG_WAVE);
        u_word[q] = (f << 16) | (c4[u] & lmask);
        u_rank[q] = (uint32_t)(r + (lane() - hl));
        if (NUMERIC) u_val[q] = v4[u];
      }
    }
  }
  __syncthreads();
  block_excl_scan<BS>(hist, loff, nbk, s_tmp);
  for (int64_t q = threadIdx.x; q < nbk; q += BS) {
    const int h = hist[q];
    if (h > 0) {
      const unsigned long long r = atomicAdd(&bin_cursor2[gb + q], (unsigned long long)h);
      dst[q] = bin_start2[gb + q] + (int64_t)r;
    }
  }
  for (int32_t q = threadIdx.x; q < nloc; q += BS) {
    const uint32_t w = u_word[q];
    s_idx[loff[w >> 16] + (int32_t)u_rank[q]] = (uint16_t)q;
  }
  __syncthreads();
  for (int32_t p = threadIdx.x; p < nloc; p += BS) {
    const int32_t q = s_idx[p];
    const uint32_t w = u_word[q];
    const uint32_t f = w >> 16;
    const int64_t d = dst[f] + (p - loff[f]);
    st_stream<HINT_WS_STORE>(&ws2_col[d], (uint16_t)(w & 0xFFFFu));
    if (NUMERIC) st_stream<HINT_WS_STORE>(&ws2_val[d], u_val[q]);
  }
}

// Fine-chunk product counts of the level-2 tiles of b2 (cnt2 zeroed before):
// per tile a histogram in LDS, added into the chunk totals.
template <int BS>
__global__ void __launch_bounds__(BS)
    k_l2_hist(ChunkGeom g2, BatchArgs b2, const int32_t* __restrict__ tile_row2,
              const int64_t* __restrict__ start1, const uint32_t* __restrict__ ws1_col,
              unsigned long long* cnt2) {
  extern __shared__ __align__(16) unsigned char dsm[];
  int32_t* hist = (int32_t*)dsm;
  const int64_t tg = b2.tile0 + blockIdx.x;
  const int64_t k = tile_row2[tg];
  const int64_t p0 = (tg - g2.tileBase[k]) * (int64_t)g2.tile;
  const int64_t v = g2.rows[k];
  const int64_t cnt = g2.ip[v];
  const int32_t nloc = (int32_t)((cnt - p0 < g2.tile) ? (cnt - p0) : g2.tile);
  const int64_t s0 = start1[v] + p0;
  const int64_t nbk = g2.nb[k], gb = g2.binBase[k];
  const int sh = g2.shift;
  for (int64_t q = threadIdx.x; q < nbk; q += BS) hist[q] = 0;
  __syncthreads();
  for (int32_t qb = threadIdx.x; qb < nloc; qb += 4 * BS) {
    uint32_t c4[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int32_t q = qb + u * BS;
      c4[u] = (q < nloc) ? ld_stream<HINT_WS_LOAD>(&ws1_col[s0 + q]) : 0u;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (qb + u * BS < nloc) {
        const uint32_t f = c4[u] >> sh;
        int hl, len;
        wave_run(f, hl, len);
        if (lane() == hl) atomicAdd(&hist[f], len);
      }
    }
  }
  __syncthreads();
  for (int64_t q = threadIdx.x; q < nbk; q += BS) {
    const int h = hist[q];
    if (h > 0) atomicAdd(&cnt2[gb + q], (unsigned long long)h);
  }
}

// the virtual row of every fine chunk (one wave per virtual row)
__global__ void k_vrow_rows(ChunkGeom g2, int32_t* row2, int64_t k0) {
  const int64_t k = k0 + (int64_t)blockIdx.x * 4 + threadIdx.x / MG_WAVE;
  if (k >= g2.nch) return;
  const int64_t bb = g2.binBase[k], nbk = g2.nb[k];
  for (int64_t q = lane(); q < nbk; q += MG_WAVE) row2[bb + q] = (int32_t)k;
}

// ---------------------------------------------------------------------------
// Chunk start / size and work items
// ---------------------------------------------------------------------------
// per row: dense chunks become single items; runs of small consecutive chunks
// (<= 64 chunks, <= group_max products) become packed sort items.  Each
// thread walks its row's chunks twice: once to count its items, then (after
// one reservation per wave on each item counter) to write them; per-item
// atomics on the two counters would serialise across the whole grid.
template <typename Emit>
MG_INLINE void group_row(const int64_t* bin_cnt, int64_t bb, int64_t nbk, int64_t dense_min,
                         int64_t group_max, Emit&& emit) {
  int64_t gs = -1, gn = 0, gc = 0;
  for (int64_t q = 0; q < nbk; ++q) {
    const int64_t cnt = bin_cnt[bb + q];
    if (cnt >= dense_min) {
      if (gs >= 0) {
        emit(1, gs, gn);
        gs = -1; gn = 0; gc = 0;
      }
      emit(0, bb + q, 1);
      continue;
    }
    if (gs >= 0 && (gc + cnt > group_max || gn >= 64)) {
      emit(1, gs, gn);
      gs = -1; gn = 0; gc = 0;
    }
    if (gs < 0) gs = bb + q;
    ++gn;
    gc += cnt;
  }
  if (gs >= 0) emit(1, gs, gn);
}

__global__ void k_bin_group(ChunkGeom g, BatchArgs b, const int64_t* bin_cnt, int64_t dense_min,
                            int64_t group_max, int64_t* dense_items, int64_t* sort_items,
                            int32_t* item_counts, int64_t item_base) {
  const int64_t k = b.k0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = k < b.k1;
  const int64_t nbk = live ? g.nb[k] : 0, bb = live ? g.binBase[k] : 0;
  int n[2] = {0, 0};
  if (live)
    group_row(bin_cnt, bb, nbk, dense_min, group_max,
              [&](int kind, int64_t, int64_t) { ++n[kind]; });
  int base[2];
  for (int kind = 0; kind < 2; ++kind) {
    const int inc = wave_incl_scan(n[kind]);
    const int tot = __shfl(inc, MG_WAVE - 1, MG_WAVE);
    int wb = 0;
    if (lane() == 0 && tot > 0) wb = atomicAdd(&item_counts[kind], tot);
    base[kind] = __shfl(wb, 0, MG_WAVE) + inc - n[kind];
  }
  if (!live) return;
  group_row(bin_cnt, bb, nbk, dense_min, group_max, [&](int kind, int64_t first, int64_t cnt) {
    const int64_t idx = item_base + base[kind]++;
    if (kind == 0) {
      dense_items[idx] = first;
    } else {
      sort_items[2 * idx] = first;
      sort_items[2 * idx + 1] = cnt;
    }
  });
}

// ---------------------------------------------------------------------------
// Dense chunk accumulation: one workgroup per chunk; LDS values (numeric) and
// one bitmap bit per column; write-out in column order.
// ---------------------------------------------------------------------------
size_t bin_dense_lds(int f64, int shift) {
  const size_t L = (size_t)1 << shift;
  return L * (f64 ? 8 : 4) + (L / 32) * 4 + 64;
}

template <typename V, bool NUMERIC>
__global__ void __launch_bounds__(1024)
    k_accum_dense(ChunkGeom g, const int64_t* __restrict__ items, const int32_t* item_counts,
                  int64_t item_base, const int64_t* __restrict__ bin_start,
                  const int64_t* __restrict__ bin_cnt, const int32_t* __restrict__ bin_row,
                  const uint16_t* __restrict__ ws_col, const V* __restrict__ ws_val,
                  int64_t* bin_nnz, const int64_t* __restrict__ bin_out, void* ccol_, int col64,
                  V* cval, unsigned int* work) {
  // persistent: each workgroup takes chunks from a counter; the accumulator
  // and bitmap are cleared once, and afterwards only the touched entries are
  // reset during the write-out, so a chunk costs O(products + chunk/32)
  extern __shared__ __align__(16) unsigned char dsm[];
  const int BS = blockDim.x;
  const int64_t L = (int64_t)1 << g.shift;
  V* acc = (V*)dsm;
  uint32_t* bits = (uint32_t*)(dsm + (NUMERIC ? L * sizeof(V) : 0));
  __shared__ int64_t sh_w[16];
  __shared__ unsigned int sh_item;
  const int t = threadIdx.x;
  const int64_t nitems = item_counts[0];
  const int64_t nwords = L / 32;
  for (int64_t q = t; q < nwords; q += BS) bits[q] = 0u;
  if (NUMERIC)
    for (int64_t q = t; q < L; q += BS) acc[q] = (V)0;
  const int64_t wpt = (nwords + BS - 1) / BS;
  const int64_t w0 = t * wpt, w1 = (w0 + wpt < nwords) ? (w0 + wpt) : nwords;
  const int wv = t / MG_WAVE, nw = BS / MG_WAVE;
  // the next item's index is fetched while the current one is processed
  unsigned int nxt = 0;
  if (t == 0) nxt = atomicAdd(work, 1u);
  for (;;) {
    __syncthreads();
    if (t == 0) sh_item = nxt;
    __syncthreads();
    const int64_t it = sh_item;
    if (it >= nitems) break;
    if (t == 0) nxt = atomicAdd(work, 1u);
    const int64_t gb = items[item_base + it];
    const int64_t s0 = bin_start[gb], cnt = bin_cnt[gb];
    int64_t q = t;
    for (; q + 3 * BS < cnt; q += 4 * BS) {
      uint32_t c4[4];
      V v4[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        c4[u] = ld_stream<HINT_WS_LOAD>(&ws_col[s0 + q + u * BS]);
        if (NUMERIC) v4[u] = ld_stream<HINT_WS_LOAD>(&ws_val[s0 + q + u * BS]);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        atomicOr(&bits[c4[u] >> 5], 1u << (c4[u] & 31));
        if (NUMERIC) atomicAdd(&acc[c4[u]], v4[u]);
      }
    }
    for (; q < cnt; q += BS) {
      const uint32_t c = ld_stream<HINT_WS_LOAD>(&ws_col[s0 + q]);
      atomicOr(&bits[c >> 5], 1u << (c & 31));
      if (NUMERIC) atomicAdd(&acc[c], ld_stream<HINT_WS_LOAD>(&ws_val[s0 + q]));
    }
    __syncthreads();
    int64_t my = 0;
    for (int64_t w = w0; w < w1; ++w) my += __popc(bits[w]);
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
      for (int64_t w = w0; w < w1; ++w) bits[w] = 0u;
      continue;
    }
    const int64_t k = bin_row[gb];
    const int64_t colbase = ((g.minc[g.rows[k]] >> g.shift) + (gb - g.binBase[k])) << g.shift;
    int64_t pos = bin_out[gb] + before + inc - my;
    for (int64_t w = w0; w < w1; ++w) {
      uint32_t bb = bits[w];
      if (!bb) continue;
      bits[w] = 0u;
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
// Dense chunk accumulation in workspace order (deterministic mode): one wave
// per chunk adds the chunk's products into the LDS accumulator one by one in
// the order they are stored, which the order-preserving reorder made the
// order of Eq. 1.  A window of 64 products is sorted by (column, position);
// the k-th products of all runs of equal columns are added together (distinct
// columns), k = 0, 1, ..., so each column's additions keep their order.
// ---------------------------------------------------------------------------
template <typename V>
__global__ void __launch_bounds__(MG_WAVE)
    k_accum_dense_det(ChunkGeom g, const int64_t* __restrict__ items, const int32_t* item_counts,
                      int64_t item_base, const int64_t* __restrict__ bin_start,
                      const int64_t* __restrict__ bin_cnt, const int32_t* __restrict__ bin_row,
                      const uint16_t* __restrict__ ws_col, const V* __restrict__ ws_val,
                      const int64_t* __restrict__ bin_out, void* ccol_, int col64, V* cval,
                      unsigned int* work) {
  extern __shared__ __align__(16) unsigned char dsm[];
  const int64_t L = (int64_t)1 << g.shift;
  V* acc = (V*)dsm;
  uint32_t* bits = (uint32_t*)(dsm + L * sizeof(V));
  const int l = lane();
  const int64_t nitems = item_counts[0];
  const int64_t nwords = L / 32;
  for (int64_t q = l; q < nwords; q += MG_WAVE) bits[q] = 0u;
  for (int64_t q = l; q < L; q += MG_WAVE) acc[q] = (V)0;
  const int64_t wpl = (nwords + MG_WAVE - 1) / MG_WAVE;
  const int64_t w0 = l * wpl, w1 = (w0 + wpl < nwords) ? (w0 + wpl) : nwords;
  const uint64_t upto = (l == MG_WAVE - 1) ? ~0ull : ((2ull << l) - 1ull);
  for (;;) {
    unsigned int it = 0;
    if (l == 0) it = atomicAdd(work, 1u);
    it = __shfl(it, 0, MG_WAVE);
    if ((int64_t)it >= nitems) break;
    const int64_t gb = items[item_base + it];
    const int64_t s0 = bin_start[gb], cnt = bin_cnt[gb];
    // DD windows of 64 products are loaded while the previous DD are added
    constexpr int DD = 4;
    uint32_t c4[DD];
    V v4[DD];
#pragma unroll
    for (int u = 0; u < DD; ++u) {
      const int64_t x = (int64_t)u * MG_WAVE + l;
      c4[u] = x < cnt ? (uint32_t)ws_col[s0 + x] : 0xFFFFFFFFu;
      v4[u] = x < cnt ? ws_val[s0 + x] : (V)0;
    }
    for (int64_t xb = 0; xb < cnt; xb += DD * MG_WAVE) {
      uint32_t n4[DD];
      V w4[DD];
#pragma unroll
      for (int u = 0; u < DD; ++u) {
        const int64_t x = xb + (int64_t)(DD + u) * MG_WAVE + l;
        n4[u] = x < cnt ? (uint32_t)ws_col[s0 + x] : 0xFFFFFFFFu;
        w4[u] = x < cnt ? ws_val[s0 + x] : (V)0;
      }
#pragma unroll
      for (int u = 0; u < DD; ++u) {
        if (xb + (int64_t)u * MG_WAVE >= cnt) break;
        const bool ok = c4[u] != 0xFFFFFFFFu;
        uint32_t kk[1] = {ok ? ((c4[u] << 6) | (uint32_t)l) : 0xFFFFFFFFu};
        bitonic_sort_keys<1>(kk);
        const bool mine = kk[0] != 0xFFFFFFFFu;
        const uint32_t cc = kk[0] >> 6;
        const V vv = __shfl(v4[u], (int)(kk[0] & 63u), MG_WAVE);
        const uint32_t pc = __shfl_up(cc, 1, MG_WAVE);
        const uint64_t hm = __ballot(l == 0 || pc != cc);
        const int r = l - (63 - __clzll(hm & upto));  // position inside the run
        const int R = wave_max(mine ? r + 1 : 0);
        for (int rr = 0; rr < R; ++rr) {
          if (mine && r == rr) {
            acc[cc] = acc[cc] + vv;
            atomicOr(&bits[cc >> 5], 1u << (cc & 31));
          }
        }
      }
#pragma unroll
      for (int u = 0; u < DD; ++u) {
        c4[u] = n4[u];
        v4[u] = w4[u];
      }
    }
    // write-out in column order: a lane owns words w0..w1
    int64_t my = 0;
    for (int64_t w = w0; w < w1; ++w) my += __popc(bits[w]);
    const int64_t inc = wave_incl_scan(my);
    const int64_t k = bin_row[gb];
    const int64_t colbase = ((g.minc[g.rows[k]] >> g.shift) + (gb - g.binBase[k])) << g.shift;
    int64_t pos = bin_out[gb] + inc - my;
    for (int64_t w = w0; w < w1; ++w) {
      uint32_t bb = bits[w];
      if (!bb) continue;
      bits[w] = 0u;
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
// Packed sort of small chunks: one wave per item of <= 64 consecutive chunks
// of one row and <= 64*E products; key = (chunk offset << shift) | local col,
// i.e. the column relative to the item's first chunk.
// ---------------------------------------------------------------------------
constexpr int AS_WAVES = 4;

template <typename V, int E, bool NUMERIC, bool DET>
MG_INLINE void accum_sort_item(const ChunkGeom& g, int64_t g0, int nbg, const int64_t* bin_start,
                               const int64_t* bin_cnt, const int32_t* bin_row,
                               const uint16_t* ws_col, const V* ws_val, int64_t* bin_nnz,
                               const int64_t* bin_out, void* ccol_, int col64, V* cval,
                               int64_t* s_bs, int32_t* s_cnt, V* s_v, uint32_t* s_k) {
  // numeric keys carry the element index in their low bits, so the network
  // moves one 32-bit word per element and the sum of a run follows the
  // elements' order in the workspace; values are fetched from LDS afterwards
  constexpr int CAP = MG_WAVE * E;
  constexpr int IDXB = NUMERIC ? ilog2c(CAP) : 0;
  const int l = lane();
  const int64_t start = bin_start[g0];
  const int64_t endp = bin_start[g0 + nbg - 1] + bin_cnt[g0 + nbg - 1];
  const int P = (int)(endp - start);
  if (l < nbg) {
    s_bs[l] = bin_start[g0 + l] - start;
    s_cnt[l] = 0;
  }
  wave_sync2();
  uint32_t k[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int x = e * MG_WAVE + l;
    if (x < P) {
      const int bo = upper_index(s_bs, 0, nbg, (int64_t)x);
      const uint32_t key = ((uint32_t)bo << g.shift) | (uint32_t)ld_stream<HINT_WS_LOAD>(&ws_col[start + x]);
      k[e] = NUMERIC ? ((key << IDXB) | (uint32_t)x) : key;
      if (NUMERIC) s_v[x] = ld_stream<HINT_WS_LOAD>(&ws_val[start + x]);
    } else {
      k[e] = 0xFFFFFFFFu;
    }
  }
  bitonic_sort_keys<E>(k);
  wave_sync2();
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
    wave_sync2();
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
    V carry = (V)0;
    if constexpr (DET) {
      // the lane holding a run's head sums the run from +0.0 in element
      // order, walking the sorted keys in LDS, and writes it
#pragma unroll
      for (int e = 0; e < E; ++e) s_k[l * E + e] = k[e];
      wave_sync2();
      const int64_t kk = bin_row[g0];
      const int64_t colbase = ((g.minc[g.rows[kk]] >> g.shift) + (g0 - g.binBase[kk])) << g.shift;
      const int64_t obase = bin_out[g0];
      int hr = hbase;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        if (!head[e]) continue;
        const uint32_t key = k[e] >> IDXB;
        V run = (V)0;
        int y = l * E + e;
        do {
          run = run + s_v[s_k[y] & (CAP - 1)];
          ++y;
        } while (y < P && (s_k[y] >> IDXB) == key);
        const int64_t pos = obase + hr;
        ++hr;
        const int64_t col = colbase + (int64_t)key;
        if (col64) st_stream<HINT_C_STORE>(&((int64_t*)ccol_)[pos], (int64_t)col);
        else st_stream<HINT_C_STORE>(&((int32_t*)ccol_)[pos], (int32_t)col);
        st_stream<HINT_C_STORE>(&cval[pos], run);
      }
      return;
    } else {
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
      carry = __shfl_up(s, 1, MG_WAVE);
      if (l == 0) carry = (V)0;
    }
    const uint32_t nextk = __shfl_down(k[0], 1, MG_WAVE) >> IDXB;
    const int64_t kk = bin_row[g0];
    const int64_t colbase = ((g.minc[g.rows[kk]] >> g.shift) + (g0 - g.binBase[kk])) << g.shift;
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

template <typename V, bool NUMERIC, bool DET>
__global__ void __launch_bounds__(AS_WAVES * MG_WAVE)
    k_accum_sort(ChunkGeom g, const int64_t* __restrict__ items, const int32_t* item_counts,
                 int64_t item_base, const int64_t* __restrict__ bin_start,
                 const int64_t* __restrict__ bin_cnt, const int32_t* __restrict__ bin_row,
                 const uint16_t* __restrict__ ws_col, const V* __restrict__ ws_val,
                 int64_t* bin_nnz, const int64_t* __restrict__ bin_out, void* ccol_, int col64,
                 V* cval, int64_t it0) {
  __shared__ int64_t s_bs[AS_WAVES][MG_WAVE];
  __shared__ int32_t s_cnt[AS_WAVES][MG_WAVE];
  __shared__ V s_v[AS_WAVES][NUMERIC ? SORT_CAP : 1];
  __shared__ uint32_t s_k[AS_WAVES][DET ? SORT_CAP : 1];
  const int w = threadIdx.x / MG_WAVE;
  const int64_t it = it0 + (int64_t)blockIdx.x * AS_WAVES + w;
  if (it >= item_counts[1]) return;
  const int64_t g0 = items[2 * (item_base + it)];
  const int nbg = (int)items[2 * (item_base + it) + 1];
  const int64_t P = bin_start[g0 + nbg - 1] + bin_cnt[g0 + nbg - 1] - bin_start[g0];
  if (P <= 64)
    accum_sort_item<V, 1, NUMERIC, DET>(g, g0, nbg, bin_start, bin_cnt, bin_row, ws_col, ws_val, bin_nnz,
                                   bin_out, ccol_, col64, cval, s_bs[w], s_cnt[w], s_v[w], s_k[w]);
  else if (P <= 128)
    accum_sort_item<V, 2, NUMERIC, DET>(g, g0, nbg, bin_start, bin_cnt, bin_row, ws_col, ws_val, bin_nnz,
                                   bin_out, ccol_, col64, cval, s_bs[w], s_cnt[w], s_v[w], s_k[w]);
  else if (P <= 256)
    accum_sort_item<V, 4, NUMERIC, DET>(g, g0, nbg, bin_start, bin_cnt, bin_row, ws_col, ws_val, bin_nnz,
                                   bin_out, ccol_, col64, cval, s_bs[w], s_cnt[w], s_v[w], s_k[w]);
  else if (P <= 512)
    accum_sort_item<V, 8, NUMERIC, DET>(g, g0, nbg, bin_start, bin_cnt, bin_row, ws_col, ws_val, bin_nnz,
                                   bin_out, ccol_, col64, cval, s_bs[w], s_cnt[w], s_v[w], s_k[w]);
  else
    accum_sort_item<V, 16, NUMERIC, DET>(g, g0, nbg, bin_start, bin_cnt, bin_row, ws_col, ws_val,
                                    bin_nnz, bin_out, ccol_, col64, cval, s_bs[w], s_cnt[w], s_v[w], s_k[w]);
}

// ---------------------------------------------------------------------------
// Coarse chunks of at most SORT_CAP products, sorted straight from the first
// workspace (no fine level): one wave per coarse chunk; key = the column
// local to the coarse chunk (< 2^cshift <= 2^22), numeric keys carry the
// element index below it; count mode writes the distinct columns, numeric
// mode the sums of each run at the chunk's offset in C.
// ---------------------------------------------------------------------------
template <typename V, int E, bool NUMERIC>
MG_INLINE void vrow_sort_item(int64_t s0, int P, int64_t colbase,
                              const uint32_t* __restrict__ ws1_col, const V* __restrict__ ws1_val,
                              int64_t* nnz_out, int64_t obase, void* ccol_, int col64, V* cval,
                              V* s_v) {
  constexpr int CAP = MG_WAVE * E;
  constexpr int IDXB = NUMERIC ? ilog2c(CAP) : 0;
  const int l = lane();
  uint32_t k[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int x = e * MG_WAVE + l;
    if (x < P) {
      const uint32_t key = ld_stream<HINT_WS_LOAD>(&ws1_col[s0 + x]);
      k[e] = NUMERIC ? ((key << IDXB) | (uint32_t)x) : key;
      if (NUMERIC) s_v[x] = ld_stream<HINT_WS_LOAD>(&ws1_val[s0 + x]);
    } else {
      k[e] = 0xFFFFFFFFu;
    }
  }
  bitonic_sort_keys<E>(k);
  wave_sync2();
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
    const int tot = wave_sum(hc);
    if (l == 0) *nnz_out = tot;
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

template <typename V, bool NUMERIC>
__global__ void __launch_bounds__(AS_WAVES * MG_WAVE)
    k_vrow_sort(const int32_t* __restrict__ small, int64_t nsmall, const int64_t* __restrict__ cnt1,
                const int64_t* __restrict__ start1, const int64_t* __restrict__ minc2,
                const uint32_t* __restrict__ ws1_col, const V* __restrict__ ws1_val,
                int64_t* nnz1, const int64_t* __restrict__ out1, void* ccol_, int col64, V* cval,
                int64_t i0) {
  __shared__ V s_v[AS_WAVES][NUMERIC ? SORT_CAP : 1];
  const int w = threadIdx.x / MG_WAVE;
  const int64_t i = i0 + (int64_t)blockIdx.x * AS_WAVES + w;
  if (i >= nsmall) return;
  const int64_t v = small[i];
  const int P = (int)cnt1[v];
  if (P == 0) {
    if (!NUMERIC && lane() == 0) nnz1[v] = 0;
    return;
  }
  const int64_t s0 = start1[v], cb = minc2[v], ob = NUMERIC ? out1[v] : 0;
  int64_t* no = nnz1 + v;
  if (P <= 64)
    vrow_sort_item<V, 1, NUMERIC>(s0, P, cb, ws1_col, ws1_val, no, ob, ccol_, col64, cval, s_v[w]);
  else if (P <= 128)
    vrow_sort_item<V, 2, NUMERIC>(s0, P, cb, ws1_col, ws1_val, no, ob, ccol_, col64, cval, s_v[w]);
  else if (P <= 256)
    vrow_sort_item<V, 4, NUMERIC>(s0, P, cb, ws1_col, ws1_val, no, ob, ccol_, col64, cval, s_v[w]);
  else if (P <= 512)
    vrow_sort_item<V, 8, NUMERIC>(s0, P, cb, ws1_col, ws1_val, no, ob, ccol_, col64, cval, s_v[w]);
  else
    vrow_sort_item<V, 16, NUMERIC>(s0, P, cb, ws1_col, ws1_val, no, ob, ccol_, col64, cval,
                                   s_v[w]);
}

// rownnz of CHUNKED rows (count) / output offset of every chunk (numeric)
__global__ void k_bin_rows(ChunkGeom g, int64_t k0, int64_t k1, const int64_t* bin_nnz,
                           int64_t* rownnz, const int64_t* crp, int64_t* bin_out, int to_out) {
  const int64_t k = k0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= k1) return;
  const int64_t nbk = g.nb[k], bb = g.binBase[k];
  const int32_t r = g.rows[k];
  int64_t s = to_out ? crp[r] : 0;
  for (int64_t q = 0; q < nbk; ++q) {
    if (to_out) bin_out[bb + q] = s;
    s += bin_nnz[bb + q];
  }
  if (!to_out) rownnz[r] = s;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_aoff(const Mats& M, const int32_t* rows, int64_t nrows, int64_t* aoff,
                       int64_t* ent, hipStream_t st) {
  const int64_t cap = max_grid(256) * 4;  // one wave per row, four per block
  for (int64_t o = 0; o < nrows; o += cap) {
    const int64_t n = std::min(cap, nrows - o);
    const unsigned grid = (unsigned)((n + 3) / 4);
    MG_DISPATCH2(M, hipLaunchKernelGGL((k_aoff<RP, CI>), grid, 256, 0, st, (const RP*)M.arp,
                                        (const CI*)M.acol, (const RP*)M.brp, rows + o, n, aoff,
                                        ent + o));
  }
  return hipGetLastError();
}

hipError_t launch_bin_hist(const Mats& M, const ChunkGeom& g, const BatchArgs& b,
                            const int32_t* tile_row, const int64_t* aoff, const int64_t* tile_e0,
                            int64_t* bin_cnt, int32_t* bin_row, int64_t max_nb, hipStream_t st) {
  if (b.ntiles <= 0) return hipSuccess;
  const size_t lds = BIN_BS * 8 * 2 + (size_t)max_nb * 4 + 64;
  const int64_t cap = max_grid(BIN_BS);
  for (int64_t o = 0; o < b.ntiles; o += cap) {
    BatchArgs bp = b;
    bp.tile0 = b.tile0 + o;
    bp.ntiles = std::min(cap, b.ntiles - o);
    MG_DISPATCH2(M, {
      auto kf = k_bin_hist<RP, CI>;
      (void)hipFuncSetAttribute((const void*)kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      hipLaunchKernelGGL(kf, (unsigned)bp.ntiles, BIN_BS, lds, st, (const RP*)M.arp,
                         (const CI*)M.acol, (const RP*)M.brp, (const CI*)M.bcol, g, bp, tile_row,
                         aoff, tile_e0, (unsigned long long*)bin_cnt, bin_row);
    });
  }
  return hipGetLastError();
}
hipError_t launch_bin_accum(const ChunkGeom& g, const BatchArgs& b, bool numeric, int f64,
                             const int64_t* bin_start, const int64_t* bin_cnt,
                             const int32_t* bin_row, const int64_t* dense_items,
                             const int64_t* sort_items, const int32_t* item_counts,
                             const uint16_t* ws_col, const void* ws_val, int64_t* bin_nnz,
                             const int64_t* bin_out, void* ccol, int col64, void* cval,
                             int dense_block, unsigned int* work, int persistent_wgs, bool det,
                             hipStream_t st) {
  if (b.nbins <= 0) return hipSuccess;
  det = det && numeric;
  const size_t lds = bin_dense_lds(f64, g.shift);
  const unsigned gd = (unsigned)std::min<int64_t>(b.nbins, persistent_wgs);
  // sort items: one wave each, as many as the host read back, else the bound
  // of one per chunk (waves past the count leave at once); the grid is cut
  // below 2^32 work-items
  const int64_t gs_all = ((b.n_sort >= 0 ? b.n_sort : b.nbins) + AS_WAVES - 1) / AS_WAVES;
  const int64_t gcap = max_grid(AS_WAVES * MG_WAVE);
#define MG_AC(V)                                                                                  \
  {                                                                                               \
    if (det) {                                                                                    \
      /* one wave per workgroup: as many workgroups as the LDS holds, twice over */             \
      auto kd = k_accum_dense_det<V>;                                                             \
      (void)hipFuncSetAttribute((const void*)kd, hipFuncAttributeMaxDynamicSharedMemorySize,      \
                                (int)lds);                                                        \
      const unsigned gdd = (unsigned)std::min<int64_t>(b.nbins, (int64_t)persistent_wgs * 8);     \
      hipLaunchKernelGGL(kd, gdd, MG_WAVE, lds, st, g, dense_items, item_counts, b.bin0,          \
                         bin_start, bin_cnt, bin_row, ws_col, (const V*)ws_val, bin_out, ccol,    \
                         col64, (V*)cval, work);                                                  \
    } else {                                                                                      \
      auto kd = numeric ? k_accum_dense<V, true> : k_accum_dense<V, false>;                       \
      (void)hipFuncSetAttribute((const void*)kd, hipFuncAttributeMaxDynamicSharedMemorySize,      \
                                (int)lds);                                                        \
      hipLaunchKernelGGL(kd, gd, dense_block, lds, st, g, dense_items, item_counts, b.bin0,       \
                         bin_start, bin_cnt, bin_row, ws_col, (const V*)ws_val, bin_nnz, bin_out, \
                         ccol, col64, (V*)cval, work);                                            \
    }                                                                                             \
    auto ks = det ? k_accum_sort<V, true, true>                                                   \
                  : (numeric ? k_accum_sort<V, true, false> : k_accum_sort<V, false, false>);     \
    for (int64_t o = 0; o < gs_all; o += gcap)                                                    \
      hipLaunchKernelGGL(ks, (unsigned)std::min(gcap, gs_all - o), AS_WAVES * MG_WAVE, 0, st, g,  \
                         sort_items, item_counts, b.bin0, bin_start, bin_cnt, bin_row, ws_col,    \
                         (const V*)ws_val, bin_nnz, bin_out, ccol, col64, (V*)cval,               \
                         o * AS_WAVES);                                                           \
  }
  if (f64) MG_AC(double) else MG_AC(float)
#undef MG_AC
  return hipGetLastError();
}

hipError_t launch_bin_scatter_det(const Mats& M, const ChunkGeom& g, const int64_t* aoff,
                                  const int64_t* tile_e0, const int32_t* seg_row,
                                  const int64_t* segBase, const int64_t* tabBase,
                                  const int64_t* tabS, int S, int64_t sg0, int64_t nsegs,
                                  const int64_t* bin_start, uint16_t* ws_col, void* ws_val,
                                  int64_t max_nb, hipStream_t st) {
  if (nsegs <= 0) return hipSuccess;
  const size_t lds = bin_scatter_det_lds(M.f64, g.tile, max_nb);
  const int64_t cap = max_grid(DS_BS);
  for (int64_t o = 0; o < nsegs; o += cap) {
#define MG_SD(V)                                                                                  \
  MG_DISPATCH2(M, {                                                                               \
    auto kf = k_bin_scatter_det<RP, CI, V>;                                                       \
    (void)hipFuncSetAttribute((const void*)kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);   \
    hipLaunchKernelGGL(kf, (unsigned)std::min(cap, nsegs - o), DS_BS, lds, st, (const RP*)M.arp,  \
                       (const CI*)M.acol, (const V*)M.aval, (const RP*)M.brp, (const CI*)M.bcol,  \
                       (const V*)M.bval, g, aoff, tile_e0, seg_row, segBase, tabBase, tabS, S,    \
                       sg0 + o, bin_start, ws_col, (V*)ws_val);                                   \
  });
    if (M.f64) { MG_SD(double) } else { MG_SD(float) }
#undef MG_SD
  }
  return hipGetLastError();
}

hipError_t launch_row_bitmap(const Mats& M, const ChunkGeom& g, const int64_t* aoff,
                             int64_t max_nb, int64_t* bin_nnz, int64_t* bin_cnt, int32_t* bin_row,
                             int64_t* rownnz, hipStream_t st) {
  if (g.nch <= 0) return hipSuccess;
  const size_t lds = row_bitmap_lds(g.shift, max_nb);
  const int64_t cap = max_grid(RB_BS);
  for (int64_t o = 0; o < g.nch; o += cap) {
    MG_DISPATCH2(M, {
      auto kf = k_row_bitmap<RP, CI>;
      (void)hipFuncSetAttribute((const void*)kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      hipLaunchKernelGGL(kf, (unsigned)std::min(cap, g.nch - o), RB_BS, lds, st, (const RP*)M.arp,
                         (const CI*)M.acol, (const RP*)M.brp, (const CI*)M.bcol, g, aoff, bin_nnz,
                         bin_cnt, bin_row, rownnz, o);
    });
  }
  return hipGetLastError();
}

hipError_t launch_tile_e0(const Mats& M, const ChunkGeom& g, const int32_t* tile_row,
                          const int64_t* aoff, int64_t ntiles, int64_t* tile_e0, hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  const unsigned grid = (unsigned)((ntiles + 255) / 256);
  if (M.rp64)
    hipLaunchKernelGGL(k_tile_e0<int64_t>, grid, 256, 0, st, (const int64_t*)M.arp, g, tile_row,
                       aoff, ntiles, tile_e0);
  else
    hipLaunchKernelGGL(k_tile_e0<int32_t>, grid, 256, 0, st, (const int32_t*)M.arp, g, tile_row,
                       aoff, ntiles, tile_e0);
  return hipGetLastError();
}

hipError_t launch_bin_scatter2(const Mats& M, const ChunkGeom& g, const BatchArgs& b, bool numeric,
                               int lc32, int sorted, int block, const int32_t* tile_row, const int64_t* aoff,
                               const int64_t* tile_e0, const int64_t* bin_start,
                               unsigned long long* bin_cursor, void* ws_col, void* ws_val,
                               int64_t max_nb, hipStream_t st) {
  if (b.ntiles <= 0) return hipSuccess;
  // the chunk-order index is 16-bit
  if (sorted && g.tile > 65536) return hipErrorInvalidValue;
  const size_t lds = bin_scatter2_lds(M.f64, g.tile, max_nb, lc32, sorted, block);
  const int bs = scatter2_block(lc32, sorted, block);
  if (bs != 256 && bs != 512 && bs != 1024) return hipErrorInvalidValue;
  const int64_t cap = max_grid(bs);
  for (int64_t o = 0; o < b.ntiles; o += cap) {
    BatchArgs bp = b;
    bp.tile0 = b.tile0 + o;
    bp.ntiles = std::min(cap, b.ntiles - o);
    // 32-bit columns: the chunk-ordered form at bs threads
#define MG_SC2_BS(BSZ, V, LC)                                                                     \
  MG_DISPATCH2(M, {                                                                               \
    auto kf = numeric ? (sorted ? k_bin_scatter2<BSZ, RP, CI, V, LC, true, true>                   \
                                : k_bin_scatter2<BIN_BS, RP, CI, V, LC, true, false>)              \
                      : (sorted ? k_bin_scatter2<BSZ, RP, CI, V, LC, false, true>                  \
                                : k_bin_scatter2<BIN_BS, RP, CI, V, LC, false, false>);            \
    (void)hipFuncSetAttribute((const void*)kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);   \
    hipLaunchKernelGGL(kf, (unsigned)bp.ntiles, bs, lds, st, (const RP*)M.arp,                    \
                       (const CI*)M.acol, (const V*)M.aval, (const RP*)M.brp, (const CI*)M.bcol,  \
                       (const V*)M.bval, g, bp, tile_row, aoff, tile_e0, bin_start, bin_cursor,   \
                       (LC*)ws_col, (V*)ws_val);                                                  \
  });
    if (lc32) {
      if (bs == 1024) {
        if (M.f64) { MG_SC2_BS(1024, double, uint32_t) } else { MG_SC2_BS(1024, float, uint32_t) }
      } else if (bs == 512) {
        if (M.f64) { MG_SC2_BS(512, double, uint32_t) } else { MG_SC2_BS(512, float, uint32_t) }
      } else {
        if (M.f64) { MG_SC2_BS(256, double, uint32_t) } else { MG_SC2_BS(256, float, uint32_t) }
      }
    } else {
      if (M.f64) { MG_SC2_BS(BIN_BS, double, uint16_t) } else { MG_SC2_BS(BIN_BS, float, uint16_t) }
    }
#undef MG_SC2_BS
  }
  return hipGetLastError();
}

hipError_t launch_l2_hist(const ChunkGeom& g2, const BatchArgs& b2, const int32_t* tile_row2,
                          const int64_t* start1, const uint32_t* ws1_col, int64_t* cnt2,
                          int64_t max_nb2, hipStream_t st) {
  if (b2.ntiles <= 0) return hipSuccess;
  const size_t lds = (size_t)max_nb2 * 4 + 64;
  const int64_t cap = max_grid(512);
  for (int64_t o = 0; o < b2.ntiles; o += cap) {
    BatchArgs bp = b2;
    bp.tile0 = b2.tile0 + o;
    bp.ntiles = std::min(cap, b2.ntiles - o);
    hipLaunchKernelGGL(k_l2_hist<512>, (unsigned)bp.ntiles, 512, lds, st, g2, bp, tile_row2,
                       start1, ws1_col, (unsigned long long*)cnt2);
  }
  return hipGetLastError();
}

hipError_t launch_vrow_rows(const ChunkGeom& g2, int32_t* row2, hipStream_t st) {
  const int64_t cap = max_grid(256) * 4;  // one wave per virtual row
  for (int64_t o = 0; o < g2.nch; o += cap)
    hipLaunchKernelGGL(k_vrow_rows, (unsigned)((std::min(cap, g2.nch - o) + 3) / 4), 256, 0, st,
                       g2, row2, o);
  return hipGetLastError();
}

hipError_t launch_vrow_geom(const ChunkGeom& g1, int fshift, int64_t* minc2, int64_t* maxc2,
                            int64_t* nb2, hipStream_t st) {
  const int64_t cap = max_grid(256) * 4;  // one wave per coarse row
  for (int64_t o = 0; o < g1.nch; o += cap)
    hipLaunchKernelGGL(k_vrow_geom, (unsigned)((std::min(cap, g1.nch - o) + 3) / 4), 256, 0, st,
                       g1, fshift, minc2, maxc2, nb2, o);
  return hipGetLastError();
}

hipError_t launch_vrow_tiles(const ChunkGeom& g2, int64_t k0, int64_t k1, hipStream_t st) {
  if (k1 <= k0) return hipSuccess;
  hipLaunchKernelGGL(k_vrow_tiles, (unsigned)((k1 - k0 + 255) / 256), 256, 0, st, g2, k0, k1);
  return hipGetLastError();
}

hipError_t launch_vrow_split(const int64_t* cnt1, int64_t k0, int64_t n, int64_t* flags,
                             int64_t* pos, int64_t* nbig, void* scan_temp, int32_t* big,
                             int32_t* small, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const unsigned g = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(k_vrow_flags, g, 256, 0, st, cnt1, k0, n, flags);
  hipError_t e = scan_excl_i64(flags, pos, n, nbig, nullptr, scan_temp, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_vrow_split, g, 256, 0, st, cnt1, k0, n, (const int64_t*)pos, big, small);
  return hipGetLastError();
}

hipError_t launch_vrow_gather(const int32_t* rows, int64_t n, const int64_t* vnb,
                              const int64_t* cnt1, int64_t* nb, int64_t* cnt, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_vrow_gather, (unsigned)((n + 255) / 256), 256, 0, st, rows, n, vnb, cnt1,
                     nb, cnt);
  return hipGetLastError();
}

hipError_t launch_vrow_sort(bool numeric, int f64, const int32_t* small, int64_t nsmall,
                            const int64_t* cnt1, const int64_t* start1, const int64_t* minc2,
                            const uint32_t* ws1_col, const void* ws1_val, int64_t* nnz1,
                            const int64_t* out1, void* ccol, int col64, void* cval,
                            hipStream_t st) {
  if (nsmall <= 0) return hipSuccess;
  const int64_t gall = (nsmall + AS_WAVES - 1) / AS_WAVES;
  const int64_t gcap = max_grid(AS_WAVES * MG_WAVE);
#define MG_VS(V)                                                                                  \
  {                                                                                               \
    auto kf = numeric ? k_vrow_sort<V, true> : k_vrow_sort<V, false>;                             \
    for (int64_t o = 0; o < gall; o += gcap)                                                      \
      hipLaunchKernelGGL(kf, (unsigned)std::min(gcap, gall - o), AS_WAVES * MG_WAVE, 0, st,       \
                         small, nsmall, cnt1, start1, minc2, ws1_col, (const V*)ws1_val, nnz1,    \
                         out1, ccol, col64, (V*)cval, o * AS_WAVES);                               \
  }
  if (f64) MG_VS(double) else MG_VS(float)
#undef MG_VS
  return hipGetLastError();
}

hipError_t launch_vrow_bitmap(const ChunkGeom& g2, int cshift, int64_t k0, int64_t k1,
                              int64_t max_nb2, const int64_t* start1, const uint32_t* ws1_col,
                              int64_t* bin_cnt2, int64_t* bin_nnz2, int32_t* bin_row2,
                              int64_t* vnnz, hipStream_t st) {
  if (k1 <= k0) return hipSuccess;
  const size_t lds = vrow_bitmap_lds(cshift, max_nb2);
  (void)hipFuncSetAttribute((const void*)k_vrow_bitmap, hipFuncAttributeMaxDynamicSharedMemorySize,
                      (int)lds);
  const int64_t cap = max_grid(VB_BS);
  for (int64_t o = k0; o < k1; o += cap)
    hipLaunchKernelGGL(k_vrow_bitmap, (unsigned)std::min(cap, k1 - o), VB_BS, lds, st, g2, o,
                       start1, ws1_col, bin_cnt2, bin_nnz2, bin_row2, vnnz);
  return hipGetLastError();
}

hipError_t launch_l2_scatter(const ChunkGeom& g2, const BatchArgs& b2, bool numeric, int f64,
                             const int32_t* tile_row2, const int64_t* start1,
                             const uint32_t* ws1_col, const void* ws1_val,
                             const int64_t* bin_start2, unsigned long long* bin_cursor2,
                             uint16_t* ws2_col, void* ws2_val, int64_t max_nb2, int block,
                             hipStream_t st) {
  if (b2.ntiles <= 0) return hipSuccess;
  if (g2.tile > 65536) return hipErrorInvalidValue;  // 16-bit positions
  const int bs = block > 0 ? block : MG_L2_BS;
  if (bs != 256 && bs != 1024) return hipErrorInvalidValue;
  const size_t lds = l2_scatter_lds(f64, g2.tile, max_nb2);
  const int64_t cap = max_grid(bs);
#define MG_L2(BSZ, V)                                                                             \
  {                                                                                               \
    auto kf = numeric ? k_l2_scatter<BSZ, V, true> : k_l2_scatter<BSZ, V, false>;                 \
    (void)hipFuncSetAttribute((const void*)kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);   \
    for (int64_t o = 0; o < b2.ntiles; o += cap) {                                                \
      BatchArgs bp = b2;                                                                          \
      bp.tile0 = b2.tile0 + o;                                                                    \
      bp.ntiles = std::min(cap, b2.ntiles - o);                                                   \
      hipLaunchKernelGGL(kf, (unsigned)bp.ntiles, BSZ, lds, st, g2, bp, tile_row2, start1,        \
                         ws1_col, (const V*)ws1_val, bin_start2, bin_cursor2, ws2_col,            \
                         (V*)ws2_val);                                                            \
    }                                                                                             \
  }
  if (bs == 1024) {
    if (f64) MG_L2(1024, double) else MG_L2(1024, float)
  } else {
    if (f64) MG_L2(256, double) else MG_L2(256, float)
  }
#undef MG_L2
  return hipGetLastError();
}

hipError_t launch_bin_group(const ChunkGeom& g, const BatchArgs& b, const int64_t* bin_cnt,
                            int64_t dense_min, int64_t group_max, int64_t* dense_items,
                            int64_t* sort_items, int32_t* item_counts, hipStream_t st) {
  const int64_t nr = b.k1 - b.k0;
  if (nr <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_bin_group, (unsigned)((nr + 255) / 256), 256, 0, st, g, b, bin_cnt,
                     dense_min, group_max, dense_items, sort_items, item_counts, b.bin0);
  return hipGetLastError();
}

hipError_t launch_bin_rows(const ChunkGeom& g, int64_t k0, int64_t k1, const int64_t* bin_nnz,
                           int64_t* rownnz, const int64_t* crp, int64_t* bin_out, bool to_out,
                           hipStream_t st) {
  if (k1 <= k0) return hipSuccess;
  hipLaunchKernelGGL(k_bin_rows, (unsigned)((k1 - k0 + 255) / 256), 256, 0, st, g, k0, k1, bin_nnz,
                     rownnz, crp, bin_out, to_out ? 1 : 0);
  return hipGetLastError();
}

}  // namespace mg
