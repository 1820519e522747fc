#pragma once
// SORT rows (expand, sort, merge; Algorithm 2) in two modes: count (precise
// symbolic phase, Section 2.1) and numeric (values written straight into C at
// the row offsets the symbolic phase produced).
#include "common.h"
#include "kernels.h"
#include "k_sort_decl.h"

namespace mg {

MG_INLINE void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

// ---------------------------------------------------------------------------
// SORT rows.  One wave per tile of R consecutive rows of one size class; the
// tile's products (<= 64*E) are gathered into wave-private LDS with a
// composite key (slot << colbits | col - minc), sorted by a register bitonic
// network, then merged: count mode counts distinct keys per row, numeric mode
// sums runs of equal keys (each run starting from +0.0) and writes them in
// ascending column order at the row's offset in C.
//
// Count mode of the classes with one row per wave (E > 1) needs no order:
// the products' keys go into a wave-private open-addressing table in LDS
// (linear probing, twice as many slots as the wave can stage, so it never
// fills), and the row's distinct columns are the inserts that found an empty
// slot.  (Packing several rows into one wave to keep more loads in flight
// measured slower: the larger table lowers occupancy more than it gains.)
// ---------------------------------------------------------------------------
constexpr int SR_WAVES = 4;

template <typename K>
MG_INLINE K key_max() { return (K)~(K)0; }

// Multiplicative (Fibonacci) hash of a key to `bits` bits: consecutive
// columns (banded rows) land far apart, so linear probing stays short.
MG_INLINE uint32_t key_hash(uint32_t k, int bits) { return (k * 2654435769u) >> (32 - bits); }
MG_INLINE uint32_t key_hash(uint64_t k, int bits) {
  return (uint32_t)((k * 0x9E3779B97F4A7C15ull) >> (64 - bits));
}

// One tile (R consecutive rows of the class list, one wave).
template <typename RP, typename CI, typename V, int E, typename K, bool NUMERIC>
MG_INLINE void sort_rows_tile(RowSrc src, const int32_t* __restrict__ list, int64_t count,
                              int R, int colbits, const int64_t* __restrict__ minc,
                              int64_t* rownnz, const int64_t* __restrict__ crp, DevStats* stats,
                              int tile_in) {
  // the tile index is wave-uniform: keep it in a scalar register
  const int64_t tile = __builtin_amdgcn_readfirstlane(tile_in);
  constexpr int CAP = MG_WAVE * E;
  constexpr bool HASH = !NUMERIC && E > 1;  // count by table inserts, no sort
  constexpr int HT = HASH ? 2 * CAP : 1;     // table slots (a power of two)
  constexpr int HTB = ilog2c(HT);
  constexpr int U = 4;  // products per lane whose loads are in flight together
  __shared__ K s_key[SR_WAVES][HASH ? 1 : CAP];
  __shared__ K s_hash[SR_WAVES][HT];
  __shared__ V s_val[SR_WAVES][NUMERIC ? CAP : 1];
  __shared__ int32_t s_pre[SR_WAVES][MG_WAVE + 1];
  __shared__ const CI* s_bcolp[SR_WAVES][MG_WAVE];
  __shared__ const V* s_bvalp[SR_WAVES][NUMERIC ? MG_WAVE : 1];
  __shared__ V s_av[SR_WAVES][NUMERIC ? MG_WAVE : 1];
  __shared__ int32_t s_wslot[SR_WAVES][MG_WAVE];
  // per-row slots: a wave takes R = 64 / 2^c rows of the classes with one
  // element per lane and a single row beyond, so only E = 1 needs 64 slots
  // (the LDS saved raises the occupancy of the larger classes)
  constexpr int RS = (E == 1) ? MG_WAVE : 1;
  __shared__ int64_t s_ent[SR_WAVES][RS];
  __shared__ int64_t s_apos[SR_WAVES][RS];
  __shared__ int64_t s_minc[SR_WAVES][RS];
  __shared__ int32_t s_row[SR_WAVES][RS];
  __shared__ int32_t s_mat[SR_WAVES][RS];
  __shared__ int64_t s_cb[SR_WAVES][NUMERIC ? RS : 1];
  __shared__ int32_t s_aux[SR_WAVES][RS];

  const int w = threadIdx.x / MG_WAVE;
  const int l = lane();
  const int64_t r0 = tile * R;
  if (r0 >= count) return;  // whole wave leaves together
  const int nr = (int)((count - r0) < R ? (count - r0) : R);
  if (nr > RS) {  // more rows per wave than the slots hold: not a launch this file makes
    if (l == 0) atomicOr(&stats->err, ERR_STAGE_OVERFLOW);
    return;
  }

  int64_t ne = 0;
  if (l < nr) {
    const int32_t row = list[r0 + l];
    const int32_t b = src.tab ? src.mat_of_row[row] : 0;
    const MatEnt& M = src.tab ? src.tab[b] : src.one;
    const int64_t lrow = row - M.row0;
    const RP* arp = (const RP*)M.arp;
    const int64_t a0 = ld_global(arp + lrow);
    ne = (int64_t)ld_global(arp + lrow + 1) - a0;
    s_row[w][l] = row;
    s_mat[w][l] = b;
    s_apos[w][l] = a0;
    s_minc[w][l] = minc[row];
    if (NUMERIC) s_cb[w][l] = src.tab ? crp[M.row0] : 0;
  }
  const int64_t einc = wave_incl_scan(ne);
  const int64_t ntot = __shfl(einc, MG_WAVE - 1, MG_WAVE);
  if (l < RS) {
    s_ent[w][l] = einc - ne;
    s_aux[w][l] = 0;
  }
  wave_sync();

  const K kmask = ((K)1 << colbits) - 1;
  int P = 0;
  int fresh = 0;  // HASH: this lane's inserts that took an empty slot
  if constexpr (HASH) {
    for (int x = l; x < HT; x += MG_WAVE) s_hash[w][x] = key_max<K>();
    wave_sync();
  }
  for (int64_t f0 = 0; f0 < ntot; f0 += MG_WAVE) {
    const int64_t f = f0 + l;
    int len = 0, slot = 0;
    const CI* bcp = nullptr;
    const V* bvp = nullptr;
    V av = (V)0;
    if (f < ntot) {
      // s_ent of the slots past nr is ntot > f
      if constexpr (RS == MG_WAVE) slot = upper_index64(s_ent[w], f);
      const MatEnt& M = src.tab ? src.tab[s_mat[w][slot]] : src.one;
      const int64_t p = s_apos[w][slot] + (f - s_ent[w][slot]);
      const int64_t j = ld_global((const CI*)M.acol + p);
      const RP* brp = (const RP*)M.brp;
      const int64_t b0 = ld_global(brp + j);
      len = (int)((int64_t)ld_global(brp + j + 1) - b0);
      bcp = (const CI*)M.bcol + b0;
      if (NUMERIC) {
        bvp = (const V*)M.bval + b0;
        av = ld_global((const V*)M.aval + p);
      }
    }
    const int inc = wave_incl_scan(len);
    const int tot = __shfl(inc, MG_WAVE - 1, MG_WAVE);
    s_pre[w][l] = inc - len;
    s_bcolp[w][l] = bcp;
    if (NUMERIC) s_bvalp[w][l] = bvp;
    if (NUMERIC) s_av[w][l] = av;
    s_wslot[w][l] = slot;
    wave_sync();
    if (P + tot > CAP) {
      if (l == 0) atomicOr(&stats->err, ERR_STAGE_OVERFLOW);
      return;
    }
    // U products per lane are located, then loaded, then staged, so their
    // loads are in flight together
    for (int qb = l; qb < tot; qb += U * MG_WAVE) {
      const CI* cp4[U];
      const V* vp4[U];
      V a4[U];
      int s4[U];
      // owner of product q: the last lane k with s_pre[k] <= q (the lanes
      // past the live A entries hold tot, and s_pre[0] = 0); searched for
      // every u without a branch, so the U searches interleave
      int k4[U];
#pragma unroll
      for (int u = 0; u < U; ++u) k4[u] = upper_index64(s_pre[w], qb + u * MG_WAVE);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = k4[u];
        const int off = qb + u * MG_WAVE - s_pre[w][k];
        cp4[u] = s_bcolp[w][k] + off;
        if (NUMERIC) {
          vp4[u] = s_bvalp[w][k] + off;
          a4[u] = s_av[w][k];
        }
        s4[u] = s_wslot[w][k];
      }
      CI c4[U];
      V v4[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool ok = qb + u * MG_WAVE < tot;
        c4[u] = ok ? ld_global(cp4[u]) : (CI)0;
        if (NUMERIC) v4[u] = ok ? ld_global(vp4[u]) : (V)0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int q = qb + u * MG_WAVE;
        if (q < tot) {
          const K key = ((K)s4[u] << colbits) | (K)((int64_t)c4[u] - s_minc[w][s4[u]]);
          if constexpr (HASH) {
            // at most CAP distinct keys in 2*CAP slots: an empty slot or the
            // key itself is always reached
            uint32_t hx = key_hash(key, HTB);
            for (;;) {
              const K old = atomicCAS(&s_hash[w][hx], key_max<K>(), key);
              if (old == key_max<K>()) {
                ++fresh;
                break;
              }
              if (old == key) break;
              hx = (hx + 1) & (HT - 1);
            }
          } else {
            s_key[w][P + q] = key;
            if (NUMERIC) s_val[w][P + q] = a4[u] * v4[u];
          }
        }
      }
    }
    P += tot;
    wave_sync();
  }
  if constexpr (HASH) {
    // one row per wave (R = 1 for E > 1)
    const int distinct = wave_sum(fresh);
    if (l == 0) rownnz[s_row[w][0]] = distinct;
  } else {

    // load (striped: the network sorts whatever order it is given).  In
    // numeric mode the key carries the element's staging index in its low
    // IDXB bits: the network moves one word per element, runs of equal keys
    // sum in staging order, and values are fetched from LDS after the sort.
    constexpr int IDXB = NUMERIC ? ilog2c(CAP) : 0;
    K k[E];
  #pragma unroll
    for (int e = 0; e < E; ++e) {
      const int x = e * MG_WAVE + l;
      k[e] = (x < P) ? ((s_key[w][x] << IDXB) | (NUMERIC ? (K)x : (K)0)) : key_max<K>();
    }
    bitonic_sort_keys<E>(k);
    V v[NUMERIC ? E : 1];
    if (NUMERIC) {
      wave_sync();
  #pragma unroll
      for (int e = 0; e < E; ++e) {
        const int x = l * E + e;
        v[e] = (x < P) ? s_val[w][(int)(k[e] & (K)(CAP - 1))] : (V)0;
      }
    }
  #pragma unroll
    for (int e = 0; e < E; ++e) k[e] >>= IDXB;

    // heads of runs of equal keys (blocked layout: element x = l*E + e)
    const K prevk = __shfl_up(k[E - 1], 1, MG_WAVE);
    bool head[E];
    int hc = 0;
  #pragma unroll
    for (int e = 0; e < E; ++e) {
      const int x = l * E + e;
      const K pk = (e == 0) ? prevk : k[e - 1];
      head[e] = (x < P) && (x == 0 || k[e] != pk);
      hc += head[e] ? 1 : 0;
    }
    if (!NUMERIC) {
      // distinct keys of a row = head rank at the next row's first element (or
      // the wave's total) minus the rank at this row's first element; every
      // row of the tile has at least one product, so each slot has a first
      const int hinc = wave_incl_scan(hc);
      const int htot = __shfl(hinc, MG_WAVE - 1, MG_WAVE);
      int hr = hinc - hc;
  #pragma unroll
      for (int e = 0; e < E; ++e) {
        const int x = l * E + e;
        const K pk = (e == 0) ? prevk : k[e - 1];
        if (head[e]) {
          if (x == 0 || (k[e] >> colbits) != (pk >> colbits)) s_aux[w][(int)(k[e] >> colbits)] = hr;
          ++hr;
        }
      }
      wave_sync();
      if (l < nr) rownnz[s_row[w][l]] = ((l + 1 < nr) ? s_aux[w][l + 1] : htot) - s_aux[w][l];
      return;
    } else {
      const int hinc = wave_incl_scan(hc);
      const int hbase = hinc - hc;
      // rank of the first head of each slot
      int hr = hbase;
  #pragma unroll
      for (int e = 0; e < E; ++e) {
        const int x = l * E + e;
        const K pk = (e == 0) ? prevk : k[e - 1];
        if (head[e]) {
          if (x == 0 || (k[e] >> colbits) != (pk >> colbits)) s_aux[w][(int)(k[e] >> colbits)] = hr;
          ++hr;
        }
      }
      // segmented sums: per lane (has_head, sum of its trailing run), then a
      // segmented inclusive scan across lanes for the carry into each lane
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
      wave_sync();
      const K nextk = __shfl_down(k[0], 1, MG_WAVE);
      V run = carry;
      hr = hbase;
  #pragma unroll
      for (int e = 0; e < E; ++e) {
        const int x = l * E + e;
        if (head[e]) { run = (V)0 + v[e]; ++hr; }
        else run = run + v[e];
        const K nk = (e == E - 1) ? nextk : k[e + 1];
        const bool tail = (x < P) && (x == P - 1 || nk != k[e]);
        if (tail) {
          const int sl = (int)(k[e] >> colbits);
          const MatEnt& M = src.tab ? src.tab[s_mat[w][sl]] : src.one;
          const int64_t pos = crp[s_row[w][sl]] - s_cb[w][sl] + (hr - 1 - s_aux[w][sl]);
          st_stream<HINT_C_STORE>(&((CI*)M.ccol)[pos],
                                  (CI)(s_minc[w][sl] + (int64_t)(k[e] & kmask)));
          st_stream<HINT_C_STORE>(&((V*)M.cval)[pos], run);
        }
      }
    }
  }  // !HASH
}

// One tile per wave from the grid (work == nullptr), or persistent waves that
// take runs of `grab` consecutive tiles from the counter *work (one atomic
// per run, so the counter is not a point of contention) until the list is
// done.
// (Two kernels rather than one with both paths: one inlined copy of the tile
// per kernel keeps its register count, and so its occupancy.)
template <typename RP, typename CI, typename V, int E, typename K, bool NUMERIC>
__global__ void __launch_bounds__(SR_WAVES * MG_WAVE)
    k_sort_rows(RowSrc src, const int32_t* __restrict__ list, int64_t count, int R, int colbits,
                const int64_t* __restrict__ minc, int64_t* rownnz, const int64_t* __restrict__ crp,
                DevStats* stats) {
  sort_rows_tile<RP, CI, V, E, K, NUMERIC>(src, list, count, R, colbits, minc, rownnz, crp, stats,
                                           (int)(blockIdx.x * SR_WAVES + threadIdx.x / MG_WAVE));
}

template <typename RP, typename CI, typename V, int E, typename K, bool NUMERIC>
__global__ void __launch_bounds__(SR_WAVES * MG_WAVE)
    k_sort_rows_persistent(RowSrc src, const int32_t* __restrict__ list, int64_t count, int R,
                           int colbits, const int64_t* __restrict__ minc, int64_t* rownnz,
                           const int64_t* __restrict__ crp, DevStats* stats, unsigned int* work,
                           int grab) {
  const int64_t ntiles = (count + R - 1) / R;
  for (;;) {
    unsigned int tt = 0;
    if (lane() == 0) tt = atomicAdd(work, (unsigned int)grab);
    const int64_t t0 = (int64_t)__shfl(tt, 0, MG_WAVE);
    if (t0 >= ntiles) return;  // the whole wave leaves together
    const int64_t t1 = (t0 + grab < ntiles) ? t0 + grab : ntiles;
    for (int64_t tile = t0; tile < t1; ++tile) {
      sort_rows_tile<RP, CI, V, E, K, NUMERIC>(src, list, count, R, colbits, minc, rownnz, crp,
                                               stats, (int)tile);
      wave_sync();  // the tile's LDS is read before the next tile writes it
    }
  }
}

template <typename RP, typename CI, typename V, int E, typename K>
static void sort_rows_launch(const RowSrc& src, bool numeric, const int32_t* list, int64_t count,
                             int R, int colbits, const int64_t* minc, int64_t* rownnz,
                             const int64_t* crp, DevStats* stats, unsigned grid, unsigned int* work,
                             int grab, hipStream_t st) {
  if (grid == 0) return;
  if (work) {
    if (numeric)
      hipLaunchKernelGGL((k_sort_rows_persistent<RP, CI, V, E, K, true>), grid, SR_WAVES * MG_WAVE,
                         0, st, src, list, count, R, colbits, minc, rownnz, crp, stats, work, grab);
    else
      hipLaunchKernelGGL((k_sort_rows_persistent<RP, CI, V, E, K, false>), grid,
                         SR_WAVES * MG_WAVE, 0, st, src, list, count, R, colbits, minc, rownnz,
                         crp, stats, work, grab);
    return;
  }
  if (numeric)
    hipLaunchKernelGGL((k_sort_rows<RP, CI, V, E, K, true>), grid, SR_WAVES * MG_WAVE, 0, st, src,
                       list, count, R, colbits, minc, rownnz, crp, stats);
  else
    hipLaunchKernelGGL((k_sort_rows<RP, CI, V, E, K, false>), grid, SR_WAVES * MG_WAVE, 0, st, src,
                       list, count, R, colbits, minc, rownnz, crp, stats);
}

template <typename RP, typename CI, typename V, int E, typename K>
static hipError_t sort_rows_t(const RowSrc& src, bool numeric, const int32_t* list, int64_t count,
                              int R, int colbits, const int64_t* minc, int64_t* rownnz,
                              const int64_t* crp, DevStats* stats, unsigned int* work,
                              int persistent_blocks, hipStream_t st) {
  if (work) {
    // persistent: as many workgroups as are resident at once (at most
    // persistent_blocks), each wave pulling tiles; the counter starts at 0
    int per_cu = 0, dev = 0, cus = 1;
    auto kf = numeric ? k_sort_rows_persistent<RP, CI, V, E, K, true>
                      : k_sort_rows_persistent<RP, CI, V, E, K, false>;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kf, SR_WAVES * MG_WAVE, 0) !=
            hipSuccess ||
        per_cu < 1)
      per_cu = 1;
    if (hipGetDevice(&dev) == hipSuccess)
      (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int64_t tiles = (count + R - 1) / R;
    int64_t grid = std::min<int64_t>((int64_t)per_cu * std::max(cus, 1),
                                     (tiles + SR_WAVES - 1) / SR_WAVES);
    if (persistent_blocks > 0) grid = std::min<int64_t>(grid, persistent_blocks);
    grid = std::max<int64_t>(grid, 1);
    // about 16 grabs per wave, each of consecutive tiles
    const int64_t grab = std::max<int64_t>(1, std::min<int64_t>(
        1 << 16, tiles / (grid * SR_WAVES * 16)));
    sort_rows_launch<RP, CI, V, E, K>(src, numeric, list, count, R, colbits, minc, rownnz, crp,
                                      stats, (unsigned)grid, work, (int)grab, st);
    return hipGetLastError();
  }
  // a wave takes R rows; pieces of at most max_grid blocks of SR_WAVES waves
  const int64_t rows_cap = max_grid(SR_WAVES * MG_WAVE) * SR_WAVES * R;
  for (int64_t o = 0; o < count; o += rows_cap) {
    const int64_t n = std::min(rows_cap, count - o);
    const int64_t tiles = (n + R - 1) / R;
    const unsigned grid = (unsigned)((tiles + SR_WAVES - 1) / SR_WAVES);
    sort_rows_launch<RP, CI, V, E, K>(src, numeric, list + o, n, R, colbits, minc, rownnz, crp,
                                      stats, grid, nullptr, 1, st);
  }
  return hipGetLastError();
}


template <typename RP, typename CI, typename V>
hipError_t sort_rows_cls(const RowSrc& src, int cls, bool numeric, const int32_t* list,
                         int64_t count, const int64_t* minc, int colbits, int64_t* rownnz,
                         const int64_t* crp, DevStats* stats, unsigned int* work,
                         int persistent_blocks, hipStream_t st) {
  // class c holds rows with ip in (2^(c-1), 2^c]: E = max(1, 2^c / 64) per
  // lane, R = 64 * E / 2^c rows per wave
  const int E = (cls <= 6) ? 1 : (1 << (cls - 6));
  const int R = (cls <= 6) ? (64 >> cls) : 1;  // R > 1 only with E = 1 (the kernel's slots)
  int slotbits = 0;
  while ((1 << slotbits) < R) ++slotbits;
  int capbits = 0;
  while ((1 << capbits) < 64 * E) ++capbits;
  // count mode keeps keys below 2^31 (all-ones marks padding); numeric keys
  // add the staging index and may use all 32 bits (see the kernel)
  const bool k64 = numeric ? (colbits + slotbits + capbits) > 32 : (colbits + slotbits) > 31;
#define MG_SR(EE)                                                                               \
  if (E == EE) {                                                                                \
    if (k64)                                                                                    \
      return sort_rows_t<RP, CI, V, EE, uint64_t>(src, numeric, list, count, R, colbits, minc,  \
                                                  rownnz, crp, stats, work, persistent_blocks,  \
                                                  st);                                          \
    return sort_rows_t<RP, CI, V, EE, uint32_t>(src, numeric, list, count, R, colbits, minc,    \
                                                rownnz, crp, stats, work, persistent_blocks,    \
                                                st);                                            \
  }
  MG_SR(1) MG_SR(2) MG_SR(4) MG_SR(8) MG_SR(16)
#undef MG_SR
  return hipErrorInvalidValue;
}

#define MG_SORT_INSTANTIATE(RP, V)                                                              \
  template hipError_t sort_rows_cls<RP, int32_t, V>(const RowSrc&, int, bool, const int32_t*,   \
                                                     int64_t, const int64_t*, int, int64_t*,    \
                                                     const int64_t*, DevStats*, unsigned int*,  \
                                                     int, hipStream_t);                         \
  template hipError_t sort_rows_cls<RP, int64_t, V>(const RowSrc&, int, bool, const int32_t*,   \
                                                     int64_t, const int64_t*, int, int64_t*,    \
                                                     const int64_t*, DevStats*, unsigned int*,  \
                                                     int, hipStream_t);

}  // namespace mg
