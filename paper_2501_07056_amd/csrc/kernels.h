// Internal launch interface between the host runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace mg {

// Row classes: 0..10 are SORT rows with ip in (2^(c-1), 2^c]; then DENSE,
// CHUNKED, EMPTY.
constexpr int NSORT_CLS = 11;
constexpr int CLS_DENSE = 11;
constexpr int CLS_CHUNKED = 12;
constexpr int CLS_EMPTY = 13;
constexpr int CLS_COARSE = 14;  // CHUNKED rows taken through the coarse level first
constexpr int NCLS = 16;
constexpr int SORT_CAP = 1024;  // products one wave sorts (64 lanes x 16)

// Device-side statistics of a plan (one struct in device memory).
struct DevStats {
  unsigned long long ip_total;
  unsigned long long max_ip;
  unsigned long long max_range;
  unsigned long long ip_cat[4];
  unsigned long long rows_cat[4];
  unsigned long long ent_cat[4];   // A entries of the rows of each category
  unsigned long long nnz_cat[4];   // nnz of C in the rows of each category
  unsigned long long range_cat[3]; // widest column range among SORT, DENSE, CHUNKED rows
  unsigned long long heavy;        // rows deferred to the long-row setup kernel
  unsigned int err;  // bit flags, see ERR_*
  unsigned int pad;
};
constexpr unsigned ERR_STAGE_OVERFLOW = 1u;
constexpr unsigned ERR_INVALID_CSR = 2u;
constexpr unsigned ERR_BIN_OVERFLOW = 4u;

// Device views of A (n x k) and B (k x m) sharing index types.
struct Mats {
  const void *arp, *acol, *aval;
  const void *brp, *bcol, *bval;
  int64_t n, k, m;
  int rp64, col64, f64;
};

// One product C = A * B (device pointers).  In a batch, its rows are rows
// row0 .. row0 + nrows - 1 of the batch's concatenated row numbering.
struct MatEnt {
  const void *arp, *acol, *aval;
  const void *brp, *bcol, *bval;
  void *ccol, *cval, *crp_out;
  int64_t row0, nrows;
  int64_t sort_max, dense_max;  // classification thresholds of this product
  int64_t mcols;                // columns of B (and C)
  int32_t crp_out64;            // crp_out holds int64 (else int32)
  int32_t pad;
};

// Batched row addressing: tab == nullptr means every row belongs to `one`.
struct RowSrc {
  MatEnt one;
  const MatEnt* tab;
  const int32_t* mat_of_row;
};

struct ClassParams {
  int64_t sort_max;   // SORT iff ip < sort_max (<= SORT_CAP)
  int64_t dense_max;  // DENSE iff column range <= dense_max
  int force;          // -1 auto, else category
  int64_t coarse_range;  // CHUNKED rows wider than this take the coarse level (<= 0: never)
};

size_t scan_temp_bytes(int64_t n);
hipError_t scan_excl_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* total,
                         const int64_t* carry, void* temp, hipStream_t st);
hipError_t scan_excl_i32(const int32_t* in, int64_t* out, int64_t n, int64_t* total,
                         const int64_t* carry, void* temp, hipStream_t st);

// --- row level (k_rows.hip) ---
// heavy: scratch of M.n int32 (rows with many A entries are listed there and
// set up by a workgroup each)
hipError_t launch_rowinfo(const Mats& M, int64_t a_nnz, const ClassParams& cp, int64_t* ip,
                          int64_t* minc, int64_t* maxc, int32_t* cls, DevStats* stats,
                          int32_t* heavy, hipStream_t st);
hipError_t launch_validate(const Mats& M, int64_t a_nnz, int64_t b_nnz, DevStats* stats,
                           hipStream_t st);
// Stable partition of rows by class: list (int32 row ids) and list_off[NCLS+1].
size_t classify_temp_bytes(int64_t n);
hipError_t launch_classify(const int32_t* cls, int64_t n, int32_t* list, int64_t* list_off,
                           void* temp, hipStream_t st);
// SORT rows of class c (count mode writes rownnz; numeric writes C).  With
// work (a device counter holding 0), persistent waves pull the tiles, on at
// most persistent_blocks workgroups (<= 0: as many as are resident).
hipError_t launch_sort_rows(const Mats& M, const RowSrc& src, int cls, bool numeric,
                            const int32_t* list, int64_t begin, int64_t count, const int64_t* minc,
                            int colbits, int64_t* rownnz, const int64_t* crp, DevStats* stats,
                            hipStream_t st, unsigned int* work = nullptr,
                            int persistent_blocks = 0);
// RowSrc for a single product
RowSrc single_src(const Mats& M, void* ccol, void* cval);
// DENSE rows: one workgroup per row, column range <= 2^shift.
hipError_t launch_dense_rows(const Mats& M, const RowSrc& src, bool numeric, const int32_t* list,
                             int64_t begin, int64_t count, const int64_t* minc,
                             const int64_t* maxc, int shift, int block, int64_t* rownnz,
                             const int64_t* crp, hipStream_t st, unsigned int* work = nullptr);
// --- batches of products (rows of all products concatenated) ---
// mat_of_row[r] = b for row0[b] <= r < row0[b + 1]
hipError_t launch_mat_of_row(const int64_t* row0, int64_t nmat, int64_t nrows, int32_t* mat_of_row,
                             hipStream_t st);
// setup over a batch; flags[b] is set to 1 when product b has CHUNKED rows
hipError_t launch_rowinfo_batch(const Mats& T, const RowSrc& src, int64_t nrows, int64_t a_nnz,
                                const ClassParams& cp, int64_t* ip, int64_t* minc, int64_t* maxc,
                                int32_t* cls, DevStats* stats, int32_t* flags, hipStream_t st);
// per row: ip_i and min(ip_i, columns of C) (the row's nnz bound)
hipError_t launch_row_bound(const Mats& T, const RowSrc& src, int64_t nrows, int64_t a_nnz,
                            int64_t* ip, int64_t* bound, hipStream_t st);
// rows of products whose flag is set become EMPTY (they are planned alone)
hipError_t launch_drop_flagged(const int32_t* flags, const int32_t* mat_of_row, int64_t nrows,
                               int32_t* cls, hipStream_t st);
// per-product row pointers of C from the batch's row offsets
hipError_t launch_write_rowptr_batch(const RowSrc& src, const int64_t* crp, int64_t nrows,
                                     int64_t nmat, const int32_t* flags, hipStream_t st);
size_t dense_rows_lds(int f64, int shift, int block);

// --- chunked rows (k_bins.hip) ---
struct ChunkGeom {
  // per CHUNKED row k (list order), all int64 arrays of nchunked(+1) entries
  const int32_t* rows;   // row ids (slice of the class list)
  const int64_t* ip;     // per-row ip (indexed by row id)
  const int64_t* minc;   // per-row min column (by row id)
  const int64_t* maxc;   // per-row max column (by row id)
  int64_t* nb;           // bins per row                      [nch]
  int64_t* nt;           // tiles per row                     [nch]
  int64_t* binBase;      // exclusive scan of nb              [nch+1]
  int64_t* tileBase;     // exclusive scan of nt              [nch+1]
  int64_t* ipBase;       // exclusive scan of ip              [nch+1]
  int64_t nch;
  int shift;             // chunk length 2^shift
  int tile;              // products per tile (power of two)
  int hints;             // HINT_* bits: non-temporal access classes
};
hipError_t launch_chunk_geom(const ChunkGeom& g, hipStream_t st);
// first_of[s] (int32, pre-filled with -1) and bases[3*s] for batch slots of W products
hipError_t launch_batch_bounds(const ChunkGeom& g, int64_t W, int32_t* first_of, int64_t* bases,
                               hipStream_t st);
// aoff of every A entry of the CHUNKED rows; ent[k] = A entries of row k
hipError_t launch_aoff(const Mats& M, const int32_t* rows, int64_t nrows, int64_t* aoff,
                       int64_t* ent, hipStream_t st);
// per category: sum of rownnz (before the scan) into stats->nnz_cat
hipError_t launch_cat_nnz(const int32_t* cls, const int64_t* rownnz, int64_t n, DevStats* stats,
                          hipStream_t st);
// out[k] = v[rows[k]]
hipError_t launch_gather_rows(const int64_t* v, const int32_t* rows, int64_t nrows, int64_t* out,
                              hipStream_t st);
hipError_t launch_stream_copy(void* dst, const void* src, size_t bytes, hipStream_t st);
hipError_t launch_tiles(const int64_t* nt, const int64_t* tileBase, int64_t k0, int64_t k1,
                        int32_t* tile_row, hipStream_t st);

struct BatchArgs {
  int64_t k0, k1;          // CHUNKED list range of the batch
  int64_t tile0, ntiles;   // global tile range
  int64_t bin0, nbins;     // global bin range
  int64_t ip0, nip;        // global product range (batch workspace offset = ip - ip0)
  int64_t nent, nnz_out;   // A entries of the batch's rows; nnz of C they produce
  int64_t n_sort = -1;     // its sort items, once read back to the host (-1: not known)
};
// per-chunk product totals of a batch (bin_cnt zeroed before), and each
// chunk's row
hipError_t launch_bin_hist(const Mats& M, const ChunkGeom& g, const BatchArgs& b,
                            const int32_t* tile_row, const int64_t* aoff, const int64_t* tile_e0,
                            int64_t* bin_cnt, int32_t* bin_row, int64_t max_nb, hipStream_t st);
hipError_t launch_bin_accum(const ChunkGeom& g, const BatchArgs& b, bool numeric, int f64,
                            const int64_t* bin_start, const int64_t* bin_cnt,
                            const int32_t* bin_row, const int64_t* dense_items,
                            const int64_t* sort_items, const int32_t* item_counts,
                            const uint16_t* ws_col, const void* ws_val, int64_t* bin_nnz,
                            const int64_t* bin_out, void* ccol, int col64, void* cval,
                            int dense_block, unsigned int* work, int persistent_wgs, bool det,
                            hipStream_t st);
// deterministic mode (CHUNKED rows): the order-preserving reorder.  A row's
// tiles form segments of S tiles; launch_det_nseg gives each row its segment
// count and table size (segments x chunks), launch_det_seg_hist fills the
// table [row][chunk][segment] with each segment's products per chunk (plan
// time, structure only), and after an exclusive scan of the table
// launch_bin_scatter_det reorders segments [sg0, sg0 + nsegs) of a batch,
// one workgroup each (bin_scatter_det_lds bytes): every chunk's run lists
// its products in the order of Eq. 1.  With det, launch_bin_accum sums each
// column's products in that order.
hipError_t launch_det_nseg(const ChunkGeom& g, int S, int64_t* nseg, int64_t* ntab,
                           hipStream_t st);
size_t det_seg_hist_lds(int64_t max_nb);
hipError_t launch_det_seg_hist(const Mats& M, const ChunkGeom& g, const int64_t* aoff,
                               const int64_t* tile_e0, const int32_t* seg_row,
                               const int64_t* segBase, const int64_t* tabBase, int S,
                               int64_t nsegs, int64_t max_nb, int64_t* tab, hipStream_t st);
size_t bin_scatter_det_lds(int f64, int tile, int64_t max_nb);
hipError_t launch_bin_scatter_det(const Mats& M, const ChunkGeom& g, const int64_t* aoff,
                                  const int64_t* tile_e0, const int32_t* seg_row,
                                  const int64_t* segBase, const int64_t* tabBase,
                                  const int64_t* tabS, int S, int64_t sg0, int64_t nsegs,
                                  const int64_t* bin_start, uint16_t* ws_col, void* ws_val,
                                  int64_t max_nb, hipStream_t st);
size_t bin_dense_lds(int f64, int shift);
// symbolic phase of CHUNKED rows with the row's bitmap in LDS (needs
// row_bitmap_lds bytes); writes chunk nnz, chunk product counts, chunk row
// and row nnz
size_t row_bitmap_lds(int shift, int64_t max_nb);
hipError_t launch_row_bitmap(const Mats& M, const ChunkGeom& g, const int64_t* aoff,
                             int64_t max_nb, int64_t* bin_nnz, int64_t* bin_cnt, int32_t* bin_row,
                             int64_t* rownnz, hipStream_t st);
// reorder with chunk ranges reserved by atomic adds on bin cursors (count
// mode: columns only); ws_col holds uint16 (lc32 = 0) or uint32 (lc32 = 1)
// chunk-local columns; sorted = 1 writes each tile out in chunk order
// (an index permutation in LDS).  block: the workgroup size of the sorted
// 32-bit form (256, 512 or 1024; 0 for the default), BIN_BS otherwise
size_t bin_scatter2_lds(int f64, int tile, int64_t max_nb, int lc32, int sorted, int block);
hipError_t launch_bin_scatter2(const Mats& M, const ChunkGeom& g, const BatchArgs& b, bool numeric,
                               int lc32, int sorted, int block, const int32_t* tile_row,
                               const int64_t* aoff,
                               const int64_t* tile_e0, const int64_t* bin_start,
                               unsigned long long* bin_cursor, void* ws_col, void* ws_val,
                               int64_t max_nb, hipStream_t st);
// --- coarse level: coarse chunks as virtual rows of a second geometry ---
// per coarse chunk (global index over the coarse rows' chunks): column base,
// last column, fine chunk count
hipError_t launch_vrow_geom(const ChunkGeom& g1, int fshift, int64_t* minc2, int64_t* maxc2,
                            int64_t* nb2, hipStream_t st);
// fine-chunk product counts of the level-2 tiles of b2 (cnt2 zeroed before)
hipError_t launch_l2_hist(const ChunkGeom& g2, const BatchArgs& b2, const int32_t* tile_row2,
                          const int64_t* start1, const uint32_t* ws1_col, int64_t* cnt2,
                          int64_t max_nb2, hipStream_t st);
// row2[fine chunk] = its virtual row
hipError_t launch_vrow_rows(const ChunkGeom& g2, int32_t* row2, hipStream_t st);
// g2.nt[k] = ceil(products / g2.tile) of listed virtual rows k in [k0, k1)
hipError_t launch_vrow_tiles(const ChunkGeom& g2, int64_t k0, int64_t k1, hipStream_t st);
// the coarse chunks [k0, k0 + n) split into those with more than SORT_CAP
// products (big, ascending) and the others (small, ascending); *nbig
// (device) receives the big count; flags, pos: n entries of scratch
hipError_t launch_vrow_split(const int64_t* cnt1, int64_t k0, int64_t n, int64_t* flags,
                             int64_t* pos, int64_t* nbig, void* scan_temp, int32_t* big,
                             int32_t* small, hipStream_t st);
// nb[k] = vnb[rows[k]], cnt[k] = cnt1[rows[k]]
hipError_t launch_vrow_gather(const int32_t* rows, int64_t n, const int64_t* vnb,
                              const int64_t* cnt1, int64_t* nb, int64_t* cnt, hipStream_t st);
// small coarse chunks sorted from the first workspace: nnz1 (count mode) or
// C at out1 (numeric); columns = minc2 + local column
hipError_t launch_vrow_sort(bool numeric, int f64, const int32_t* small, int64_t nsmall,
                            const int64_t* cnt1, const int64_t* start1, const int64_t* minc2,
                            const uint32_t* ws1_col, const void* ws1_val, int64_t* nnz1,
                            const int64_t* out1, void* ccol, int col64, void* cval,
                            hipStream_t st);
// symbolic phase of virtual rows [k0, k1): fine chunk products, nnz, row;
// virtual row nnz
size_t vrow_bitmap_lds(int cshift, int64_t max_nb2);
hipError_t launch_vrow_bitmap(const ChunkGeom& g2, int cshift, int64_t k0, int64_t k1,
                              int64_t max_nb2, const int64_t* start1, const uint32_t* ws1_col,
                              int64_t* bin_cnt2, int64_t* bin_nnz2, int32_t* bin_row2,
                              int64_t* vnnz, hipStream_t st);
// level-2 reorder of the tiles of b2 (first workspace -> second; count
// mode: columns only); block: 256 or 1024 threads per tile (0: 1024)
size_t l2_scatter_lds(int f64, int tile, int64_t max_nb2);
hipError_t launch_l2_scatter(const ChunkGeom& g2, const BatchArgs& b2, bool numeric, int f64,
                             const int32_t* tile_row2, const int64_t* start1,
                             const uint32_t* ws1_col, const void* ws1_val,
                             const int64_t* bin_start2, unsigned long long* bin_cursor2,
                             uint16_t* ws2_col, void* ws2_val, int64_t max_nb2, int block,
                             hipStream_t st);
// first A entry of every tile
hipError_t launch_tile_e0(const Mats& M, const ChunkGeom& g, const int32_t* tile_row,
                          const int64_t* aoff, int64_t ntiles, int64_t* tile_e0, hipStream_t st);
hipError_t launch_bin_group(const ChunkGeom& g, const BatchArgs& b, const int64_t* bin_cnt,
                            int64_t dense_min, int64_t group_max, int64_t* dense_items,
                            int64_t* sort_items, int32_t* item_counts, hipStream_t st);
// per CHUNKED row: rownnz = sum of its bins' nnz (count mode) / bin output
// offsets from crp (numeric prep)
hipError_t launch_bin_rows(const ChunkGeom& g, int64_t k0, int64_t k1, const int64_t* bin_nnz,
                           int64_t* rownnz, const int64_t* crp, int64_t* bin_out, bool to_out,
                           hipStream_t st);

// --- CHUNKED rows binned by runs (k_runs.hip) ---
// Chunk index of B (chunks of 2^shift columns): count pass (fill = false)
// writes cnt[j] = runs of row j + 1; after an exclusive scan into ptr
// (nrows + 1 entries), the fill pass writes pos (run starts, then the row's
// end) and chunk (each run's column >> shift).  Needs nnz(B) < 2^32.
hipError_t launch_bci(const Mats& M, int shift, bool fill, int64_t* cnt, const int64_t* ptr,
                      uint32_t* pos, uint32_t* chunk, hipStream_t st);
// out[0] += runs of the listed rows; out[1] = max(out[1], A entries of a
// row); out[2] += their products (ip, by row id)
hipError_t launch_run_count(const Mats& M, const int32_t* rows, int64_t nrows, const int64_t* bptr,
                            const int64_t* ip, unsigned long long* out, hipStream_t st);
// One run of a chunk, 16 bytes written and read whole: the product offset
// of its first product (64 bits, low word first), its start in B's column
// array and its A entry.  One record instead of three arrays halves the
// partly written cache lines of the scatter, whose runs of one chunk land
// a few at a time.
typedef uint32_t run_t __attribute__((ext_vector_type(4)));
// hist: runs and products per chunk (bin_seg, bin_cnt) and each chunk's row;
// otherwise the runs' scatter: every run's record, the runs of chunk b at
// [seg_beg[b], seg_beg[b + 1])
size_t run_rows_lds(int64_t max_nb);
hipError_t launch_run_rows(const Mats& M, const ChunkGeom& g, bool hist, const int64_t* bptr,
                           const uint32_t* bpos, const uint32_t* bchunk, int64_t max_nb,
                           int64_t* bin_seg, int64_t* bin_cnt, int32_t* bin_row,
                           const int64_t* seg_beg, const int64_t* bin_start, run_t* runs,
                           hipStream_t st);
// Dense items are dealt to the XCDs by column chunk: chunk index c goes to
// XCD c % N_XCD, and each XCD's items are ordered by c, so the workgroups of
// one XCD (ids congruent mod N_XCD: the dispatcher deals workgroups to the
// XCDs round-robin) work on the same few column chunks at a time and find
// those chunks' B entries in their L2.  key = (c % N_XCD) * cpx + c / N_XCD
// with cpx = ceil(column chunks / N_XCD); xcd_start (N_XCD * cpx + 1
// entries) receives the exclusive scan of the keys' counts, xcd_cur a copy
// (the records' cursors).  temp: scan_temp_bytes(N_XCD * cpx + 1).
constexpr int N_XCD = 8;
// (nitems: a bound on the dense items, the launches' size)
hipError_t launch_dense_order(const ChunkGeom& g, int64_t nitems, const int64_t* dense_items,
                              const int32_t* item_counts, const int32_t* bin_row, int64_t cpx,
                              int64_t* xcd_start, int64_t* xcd_cur, void* temp, hipStream_t st);
// the dense items' records (6 int64 each: product start, run start,
// products, runs, first column, chunk), built once after the grouping, each
// at its place in the XCD order (xcd_cur advanced)
hipError_t launch_run_records(const ChunkGeom& g, int64_t nitems, const int64_t* dense_items,
                              const int32_t* item_counts, const int64_t* bin_start,
                              const int64_t* bin_cnt, const int32_t* bin_row,
                              const int64_t* seg_beg, int64_t cpx, int64_t* xcd_cur,
                              int64_t* rec, hipStream_t st);
// the accumulators over chunks whose products are read through their runs
// (count mode: bin_nnz; numeric: C at bin_out).  The dense items' workgroups
// have dense_block threads in numeric mode and RUN_COUNT_BLOCK in count
// mode, whose LDS (the bitmap and the run window) allows eight per CU:
// persistent_wgs is the grid of the mode launched.
constexpr int RUN_COUNT_BLOCK = 256;
size_t run_dense_lds(int f64, int shift, int block);
hipError_t launch_run_accum(const Mats& M, const ChunkGeom& g, int64_t nbins, bool numeric,
                            const int64_t* bin_start, const int64_t* bin_cnt,
                            const int32_t* bin_row, const int64_t* dense_rec,
                            const int64_t* sort_items, const int32_t* item_counts,
                            const int64_t* seg_beg, const run_t* runs, int64_t* bin_nnz,
                            const int64_t* bin_out,
                            void* ccol, int col64, void* cval, int dense_block,
                            unsigned int* work, int persistent_wgs, uint32_t* chunk_bm,
                            int64_t n_sort_items, const int64_t* xcd_start, int64_t cpx,
                            hipStream_t st);

// --- misc (k_rows.hip) ---
hipError_t launch_fill_i64(int64_t* p, int64_t n, int64_t v, hipStream_t st);
hipError_t launch_write_rowptr(const int64_t* crp, int64_t n, void* out, int out64,
                               hipStream_t st);

}  // namespace mg
