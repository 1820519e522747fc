// Building blocks on one stream of intermediate products (the reordering and
// accumulation microbenchmarks of Section 4.1): the stream is one virtual
// row with columns [0, m); the level-2 reorder and the chunk accumulators
// of CHUNKED rows run on it, each stage timed with events.
#include "runtime_int.h"

using namespace mgrt;

extern "C" magnus_status_t magnus_stream_chunks(magnus_handle_t h, const uint32_t* cols,
                                                const void* vals, int32_t val_type, int64_t n,
                                                int64_t m, int32_t chunk_shift, int32_t dense_min,
                                                int32_t* out_cols, void* out_vals, int64_t* nnz,
                                                void* stream, magnus_stream_times_t* times) {
  if (!h || !nnz || n < 0 || m <= 0 || m >= ((int64_t)1 << 31) || chunk_shift < 1 ||
      chunk_shift > 16 || dense_min < 0 || dense_min > SORT_CAP + 1 ||
      (val_type != MAGNUS_F32 && val_type != MAGNUS_F64) ||
      (n > 0 && (!cols || !vals || !out_cols || !out_vals)))
    return MAGNUS_ERR_INVALID_ARG;
  const int f64 = val_type == MAGNUS_F64;
  const int64_t nb = ((m - 1) >> chunk_shift) + 1;
  if (nb > 8191 || bin_dense_lds(f64, chunk_shift) > (size_t)h->lds_max) {
    h->err = "too many chunks, or a chunk accumulator larger than the LDS";
    return MAGNUS_ERR_INVALID_ARG;
  }
  int tile = 2048;
  while (tile > 256 && l2_scatter_lds(f64, tile, nb) > (size_t)h->lds_max) tile /= 2;
  if (l2_scatter_lds(f64, tile, nb) > (size_t)h->lds_max) return MAGNUS_ERR_INVALID_ARG;
  HIPCHK(hipSetDevice(h->device));
  *nnz = 0;
  if (times) *times = magnus_stream_times_t{};
  if (n == 0) return MAGNUS_OK;

  magnus_plan_s tmp;
  tmp.h = h;
  tmp.st = (hipStream_t)stream;
  const int64_t nt = (n + tile - 1) / tile;
  const size_t vs = f64 ? 8 : 4;
  // geometry of the one virtual row: ip, minc, maxc, nb, nt, binBase[2],
  // tileBase[2], product start
  int64_t* geo = (int64_t*)palloc(&tmp, sizeof(int64_t) * 10);
  int32_t* rows = (int32_t*)palloc(&tmp, 64);
  int64_t* tile_row8 = (int64_t*)palloc(&tmp, sizeof(int64_t) * ((nt + 1) / 2 + 1));
  int64_t* cnt = (int64_t*)palloc(&tmp, sizeof(int64_t) * nb);
  int64_t* start = (int64_t*)palloc(&tmp, sizeof(int64_t) * nb);
  int64_t* cnz = (int64_t*)palloc(&tmp, sizeof(int64_t) * nb);
  int64_t* out = (int64_t*)palloc(&tmp, sizeof(int64_t) * (nb + 1));
  int64_t* row8 = (int64_t*)palloc(&tmp, sizeof(int64_t) * ((nb + 1) / 2 + 1));
  int64_t* dense_items = (int64_t*)palloc(&tmp, sizeof(int64_t) * nb);
  int64_t* sort_items = (int64_t*)palloc(&tmp, sizeof(int64_t) * 2 * nb);
  unsigned long long* cursor = (unsigned long long*)palloc(&tmp, sizeof(int64_t) * nb);
  int64_t* counters = (int64_t*)palloc(&tmp, sizeof(int64_t) * 4);  // item counts, work x2
  uint16_t* ws_col = (uint16_t*)palloc(&tmp, sizeof(uint16_t) * n);
  void* ws_val = palloc(&tmp, vs * n);
  void* stmp = palloc(&tmp, scan_temp_bytes(nb + 1));
  if (!geo || !rows || !tile_row8 || !cnt || !start || !cnz || !out || !row8 || !dense_items ||
      !sort_items || !cursor || !counters || !ws_col || !ws_val || !stmp) {
    plan_free_all(&tmp);
    return MAGNUS_ERR_OOM;
  }
  const int64_t h_geo[10] = {n, 0, m - 1, nb, nt, 0, nb, 0, nt, 0};
  ChunkGeom g{};
  g.rows = rows;
  g.ip = geo;
  g.minc = geo + 1;
  g.maxc = geo + 2;
  g.nb = geo + 3;
  g.nt = geo + 4;
  g.binBase = geo + 5;
  g.tileBase = geo + 7;
  g.ipBase = nullptr;
  g.nch = 1;
  g.shift = chunk_shift;
  g.tile = tile;
  g.hints = 0;
  BatchArgs b{};
  b.k0 = 0;
  b.k1 = 1;
  b.tile0 = 0;
  b.ntiles = nt;
  b.bin0 = 0;
  b.nbins = nb;
  b.nip = n;
  const int32_t* tile_row = (const int32_t*)tile_row8;  // every tile belongs to row 0
  int32_t* bin_row = (int32_t*)row8;
  int32_t* item_counts = (int32_t*)counters;
  unsigned int* work = (unsigned int*)(counters + 1);
  const int64_t dmin = dense_min > 0 ? dense_min : SORT_CAP;
  const size_t dl = bin_dense_lds(f64, chunk_shift);
  const int per_cu = std::max<int>(1, (int)(h->lds_max / std::max<size_t>(dl, 1)));
  const int pwgs = std::max(1, h->cus) * std::min(per_cu, 2048 / 256);

  hipEvent_t ev[7];
  for (auto& e : ev) e = nullptr;
  magnus_status_t r = MAGNUS_OK;
  hipError_t e = hipSuccess;
  for (int i = 0; i < 7 && e == hipSuccess; ++i) e = hipEventCreate(&ev[i]);
#define SB(expr)                                 \
  do {                                           \
    if (e == hipSuccess) e = (expr);             \
  } while (0)
  SB(hipMemcpyAsync(geo, h_geo, sizeof(h_geo), hipMemcpyHostToDevice, tmp.st));
  SB(launch_fill_i64((int64_t*)rows, 1, 0, tmp.st));
  SB(launch_fill_i64(tile_row8, (nt + 1) / 2 + 1, 0, tmp.st));
  SB(launch_fill_i64(row8, (nb + 1) / 2 + 1, 0, tmp.st));
  SB(launch_fill_i64(counters, 4, 0, tmp.st));
  SB(hipEventRecord(ev[0], tmp.st));
  // histogram of the products per chunk
  SB(launch_fill_i64(cnt, nb, 0, tmp.st));
  SB(launch_l2_hist(g, b, tile_row, geo + 9, cols, cnt, nb, tmp.st));
  SB(hipEventRecord(ev[1], tmp.st));
  // prefix sum: each chunk's start in the workspace
  SB(scan_excl_i64(cnt, start, nb, nullptr, nullptr, stmp, tmp.st));
  SB(hipEventRecord(ev[2], tmp.st));
  // reorder
  SB(launch_fill_i64((int64_t*)cursor, nb, 0, tmp.st));
  SB(launch_l2_scatter(g, b, true, f64, tile_row, geo + 9, cols, vals, start, cursor, ws_col,
                       ws_val, nb, 0, tmp.st));
  SB(hipEventRecord(ev[3], tmp.st));
  // chunks to work items: dense chunks, packed sorts of small ones
  SB(launch_bin_group(g, b, cnt, dmin, SORT_CAP, dense_items, sort_items, item_counts, tmp.st));
  SB(hipEventRecord(ev[4], tmp.st));
  // distinct columns per chunk, and the output offsets
  SB(launch_bin_accum(g, b, false, f64, start, cnt, bin_row, dense_items, sort_items,
                      item_counts, ws_col, ws_val, cnz, out, nullptr, 0, nullptr, 256, work,
                      pwgs, false, tmp.st));
  SB(scan_excl_i64(cnz, out, nb, out + nb, nullptr, stmp, tmp.st));
  SB(hipEventRecord(ev[5], tmp.st));
  // sums into the output
  SB(launch_bin_accum(g, b, true, f64, start, cnt, bin_row, dense_items, sort_items,
                      item_counts, ws_col, ws_val, cnz, out, out_cols, 0, out_vals, 256, work + 1,
                      pwgs, false, tmp.st));
  SB(hipEventRecord(ev[6], tmp.st));
#undef SB
  if (e != hipSuccess) r = fail_hip(h, e, "magnus_stream_chunks");
  int32_t ic[2] = {0, 0};
  if (r == MAGNUS_OK) r = readback(&tmp, {{out + nb, 8}, {item_counts, 8}}, {nnz, ic});
  if (r == MAGNUS_OK && times) {
    float t[6] = {0, 0, 0, 0, 0, 0};
    for (int i = 0; i < 6; ++i) (void)hipEventElapsedTime(&t[i], ev[i], ev[i + 1]);
    times->histogram_ms = t[0];
    times->scan_ms = t[1];
    times->reorder_ms = t[2];
    times->group_ms = t[3];
    times->count_ms = t[4];
    times->accumulate_ms = t[5];
    times->chunks = nb;
    times->dense_chunks = ic[0];
    times->sort_groups = ic[1];
  }
  (void)hipStreamSynchronize(tmp.st);
  for (auto& x : ev)
    if (x) (void)hipEventDestroy(x);
  plan_free_all(&tmp);
  return r;
}
