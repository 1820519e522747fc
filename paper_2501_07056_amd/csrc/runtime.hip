// Host runtime and C ABI: plans the setup and precise symbolic phases, then
// runs the numeric phase into caller-owned C (see include/magnus.h).
#include "runtime_int.h"

using namespace mgrt;

namespace {

// Products per row batch: the batch_products option, else the workspace cap
// (max_workspace_bytes, else an eighth of the device memory, the same batches
// on every call whatever the caching allocator holds) over the workspace
// bytes per product; a batch always holds the longest row.
magnus_status_t batch_width(magnus_plan_s* P, int64_t bytes_per_product, int64_t& W) {
  magnus_handle_s* h = P->h;
  const magnus_options_t& o = h->opts;
  W = o.batch_products;
  if (W <= 0) {
    int64_t budget = o.max_workspace_bytes;
    if (budget <= 0) {
      size_t fr = 0, tot = 0;
      HIPCHK(hipMemGetInfo(&fr, &tot));
      budget = (int64_t)(tot / 8);
    }
    W = budget / bytes_per_product;
  }
  // a retry after the allocator failed asks for batches half as wide each time
  W /= std::max<int64_t>(1, P->ws_div);
  if (W <= (int64_t)P->h_stats.max_ip) P->w_at_min = true;
  if (W < (int64_t)P->h_stats.max_ip) W = (int64_t)P->h_stats.max_ip;
  if (W < 1) W = 1;
  return MAGNUS_OK;
}

// Geometry of the rows of g (g.rows, g.ip, g.minc, g.maxc, g.nch, g.shift,
// g.tile set): chunks, tiles and products per row and their exclusive scans,
// then the row batches of at most W products each (whole rows).  tots =
// products, tiles, chunks over all rows.
magnus_status_t geometry_and_batches(magnus_plan_s* P, ChunkGeom& g, int64_t W,
                                     std::vector<BatchArgs>& batches, int64_t& ws_products,
                                     int64_t tots[3]) {
  magnus_handle_s* h = P->h;
  const int64_t nch = g.nch;
  int64_t* geo = (int64_t*)palloc(P, sizeof(int64_t) * (2 * nch + 3 * (nch + 1)));
  if (!geo) return MAGNUS_ERR_OOM;
  g.nb = geo;
  g.nt = geo + nch;
  g.binBase = geo + 2 * nch;
  g.tileBase = g.binBase + (nch + 1);
  g.ipBase = g.tileBase + (nch + 1);
  void* tmp = P->temp;  // sized for a scan of n + 1 >= nch + 1 entries
  HIPCHK(launch_chunk_geom(g, P->st));
  HIPCHK(scan_excl_i64(g.nb, g.binBase, nch, g.binBase + nch, nullptr, tmp, P->st));
  HIPCHK(scan_excl_i64(g.nt, g.tileBase, nch, g.tileBase + nch, nullptr, tmp, P->st));
  HIPCHK(scan_excl_i64(g.ipBase, g.ipBase, nch, g.ipBase + nch, nullptr, tmp, P->st));
  const int64_t ipch = (int64_t)P->h_stats.ip_cat[2];
  const int64_t nslots = ipch / W + 1;
  int32_t* first_of = (int32_t*)palloc(P, sizeof(int32_t) * nslots);
  int64_t* bases = (int64_t*)palloc(P, sizeof(int64_t) * 3 * nslots);
  if (!first_of || !bases) return MAGNUS_ERR_OOM;
  HIPCHK(hipMemsetAsync(first_of, 0xFF, sizeof(int32_t) * nslots, P->st));
  HIPCHK(launch_batch_bounds(g, W, first_of, bases, P->st));
  std::vector<int32_t> h_first(nslots);
  std::vector<int64_t> h_bases(3 * nslots);
  magnus_status_t s = readback(
      P,
      {{first_of, sizeof(int32_t) * nslots},
       {bases, sizeof(int64_t) * 3 * nslots},
       {g.ipBase + nch, 8},
       {g.tileBase + nch, 8},
       {g.binBase + nch, 8}},
      {h_first.data(), h_bases.data(), &tots[0], &tots[1], &tots[2]});
  if (s != MAGNUS_OK) return s;
  // batches in slot order
  std::vector<int64_t> starts;
  for (int64_t q = 0; q < nslots; ++q)
    if (h_first[q] >= 0) starts.push_back(q);
  batches.clear();
  ws_products = 0;
  int64_t max_tiles = 0;
  for (size_t b = 0; b < starts.size(); ++b) {
    const int64_t q = starts[b];
    BatchArgs ba{};
    ba.k0 = h_first[q];
    ba.ip0 = h_bases[3 * q + 0];
    ba.tile0 = h_bases[3 * q + 1];
    ba.bin0 = h_bases[3 * q + 2];
    if (b + 1 < starts.size()) {
      const int64_t q2 = starts[b + 1];
      ba.k1 = h_first[q2];
      ba.nip = h_bases[3 * q2 + 0] - ba.ip0;
      ba.ntiles = h_bases[3 * q2 + 1] - ba.tile0;
      ba.nbins = h_bases[3 * q2 + 2] - ba.bin0;
    } else {
      ba.k1 = nch;
      ba.nip = tots[0] - ba.ip0;
      ba.ntiles = tots[1] - ba.tile0;
      ba.nbins = tots[2] - ba.bin0;
    }
    ws_products = std::max(ws_products, ba.nip);
    max_tiles = std::max(max_tiles, ba.ntiles);
    batches.push_back(ba);
  }
  if (max_tiles > INT32_MAX) return MAGNUS_ERR_INDEX_OVERFLOW;
  return MAGNUS_OK;
}

// Deterministic mode: segments of S tiles per CHUNKED row and, per segment,
// the products its earlier segments put into each chunk of the row (count
// table [row][chunk][segment] and its exclusive scan).  S doubles from 16
// until the table (16 bytes an entry with its scan) stays within a quarter
// of the workspace cap.
magnus_status_t det_setup(magnus_plan_s* P, int64_t ntiles, int64_t nbins) {
  magnus_handle_s* h = P->h;
  const ChunkGeom& g = P->g;
  const int64_t nch = P->nch;
  int64_t cap = h->opts.max_workspace_bytes;
  if (cap <= 0) {
    size_t fr = 0, tot = 0;
    HIPCHK(hipMemGetInfo(&fr, &tot));
    cap = (int64_t)(tot / 8);
  }
  const int64_t cap_entries = std::max<int64_t>((int64_t)1 << 20, cap / 4 / 16);
  int S = 16;
  while ((int64_t)S * P->tile < ((int64_t)1 << 30) && P->max_nb * (ntiles / S + 1) + nbins > cap_entries)
    S *= 2;
  P->det_S = S;
  int64_t* nseg = (int64_t*)palloc(P, sizeof(int64_t) * 2 * (nch + 1));
  P->det_segBase = (int64_t*)palloc(P, sizeof(int64_t) * (nch + 1));
  P->det_tabBase = (int64_t*)palloc(P, sizeof(int64_t) * (nch + 1));
  if (!nseg || !P->det_segBase || !P->det_tabBase) return MAGNUS_ERR_OOM;
  int64_t* ntab = nseg + nch + 1;
  HIPCHK(launch_det_nseg(g, S, nseg, ntab, P->st));
  HIPCHK(scan_excl_i64(nseg, P->det_segBase, nch, P->det_segBase + nch, nullptr, P->temp, P->st));
  HIPCHK(scan_excl_i64(ntab, P->det_tabBase, nch, P->det_tabBase + nch, nullptr, P->temp, P->st));
  P->h_det_segBase.assign(nch + 1, 0);
  int64_t tt = 0;
  magnus_status_t s = readback(P, {{P->det_segBase, sizeof(int64_t) * (nch + 1)},
                                   {P->det_tabBase + nch, sizeof(int64_t)}},
                               {P->h_det_segBase.data(), &tt});
  if (s != MAGNUS_OK) return s;
  const int64_t nsegs = P->h_det_segBase[nch];
  P->det_seg_row = (int32_t*)palloc(P, sizeof(int32_t) * std::max<int64_t>(1, nsegs));
  int64_t* tab = (int64_t*)palloc(P, sizeof(int64_t) * std::max<int64_t>(1, tt));
  P->det_tabS = (int64_t*)palloc(P, sizeof(int64_t) * std::max<int64_t>(1, tt));
  void* stmp = palloc(P, scan_temp_bytes(std::max<int64_t>(1, tt)));
  if (!P->det_seg_row || !tab || !P->det_tabS || !stmp) return MAGNUS_ERR_OOM;
  HIPCHK(launch_tiles(nseg, P->det_segBase, 0, nch, P->det_seg_row, P->st));
  {
    // per product: B column; per table entry: one count written
    ProfScope ps(h, P->st, "det_counts (symbolic, segment chunks)",
                 (double)P->h_stats.ip_cat[2] * P->s_col + (double)tt * 8);
    HIPCHK(launch_det_seg_hist(P->M, g, P->aoff, P->tile_e0, P->det_seg_row, P->det_segBase,
                               P->det_tabBase, S, nsegs, P->max_nb, tab, P->st));
  }
  HIPCHK(scan_excl_i64(tab, P->det_tabS, tt, nullptr, nullptr, stmp, P->st));
  return MAGNUS_OK;
}

// Run binning of the CHUNKED rows (k_runs.hip), when options.chunk_runs
// allows it: B's chunk index, then the rows' run total; the rows are binned
// by runs when they hold at least RUN_MIN_LEN products per run (or the option
// forces it) and the run lists fit the workspace cap.  *chosen reports
// whether the plan goes this way; the arrays of the chunk geometry are then
// set up for one batch of all CHUNKED rows.
constexpr int64_t RUN_MIN_LEN = 8;

magnus_status_t runs_setup(magnus_plan_s* P, bool& chosen) {
  magnus_handle_s* h = P->h;
  const magnus_options_t& o = h->opts;
  chosen = false;
  const int64_t kB = P->M.k;
  if (P->det || o.chunk_runs < 0 || P->b_nnz >= ((int64_t)1 << 32) - 1 ||
      P->a_nnz >= ((int64_t)1 << 32) || P->h_stats.max_ip >= ((unsigned long long)1 << 31) ||
      run_rows_lds(P->max_nb) > (size_t)P->lds_budget ||
      run_dense_lds(P->M.f64, P->shift, P->dense_block) > (size_t)h->lds_max)
    return MAGNUS_OK;
  // B's chunk index: runs per row (+1), their scan, then starts and chunks
  P->bci_ptr = (int64_t*)palloc(P, sizeof(int64_t) * (kB + 1));
  void* btmp = palloc(P, scan_temp_bytes(kB + 1) + 64);
  unsigned long long* cnt = (unsigned long long*)palloc(P, 64);  // runs, max entries, products
  if (!P->bci_ptr || !btmp || !cnt) return MAGNUS_ERR_OOM;
  HIPCHK(launch_bci(P->M, P->shift, false, P->bci_ptr, nullptr, nullptr, nullptr, P->st));
  HIPCHK(scan_excl_i64(P->bci_ptr, P->bci_ptr, kB, P->bci_ptr + kB, nullptr, btmp, P->st));
  HIPCHK(hipMemsetAsync(cnt, 0, 24, P->st));
  HIPCHK(launch_run_count(P->M, P->list + P->h_list_off[CLS_CHUNKED], P->nch, P->bci_ptr, P->ip,
                          cnt, P->st));
  int64_t nbci = 0;
  unsigned long long hc[3] = {0, 0, 0};
  magnus_status_t s = readback(P, {{P->bci_ptr + kB, 8}, {cnt, 24}}, {&nbci, hc});
  if (s != MAGNUS_OK) return s;
  const int64_t runs = (int64_t)hc[0];
  // products of the rows listed as CHUNKED (coarse-level rows excluded)
  const int64_t ipch = (int64_t)hc[2];
  int64_t cap = o.max_workspace_bytes;
  if (cap <= 0) {
    size_t fr = 0, tot = 0;
    HIPCHK(hipMemGetInfo(&fr, &tot));
    cap = (int64_t)(tot / 8);
  }
  cap /= std::max<int64_t>(1, P->ws_div);
  const bool fits = runs * 16 <= cap && hc[1] < ((unsigned long long)1 << 24);
  const bool want = o.chunk_runs > 0 || (runs > 0 && ipch >= RUN_MIN_LEN * runs);
  if (!fits || !want) return MAGNUS_OK;
  P->bci_pos = (uint32_t*)palloc(P, sizeof(uint32_t) * std::max<int64_t>(1, nbci));
  P->bci_chunk = (uint32_t*)palloc(P, sizeof(uint32_t) * std::max<int64_t>(1, nbci));
  if (!P->bci_pos || !P->bci_chunk) return MAGNUS_ERR_OOM;
  HIPCHK(launch_bci(P->M, P->shift, true, nullptr, P->bci_ptr, P->bci_pos, P->bci_chunk, P->st));
  P->n_runs = runs;
  chosen = true;
  P->runs = true;
  // packed sorts of up to 1024 products unless set (config 2: 301.6 -> 298.0
  // ms per step against 512; 256 is slower)
  if (o.sort_group_max <= 0) P->group_max = SORT_CAP;
  // 512-thread dense workgroups unless set (config 2: 360 -> 324 ms per step
  // against 256; 1024 is slower)
  if (o.dense_block != 256 && o.dense_block != 512 && o.dense_block != 1024) {
    P->dense_block = 512;
    const size_t dl = run_dense_lds(P->M.f64, P->shift, P->dense_block);
    const int per_cu = std::max<int>(1, (int)(h->lds_max / std::max<size_t>(dl, 1)));
    P->persistent_wgs = std::max(1, h->cus) * std::min(per_cu, 2048 / P->dense_block);
  }
  {
    // count mode: 256-thread workgroups whatever dense_block is (R-MAT scale
    // 20: run_count 62.4 -> 60.0 ms against the numeric phase's 512)
    const size_t dlc = ((size_t)1 << P->shift) / 8 + (size_t)RUN_COUNT_BLOCK * 8 + 4096;
    const int per_cu_c = std::max<int>(1, (int)(h->lds_max / dlc));
    P->persistent_wgs_count = std::max(1, h->cus) * std::min(per_cu_c, 2048 / RUN_COUNT_BLOCK);
  }

  // the chunk geometry of one batch of all CHUNKED rows
  ChunkGeom& g = P->g;
  int64_t tots[3];
  s = geometry_and_batches(P, g, INT64_MAX / 4, P->batches, P->ws_products, tots);
  if (s != MAGNUS_OK) return s;
  const int64_t nbins = tots[2], nch = P->nch;
  P->ws_products = 0;
  P->scan_temp = palloc(P, scan_temp_bytes(nbins + 1));
  // dense item counters: N_XCD for the count pass, N_XCD for the numeric one
  P->work_ctr = (unsigned int*)palloc(P, sizeof(unsigned int) * 2 * N_XCD);
  P->xcd_cpx = ((((P->M.m > 0 ? P->M.m - 1 : 0) >> P->shift) + 1) + N_XCD - 1) / N_XCD;
  P->xcd_start = (int64_t*)palloc(P, sizeof(int64_t) * (N_XCD * P->xcd_cpx + 1));
  P->xcd_cur = (int64_t*)palloc(P, sizeof(int64_t) * (N_XCD * P->xcd_cpx + 1));
  P->xcd_temp = palloc(P, scan_temp_bytes(N_XCD * P->xcd_cpx + 1));
  if (!P->xcd_start || !P->xcd_cur || !P->xcd_temp) return MAGNUS_ERR_OOM;
  P->bin_start = (int64_t*)palloc(P, sizeof(int64_t) * nbins);
  P->bin_cnt = (int64_t*)palloc(P, sizeof(int64_t) * nbins);
  P->bin_nnz = (int64_t*)palloc(P, sizeof(int64_t) * nbins);
  P->bin_out = (int64_t*)palloc(P, sizeof(int64_t) * nbins);
  P->bin_row = (int32_t*)palloc(P, sizeof(int32_t) * nbins);
  P->bin_seg = (int64_t*)palloc(P, sizeof(int64_t) * nbins);
  P->seg_beg = (int64_t*)palloc(P, sizeof(int64_t) * (nbins + 1));
  P->dense_items = (int64_t*)palloc(P, sizeof(int64_t) * nbins);
  P->sort_items = (int64_t*)palloc(P, sizeof(int64_t) * 2 * nbins);
  P->item_counts = (int32_t*)palloc(P, sizeof(int32_t) * 2);
  // dense items are the chunks of >= dense_min products: at most
  // products / dense_min of them
  P->run_rec = (int64_t*)palloc(
      P, sizeof(int64_t) * 6 * std::max<int64_t>(1, std::min(nbins, tots[0] / std::max<int64_t>(1, P->dense_min) + 1)));
  P->run_list = (run_t*)palloc(P, sizeof(run_t) * std::max<int64_t>(1, runs));
  P->ent = (int64_t*)palloc(P, sizeof(int64_t) * (4 * nch + 2));
  if (!P->aoff) P->aoff = (int64_t*)palloc(P, sizeof(int64_t) * std::max<int64_t>(1, P->a_nnz));
  if (!P->scan_temp || !P->work_ctr || !P->bin_start || !P->bin_cnt || !P->bin_nnz ||
      !P->bin_out || !P->bin_row || !P->bin_seg || !P->seg_beg || !P->dense_items ||
      !P->sort_items || !P->item_counts || !P->run_list || !P->ent ||
      !P->run_rec ||
      !P->aoff)
    return MAGNUS_ERR_OOM;
  HIPCHK(hipMemsetAsync(P->item_counts, 0, sizeof(int32_t) * 2, P->st));
  HIPCHK(hipMemsetAsync(P->bin_nnz, 0, sizeof(int64_t) * nbins, P->st));
  P->entBase = P->ent + nch;
  P->nnzr = P->entBase + nch + 1;
  P->nnzBase = P->nnzr + nch;
  // A entries per row (for the batch's profiling bytes and nnz offsets)
  HIPCHK(launch_aoff(P->M, g.rows, nch, P->aoff, P->ent, P->st));
  HIPCHK(scan_excl_i64(P->ent, P->entBase, nch, P->entBase + nch, nullptr, P->temp, P->st));
  P->info.n_batches = 1;
  P->info.n_bins = nbins;
  return MAGNUS_OK;
}

magnus_status_t setup_chunked(magnus_plan_s* P) {
  magnus_handle_s* h = P->h;
  const int64_t nch = P->nch;
  ChunkGeom& g = P->g;
  g.rows = P->list + P->h_list_off[CLS_CHUNKED];
  g.ip = P->ip;
  g.minc = P->minc;
  g.maxc = P->maxc;
  g.nch = nch;
  g.shift = P->shift;
  g.tile = P->tile;
  g.hints = P->hints;
  {
    bool chosen = false;
    magnus_status_t sr = runs_setup(P, chosen);
    if (sr != MAGNUS_OK || chosen) return sr;
  }
  void* tmp = P->temp;
  const int64_t vs = P->M.f64 ? 8 : 4;
  int64_t W = 0, tots[3];
  magnus_status_t s = batch_width(P, 2 + vs, W);
  if (s != MAGNUS_OK) return s;
  s = geometry_and_batches(P, g, W, P->batches, P->ws_products, tots);
  if (s != MAGNUS_OK) return s;
  const int64_t ntiles = tots[1], nbins = tots[2];
  const int64_t nbat = (int64_t)P->batches.size();
  P->bitmap_symbolic = row_bitmap_lds(P->shift, P->max_nb) <= (size_t)P->lds_budget;
  if (!P->aoff) P->aoff = (int64_t*)palloc(P, sizeof(int64_t) * std::max<int64_t>(1, P->a_nnz));
  P->tile_row = (int32_t*)palloc(P, sizeof(int32_t) * ntiles);
  P->scan_temp = palloc(P, scan_temp_bytes(nbins));
  if (!P->scan_temp) return MAGNUS_ERR_OOM;
  P->bin_cursor = (unsigned long long*)palloc(P, sizeof(unsigned long long) * nbins);
  P->work_ctr = (unsigned int*)palloc(P, sizeof(int64_t) * 2 * nbat);
  if (!P->work_ctr) return MAGNUS_ERR_OOM;
  P->bin_start = (int64_t*)palloc(P, sizeof(int64_t) * nbins);
  P->bin_cnt = (int64_t*)palloc(P, sizeof(int64_t) * nbins);
  P->bin_nnz = (int64_t*)palloc(P, sizeof(int64_t) * nbins);
  P->bin_out = (int64_t*)palloc(P, sizeof(int64_t) * nbins);
  P->bin_row = (int32_t*)palloc(P, sizeof(int32_t) * nbins);
  P->dense_items = (int64_t*)palloc(P, sizeof(int64_t) * nbins);
  P->sort_items = (int64_t*)palloc(P, sizeof(int64_t) * 2 * nbins);
  P->item_counts = (int32_t*)palloc(P, sizeof(int32_t) * 2 * nbat);
  P->ws_col = (uint16_t*)palloc(P, sizeof(uint16_t) * P->ws_products);
  P->ws_val = palloc(P, (size_t)vs * P->ws_products);
  if (!P->aoff || !P->tile_row || !P->bin_start || !P->bin_cnt || !P->bin_nnz || !P->bin_out ||
      !P->bin_row || !P->dense_items || !P->sort_items || !P->item_counts || !P->ws_col ||
      !P->ws_val || !P->bin_cursor)
    return MAGNUS_ERR_OOM;
  HIPCHK(hipMemsetAsync(P->item_counts, 0, sizeof(int32_t) * 2 * nbat, P->st));
  HIPCHK(hipMemsetAsync(P->bin_nnz, 0, sizeof(int64_t) * nbins, P->st));
  P->ent = (int64_t*)palloc(P, sizeof(int64_t) * (4 * nch + 2));
  if (!P->ent) return MAGNUS_ERR_OOM;
  P->entBase = P->ent + nch;
  P->nnzr = P->entBase + nch + 1;
  P->nnzBase = P->nnzr + nch;
  HIPCHK(launch_aoff(P->M, g.rows, nch, P->aoff, P->ent, P->st));
  HIPCHK(scan_excl_i64(P->ent, P->entBase, nch, P->entBase + nch, nullptr, tmp, P->st));
  HIPCHK(launch_tiles(g.nt, g.tileBase, 0, nch, P->tile_row, P->st));
  P->tile_e0 = (int64_t*)palloc(P, sizeof(int64_t) * std::max<int64_t>(1, ntiles));
  if (!P->tile_e0) return MAGNUS_ERR_OOM;
  HIPCHK(launch_tile_e0(P->M, g, P->tile_row, P->aoff, ntiles, P->tile_e0, P->st));
  if (P->det) {
    magnus_status_t sd = det_setup(P, ntiles, nbins);
    if (sd != MAGNUS_OK) return sd;
  }
  P->info.n_batches = nbat;
  P->info.n_bins = nbins;
  return MAGNUS_OK;
}

// Symbolic phase of CHUNKED rows: exact nnz per chunk and per row, chunk
// sizes and starts, and the accumulation work items of every batch.
magnus_status_t chunked_symbolic(magnus_plan_s* P) {
  magnus_handle_s* h = P->h;
  if (P->runs) {
    // runs per chunk and products per chunk, their scans, the runs'
    // scatter, the accumulation items, then the accumulators in count mode
    const BatchArgs& b = P->batches[0];
    const int64_t nbins = b.nbins;
    {
      const double ent = (double)P->h_stats.ent_cat[2];
      ProfScope ps(h, P->st, "run_bin (symbolic, runs per chunk)",
                   2.0 * (ent * (P->s_col + 16) + (double)P->n_runs * 8) +
                       (double)P->n_runs * 16 + (double)nbins * 36);
      HIPCHK(launch_run_rows(P->M, P->g, true, P->bci_ptr, P->bci_pos, P->bci_chunk, P->max_nb,
                             P->bin_seg, P->bin_cnt, P->bin_row, nullptr, nullptr, nullptr,
                             P->st));
      HIPCHK(scan_excl_i64(P->bin_cnt, P->bin_start, nbins, nullptr, nullptr, P->scan_temp,
                           P->st));
      HIPCHK(scan_excl_i64(P->bin_seg, P->seg_beg, nbins, P->seg_beg + nbins, nullptr,
                           P->scan_temp, P->st));
      HIPCHK(launch_run_rows(P->M, P->g, false, P->bci_ptr, P->bci_pos, P->bci_chunk, P->max_nb,
                             nullptr, nullptr, nullptr, P->seg_beg, P->bin_start,
                             P->run_list, P->st));
    }
    HIPCHK(launch_bin_group(P->g, b, P->bin_cnt, P->dense_min, P->group_max, P->dense_items,
                            P->sort_items, P->item_counts, P->st));
    // the item counts size the launches over the items, and the dense
    // items' column bitmaps (2^shift bits each), written by the count pass
    // and read by the numeric one
    {
      int32_t ic[2] = {0, 0};
      magnus_status_t sr = readback(P, {{P->item_counts, 8}}, {ic});
      if (sr != MAGNUS_OK) return sr;
      P->n_dense_run = ic[0];
      P->n_sort_run = ic[1];
      P->chunk_bm = (uint32_t*)palloc(
          P, (size_t)std::max<int64_t>(1, P->n_dense_run) * (((size_t)1 << P->shift) / 8));
      if (!P->chunk_bm) return MAGNUS_ERR_OOM;
    }
    HIPCHK(launch_dense_order(P->g, P->n_dense_run, P->dense_items, P->item_counts, P->bin_row,
                              P->xcd_cpx, P->xcd_start, P->xcd_cur, P->xcd_temp, P->st));
    HIPCHK(launch_run_records(P->g, P->n_dense_run, P->dense_items, P->item_counts,
                              P->bin_start, P->bin_cnt, P->bin_row, P->seg_beg, P->xcd_cpx,
                              P->xcd_cur, P->run_rec, P->st));
    unsigned int* wk = P->work_ctr;
    HIPCHK(launch_fill_i64((int64_t*)wk, N_XCD / 2, 0, P->st));
    {
      ProfScope ps(h, P->st, "run_count (symbolic, chunks from runs)",
                   (double)b.nip * P->s_col + (double)P->n_runs * 16 + (double)nbins * 40);
      HIPCHK(launch_run_accum(P->M, P->g, nbins, false, P->bin_start, P->bin_cnt, P->bin_row,
                              P->run_rec, P->sort_items, P->item_counts, P->seg_beg,
                              P->run_list, P->bin_nnz, nullptr, nullptr, 0,
                              nullptr, P->dense_block, wk, P->persistent_wgs_count, P->chunk_bm,
                              P->n_sort_run, P->xcd_start, P->xcd_cpx, P->st));
    }
    HIPCHK(launch_bin_rows(P->g, b.k0, b.k1, P->bin_nnz, P->crp, nullptr, nullptr, false, P->st));
    return MAGNUS_OK;
  }
  if (P->bitmap_symbolic) {
    {
      const double ipc = (double)P->h_stats.ip_cat[2], ec = (double)P->h_stats.ent_cat[2];
      ProfScope ps(h, P->st, "row_bitmap (symbolic, chunked rows)",
                   ipc * P->s_col + ec * (P->s_col + 8 + P->s_rp) +
                       (double)P->info.n_bins * 20 + (double)P->nch * 8);
      HIPCHK(launch_row_bitmap(P->M, P->g, P->aoff, P->max_nb, P->bin_nnz, P->bin_cnt, P->bin_row,
                               P->crp, P->st));
    }
    for (size_t bi = 0; bi < P->batches.size(); ++bi) {
      const BatchArgs& b = P->batches[bi];
      HIPCHK(scan_excl_i64(P->bin_cnt + b.bin0, P->bin_start + b.bin0, b.nbins, nullptr, nullptr,
                           P->scan_temp, P->st));
      HIPCHK(launch_bin_group(P->g, b, P->bin_cnt, P->dense_min, P->group_max, P->dense_items,
                              P->sort_items, P->item_counts + 2 * bi, P->st));
    }
    return MAGNUS_OK;
  }
  // the row bitmap does not fit the LDS: per batch, per-chunk product totals
  // (tile histograms added atomically), their scan, a reorder of the
  // chunk-local columns, and a count of the distinct columns of every chunk
  for (size_t bi = 0; bi < P->batches.size(); ++bi) {
    const BatchArgs& b = P->batches[bi];
    int32_t* ic = P->item_counts + 2 * bi;
    HIPCHK(launch_fill_i64(P->bin_cnt + b.bin0, b.nbins, 0, P->st));
    HIPCHK(launch_bin_hist(P->M, P->g, b, P->tile_row, P->aoff, P->tile_e0, P->bin_cnt,
                           P->bin_row, P->max_nb, P->st));
    HIPCHK(scan_excl_i64(P->bin_cnt + b.bin0, P->bin_start + b.bin0, b.nbins, nullptr, nullptr,
                         P->scan_temp, P->st));
    HIPCHK(launch_bin_group(P->g, b, P->bin_cnt, P->dense_min, P->group_max, P->dense_items,
                            P->sort_items, ic, P->st));
    HIPCHK(launch_fill_i64((int64_t*)P->bin_cursor + b.bin0, b.nbins, 0, P->st));
    HIPCHK(launch_bin_scatter2(P->M, P->g, b, false, 0, P->sorted_out, 0, P->tile_row, P->aoff,
                               P->tile_e0, P->bin_start, P->bin_cursor, P->ws_col, P->ws_val,
                               P->max_nb, P->st));
    unsigned int* wk = P->work_ctr + 4 * bi;
    HIPCHK(launch_fill_i64((int64_t*)wk, 1, 0, P->st));
    HIPCHK(launch_bin_accum(P->g, b, false, P->M.f64, P->bin_start, P->bin_cnt, P->bin_row,
                            P->dense_items, P->sort_items, ic, P->ws_col, P->ws_val, P->bin_nnz,
                            P->bin_out, nullptr, 0, nullptr, P->dense_block, wk,
                            P->persistent_wgs, false, P->st));
    HIPCHK(launch_bin_rows(P->g, b.k0, b.k1, P->bin_nnz, P->crp, nullptr, nullptr, false, P->st));
  }
  return MAGNUS_OK;
}

// Numeric phase of CHUNKED rows, batch by batch: chunk output offsets in C,
// reorder into the workspace, accumulate every chunk into C.
magnus_status_t chunked_numeric(magnus_plan_s* P, void* ccol, int col64, void* cval) {
  magnus_handle_s* h = P->h;
  if (P->runs) {
    const BatchArgs& b = P->batches[0];
    HIPCHK(launch_bin_rows(P->g, b.k0, b.k1, P->bin_nnz, nullptr, P->crp, P->bin_out, true,
                           P->st));
    unsigned int* wk = P->work_ctr + N_XCD;
    HIPCHK(launch_fill_i64((int64_t*)wk, N_XCD / 2, 0, P->st));
    // per product: B column and value; per run: its record and A value; per
    // output: C written
    ProfScope ps(h, P->st, "run_accum (numeric, chunks from runs)",
                 (double)b.nip * (P->s_col + P->s_val) +
                     (double)P->n_runs * (16 + P->s_val) +
                     (double)b.nnz_out * (P->s_col + P->s_val));
    HIPCHK(launch_run_accum(P->M, P->g, b.nbins, true, P->bin_start, P->bin_cnt, P->bin_row,
                            P->run_rec, P->sort_items, P->item_counts, P->seg_beg,
                            P->run_list, P->bin_nnz, P->bin_out, ccol, col64, cval,
                            P->dense_block, wk, P->persistent_wgs, P->chunk_bm, P->n_sort_run,
                            P->xcd_start, P->xcd_cpx, P->st));
    return MAGNUS_OK;
  }
  for (size_t bi = 0; bi < P->batches.size(); ++bi) {
    const BatchArgs& b = P->batches[bi];
    int32_t* ic = P->item_counts + 2 * bi;
    HIPCHK(launch_bin_rows(P->g, b.k0, b.k1, P->bin_nnz, nullptr, P->crp, P->bin_out, true,
                           P->st));
    HIPCHK(launch_fill_i64((int64_t*)P->bin_cursor + b.bin0, b.nbins, 0, P->st));
    {
      // per product: B column and value read, chunk-local column and
      // product written; per A entry: column, value, product offset, B row
      const double bytes = (double)b.nip * (P->s_col + P->s_val + 2 + P->s_val) +
                           (double)b.nent * (P->s_col + P->s_val + 8 + P->s_rp);
      if (P->det) {
        ProfScope ps(h, P->st, "bin_scatter_det (ordered reorder)", bytes);
        const int64_t sg0 = P->h_det_segBase[b.k0];
        HIPCHK(launch_bin_scatter_det(P->M, P->g, P->aoff, P->tile_e0, P->det_seg_row,
                                      P->det_segBase, P->det_tabBase, P->det_tabS, P->det_S,
                                      sg0, P->h_det_segBase[b.k1] - sg0, P->bin_start, P->ws_col,
                                      P->ws_val, P->max_nb, P->st));
      } else {
        ProfScope ps(h, P->st, "bin_scatter (numeric reorder)", bytes);
        HIPCHK(launch_bin_scatter2(P->M, P->g, b, true, 0, P->sorted_out, 0, P->tile_row, P->aoff,
                                   P->tile_e0, P->bin_start, P->bin_cursor, P->ws_col, P->ws_val,
                                   P->max_nb, P->st));
      }
    }
    unsigned int* wk = P->work_ctr + 4 * bi + 2;
    HIPCHK(launch_fill_i64((int64_t*)wk, 1, 0, P->st));
    {
      // per product: chunk-local column and value read; per output: C write
      ProfScope ps(h, P->st,
                   P->det ? "bin_accum_det (ordered dense+sort)"
                          : "bin_accum (numeric, dense+sort chunks)",
                   (double)b.nip * (2 + P->s_val) + (double)b.nnz_out * (P->s_col + P->s_val));
      HIPCHK(launch_bin_accum(P->g, b, true, P->M.f64, P->bin_start, P->bin_cnt, P->bin_row,
                              P->dense_items, P->sort_items, ic, P->ws_col, P->ws_val, P->bin_nnz,
                              P->bin_out, ccol, col64, cval, P->dense_block, wk,
                              P->persistent_wgs, P->det, P->st));
    }
  }
  return MAGNUS_OK;
}

// ---------------------------------------------------------------------------
// Coarse-level rows (Section 3.3, Algorithm 4)
// ---------------------------------------------------------------------------
magnus_status_t setup_coarse(magnus_plan_s* P) {
  magnus_handle_s* h = P->h;
  auto& C = P->co;
  const int64_t n1 = C.nrows;
  ChunkGeom& g1 = C.g1;
  g1.rows = P->list + P->h_list_off[CLS_COARSE];
  g1.ip = P->ip;
  g1.minc = P->minc;
  g1.maxc = P->maxc;
  g1.nch = n1;
  g1.shift = C.cshift;
  g1.tile = C.tile1;
  g1.hints = P->hints;
  const int64_t vs = P->M.f64 ? 8 : 4;
  int64_t W = 0, tots[3];
  // per product: the first workspace (32-bit column, value) and the second
  // (16-bit column, value)
  magnus_status_t s = batch_width(P, (4 + vs) + (2 + vs), W);
  if (s != MAGNUS_OK) return s;
  s = geometry_and_batches(P, g1, W, C.b1, C.ws_products, tots);
  if (s != MAGNUS_OK) return s;
  const int64_t ntiles1 = tots[1], nv = tots[2];
  const int64_t nbat = (int64_t)C.b1.size();
  C.nv = nv;
  if (nv > INT32_MAX) return MAGNUS_ERR_INDEX_OVERFLOW;
  if (!P->aoff) P->aoff = (int64_t*)palloc(P, sizeof(int64_t) * std::max<int64_t>(1, P->a_nnz));
  C.tile_row1 = (int32_t*)palloc(P, sizeof(int32_t) * std::max<int64_t>(1, ntiles1));
  C.tile_e0 = (int64_t*)palloc(P, sizeof(int64_t) * std::max<int64_t>(1, ntiles1));
  C.ent = (int64_t*)palloc(P, sizeof(int64_t) * (2 * n1 + 1));
  if (!P->aoff || !C.tile_row1 || !C.tile_e0 || !C.ent) return MAGNUS_ERR_OOM;
  C.entBase = C.ent + n1;
  HIPCHK(launch_aoff(P->M, g1.rows, n1, P->aoff, C.ent, P->st));
  HIPCHK(scan_excl_i64(C.ent, C.entBase, n1, C.entBase + n1, nullptr, P->temp, P->st));
  HIPCHK(launch_tiles(g1.nt, g1.tileBase, 0, n1, C.tile_row1, P->st));
  HIPCHK(launch_tile_e0(P->M, g1, C.tile_row1, P->aoff, ntiles1, C.tile_e0, P->st));

  // per coarse chunk: counts, starts, nnz, output offsets, column range and
  // fine chunk count; the size split's lists and scratch
  int64_t max_nb1b = 1;
  for (auto& b : C.b1) max_nb1b = std::max(max_nb1b, b.nbins);
  C.cnt1 = (int64_t*)palloc(P, sizeof(int64_t) * nv);
  C.start1 = (int64_t*)palloc(P, sizeof(int64_t) * nv);
  C.nnz1 = (int64_t*)palloc(P, sizeof(int64_t) * nv);
  C.out1 = (int64_t*)palloc(P, sizeof(int64_t) * (nv + 1));
  C.row1 = (int32_t*)palloc(P, sizeof(int32_t) * nv);
  C.cur1 = (unsigned long long*)palloc(P, sizeof(unsigned long long) * nv);
  C.minc2 = (int64_t*)palloc(P, sizeof(int64_t) * 3 * nv);
  C.big_all = (int32_t*)palloc(P, sizeof(int32_t) * nv);
  C.small_all = (int32_t*)palloc(P, sizeof(int32_t) * nv);
  C.flags = (int64_t*)palloc(P, sizeof(int64_t) * 2 * max_nb1b);
  C.nbig_dev = (int64_t*)palloc(P, sizeof(int64_t) * std::max<int64_t>(1, nbat));
  C.scan_temp = palloc(P, scan_temp_bytes(nv + 1));
  C.item_counts = (int32_t*)palloc(P, sizeof(int32_t) * 2 * std::max<int64_t>(1, nbat));
  C.work = (unsigned int*)palloc(P, sizeof(int64_t) * 2 * std::max<int64_t>(1, nbat));
  // the first reorder is done once, with values, in the symbolic phase when
  // all the coarse rows' products fit the workspace cap (max_workspace_bytes,
  // else a quarter of the device memory)
  C.ip_total = tots[0];
  // coarse chunks of few products on average (rows over 512 coarse chunks
  // wide): level-2 tiles of 2048 products at 256 threads, where one coarse
  // chunk of about a thousand products would leave most of 1024 threads idle
  // (uniform 2^30 columns: level-2 count and reorder 42.6 + 12.9 ms at
  // 2048 x 256, 51.7 + 22.4 at 4096 x 1024)
  C.l2_block = 1024;
  if (C.ip_total < (int64_t)MG_L2_SMALL * std::max<int64_t>(1, nv)) {
    C.tile2 = std::min(C.tile2, 2048);
    C.l2_block = 256;
  }
  {
    int64_t cap = h->opts.max_workspace_bytes;
    if (cap <= 0) {
      size_t fr = 0, tot = 0;
      HIPCHK(hipMemGetInfo(&fr, &tot));
      cap = (int64_t)(tot / 4);
    }
    cap /= std::max<int64_t>(1, P->ws_div);
    C.keep_ws1 = C.ip_total * (4 + vs) <= cap;
  }
  const int64_t n_ws1 = C.keep_ws1 ? C.ip_total : C.ws_products;
  C.ws1_col = (uint32_t*)palloc(P, sizeof(uint32_t) * std::max<int64_t>(1, n_ws1));
  C.ws1_val = palloc(P, (size_t)vs * std::max<int64_t>(1, n_ws1));
  C.ws2_col = (uint16_t*)palloc(P, sizeof(uint16_t) * C.ws_products);
  C.ws2_val = palloc(P, (size_t)vs * C.ws_products);
  if (!C.cnt1 || !C.start1 || !C.nnz1 || !C.out1 || !C.row1 || !C.cur1 || !C.minc2 ||
      !C.big_all || !C.small_all || !C.flags || !C.nbig_dev || !C.scan_temp ||
      !C.item_counts || !C.work || !C.ws1_col || !C.ws1_val || !C.ws2_col || !C.ws2_val)
    return MAGNUS_ERR_OOM;
  C.maxc2 = C.minc2 + nv;
  C.vnb = C.minc2 + 2 * nv;
  C.pos = C.flags + max_nb1b;
  HIPCHK(launch_vrow_geom(g1, P->shift, C.minc2, C.maxc2, C.vnb, P->st));
  HIPCHK(hipMemsetAsync(C.item_counts, 0, sizeof(int32_t) * 2 * std::max<int64_t>(1, nbat),
                        P->st));
  C.cb.assign(nbat, magnus_plan_s::CBatch{});
  return MAGNUS_OK;
}

// Level-2 geometry of a batch's big coarse chunks (known after the first
// reorder has counted them): their fine chunks and tiles, and the per fine
// chunk arrays, allocated for this batch.
magnus_status_t coarse_fine_setup(magnus_plan_s* P, size_t bi) {
  magnus_handle_s* h = P->h;
  auto& C = P->co;
  magnus_plan_s::CBatch& cb = C.cb[bi];
  const int64_t nb = cb.nbig;
  int64_t* geo = (int64_t*)palloc(P, sizeof(int64_t) * (3 * nb + 2 * (nb + 1) + 1));
  if (!geo) return MAGNUS_ERR_OOM;
  ChunkGeom& g2 = cb.g2;
  g2.rows = cb.big;
  g2.ip = C.cnt1;
  g2.minc = C.minc2;
  g2.maxc = C.maxc2;
  g2.nb = geo;
  g2.nt = geo + nb;
  int64_t* cntL = geo + 2 * nb;
  g2.binBase = geo + 3 * nb;
  g2.tileBase = g2.binBase + (nb + 1);
  int64_t* ptot = g2.tileBase + (nb + 1);
  g2.ipBase = nullptr;
  g2.nch = nb;
  g2.shift = P->shift;
  g2.tile = C.tile2;
  g2.hints = P->hints;
  HIPCHK(launch_vrow_gather(cb.big, nb, C.vnb, C.cnt1, g2.nb, cntL, P->st));
  HIPCHK(launch_vrow_tiles(g2, 0, nb, P->st));
  HIPCHK(scan_excl_i64(g2.nb, g2.binBase, nb, g2.binBase + nb, nullptr, C.scan_temp, P->st));
  HIPCHK(scan_excl_i64(g2.nt, g2.tileBase, nb, g2.tileBase + nb, nullptr, C.scan_temp, P->st));
  HIPCHK(scan_excl_i64(cntL, cntL, nb, ptot, nullptr, C.scan_temp, P->st));
  int64_t tot[3] = {0, 0, 0};
  magnus_status_t s = readback(P, {{g2.binBase + nb, 8}, {g2.tileBase + nb, 8}, {ptot, 8}},
                               {&tot[0], &tot[1], &tot[2]});
  if (s != MAGNUS_OK) return s;
  const int64_t F = tot[0], T = tot[1];
  if (T > INT32_MAX) return MAGNUS_ERR_INDEX_OVERFLOW;
  cb.nbins2 = F;
  cb.nip2 = tot[2];
  C.nbins2 += F;
  cb.cnt2 = (int64_t*)palloc(P, sizeof(int64_t) * F);
  cb.start2 = (int64_t*)palloc(P, sizeof(int64_t) * F);
  cb.nnz2 = (int64_t*)palloc(P, sizeof(int64_t) * F);
  cb.out2 = (int64_t*)palloc(P, sizeof(int64_t) * F);
  cb.dense2 = (int64_t*)palloc(P, sizeof(int64_t) * F);
  cb.sort2 = (int64_t*)palloc(P, sizeof(int64_t) * 2 * F);
  cb.row2 = (int32_t*)palloc(P, sizeof(int32_t) * F);
  cb.cur2 = (unsigned long long*)palloc(P, sizeof(unsigned long long) * F);
  cb.tile_row2 = (int32_t*)palloc(P, sizeof(int32_t) * std::max<int64_t>(1, T));
  cb.scan_temp = palloc(P, scan_temp_bytes(F + 1));
  if (!cb.cnt2 || !cb.start2 || !cb.nnz2 || !cb.out2 || !cb.dense2 || !cb.sort2 || !cb.row2 ||
      !cb.cur2 || !cb.tile_row2 || !cb.scan_temp)
    return MAGNUS_ERR_OOM;
  HIPCHK(launch_tiles(g2.nt, g2.tileBase, 0, nb, cb.tile_row2, P->st));
  HIPCHK(launch_vrow_rows(g2, cb.row2, P->st));
  BatchArgs& b2 = cb.b2;
  b2 = BatchArgs{};
  b2.k0 = 0;
  b2.k1 = nb;
  b2.tile0 = 0;
  b2.ntiles = T;
  b2.bin0 = 0;
  b2.nbins = F;
  b2.nip = tot[2];
  // the bitmap of a coarse chunk (2^cshift bits) pays when its products are
  // dense enough
  cb.bitmap_sym = (tot[2] / std::max<int64_t>(1, nb)) * MG_BITMAP_DENSITY >=
                  ((int64_t)1 << C.cshift);
  return MAGNUS_OK;
}

// Symbolic phase of coarse-level rows: per batch, the coarse chunks' product
// counts and the first reorder (columns only), the split of the coarse
// chunks by size; small ones counted by sorting; for big ones each fine
// chunk's products and nnz, either from a bitmap of the coarse chunk (dense
// coarse chunks) or from the level-2 reorder of the columns and the
// accumulators in count mode (sparse ones, where clearing and scanning a
// bitmap would cost more than the products); row nnz.
magnus_status_t coarse_symbolic(magnus_plan_s* P) {
  magnus_handle_s* h = P->h;
  auto& C = P->co;
  ChunkGeom& g1 = C.g1;
  for (size_t bi = 0; bi < C.b1.size(); ++bi) {
    const BatchArgs& b = C.b1[bi];
    magnus_plan_s::CBatch& cb = C.cb[bi];
    int32_t* ic = C.item_counts + 2 * bi;
    uint32_t* w1c = C.col1(b);
    void* w1v = C.val1(b, (int64_t)P->s_val);
    {
      // per product: B column read (twice: histogram and reorder), 32-bit
      // column written (with the kept workspace, B value read and product
      // written too); per tile the A entries' metadata
      const double pv = C.keep_ws1 ? 2 * P->s_val : 0;
      ProfScope ps(h, P->st,
                   C.keep_ws1 ? "coarse_reorder (symbolic, L1, values)"
                              : "coarse_reorder (symbolic, level 1)",
                   (double)b.nip * (2 * P->s_col + 4 + pv) +
                       2.0 * (double)b.nip / std::max<int64_t>(1, g1.tile) * 64);
      HIPCHK(launch_fill_i64(C.cnt1 + b.bin0, b.nbins, 0, P->st));
      HIPCHK(launch_bin_hist(P->M, g1, b, C.tile_row1, P->aoff, C.tile_e0, C.cnt1, C.row1,
                             C.max_nb1, P->st));
      HIPCHK(scan_excl_i64(C.cnt1 + b.bin0, C.start1 + b.bin0, b.nbins, nullptr, nullptr,
                           C.scan_temp, P->st));
      HIPCHK(launch_fill_i64((int64_t*)C.cur1 + b.bin0, b.nbins, 0, P->st));
      HIPCHK(launch_bin_scatter2(P->M, g1, b, C.keep_ws1, 1,
                                 C.keep_ws1 ? C.sorted1 : C.sorted1_sym, C.block1, C.tile_row1,
                                 P->aoff,
                                 C.tile_e0, C.start1, C.cur1, w1c, w1v, C.max_nb1, P->st));
    }
    cb.big = C.big_all + b.bin0;
    cb.small = C.small_all + b.bin0;
    HIPCHK(launch_vrow_split(C.cnt1, b.bin0, b.nbins, C.flags, C.pos, C.nbig_dev + bi,
                             C.scan_temp, cb.big, cb.small, P->st));
    magnus_status_t s = readback(P, {{C.nbig_dev + bi, 8}}, {&cb.nbig});
    if (s != MAGNUS_OK) return s;
    cb.nsmall = b.nbins - cb.nbig;
    {
      // per product of a small coarse chunk: 32-bit column read
      ProfScope ps(h, P->st, "coarse_sort (symbolic, small chunks)",
                   (double)(b.nip) * 4);
      HIPCHK(launch_vrow_sort(false, P->M.f64, cb.small, cb.nsmall, C.cnt1, C.start1, C.minc2,
                              w1c, w1v, C.nnz1, nullptr, nullptr, 0, nullptr, P->st));
    }
    if (cb.nbig > 0) {
      s = coarse_fine_setup(P, bi);
      if (s != MAGNUS_OK) return s;
      ChunkGeom& g2 = cb.g2;
      const BatchArgs& b2 = cb.b2;
      if (cb.bitmap_sym) {
        // per product: 32-bit column read; per fine chunk: three words out
        ProfScope ps(h, P->st, "coarse_bitmap (symbolic, level 2)",
                     (double)b2.nip * 4 + (double)b2.nbins * 20);
        HIPCHK(launch_vrow_bitmap(g2, C.cshift, 0, cb.nbig, C.max_nb2, C.start1, w1c, cb.cnt2,
                                  cb.nnz2, cb.row2, C.nnz1, P->st));
        HIPCHK(scan_excl_i64(cb.cnt2, cb.start2, b2.nbins, nullptr, nullptr, cb.scan_temp,
                             P->st));
        HIPCHK(launch_bin_group(g2, b2, cb.cnt2, P->dense_min, P->group_max, cb.dense2,
                                cb.sort2, ic, P->st));
      } else {
        // per product: 32-bit column read twice (histogram, reorder), 16-bit
        // column written and read; per fine chunk: count, start, nnz
        ProfScope ps(h, P->st, "coarse_count (symbolic, level 2)",
                     (double)b2.nip * (4 + 4 + 2 + 2) + (double)b2.nbins * 24);
        HIPCHK(launch_fill_i64(cb.cnt2, b2.nbins, 0, P->st));
        HIPCHK(launch_l2_hist(g2, b2, cb.tile_row2, C.start1, w1c, cb.cnt2, C.max_nb2, P->st));
        HIPCHK(scan_excl_i64(cb.cnt2, cb.start2, b2.nbins, nullptr, nullptr, cb.scan_temp,
                             P->st));
        HIPCHK(launch_bin_group(g2, b2, cb.cnt2, P->dense_min, P->group_max, cb.dense2,
                                cb.sort2, ic, P->st));
        HIPCHK(launch_fill_i64((int64_t*)cb.cur2, b2.nbins, 0, P->st));
        HIPCHK(launch_l2_scatter(g2, b2, false, P->M.f64, cb.tile_row2, C.start1, w1c, w1v,
                                 cb.start2, cb.cur2, C.ws2_col, C.ws2_val, C.max_nb2, C.l2_block,
                                 P->st));
        unsigned int* wk = C.work + 4 * bi + 2;
        HIPCHK(launch_fill_i64((int64_t*)wk, 1, 0, P->st));
        HIPCHK(launch_bin_accum(g2, b2, false, P->M.f64, cb.start2, cb.cnt2, cb.row2, cb.dense2,
                                cb.sort2, ic, C.ws2_col, C.ws2_val, cb.nnz2, cb.out2, nullptr, 0,
                                nullptr, P->dense_block, wk, P->persistent_wgs, false, P->st));
        HIPCHK(launch_bin_rows(g2, 0, cb.nbig, cb.nnz2, C.nnz1, nullptr, nullptr, false,
                               P->st));
      }
    }
    HIPCHK(launch_bin_rows(g1, b.k0, b.k1, C.nnz1, P->crp, nullptr, nullptr, false, P->st));
  }
  return MAGNUS_OK;
}

// Numeric phase of coarse-level rows, batch by batch: output offsets of the
// coarse and fine chunks, the first reorder, the sorts of the small coarse
// chunks, the second reorder and the accumulation of the big ones' fine
// chunks into C.
magnus_status_t coarse_numeric(magnus_plan_s* P, void* ccol, int col64, void* cval) {
  magnus_handle_s* h = P->h;
  auto& C = P->co;
  const double vs = P->s_val;
  for (size_t bi = 0; bi < C.b1.size(); ++bi) {
    const BatchArgs& b = C.b1[bi];
    magnus_plan_s::CBatch& cb = C.cb[bi];
    HIPCHK(launch_bin_rows(C.g1, b.k0, b.k1, C.nnz1, nullptr, P->crp, C.out1, true, P->st));
    uint32_t* w1c = C.col1(b);
    void* w1v = C.val1(b, (int64_t)vs);
    if (!C.keep_ws1) {
      HIPCHK(launch_fill_i64((int64_t*)C.cur1 + b.bin0, b.nbins, 0, P->st));
      // per product: B column and value read, 32-bit column and product
      // written; per A entry: column, value, product offset, B row
      ProfScope ps(h, P->st, "coarse_scatter (numeric, level 1)",
                   (double)b.nip * (P->s_col + vs + 4 + vs) +
                       (double)b.nent * (P->s_col + vs + 8 + P->s_rp));
      HIPCHK(launch_bin_scatter2(P->M, C.g1, b, true, 1, C.sorted1, C.block1, C.tile_row1, P->aoff,
                                 C.tile_e0, C.start1, C.cur1, w1c, w1v, C.max_nb1, P->st));
    }
    {
      // per product of a small coarse chunk: column and value read; per
      // output: C column and value
      ProfScope ps(h, P->st, "coarse_sort (numeric, small chunks)",
                   (double)(b.nip - cb.nip2) * (4 + vs));
      HIPCHK(launch_vrow_sort(true, P->M.f64, cb.small, cb.nsmall, C.cnt1, C.start1, C.minc2,
                              w1c, w1v, C.nnz1, C.out1, ccol, col64, cval, P->st));
    }
    if (cb.nbig == 0) continue;
    const BatchArgs& b2 = cb.b2;
    HIPCHK(launch_bin_rows(cb.g2, 0, cb.nbig, cb.nnz2, nullptr, C.out1, cb.out2, true, P->st));
    HIPCHK(launch_fill_i64((int64_t*)cb.cur2, b2.nbins, 0, P->st));
    {
      // per product: 32-bit column and value read, 16-bit column and value
      // written
      ProfScope ps(h, P->st, "fine_scatter (numeric, level 2)",
                   (double)b2.nip * (4 + vs + 2 + vs));
      HIPCHK(launch_l2_scatter(cb.g2, b2, true, P->M.f64, cb.tile_row2, C.start1, w1c, w1v,
                               cb.start2, cb.cur2, C.ws2_col, C.ws2_val, C.max_nb2, C.l2_block,
                               P->st));
    }
    unsigned int* wk = C.work + 4 * bi;
    HIPCHK(launch_fill_i64((int64_t*)wk, 1, 0, P->st));
    {
      // the kernels of the CHUNKED rows' accumulation, under the same name
      ProfScope ps(h, P->st, "bin_accum (numeric, dense+sort chunks)",
                   (double)b2.nip * (2 + vs) + (double)b.nnz_out * (P->s_col + vs));
      HIPCHK(launch_bin_accum(cb.g2, b2, true, P->M.f64, cb.start2, cb.cnt2, cb.row2, cb.dense2,
                              cb.sort2, C.item_counts + 2 * bi, C.ws2_col, C.ws2_val, cb.nnz2,
                              cb.out2, ccol, col64, cval, P->dense_block, wk, P->persistent_wgs,
                              false, P->st));
    }
  }
  return MAGNUS_OK;
}

magnus_status_t run_rows(magnus_plan_s* P, bool numeric, void* ccol, void* cval) {
  magnus_handle_s* h = P->h;
  const DevStats& S = P->h_stats;
  const double cv = P->s_col + (numeric ? P->s_val : 0);
  const double nzs = numeric ? (double)P->info.nnz_by_category[0] * (P->s_col + P->s_val) : 0;
  const double nzd = numeric ? (double)P->info.nnz_by_category[1] * (P->s_col + P->s_val) : 0;
  // per product: B column (and value); per A entry: column (value) and both
  // B row pointers; per row: list entry, minc, row offset or count; per
  // output (numeric): C column and value
  {
    ProfScope ps_sort(h, P->st, numeric ? "sort_rows (numeric)" : "sort_rows (symbolic)",
                      (double)S.ip_cat[0] * cv + (double)S.ent_cat[0] * (cv + 2 * P->s_rp) +
                          (double)S.rows_cat[0] * 20 + nzs);
    for (int c = 0; c < NSORT_CLS; ++c) {
      const int64_t cnt = P->h_list_off[c + 1] - P->h_list_off[c];
      if (cnt > 0)
        HIPCHK(launch_sort_rows(P->M, single_src(P->M, ccol, cval), c, numeric, P->list,
                                P->h_list_off[c], cnt, P->minc, P->colbits, P->crp, P->crp,
                                P->stats, P->st));
    }
  }
  const int64_t nd = P->h_list_off[CLS_DENSE + 1] - P->h_list_off[CLS_DENSE];
  {
    ProfScope ps_dense(h, P->st, numeric ? "dense_rows (numeric)" : "dense_rows (symbolic)",
                       (double)S.ip_cat[1] * cv + (double)S.ent_cat[1] * (cv + 2 * P->s_rp) +
                           (double)S.rows_cat[1] * 28 + nzd);
    if (nd > 0)
      HIPCHK(launch_dense_rows(P->M, single_src(P->M, ccol, cval), numeric, P->list,
                               P->h_list_off[CLS_DENSE], nd, P->minc, P->maxc, P->dense_shift,
                               P->dense_block, P->crp, P->crp, P->st));
  }
  return MAGNUS_OK;
}

}  // namespace

extern "C" {

const char* magnus_status_string(magnus_status_t s) {
  switch (s) {
    case MAGNUS_OK: return "MAGNUS_OK";
    case MAGNUS_ERR_INVALID_ARG: return "MAGNUS_ERR_INVALID_ARG";
    case MAGNUS_ERR_SHAPE: return "MAGNUS_ERR_SHAPE";
    case MAGNUS_ERR_DTYPE: return "MAGNUS_ERR_DTYPE";
    case MAGNUS_ERR_INVALID_CSR: return "MAGNUS_ERR_INVALID_CSR";
    case MAGNUS_ERR_INDEX_OVERFLOW: return "MAGNUS_ERR_INDEX_OVERFLOW";
    case MAGNUS_ERR_CAPACITY: return "MAGNUS_ERR_CAPACITY";
    case MAGNUS_ERR_WORKSPACE: return "MAGNUS_ERR_WORKSPACE";
    case MAGNUS_ERR_OOM: return "MAGNUS_ERR_OOM";
    case MAGNUS_ERR_REJECTED: return "MAGNUS_ERR_REJECTED";
    case MAGNUS_ERR_HIP: return "MAGNUS_ERR_HIP";
    case MAGNUS_ERR_NOT_READY: return "MAGNUS_ERR_NOT_READY";
    case MAGNUS_ERR_INTERNAL: return "MAGNUS_ERR_INTERNAL";
  }
  return "MAGNUS_ERR_UNKNOWN";
}

const char* magnus_last_error(magnus_handle_t h) { return h ? h->err.c_str() : ""; }

void magnus_options_default(magnus_options_t* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->force_category = MAGNUS_CAT_AUTO;
  o->sort_max = 0;
  o->chunk_shift = 0;
  o->bin_dense_min = 0;
  o->tile_products = 0;
  o->dense_block = 0;
  o->batch_products = 0;
  o->max_workspace_bytes = 0;
  o->validate = 0;
  o->lds_bytes = 0;
  o->sort_group_max = 0;
}

magnus_status_t magnus_create(magnus_handle_t* out, int device, const magnus_options_t* opts) {
  if (!out) return MAGNUS_ERR_INVALID_ARG;
  *out = nullptr;
  magnus_handle_s* h = new magnus_handle_s();
  h->device = device;
  magnus_options_default(&h->opts);
  if (opts) h->opts = *opts;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || device < 0 || device >= ndev) {
    h->err = "no such HIP device";
    delete h;
    return e != hipSuccess ? MAGNUS_ERR_HIP : MAGNUS_ERR_INVALID_ARG;
  }
  int v = 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess)
    h->lds_max = v;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess)
    h->cus = v;
  {
    // the allocation-free entry points' scratch: its address on this device
    void* p = nullptr;
    e = hipSetDevice(device);
    if (e == hipSuccess) e = noalloc_scratch(device, &p);
    if (e != hipSuccess) {
      delete h;
      return MAGNUS_ERR_HIP;
    }
  }
  *out = h;
  return MAGNUS_OK;
}

magnus_status_t magnus_destroy(magnus_handle_t h) {
  delete h;
  return MAGNUS_OK;
}

magnus_status_t magnus_set_options(magnus_handle_t h, const magnus_options_t* o) {
  if (!h || !o) return MAGNUS_ERR_INVALID_ARG;
  h->opts = *o;
  return MAGNUS_OK;
}

magnus_status_t magnus_set_allocator(magnus_handle_t h, magnus_alloc_fn a, magnus_free_fn f,
                                     void* ctx) {
  if (!h || (!a) != (!f)) return MAGNUS_ERR_INVALID_ARG;
  h->alloc_fn = a;
  h->free_fn = f;
  h->alloc_ctx = ctx;
  return MAGNUS_OK;
}

magnus_status_t magnus_gpu_chunk_shift(int32_t val_type, int64_t lds_bytes, int32_t* shift) {
  if (!shift || lds_bytes <= 0 || (val_type != MAGNUS_F32 && val_type != MAGNUS_F64))
    return MAGNUS_ERR_INVALID_ARG;
  *shift = default_shift(val_type == MAGNUS_F64, (int)std::min<int64_t>(lds_bytes, 1 << 30));
  return MAGNUS_OK;
}

magnus_status_t magnus_paper_chunk_model(int64_t m_c, int64_t s_cache, int64_t s_line,
                                         double s_dense_accum, int64_t* nf, int64_t* nco,
                                         int64_t* mcmax) {
  if (m_c < 1 || s_cache < 1 || s_line < 1 || !(s_dense_accum > 0) || !nf || !nco || !mcmax)
    return MAGNUS_ERR_INVALID_ARG;
  // Eq. 2-7 of Section 3.5; m_C ceiled to a power of two, m_CmaxL2 floored,
  // fine chunk counts rounded to the power of two nearest in log2
  int64_t mc = 1;
  while (mc < m_c) mc <<= 1;
  const double sc = 4.0 + 4.0 + 2.0 * (double)s_line;
  auto nearest = [](double x) -> int64_t {
    if (x <= 1.0) return 1;
    const double e = std::log2(x);
    const double lo = std::floor(e);
    return (int64_t)1 << (int)((e - lo >= 0.5) ? lo + 1 : lo);
  };
  const double mx = (double)s_cache * (double)s_cache / (4.0 * s_dense_accum * sc);
  int64_t m2 = 1;
  while ((double)(m2 * 2) <= mx) m2 <<= 1;
  *mcmax = m2;
  const bool fits = 2.0 * std::sqrt((double)mc * s_dense_accum * sc) < (double)s_cache;
  if (fits) {
    *nf = std::min<int64_t>(nearest(std::sqrt((double)mc * s_dense_accum / sc)), mc);
    *nco = 1;
  } else {
    *nf = std::min<int64_t>(nearest(std::sqrt((double)m2 * s_dense_accum / sc)), m2);
    *nco = std::max<int64_t>(1, mc / m2);
  }
  return MAGNUS_OK;
}

}  // extern "C"

namespace {

// One attempt at a plan; ws_div divides the row-batch width and the kept
// workspace cap.  *shrinkable reports whether a smaller divisor's retry could
// need less memory (some row batch was wider than the longest row).
magnus_status_t plan_once(magnus_handle_t h, const magnus_csr_t* A, const magnus_csr_t* B,
                          void* stream, magnus_plan_t* out, magnus_plan_info_t* info,
                          int64_t ws_div, bool* shrinkable) {
  *shrinkable = false;
  Mats M{};
  magnus_status_t s = make_mats(A, B, M);
  if (s != MAGNUS_OK) return s;
  HIPCHK(hipSetDevice(h->device));
  magnus_plan_s* P = new magnus_plan_s();
  P->ws_div = ws_div;
  P->h = h;
  P->st = (hipStream_t)stream;
  P->M = M;
  P->a_nnz = A->nnz;
  P->b_nnz = B->nnz;
  P->n = A->nrows;
  P->vtype = A->val_type;
  P->itype_rp = A->rowptr_type;
  P->itype_col = A->col_type;
  const magnus_options_t& o = h->opts;
  const int lds = o.lds_bytes > 0 ? std::min(o.lds_bytes, h->lds_max) : h->lds_max;
  P->lds_budget = lds;
  // deterministic mode defaults to chunks a quarter as long: its dense
  // accumulator is one wave per accumulator, and smaller chunks move most
  // products to the packed sorts, which keep more of the device busy
  P->shift = o.chunk_shift > 0 ? std::min(o.chunk_shift, 16)
                               : default_shift(M.f64, lds) - (o.deterministic ? 2 : 0);
  P->sort_max = o.sort_max > 0 ? std::min<int64_t>(o.sort_max, SORT_CAP + 1) : SORT_CAP + 1;
  // packed sort items of at most 512 products: a smaller network per
  // product than 1024 (config 2 accumulate 144.6 -> 142.0 ms; 256 is slower)
  P->group_max = o.sort_group_max > 0 ? std::min<int64_t>(o.sort_group_max, SORT_CAP) : SORT_CAP / 2;
  // chunks below dense_min are sorted: several packed up to group_max
  // products, or one alone when it holds more than group_max itself
  P->dense_min = o.bin_dense_min > 0 ? o.bin_dense_min : SORT_CAP;
  if (P->dense_min > SORT_CAP + 1) P->dense_min = SORT_CAP + 1;
  P->tile = o.tile_products > 0 ? o.tile_products : 1024;
  if (P->tile < 256 || P->tile > 16384 || (P->tile & (P->tile - 1))) P->tile = 1024;
  P->dense_block = (o.dense_block == 512 || o.dense_block == 1024) ? o.dense_block : 256;
  P->hints = o.stream_hints & 7;
  {
    // dense accumulator workgroups resident per CU, from its LDS footprint
    const size_t dl = bin_dense_lds(M.f64, P->shift);
    const int per_cu = std::max<int>(1, (int)(h->lds_max / std::max<size_t>(dl, 1)));
    P->persistent_wgs = std::max(1, h->cus) * std::min(per_cu, 2048 / P->dense_block);
    // count mode keeps only the bitmap in LDS: the waves per CU bound it
    const size_t dlc = ((size_t)1 << P->shift) / 8 + (size_t)P->dense_block * 8 + 4096;
    const int per_cu_c = std::max<int>(1, (int)(h->lds_max / dlc));
    P->persistent_wgs_count = std::max(1, h->cus) * std::min(per_cu_c, 2048 / P->dense_block);
  }

  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  auto cleanup = [&](magnus_status_t st) {
    *shrinkable = (P->nch > 0 || P->co.nrows > 0) && !P->w_at_min;
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    plan_free_all(P);
    delete P;
    return st;
  };
  const int64_t n = P->n;
  P->stats = (DevStats*)palloc(P, sizeof(DevStats));
  P->ip = (int64_t*)palloc(P, sizeof(int64_t) * std::max<int64_t>(n, 1));
  P->minc = (int64_t*)palloc(P, sizeof(int64_t) * std::max<int64_t>(n, 1));
  P->maxc = (int64_t*)palloc(P, sizeof(int64_t) * std::max<int64_t>(n, 1));
  P->crp = (int64_t*)palloc(P, sizeof(int64_t) * (n + 1));
  P->cls = (int32_t*)palloc(P, sizeof(int32_t) * std::max<int64_t>(n, 1));
  P->list = (int32_t*)palloc(P, sizeof(int32_t) * std::max<int64_t>(n, 1));
  P->list_off = (int64_t*)palloc(P, sizeof(int64_t) * (NCLS + 1));
  P->temp = palloc(P, std::max(classify_temp_bytes(n), scan_temp_bytes(n + 1)) + 1024);
  if (!P->stats || !P->ip || !P->minc || !P->maxc || !P->crp || !P->cls || !P->list ||
      !P->list_off || !P->temp)
    return cleanup(MAGNUS_ERR_OOM);

#define PCHK(expr)                                        \
  do {                                                    \
    hipError_t e_ = (expr);                               \
    if (e_ != hipSuccess) return cleanup(fail_hip(h, e_, #expr)); \
  } while (0)
#define SCHK(expr)                                        \
  do {                                                    \
    magnus_status_t s_ = (expr);                          \
    if (s_ != MAGNUS_OK) return cleanup(s_);              \
  } while (0)

  PCHK(hipEventCreate(&ev0));
  PCHK(hipEventCreate(&ev1));
  PCHK(hipEventRecord(ev0, P->st));
  PCHK(hipMemsetAsync(P->stats, 0, sizeof(DevStats), P->st));
  if (o.validate) {
    // an invalid column would index B's row pointers out of range in the
    // setup pass: the check is read back before anything else runs
    PCHK(launch_validate(M, A->nnz, B->nnz, P->stats, P->st));
    SCHK(readback(P, {{P->stats, sizeof(DevStats)}}, {&P->h_stats}));
    if (P->h_stats.err & ERR_INVALID_CSR) return cleanup(MAGNUS_ERR_INVALID_CSR);
  }
  ClassParams cp{};
  cp.sort_max = P->sort_max;
  cp.dense_max = (int64_t)1 << P->shift;
  P->det = o.deterministic != 0;
  // deterministic mode: every non-empty row takes the CHUNKED path
  cp.force = P->det ? (int)MAGNUS_CAT_CHUNKED
                    : ((o.force_category >= 0 && o.force_category <= 2) ? o.force_category : -1);
  {
    // coarse level (the paper's m_CmaxL2 with the LDS for the L2 cache):
    // chunks of 2^cshift columns, the widest whose bitmap (the symbolic
    // phase's accumulator, one bit per column) and chunk counts fit the LDS
    // budget, at most 2^12 chunks each, or coarse_chunks chunks; CHUNKED rows
    // wider than one coarse chunk take it
    auto& Co = P->co;
    const int sh = P->shift;
    auto fits = [&](int c) {
      return vrow_bitmap_lds(c, ((int64_t)1 << (c - sh)) + 1) + 1024 <= (size_t)lds;
    };
    int cs = sh + 1;
    while (cs < sh + 12 && fits(cs + 1)) ++cs;
    if (o.coarse_chunks > 0) {
      int lg = 1;
      while (lg < 12 && ((int64_t)2 << lg) <= o.coarse_chunks) ++lg;
      cs = std::min(cs, sh + lg);
    }
    Co.cshift = cs;
    Co.coarse_range = (!P->det && o.coarse_chunks >= 0 && fits(cs)) ? ((int64_t)1 << cs) : 0;
    cp.coarse_range = Co.coarse_range;
  }
  P->s_rp = M.rp64 ? 8 : 4;
  P->s_col = M.col64 ? 8 : 4;
  P->s_val = M.f64 ? 8 : 4;
  {
    ProfScope ps(h, P->st, "rowinfo (setup)",
                 (double)(n + 1) * P->s_rp + (double)A->nnz * (3 * P->s_col + 2 * P->s_rp) +
                     (double)n * 28);
    PCHK(launch_rowinfo(M, A->nnz, cp, P->ip, P->minc, P->maxc, P->cls, P->stats, P->list,
                        P->st));
  }
  PCHK(launch_classify(P->cls, n, P->list, P->list_off, P->temp, P->st));
  SCHK(readback(P, {{P->stats, sizeof(DevStats)}, {P->list_off, sizeof(int64_t) * (NCLS + 1)}},
                {&P->h_stats, P->h_list_off}));
  if (P->h_stats.err & ERR_INVALID_CSR) return cleanup(MAGNUS_ERR_INVALID_CSR);
  P->colbits = bits_for((int64_t)std::max<unsigned long long>(1, P->h_stats.range_cat[0]));
  P->dense_shift = dense_rows_shift(P->h_stats.range_cat[1], P->shift);
  if (o.tile_products <= 0 && P->h_stats.rows_cat[2] > 0 &&
      P->h_stats.ip_cat[2] / P->h_stats.rows_cat[2] >= ((unsigned long long)1 << 18))
    P->tile = 2048;  // long CHUNKED rows: longer tiles amortise each tile's A-entry staging
  P->max_nb = (int64_t)(P->h_stats.range_cat[2] >> P->shift) + 2;
  P->nch = P->h_list_off[CLS_CHUNKED + 1] - P->h_list_off[CLS_CHUNKED];
  if (P->max_nb > 65535 && P->nch > 0) return cleanup(MAGNUS_ERR_INVALID_ARG);
  if (P->nch > 0) {
    // the reorder kernels keep per-chunk counters of a row in LDS: shrink the
    // tile if they and the staged tile do not fit
    auto fits = [&](int tile) {
      return bin_scatter2_lds(M.f64, tile, P->max_nb, 0, P->sorted_out, 0) <= (size_t)h->lds_max &&
             (!P->det || bin_scatter_det_lds(M.f64, tile, P->max_nb) <= (size_t)h->lds_max);
    };
    while (P->tile > 256 && !fits(P->tile)) P->tile /= 2;
    if (!fits(P->tile)) {
      h->err = "too many chunks per row for the LDS: raise chunk_shift";
      return cleanup(MAGNUS_ERR_INVALID_ARG);
    }
    SCHK(setup_chunked(P));
  }
  P->co.nrows = P->h_list_off[CLS_COARSE + 1] - P->h_list_off[CLS_COARSE];
  if (P->co.nrows > 0) {
    auto& Co = P->co;
    Co.max_nb1 = (int64_t)(P->h_stats.range_cat[2] >> Co.cshift) + 2;
    Co.max_nb2 = ((int64_t)1 << (Co.cshift - P->shift)) + 1;
    if (Co.max_nb1 > 65535) {
      h->err = "too many coarse chunks per row";
      return cleanup(MAGNUS_ERR_INVALID_ARG);
    }
    // expansion-order write-out with short tiles while the rows span few
    // coarse chunks (long runs per chunk); chunk-ordered with long tiles
    // beyond
    Co.sorted1 = Co.max_nb1 > MG_COARSE_SORTED_MIN ? 1 : 0;
    Co.sorted1_sym = Co.max_nb1 > MG_COARSE_SORTED_SYM_MIN ? 1 : 0;
    // chunk-ordered tiles fill the LDS of a CU, one workgroup each: the
    // longest tile (up to 8192 products, longer runs per chunk) that fits
    // with 1024 threads, else with 512 (the gathers of more waves in flight).
    // Uniform 2^28 columns, first reorder: 8192 x 256 threads 86.7 ms, 8192 x
    // 512 58.9, 8192 x 1024 48.0; 2^30: 8192 x 512 72.8, 4096 x 1024 103.9
    Co.tile1 = Co.sorted1 ? 8192 : 1024;
    Co.block1 = 0;
    if (o.tile_products > 0) Co.tile1 = P->tile;
    if (Co.sorted1) {
      auto fits1 = [&](int t, int bk) {
        return bin_scatter2_lds(M.f64, t, Co.max_nb1, 1, 1, bk) <= (size_t)h->lds_max;
      };
      const int t0 = Co.tile1;
      Co.block1 = 256;
      for (int t = t0; t >= 256; t /= 2) {
        if (fits1(t, 1024)) { Co.tile1 = t; Co.block1 = 1024; break; }
        if (fits1(t, 512)) { Co.tile1 = t; Co.block1 = 512; break; }
        if (o.tile_products > 0) break;  // the set tile at 256 threads
      }
    }
    while (Co.tile1 > 256 && bin_scatter2_lds(M.f64, Co.tile1, Co.max_nb1, 1, Co.sorted1,
                                              Co.block1) > (size_t)h->lds_max)
      Co.tile1 /= 2;
    while (Co.tile2 > 256 && l2_scatter_lds(M.f64, Co.tile2, Co.max_nb2) > (size_t)h->lds_max)
      Co.tile2 /= 2;
    if (bin_scatter2_lds(M.f64, Co.tile1, Co.max_nb1, 1, Co.sorted1, Co.block1) >
            (size_t)h->lds_max ||
        l2_scatter_lds(M.f64, Co.tile2, Co.max_nb2) > (size_t)h->lds_max) {
      h->err = "too many coarse chunks per row for the LDS";
      return cleanup(MAGNUS_ERR_INVALID_ARG);
    }
    SCHK(setup_coarse(P));
  }

  // precise symbolic phase: exact nnz per row, then the row offsets of C
  PCHK(launch_fill_i64(P->crp, n + 1, 0, P->st));
  SCHK(run_rows(P, false, nullptr, nullptr));
  if (P->nch > 0) SCHK(chunked_symbolic(P));
  if (P->co.nrows > 0) {
    SCHK(coarse_symbolic(P));
    // nnz of C per coarse-level batch (profiling bytes): scan of the coarse
    // chunks' nnz, overwritten by their output offsets in the numeric phase
    PCHK(scan_excl_i64(P->co.nnz1, P->co.out1, P->co.nv, P->co.out1 + P->co.nv, nullptr,
                       P->co.scan_temp, P->st));
  }
  PCHK(launch_cat_nnz(P->cls, P->crp, n, P->stats, P->st));
  if (P->nch > 0) {
    PCHK(launch_gather_rows(P->crp, P->g.rows, P->nch, P->nnzr, P->st));
    PCHK(scan_excl_i64(P->nnzr, P->nnzBase, P->nch, P->nnzBase + P->nch, nullptr, P->temp, P->st));
  }
  PCHK(scan_excl_i64(P->crp, P->crp, n + 1, nullptr, nullptr, P->temp, P->st));
  PCHK(hipEventRecord(ev1, P->st));
  int64_t nnzc = 0;
  DevStats st2{};
  std::vector<int32_t> icounts(2 * P->batches.size() + 2, 0);
  const size_t nb_ = P->batches.size();
  std::vector<int64_t> bent(nb_ + 1, 0), bnnz(nb_ + 1, 0);
  std::vector<std::pair<const void*, size_t>> src = {
      {P->crp + n, 8}, {P->stats, sizeof(DevStats)}, {P->item_counts, sizeof(int32_t) * 2 * nb_}};
  std::vector<void*> dst = {&nnzc, &st2, icounts.data()};
  for (size_t b = 0; b <= nb_ && P->nch > 0; ++b) {
    const int64_t kk = (b < nb_) ? P->batches[b].k0 : P->nch;
    src.push_back({P->entBase + kk, 8});
    dst.push_back(&bent[b]);
    src.push_back({P->nnzBase + kk, 8});
    dst.push_back(&bnnz[b]);
  }
  const size_t nbc = P->co.b1.size();
  std::vector<int64_t> cent(nbc + 1, 0), cnnz(nbc + 1, 0);
  std::vector<int32_t> cicounts(2 * nbc + 2, 0);
  if (P->co.nrows > 0) {
    auto& Co = P->co;
    src.push_back({Co.item_counts, sizeof(int32_t) * 2 * nbc});
    dst.push_back(cicounts.data());
    for (size_t b = 0; b <= nbc; ++b) {
      src.push_back({Co.entBase + ((b < nbc) ? Co.b1[b].k0 : Co.nrows), 8});
      dst.push_back(&cent[b]);
      src.push_back({Co.out1 + ((b < nbc) ? Co.b1[b].bin0 : Co.nv), 8});
      dst.push_back(&cnnz[b]);
    }
  }
  SCHK(readback(P, src, dst));
  for (size_t b = 0; b < nb_; ++b) {
    P->batches[b].nent = bent[b + 1] - bent[b];
    P->batches[b].nnz_out = bnnz[b + 1] - bnnz[b];
  }
  for (size_t b = 0; b < nbc; ++b) {
    P->co.b1[b].nent = cent[b + 1] - cent[b];
    P->co.b1[b].nnz_out = cnnz[b + 1] - cnnz[b];
    P->co.cb[b].b2.n_sort = cicounts[2 * b + 1];
    P->info.n_dense_chunks += cicounts[2 * b];
    P->info.n_sort_groups += cicounts[2 * b + 1];
  }
  for (int k = 0; k < 4; ++k) P->info.nnz_by_category[k] = (int64_t)st2.nnz_cat[k];
  P->h_stats.nnz_cat[0] = st2.nnz_cat[0];
  for (size_t b = 0; b < P->batches.size(); ++b) {
    P->info.n_dense_chunks += icounts[2 * b];
    P->info.n_sort_groups += icounts[2 * b + 1];
    P->batches[b].n_sort = icounts[2 * b + 1];
  }
  float ms = 0;
  (void)hipEventElapsedTime(&ms, ev0, ev1);
  (void)hipEventDestroy(ev0);
  (void)hipEventDestroy(ev1);
  ev0 = ev1 = nullptr;
  if (st2.err & (ERR_STAGE_OVERFLOW | ERR_BIN_OVERFLOW)) {
    h->err = "device consistency check failed in the symbolic phase";
    return cleanup(MAGNUS_ERR_INTERNAL);
  }
  P->nnz_c = nnzc;

  magnus_plan_info_t& I = P->info;
  I.ip_total = (int64_t)P->h_stats.ip_total;
  I.flops = 2 * I.ip_total;
  I.nnz_c = nnzc;
  I.max_row_ip = (int64_t)P->h_stats.max_ip;
  for (int k = 0; k < 4; ++k) {
    I.rows_by_category[k] = (int64_t)P->h_stats.rows_cat[k];
    I.ip_by_category[k] = (int64_t)P->h_stats.ip_cat[k];
  }
  size_t held = 0;
  for (auto& a : P->allocs) held += a.n;
  I.plan_bytes = (int64_t)held;
  I.chunk_shift = P->shift;
  I.sort_max = (int32_t)P->sort_max;
  I.bin_dense_min = (int32_t)P->dense_min;
  I.tile_products = P->tile;
  I.symbolic_ms = ms;
  I.coarse_rows = P->co.nrows;
  I.coarse_chunks = P->co.nv;
  I.coarse_fine_chunks = P->co.nbins2;
  I.coarse_shift = P->co.nrows > 0 ? P->co.cshift : 0;
  I.run_binned = P->runs ? 1 : 0;
  I.n_runs = P->runs ? P->n_runs : 0;
  if (info) *info = I;
  *out = P;
  return MAGNUS_OK;
#undef PCHK
#undef SCHK
}

}  // namespace

extern "C" {

magnus_status_t magnus_plan(magnus_handle_t h, const magnus_csr_t* A, const magnus_csr_t* B,
                            void* stream, magnus_plan_t* out, magnus_plan_info_t* info) {
  if (!h || !out) return MAGNUS_ERR_INVALID_ARG;
  *out = nullptr;
  // when the allocator fails, row batches (Section 3.3's batching of rows
  // until the memory limit) are halved and the plan is made again, up to
  // four times, while a batch is still wider than the longest row
  magnus_status_t s = MAGNUS_OK;
  for (int64_t div = 1; div <= 16; div *= 2) {
    bool shrinkable = false;
    s = plan_once(h, A, B, stream, out, info, div, &shrinkable);
    if (s != MAGNUS_ERR_OOM || !shrinkable) break;
  }
  if (s == MAGNUS_OK && MG_GUARD) {
    s = plan_check_guards(*out);
    if (s != MAGNUS_OK) {
      magnus_plan_destroy(*out);
      *out = nullptr;
    }
  }
  return s;
}

magnus_status_t magnus_plan_get_info(magnus_plan_t P, magnus_plan_info_t* info) {
  if (!P || !info) return MAGNUS_ERR_INVALID_ARG;
  *info = P->info;
  return MAGNUS_OK;
}

magnus_status_t magnus_execute(magnus_handle_t h, magnus_plan_t P, const magnus_csr_t* A,
                               const magnus_csr_t* B, const magnus_csr_out_t* C, int64_t* nnz_out,
                               void* stream) {
  if (!h || !P || !C) return MAGNUS_ERR_INVALID_ARG;
  Mats M{};
  magnus_status_t s = make_mats(A, B, M);
  if (s != MAGNUS_OK) return s;
  if (M.n != P->n || A->nnz != P->a_nnz || B->nnz != P->b_nnz) return MAGNUS_ERR_SHAPE;
  if (C->nrows != A->nrows || C->ncols != B->ncols) return MAGNUS_ERR_SHAPE;
  if (C->val_type != A->val_type || C->col_type != B->col_type) return MAGNUS_ERR_DTYPE;
  if (C->rowptr_type != MAGNUS_I32 && C->rowptr_type != MAGNUS_I64) return MAGNUS_ERR_INVALID_ARG;
  if (nnz_out) *nnz_out = P->nnz_c;
  if (C->rowptr_type == MAGNUS_I32 && P->nnz_c > INT32_MAX) return MAGNUS_ERR_INDEX_OVERFLOW;
  if (C->capacity < P->nnz_c) return MAGNUS_ERR_CAPACITY;
  if (!C->rowptr || (P->nnz_c > 0 && (!C->col || !C->val))) return MAGNUS_ERR_INVALID_ARG;
  HIPCHK(hipSetDevice(h->device));
  P->M = M;  // same shapes; the pointers of this call are used
  P->st = (hipStream_t)stream;
  magnus_status_t r = run_rows(P, true, C->col, C->val);
  if (r != MAGNUS_OK) return r;
  if (P->nch > 0) {
    r = chunked_numeric(P, C->col, C->col_type == MAGNUS_I64, C->val);
    if (r != MAGNUS_OK) return r;
  }
  if (P->co.nrows > 0) {
    r = coarse_numeric(P, C->col, C->col_type == MAGNUS_I64, C->val);
    if (r != MAGNUS_OK) return r;
  }
  HIPCHK(launch_write_rowptr(P->crp, P->n, C->rowptr, C->rowptr_type == MAGNUS_I64, P->st));
  if (MG_GUARD) {
    // checked builds: the guards after the numeric phase (not inside a
    // graph capture, where the stream cannot be waited for)
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIPCHK(hipStreamIsCapturing(P->st, &cs));
    if (cs == hipStreamCaptureStatusNone) return plan_check_guards(P);
  }
  return MAGNUS_OK;
}

magnus_status_t magnus_plan_destroy(magnus_plan_t P) {
  if (!P) return MAGNUS_OK;
  plan_free_all(P);
  delete P;
  return MAGNUS_OK;
}

}  // extern "C"

namespace {

// Bytes of the three arrays of C as magnus_spgemm allocates them.
void csr_out_bytes(const magnus_csr_out_t* C, size_t b[3]) {
  b[0] = align256((size_t)(C->nrows + 1) * (C->rowptr_type == MAGNUS_I64 ? 8 : 4));
  b[1] = align256(std::max<size_t>(1, (size_t)C->capacity * (C->col_type == MAGNUS_I64 ? 8 : 4)));
  b[2] = align256(std::max<size_t>(1, (size_t)C->capacity * (C->val_type == MAGNUS_F64 ? 8 : 4)));
}

void csr_out_release(magnus_handle_s* h, magnus_csr_out_t* C, void* stream) {
  size_t b[3];
  csr_out_bytes(C, b);
  void* p[3] = {C->rowptr, C->col, C->val};
  for (int k = 0; k < 3; ++k) {
    if (!p[k]) continue;
    if (h->free_fn) h->free_fn(p[k], b[k], stream, h->alloc_ctx);
    else default_free(p[k], b[k], nullptr, nullptr);
  }
  C->rowptr = C->col = C->val = nullptr;
}

}  // namespace

extern "C" {

magnus_status_t magnus_spgemm(magnus_handle_t h, const magnus_csr_t* A, const magnus_csr_t* B,
                              int32_t c_rowptr_type, magnus_csr_out_t* C, void* stream) {
  if (!h || !C) return MAGNUS_ERR_INVALID_ARG;
  memset(C, 0, sizeof(*C));
  if (c_rowptr_type != MAGNUS_I32 && c_rowptr_type != MAGNUS_I64) return MAGNUS_ERR_INVALID_ARG;
  magnus_plan_t P = nullptr;
  magnus_status_t s = magnus_plan(h, A, B, stream, &P, nullptr);
  if (s != MAGNUS_OK) return s;
  const int64_t nnz = P->nnz_c;
  if (c_rowptr_type == MAGNUS_I32 && nnz > INT32_MAX) {
    magnus_plan_destroy(P);
    return MAGNUS_ERR_INDEX_OVERFLOW;
  }
  magnus_csr_out_t c{};
  c.nrows = A->nrows;
  c.ncols = B->ncols;
  c.capacity = nnz;
  c.rowptr_type = c_rowptr_type;
  c.col_type = B->col_type;
  c.val_type = A->val_type;
  size_t b[3];
  csr_out_bytes(&c, b);
  void* p[3] = {nullptr, nullptr, nullptr};
  for (int k = 0; k < 3; ++k) {
    p[k] = h->alloc_fn ? h->alloc_fn(b[k], stream, h->alloc_ctx) : default_alloc(b[k], nullptr, nullptr);
    if (!p[k]) break;
  }
  c.rowptr = p[0];
  c.col = p[1];
  c.val = p[2];
  if (!p[0] || !p[1] || !p[2]) {
    csr_out_release(h, &c, stream);
    magnus_plan_destroy(P);
    h->err = "the allocator returned no memory for C";
    return MAGNUS_ERR_OOM;
  }
  int64_t got = 0;
  s = magnus_execute(h, P, A, B, &c, &got, stream);
  // the plan's memory goes back to the allocator in stream order (or after
  // the device finishes, with the default hipFree)
  magnus_plan_destroy(P);
  if (s != MAGNUS_OK) {
    csr_out_release(h, &c, stream);
    return s;
  }
  *C = c;
  return MAGNUS_OK;
}

magnus_status_t magnus_csr_free(magnus_handle_t h, magnus_csr_out_t* C, void* stream) {
  if (!h || !C) return MAGNUS_ERR_INVALID_ARG;
  csr_out_release(h, C, stream);
  C->capacity = 0;
  return MAGNUS_OK;
}

magnus_status_t magnus_row_ip(magnus_handle_t h, const magnus_csr_t* A, const magnus_csr_t* B,
                              int64_t* ip_out, int64_t* ip_total, void* stream) {
  if (!h || !ip_out) return MAGNUS_ERR_INVALID_ARG;
  Mats M{};
  magnus_status_t s = make_mats(A, B, M);
  if (s != MAGNUS_OK) return s;
  HIPCHK(hipSetDevice(h->device));
  magnus_plan_s tmp;
  tmp.h = h;
  tmp.st = (hipStream_t)stream;
  const int64_t n = A->nrows;
  int64_t* minc = (int64_t*)palloc(&tmp, sizeof(int64_t) * std::max<int64_t>(n, 1));
  int64_t* maxc = (int64_t*)palloc(&tmp, sizeof(int64_t) * std::max<int64_t>(n, 1));
  int32_t* cls = (int32_t*)palloc(&tmp, sizeof(int32_t) * std::max<int64_t>(n, 1));
  int32_t* heavy = (int32_t*)palloc(&tmp, sizeof(int32_t) * std::max<int64_t>(n, 1));
  DevStats* stats = (DevStats*)palloc(&tmp, sizeof(DevStats));
  if (!minc || !maxc || !cls || !heavy || !stats) {
    plan_free_all(&tmp);
    return MAGNUS_ERR_OOM;
  }
  ClassParams cp{SORT_CAP + 1, 1 << 13, -1};
  hipError_t e = hipMemsetAsync(stats, 0, sizeof(DevStats), tmp.st);
  if (e == hipSuccess)
    e = launch_rowinfo(M, A->nnz, cp, ip_out, minc, maxc, cls, stats, heavy, tmp.st);
  DevStats hs{};
  magnus_status_t r = MAGNUS_OK;
  if (e != hipSuccess) r = fail_hip(h, e, "launch_rowinfo");
  else r = readback(&tmp, {{stats, sizeof(DevStats)}}, {&hs});
  plan_free_all(&tmp);
  if (r == MAGNUS_OK && ip_total) *ip_total = (int64_t)hs.ip_total;
  return r;
}

magnus_status_t magnus_profile_enable(magnus_handle_t h, int on) {
  if (!h) return MAGNUS_ERR_INVALID_ARG;
  h->prof = on != 0;
  return MAGNUS_OK;
}

magnus_status_t magnus_profile_read(magnus_handle_t h, magnus_kernel_stat_t* out, int max, int* n) {
  if (!h || !n || (max > 0 && !out)) return MAGNUS_ERR_INVALID_ARG;
  std::vector<magnus_kernel_stat_t> agg;
  magnus_status_t r = MAGNUS_OK;
  for (auto& rec : h->recs) {
    float ms = 0;
    if (hipEventSynchronize(rec.b) != hipSuccess ||
        hipEventElapsedTime(&ms, rec.a, rec.b) != hipSuccess)
      r = MAGNUS_ERR_HIP;
    (void)hipEventDestroy(rec.a);
    (void)hipEventDestroy(rec.b);
    magnus_kernel_stat_t* s = nullptr;
    for (auto& x : agg)
      if (strncmp(x.name, rec.name, sizeof(x.name) - 1) == 0) s = &x;
    if (!s) {
      magnus_kernel_stat_t z{};
      strncpy(z.name, rec.name, sizeof(z.name) - 1);
      agg.push_back(z);
      s = &agg.back();
    }
    s->launches += 1;
    s->ms += ms;
    s->bytes += rec.bytes;
  }
  h->recs.clear();
  *n = (int)agg.size();
  for (int i = 0; i < (int)agg.size() && i < max; ++i) out[i] = agg[i];
  if (r != MAGNUS_OK) h->err = "event timing failed";
  return r;
}

magnus_status_t magnus_stream_copy(magnus_handle_t h, void* dst, const void* src, size_t bytes,
                                   void* stream) {
  if (!h || (bytes > 0 && (!dst || !src))) return MAGNUS_ERR_INVALID_ARG;
  HIPCHK(hipSetDevice(h->device));
  ProfScope ps(h, (hipStream_t)stream, "stream_copy", 2.0 * (double)bytes);
  HIPCHK(launch_stream_copy(dst, src, bytes, (hipStream_t)stream));
  return MAGNUS_OK;
}

magnus_status_t magnus_exclusive_scan_i64(magnus_handle_t h, const int64_t* in, int64_t* out,
                                          int64_t n, int64_t* total, void* stream) {
  if (!h || n < 0 || (n > 0 && (!in || !out))) return MAGNUS_ERR_INVALID_ARG;
  HIPCHK(hipSetDevice(h->device));
  magnus_plan_s tmp;
  tmp.h = h;
  tmp.st = (hipStream_t)stream;
  void* t = palloc(&tmp, scan_temp_bytes(n) + 64);
  int64_t* dtot = (int64_t*)palloc(&tmp, 64);
  if (!t || !dtot) {
    plan_free_all(&tmp);
    return MAGNUS_ERR_OOM;
  }
  hipError_t e = scan_excl_i64(in, out, n, dtot, nullptr, t, tmp.st);
  magnus_status_t r = MAGNUS_OK;
  if (e != hipSuccess) r = fail_hip(h, e, "scan");
  else if (total) r = readback(&tmp, {{dtot, 8}}, {total});
  else {
    // the scratch is released below; wait for the scan to finish with it
    e = hipStreamSynchronize(tmp.st);
    if (e != hipSuccess) r = fail_hip(h, e, "sync");
  }
  plan_free_all(&tmp);
  return r;
}

}  // extern "C"
