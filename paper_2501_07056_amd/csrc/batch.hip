// Batches of independent products: the rows of all products are numbered one
// after another and each phase of the method (setup and categorisation,
// Section 3.1; precise symbolic count and prefix sum, Section 2.1; numeric
// accumulation of SORT and DENSE rows, Algorithms 1 and 2) is one set of
// launches over the whole batch.  In the numeric phase every stage (one SORT
// size class, or the DENSE rows) is one grid over the rows of all products,
// or, on request, one persistent kernel whose waves or workgroups pull
// (product, row range) tiles from a device counter.  Products with CHUNKED
// rows (Algorithm 3) are planned on their own.  The numeric launches of the
// whole batch, those of the CHUNKED products included, are captured once into
// a HIP graph whose stages are independent branches (they write disjoint rows
// of C), so the device overlaps them; replays read a pointer table refreshed
// before each launch.
#include <array>

#include "runtime_int.h"

using namespace mgrt;

struct magnus_batch_plan_s {
  magnus_plan_s core;  // allocations, pinned readback buffer, stream
  int32_t nmat = 0;
  int64_t N = 0;       // rows over all products
  Mats T{};            // index / value types of the batch (pointers unused)
  // per product (host)
  std::vector<int64_t> n, k, m, annz, bnnz, row0, nnz;
  std::vector<magnus_plan_s*> alone;  // products planned on their own
  std::vector<int32_t> h_flags;
  // device
  MatEnt* d_tab = nullptr;
  int64_t* d_row0 = nullptr;
  int32_t* d_row0_i32 = nullptr;
  int32_t* mat_of_row = nullptr;
  int32_t* flags = nullptr;
  int64_t* mat_off = nullptr;
  RowSrc src{};
  // pinned staging of the pointer table, and the event that frees it
  MatEnt* h_tab = nullptr;
  hipEvent_t tab_ev = nullptr;
  // captured numeric launches: the capture stream, the branch streams and
  // their events, and the CHUNKED products' buffers the graph was made with
  hipStream_t cap_st = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<hipStream_t> br_st;
  std::vector<hipEvent_t> br_ev;
  hipEvent_t fork_ev = nullptr;
  std::vector<std::array<const void*, 9>> cap_ptrs;
  bool cap_persistent = false;   // the stage kind the graph was captured with
  unsigned int* work = nullptr;  // one tile counter per stage
  double numeric_bytes = 0;
};

namespace {

void batch_free(magnus_batch_plan_s* P) {
  for (auto* a : P->alone)
    if (a) magnus_plan_destroy(a);
  P->alone.clear();
  if (P->exec) (void)hipGraphExecDestroy(P->exec);
  if (P->graph) (void)hipGraphDestroy(P->graph);
  if (P->cap_st) (void)hipStreamDestroy(P->cap_st);
  for (auto s_ : P->br_st) (void)hipStreamDestroy(s_);
  for (auto e_ : P->br_ev) (void)hipEventDestroy(e_);
  if (P->fork_ev) (void)hipEventDestroy(P->fork_ev);
  if (P->tab_ev) {
    (void)hipEventSynchronize(P->tab_ev);
    (void)hipEventDestroy(P->tab_ev);
  }
  if (P->h_tab) P->core.h->put_pinned(P->h_tab);
  plan_free_all(&P->core);
  delete P;
}

constexpr int NBRANCH = 4;

// The numeric launches of the batch.  Eager: every stage in stream order on
// st, then the CHUNKED products.  Branched (for the graph): the stages and
// the CHUNKED products are spread over NBRANCH streams forked from st and
// joined back into it.  persistent: each stage is a persistent kernel
// pulling tiles from its counter in P->work (plain grids otherwise).
magnus_status_t batch_numeric(magnus_batch_plan_s* P, hipStream_t st, bool branched,
                              bool persistent, int32_t count, const magnus_csr_t* A,
                              const magnus_csr_t* B, const magnus_csr_out_t* Cout) {
  magnus_plan_s* C = &P->core;
  magnus_handle_s* h = C->h;
  // the stages' tile counters start at 0 (a kernel, not a memset node)
  HIPCHK(launch_fill_i64((int64_t*)P->work, (NCLS + 2) / 2, 0, st));
  std::vector<hipStream_t> used;
  int next = 0;
  auto stream_for = [&](hipStream_t& s) -> hipError_t {
    if (!branched) {
      s = st;
      return hipSuccess;
    }
    s = P->br_st[next % NBRANCH];
    if (next < NBRANCH) {
      hipError_t e = hipStreamWaitEvent(s, P->fork_ev, 0);
      if (e != hipSuccess) return e;
      used.push_back(s);
    }
    ++next;
    return hipSuccess;
  };
  if (branched) HIPCHK(hipEventRecord(P->fork_ev, st));
  for (int c = 0; c < NSORT_CLS; ++c) {
    const int64_t cnt = C->h_list_off[c + 1] - C->h_list_off[c];
    if (cnt <= 0) continue;
    hipStream_t s = nullptr;
    HIPCHK(stream_for(s));
    HIPCHK(launch_sort_rows(P->T, P->src, c, true, C->list, C->h_list_off[c], cnt, C->minc,
                            C->colbits, C->crp, C->crp, C->stats, s,
                            persistent ? P->work + c : nullptr));
  }
  const int64_t nd = C->h_list_off[CLS_DENSE + 1] - C->h_list_off[CLS_DENSE];
  if (nd > 0) {
    hipStream_t s = nullptr;
    HIPCHK(stream_for(s));
    HIPCHK(launch_dense_rows(P->T, P->src, true, C->list, C->h_list_off[CLS_DENSE], nd, C->minc,
                             C->maxc, C->dense_shift, C->dense_block, C->crp, C->crp, s,
                             persistent ? P->work + CLS_DENSE : nullptr));
  }
  for (int32_t b = 0; b < count; ++b) {
    if (!P->alone[b]) continue;
    hipStream_t s = nullptr;
    HIPCHK(stream_for(s));
    int64_t nz = 0;
    magnus_status_t r = magnus_execute(h, P->alone[b], &A[b], &B[b], &Cout[b], &nz, s);
    if (r != MAGNUS_OK) return r;
  }
  for (size_t k = 0; k < used.size(); ++k) {
    HIPCHK(hipEventRecord(P->br_ev[k], used[k]));
    HIPCHK(hipStreamWaitEvent(st, P->br_ev[k], 0));
  }
  HIPCHK(launch_write_rowptr_batch(P->src, C->crp, P->N, P->nmat, P->flags, st));
  return MAGNUS_OK;
}

// The buffers of the CHUNKED products (their launches take them directly).
std::vector<std::array<const void*, 9>> alone_ptrs(const magnus_batch_plan_s* P, int32_t count,
                                                   const magnus_csr_t* A, const magnus_csr_t* B,
                                                   const magnus_csr_out_t* Cout) {
  std::vector<std::array<const void*, 9>> v;
  for (int32_t b = 0; b < count; ++b)
    if (P->alone[b])
      v.push_back({A[b].rowptr, A[b].col, A[b].val, B[b].rowptr, B[b].col, B[b].val,
                   Cout[b].rowptr, Cout[b].col, Cout[b].val});
  return v;
}

}  // namespace

extern "C" {

magnus_status_t magnus_batch_plan(magnus_handle_t h, int32_t count, const magnus_csr_t* A,
                                  const magnus_csr_t* B, const int32_t* sort_max, void* stream,
                                  magnus_batch_plan_t* out, int64_t* nnz_out,
                                  magnus_plan_info_t* info) {
  if (!h || !out || count < 1 || !A || !B || !nnz_out) return MAGNUS_ERR_INVALID_ARG;
  *out = nullptr;
  if (h->opts.deterministic) {
    h->err = "deterministic mode covers single products (magnus_plan) only";
    return MAGNUS_ERR_INVALID_ARG;
  }
  // descriptors, shared types, row numbering
  std::vector<Mats> mats(count);
  int64_t N = 0, annz_tot = 0;
  for (int32_t b = 0; b < count; ++b) {
    magnus_status_t s = make_mats(&A[b], &B[b], mats[b]);
    if (s != MAGNUS_OK) return s;
    if (b > 0 && (mats[b].rp64 != mats[0].rp64 || mats[b].col64 != mats[0].col64 ||
                  mats[b].f64 != mats[0].f64))
      return MAGNUS_ERR_DTYPE;
    N += A[b].nrows;
    annz_tot += A[b].nnz;
    if (N > INT32_MAX) return MAGNUS_ERR_INDEX_OVERFLOW;
  }
  if (sort_max)
    for (int32_t b = 0; b < count; ++b)
      if (sort_max[b] < 1) return MAGNUS_ERR_INVALID_ARG;
  HIPCHK(hipSetDevice(h->device));

  magnus_batch_plan_s* P = new magnus_batch_plan_s();
  magnus_plan_s* C = &P->core;
  C->h = h;
  C->st = (hipStream_t)stream;
  P->nmat = count;
  P->N = N;
  P->T = mats[0];
  C->n = N;
  C->M = mats[0];
  const magnus_options_t& o = h->opts;
  const int lds = o.lds_bytes > 0 ? std::min(o.lds_bytes, h->lds_max) : h->lds_max;
  C->lds_budget = lds;
  C->shift = o.chunk_shift > 0 ? std::min(o.chunk_shift, 16) : default_shift(P->T.f64, lds);
  C->sort_max = o.sort_max > 0 ? std::min<int64_t>(o.sort_max, SORT_CAP + 1) : SORT_CAP + 1;
  C->dense_block = (o.dense_block == 512 || o.dense_block == 1024) ? o.dense_block : 256;
  C->s_rp = P->T.rp64 ? 8 : 4;
  C->s_col = P->T.col64 ? 8 : 4;
  C->s_val = P->T.f64 ? 8 : 4;

  auto cleanup = [&](magnus_status_t st) {
    batch_free(P);
    return st;
  };
#define BCHK(expr)                                                 \
  do {                                                             \
    hipError_t e_ = (expr);                                        \
    if (e_ != hipSuccess) return cleanup(fail_hip(h, e_, #expr));  \
  } while (0)
#define BSCHK(expr)                              \
  do {                                           \
    magnus_status_t s_ = (expr);                 \
    if (s_ != MAGNUS_OK) return cleanup(s_);     \
  } while (0)

  P->n.resize(count);
  P->k.resize(count);
  P->m.resize(count);
  P->annz.resize(count);
  P->bnnz.resize(count);
  P->row0.resize(count + 1);
  P->nnz.assign(count, 0);
  P->alone.assign(count, nullptr);
  P->h_flags.assign(count, 0);
  P->h_tab = (MatEnt*)h->get_pinned(sizeof(MatEnt) * count);
  if (!P->h_tab) return cleanup(MAGNUS_ERR_OOM);
  std::vector<int32_t> row0_i32(count + 1);
  int64_t r0 = 0;
  for (int32_t b = 0; b < count; ++b) {
    P->n[b] = A[b].nrows;
    P->k[b] = A[b].ncols;
    P->m[b] = B[b].ncols;
    P->annz[b] = A[b].nnz;
    P->bnnz[b] = B[b].nnz;
    P->row0[b] = r0;
    row0_i32[b] = (int32_t)r0;
    MatEnt& E = P->h_tab[b];
    memset(&E, 0, sizeof(E));
    E.arp = A[b].rowptr;
    E.acol = A[b].col;
    E.aval = A[b].val;
    E.brp = B[b].rowptr;
    E.bcol = B[b].col;
    E.bval = B[b].val;
    E.row0 = r0;
    E.nrows = A[b].nrows;
    E.sort_max = sort_max ? std::min<int64_t>(sort_max[b], SORT_CAP + 1) : C->sort_max;
    E.dense_max = (int64_t)1 << C->shift;
    E.mcols = B[b].ncols;
    E.crp_out64 = 1;
    r0 += A[b].nrows;
  }
  P->row0[count] = r0;
  row0_i32[count] = (int32_t)r0;

  const int64_t n1 = std::max<int64_t>(N, 1);
  P->d_tab = (MatEnt*)palloc(C, sizeof(MatEnt) * count);
  P->d_row0 = (int64_t*)palloc(C, sizeof(int64_t) * (count + 1));
  P->d_row0_i32 = (int32_t*)palloc(C, sizeof(int32_t) * (count + 1));
  P->mat_of_row = (int32_t*)palloc(C, sizeof(int32_t) * n1);
  P->flags = (int32_t*)palloc(C, sizeof(int32_t) * count);
  P->mat_off = (int64_t*)palloc(C, sizeof(int64_t) * (count + 1));
  P->work = (unsigned int*)palloc(C, sizeof(unsigned int) * (NCLS + 2));
  C->stats = (DevStats*)palloc(C, sizeof(DevStats));
  C->ip = (int64_t*)palloc(C, sizeof(int64_t) * n1);
  C->minc = (int64_t*)palloc(C, sizeof(int64_t) * n1);
  C->maxc = (int64_t*)palloc(C, sizeof(int64_t) * n1);
  C->crp = (int64_t*)palloc(C, sizeof(int64_t) * (N + 1));
  C->cls = (int32_t*)palloc(C, sizeof(int32_t) * n1);
  C->list = (int32_t*)palloc(C, sizeof(int32_t) * n1);
  C->list_off = (int64_t*)palloc(C, sizeof(int64_t) * (NCLS + 1));
  C->temp = palloc(C, std::max(classify_temp_bytes(N), scan_temp_bytes(N + 1)) + 1024);
  if (!P->d_tab || !P->d_row0 || !P->d_row0_i32 || !P->mat_of_row || !P->flags || !P->mat_off ||
      !P->work || !C->stats || !C->ip || !C->minc || !C->maxc || !C->crp || !C->cls || !C->list ||
      !C->list_off || !C->temp)
    return cleanup(MAGNUS_ERR_OOM);
  P->src.one = P->h_tab[0];
  P->src.tab = P->d_tab;
  P->src.mat_of_row = P->mat_of_row;

  hipEvent_t ev0, ev1;
  BCHK(hipEventCreate(&ev0));
  BCHK(hipEventCreate(&ev1));
  BCHK(hipEventRecord(ev0, C->st));
  // the pinned table is read by this copy: the event guards its reuse
  BCHK(hipMemcpyAsync(P->d_tab, P->h_tab, sizeof(MatEnt) * count, hipMemcpyHostToDevice, C->st));
  BCHK(hipMemcpyAsync(P->d_row0, P->row0.data(), sizeof(int64_t) * (count + 1),
                      hipMemcpyHostToDevice, C->st));
  BCHK(hipMemcpyAsync(P->d_row0_i32, row0_i32.data(), sizeof(int32_t) * (count + 1),
                      hipMemcpyHostToDevice, C->st));
  BCHK(hipEventCreate(&P->tab_ev));
  BCHK(hipEventRecord(P->tab_ev, C->st));
  BCHK(hipMemsetAsync(C->stats, 0, sizeof(DevStats), C->st));
  BCHK(hipMemsetAsync(P->flags, 0, sizeof(int32_t) * count, C->st));
  if (o.validate)
    for (int32_t b = 0; b < count; ++b)
      BCHK(launch_validate(mats[b], A[b].nnz, B[b].nnz, C->stats, C->st));
  BCHK(launch_mat_of_row(P->d_row0, count, N, P->mat_of_row, C->st));
  ClassParams cp{};
  cp.sort_max = C->sort_max;
  cp.dense_max = (int64_t)1 << C->shift;
  cp.force = (o.force_category >= 0 && o.force_category <= 1) ? o.force_category : -1;
  {
    ProfScope ps(h, C->st, "batch rowinfo (setup)",
                 (double)(N + count) * C->s_rp + (double)annz_tot * (3 * C->s_col + 2 * C->s_rp) +
                     (double)N * 32);
    BCHK(launch_rowinfo_batch(P->T, P->src, N, annz_tot, cp, C->ip, C->minc, C->maxc, C->cls,
                              C->stats, P->flags, C->st));
  }
  BCHK(launch_classify(C->cls, N, C->list, C->list_off, C->temp, C->st));
  // the host vectors' storage is read by the copies above: wait here, before
  // they can go out of scope
  BSCHK(readback(C, {{C->stats, sizeof(DevStats)},
                     {C->list_off, sizeof(int64_t) * (NCLS + 1)},
                     {P->flags, sizeof(int32_t) * count}},
                 {&C->h_stats, C->h_list_off, P->h_flags.data()}));
  if (C->h_stats.err & ERR_INVALID_CSR) return cleanup(MAGNUS_ERR_INVALID_CSR);
  C->colbits = bits_for((int64_t)std::max<unsigned long long>(1, C->h_stats.range_cat[0]));
  C->dense_shift = dense_rows_shift(C->h_stats.range_cat[1], C->shift);
  bool any_alone = false;
  for (int32_t b = 0; b < count; ++b) any_alone |= P->h_flags[b] != 0;
  if (any_alone) {
    // products with CHUNKED rows: plan them alone, drop their rows here
    for (int32_t b = 0; b < count; ++b) {
      if (!P->h_flags[b]) continue;
      magnus_plan_info_t bi{};
      BSCHK(magnus_plan(h, &A[b], &B[b], stream, &P->alone[b], &bi));
      P->nnz[b] = bi.nnz_c;
      for (int c = 0; c < 4; ++c) P->core.info.nnz_by_category[c] += bi.nnz_by_category[c];
    }
    BCHK(launch_drop_flagged(P->flags, P->mat_of_row, N, C->cls, C->st));
    BCHK(launch_classify(C->cls, N, C->list, C->list_off, C->temp, C->st));
    BSCHK(readback(C, {{C->list_off, sizeof(int64_t) * (NCLS + 1)}}, {C->h_list_off}));
  }

  // precise symbolic phase over the batch, then the row offsets and the
  // first offset of every product
  const DevStats& S = C->h_stats;
  BCHK(launch_fill_i64(C->crp, N + 1, 0, C->st));
  {
    ProfScope ps(h, C->st, "batch sort_rows (symbolic)",
                 (double)S.ip_cat[0] * C->s_col + (double)S.ent_cat[0] * (C->s_col + 2 * C->s_rp) +
                     (double)S.rows_cat[0] * 24);
    for (int c = 0; c < NSORT_CLS; ++c) {
      const int64_t cnt = C->h_list_off[c + 1] - C->h_list_off[c];
      if (cnt > 0)
        BCHK(launch_sort_rows(P->T, P->src, c, false, C->list, C->h_list_off[c], cnt, C->minc,
                              C->colbits, C->crp, C->crp, C->stats, C->st));
    }
  }
  const int64_t nd = C->h_list_off[CLS_DENSE + 1] - C->h_list_off[CLS_DENSE];
  {
    ProfScope ps(h, C->st, "batch dense_rows (symbolic)",
                 (double)S.ip_cat[1] * C->s_col + (double)S.ent_cat[1] * (C->s_col + 2 * C->s_rp) +
                     (double)S.rows_cat[1] * 32);
    if (nd > 0)
      BCHK(launch_dense_rows(P->T, P->src, false, C->list, C->h_list_off[CLS_DENSE], nd, C->minc,
                             C->maxc, C->dense_shift, C->dense_block, C->crp, C->crp, C->st));
  }
  BCHK(launch_cat_nnz(C->cls, C->crp, N, C->stats, C->st));
  BCHK(scan_excl_i64(C->crp, C->crp, N + 1, nullptr, nullptr, C->temp, C->st));
  BCHK(launch_gather_rows(C->crp, P->d_row0_i32, count + 1, P->mat_off, C->st));
  BCHK(hipEventRecord(ev1, C->st));
  std::vector<int64_t> off(count + 1, 0);
  DevStats st2{};
  BSCHK(readback(C, {{P->mat_off, sizeof(int64_t) * (count + 1)}, {C->stats, sizeof(DevStats)}},
                 {off.data(), &st2}));
  float ms = 0;
  (void)hipEventElapsedTime(&ms, ev0, ev1);
  (void)hipEventDestroy(ev0);
  (void)hipEventDestroy(ev1);
  if (st2.err & ERR_STAGE_OVERFLOW) {
    h->err = "device consistency check failed in the batched symbolic phase";
    return cleanup(MAGNUS_ERR_INTERNAL);
  }
  int64_t nnz_tot = 0;
  for (int32_t b = 0; b < count; ++b) {
    if (!P->h_flags[b]) P->nnz[b] = off[b + 1] - off[b];
    nnz_out[b] = P->nnz[b];
    nnz_tot += P->nnz[b];
  }

  magnus_plan_info_t& I = C->info;
  I.ip_total = (int64_t)S.ip_total;
  I.flops = 2 * I.ip_total;
  I.nnz_c = nnz_tot;
  I.max_row_ip = (int64_t)S.max_ip;
  for (int c = 0; c < 4; ++c) {
    I.rows_by_category[c] = (int64_t)S.rows_cat[c];
    I.ip_by_category[c] = (int64_t)S.ip_cat[c];
    I.nnz_by_category[c] += (int64_t)st2.nnz_cat[c];
  }
  size_t held = 0;
  for (auto& a : C->allocs) held += a.n;
  for (auto* a : P->alone)
    if (a) held += (size_t)a->info.plan_bytes;
  I.plan_bytes = (int64_t)held;
  I.chunk_shift = C->shift;
  I.sort_max = (int32_t)C->sort_max;
  I.symbolic_ms = ms;
  // algorithmic bytes of the numeric launches (products, A entries, rows,
  // outputs), for the execute's profile record
  const double cv = C->s_col + C->s_val;
  P->numeric_bytes = (double)(S.ip_cat[0] + S.ip_cat[1]) * cv +
                     (double)(S.ent_cat[0] + S.ent_cat[1]) * (cv + 2 * C->s_rp) +
                     (double)(S.rows_cat[0] + S.rows_cat[1]) * 24 +
                     (double)(st2.nnz_cat[0] + st2.nnz_cat[1]) * cv + (double)(N + count) * 16;
  if (info) *info = I;
  *out = P;
  return MAGNUS_OK;
#undef BCHK
#undef BSCHK
}

magnus_status_t magnus_batch_execute(magnus_handle_t h, magnus_batch_plan_t P, int32_t count,
                                     const magnus_csr_t* A, const magnus_csr_t* B,
                                     const magnus_csr_out_t* Cout, int32_t mode, void* stream) {
  if (!h || !P || !A || !B || !Cout || count != P->nmat) return MAGNUS_ERR_INVALID_ARG;
  const bool persistent = (mode & MAGNUS_BATCH_PERSISTENT) != 0;
  mode &= ~MAGNUS_BATCH_PERSISTENT;
  if (mode != MAGNUS_BATCH_GRAPH && mode != MAGNUS_BATCH_EAGER) return MAGNUS_ERR_INVALID_ARG;
  magnus_plan_s* C = &P->core;
  // every descriptor is checked before anything is launched
  for (int32_t b = 0; b < count; ++b) {
    Mats M{};
    magnus_status_t s = make_mats(&A[b], &B[b], M);
    if (s != MAGNUS_OK) return s;
    if (M.rp64 != P->T.rp64 || M.col64 != P->T.col64 || M.f64 != P->T.f64) return MAGNUS_ERR_DTYPE;
    if (A[b].nrows != P->n[b] || A[b].ncols != P->k[b] || B[b].ncols != P->m[b] ||
        A[b].nnz != P->annz[b] || B[b].nnz != P->bnnz[b])
      return MAGNUS_ERR_SHAPE;
    const magnus_csr_out_t& O = Cout[b];
    if (O.nrows != P->n[b] || O.ncols != P->m[b]) return MAGNUS_ERR_SHAPE;
    if (O.val_type != A[b].val_type || O.col_type != B[b].col_type) return MAGNUS_ERR_DTYPE;
    if (O.rowptr_type != MAGNUS_I32 && O.rowptr_type != MAGNUS_I64) return MAGNUS_ERR_INVALID_ARG;
    if (O.capacity < P->nnz[b]) return MAGNUS_ERR_CAPACITY;
    if (O.rowptr_type == MAGNUS_I32 && P->nnz[b] > INT32_MAX) return MAGNUS_ERR_INDEX_OVERFLOW;
    if (!O.rowptr || (P->nnz[b] > 0 && (!O.col || !O.val))) return MAGNUS_ERR_INVALID_ARG;
  }
  HIPCHK(hipSetDevice(h->device));
  hipStream_t st = (hipStream_t)stream;
  // the previous call's table copy must have read the pinned table
  HIPCHK(hipEventSynchronize(P->tab_ev));
  for (int32_t b = 0; b < count; ++b) {
    MatEnt& E = P->h_tab[b];
    E.arp = A[b].rowptr;
    E.acol = A[b].col;
    E.aval = A[b].val;
    E.brp = B[b].rowptr;
    E.bcol = B[b].col;
    E.bval = B[b].val;
    E.ccol = Cout[b].col;
    E.cval = Cout[b].val;
    E.crp_out = Cout[b].rowptr;
    E.crp_out64 = Cout[b].rowptr_type == MAGNUS_I64;
  }
  HIPCHK(hipMemcpyAsync(P->d_tab, P->h_tab, sizeof(MatEnt) * count, hipMemcpyHostToDevice, st));
  HIPCHK(hipEventRecord(P->tab_ev, st));
  {
    ProfScope ps(h, st, mode == MAGNUS_BATCH_GRAPH ? "batch execute (graph)" : "batch execute",
                 P->numeric_bytes);
    if (mode == MAGNUS_BATCH_EAGER) {
      magnus_status_t r = batch_numeric(P, st, false, persistent, count, A, B, Cout);
      if (r != MAGNUS_OK) return r;
    } else {
      // the CHUNKED products' launches hold their buffers: a call with other
      // buffers for them, or with the other stage kind, captures the graph
      // again
      const auto ptrs = alone_ptrs(P, count, A, B, Cout);
      if (P->exec && (ptrs != P->cap_ptrs || persistent != P->cap_persistent)) {
        (void)hipGraphExecDestroy(P->exec);
        (void)hipGraphDestroy(P->graph);
        P->exec = nullptr;
        P->graph = nullptr;
      }
      if (!P->exec) {
        // capture on a private stream: nothing runs while capturing, and the
        // caller's stream may be the null stream, which cannot be captured
        if (!P->cap_st) HIPCHK(hipStreamCreateWithFlags(&P->cap_st, hipStreamNonBlocking));
        if (P->br_st.empty()) {
          for (int k = 0; k < NBRANCH; ++k) {
            hipStream_t bs = nullptr;
            hipEvent_t be = nullptr;
            HIPCHK(hipStreamCreateWithFlags(&bs, hipStreamNonBlocking));
            P->br_st.push_back(bs);
            HIPCHK(hipEventCreateWithFlags(&be, hipEventDisableTiming));
            P->br_ev.push_back(be);
          }
          HIPCHK(hipEventCreateWithFlags(&P->fork_ev, hipEventDisableTiming));
        }
        // no profiling events inside the captured launches
        const bool prof = h->prof;
        h->prof = false;
        HIPCHK(hipStreamBeginCapture(P->cap_st, hipStreamCaptureModeRelaxed));
        magnus_status_t r = batch_numeric(P, P->cap_st, true, persistent, count, A, B, Cout);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(P->cap_st, &g);
        h->prof = prof;
        if (r != MAGNUS_OK) {
          if (g) (void)hipGraphDestroy(g);
          return r;
        }
        if (e != hipSuccess) return fail_hip(h, e, "hipStreamEndCapture");
        P->graph = g;
        HIPCHK(hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0));
        P->cap_ptrs = ptrs;
        P->cap_persistent = persistent;
      }
      HIPCHK(hipGraphLaunch(P->exec, st));
    }
  }
  (void)C;
  if (MG_GUARD) {
    // checked builds: the guards of the batch's and its alone products' plans
    HIPCHK(hipStreamSynchronize(st));
    magnus_status_t g = plan_check_guards(&P->core);
    for (size_t b = 0; g == MAGNUS_OK && b < P->alone.size(); ++b)
      if (P->alone[b]) g = plan_check_guards(P->alone[b]);
    return g;
  }
  return MAGNUS_OK;
}

magnus_status_t magnus_batch_bound(magnus_handle_t h, int32_t count, const magnus_csr_t* A,
                                   const magnus_csr_t* B, void* stream, int64_t* ip_out,
                                   int64_t* nnz_bound_out) {
  if (!h || count < 1 || !A || !B || !ip_out || !nnz_bound_out) return MAGNUS_ERR_INVALID_ARG;
  Mats T{};
  int64_t N = 0, annz = 0;
  for (int32_t b = 0; b < count; ++b) {
    Mats M{};
    magnus_status_t s = make_mats(&A[b], &B[b], M);
    if (s != MAGNUS_OK) return s;
    if (b == 0) T = M;
    else if (M.rp64 != T.rp64 || M.col64 != T.col64 || M.f64 != T.f64) return MAGNUS_ERR_DTYPE;
    N += A[b].nrows;
    annz += A[b].nnz;
    if (N > INT32_MAX) return MAGNUS_ERR_INDEX_OVERFLOW;
  }
  HIPCHK(hipSetDevice(h->device));
  magnus_plan_s tmp;
  tmp.h = h;
  tmp.st = (hipStream_t)stream;
  std::vector<MatEnt> tab(count);
  std::vector<int64_t> row0(count + 1);
  std::vector<int32_t> row0_i32(count + 1);
  int64_t r0 = 0;
  for (int32_t b = 0; b < count; ++b) {
    MatEnt& E = tab[b];
    memset(&E, 0, sizeof(E));
    E.arp = A[b].rowptr;
    E.acol = A[b].col;
    E.brp = B[b].rowptr;
    E.bcol = B[b].col;
    E.row0 = r0;
    E.nrows = A[b].nrows;
    E.mcols = B[b].ncols;
    row0[b] = r0;
    row0_i32[b] = (int32_t)r0;
    r0 += A[b].nrows;
  }
  row0[count] = r0;
  row0_i32[count] = (int32_t)r0;
  MatEnt* d_tab = (MatEnt*)palloc(&tmp, sizeof(MatEnt) * count);
  int64_t* d_row0 = (int64_t*)palloc(&tmp, sizeof(int64_t) * (count + 1));
  int32_t* d_row0_i32 = (int32_t*)palloc(&tmp, sizeof(int32_t) * (count + 1));
  int32_t* mor = (int32_t*)palloc(&tmp, sizeof(int32_t) * std::max<int64_t>(N, 1));
  int64_t* vip = (int64_t*)palloc(&tmp, sizeof(int64_t) * (N + 1));
  int64_t* vbd = (int64_t*)palloc(&tmp, sizeof(int64_t) * (N + 1));
  int64_t* out = (int64_t*)palloc(&tmp, sizeof(int64_t) * 2 * (count + 1));
  void* temp = palloc(&tmp, scan_temp_bytes(N + 1) + 1024);
  magnus_status_t r = MAGNUS_OK;
  if (!d_tab || !d_row0 || !d_row0_i32 || !mor || !vip || !vbd || !out || !temp) {
    r = MAGNUS_ERR_OOM;
  } else {
    RowSrc src{};
    src.tab = d_tab;
    src.mat_of_row = mor;
    hipError_t e = hipMemcpyAsync(d_tab, tab.data(), sizeof(MatEnt) * count,
                                  hipMemcpyHostToDevice, tmp.st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(d_row0, row0.data(), sizeof(int64_t) * (count + 1),
                         hipMemcpyHostToDevice, tmp.st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(d_row0_i32, row0_i32.data(), sizeof(int32_t) * (count + 1),
                         hipMemcpyHostToDevice, tmp.st);
    if (e == hipSuccess) e = launch_fill_i64(vip + N, 1, 0, tmp.st);
    if (e == hipSuccess) e = launch_fill_i64(vbd + N, 1, 0, tmp.st);
    if (e == hipSuccess) e = launch_mat_of_row(d_row0, count, N, mor, tmp.st);
    if (e == hipSuccess) {
      ProfScope ps(h, tmp.st, "batch row_bound", (double)annz * (T.col64 ? 8 : 4) * 3 +
                                                     (double)N * 20);
      e = launch_row_bound(T, src, N, annz, vip, vbd, tmp.st);
    }
    if (e == hipSuccess) e = scan_excl_i64(vip, vip, N + 1, nullptr, nullptr, temp, tmp.st);
    if (e == hipSuccess) e = scan_excl_i64(vbd, vbd, N + 1, nullptr, nullptr, temp, tmp.st);
    if (e == hipSuccess) e = launch_gather_rows(vip, d_row0_i32, count + 1, out, tmp.st);
    if (e == hipSuccess) e = launch_gather_rows(vbd, d_row0_i32, count + 1, out + count + 1, tmp.st);
    std::vector<int64_t> h_out(2 * (count + 1));
    if (e != hipSuccess) r = fail_hip(h, e, "magnus_batch_bound");
    else r = readback(&tmp, {{out, sizeof(int64_t) * 2 * (count + 1)}}, {h_out.data()});
    if (r == MAGNUS_OK)
      for (int32_t b = 0; b < count; ++b) {
        ip_out[b] = h_out[b + 1] - h_out[b];
        nnz_bound_out[b] = h_out[count + 1 + b + 1] - h_out[count + 1 + b];
      }
  }
  if (r != MAGNUS_OK) (void)hipStreamSynchronize(tmp.st);
  plan_free_all(&tmp);
  return r;
}

magnus_status_t magnus_batch_plan_destroy(magnus_batch_plan_t P) {
  if (!P) return MAGNUS_OK;
  batch_free(P);
  return MAGNUS_OK;
}

}  // extern "C"
