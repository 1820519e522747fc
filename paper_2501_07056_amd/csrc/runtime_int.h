// Host-side state shared by the runtime's translation units: the handle, the
// plan of one product, allocation, readback and profiling helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "kernels.h"
#include "magnus.h"

// default write-out order of the one-level CHUNKED reorder (1: chunk order)
#ifndef MG_SORTED_OUT
#define MG_SORTED_OUT 0
#endif
// the coarse level's first reorder writes in chunk order when rows span more
// coarse chunks than this (short runs per chunk in the expansion order;
// uniform 2^26 columns, 66 coarse chunks: 133.4 -> 124.0 ms per step, 2^27:
// 158.2 -> 132.2); the symbolic phase's reorder (columns only) gains from
// it only further on
#ifndef MG_COARSE_SORTED_MIN
#define MG_COARSE_SORTED_MIN 32
#endif
#ifndef MG_COARSE_SORTED_SYM_MIN
#define MG_COARSE_SORTED_SYM_MIN 512
#endif
// products per tile of the level-2 reorder (1024 threads each; uniform 2^28
// columns: fine_scatter 30.2 -> 24.3 ms against 2048 at 256 threads with a
// second staged copy)
#ifndef MG_L2_TILE
#define MG_L2_TILE 4096
#endif
// below this many products per coarse chunk on average, level-2 tiles of
// 2048 at 256 threads
#ifndef MG_L2_SMALL
#define MG_L2_SMALL 2048
#endif
// coarse chunks with at least 2^cshift / MG_BITMAP_DENSITY products (on
// average) are counted with a bitmap in the symbolic phase (measured on
// uniform rows: the bitmap is faster at 1/128, the count-mode accumulators
// at 1/1024)
#ifndef MG_BITMAP_DENSITY
#define MG_BITMAP_DENSITY 512
#endif

using namespace mg;

struct magnus_handle_s {
  struct PRec {
    const char* name;
    hipEvent_t a, b;
    double bytes;
  };
  bool prof = false;
  std::vector<PRec> recs;
  int device = 0;
  magnus_options_t opts{};
  magnus_alloc_fn alloc_fn = nullptr;
  magnus_free_fn free_fn = nullptr;
  void* alloc_ctx = nullptr;
  std::string err;
  // device bytes held by this handle's plans, and an optional cap on them: an
  // allocation past the cap fails like any other (0: no cap).  A serving
  // loop caps the planning of each group at the memory reserved for it.
  std::atomic<int64_t> plan_live{0};
  int64_t plan_cap = 0;
  int lds_max = 65536;
  int cus = 0;
  // pinned host buffers, kept until the handle is destroyed: freeing pinned
  // memory waits for the whole device, which would stall work on other
  // streams (a serving loop plans on one stream while others execute)
  struct Pinned {
    void* p;
    size_t n;
    bool busy;
  };
  std::vector<Pinned> pinned;
  void* get_pinned(size_t n) {
    for (auto& b : pinned)
      if (!b.busy && b.n >= n) {
        b.busy = true;
        return b.p;
      }
    void* p = nullptr;
    if (hipHostMalloc(&p, n, hipHostMallocDefault) != hipSuccess) return nullptr;
    pinned.push_back({p, n, true});
    return p;
  }
  void put_pinned(void* p) {
    for (auto& b : pinned)
      if (b.p == p) b.busy = false;
  }
  ~magnus_handle_s() {
    for (auto& b : pinned) (void)hipHostFree(b.p);
  }
};

namespace mgrt {

struct Alloc {
  void* p;
  size_t n;
};

inline void* default_alloc(size_t n, void*, void*) {
  void* p = nullptr;
  if (hipMalloc(&p, n ? n : 1) != hipSuccess) return nullptr;
  return p;
}
inline void default_free(void* p, size_t, void*, void*) { (void)hipFree(p); }

// Device address of this device's fixed scratch array (noalloc.hip), looked
// up with the device current once per device.
hipError_t noalloc_scratch(int device, void** out);

inline int bits_for(int64_t range) {
  int b = 1;
  while (b < 62 && ((int64_t)1 << b) < range) ++b;
  return b;
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace mgrt

struct magnus_plan_s {
  magnus_handle_s* h = nullptr;
  hipStream_t st = nullptr;
  std::vector<mgrt::Alloc> allocs;
  Mats M{};
  int64_t a_nnz = 0, b_nnz = 0, n = 0;
  int vtype = 0, itype_rp = 0, itype_col = 0;
  // per-row arrays
  int64_t *ip = nullptr, *minc = nullptr, *maxc = nullptr, *crp = nullptr;
  int32_t *cls = nullptr, *list = nullptr;
  int64_t* list_off = nullptr;
  DevStats* stats = nullptr;
  void* temp = nullptr;
  int64_t h_list_off[NCLS + 1]{};
  DevStats h_stats{};
  int shift = 13, colbits = 1, dense_block = 256, tile = 2048, lds_budget = 65536;
  int dense_shift = 13;  // DENSE rows: accumulator length 2^dense_shift covers their widest range
  int persistent_wgs = 512;
  int hints = 0;
  int64_t sort_max = 1025, dense_min = 1024, group_max = 1024;
  // workspace divisor of this attempt (an allocation failure retries with a
  // larger one), and whether some row batch came out no wider than its
  // longest row (then a larger divisor changes nothing)
  int64_t ws_div = 1;
  bool w_at_min = false;
  // CHUNKED rows binned by runs (k_runs.hip): B's chunk index, the runs'
  // count per chunk and their starts, and per run its B position, A entry
  // and product offset
  bool runs = false;
  int64_t n_runs = 0;
  int64_t *bci_ptr = nullptr, *bin_seg = nullptr, *seg_beg = nullptr;
  run_t* run_list = nullptr;  // every run's record, grouped by chunk
  int64_t* run_rec = nullptr;  // 6 int64 per dense item
  uint32_t* chunk_bm = nullptr;  // column bitmap of every dense item
  int64_t n_dense_run = 0;
  int64_t n_sort_run = -1;  // sort items of the runs path (read back; -1: not known)
  // dense items of the runs path in XCD order (see launch_dense_order)
  int64_t xcd_cpx = 1;
  int64_t *xcd_start = nullptr, *xcd_cur = nullptr;
  void* xcd_temp = nullptr;
  uint32_t *bci_pos = nullptr, *bci_chunk = nullptr;
  int persistent_wgs_count = 512;  // count-mode accumulator workgroups (bitmap only in LDS)
  // CHUNKED rows
  int64_t nch = 0, max_nb = 1;
  ChunkGeom g{};
  int64_t *aoff = nullptr, *tile_e0 = nullptr;
  int32_t *tile_row = nullptr, *bin_row = nullptr, *item_counts = nullptr;
  int64_t *bin_start = nullptr, *bin_cnt = nullptr, *bin_nnz = nullptr, *bin_out = nullptr;
  int64_t *dense_items = nullptr, *sort_items = nullptr;
  unsigned long long* bin_cursor = nullptr;
  unsigned int* work_ctr = nullptr;  // one counter per batch and phase
  bool bitmap_symbolic = false;
  bool det = false;  // deterministic mode: order-preserving reorder, sums in Eq. 1 order
  // deterministic mode: segments of det_S tiles, their rows, per-row segment
  // and table bases, the count table and its exclusive scan
  int det_S = 16;
  int32_t* det_seg_row = nullptr;
  int64_t *det_segBase = nullptr, *det_tabBase = nullptr, *det_tabS = nullptr;
  std::vector<int64_t> h_det_segBase;
  int sorted_out = MG_SORTED_OUT;  // CHUNKED reorder writes each tile out in chunk order
  uint16_t* ws_col = nullptr;
  void* ws_val = nullptr;
  void* scan_temp = nullptr;
  int64_t ws_products = 0;
  std::vector<BatchArgs> batches;
  int64_t nnz_c = 0;
  magnus_plan_info_t info{};
  int64_t *ent = nullptr, *entBase = nullptr, *nnzr = nullptr, *nnzBase = nullptr;
  double s_rp = 4, s_col = 4, s_val = 8;
  // Coarse-level rows (CHUNKED rows wider than coarse_range): a first reorder
  // into coarse chunks of 2^cshift columns (geometry g1, 32-bit chunk-local
  // columns in ws1).  Per batch the coarse chunks split by size: those with
  // at most SORT_CAP products are sorted straight from ws1; the others are
  // the rows of a second geometry whose chunks of 2^shift columns are
  // reordered into ws2 and accumulated like the chunks of CHUNKED rows.
  struct CBatch {
    int64_t nbig = 0, nsmall = 0, nbins2 = 0, nip2 = 0;
    int32_t *big = nullptr, *small = nullptr;  // coarse chunk ids (slices of big_all/small_all)
    ChunkGeom g2{};
    BatchArgs b2{};
    int64_t *cnt2 = nullptr, *start2 = nullptr, *nnz2 = nullptr, *out2 = nullptr;
    int64_t *dense2 = nullptr, *sort2 = nullptr;
    int32_t *row2 = nullptr, *tile_row2 = nullptr;
    unsigned long long* cur2 = nullptr;
    void* scan_temp = nullptr;
    bool bitmap_sym = true;
  };
  struct Coarse {
    int64_t nrows = 0, coarse_range = 0, max_nb1 = 1, max_nb2 = 1, nv = 0, nbins2 = 0;
    int cshift = 20, tile1 = 4096, tile2 = MG_L2_TILE, sorted1 = 1, sorted1_sym = 1;
    int block1 = 0;  // workgroup size of the chunk-ordered first reorder (0: default)
    int l2_block = 1024;  // workgroup size of the level-2 reorder
    ChunkGeom g1{};
    std::vector<BatchArgs> b1;  // level-1 batches
    std::vector<CBatch> cb;     // their level-2 parts
    int64_t *tile_e0 = nullptr, *ent = nullptr, *entBase = nullptr;
    int32_t* tile_row1 = nullptr;
    // per coarse chunk
    int64_t *cnt1 = nullptr, *start1 = nullptr, *nnz1 = nullptr, *out1 = nullptr;
    int64_t *minc2 = nullptr, *maxc2 = nullptr, *vnb = nullptr;
    int32_t *row1 = nullptr, *big_all = nullptr, *small_all = nullptr;
    unsigned long long* cur1 = nullptr;
    int64_t *flags = nullptr, *pos = nullptr, *nbig_dev = nullptr;  // split scratch
    int32_t* item_counts = nullptr;  // per batch: dense items, sort items
    unsigned int* work = nullptr;    // per batch: persistent-kernel counters
    // first workspace: one batch's products, or, when every coarse row's
    // products fit the budget (keep_ws1), all of them, written with their
    // values by the symbolic phase and read again by the numeric phase
    uint32_t* ws1_col = nullptr;
    void* ws1_val = nullptr;
    bool keep_ws1 = false;
    uint16_t* ws2_col = nullptr;
    void* ws2_val = nullptr;
    int64_t ws_products = 0, ip_total = 0;
    void* scan_temp = nullptr;  // scans of up to nv + 1 entries
    uint32_t* col1(const BatchArgs& b) const { return ws1_col + (keep_ws1 ? b.ip0 : 0); }
    void* val1(const BatchArgs& b, int64_t vs) const {
      return (char*)ws1_val + (keep_ws1 ? b.ip0 * vs : 0);
    }
  } co;
};

namespace mgrt {

inline magnus_status_t fail_hip(magnus_handle_s* h, hipError_t e, const char* where) {
  if (h) h->err = std::string(where) + ": " + hipGetErrorString(e);
  return MAGNUS_ERR_HIP;
}

#define HIPCHK(expr)                                      \
  do {                                                    \
    hipError_t e_ = (expr);                               \
    if (e_ != hipSuccess) return fail_hip(h, e_, #expr);  \
  } while (0)

// Checked builds (MG_CHECKED) put MG_GUARD bytes of a fixed pattern before
// and after every plan allocation; plan_check_guards reads them back after
// the plan's work and reports an overwrite.
#ifdef MG_CHECKED
constexpr size_t MG_GUARD = 256;
constexpr int MG_GUARD_BYTE = 0xA5;
#else
constexpr size_t MG_GUARD = 0;
#endif

inline void* palloc(magnus_plan_s* P, size_t bytes) {
  magnus_handle_s* h = P->h;
  bytes = align256(bytes ? bytes : 1);
  const size_t total = bytes + 2 * MG_GUARD;
  if (h->plan_cap > 0 && h->plan_live.load() + (int64_t)total > h->plan_cap) return nullptr;
  void* base = h->alloc_fn ? h->alloc_fn(total, (void*)P->st, h->alloc_ctx)
                           : default_alloc(total, nullptr, nullptr);
  if (!base) return nullptr;
  void* p = (char*)base + MG_GUARD;
#ifdef MG_CHECKED
  if (hipMemsetAsync(base, MG_GUARD_BYTE, MG_GUARD, P->st) != hipSuccess ||
      hipMemsetAsync((char*)p + bytes, MG_GUARD_BYTE, MG_GUARD, P->st) != hipSuccess) {
    if (h->free_fn) h->free_fn(base, total, (void*)P->st, h->alloc_ctx);
    else default_free(base, total, nullptr, nullptr);
    return nullptr;
  }
#endif
  P->allocs.push_back({p, bytes});
  h->plan_live += (int64_t)total;
  return p;
}

inline void plan_free_all(magnus_plan_s* P) {
  magnus_handle_s* h = P->h;
  for (auto& a : P->allocs) {
    void* base = (char*)a.p - MG_GUARD;
    const size_t total = a.n + 2 * MG_GUARD;
    if (h && h->free_fn) h->free_fn(base, total, (void*)P->st, h->alloc_ctx);
    else default_free(base, total, nullptr, nullptr);
    if (h) h->plan_live -= (int64_t)total;
  }
  P->allocs.clear();
}

// Checked builds: waits for the plan's stream and compares every guard with
// its pattern; MAGNUS_ERR_INTERNAL (with the allocation named in the
// handle's error text) on an overwrite.  Other builds: MAGNUS_OK.
inline magnus_status_t plan_check_guards(magnus_plan_s* P) {
#ifdef MG_CHECKED
  if (hipStreamSynchronize(P->st) != hipSuccess) return fail_hip(P->h, hipGetLastError(), "guards");
  std::vector<unsigned char> g(MG_GUARD);
  for (size_t k = 0; k < P->allocs.size(); ++k) {
    const Alloc& a = P->allocs[k];
    for (int side = 0; side < 2; ++side) {
      const char* at = side ? (const char*)a.p + a.n : (const char*)a.p - MG_GUARD;
      if (hipMemcpy(g.data(), at, MG_GUARD, hipMemcpyDeviceToHost) != hipSuccess)
        return fail_hip(P->h, hipGetLastError(), "guards");
      for (size_t i = 0; i < MG_GUARD; ++i)
        if (g[i] != (unsigned char)MG_GUARD_BYTE) {
          char msg[160];
          snprintf(msg, sizeof msg, "guard %s allocation %zu of %zu (%zu bytes) overwritten",
                   side ? "after" : "before", k, P->allocs.size(), a.n);
          P->h->err = msg;
          return MAGNUS_ERR_INTERNAL;
        }
    }
  }
#else
  (void)P;
#endif
  return MAGNUS_OK;
}


// Brackets one launch (or a group of launches) with events when profiling.
struct ProfScope {
  magnus_handle_s* h;
  hipStream_t st;
  const char* name;
  double bytes;
  hipEvent_t a{}, b{};
  bool on;
  ProfScope(magnus_handle_s* h_, hipStream_t st_, const char* name_, double bytes_)
      : h(h_), st(st_), name(name_), bytes(bytes_), on(h_ && h_->prof) {
    if (on) {
      if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess ||
          hipEventRecord(a, st) != hipSuccess)
        on = false;
    }
  }
  ~ProfScope() {
    if (on && hipEventRecord(b, st) == hipSuccess) h->recs.push_back({name, a, b, bytes});
  }
};

inline magnus_status_t check_csr(const magnus_csr_t* X) {
  if (!X) return MAGNUS_ERR_INVALID_ARG;
  if (X->nrows < 0 || X->ncols < 0 || X->nnz < 0) return MAGNUS_ERR_INVALID_ARG;
  if ((X->rowptr_type != MAGNUS_I32 && X->rowptr_type != MAGNUS_I64) ||
      (X->col_type != MAGNUS_I32 && X->col_type != MAGNUS_I64) ||
      (X->val_type != MAGNUS_F32 && X->val_type != MAGNUS_F64))
    return MAGNUS_ERR_INVALID_ARG;
  if (!X->rowptr) return MAGNUS_ERR_INVALID_ARG;
  if (X->nnz > 0 && (!X->col || !X->val)) return MAGNUS_ERR_INVALID_ARG;
  if (X->rowptr_type == MAGNUS_I32 && X->nnz > INT32_MAX) return MAGNUS_ERR_INDEX_OVERFLOW;
  if (X->col_type == MAGNUS_I32 && X->ncols > (int64_t)INT32_MAX + 1) return MAGNUS_ERR_INDEX_OVERFLOW;
  return MAGNUS_OK;
}

inline magnus_status_t readback(magnus_plan_s* P,
                                const std::vector<std::pair<const void*, size_t>>& src,
                                std::vector<void*> dst) {
  magnus_handle_s* h = P->h;
  size_t tot = 0;
  for (auto& s : src) tot += align256(s.second);
  char* buf = (char*)h->get_pinned(std::max<size_t>(tot, 4096));
  if (!buf) {
    h->err = "hipHostMalloc failed";
    return MAGNUS_ERR_OOM;
  }
  size_t off = 0;
  hipError_t e = hipSuccess;
  for (auto& s : src) {
    if (s.second && e == hipSuccess)
      e = hipMemcpyAsync(buf + off, s.first, s.second, hipMemcpyDeviceToHost, P->st);
    off += align256(s.second);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(P->st);
  if (e == hipSuccess) {
    off = 0;
    for (size_t i = 0; i < src.size(); ++i) {
      if (src[i].second) memcpy(dst[i], buf + off, src[i].second);
      off += align256(src[i].second);
    }
  } else {
    (void)hipStreamSynchronize(P->st);
  }
  h->put_pinned(buf);
  if (e != hipSuccess) return fail_hip(h, e, "readback");
  return MAGNUS_OK;
}

inline int dense_rows_shift(unsigned long long widest, int shift) {
  int s = 5;
  while (s < shift && ((unsigned long long)1 << s) < widest) ++s;
  return s;
}

inline int default_shift(int f64, int lds_budget) {
  // largest 2^s with s_val * 2^s + 2^s / 8 bytes <= half the LDS budget (two
  // dense workgroups per CU), capped at 2^16 (16-bit chunk-local columns)
  const double per = (f64 ? 8.0 : 4.0) + 0.125;
  int s = 8;
  while (s < 16 && per * (double)((int64_t)1 << (s + 1)) + 1024 <= lds_budget / 2.0) ++s;
  return s;
}

inline magnus_status_t make_mats(const magnus_csr_t* A, const magnus_csr_t* B, Mats& M) {
  magnus_status_t s = check_csr(A);
  if (s != MAGNUS_OK) return s;
  s = check_csr(B);
  if (s != MAGNUS_OK) return s;
  if (A->ncols != B->nrows) return MAGNUS_ERR_SHAPE;
  if (A->rowptr_type != B->rowptr_type || A->col_type != B->col_type ||
      A->val_type != B->val_type)
    return MAGNUS_ERR_DTYPE;
  if (A->nrows > INT32_MAX) return MAGNUS_ERR_INDEX_OVERFLOW;
  M.arp = A->rowptr;
  M.acol = A->col;
  M.aval = A->val;
  M.brp = B->rowptr;
  M.bcol = B->col;
  M.bval = B->val;
  M.n = A->nrows;
  M.k = A->ncols;
  M.m = B->ncols;
  M.rp64 = A->rowptr_type == MAGNUS_I64;
  M.col64 = A->col_type == MAGNUS_I64;
  M.f64 = A->val_type == MAGNUS_F64;
  return MAGNUS_OK;
}

}  // namespace mgrt
