// Dispatch of SORT rows to the instantiation for A's and B's types.
#include "k_sort_decl.h"
#include "dispatch.h"

namespace mg {

RowSrc single_src(const Mats& M, void* ccol, void* cval) {
  RowSrc s{};
  s.one.arp = M.arp;
  s.one.acol = M.acol;
  s.one.aval = M.aval;
  s.one.brp = M.brp;
  s.one.bcol = M.bcol;
  s.one.bval = M.bval;
  s.one.ccol = ccol;
  s.one.cval = cval;
  s.one.crp_out = nullptr;
  s.one.row0 = 0;
  s.one.nrows = M.n;
  s.one.sort_max = 0;
  s.one.dense_max = 0;
  s.one.mcols = M.m;
  s.one.crp_out64 = 1;
  s.one.pad = 0;
  s.tab = nullptr;
  s.mat_of_row = nullptr;
  return s;
}

hipError_t launch_sort_rows(const Mats& M, const RowSrc& src, int cls, bool numeric,
                            const int32_t* list, int64_t begin, int64_t count, const int64_t* minc,
                            int colbits, int64_t* rownnz, const int64_t* crp, DevStats* stats,
                            hipStream_t st, unsigned int* work, int persistent_blocks) {
  if (count <= 0) return hipSuccess;
  hipError_t e = hipSuccess;
  MG_DISPATCH3(M, e = (sort_rows_cls<RP, CI, V>(src, cls, numeric, list + begin, count, minc,
                                                 colbits, rownnz, crp, stats, work,
                                                 persistent_blocks, st)));
  return e;
}

}  // namespace mg
