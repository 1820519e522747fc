// Dispatch of SORT rows to the instantiation for A's and B's types.
#include "k_sort_decl.h"
#include "dispatch.h"

namespace mg {

hipError_t launch_sort_rows(const Mats& M, int cls, bool numeric, const int32_t* list,
                            int64_t begin, int64_t count, const int64_t* minc, int colbits,
                            int64_t* rownnz, const int64_t* crp, void* ccol, void* cval,
                            DevStats* stats, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipError_t e = hipSuccess;
  MG_DISPATCH3(M, e = (sort_rows_cls<RP, CI, V>(M, cls, numeric, list + begin, count, minc,
                                                 colbits, rownnz, crp, ccol, cval, stats, st)));
  return e;
}

}  // namespace mg
