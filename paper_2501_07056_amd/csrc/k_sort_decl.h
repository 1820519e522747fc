// Declaration of the SORT-row launcher template (defined in k_sort_impl.h,
// instantiated per value and row-pointer type in k_sort_*.hip).
#pragma once
#include "kernels.h"

namespace mg {
template <typename RP, typename CI, typename V>
hipError_t sort_rows_cls(const RowSrc& src, int cls, bool numeric, const int32_t* list,
                         int64_t count, const int64_t* minc, int colbits, int64_t* rownnz,
                         const int64_t* crp, DevStats* stats, unsigned int* work,
                         int persistent_blocks, hipStream_t st);
}  // namespace mg
