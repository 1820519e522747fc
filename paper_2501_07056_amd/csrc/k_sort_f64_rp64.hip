// SORT-row kernels instantiated for double values and int64_t row pointers.
#include "k_sort_impl.h"

namespace mg {
MG_SORT_INSTANTIATE(int64_t, double)
}  // namespace mg
