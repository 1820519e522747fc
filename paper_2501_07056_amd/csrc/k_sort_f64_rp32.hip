// SORT-row kernels instantiated for double values and int32_t row pointers.
#include "k_sort_impl.h"

namespace mg {
MG_SORT_INSTANTIATE(int32_t, double)
}  // namespace mg
