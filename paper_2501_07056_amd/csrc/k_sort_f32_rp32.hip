// SORT-row kernels instantiated for float values and int32_t row pointers.
#include "k_sort_impl.h"

namespace mg {
MG_SORT_INSTANTIATE(int32_t, float)
}  // namespace mg
