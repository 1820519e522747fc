// SORT-row kernels instantiated for float values and int64_t row pointers.
#include "k_sort_impl.h"

namespace mg {
MG_SORT_INSTANTIATE(int64_t, float)
}  // namespace mg
