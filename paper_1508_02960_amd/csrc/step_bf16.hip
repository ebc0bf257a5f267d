// Step kernels for BF16 storage (stochastic and round-to-nearest rounding),
// instantiated here for the entry points of step_table.hpp.
#include <hip/hip_runtime.h>

#include "step_impl.hpp"

namespace lbm {
template const void* step_kernel_entry<bf16s_t>(bool, bool, bool, int, int);
template const void* step_kernel_entry<bf16_t>(bool, bool, bool, int, int);
}  // namespace lbm
