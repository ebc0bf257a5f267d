// Step kernels for FP32 storage,
// instantiated here for the entry points of step_table.hpp.
#include <hip/hip_runtime.h>

#include "step_impl.hpp"

namespace lbm {
template const void* step_kernel_entry<float>(bool, bool, bool, int, int);
template const void* batch_kernel_entry<float>(bool, bool, int, int);
}  // namespace lbm
