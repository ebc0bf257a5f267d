// Entry points of the step kernels by template arguments.  The kernels of
// each storage type are instantiated in a translation unit of their own
// (step_f64.hip, step_f32.hip, step_f16.hip, step_bf16.hip), so that they
// compile in parallel; the host code only sees these declarations.
#pragma once

#include <type_traits>

#include "kernels.hpp"

namespace lbm {

// FP32 and FP64 store g directly; only they run the general wall rules.
template <typename S>
constexpr bool kUnscaledStorage = std::is_same_v<S, float> || std::is_same_v<S, double>;

// Single-domain step (step_kernel, or step_pair_kernel with pairs) for the
// collision operator (kSRT, kTRT, kMRT) and wall template (kSBB, kCLI,
// kGEN); red adds the block partial sums, nt stores non-temporally.
template <typename S>
const void* step_kernel_entry(bool red, bool nt, bool pairs, int collision, int wall_tmpl);

// Batch step (batch_step_kernel), FP32 and FP64 storage.
template <typename S>
const void* batch_kernel_entry(bool red, bool nt, int collision, int wall_tmpl);

}  // namespace lbm
