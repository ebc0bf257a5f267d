// Definitions behind step_table.hpp; included only by the per-storage
// translation units that instantiate them.
#pragma once

#define LBM_STEP_TU
#include "step_table.hpp"

namespace lbm {

template <typename S, bool RED, bool NT>
const void* step_pair_fn(int collision, int wall_tmpl) {
  if constexpr (sizeof(S) == 2) {
    switch (collision * 2 + wall_tmpl) {
      case 0: return (const void*)step_pair_kernel<S, kSRT, kSBB, RED, NT>;
      case 1: return (const void*)step_pair_kernel<S, kSRT, kCLI, RED, NT>;
      case 2: return (const void*)step_pair_kernel<S, kTRT, kSBB, RED, NT>;
      case 3: return (const void*)step_pair_kernel<S, kTRT, kCLI, RED, NT>;
      case 4: return (const void*)step_pair_kernel<S, kMRT, kSBB, RED, NT>;
      default: return (const void*)step_pair_kernel<S, kMRT, kCLI, RED, NT>;
    }
  }
  return nullptr;
}

template <typename S, bool RED, bool NT>
const void* step_fn(int collision, int wall_tmpl) {
  if constexpr (kUnscaledStorage<S>) {
    if (wall_tmpl == kGEN) {
      switch (collision) {
        case 0: return (const void*)step_kernel<S, kSRT, kGEN, RED, NT>;
        case 1: return (const void*)step_kernel<S, kTRT, kGEN, RED, NT>;
        default: return (const void*)step_kernel<S, kMRT, kGEN, RED, NT>;
      }
    }
  }
  switch (collision * 2 + wall_tmpl) {
    case 0: return (const void*)step_kernel<S, kSRT, kSBB, RED, NT>;
    case 1: return (const void*)step_kernel<S, kSRT, kCLI, RED, NT>;
    case 2: return (const void*)step_kernel<S, kTRT, kSBB, RED, NT>;
    case 3: return (const void*)step_kernel<S, kTRT, kCLI, RED, NT>;
    case 4: return (const void*)step_kernel<S, kMRT, kSBB, RED, NT>;
    default: return (const void*)step_kernel<S, kMRT, kCLI, RED, NT>;
  }
}

template <typename S>
const void* step_kernel_entry(bool red, bool nt, bool pairs, int collision, int wall_tmpl) {
  if (pairs) {
    if (red) return nt ? step_pair_fn<S, true, true>(collision, wall_tmpl)
                       : step_pair_fn<S, true, false>(collision, wall_tmpl);
    return nt ? step_pair_fn<S, false, true>(collision, wall_tmpl)
              : step_pair_fn<S, false, false>(collision, wall_tmpl);
  }
  if (red) return nt ? step_fn<S, true, true>(collision, wall_tmpl)
                     : step_fn<S, true, false>(collision, wall_tmpl);
  return nt ? step_fn<S, false, true>(collision, wall_tmpl)
            : step_fn<S, false, false>(collision, wall_tmpl);
}

template <typename S, bool RED, bool NT>
const void* batch_fn(int collision, int wall_tmpl) {
  if (wall_tmpl == kGEN) {
    switch (collision) {
      case 0: return (const void*)batch_step_kernel<S, kSRT, kGEN, RED, NT>;
      case 1: return (const void*)batch_step_kernel<S, kTRT, kGEN, RED, NT>;
      default: return (const void*)batch_step_kernel<S, kMRT, kGEN, RED, NT>;
    }
  }
  switch (collision * 2 + wall_tmpl) {
    case 0: return (const void*)batch_step_kernel<S, kSRT, kSBB, RED, NT>;
    case 1: return (const void*)batch_step_kernel<S, kSRT, kCLI, RED, NT>;
    case 2: return (const void*)batch_step_kernel<S, kTRT, kSBB, RED, NT>;
    case 3: return (const void*)batch_step_kernel<S, kTRT, kCLI, RED, NT>;
    case 4: return (const void*)batch_step_kernel<S, kMRT, kSBB, RED, NT>;
    default: return (const void*)batch_step_kernel<S, kMRT, kCLI, RED, NT>;
  }
}

template <typename S>
const void* batch_kernel_entry(bool red, bool nt, int collision, int wall_tmpl) {
  if (red) return nt ? batch_fn<S, true, true>(collision, wall_tmpl)
                     : batch_fn<S, true, false>(collision, wall_tmpl);
  return nt ? batch_fn<S, false, true>(collision, wall_tmpl)
            : batch_fn<S, false, false>(collision, wall_tmpl);
}

}  // namespace lbm
