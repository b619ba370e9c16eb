// Which GEMM-class contractions take the few-summed-values kernel.
#pragma once

#include "tn_internal.h"

namespace tn {

// Whether a GEMM-class contraction takes the few-summed-values kernel: at most
// three summed bits (K <= 8 values), no split over the summed range, and at
// least 2^5 values on each free side.
inline bool gemm_smallk_ok(const GemmOp& op) {
  return op.n_k <= 3 && op.k_split_bits <= 0 && op.n_m >= 5 && op.n_n >= 5 && op.n_m + op.n_n <= 40;
}

}  // namespace tn
