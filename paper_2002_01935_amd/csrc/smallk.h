// Write-bound complex GEMM with few summed values (smallk.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "smallk_rule.h"

namespace tn {

hipError_t launch_gemm_smallk(const Ctx& ctx, const GemmOp& op, int prec, hipStream_t s);
// kernel (template name) that launch_gemm_smallk runs for op at precision prec
const char* smallk_kernel_name(const GemmOp& op, int prec);

}  // namespace tn
