// Pieces of the executor (exec.hip) shared with the many-network batch
// (batch.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "plan.h"

namespace tn {

// Sets the calling thread's tn_last_error message; returns code.
int set_error(int code, const std::string& msg);
// Launch context of a plan's program over workspace `ws`.
Ctx make_ctx(const tn_plan_s* p, void* ws, uint64_t arena_stride);
// Launch one op of a program of precision `prec` (a tn_precision).
hipError_t launch_op(int prec, const Ctx& ctx, const Op& op, hipStream_t s);
// A plan's forward program with its tail: mode 0 writes the root to the output
// slot in the storage type (unsliced contraction), mode 1 adds every in-flight
// slice's root to the complex128 output slot.  Ends with the batch-counter op.
std::vector<Op> forward_program(const tn_plan_s* p, int mode);

}  // namespace tn
