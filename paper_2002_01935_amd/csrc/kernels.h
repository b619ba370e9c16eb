// Launchers for the gfx950 kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/tn.h"
#include "tn_internal.h"

namespace tn {

hipError_t launch_row(const Ctx& ctx, const RowOp& op, bool f64, hipStream_t s);
hipError_t launch_reduce(const Ctx& ctx, const RowOp& op, bool f64, hipStream_t s);
hipError_t launch_gemm(const Ctx& ctx, const GemmOp& op, int prec, hipStream_t s);
hipError_t launch_permute(const Ctx& ctx, const PermuteOp& op, bool f64, hipStream_t s);
hipError_t launch_accum(const Ctx& ctx, const AccumOp& op, bool f64, hipStream_t s);
hipError_t launch_counter(const Ctx& ctx, int64_t value, int add, hipStream_t s);
hipError_t launch_fill(uint64_t base, uint64_t bytes, hipStream_t s);
hipError_t launch_split(const Ctx& ctx, const SplitOp& op, hipStream_t s);
// log2 tile sizes of a gemm tile variant; -1 if unknown
int gemm_tile_bits(int tile, int* bm, int* bn);
// whether tile variant `tile` can run op at precision prec
bool gemm_tile_ok(const GemmOp& op, int tile, int prec);
// kernel (template instance) that launch_gemm runs for op's tile at precision prec
const char* gemm_kernel_name(const GemmOp& op, int prec);
constexpr int kNumGemmTiles = 13;
constexpr int kSplitTile = 10;      // first BF16x3 variant on pre-split operands (direct-to-LDS)
constexpr int kNumSplitTiles = 3;   // variants 10, 11, 12
constexpr int kNumTilesShared = 4;   // tiles 0..3 exist for every matrix-core kernel
constexpr int kValuTile = 4;   // vector-ALU variant (complex128 and reference)

}  // namespace tn
