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
// Workgroups (of 4 wavefronts) along x of a persistent launch of `kernel`
// that needs `waves` wavefronts per grid row, with gy grid rows: about
// kStreamWavesPerCU wavefronts per compute unit over the whole grid, fewer
// when the kernel's registers let a compute unit hold fewer at once.
constexpr int kStreamWavesPerCU = 16;
// Streaming row kernel: blocks of 64 rows per unit (1 or 2), and the store
// mode for contiguous complex64 output blocks (1: coalesced pieces, 2: LDS
// staging) by in-thread value count.  Measured on MI355X (ms per launch,
// 1 / 2 blocks per unit): 2^26 x 16 outputs from one summed value: staging
// 1.79 / 1.77, coalesced 2.00 / 2.01; 2^25 x 8 from two: staging 0.559 /
// 0.537, coalesced 0.575 / 0.561; 2^28 x 4 from four: staging 3.63 / 3.64,
// coalesced 3.45 / 3.29.
constexpr int kRowStreamBlocks = 2;
constexpr int kRowStreamMode(int nin) { return nin >= 8 ? 2 : 1; }
unsigned stream_grid_x(uint64_t waves, unsigned gy, const void* kernel);
// log2 tile sizes of a gemm tile variant; -1 if unknown
int gemm_tile_bits(int tile, int* bm, int* bn);
// whether tile variant `tile` can run op at precision prec
bool gemm_tile_ok(const GemmOp& op, int tile, int prec);
// kernel (template instance) that launch_gemm runs for op's tile at precision prec
const char* gemm_kernel_name(const GemmOp& op, int prec);
constexpr int kNumGemmTiles = 15;
constexpr int kSplitTile = 10;      // first BF16x3 variant on pre-split operands (direct-to-LDS)
constexpr int kNumSplitTiles = 4;   // variants 10, 11, 12, 13
constexpr int kNumTilesShared = 4;   // tiles 0..3 exist for every matrix-core kernel
constexpr int kValuTile = 4;   // vector-ALU variant (complex128 and reference)

}  // namespace tn
