// Complex GEMM with at most eight summed values, C[h][m][n] = sum_k A[h][m][k] B[h][n][k]
// (Sec. 2: a pairwise contraction whose shared indices span at most three
// bits).  Each output needs at most 8 complex multiply-adds per 8 or 16 bytes
// written, so these contractions are bound by the HBM write of C, not by
// arithmetic (eight values take about 60 % of the vector ALU's FP32 rate at
// 6 TB/s of output):
// a tile through LDS and matrix cores would spend its time in the load ->
// product -> store chain of each block.  Here every thread owns one index of
// the free side that holds C's lowest bit (consecutive lanes write consecutive
// elements) and R indices of the other side: it loads its own K operand
// values once and, per output, the other operand's K values, which all lanes
// of a wavefront share (one cached address).  Without accumulation into C
// and with a fast side of at least 64 threads, a one-shot variant runs when
// the fast side's operand fits the L2 (each wavefront writes a few
// consecutive 1 KiB pieces of C), else the streaming variant (persistent
// wavefronts, the next unit's operands loaded before the current unit's
// stores).  The sum over k runs in index order in the storage
// precision (FP32 for complex64, FP64 for complex128).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "../../include/tn.h"
#include "kernels.h"
#include "smallk.h"

namespace tn {

#define GMEM __attribute__((address_space(1)))
#define CMEM __attribute__((address_space(4)))
#define TN_WAVE_SYNC() __builtin_amdgcn_wave_barrier()
// A value the same in every lane of the wavefront, made known to the compiler as such.
#define TN_UNIFORM(x) __builtin_amdgcn_readfirstlane(x)

#include "rowops.h"
#include "smallk_kernel.h"

hipError_t launch_gemm_smallk(const Ctx& ctx, const GemmOp& in, int prec, hipStream_t s) {
  constexpr int R = kSmallkRows;
  GemmOp op = in;
  SmallkTables kt;
  SmallkLaunch L;
  if (!smallk_prepare(op, prec, ctx.n_batch, kt, L)) return hipErrorInvalidValue;
  if (L.blocks > 0x7fffffffULL || L.gy > 65535) return hipErrorInvalidConfiguration;
  const dim3 grid((unsigned)L.blocks, (unsigned)L.gy, 1);
  const dim3 wgrid((unsigned)((L.units + 3) / 4), (unsigned)L.gy, 1);   // units <= 2^25: at most 2^23 workgroups
  smallk_dispatch(L, prec, [&](auto t, auto fastn, auto p, auto kn, auto variant) {
    using T = decltype(t);
    constexpr bool FN = decltype(fastn)::value;
    constexpr int P = decltype(p)::value, KN = decltype(kn)::value, VAR = decltype(variant)::value;
    if constexpr (VAR == kSmallkWide) {
      if constexpr (KN <= kWideMaxSummed) gemm_smallk_wide<T, FN, P, KN><<<wgrid, 256, 0, s>>>(ctx, op, kt);
    }
    else if constexpr (VAR == kSmallkStream) {
      auto k = gemm_smallk_stream<T, FN, P, KN>;
      const dim3 sgrid(stream_grid_x(L.units, (unsigned)L.gy, (const void*)k), (unsigned)L.gy, 1);
      k<<<sgrid, 256, 0, s>>>(ctx, op, kt);
    }
    else gemm_smallk<T, FN, P, R, KN><<<grid, 256, 0, s>>>(ctx, op, kt);
  });
  return hipGetLastError();
}

const char* smallk_kernel_name(const GemmOp& in, int prec) {
  GemmOp op = in;
  SmallkTables kt;
  SmallkLaunch L;
  if (!smallk_prepare(op, prec, 1, kt, L)) return "gemm_smallk";
  return L.variant == kSmallkWide ? "gemm_smallk_wide" : (L.variant == kSmallkStream ? "gemm_smallk_stream" : "gemm_smallk");
}

}  // namespace tn
