// Complex GEMM with at most four summed values, C[h][m][n] = sum_k A[h][m][k] B[h][n][k]
// (Sec. 2: a pairwise contraction whose shared indices span at most two bits).
// Each output needs at most 4 complex multiply-adds per 8 or 16 bytes written,
// so these contractions are bound by the HBM write of C, not by arithmetic:
// a tile through LDS and matrix cores would spend its time in the load ->
// product -> store chain of each block.  Here every thread owns one index of
// the free side that holds C's lowest bit (consecutive lanes write consecutive
// elements) and R indices of the other side: it loads its own K operand
// values once and, per output, the other operand's K values, which all lanes
// of a wavefront share (one cached address).  The sum over k runs in index
// order in the storage precision (FP32 for complex64, FP64 for complex128).
#include <hip/hip_runtime.h>

#include "../../include/tn.h"
#include "smallk.h"

namespace tn {

#define GMEM __attribute__((address_space(1)))
#define CMEM __attribute__((address_space(4)))
#define TN_WAVE_SYNC() __builtin_amdgcn_wave_barrier()

#include "rowops.h"

typedef float f4 __attribute__((ext_vector_type(4)));

// Offsets the host computes once per launch: of summed value k in the
// thread's own operand (kf) and in the shared one (ks); of row i < R of the
// shared index in that operand (si) and in C (ci), added to the deposit of
// the thread's first row (a multiple of R, so the bit sets are disjoint);
// of the thread's second own index (P = 2) in its operand (f1).
struct SmallkTables {
  uint32_t kf[4], ks[4], si[16], ci[16], f1;
};

template <typename T, bool FASTN, int P, int R>
__global__ __launch_bounds__(256) void gemm_smallk(Ctx ctx, GemmOp op, SmallkTables kt) {
  using V = typename C2<T>::t;
  static_assert(P == 1 || (P == 2 && sizeof(T) == 4), "paired stores are 16-byte complex64 pairs");
  constexpr int LP = P == 2 ? 1 : 0;
  const int nzh = ctx.n_batch;
  const int z = blockIdx.y % nzh;
  const uint32_t h = blockIdx.y / nzh;
  const int64_t sid = slice_id(ctx, z);
  if (sid < 0) return;
  const int nf = FASTN ? op.n_n : op.n_m;
  const int ns = FASTN ? op.n_m : op.n_n;
  const uint64_t t = uint64_t(blockIdx.x) * 256 + threadIdx.x;
  const uint32_t f = uint32_t(t & ((uint64_t(1) << (nf - LP)) - 1)) << LP;
  const uint64_t s0 = (t >> (nf - LP)) * R;
  if (s0 >= (uint64_t(1) << ns)) return;
  const int eb = sizeof(V);
  GMEM const V* A = reinterpret_cast<GMEM const V*>(resolve(ctx, op.a, z, sid, eb)) + deposit_runs32(h, op.run_a_h);
  GMEM const V* B = reinterpret_cast<GMEM const V*>(resolve(ctx, op.b, z, sid, eb)) + deposit_runs32(h, op.run_b_h);
  GMEM V* C = reinterpret_cast<GMEM V*>(resolve(ctx, op.c, z, sid, eb)) + deposit_runs32(h, op.run_c_h);
  const int K = 1 << op.n_k;
  GMEM const V* F = (FASTN ? B : A) + deposit_runs32(f, FASTN ? op.run_b_n : op.run_a_m);
  GMEM const V* S = (FASTN ? A : B) + deposit_runs32(uint32_t(s0), FASTN ? op.run_a_m : op.run_b_n);
  GMEM V* Cr = C + deposit_runs32(f, FASTN ? op.run_c_n : op.run_c_m) +
               deposit_runs32(uint32_t(s0), FASTN ? op.run_c_m : op.run_c_n);
  const int cjf = FASTN ? op.conj_b : op.conj_a, cjs = FASTN ? op.conj_a : op.conj_b;
  V fv[P][4];
#pragma unroll
  for (int p = 0; p < P; p++)
#pragma unroll
    for (int k = 0; k < 4; k++)
      if (k < K) fv[p][k] = conjv(ld(F + (p ? kt.f1 : 0u) + kt.kf[k]), cjf);
#pragma unroll
  for (int i = 0; i < R; i++) {
    V acc[P];
#pragma unroll
    for (int p = 0; p < P; p++) {
      acc[p].x = 0;
      acc[p].y = 0;
    }
#pragma unroll
    for (int k = 0; k < 4; k++)
      if (k < K) {
        const V sv = conjv(ld(S + kt.si[i] + kt.ks[k]), cjs);
#pragma unroll
        for (int p = 0; p < P; p++) acc[p] = FASTN ? cfma(acc[p], sv, fv[p][k]) : cfma(acc[p], fv[p][k], sv);
      }
    GMEM V* d = Cr + kt.ci[i];
    if (op.accumulate) {
#pragma unroll
      for (int p = 0; p < P; p++) {
        const V o = ld(d + p);
        acc[p].x += o.x;
        acc[p].y += o.y;
      }
    }
    if constexpr (P == 2) {
      // the pair is adjacent in C (its two lowest positions are this
      // thread's index bits 0 and 1, f even): one 16-byte store where the
      // address allows it (a caller's output may be only 8-byte aligned)
      if ((reinterpret_cast<uint64_t>(d) & 15) == 0) {
        f4 v = {acc[0].x, acc[0].y, acc[1].x, acc[1].y};
        *reinterpret_cast<GMEM f4*>(d) = v;
      } else {
        st(d, acc[0]);
        st(d + 1, acc[1]);
      }
    } else {
      st(d, acc[0]);
    }
  }
}

// Offset of a small value v (its set bits among the first n of a position list).
static uint32_t deposit_small(uint32_t v, const int8_t* pos, int n) {
  uint32_t off = 0;
  for (int i = 0; i < n && (v >> i); i++)
    if ((v >> i) & 1) off += uint32_t(1) << pos[i];
  return off;
}

hipError_t launch_gemm_smallk(const Ctx& ctx, const GemmOp& in, int prec, hipStream_t s) {
  constexpr int R = 16;
  if (!gemm_smallk_ok(in)) return hipErrorInvalidValue;
  GemmOp op = in;
  make_runs(op.a_h, op.n_h, op.run_a_h);
  make_runs(op.b_h, op.n_h, op.run_b_h);
  make_runs(op.c_h, op.n_h, op.run_c_h);
  make_runs(op.a_m, op.n_m, op.run_a_m);
  make_runs(op.c_m, op.n_m, op.run_c_m);
  make_runs(op.b_n, op.n_n, op.run_b_n);
  make_runs(op.c_n, op.n_n, op.run_c_n);
  for (int i = 0; i < op.n_k; i++)
    if (op.a_k[i] < 0 || op.b_k[i] < 0) return hipErrorInvalidValue;
  // the thread's own index runs over the free side holding C's position 0
  const bool fastn = op.c_m[0] != 0;
  const int8_t* f_op = fastn ? op.b_n : op.a_m;
  const int8_t* f_c = fastn ? op.c_n : op.c_m;
  const int8_t* s_op = fastn ? op.a_m : op.b_n;
  const int8_t* s_c = fastn ? op.c_m : op.c_n;
  const int nf = fastn ? op.n_n : op.n_m, ns = fastn ? op.n_m : op.n_n;
  const bool pair = prec != TN_C128 && f_c[0] == 0 && f_c[1] == 1;
  SmallkTables kt{};
  for (int k = 0; k < (1 << op.n_k); k++) {
    kt.kf[k] = deposit_small(k, fastn ? op.b_k : op.a_k, op.n_k);
    kt.ks[k] = deposit_small(k, fastn ? op.a_k : op.b_k, op.n_k);
  }
  for (int i = 0; i < R; i++) {
    kt.si[i] = deposit_small(i, s_op, ns);
    kt.ci[i] = deposit_small(i, s_c, ns);
  }
  kt.f1 = deposit_small(1, f_op, nf);
  const uint64_t threads = (uint64_t(1) << (nf + ns)) / R / (pair ? 2 : 1);
  const uint64_t blocks = (threads + 255) / 256;
  const uint64_t gy = uint64_t(ctx.n_batch) << op.n_h;
  if (blocks > 0x7fffffffULL || gy > 65535) return hipErrorInvalidConfiguration;
  const dim3 grid((unsigned)blocks, (unsigned)gy, 1);
  if (prec == TN_C128) {
    if (fastn) gemm_smallk<double, true, 1, R><<<grid, 256, 0, s>>>(ctx, op, kt);
    else gemm_smallk<double, false, 1, R><<<grid, 256, 0, s>>>(ctx, op, kt);
  } else if (pair) {
    if (fastn) gemm_smallk<float, true, 2, R><<<grid, 256, 0, s>>>(ctx, op, kt);
    else gemm_smallk<float, false, 2, R><<<grid, 256, 0, s>>>(ctx, op, kt);
  } else {
    if (fastn) gemm_smallk<float, true, 1, R><<<grid, 256, 0, s>>>(ctx, op, kt);
    else gemm_smallk<float, false, 1, R><<<grid, 256, 0, s>>>(ctx, op, kt);
  }
  return hipGetLastError();
}

}  // namespace tn
