// The few-summed-values GEMM kernel (gemm_smallk) and its launch-time
// preparation.  Included inside namespace tn, after rowops.h, by smallk.hip;
// written in plain C++ over the HIP names rowops.h uses so that the host
// emulation in the tests runs the same code on the CPU.
#pragma once

typedef float smallk_f4 __attribute__((ext_vector_type(4)));

constexpr int kSmallkRows = 32;   // rows of the shared index per thread

// Offsets the host computes once per launch: of summed value k in the
// thread's own operand (kf) and in the shared one (ks); of row i < R of the
// shared index in that operand (si) and in C (ci), added to the deposit of
// the thread's first row (a multiple of R, so the bit sets are disjoint);
// of the thread's second own index (P = 2) in its operand (f1).
struct SmallkTables {
  uint32_t kf[4], ks[4], si[32], ci[32], f1;
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
        smallk_f4 v = {acc[0].x, acc[0].y, acc[1].x, acc[1].y};
        *reinterpret_cast<GMEM smallk_f4*>(d) = v;
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
inline uint32_t deposit_small(uint32_t v, const int8_t* pos, int n) {
  uint32_t off = 0;
  for (int i = 0; i < n && (v >> i); i++)
    if ((v >> i) & 1) off += uint32_t(1) << pos[i];
  return off;
}


// Grid and variant of one launch.
struct SmallkLaunch {
  bool fastn, pair;
  uint64_t blocks, gy;
};

// Host side of a launch: the op's position lists as runs, the offset tables
// and the grid.  False when the op does not qualify.
inline bool smallk_prepare(GemmOp& op, int prec, int n_batch, SmallkTables& kt, SmallkLaunch& L) {
  constexpr int R = kSmallkRows;
  if (!gemm_smallk_ok(op)) return false;
  make_runs(op.a_h, op.n_h, op.run_a_h);
  make_runs(op.b_h, op.n_h, op.run_b_h);
  make_runs(op.c_h, op.n_h, op.run_c_h);
  make_runs(op.a_m, op.n_m, op.run_a_m);
  make_runs(op.c_m, op.n_m, op.run_c_m);
  make_runs(op.b_n, op.n_n, op.run_b_n);
  make_runs(op.c_n, op.n_n, op.run_c_n);
  for (int i = 0; i < op.n_k; i++)
    if (op.a_k[i] < 0 || op.b_k[i] < 0) return false;
  // the thread's own index runs over the free side holding C's position 0
  L.fastn = op.c_m[0] != 0;
  const int8_t* f_op = L.fastn ? op.b_n : op.a_m;
  const int8_t* f_c = L.fastn ? op.c_n : op.c_m;
  const int8_t* s_op = L.fastn ? op.a_m : op.b_n;
  const int8_t* s_c = L.fastn ? op.c_m : op.c_n;
  const int nf = L.fastn ? op.n_n : op.n_m, ns = L.fastn ? op.n_m : op.n_n;
  L.pair = prec != TN_C128 && f_c[0] == 0 && f_c[1] == 1;
  kt = SmallkTables{};
  for (int k = 0; k < (1 << op.n_k); k++) {
    kt.kf[k] = deposit_small(k, L.fastn ? op.b_k : op.a_k, op.n_k);
    kt.ks[k] = deposit_small(k, L.fastn ? op.a_k : op.b_k, op.n_k);
  }
  for (int i = 0; i < R; i++) {
    kt.si[i] = deposit_small(i, s_op, ns);
    kt.ci[i] = deposit_small(i, s_c, ns);
  }
  kt.f1 = deposit_small(1, f_op, nf);
  const uint64_t threads = (uint64_t(1) << (nf + ns)) / R / (L.pair ? 2 : 1);
  L.blocks = (threads + 255) / 256;
  L.gy = uint64_t(n_batch) << op.n_h;
  return true;
}
