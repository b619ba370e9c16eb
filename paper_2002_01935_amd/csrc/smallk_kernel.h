// The few-summed-values GEMM kernel (gemm_smallk) and its launch-time
// preparation.  Included inside namespace tn, after rowops.h, by smallk.hip;
// written in plain C++ over the HIP names rowops.h uses so that the host
// emulation in the tests runs the same code on the CPU.
#pragma once

typedef float smallk_f4 __attribute__((ext_vector_type(4)));

constexpr int kSmallkRows = 32;   // rows of the shared index per thread
// log2 rows of the shared index per unit of the streaming variant (<= 5).
// Measured on MI355X with 2^4 instead: (2^14, 2^14, 4) and (2^13, 2^13, 2) 3 %
// and 8 % faster, (2^15, 2^15, 1) 1 % and (2^12, 2^12, 4) 9 % slower; with 2^3
// (2^15, 2^15, 1) 16 % slower.
constexpr int kStreamRowBits = 5;
// One-shot variant (gemm_smallk_wide): log2 of the 64-lane pieces of one row
// that a wavefront writes and of its rows, by summed-value count KN; the
// largest fast-side operand (log2 bytes per batch index) it takes, so that
// the operand every row re-reads stays in the L2; the fewest outputs (log2)
// for which it runs.  Measured on MI355X (ms per launch, streaming variant /
// one-shot; C = A B with N lowest in C): 2^15 x 2^15 from one summed value
// 1.49-1.51 / 1.40-1.41; 2^15 x 2^14 from two 0.761 / 0.622; 2^13 x 2^13 from
// two 0.109 / 0.090; 2^14 x 2^14 from four 0.418-0.421 / 0.361-0.370; 2^12 x
// 2^12 from four 0.032 / 0.037 (below the output threshold).  Four pieces of
// one row for KN = 1 beat two pieces (2.17 ms on the first node) and eight
// (1.49); for KN = 4 one row of four pieces made 2^14 x 2^14 take 0.97 ms
// (eight operand loads per store).
constexpr int wide_piece_bits(int kn) { return kn == 1 ? 2 : (kn == 2 ? 0 : 1); }
constexpr int wide_row_bits(int kn) { return kn == 1 ? 0 : 2; }
constexpr int kWideOperandBits = 22;
constexpr int kWideMinOutputBits = 25;
// Eight summed values stay on the streaming variant: one-shot wavefronts then
// need eight operand loads per store or an LDS exchange of the shared values,
// and both ran slower (2^15 x 2^15 from eight: streaming 1.63 ms; one-shot
// with vector loads of the shared values 3.83 ms, through LDS 2.29 ms; the
// matrix-core GEMM 2.03 ms).
constexpr int kWideMaxSummed = 4;

// Offsets the host computes once per launch: of summed value k in the
// thread's own operand (kf) and in the shared one (ks); of row i < R of the
// shared index in that operand (si) and in C (ci), added to the deposit of
// the thread's first row (a multiple of R, so the bit sets are disjoint);
// of the thread's second own index (P = 2) in its operand (f1).
struct SmallkTables {
  uint32_t kf[8], ks[8], si[32], ci[32], f1;
  uint32_t dci[5];   // ci[i + 1] - ci[i] when i has t trailing ones (streaming variant)
};

// KN = 2^n_k summed values (a template parameter: every load is issued
// unconditionally, none waits behind a branch).
template <typename T, bool FASTN, int P, int R, int KN>
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
  GMEM const V* F = (FASTN ? B : A) + deposit_runs32(f, FASTN ? op.run_b_n : op.run_a_m);
  GMEM const V* S = (FASTN ? A : B) + deposit_runs32(uint32_t(s0), FASTN ? op.run_a_m : op.run_b_n);
  GMEM V* Cr = C + deposit_runs32(f, FASTN ? op.run_c_n : op.run_c_m) +
               deposit_runs32(uint32_t(s0), FASTN ? op.run_c_m : op.run_c_n);
  const int cjf = FASTN ? op.conj_b : op.conj_a, cjs = FASTN ? op.conj_a : op.conj_b;
  V fv[P][KN];
#pragma unroll
  for (int p = 0; p < P; p++)
#pragma unroll
    for (int k = 0; k < KN; k++) fv[p][k] = conjv(ld(F + (p ? kt.f1 : 0u) + kt.kf[k]), cjf);
#pragma unroll
  for (int i = 0; i < R; i++) {
    V acc[P];
#pragma unroll
    for (int p = 0; p < P; p++) {
      acc[p].x = 0;
      acc[p].y = 0;
    }
#pragma unroll
    for (int k = 0; k < KN; k++) {
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

// Streaming variant (no accumulation into C, and a fast side of at least 64
// threads, so that the 64 lanes of a wavefront share their R rows):
// persistent wavefronts walk units of 64 lanes x R rows.  Per unit a lane
// loads its own operand's K values and one or two of the R x K values of the
// other operand that the wavefront shares (lane l holds row l mod R, summed
// value l / R, ...); the wavefront puts those into its LDS area and each row
// reads its shared values back at one address for all lanes (a broadcast),
// so a unit needs no vector memory loads between its stores.  The loads
// of the wavefront's next unit are issued before the current unit's stores
// (stream_walk).
template <typename T, bool FASTN, int P, int KN>
__global__ __launch_bounds__(256) void gemm_smallk_stream(Ctx ctx, GemmOp op, SmallkTables kt) {
  using V = typename C2<T>::t;
  static_assert(P == 1 || (P == 2 && sizeof(T) == 4), "paired stores are 16-byte complex64 pairs");
  constexpr int R = 1 << kStreamRowBits;
  static_assert(R <= kSmallkRows, "row offsets come from the launch tables");
  constexpr int LP = P == 2 ? 1 : 0;
  constexpr int Q = (R * KN + 63) / 64;   // shared-operand values per lane and unit
  const int nzh = ctx.n_batch;
  const int z = blockIdx.y % nzh;
  const uint32_t h = blockIdx.y / nzh;
  const int64_t sid = slice_id(ctx, z);
  if (sid < 0) return;
  const int nf = FASTN ? op.n_n : op.n_m;
  const int ns = FASTN ? op.n_m : op.n_n;
  const int fbits = nf - LP - 6;                        // >= 0 (the launcher checks)
  const uint32_t units = 1u << (fbits + ns - kStreamRowBits);
  const uint32_t lane = threadIdx.x & 63;
  // uniform over the wavefront (the compiler cannot tell by itself): the
  // unit offsets below are then scalar work
  const uint32_t wave = TN_UNIFORM(blockIdx.x * 4 + (threadIdx.x >> 6));
  const uint32_t nwave = gridDim.x * 4;
  if (wave >= units) return;
  const int eb = sizeof(V);
  GMEM const V* A = reinterpret_cast<GMEM const V*>(resolve(ctx, op.a, z, sid, eb)) + deposit_runs32(h, op.run_a_h);
  GMEM const V* B = reinterpret_cast<GMEM const V*>(resolve(ctx, op.b, z, sid, eb)) + deposit_runs32(h, op.run_b_h);
  GMEM V* C = reinterpret_cast<GMEM V*>(resolve(ctx, op.c, z, sid, eb)) + deposit_runs32(h, op.run_c_h);
  GMEM const V* F = FASTN ? B : A;
  GMEM const V* S = FASTN ? A : B;
  const BitRuns& rf = FASTN ? op.run_b_n : op.run_a_m;
  const BitRuns& rs = FASTN ? op.run_a_m : op.run_b_n;
  const BitRuns& rcf = FASTN ? op.run_c_n : op.run_c_m;
  const BitRuns& rcs = FASTN ? op.run_c_m : op.run_c_n;
  const int cjf = FASTN ? op.conj_b : op.conj_a, cjs = FASTN ? op.conj_a : op.conj_b;
  const uint32_t fmask = (1u << fbits) - 1;
  // summed value of this lane's q-th shared load: k = (lane + 64 q) / R
  uint32_t ksl[Q];
#pragma unroll
  for (int q = 0; q < Q; q++) {
    const uint32_t k = ((lane + 64 * q) / R) % KN;
    // selects over the table (no lane-dependent index into the kernel's arguments)
    uint32_t v = kt.ks[0];
#pragma unroll
    for (int j = 1; j < KN; j++) v = k == uint32_t(j) ? kt.ks[j] : v;
    ksl[q] = v;
  }
  // offsets split into the unit's part (uniform) and the lane's part: the
  // lane's fast-side index bits, and the shared row its loads cover
  const uint32_t lf = deposit_runs32(lane << LP, rf), lcf = deposit_runs32(lane << LP, rcf);
  uint32_t ls[Q];
#pragma unroll
  for (int q = 0; q < Q; q++) ls[q] = deposit_runs32((lane + 64 * q) & (R - 1), rs) + ksl[q];
  struct Set {
    V f[P][KN];
    V s[Q];
  };
  auto load = [&](Set& st_, uint32_t u) {
    GMEM const V* Fp = F + deposit_runs_u((u & fmask) << (6 + LP), rf) + lf;
    GMEM const V* Sp = S + deposit_runs_u((u >> fbits) * R, rs);
#pragma unroll
    for (int p = 0; p < P; p++)
#pragma unroll
      for (int k = 0; k < KN; k++) st_.f[p][k] = ld(Fp + (p ? kt.f1 : 0u) + kt.kf[k]);
#pragma unroll
    for (int q = 0; q < Q; q++) st_.s[q] = ld(Sp + ls[q]);
  };
  // the wavefront's shared values of one unit: [64 Q] values, entry i + R k
  // holding row i, summed value k
  __shared__ __attribute__((aligned(16))) char bcast[4][64 * Q * sizeof(V)];
  V* Sw = reinterpret_cast<V*>(&bcast[threadIdx.x >> 6][0]);
  auto body = [&](const Set& st_, uint32_t u, auto aligned) {
    GMEM V* Cr = C + (deposit_runs_u((u & fmask) << (6 + LP), rcf) + deposit_runs_u((u >> fbits) * R, rcs)) + lcf;
#pragma unroll
    for (int q = 0; q < Q; q++) Sw[lane + 64 * q] = st_.s[q];
    // one wavefront's area only: its LDS accesses are performed in order
    TN_WAVE_SYNC();
    uint32_t ci = 0;                              // offset of row i in C (rows walked in order)
#pragma unroll
    for (int i = 0; i < R; i++) {
      if (i) ci += kt.dci[__builtin_ctz(~uint32_t(i - 1))];
      V acc[P];
#pragma unroll
      for (int p = 0; p < P; p++) {
        acc[p].x = 0;
        acc[p].y = 0;
      }
#pragma unroll
      for (int k = 0; k < KN; k++) {
        const V s = conjv(Sw[i + R * k], cjs);
#pragma unroll
        for (int p = 0; p < P; p++) {
          const V f = conjv(st_.f[p][k], cjf);
          acc[p] = FASTN ? cfma(acc[p], s, f) : cfma(acc[p], f, s);
        }
      }
      GMEM V* d = Cr + ci;
      if constexpr (P == 2) {
        if constexpr (decltype(aligned)::value) {
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
    // the next unit's LDS writes follow this wavefront's reads
    TN_WAVE_SYNC();
  };
  auto run = [&](auto aligned) {
    Set s0, s1;
    stream_walk(wave, nwave, units, s0, s1, load, [&](const Set& st_, uint32_t u) { body(st_, u, aligned); });
  };
  // the pair's offsets in C are multiples of two elements: 16-byte alignment
  // of every store follows from C's own
  if (P == 2 && (reinterpret_cast<uint64_t>(C) & 15) == 0) run(std::true_type());
  else run(std::false_type());
}

// One-shot variant for ops whose fast-side operand stays in the L2 (without
// accumulation into C): each wavefront writes 2^wide_piece_bits(KN)
// consecutive 64-lane pieces of the fast index for 2^wide_row_bits(KN) rows
// of the shared index, after loading its own operand values (vector loads,
// L2 hits) and the rows' shared values (scalar loads), and ends.  Consecutive
// wavefronts take consecutive pieces, and workgroups start in index order, so
// the stores in flight over the whole chip stay within a narrow window of C;
// persistent wavefronts (the streaming variant) drift apart and spread
// theirs, which the HBM takes more slowly.  The sum over k runs in index
// order from zero, as in the other variants (the same bits whichever runs).
template <typename T, bool FASTN, int P, int KN>
__global__ __launch_bounds__(256) void gemm_smallk_wide(Ctx ctx, GemmOp op, SmallkTables kt) {
  using V = typename C2<T>::t;
  static_assert(P == 1 || (P == 2 && sizeof(T) == 4), "paired stores are 16-byte complex64 pairs");
  constexpr int PB = wide_piece_bits(KN), RB = wide_row_bits(KN);
  constexpr int TP = 1 << PB, RW = 1 << RB;
  static_assert(RW <= kSmallkRows, "row offsets come from the launch tables");
  constexpr int LP = P == 2 ? 1 : 0;
  const int nzh = ctx.n_batch;
  const int z = blockIdx.y % nzh;
  const uint32_t h = blockIdx.y / nzh;
  const int64_t sid = slice_id(ctx, z);
  if (sid < 0) return;
  const int nf = FASTN ? op.n_n : op.n_m;
  const int ns = FASTN ? op.n_m : op.n_n;
  const int gbits = nf - LP - 6 - PB;                   // >= 0 (the launcher checks)
  const uint64_t units = uint64_t(1) << (gbits + ns - RB);
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t u = TN_UNIFORM(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (u >= units) return;
  const int eb = sizeof(V);
  GMEM const V* A = reinterpret_cast<GMEM const V*>(resolve(ctx, op.a, z, sid, eb)) + deposit_runs32(h, op.run_a_h);
  GMEM const V* B = reinterpret_cast<GMEM const V*>(resolve(ctx, op.b, z, sid, eb)) + deposit_runs32(h, op.run_b_h);
  GMEM V* C = reinterpret_cast<GMEM V*>(resolve(ctx, op.c, z, sid, eb)) + deposit_runs32(h, op.run_c_h);
  GMEM const V* F = FASTN ? B : A;
  CMEM const V* S = reinterpret_cast<CMEM const V*>(reinterpret_cast<uintptr_t>(FASTN ? A : B));
  const BitRuns& rf = FASTN ? op.run_b_n : op.run_a_m;
  const BitRuns& rs = FASTN ? op.run_a_m : op.run_b_n;
  const BitRuns& rcf = FASTN ? op.run_c_n : op.run_c_m;
  const BitRuns& rcs = FASTN ? op.run_c_m : op.run_c_n;
  const int cjf = FASTN ? op.conj_b : op.conj_a, cjs = FASTN ? op.conj_a : op.conj_b;
  // pieces: fast index ((g TP + t) 64 + lane) 2^LP; rows r0 .. r0 + RW - 1
  const uint32_t g = u & ((1u << gbits) - 1), r0 = (u >> gbits) << RB;
  const uint32_t lf = deposit_runs32(lane << LP, rf), lcf = deposit_runs32(lane << LP, rcf);
  V fv[TP][P][KN], sv[RW][KN];
#pragma unroll
  for (int t = 0; t < TP; t++) {
    GMEM const V* Fp = F + deposit_runs_u(((g << PB) + t) << (6 + LP), rf) + lf;
#pragma unroll
    for (int p = 0; p < P; p++)
#pragma unroll
      for (int k = 0; k < KN; k++) fv[t][p][k] = conjv(ld(Fp + (p ? kt.f1 : 0u) + kt.kf[k]), cjf);
  }
  const uint32_t so = deposit_runs_u(r0, rs);
#pragma unroll
  for (int i = 0; i < RW; i++)
#pragma unroll
    for (int k = 0; k < KN; k++) sv[i][k] = conjv(ldc(S + so + kt.si[i] + kt.ks[k]), cjs);
  const uint32_t co = deposit_runs_u(r0, rcs);
  uint32_t cp[TP];
#pragma unroll
  for (int t = 0; t < TP; t++) cp[t] = deposit_runs_u(((g << PB) + t) << (6 + LP), rcf);
  auto run = [&](auto aligned) {
#pragma unroll
    for (int i = 0; i < RW; i++)
#pragma unroll
      for (int t = 0; t < TP; t++) {
        V acc[P];
#pragma unroll
        for (int p = 0; p < P; p++) {
          acc[p].x = 0;
          acc[p].y = 0;
        }
#pragma unroll
        for (int k = 0; k < KN; k++)
#pragma unroll
          for (int p = 0; p < P; p++)
            acc[p] = FASTN ? cfma(acc[p], sv[i][k], fv[t][p][k]) : cfma(acc[p], fv[t][p][k], sv[i][k]);
        GMEM V* d = C + co + kt.ci[i] + cp[t] + lcf;
        if constexpr (P == 2) {
          if constexpr (decltype(aligned)::value) {
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
  };
  // as in the streaming variant: 16-byte alignment of every paired store
  // follows from C's own
  if (P == 2 && (reinterpret_cast<uint64_t>(C) & 15) == 0) run(std::true_type());
  else run(std::false_type());
}

// Offset of a small value v (its set bits among the first n of a position list).
inline uint32_t deposit_small(uint32_t v, const int8_t* pos, int n) {
  uint32_t off = 0;
  for (int i = 0; i < n && (v >> i); i++)
    if ((v >> i) & 1) off += uint32_t(1) << pos[i];
  return off;
}


// Kernel variants of a launch.
enum SmallkVariant { kSmallkPlain = 0, kSmallkStream = 1, kSmallkWide = 2 };

// Grid and variant of one launch: units = wavefronts per grid row of the
// streaming and one-shot variants, blocks = workgroups per grid row of the
// plain one.
struct SmallkLaunch {
  bool fastn, pair;
  int variant;
  int kn;
  uint64_t blocks, gy, units;
};

// When the one-shot variant may run (smallk_prepare): never, by the rule
// above, or whatever the output size (the last two for the host emulation's
// tests on small operands).
enum SmallkWideRule { kWideNever = 0, kWideDefault = 1, kWideAnySize = 2 };

// Host side of a launch: the op's position lists as runs, the offset tables
// and the grid.  False when the op does not qualify.
inline bool smallk_prepare(GemmOp& op, int prec, int n_batch, SmallkTables& kt, SmallkLaunch& L,
                           int wide_rule = kWideDefault) {
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
  for (int t = 0; t < 5; t++) kt.dci[t] = kt.ci[1 << t] - kt.ci[(1 << t) - 1];   // i = 2^t - 1 -> 2^t
  const uint64_t threads = (uint64_t(1) << (nf + ns)) / R / (L.pair ? 2 : 1);
  L.blocks = (threads + 255) / 256;
  L.gy = uint64_t(n_batch) << op.n_h;
  L.kn = 1 << op.n_k;
  const int lp = L.pair ? 1 : 0, eb = prec == TN_C128 ? 16 : 8;
  const int kn = 1 << op.n_k, pb = wide_piece_bits(kn), rb = wide_row_bits(kn);
  const int wide_bits = nf - lp - 6 - pb + ns - rb;         // log2 wavefronts per grid row
  if (wide_rule != kWideNever && kn <= kWideMaxSummed && !op.accumulate && nf - lp >= 6 + pb && ns >= rb &&
      wide_bits + 6 <= 31 &&
      (nf + ns >= kWideMinOutputBits || wide_rule == kWideAnySize) &&
      nf + op.n_k + __builtin_ctz(eb) <= kWideOperandBits) {
    L.variant = kSmallkWide;
    L.units = uint64_t(1) << wide_bits;
  } else if (!op.accumulate && nf - lp >= 6) {
    L.variant = kSmallkStream;
    L.units = (threads << (5 - kStreamRowBits)) / 64;        // units of 64 lanes x 2^kStreamRowBits rows
  } else {
    L.variant = kSmallkPlain;
    L.units = 0;
  }
  return true;
}

// Calls f(T(), fastn, p, kn, variant) with the launch's variant as
// std::integral_constant / bool_constant values.
template <class Fn>
inline void smallk_dispatch(const SmallkLaunch& L, int prec, Fn&& f) {
  auto with_kn = [&](auto t, auto fastn, auto p, auto variant) {
    if (L.kn == 1) f(t, fastn, p, std::integral_constant<int, 1>(), variant);
    else if (L.kn == 2) f(t, fastn, p, std::integral_constant<int, 2>(), variant);
    else if (L.kn == 4) f(t, fastn, p, std::integral_constant<int, 4>(), variant);
    else f(t, fastn, p, std::integral_constant<int, 8>(), variant);
  };
  auto with_variant = [&](auto t, auto fastn, auto p) {
    if (L.variant == kSmallkWide) with_kn(t, fastn, p, std::integral_constant<int, kSmallkWide>());
    else if (L.variant == kSmallkStream) with_kn(t, fastn, p, std::integral_constant<int, kSmallkStream>());
    else with_kn(t, fastn, p, std::integral_constant<int, kSmallkPlain>());
  };
  auto with_fastn = [&](auto t, auto p) {
    if (L.fastn) with_variant(t, std::true_type(), p);
    else with_variant(t, std::false_type(), p);
  };
  if (prec == TN_C128) with_fastn(double(), std::integral_constant<int, 1>());
  else if (L.pair) with_fastn(float(), std::integral_constant<int, 2>());
  else with_fastn(float(), std::integral_constant<int, 1>());
}
