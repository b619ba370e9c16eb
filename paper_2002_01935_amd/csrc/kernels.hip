// gfx950 kernels for pairwise tensor contraction (Sec. 2: a vertex
// contraction is the product of two tensors summed over their common,
// no-longer-needed indices).
//
// Every operand is addressed through bit positions (tn_internal.h): element
// offset = sum over bit indices of (bit << position).  Loads therefore read an
// operand in whatever axis order it is stored and writes produce the order
// the consumer asked for; no transpose is ever materialised.
//
// Kernel classes:
//   row_kernel     one thread per output "row" (batch + large free side), the
//                  small free side (<= 16 values) and the summed range inside
//                  the thread; bandwidth-bound gate applications and
//                  absorptions of small tensors into large ones.
//   splitk_kernel  one 64-lane wavefront per (row, K chunk), lanes striding
//                  over the summed indices; long reductions with few outputs
//                  (dot products, skinny contractions).  Chunks are reduced in
//                  a fixed order by reduce_kernel, so results are
//                  deterministic.
//   gemm_mfma_4m   complex GEMM on FP32 matrix cores: the complex product is
//                  embedded as a real product of [Ar Ai] (M x 2K) with
//                  [[Br Bi] [-Bi Br]] (2K x 2N), so one v_mfma_f32_32x32x2f32
//                  with k = (re, im) is one complex multiply-add of a 32 x 16
//                  complex tile: 4 real products (4M), FP32 accumulation.
//   gemm_valu      tiled vector-ALU complex GEMM, used for complex128.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <type_traits>
#include <unordered_map>

#include "kernels.h"

namespace tn {

// Operand pointers are built from integer addresses (workspace offsets and a
// device pointer table); tagging them with the global address space makes the
// compiler emit global (not flat) loads and stores, whose completion counters
// are independent of LDS traffic, so prefetches overlap computation.
#define GMEM __attribute__((address_space(1)))
// Constant address space: uniform read-only data, loaded with scalar loads.
#define CMEM __attribute__((address_space(4)))
// Point where all lanes of a wavefront have passed the preceding LDS writes
// (a wavefront runs its lanes together: only compiler reordering is fenced).
#define TN_WAVE_SYNC() __builtin_amdgcn_wave_barrier()
// A value the same in every lane of the wavefront, made known to the compiler as such.
#define TN_UNIFORM(x) __builtin_amdgcn_readfirstlane(x)

#include "rowops.h"

// ------------------------------------------------------------------ permute / accumulate

template <typename TS, typename TD>
__global__ __launch_bounds__(256) void permute_kernel(Ctx ctx, PermuteOp op) {
  using VS = typename C2<TS>::t;
  using VD = typename C2<TD>::t;
  const uint64_t e = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >> op.n_bits) return;
  const uint64_t so = deposit_runs(e, op.run_src);
  const uint64_t dof = deposit_runs(e, op.run_dst);
  const int z0 = op.per_slice_serial ? 0 : blockIdx.y;
  const int z1 = op.per_slice_serial ? ctx.n_batch : blockIdx.y + 1;
  for (int z = z0; z < z1; z++) {
    const int64_t sid = slice_id(ctx, z);
    if (sid < 0) continue;
    GMEM const VS* S = reinterpret_cast<GMEM const VS*>(resolve(ctx, op.src, z, sid, sizeof(VS)));
    GMEM VD* D = reinterpret_cast<GMEM VD*>(resolve(ctx, op.dst, z, sid, sizeof(VD)));
    const VS s = ld(S + so);
    VD d;
    if (op.accumulate) {
      d = ld(D + dof);
      d.x += (TD)s.x;
      d.y += (TD)s.y;
    } else {
      d.x = (TD)s.x;
      d.y = (TD)s.y;
    }
    st(D + dof, d);
  }
}

// dst (complex128) += root of every in-flight slice, one slice after the
// other in slice order: the FP64 sum has the same rounding whatever the batch.
template <typename T>
__global__ __launch_bounds__(256) void accum_kernel(Ctx ctx, AccumOp op) {
  using V = typename C2<T>::t;
  const int64_t o = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (o >= op.n) return;
  GMEM double2* D = reinterpret_cast<GMEM double2*>(resolve(ctx, op.dst, 0, 0, 16));
  double2 d = ld(D + o);
  for (int z = 0; z < ctx.n_batch; z++) {
    const int64_t sid = slice_id(ctx, z);
    if (sid < 0) continue;
    GMEM const V* S = reinterpret_cast<GMEM const V*>(resolve(ctx, op.src, z, sid, sizeof(V)));
    const V s = ld(S + o);
    d.x += (double)s.x;
    d.y += (double)s.y;
  }
  st(D + o, d);
}

__global__ void counter_kernel(Ctx ctx, int64_t value, int add) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    int64_t* c = reinterpret_cast<int64_t*>(ctx.ws + ctx.counter_off);
    *c = add ? *c + value : value;
  }
}

// Zeroes n_words 8-byte words: one per work-item up to 2^31 words (the
// stores in flight then cover a narrow window of memory), grid-stride beyond
// (a launch holds fewer than 2^32 work-items per grid dimension, and arenas
// or complex128 outputs can hold more words than that).
__global__ __launch_bounds__(256) void fill_kernel(uint64_t base, uint64_t n_words) {
  const uint64_t step = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n_words; i += step)
    reinterpret_cast<uint64_t*>(base)[i] = 0;
}

// ------------------------------------------------------------------ tile loaders

// Enumerates the elements of an R x Kt tile of a bit-addressed operand in the
// order of their memory addresses (tile bits sorted by position), so that
// consecutive threads touch consecutive addresses whenever the operand's
// lowest bits lie inside the tile; returns the element offset within the tile
// and its (row, k) position in the tile.
struct TileMap {
  int nbits;
  int8_t pos[kMaxTileBits];   // operand position of tile bit i (rows first, then k)
  int8_t dst[kMaxTileBits];   // its bit in the tile index (row | k << rlog)
  int8_t rank[kMaxTileBits];  // its place in increasing position order = bit of the enumeration index
};

// All loops run over the fixed maximum with predication, so the arrays are
// indexed statically and stay in registers.
__device__ __forceinline__ void make_tilemap(TileMap& tm, const int8_t* rowpos, int rbits,
                                             const int8_t* kpos, int kbits, int rlog) {
#pragma unroll
  for (int i = 0; i < kMaxTileBits; i++) {
    const bool isr = i < rbits, isk = !isr && i < rbits + kbits;
    tm.pos[i] = (int8_t)(isr ? pos_at(rowpos, i) : (isk ? pos_at(kpos, i - rbits) : 127));
    tm.dst[i] = (int8_t)(isr ? i : (isk ? rlog + i - rbits : 0));
  }
#pragma unroll
  for (int i = 0; i < kMaxTileBits; i++) {
    int r = 0;
#pragma unroll
    for (int j = 0; j < kMaxTileBits; j++) r += tm.pos[j] < tm.pos[i];
    tm.rank[i] = (int8_t)r;
  }
  tm.nbits = rbits + kbits;
}

// Operand offset and tile index of enumeration element e.
__device__ __forceinline__ void tile_elem(const TileMap& m, uint32_t e, uint64_t& off, int& d) {
  off = 0;
  d = 0;
#pragma unroll
  for (int i = 0; i < kMaxTileBits; i++)
    if (i < m.nbits) {
      const uint32_t bit = (e >> m.rank[i]) & 1u;
      off |= uint64_t(bit) << m.pos[i];
      d |= int(bit) << m.dst[i];
    }
}

// ------------------------------------------------------------------ matrix-core GEMMs

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Per-thread load slots of one operand tile: element offset in the operand and
// destination (row | k << rbits) in the tile; unused slots read element 0.
template <int L, int NT>
__device__ __forceinline__ void tile_slots(const TileMap& m, int tid, uint32_t* off, int16_t* dst) {
#pragma unroll
  for (int i = 0; i < L; i++) {
    const int e = tid + NT * i;
    uint64_t o;
    int d;
    tile_elem(m, e, o, d);
    const bool ok = (e >> m.nbits) == 0;
    off[i] = ok ? (uint32_t)o : 0u;
    dst[i] = ok ? (int16_t)d : (int16_t)-1;
  }
}

// XCD-aware tile order: consecutive block ids land on different XCDs (8 per
// chip), so each XCD gets a contiguous range of output tiles (shared A rows and
// B columns stay in its own L2).
__device__ __forceinline__ uint64_t xcd_tile(uint64_t bid, uint64_t ntiles) {
  return (ntiles & 7) == 0 ? (bid & 7) * (ntiles >> 3) + (bid >> 3) : bid;
}

struct GemmSetup {
  int tm, tn, tk;
  uint64_t tile_m, tile_n, h;
  int z;
  int64_t sid;
  uint64_t ka, kb, cs;   // split-K offsets of this block's summed range in A and B, and of its partial tile
};

__device__ __forceinline__ bool gemm_setup(const Ctx& ctx, const GemmOp& op, int rm, int rn, int rk, GemmSetup& g) {
  const int nzh = ctx.n_batch;
  g.z = blockIdx.y % nzh;
  g.h = blockIdx.y / nzh;
  g.sid = slice_id(ctx, g.z);
  if (g.sid < 0) return false;
  g.tm = op.n_m < rm ? op.n_m : rm;
  g.tn = op.n_n < rn ? op.n_n : rn;
  g.tk = op.n_k < rk ? op.n_k : rk;
  const uint64_t ntiles_n = uint64_t(1) << (op.n_n - g.tn);
  const uint64_t ntiles = (uint64_t(1) << (op.n_m - g.tm)) * ntiles_n;
  if (blockIdx.x >= ntiles) return false;
  // Within an XCD's range, tiles run in groups of up to 8 tile rows with the
  // row index fastest: the ~64 tiles resident on one XCD at a time then span
  // about 8 x 8 tiles, so each A row panel and B column panel they stream is
  // shared by ~8 of them through that XCD's L2 (instead of one A panel shared
  // by all and every B panel fetched separately).
  const uint64_t t = xcd_tile(blockIdx.x, ntiles);
  const int gm_bits = (op.n_m - g.tm) < 3 ? (op.n_m - g.tm) : 3;
  const uint64_t in_group = ntiles_n << gm_bits;
  const uint64_t r = t & (in_group - 1);
  g.tile_m = ((t >> (op.n_n - g.tn + gm_bits)) << gm_bits) + (r & ((uint64_t(1) << gm_bits) - 1));
  g.tile_n = r >> gm_bits;
  g.ka = deposit_runs(blockIdx.z, op.run_a_s);
  g.kb = deposit_runs(blockIdx.z, op.run_b_s);
  g.cs = uint64_t(blockIdx.z) << op.c_split_shift;
  return true;
}

// Epilogue shared by the matrix-core kernels: C[row, col] at
// deposit(row, c_m) + deposit(col, c_n) (+ batch) from the 32 x 32 FP32
// accumulator layout (lane l holds column l % 32, rows 8 (r / 4) + 4 (l / 32) +
// r % 4); real column 2 n + p is part p of complex column n.
template <int BM, int BN, int FM, int FN>
__device__ __forceinline__ void gemm_store(const Ctx& ctx, const GemmOp& op, const GemmSetup& g, uint64_t* tab,
                                           const floatx16 (&acc)[FM][FN], int wm, int wn, int tid, int nthreads) {
  constexpr int WM = FM * 32, WN = FN * 16;
  GMEM float* C = reinterpret_cast<GMEM float*>(resolve(ctx, op.c, g.z, g.sid, 8));
  const uint64_t cbase = g.cs + deposit_runs(g.h, op.run_c_h) + deposit_runs(g.tile_m << g.tm, op.run_c_m) +
                         deposit_runs(g.tile_n << g.tn, op.run_c_n);
  uint64_t* rowoff = tab;
  uint64_t* coloff = tab + BM;
  // tile-local offsets from the run tables (bits below tm / tn; deposits of
  // disjoint bit sets add)
  for (int i = tid; i < BM; i += nthreads) rowoff[i] = deposit_runs(uint64_t(i), op.run_c_m);
  for (int i = tid; i < BN; i += nthreads) coloff[i] = deposit_runs(uint64_t(i), op.run_c_n);
  __syncthreads();
  const int lane = tid & 63, hi = lane >> 5, c32 = lane & 31, odd = c32 & 1;
  const int mvalid = 1 << g.tm, nvalid = 1 << g.tn;
  GMEM float2* C2 = reinterpret_cast<GMEM float2*>(C);
  // Lanes 2c and 2c+1 hold the real and imaginary parts of column c for the
  // same rows.  They swap one value per row pair (r, r+1) so that the even
  // lane owns the complex value of row r and the odd lane that of row r+1:
  // one 8-byte store per complex output.
#pragma unroll
  for (int i = 0; i < FM; i++)
#pragma unroll
    for (int j = 0; j < FN; j++) {
      const int col = wn * WN + j * 16 + (c32 >> 1);
      const uint64_t co = col < nvalid ? coloff[col] : 0;
#pragma unroll
      for (int r = 0; r < 16; r += 2) {
        const float send = odd ? acc[i][j][r] : acc[i][j][r + 1];
        // quad permutation [1, 0, 3, 2]: exchange with the neighbouring lane
        const float recv = __builtin_bit_cast(
            float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, send), 0xB1, 0xF, 0xF, false));
        float2 v;
        v.x = odd ? recv : acc[i][j][r];
        v.y = odd ? acc[i][j][r + 1] : recv;
        const int rr = r + odd;
        const int row = wm * WM + i * 32 + 8 * (rr >> 2) + 4 * hi + (rr & 3);
        if (col >= nvalid || row >= mvalid) continue;
        GMEM float2* dst = C2 + cbase + rowoff[row] + co;
        if (op.accumulate) {
          const float2 o = ld(dst);
          v.x += o.x;
          v.y += o.y;
        }
        st(dst, v);
      }
    }
}

// 4M on FP32 matrix cores.  The complex product is the real product of
// [Ar Ai] (M x 2K) with [[Br Bi] [-Bi Br]] (2K x 2N): one
// v_mfma_f32_32x32x2f32 whose k pair is (re, im) is one complex multiply-add
// of a 32 x 16 complex tile.  BM x BN complex outputs per block of
// WGM x WGN waves, each wave 64 x 64; 8 complex k values per pipeline stage.
// LDS keeps A and B as re / im planes with k contiguous per row (row stride
// 12 floats: 128-bit reads of 16 lanes hit disjoint banks).  Each lane reads
// the fragments of 4 k values with one 128-bit load per fragment, and the
// loads for k 4..7 are in flight while the matrix cores work on k 0..3.
template <int BM, int BN, int WGM, int WGN, int PRIO = 0>
__global__ __launch_bounds__(64 * WGM * WGN) __attribute__((amdgpu_waves_per_eu(2))) void gemm_mfma_4m(Ctx ctx, GemmOp op) {
  constexpr int BK = 8, LDR = 12;
  constexpr int NT = 64 * WGM * WGN;
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int FM = WM / 32, FN = WN / 16;
  constexpr int LA = BM * BK / NT, LB = BN * BK / NT;
  constexpr int RM = __builtin_ctz(BM), RN = __builtin_ctz(BN), RK = 3;
  static_assert(FM >= 1 && FN >= 1 && LA >= 1 && LB >= 1, "tile too small");
  // [buffer][plane re / im][A rows | B cols][k]; the planes are 32 words
  // apart modulo the 64 LDS banks, so the lanes of a B fragment read, which
  // mix the two planes, stay conflict-free
  constexpr int PS = (BM + BN) * LDR + 32;
  __shared__ __attribute__((aligned(16))) float lds[4 * PS];
  static_assert(sizeof(lds) >= (BM + BN) * sizeof(uint64_t), "lds too small for epilogue tables");
  auto L = [&](int buf, int plane, int row) -> float* { return &lds[(2 * buf + plane) * PS + row * LDR]; };

  GemmSetup g;
  if (!gemm_setup(ctx, op, RM, RN, RK, g)) return;
  GMEM const float2* A = reinterpret_cast<GMEM const float2*>(resolve(ctx, op.a, g.z, g.sid, 8)) + g.ka +
                         deposit_runs(g.h, op.run_a_h) + deposit_runs(g.tile_m << g.tm, op.run_a_m);
  GMEM const float2* B = reinterpret_cast<GMEM const float2*>(resolve(ctx, op.b, g.z, g.sid, 8)) + g.kb +
                         deposit_runs(g.h, op.run_b_h) + deposit_runs(g.tile_n << g.tn, op.run_b_n);
  const int tid = threadIdx.x;
  uint32_t a_off[LA], b_off[LB];
  int16_t a_dst[LA], b_dst[LB];
  {
    TileMap ma, mb;
    make_tilemap(ma, op.a_m, g.tm, op.a_k, g.tk, RM);
    make_tilemap(mb, op.b_n, g.tn, op.b_k, g.tk, RN);
    tile_slots<LA, NT>(ma, tid, a_off, a_dst);
    tile_slots<LB, NT>(mb, tid, b_off, b_dst);
  }
  for (int i = tid; i < 4 * PS; i += NT) lds[i] = 0.f;
  // k offsets of consecutive pipeline stages, advanced stage by stage with
  // the per-carry deltas of each operand (LDS table: no scalar loads, whose
  // completion wait would also drain the LDS reads in flight, in the loop)
  __shared__ uint64_t kdel[2][kMaxBits];
  for (int t = tid; t < op.n_k - g.tk; t += NT) {
    const uint64_t c = (uint64_t(1) << t) - 1;
    kdel[0][t] = step_delta(c, op.a_k, g.tk);
    kdel[1][t] = step_delta(c, op.b_k, g.tk);
  }
  __syncthreads();

  const uint64_t nsteps = uint64_t(1) << (op.n_k - g.tk);
  const float sa = op.conj_a ? -1.f : 1.f, sb = op.conj_b ? -1.f : 1.f;
  float2 ra[LA], rb[LB];
  uint64_t ka = 0, kb = 0, kstep = 0;
  auto gload = [&]() {
#pragma unroll
    for (int i = 0; i < LA; i++) ra[i] = ld(A + ka + a_off[i]);
#pragma unroll
    for (int i = 0; i < LB; i++) rb[i] = ld(B + kb + b_off[i]);
    if (kstep + 1 < nsteps) {
      const int t = __builtin_ctzll(~kstep);
      ka += kdel[0][t];
      kb += kdel[1][t];
    }
    kstep++;
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < LA; i++)
      if (a_dst[i] >= 0) {
        const int row = a_dst[i] & (BM - 1), k = a_dst[i] >> RM;
        L(buf, 0, row)[k] = ra[i].x;
        L(buf, 1, row)[k] = sa * ra[i].y;
      }
#pragma unroll
    for (int i = 0; i < LB; i++)
      if (b_dst[i] >= 0) {
        const int col = b_dst[i] & (BN - 1), k = b_dst[i] >> RN;
        L(buf, 0, BM + col)[k] = rb[i].x;
        L(buf, 1, BM + col)[k] = sb * rb[i].y;
      }
  };

  const int wave = tid >> 6, lane = tid & 63;
  const int wm = wave / WGN, wn = wave % WGN;
  const int hi = lane >> 5;                 // 0: real part of k, 1: imaginary part
  const int c32 = lane & 31;
  const int bpar = c32 & 1;                 // output column parity: re / im
  const int bsel = bpar ^ hi;               // which part of B feeds this lane
  const float bsign = (bpar == 0 && hi == 1) ? -1.f : 1.f;
  const int arow = wm * WM + c32;
  const int bcol = BM + wn * WN + (c32 >> 1);
  floatx16 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; i++)
#pragma unroll
    for (int j = 0; j < FN; j++)
#pragma unroll
      for (int r = 0; r < 16; r++) acc[i][j][r] = 0.f;

  f4 fa[2][FM], fb[2][FN];
  auto fread = [&](int buf, int half) {
#pragma unroll
    for (int i = 0; i < FM; i++) fa[half][i] = *reinterpret_cast<const f4*>(L(buf, hi, arow + i * 32) + 4 * half);
#pragma unroll
    for (int j = 0; j < FN; j++) fb[half][j] = *reinterpret_cast<const f4*>(L(buf, bsel, bcol + j * 16) + 4 * half);
  };

  gload();
  sstore(0);
  __syncthreads();
  for (uint64_t s = 0; s < nsteps; s++) {
    const int buf = s & 1;
    if (s + 1 < nsteps) gload();
    fread(buf, 0);
    fread(buf, 1);
    if (PRIO) __builtin_amdgcn_s_setprio(1);   // keep this wave's matrix-core issue ahead of the other wave's loads
#pragma unroll
    for (int half = 0; half < 2; half++) {
#pragma unroll
      for (int j = 0; j < FN; j++) fb[half][j] *= bsign;
#pragma unroll
      for (int kk = 0; kk < 4; kk++)
#pragma unroll
        for (int i = 0; i < FM; i++)
#pragma unroll
          for (int j = 0; j < FN; j++)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa[half][i][kk], fb[half][j][kk], acc[i][j], 0, 0, 0);
    }
    if (PRIO) __builtin_amdgcn_s_setprio(0);
    if (s + 1 < nsteps) sstore(buf ^ 1);
    __syncthreads();
  }
  gemm_store<BM, BN, FM, FN>(ctx, op, g, reinterpret_cast<uint64_t*>(&lds[0]), acc, wm, wn, tid, NT);
}

// Operand ring of the direct-to-LDS kernels, for operands whose summed bits
// are their lowest positions, in order (k bit i at position i: every
// intermediate the planner lays out, and most leaves).  Each tile row is then
// 8 contiguous complex values per stage, so the stage is copied straight from
// global memory into LDS by global_load_lds_dwordx4 (16 bytes = two complex
// values per lane, no registers in between), into a ring of three LDS
// buffers: two stages are in flight while the matrix cores work on the third,
// with one barrier per stage.  LDS keeps the complex values interleaved, 4
// units of 16 bytes per row (the BM A rows, then the BN B rows); the unit
// holding k pair kp of row r sits at r * 4 + (kp ^ ((r >> 2) & 3)), a swizzle
// applied by choosing which element each lane loads (the lane's LDS slot is
// fixed), so that the 128-bit fragment reads of 16 lanes on distinct rows
// hit disjoint banks.
__device__ __forceinline__ int dl_unit(int r, int kp) { return r * 4 + (kp ^ ((r >> 2) & 3)); }

template <int BM, int BN, int NW, int NB = 3>
struct DlRing {
  static constexpr int IA = BM * 4 / 64 / NW, IB = BN * 4 / 64 / NW;   // load instructions per wave and stage
  static constexpr int NBUF = NB;
  static constexpr int UNITS = (BM + BN) * 4;                            // 16-byte units per buffer
  static_assert(IA >= 1 && IB >= 1, "tile too small");
  static_assert(IA * NW * 64 == BM * 4 && IB * NW * 64 == BN * 4, "tile / wave mismatch");
  GMEM const float2* A;
  GMEM const float2* B;
  uint32_t a_off[IA], b_off[IB];          // element offset (tile row, k pair) of every unit this lane loads

  __device__ __forceinline__ DlRing(const Ctx& ctx, const GemmOp& op, const GemmSetup& g, int wave, int lane) {
    A = reinterpret_cast<GMEM const float2*>(resolve(ctx, op.a, g.z, g.sid, 8)) + deposit_runs(g.h, op.run_a_h) + g.ka;
    B = reinterpret_cast<GMEM const float2*>(resolve(ctx, op.b, g.z, g.sid, 8)) + deposit_runs(g.h, op.run_b_h) + g.kb;
    const uint64_t mrows = uint64_t(1) << g.tm, nrows = uint64_t(1) << g.tn;
#pragma unroll
    for (int i = 0; i < IA; i++) {
      const int slot = (wave * IA + i) * 64 + lane;
      const int r = slot >> 2, kp = (slot & 3) ^ ((r >> 2) & 3);
      const uint64_t rr = uint64_t(r) < mrows ? uint64_t(r) : 0;      // rows past a partial tile repeat row 0
      a_off[i] = (uint32_t)deposit_runs((g.tile_m << g.tm) | rr, op.run_a_m) + 2 * kp;   // tensors hold < 2^32 elements
    }
#pragma unroll
    for (int i = 0; i < IB; i++) {
      const int slot = (wave * IB + i) * 64 + lane;
      const int r = slot >> 2, kp = (slot & 3) ^ ((r >> 2) & 3);
      const uint64_t rr = uint64_t(r) < nrows ? uint64_t(r) : 0;
      b_off[i] = (uint32_t)deposit_runs((g.tile_n << g.tn) | rr, op.run_b_n) + 2 * kp;
    }
  }

  // start the loads of stage `step` into its ring buffer
  __device__ __forceinline__ void issue(f4* lds, uint64_t step, int wave) const {
    issue_into(lds, step, (int)(step % NBUF), wave);
  }
  __device__ __forceinline__ void issue_into(f4* lds, uint64_t step, int buf, int wave) const {
    const uint32_t k0 = (uint32_t)(step << 3);
#pragma unroll
    for (int i = 0; i < IA; i++)
      __builtin_amdgcn_global_load_lds((GMEM const void*)(A + a_off[i] + k0),
                                       (__attribute__((address_space(3))) void*)(&lds[buf * UNITS + (wave * IA + i) * 64]),
                                       16, 0, 0);
#pragma unroll
    for (int i = 0; i < IB; i++)
      __builtin_amdgcn_global_load_lds((GMEM const void*)(B + b_off[i] + k0),
                                       (__attribute__((address_space(3))) void*)(&lds[buf * UNITS + BM * 4 + (wave * IB + i) * 64]),
                                       16, 0, 0);
  }

  // Waits until stage s is in LDS for every wave and every wave is done with
  // the buffer of stage s - 1 (its fragment reads were consumed by the matrix
  // cores).  This wave's loads of stage s are done once at most those of
  // stage s + 1 remain (the direct-to-LDS data is in LDS when its load
  // retires); then a plain barrier: a fence would also drain the stage s + 1
  // loads.
  __device__ __forceinline__ static void wait(bool more) {
    if (more) __builtin_amdgcn_s_waitcnt((IA + IB) | (0x7 << 4) | (0xF << 8));
    else __builtin_amdgcn_s_waitcnt(0 | (0x7 << 4) | (0xF << 8));
    __builtin_amdgcn_s_barrier();
  }
  // the same with the loads of the `ahead` (constant) later stages still in flight
  template <int AHEAD>
  __device__ __forceinline__ static void wait_ahead() {
    static_assert(AHEAD * (IA + IB) < 16, "wait counter field");
    __builtin_amdgcn_s_waitcnt((AHEAD * (IA + IB)) | (0x7 << 4) | (0xF << 8));
    __builtin_amdgcn_s_barrier();
  }
};

// 4M on the direct-to-LDS ring.  A lane of half hi reads complex
// k = 4q + 2hi, 4q + 2hi + 1 of its row as (re, im, re, im); the four
// matrix-core ops of k group q pair the real k indices (re, im, re, im of
// 4q + {0, 1}) of the lower half with those of 4q + {2, 3} of the upper half,
// and each lane forms the matching entries of [[Br Bi] [-Bi Br]] from its B
// unit with selects.
template <int BM, int BN, int WGM, int WGN, int OCC = 2>
__global__ __launch_bounds__(64 * WGM * WGN) __attribute__((amdgpu_waves_per_eu(OCC))) void gemm_mfma_4m_dl(Ctx ctx, GemmOp op) {
  constexpr int NT = 64 * WGM * WGN, NW = WGM * WGN;
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int FM = WM / 32, FN = WN / 16;
  constexpr int RM = __builtin_ctz(BM), RN = __builtin_ctz(BN), RK = 3;
  static_assert(FM >= 1 && FN >= 1, "tile too small");
  typedef DlRing<BM, BN, NW> Ring;
  __shared__ __attribute__((aligned(16))) f4 lds[Ring::NBUF * Ring::UNITS];
  static_assert(sizeof(lds) >= (BM + BN) * sizeof(uint64_t), "lds too small for epilogue tables");

  GemmSetup g;
  if (!gemm_setup(ctx, op, RM, RN, RK, g)) return;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const Ring ring(ctx, op, g, wave, lane);
  const uint64_t nsteps = uint64_t(1) << (op.n_k - RK);

  const int wm = wave / WGN, wn = wave % WGN;
  const int hi = lane >> 5, c32 = lane & 31, p = c32 & 1;
  const float sa = op.conj_a ? -1.f : 1.f, sb = op.conj_b ? -1.f : 1.f;
  floatx16 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; i++)
#pragma unroll
    for (int j = 0; j < FN; j++)
#pragma unroll
      for (int r = 0; r < 16; r++) acc[i][j][r] = 0.f;

  ring.issue(lds, 0, wave);
  if (nsteps > 1) ring.issue(lds, 1, wave);
  for (uint64_t s = 0; s < nsteps; s++) {
    Ring::wait(s + 1 < nsteps);
    if (s + 2 < nsteps) ring.issue(lds, s + 2, wave);
    const f4* L = &lds[(int)(s % Ring::NBUF) * Ring::UNITS];
#pragma unroll
    for (int q = 0; q < 2; q++) {
      const int kp = 2 * q + hi;
      f4 fa[FM];
#pragma unroll
      for (int i = 0; i < FM; i++) {
        fa[i] = L[dl_unit(wm * WM + i * 32 + c32, kp)];
        fa[i][1] *= sa;
        fa[i][3] *= sa;
      }
      // one B fragment at a time (fewer live registers), the next one read
      // while the matrix cores work on this one; consecutive matrix-core ops
      // alternate between the FM accumulators of column block j
      auto bunit = [&](int j) { return L[BM * 4 + dl_unit(wn * WN + j * 16 + (c32 >> 1), kp)]; };
      f4 u = bunit(0);
#pragma unroll
      for (int j = 0; j < FN; j++) {
        const f4 uj = u;
        if (j + 1 < FN) u = bunit(j + 1);
        const float br0 = uj[0], bi0 = sb * uj[1], br1 = uj[2], bi1 = sb * uj[3];
        f4 v;
        v[0] = p ? bi0 : br0;       // real k = re of the first complex k
        v[1] = p ? br0 : -bi0;      // im of the first
        v[2] = p ? bi1 : br1;       // re of the second
        v[3] = p ? br1 : -bi1;      // im of the second
#pragma unroll
        for (int e = 0; e < 4; e++)
#pragma unroll
          for (int i = 0; i < FM; i++)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa[i][e], v[e], acc[i][j], 0, 0, 0);
      }
    }
  }
  __syncthreads();                         // the epilogue reuses the LDS ring for its tables
  gemm_store<BM, BN, FM, FN>(ctx, op, g, reinterpret_cast<uint64_t*>(&lds[0]), acc, wm, wn, tid, NT);
}

// 4M on a ring of four stages with the next stage's fragments read during
// the matrix-core work: at stage s the wave waits for stage s + 1's loads
// (s + 2 stays in flight), passes the barrier (after which the buffer of
// stage s - 1, whose fragments every wave read one stage earlier, is free),
// starts the loads of stage s + 3 into it, and then issues stage s's
// matrix-core ops block by block (k group q, column block j), reading stage
// s + 1's B unit of a block into its registers right after the block's last
// op and stage s + 1's A fragments of a k group after its last block.  Every
// stage runs the same operations (past the last stage the loads fetch the
// last stage again, into a buffer no later read uses, and the reads re-read
// it), so the compiler's wait counts hold on every pass.  A's conjugation is
// folded into the B entries it multiplies.
template <int BM, int BN, int WGM, int WGN, int OCC>
__global__ __launch_bounds__(64 * WGM * WGN) __attribute__((amdgpu_waves_per_eu(OCC))) void gemm_mfma_4m_dlp(Ctx ctx, GemmOp op) {
  constexpr int NT = 64 * WGM * WGN, NW = WGM * WGN, NB = 4;
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int FM = WM / 32, FN = WN / 16;
  constexpr int RM = __builtin_ctz(BM), RN = __builtin_ctz(BN), RK = 3;
  static_assert(FM >= 1 && FN >= 1, "tile too small");
  typedef DlRing<BM, BN, NW, NB> Ring;
  __shared__ __attribute__((aligned(16))) f4 lds[NB * Ring::UNITS];
  static_assert(sizeof(lds) >= (BM + BN) * sizeof(uint64_t), "lds too small for epilogue tables");

  GemmSetup g;
  if (!gemm_setup(ctx, op, RM, RN, RK, g)) return;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const Ring ring(ctx, op, g, wave, lane);
  const uint32_t nsteps = 1u << (op.n_k - RK);                 // a power of two (tensors hold < 2^32 elements)
  const int wm = wave / WGN, wn = wave % WGN;
  const int hi = lane >> 5, c32 = lane & 31, p = c32 & 1;
  const float sa = op.conj_a ? -1.f : 1.f, sb = op.conj_b ? -1.f : 1.f;
  floatx16 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; i++)
#pragma unroll
    for (int j = 0; j < FN; j++)
#pragma unroll
      for (int r = 0; r < 16; r++) acc[i][j][r] = 0.f;

  auto buf = [&](uint32_t s) { return &lds[(s & (NB - 1)) * Ring::UNITS]; };   // stage s's buffer
  f4 fa[2][FM], fb[2][FN];                                     // raw LDS units, refilled as they die
  auto read_a = [&](int q, uint32_t s) {
    const f4* L = buf(s);
#pragma unroll
    for (int i = 0; i < FM; i++) fa[q][i] = L[dl_unit(wm * WM + i * 32 + c32, 2 * q + hi)];
  };
  auto read_b = [&](int q, int j, uint32_t s) {
    fb[q][j] = buf(s)[BM * 4 + dl_unit(wn * WN + j * 16 + (c32 >> 1), 2 * q + hi)];
  };
  auto block = [&](int q, int j) {
    const f4 u = fb[q][j];
    const float br0 = u[0], bi0 = sb * u[1], br1 = u[2], bi1 = sb * u[3];
    f4 v;
    v[0] = p ? bi0 : br0;           // real k = re of the first complex k
    v[1] = sa * (p ? br0 : -bi0);   // im of the first (A's imaginary part, conjugated when conj_a)
    v[2] = p ? bi1 : br1;           // re of the second
    v[3] = sa * (p ? br1 : -bi1);   // im of the second
#pragma unroll
    for (int e = 0; e < 4; e++)
#pragma unroll
      for (int i = 0; i < FM; i++)
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa[q][i][e], v[e], acc[i][j], 0, 0, 0);
  };
  const uint32_t last = nsteps - 1;
  auto clamp = [&](uint32_t t) { return t < last ? t : last; };
  for (int q = 0; q < NB - 1; q++) ring.issue_into(lds, clamp((uint32_t)q), q, wave);
  Ring::template wait_ahead<2>();                             // stage 0 loaded
#pragma unroll
  for (int q = 0; q < 2; q++) {
    read_a(q, 0);
#pragma unroll
    for (int j = 0; j < FN; j++) read_b(q, j, 0);
  }
  for (uint32_t s = 0; s < nsteps; s++) {
    Ring::template wait_ahead<1>();                           // stage s + 1 loaded, s + 2 in flight
    ring.issue_into(lds, clamp(s + 3), (s + 3) & (NB - 1), wave);
    const uint32_t nx = clamp(s + 1);
    // (scheduling barriers keep the compiler from reordering the blocks)
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int q = 0; q < 2; q++)
#pragma unroll
      for (int j = 0; j < FN; j++) {
        block(q, j);
        read_b(q, j, nx);
        if (j == FN - 1) read_a(q, nx);
        __builtin_amdgcn_sched_barrier(0);
      }
  }
  Ring::template wait_ahead<0>();          // no load into the ring still in flight
  __syncthreads();                         // the epilogue reuses the LDS ring for its tables
  gemm_store<BM, BN, FM, FN>(ctx, op, g, reinterpret_cast<uint64_t*>(&lds[0]), acc, wm, wn, tid, NT);
}

// Epilogue of the 3M kernels: with T1, T2, T3 the three real accumulator
// planes of a 32 x 32 complex tile (lane l holds complex column l % 32, rows
// 8 (r / 4) + 4 (l / 32) + r % 4), C = (T1 - T2) + i (T3 - T1 - T2) at
// deposit(row, c_m) + deposit(col, c_n) (+ batch).
template <int BM, int BN, int FM, int FN>
__device__ __forceinline__ void gemm_store_3m(const Ctx& ctx, const GemmOp& op, const GemmSetup& g, uint64_t* tab,
                                              const floatx16 (&acc)[3][FM][FN], int wm, int wn, int tid, int nthreads) {
  constexpr int WM = FM * 32, WN = FN * 32;
  GMEM float2* C = reinterpret_cast<GMEM float2*>(resolve(ctx, op.c, g.z, g.sid, 8));
  const uint64_t cbase = g.cs + deposit_runs(g.h, op.run_c_h) + deposit_runs(g.tile_m << g.tm, op.run_c_m) +
                         deposit_runs(g.tile_n << g.tn, op.run_c_n);
  uint64_t* rowoff = tab;
  uint64_t* coloff = tab + BM;
  // tile-local offsets from the run tables (bits below tm / tn; deposits of
  // disjoint bit sets add)
  for (int i = tid; i < BM; i += nthreads) rowoff[i] = deposit_runs(uint64_t(i), op.run_c_m);
  for (int i = tid; i < BN; i += nthreads) coloff[i] = deposit_runs(uint64_t(i), op.run_c_n);
  __syncthreads();
  const int lane = tid & 63, hi = lane >> 5, c32 = lane & 31;
  const int mvalid = 1 << g.tm, nvalid = 1 << g.tn;
#pragma unroll
  for (int i = 0; i < FM; i++)
#pragma unroll
    for (int j = 0; j < FN; j++) {
      const int col = wn * WN + j * 32 + c32;
      if (col >= nvalid) continue;
      const uint64_t co = coloff[col];
#pragma unroll
      for (int r = 0; r < 16; r++) {
        const int row = wm * WM + i * 32 + 8 * (r >> 2) + 4 * hi + (r & 3);
        if (row >= mvalid) continue;
        const float t1 = acc[0][i][j][r], t2 = acc[1][i][j][r], t3 = acc[2][i][j][r];
        float2 v;
        v.x = t1 - t2;
        v.y = t3 - t1 - t2;
        GMEM float2* dst = C + cbase + rowoff[row] + co;
        if (op.accumulate) {
          const float2 o = ld(dst);
          v.x += o.x;
          v.y += o.y;
        }
        st(dst, v);
      }
    }
}

// 3M (Gauss) on FP32 matrix cores: with T1 = Ar Br, T2 = Ai Bi and
// T3 = (Ar + Ai)(Br + Bi), Re = T1 - T2 and Im = T3 - T1 - T2: three real
// products per complex product instead of four.  Each v_mfma_f32_32x32x2f32
// takes two complex k values of one real plane for a 32 x 32 complex tile.
// LDS keeps the planes A: re, im, re + im and B: re, im, re + im, k
// contiguous per row, with the k order (k & 1) * 4 + (k >> 1) inside each
// 8-value stage so that the four k values a lane feeds (its half of the k
// pairs) are one 128-bit read.  BM x BN complex outputs per block of
// WGM x WGN waves, each wave 64 x 32.
template <int BM, int BN, int WGM, int WGN>
__global__ __launch_bounds__(64 * WGM * WGN) __attribute__((amdgpu_waves_per_eu(2))) void gemm_mfma_3m(Ctx ctx, GemmOp op) {
  constexpr int BK = 8, LDR = 12;
  constexpr int NT = 64 * WGM * WGN;
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int FM = WM / 32, FN = WN / 32;
  constexpr int LA = BM * BK / NT, LB = BN * BK / NT;
  constexpr int RM = __builtin_ctz(BM), RN = __builtin_ctz(BN), RK = 3;
  static_assert(FM >= 1 && FN >= 1 && LA >= 1 && LB >= 1, "tile too small");
  __shared__ __attribute__((aligned(16))) float lds[2][3][BM + BN][LDR];   // [buffer][re, im, re+im][rows | cols][k]
  static_assert(sizeof(lds) >= (BM + BN) * sizeof(uint64_t), "lds too small for epilogue tables");

  GemmSetup g;
  if (!gemm_setup(ctx, op, RM, RN, RK, g)) return;
  GMEM const float2* A = reinterpret_cast<GMEM const float2*>(resolve(ctx, op.a, g.z, g.sid, 8)) + g.ka +
                         deposit_runs(g.h, op.run_a_h) + deposit_runs(g.tile_m << g.tm, op.run_a_m);
  GMEM const float2* B = reinterpret_cast<GMEM const float2*>(resolve(ctx, op.b, g.z, g.sid, 8)) + g.kb +
                         deposit_runs(g.h, op.run_b_h) + deposit_runs(g.tile_n << g.tn, op.run_b_n);
  const int tid = threadIdx.x;
  uint32_t a_off[LA], b_off[LB];
  int16_t a_dst[LA], b_dst[LB];
  {
    TileMap ma, mb;
    make_tilemap(ma, op.a_m, g.tm, op.a_k, g.tk, RM);
    make_tilemap(mb, op.b_n, g.tn, op.b_k, g.tk, RN);
    tile_slots<LA, NT>(ma, tid, a_off, a_dst);
    tile_slots<LB, NT>(mb, tid, b_off, b_dst);
  }
  for (int i = tid; i < 2 * 3 * (BM + BN) * LDR; i += NT) (&lds[0][0][0][0])[i] = 0.f;
  // k offsets of consecutive pipeline stages, advanced stage by stage with
  // the per-carry deltas of each operand (LDS table: no scalar loads, whose
  // completion wait would also drain the LDS reads in flight, in the loop)
  __shared__ uint64_t kdel[2][kMaxBits];
  for (int t = tid; t < op.n_k - g.tk; t += NT) {
    const uint64_t c = (uint64_t(1) << t) - 1;
    kdel[0][t] = step_delta(c, op.a_k, g.tk);
    kdel[1][t] = step_delta(c, op.b_k, g.tk);
  }
  __syncthreads();

  const uint64_t nsteps = uint64_t(1) << (op.n_k - g.tk);
  const float sa = op.conj_a ? -1.f : 1.f, sb = op.conj_b ? -1.f : 1.f;
  float2 ra[LA], rb[LB];
  uint64_t ka = 0, kb = 0, kstep = 0;
  auto gload = [&]() {
#pragma unroll
    for (int i = 0; i < LA; i++) ra[i] = ld(A + ka + a_off[i]);
#pragma unroll
    for (int i = 0; i < LB; i++) rb[i] = ld(B + kb + b_off[i]);
    if (kstep + 1 < nsteps) {
      const int t = __builtin_ctzll(~kstep);
      ka += kdel[0][t];
      kb += kdel[1][t];
    }
    kstep++;
  };
  auto kpos = [](int k) { return (k & 1) * 4 + (k >> 1); };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < LA; i++)
      if (a_dst[i] >= 0) {
        const int row = a_dst[i] & (BM - 1), k = kpos(a_dst[i] >> RM);
        const float re = ra[i].x, im = sa * ra[i].y;
        lds[buf][0][row][k] = re;
        lds[buf][1][row][k] = im;
        lds[buf][2][row][k] = re + im;
      }
#pragma unroll
    for (int i = 0; i < LB; i++)
      if (b_dst[i] >= 0) {
        const int col = b_dst[i] & (BN - 1), k = kpos(b_dst[i] >> RN);
        const float re = rb[i].x, im = sb * rb[i].y;
        lds[buf][0][BM + col][k] = re;
        lds[buf][1][BM + col][k] = im;
        lds[buf][2][BM + col][k] = re + im;
      }
  };

  const int wave = tid >> 6, lane = tid & 63;
  const int wm = wave / WGN, wn = wave % WGN;
  const int hi = lane >> 5, c32 = lane & 31;
  const int arow = wm * WM + c32, bcol = BM + wn * WN + c32;
  floatx16 acc[3][FM][FN];
#pragma unroll
  for (int t = 0; t < 3; t++)
#pragma unroll
    for (int i = 0; i < FM; i++)
#pragma unroll
      for (int j = 0; j < FN; j++)
#pragma unroll
        for (int r = 0; r < 16; r++) acc[t][i][j][r] = 0.f;

  gload();
  sstore(0);
  __syncthreads();
  for (uint64_t s = 0; s < nsteps; s++) {
    const int buf = s & 1;
    if (s + 1 < nsteps) gload();
    f4 fa[3][FM], fb[3][FN];
#pragma unroll
    for (int t = 0; t < 3; t++) {
#pragma unroll
      for (int i = 0; i < FM; i++) fa[t][i] = *reinterpret_cast<const f4*>(&lds[buf][t][arow + i * 32][4 * hi]);
#pragma unroll
      for (int j = 0; j < FN; j++) fb[t][j] = *reinterpret_cast<const f4*>(&lds[buf][t][bcol + j * 32][4 * hi]);
    }
#pragma unroll
    for (int kk = 0; kk < 4; kk++)
#pragma unroll
      for (int t = 0; t < 3; t++)
#pragma unroll
        for (int i = 0; i < FM; i++)
#pragma unroll
          for (int j = 0; j < FN; j++)
            acc[t][i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa[t][i][kk], fb[t][j][kk], acc[t][i][j], 0, 0, 0);
    if (s + 1 < nsteps) sstore(buf ^ 1);
    __syncthreads();
  }

  gemm_store_3m<BM, BN, FM, FN>(ctx, op, g, reinterpret_cast<uint64_t*>(&lds[0][0][0][0]), acc, wm, wn, tid, NT);
}

// 3M on the direct-to-LDS ring of the 4M kernel: the ring holds the raw
// (re, im) units and each lane forms the re + im plane of its fragments in
// registers.  A lane of half hi reads complex k = 4q + 2hi, 4q + 2hi + 1 of
// its A row and of its B column; matrix-core op e of k group q pairs complex
// k = 4q + e (lower half) with 4q + 2 + e (upper half) in each of the three
// real planes, 12 ops per 32 x 32 complex tile and stage (the 4M kernel
// takes 16).  Each wave holds WM x WN complex outputs.
template <int BM, int BN, int WGM, int WGN, int OCC = 2>
__global__ __launch_bounds__(64 * WGM * WGN) __attribute__((amdgpu_waves_per_eu(OCC))) void gemm_mfma_3m_dl(Ctx ctx, GemmOp op) {
  constexpr int NT = 64 * WGM * WGN, NW = WGM * WGN;
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int FM = WM / 32, FN = WN / 32;
  constexpr int RM = __builtin_ctz(BM), RN = __builtin_ctz(BN), RK = 3;
  static_assert(FM >= 1 && FN >= 1, "tile too small");
  typedef DlRing<BM, BN, NW> Ring;
  __shared__ __attribute__((aligned(16))) f4 lds[Ring::NBUF * Ring::UNITS];
  static_assert(sizeof(lds) >= (BM + BN) * sizeof(uint64_t), "lds too small for epilogue tables");

  GemmSetup g;
  if (!gemm_setup(ctx, op, RM, RN, RK, g)) return;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const Ring ring(ctx, op, g, wave, lane);
  const uint64_t nsteps = uint64_t(1) << (op.n_k - RK);

  const int wm = wave / WGN, wn = wave % WGN;
  const int hi = lane >> 5, c32 = lane & 31;
  const float sa = op.conj_a ? -1.f : 1.f, sb = op.conj_b ? -1.f : 1.f;
  floatx16 acc[3][FM][FN];
#pragma unroll
  for (int t = 0; t < 3; t++)
#pragma unroll
    for (int i = 0; i < FM; i++)
#pragma unroll
      for (int j = 0; j < FN; j++)
#pragma unroll
        for (int r = 0; r < 16; r++) acc[t][i][j][r] = 0.f;

  ring.issue(lds, 0, wave);
  if (nsteps > 1) ring.issue(lds, 1, wave);
  for (uint64_t s = 0; s < nsteps; s++) {
    Ring::wait(s + 1 < nsteps);
    if (s + 2 < nsteps) ring.issue(lds, s + 2, wave);
    const f4* L = &lds[(int)(s % Ring::NBUF) * Ring::UNITS];
#pragma unroll
    for (int q = 0; q < 2; q++) {
      const int kp = 2 * q + hi;
      f4 fa[FM], fb[FN];
#pragma unroll
      for (int i = 0; i < FM; i++) {
        fa[i] = L[dl_unit(wm * WM + i * 32 + c32, kp)];
        fa[i][1] *= sa;
        fa[i][3] *= sa;
      }
#pragma unroll
      for (int j = 0; j < FN; j++) {
        fb[j] = L[BM * 4 + dl_unit(wn * WN + j * 32 + c32, kp)];
        fb[j][1] *= sb;
        fb[j][3] *= sb;
      }
#pragma unroll
      for (int e = 0; e < 2; e++) {
        float pa[FM], pb[FN];
#pragma unroll
        for (int i = 0; i < FM; i++) pa[i] = fa[i][2 * e] + fa[i][2 * e + 1];
#pragma unroll
        for (int j = 0; j < FN; j++) pb[j] = fb[j][2 * e] + fb[j][2 * e + 1];
#pragma unroll
        for (int i = 0; i < FM; i++)
#pragma unroll
          for (int j = 0; j < FN; j++) {
            acc[0][i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa[i][2 * e], fb[j][2 * e], acc[0][i][j], 0, 0, 0);
            acc[1][i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa[i][2 * e + 1], fb[j][2 * e + 1], acc[1][i][j], 0, 0, 0);
            acc[2][i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(pa[i], pb[j], acc[2][i][j], 0, 0, 0);
          }
      }
    }
  }
  __syncthreads();                         // the epilogue reuses the LDS ring for its tables
  gemm_store_3m<BM, BN, FM, FN>(ctx, op, g, reinterpret_cast<uint64_t*>(&lds[0]), acc, wm, wn, tid, NT);
}

// BF16x3 on BF16 matrix cores: every FP32 operand x is split into
// hi = bf16(x) and lo = bf16(x - hi) (x - hi is exact in FP32; both rounded to
// nearest even by the hardware conversion) and each real product is formed as
// hi*hi + hi*lo + lo*hi with FP32 accumulation (the lo*lo term, below 2^-16
// relative, is dropped).  The complex product uses the same real embedding as
// the 4M kernel; one v_mfma_f32_32x32x16_bf16 takes 8 complex k values (16
// real) per lane pair of a 32 x 16 complex tile.  LDS holds hi and lo of A as
// (re, im) bf16 pairs and of B in the two patterns the output column parity
// needs, (Br, -Bi) and (Bi, Br), k fastest: formed once per element when the
// stage is stored (negation and swap commute with the rounding), not at every
// fragment read.  The two patterns of a B column sit in adjacent rows, so the
// 16 lanes of a fragment read (8 columns x 2 parities) hit 16 consecutive
// rows, whose 128-bit pieces fall in disjoint banks.
template <int BM, int BN, int BK, int WGM, int WGN, int OCC = 2>
__global__ __launch_bounds__(64 * WGM * WGN) __attribute__((amdgpu_waves_per_eu(OCC))) void gemm_mfma_bf16x3(Ctx ctx, GemmOp op) {
  static_assert(((BK + 4) * 4) % 16 == 0, "fragment rows must stay 16-byte aligned");
  constexpr int NT = 64 * WGM * WGN;
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int FM = WM / 32, FN = WN / 16;
  constexpr int LA = BM * BK / NT, LB = BN * BK / NT;
  constexpr int RM = __builtin_ctz(BM), RN = __builtin_ctz(BN), RK = __builtin_ctz(BK);
  constexpr int LDK = BK + 4;                      // dwords per row: BK (re, im) pairs + pad (16-byte rows)
  static_assert(BK % 8 == 0, "BK must hold whole MFMA k steps");
  __shared__ uint32_t lds[2][2][BM + 2 * BN][LDK];  // [buffer][hi/lo][A rows | B col 0 even, odd pattern, col 1 ...][k]
  static_assert(sizeof(lds) >= (BM + BN) * sizeof(uint64_t), "lds too small for epilogue tables");

  GemmSetup g;
  if (!gemm_setup(ctx, op, RM, RN, RK, g)) return;
  GMEM const float2* A = reinterpret_cast<GMEM const float2*>(resolve(ctx, op.a, g.z, g.sid, 8)) + g.ka +
                         deposit_runs(g.h, op.run_a_h) + deposit_runs(g.tile_m << g.tm, op.run_a_m);
  GMEM const float2* B = reinterpret_cast<GMEM const float2*>(resolve(ctx, op.b, g.z, g.sid, 8)) + g.kb +
                         deposit_runs(g.h, op.run_b_h) + deposit_runs(g.tile_n << g.tn, op.run_b_n);
  const int tid = threadIdx.x;
  uint32_t a_off[LA], b_off[LB];
  int16_t a_dst[LA], b_dst[LB];
  {
    TileMap ma, mb;
    make_tilemap(ma, op.a_m, g.tm, op.a_k, g.tk, RM);
    make_tilemap(mb, op.b_n, g.tn, op.b_k, g.tk, RN);
    tile_slots<LA, NT>(ma, tid, a_off, a_dst);
    tile_slots<LB, NT>(mb, tid, b_off, b_dst);
  }
  for (int i = tid; i < 2 * 2 * (BM + 2 * BN) * LDK; i += NT) (&lds[0][0][0][0])[i] = 0u;
  // k offsets of consecutive pipeline stages, advanced stage by stage with
  // the per-carry deltas of each operand (LDS table: no scalar loads, whose
  // completion wait would also drain the LDS reads in flight, in the loop)
  __shared__ uint64_t kdel[2][kMaxBits];
  for (int t = tid; t < op.n_k - g.tk; t += NT) {
    const uint64_t c = (uint64_t(1) << t) - 1;
    kdel[0][t] = step_delta(c, op.a_k, g.tk);
    kdel[1][t] = step_delta(c, op.b_k, g.tk);
  }
  __syncthreads();

  const uint64_t nsteps = uint64_t(1) << (op.n_k - g.tk);
  const float sa = op.conj_a ? -1.f : 1.f, sb = op.conj_b ? -1.f : 1.f;
  float2 ra[LA], rb[LB];
  uint64_t ka = 0, kb = 0, kstep = 0;
  auto gload = [&]() {
#pragma unroll
    for (int i = 0; i < LA; i++) ra[i] = ld(A + ka + a_off[i]);
#pragma unroll
    for (int i = 0; i < LB; i++) rb[i] = ld(B + kb + b_off[i]);
    if (kstep + 1 < nsteps) {
      const int t = __builtin_ctzll(~kstep);
      ka += kdel[0][t];
      kb += kdel[1][t];
    }
    kstep++;
  };
  typedef float f2v __attribute__((ext_vector_type(2)));
  typedef __bf16 bf2v __attribute__((ext_vector_type(2)));
  auto split = [](float re, float im, uint32_t& h, uint32_t& l) {
    const bf2v hb = __builtin_convertvector(f2v{re, im}, bf2v);
    const f2v back = __builtin_convertvector(hb, f2v);
    const bf2v lb = __builtin_convertvector(f2v{re - back.x, im - back.y}, bf2v);
    h = __builtin_bit_cast(uint32_t, hb);     // re in the low half
    l = __builtin_bit_cast(uint32_t, lb);
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < LA; i++)
      if (a_dst[i] >= 0) {
        const int row = a_dst[i] & (BM - 1), k = a_dst[i] >> RM;
        uint32_t h, l;
        split(ra[i].x, sa * ra[i].y, h, l);
        lds[buf][0][row][k] = h;
        lds[buf][1][row][k] = l;
      }
#pragma unroll
    for (int i = 0; i < LB; i++)
      if (b_dst[i] >= 0) {
        const int col = b_dst[i] & (BN - 1), k = b_dst[i] >> RN;
        uint32_t h, l;
        split(rb[i].x, sb * rb[i].y, h, l);
        // even output columns take (Br, -Bi): the sign of the high half
        // flips; odd ones (Bi, Br): the halves swap
        lds[buf][0][BM + 2 * col][k] = h ^ 0x80000000u;
        lds[buf][1][BM + 2 * col][k] = l ^ 0x80000000u;
        lds[buf][0][BM + 2 * col + 1][k] = (h >> 16) | (h << 16);
        lds[buf][1][BM + 2 * col + 1][k] = (l >> 16) | (l << 16);
      }
  };

  const int wave = tid >> 6, lane = tid & 63;
  const int wm = wave / WGN, wn = wave % WGN;
  const int kg = lane >> 5;                 // which 4 complex k of the 8
  const int c32 = lane & 31;
  const int bpar = c32 & 1;
  floatx16 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; i++)
#pragma unroll
    for (int j = 0; j < FN; j++)
#pragma unroll
      for (int r = 0; r < 16; r++) acc[i][j][r] = 0.f;
  gload();
  sstore(0);
  __syncthreads();
  for (uint64_t s = 0; s < nsteps; s++) {
    const int buf = s & 1;
    if (s + 1 < nsteps) gload();
#pragma unroll
    for (int kt = 0; kt < BK / 8; kt++) {
      const int k0 = kt * 8 + kg * 4;
      u32x4 ah[FM], al[FM];
#pragma unroll
      for (int i = 0; i < FM; i++) {
        const int row = wm * WM + i * 32 + c32;
        ah[i] = *reinterpret_cast<const u32x4*>(&lds[buf][0][row][k0]);
        al[i] = *reinterpret_cast<const u32x4*>(&lds[buf][1][row][k0]);
      }
#pragma unroll
      for (int j = 0; j < FN; j++) {
        // the pattern of this lane's output column parity
        const int col = BM + 2 * (wn * WN + j * 16 + (c32 >> 1)) + bpar;
        const u32x4 bh = *reinterpret_cast<const u32x4*>(&lds[buf][0][col][k0]);
        const u32x4 bl = *reinterpret_cast<const u32x4*>(&lds[buf][1][col][k0]);
        // hi*hi, hi*lo, lo*hi, interleaved over the row fragments so that no
        // two consecutive matrix-core ops write the same accumulator
#pragma unroll
        for (int i = 0; i < FM; i++)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, ah[i]),
                                                              __builtin_bit_cast(bf16x8, bh), acc[i][j], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < FM; i++)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, ah[i]),
                                                              __builtin_bit_cast(bf16x8, bl), acc[i][j], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < FM; i++)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, al[i]),
                                                              __builtin_bit_cast(bf16x8, bh), acc[i][j], 0, 0, 0);
      }
    }
    if (s + 1 < nsteps) sstore(buf ^ 1);
    __syncthreads();
  }
  gemm_store<BM, BN, FM, FN>(ctx, op, g, reinterpret_cast<uint64_t*>(&lds[0][0][0][0]), acc, wm, wn, tid, NT);
}

// ------------------------------------------------------------------ BF16x3 on pre-split operands

// Splits a complex64 GEMM operand into the bf16 hi / lo units of SplitOp
// (tn_internal.h): one thread per row and group of four summed values.
__global__ __launch_bounds__(256) void split_kernel(Ctx ctx, SplitOp op) {
  const uint64_t q = uint64_t(blockIdx.x) * 256 + threadIdx.x;
  const int gbits = op.n_k - 2;                    // groups of four summed values per row
  if (q >> (op.n_rows + gbits)) return;
  const int z = blockIdx.y;
  const int64_t sid = slice_id(ctx, z);
  if (sid < 0) return;
  const uint64_t r = q >> gbits, kg = q & ((uint64_t(1) << gbits) - 1);
  GMEM const float2* S = reinterpret_cast<GMEM const float2*>(resolve(ctx, op.src, z, sid, 8));
  GMEM u32x4* D = reinterpret_cast<GMEM u32x4*>(resolve(ctx, op.dst, z, sid, 8));
  const uint64_t base = deposit_runs(r, op.run_row) + deposit_runs(kg, op.run_khi);
  typedef float f2v __attribute__((ext_vector_type(2)));
  typedef __bf16 bf2v __attribute__((ext_vector_type(2)));
  u32x4 hi, lo;
#pragma unroll
  for (int j = 0; j < 4; j++) {
    const float2 v = ld(S + base + op.j_off[j]);
    const float re = v.x, im = op.conj ? -v.y : v.y;
    const bf2v hb = __builtin_convertvector(f2v{re, im}, bf2v);      // round to nearest even
    const f2v back = __builtin_convertvector(hb, f2v);
    const bf2v lb = __builtin_convertvector(f2v{re - back.x, im - back.y}, bf2v);
    hi[j] = __builtin_bit_cast(uint32_t, hb);                           // re in the low half
    lo[j] = __builtin_bit_cast(uint32_t, lb);
  }
  const uint64_t kb = kg >> 1, g = kg & 1;
  const uint64_t blk = (r << (op.n_k - 3)) + kb;
  if (op.patterns == 1) {
    GMEM u32x4* d = D + blk * 4 + 2 * g;
    d[0] = hi;
    d[1] = lo;
  } else {
    // (re, -im): flip the sign of the high half; (im, re): swap the halves
    u32x4 h0, l0, h1, l1;
#pragma unroll
    for (int j = 0; j < 4; j++) {
      h0[j] = hi[j] ^ 0x80000000u;
      l0[j] = lo[j] ^ 0x80000000u;
      h1[j] = (hi[j] >> 16) | (hi[j] << 16);
      l1[j] = (lo[j] >> 16) | (lo[j] << 16);
    }
    GMEM u32x4* d = D + blk * 8 + 2 * g;
    d[0] = h0;
    d[1] = l0;
    d[4] = h1;
    d[5] = l1;
  }
}

// Direct-to-LDS ring for the pre-split BF16x3 operands: per stage (8 summed
// values) a tile row of A is 4 units (64 contiguous bytes), a tile column of
// B 8 units (128 contiguous bytes).  LDS slot swizzles (each group of 16
// lanes of a fragment read hits 16 different 16-byte bank groups): A unit u
// of row r at r * 4 + (u ^ ((r >> 2) & 3)); B unit u = 4 p + v of column c
// at c * 8 + 4 p + (v ^ ((c >> 1) & 3)).
__device__ __forceinline__ int sa_unit(int r, int u) { return r * 4 + (u ^ ((r >> 2) & 3)); }
__device__ __forceinline__ int sb_unit(int c, int p, int v) { return c * 8 + 4 * p + (v ^ ((c >> 1) & 3)); }

template <int BM, int BN, int NW, int NB>
struct SplitRing {
  static constexpr int UA = BM * 4, UB = BN * 8;          // 16-byte units per stage
  static constexpr int IA = UA / 64 / NW, IB = UB / 64 / NW;
  static constexpr int NBUF = NB;                          // NB - 1 stages in flight
  static constexpr int UNITS = UA + UB;
  static_assert(IA >= 1 && IB >= 1 && IA * NW * 64 == UA && IB * NW * 64 == UB, "tile / wave mismatch");
  static_assert(IA + IB < 16, "loads in flight per stage must fit the wait counter field");
  GMEM const u32x4* A;
  GMEM const u32x4* B;
  uint32_t a_off[IA], b_off[IB];   // unit offset of every unit this lane loads, at the first stage

  __device__ __forceinline__ SplitRing(const Ctx& ctx, const GemmOp& op, const GemmSetup& g, int wave, int lane) {
    A = reinterpret_cast<GMEM const u32x4*>(resolve(ctx, op.a, g.z, g.sid, 8));
    B = reinterpret_cast<GMEM const u32x4*>(resolve(ctx, op.b, g.z, g.sid, 8));
    const uint64_t mrows = uint64_t(1) << g.tm, nrows = uint64_t(1) << g.tn;
    const uint64_t kb0 = uint64_t(blockIdx.z) << (op.n_k - 3);    // this split's first block of 8
    const int kbt = op.ab_k_bits - 3;                                // blocks of 8 per row
#pragma unroll
    for (int i = 0; i < IA; i++) {
      const int slot = (wave * IA + i) * 64 + lane;
      const int r = slot >> 2, u = (slot & 3) ^ ((r >> 2) & 3);
      const uint64_t rr = uint64_t(r) < mrows ? uint64_t(r) : 0;      // rows past a partial tile repeat row 0
      const uint64_t row = (g.h << op.n_m) | (g.tile_m << g.tm) | rr;
      a_off[i] = (uint32_t)((((row << kbt) + kb0) << 2) + u);
    }
#pragma unroll
    for (int i = 0; i < IB; i++) {
      const int slot = (wave * IB + i) * 64 + lane;
      const int c = slot >> 3, pv = slot & 7;
      const int u = (pv & 4) | ((pv & 3) ^ ((c >> 1) & 3));
      const uint64_t cc = uint64_t(c) < nrows ? uint64_t(c) : 0;
      const uint64_t col = (g.h << op.n_n) | (g.tile_n << g.tn) | cc;
      b_off[i] = (uint32_t)((((col << kbt) + kb0) << 3) + u);
    }
  }

  // start the loads of stage `step` into ring buffer `buf`
  __device__ __forceinline__ void issue(u32x4* lds, uint32_t step, int buf, int wave) const {
    const uint32_t sa = step << 2, sb = step << 3;
#pragma unroll
    for (int i = 0; i < IA; i++)
      __builtin_amdgcn_global_load_lds((GMEM const void*)(A + a_off[i] + sa),
                                       (__attribute__((address_space(3))) void*)(&lds[buf * UNITS + (wave * IA + i) * 64]),
                                       16, 0, 0);
#pragma unroll
    for (int i = 0; i < IB; i++)
      __builtin_amdgcn_global_load_lds((GMEM const void*)(B + b_off[i] + sb),
                                       (__attribute__((address_space(3))) void*)(&lds[buf * UNITS + UA + (wave * IB + i) * 64]),
                                       16, 0, 0);
  }

  // as DlRing::wait: this wave's loads of stage s are done once at most those
  // of the `ahead` later stages in flight remain; then a plain barrier
  __device__ __forceinline__ static void wait(int ahead) {
    if (ahead >= 2 && NB >= 4) __builtin_amdgcn_s_waitcnt((2 * (IA + IB)) | (0x7 << 4) | (0xF << 8));
    else if (ahead >= 1) __builtin_amdgcn_s_waitcnt((IA + IB) | (0x7 << 4) | (0xF << 8));
    else __builtin_amdgcn_s_waitcnt(0 | (0x7 << 4) | (0xF << 8));
    __builtin_amdgcn_s_barrier();
  }
};

// BF16x3 on pre-split operands: the 4M embedding on v_mfma_f32_32x32x16_bf16
// (one op covers 8 complex summed values: lanes of half kg supply complex k
// 4 kg .. 4 kg + 3 as (re, im) pairs), products hi*hi + hi*lo + lo*hi with
// FP32 accumulation.  The operands arrive split (split_kernel) and stream
// global -> LDS through the ring with no staging registers and no vector-ALU
// work in the loop; lane c32 of a B read takes its column's pattern c32 & 1
// (even real column: (re, -im) -> real part, odd: (im, re) -> imaginary).
template <int BM, int BN, int WGM, int WGN, int OCC, int NB>
__global__ __launch_bounds__(64 * WGM * WGN) __attribute__((amdgpu_waves_per_eu(OCC))) void gemm_mfma_bf16x3_dl(Ctx ctx, GemmOp op) {
  constexpr int NT = 64 * WGM * WGN, NW = WGM * WGN;
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int FM = WM / 32, FN = WN / 16;
  constexpr int RM = __builtin_ctz(BM), RN = __builtin_ctz(BN), RK = 3;
  static_assert(FM >= 1 && FN >= 1, "tile too small");
  typedef SplitRing<BM, BN, NW, NB> Ring;
  static_assert(NB == 3 || (NB == 4 && 2 * (Ring::IA + Ring::IB) < 16), "ring depth");
  __shared__ __attribute__((aligned(16))) u32x4 lds[Ring::NBUF * Ring::UNITS];
  static_assert(sizeof(lds) >= (BM + BN) * sizeof(uint64_t), "lds too small for epilogue tables");

  GemmSetup g;
  if (!gemm_setup(ctx, op, RM, RN, RK, g)) return;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const Ring ring(ctx, op, g, wave, lane);
  const uint32_t nsteps = 1u << (op.n_k - RK);                 // per split: at most 2^28
  const int wm = wave / WGN, wn = wave % WGN;
  const int kg = lane >> 5, c32 = lane & 31, p = c32 & 1;
  floatx16 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; i++)
#pragma unroll
    for (int j = 0; j < FN; j++)
#pragma unroll
      for (int r = 0; r < 16; r++) acc[i][j][r] = 0.f;

  // NB - 1 stages in flight; buffer indices rotate (no division in the loop)
  for (int q = 0; q < NB - 1; q++)
    if ((uint32_t)q < nsteps) ring.issue(lds, (uint32_t)q, q, wave);
  int cur = 0, nxt = NB - 1;
  for (uint32_t s = 0; s < nsteps; s++) {
    const uint32_t left = nsteps - 1 - s;                      // stages after this one
    Ring::wait(left >= (uint32_t)(NB - 2) ? NB - 2 : (int)left);
    if (s + NB - 1 < nsteps) ring.issue(lds, s + NB - 1, nxt, wave);
    nxt = nxt + 1 == NB ? 0 : nxt + 1;
    const u32x4* L = &lds[cur * Ring::UNITS];
    cur = cur + 1 == NB ? 0 : cur + 1;
    u32x4 ah[FM], al[FM];
#pragma unroll
    for (int i = 0; i < FM; i++) {
      const int row = wm * WM + i * 32 + c32;
      ah[i] = L[sa_unit(row, 2 * kg)];
      al[i] = L[sa_unit(row, 2 * kg + 1)];
    }
#pragma unroll
    for (int j = 0; j < FN; j++) {
      const int col = wn * WN + j * 16 + (c32 >> 1);
      const u32x4 bh = L[Ring::UA + sb_unit(col, p, 2 * kg)];
      const u32x4 bl = L[Ring::UA + sb_unit(col, p, 2 * kg + 1)];
#pragma unroll
      for (int i = 0; i < FM; i++)
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, ah[i]),
                                                            __builtin_bit_cast(bf16x8, bh), acc[i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < FM; i++)
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, ah[i]),
                                                            __builtin_bit_cast(bf16x8, bl), acc[i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < FM; i++)
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, al[i]),
                                                            __builtin_bit_cast(bf16x8, bh), acc[i][j], 0, 0, 0);
    }
  }
  __syncthreads();                         // the epilogue reuses the LDS ring for its tables
  gemm_store<BM, BN, FM, FN>(ctx, op, g, reinterpret_cast<uint64_t*>(&lds[0]), acc, wm, wn, tid, NT);
}

// The same products with the fragments of the next stage read from LDS while
// the matrix cores work on the current one.  A ring of four stages: at stage
// s the wave waits for stage s + 1's loads (s + 2 stays in flight), passes the
// barrier (after which the buffer of stage s - 1, whose fragments every wave
// read one stage earlier, is free) and starts the loads of stage s + 3 into
// it; it then issues stage s's matrix-core ops column block by column block,
// reading stage s + 1's B fragments of a block into the block's registers
// right after the block's last op has used them, and stage s + 1's A
// fragments after the last block.  The LDS read latency overlaps the matrix
// cores' work and the next stage's barrier, and one register set holds the
// fragments.
template <int BM, int BN, int WGM, int WGN, int OCC>
__global__ __launch_bounds__(64 * WGM * WGN) __attribute__((amdgpu_waves_per_eu(OCC))) void gemm_mfma_bf16x3_dlp(Ctx ctx, GemmOp op) {
  constexpr int NT = 64 * WGM * WGN, NW = WGM * WGN, NB = 4;
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int FM = WM / 32, FN = WN / 16;
  constexpr int RM = __builtin_ctz(BM), RN = __builtin_ctz(BN), RK = 3;
  static_assert(FM >= 1 && FN >= 1, "tile too small");
  typedef SplitRing<BM, BN, NW, NB> Ring;
  static_assert(Ring::IA + Ring::IB < 16, "loads in flight per stage must fit the wait counter field");
  __shared__ __attribute__((aligned(16))) u32x4 lds[NB * Ring::UNITS];
  static_assert(sizeof(lds) >= (BM + BN) * sizeof(uint64_t), "lds too small for epilogue tables");

  GemmSetup g;
  if (!gemm_setup(ctx, op, RM, RN, RK, g)) return;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const Ring ring(ctx, op, g, wave, lane);
  const uint32_t nsteps = 1u << (op.n_k - RK);                 // per split: a power of two
  const int wm = wave / WGN, wn = wave % WGN;
  const int kg = lane >> 5, c32 = lane & 31, p = c32 & 1;
  floatx16 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; i++)
#pragma unroll
    for (int j = 0; j < FN; j++)
#pragma unroll
      for (int r = 0; r < 16; r++) acc[i][j][r] = 0.f;

  auto buf = [&](uint32_t s) { return &lds[(s & (NB - 1)) * Ring::UNITS]; };   // stage s's buffer
  u32x4 ah[FM], al[FM], bh[FN], bl[FN];                        // fragments, refilled as they die
  auto read_a = [&](uint32_t s) {
    const u32x4* L = buf(s);
#pragma unroll
    for (int i = 0; i < FM; i++) {
      const int row = wm * WM + i * 32 + c32;
      ah[i] = L[sa_unit(row, 2 * kg)];
      al[i] = L[sa_unit(row, 2 * kg + 1)];
    }
  };
  auto read_b = [&](int j, uint32_t s) {
    const u32x4* L = buf(s);
    const int col = wn * WN + j * 16 + (c32 >> 1);
    bh[j] = L[Ring::UA + sb_unit(col, p, 2 * kg)];
    bl[j] = L[Ring::UA + sb_unit(col, p, 2 * kg + 1)];
  };
  auto mma = [&](int j) {
#pragma unroll
    for (int i = 0; i < FM; i++)
      acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, ah[i]),
                                                          __builtin_bit_cast(bf16x8, bh[j]), acc[i][j], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < FM; i++)
      acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, ah[i]),
                                                          __builtin_bit_cast(bf16x8, bl[j]), acc[i][j], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < FM; i++)
      acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, al[i]),
                                                          __builtin_bit_cast(bf16x8, bh[j]), acc[i][j], 0, 0, 0);
  };
  // Every stage runs the same operations, so that the compiler's wait counts
  // hold on every pass: past the last stage the loads fetch the last stage
  // again (into a buffer no later read uses) and the reads re-read it.
  const uint32_t last = nsteps - 1;
  auto clamp = [&](uint32_t t) { return t < last ? t : last; };
  for (int q = 0; q < NB - 1; q++) ring.issue(lds, clamp((uint32_t)q), q, wave);
  Ring::wait(2);                                               // stage 0 loaded
  read_a(0);
#pragma unroll
  for (int j = 0; j < FN; j++) read_b(j, 0);
  for (uint32_t s = 0; s < nsteps; s++) {
    Ring::wait(1);                                             // stage s + 1 loaded, s + 2 in flight
    ring.issue(lds, clamp(s + 3), (s + 3) & (NB - 1), wave);
    const uint32_t nx = clamp(s + 1);
    // (scheduling barriers keep the compiler from reordering the blocks)
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < FN; j++) {
      mma(j);
      read_b(j, nx);
      if (j == FN - 1) read_a(nx);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  Ring::wait(0);                           // no load into the ring still in flight
  __syncthreads();                         // the epilogue reuses the LDS ring for its tables
  gemm_store<BM, BN, FM, FN>(ctx, op, g, reinterpret_cast<uint64_t*>(&lds[0]), acc, wm, wn, tid, NT);
}

// ------------------------------------------------------------------ split-K sum

// Fixed-order sum of the split-K partial products of a GEMM (splits in
// increasing order, so the result does not depend on scheduling): element e
// = (h, m, n) of every split, n fastest, goes to C at the positions of its h,
// m and n bits.
struct SplitReduceOp {
  Ref part, c;
  BitRuns run_c;       // C positions of the bits of e
  int32_t n_e;         // log2 elements per split
  int32_t n_split;     // log2 splits
  int32_t accumulate;  // add into C instead of overwriting
};

template <typename T>
__global__ __launch_bounds__(256) void split_reduce_kernel(Ctx ctx, SplitReduceOp op) {
  using V = typename C2<T>::t;
  const int z = blockIdx.y;
  const int64_t sid = slice_id(ctx, z);
  if (sid < 0) return;
  const uint64_t e = uint64_t(blockIdx.x) * 256 + threadIdx.x;
  if (e >> op.n_e) return;
  GMEM const V* P = reinterpret_cast<GMEM const V*>(resolve(ctx, op.part, z, sid, sizeof(V))) + e;
  V acc = ld(P);
  const uint64_t ns = uint64_t(1) << op.n_split;
#pragma unroll 8
  for (uint64_t sp = 1; sp < ns; sp++) {
    const V v = ld(P + (sp << op.n_e));
    acc.x += v.x;
    acc.y += v.y;
  }
  GMEM V* C = reinterpret_cast<GMEM V*>(resolve(ctx, op.c, z, sid, sizeof(V))) + deposit_runs(e, op.run_c);
  if (op.accumulate) {
    const V o = ld(C);
    acc.x += o.x;
    acc.y += o.y;
  }
  st(C, acc);
}

// ------------------------------------------------------------------ VALU tiled GEMM

// 64 x 64 complex tile, 256 threads, each thread 4 x 4 outputs; used for
// complex128 and as the FP32 reference variant of the tile autotuner.
template <typename T>
__global__ __launch_bounds__(256) void gemm_valu(Ctx ctx, GemmOp op) {
  using V = typename C2<T>::t;
  constexpr int BM = 64, BN = 64, BK = 8, RM = 6, RN = 6, RK = 3;
  constexpr int LA = BM * BK / 256, LB = BN * BK / 256;
  __shared__ V As[BK][BM];
  __shared__ V Bs[BK][BN];
  const int nzh = ctx.n_batch;
  const int z = blockIdx.y % nzh;
  const uint64_t h = blockIdx.y / nzh;
  const int64_t sid = slice_id(ctx, z);
  if (sid < 0) return;
  const int tm = op.n_m < RM ? op.n_m : RM;
  const int tn = op.n_n < RN ? op.n_n : RN;
  const int tk = op.n_k < RK ? op.n_k : RK;
  const uint64_t ntiles_n = uint64_t(1) << (op.n_n - tn);
  const uint64_t tile_m = blockIdx.x / ntiles_n, tile_n = blockIdx.x % ntiles_n;
  const int eb = sizeof(V);
  GMEM const V* A = reinterpret_cast<GMEM const V*>(resolve(ctx, op.a, z, sid, eb)) + deposit_runs(h, op.run_a_h) +
               deposit_runs(tile_m << tm, op.run_a_m) + deposit_runs(blockIdx.z, op.run_a_s);
  GMEM const V* B = reinterpret_cast<GMEM const V*>(resolve(ctx, op.b, z, sid, eb)) + deposit_runs(h, op.run_b_h) +
               deposit_runs(tile_n << tn, op.run_b_n) + deposit_runs(blockIdx.z, op.run_b_s);
  GMEM V* C = reinterpret_cast<GMEM V*>(resolve(ctx, op.c, z, sid, eb)) + deposit_runs(h, op.run_c_h) +
         deposit_runs(tile_m << tm, op.run_c_m) + deposit_runs(tile_n << tn, op.run_c_n) +
         (uint64_t(blockIdx.z) << op.c_split_shift);
  TileMap ma, mb;
  make_tilemap(ma, op.a_m, tm, op.a_k, tk, RM);
  make_tilemap(mb, op.b_n, tn, op.b_k, tk, RN);
  const int tid = threadIdx.x;
  uint64_t a_off[LA], b_off[LB];
  int a_dst[LA], b_dst[LB];
  for (int i = 0; i < LA; i++) {
    const int e = tid + 256 * i;
    uint64_t off;
    int d;
    tile_elem(ma, e, off, d);
    a_off[i] = off;
    a_dst[i] = (e >> ma.nbits) == 0 ? d : -1;
  }
  for (int i = 0; i < LB; i++) {
    const int e = tid + 256 * i;
    uint64_t off;
    int d;
    tile_elem(mb, e, off, d);
    b_off[i] = off;
    b_dst[i] = (e >> mb.nbits) == 0 ? d : -1;
  }
  for (int i = tid; i < BK * BM; i += 256) { (&As[0][0])[i].x = 0; (&As[0][0])[i].y = 0; }
  for (int i = tid; i < BK * BN; i += 256) { (&Bs[0][0])[i].x = 0; (&Bs[0][0])[i].y = 0; }
  const int ty = tid >> 4, tx = tid & 15;
  V acc[4][4];
  for (int i = 0; i < 4; i++)
    for (int j = 0; j < 4; j++) { acc[i][j].x = 0; acc[i][j].y = 0; }
  const uint64_t nsteps = uint64_t(1) << (op.n_k - tk);
  for (uint64_t s = 0; s < nsteps; s++) {
    const uint64_t ka = deposit(s, op.a_k, tk, op.n_k - tk);
    const uint64_t kb = deposit(s, op.b_k, tk, op.n_k - tk);
    __syncthreads();
    for (int i = 0; i < LA; i++)
      if (a_dst[i] >= 0) (&As[0][0])[(a_dst[i] >> RM) * BM + (a_dst[i] & (BM - 1))] = conjv(ld(A + ka + a_off[i]), op.conj_a);
    for (int i = 0; i < LB; i++)
      if (b_dst[i] >= 0) (&Bs[0][0])[(b_dst[i] >> RN) * BN + (b_dst[i] & (BN - 1))] = conjv(ld(B + kb + b_off[i]), op.conj_b);
    __syncthreads();
    for (int k = 0; k < BK; k++) {
      V a[4], b[4];
      for (int i = 0; i < 4; i++) a[i] = As[k][ty + 16 * i];
      for (int j = 0; j < 4; j++) b[j] = Bs[k][tx + 16 * j];
      for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) acc[i][j] = cfma(acc[i][j], a[i], b[j]);
    }
  }
  const int mvalid = 1 << tm, nvalid = 1 << tn;
  for (int i = 0; i < 4; i++) {
    const int row = ty + 16 * i;
    if (row >= mvalid) continue;
    const uint64_t ro = deposit_runs(uint64_t(row), op.run_c_m);
    for (int j = 0; j < 4; j++) {
      const int col = tx + 16 * j;
      if (col >= nvalid) continue;
      GMEM V* d = C + ro + deposit_runs(uint64_t(col), op.run_c_n);
      if (op.accumulate) { V o = ld(d); o.x += acc[i][j].x; o.y += acc[i][j].y; st(d, o); }
      else st(d, acc[i][j]);
    }
  }
}

// ------------------------------------------------------------------ launchers

static inline unsigned blocks_for(uint64_t n, unsigned per) { return (unsigned)((n + per - 1) / per); }

unsigned stream_grid_x(uint64_t waves, unsigned gy, const void* kernel) {
  static std::atomic<int> cus[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  int n = cus[dev].load(std::memory_order_relaxed);
  if (n <= 0) {
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    cus[dev].store(n, std::memory_order_relaxed);
  }
  // workgroups of this kernel one compute unit holds at once (its register
  // count decides): a persistent workgroup that has to wait for another to
  // finish would walk all its units only afterwards
  static std::mutex mu;
  static std::unordered_map<const void*, int> resident;
  int per_cu = kStreamWavesPerCU / 4;                               // 4 wavefronts per workgroup
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = resident.find(kernel);
    if (it == resident.end()) {
      int nb = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, 256, 0) != hipSuccess || nb <= 0) nb = per_cu;
      it = resident.emplace(kernel, nb).first;
    }
    per_cu = std::min(per_cu, it->second);
  }
  const uint64_t want = uint64_t(n) * per_cu;
  const uint64_t per_y = want / gy > 0 ? want / gy : 1;
  const uint64_t need = (waves + 3) / 4;
  return (unsigned)(need < per_y ? need : per_y);
}

// Summed-range steps per batch of loads: row_ku(NIN), or the whole range when
// it is shorter (log2 given in ubits).
template <typename T, int NIN>
static void launch_row_u(bool splitk, dim3 grid, const Ctx& ctx, const RowOp& op, int ubits, hipStream_t s) {
  constexpr int KB = row_ku(NIN) == 8 ? 3 : (row_ku(NIN) == 4 ? 2 : 1);
  const int ub = ubits < KB ? ubits : KB;
  const bool stage = !splitk && op.stage_c && sizeof(T) == 4;
#define TN_ROW_LAUNCH(U)                                                                            \
  do {                                                                                              \
    if (splitk) hipLaunchKernelGGL((splitk_kernel<T, NIN, U>), grid, dim3(kRowThreads), 0, s, ctx, op); \
    else if (stage) hipLaunchKernelGGL((row_kernel<T, NIN, U, true>), grid, dim3(kRowThreads), 0, s, ctx, op); \
    else hipLaunchKernelGGL((row_kernel<T, NIN, U>), grid, dim3(kRowThreads), 0, s, ctx, op);          \
  } while (0)
  switch (ub) {
    case 0: TN_ROW_LAUNCH(1); break;
    case 1: TN_ROW_LAUNCH(2); break;
    case 2: if constexpr (KB >= 2) TN_ROW_LAUNCH(4); break;
    default: if constexpr (KB >= 3) TN_ROW_LAUNCH(8); break;
  }
#undef TN_ROW_LAUNCH
}

template <typename T, int NIN>
static void launch_row_stream_n(const Ctx& ctx, const RowOp& op, hipStream_t s) {
  const RowKOffsets ko = row_k_offsets(op);
  const bool contiguous = op.stage_c && sizeof(T) == 4 && NIN >= 2;
  const int rb = op.n_rows >= 7 ? kRowStreamBlocks : 1;
  const uint64_t waves = (uint64_t(1) << (op.n_rows - 6)) / rb;
  auto grid = [&](const void* k) { return dim3(stream_grid_x(waves, (unsigned)ctx.n_batch, k), ctx.n_batch); };
  auto go = [&](auto kn) {
    constexpr int KN = decltype(kn)::value;
    auto with_rb = [&](auto mode) {
      constexpr int M = decltype(mode)::value;
      if (rb == 2) {
        auto k = row_stream_kernel<T, NIN, KN, M, 2>;
        hipLaunchKernelGGL(k, grid((const void*)k), dim3(kRowThreads), 0, s, ctx, op, ko);
      } else {
        auto k = row_stream_kernel<T, NIN, KN, M, 1>;
        hipLaunchKernelGGL(k, grid((const void*)k), dim3(kRowThreads), 0, s, ctx, op, ko);
      }
    };
    if constexpr (sizeof(T) == 4 && NIN >= 2)
      if (contiguous) {
        if (kRowStreamMode(NIN) == 1) with_rb(std::integral_constant<int, 1>());
        else with_rb(std::integral_constant<int, 2>());
        return;
      }
    with_rb(std::integral_constant<int, 0>());
  };
  if (op.n_k == 0) go(std::integral_constant<int, 1>());
  else if constexpr (NIN <= 8) {
    if (op.n_k == 1) go(std::integral_constant<int, 2>());
    else if constexpr (NIN <= 4) go(std::integral_constant<int, 4>());
  }
}

template <typename T>
static hipError_t launch_row_stream(const Ctx& ctx, const RowOp& op, hipStream_t s) {
  switch (op.n_in) {
    case 0: launch_row_stream_n<T, 1>(ctx, op, s); break;
    case 1: launch_row_stream_n<T, 2>(ctx, op, s); break;
    case 2: launch_row_stream_n<T, 4>(ctx, op, s); break;
    case 3: launch_row_stream_n<T, 8>(ctx, op, s); break;
    case 4: launch_row_stream_n<T, 16>(ctx, op, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_row_t(const Ctx& ctx, const RowOp& op, hipStream_t s) {
  const bool splitk = op.k_split_bits >= 0;
  if (row_stream_ok(op)) return launch_row_stream<T>(ctx, op, s);
  uint64_t units;
  int ubits;
  if (splitk) {
    const int ks = op.k_split_bits > 0 ? op.k_split_bits : 0;
    units = uint64_t(1) << (op.n_rows + ks);                 // wavefronts
    ubits = op.n_k - ks - 6;                                 // steps of 64 k per lane
  } else {
    units = uint64_t(1) << op.n_rows;                        // threads
    ubits = op.pair_a ? op.n_k - 1 : op.n_k;                 // (paired) k steps per thread
  }
  if (ubits < 0) return hipErrorInvalidValue;
  dim3 grid(blocks_for(units, splitk ? kRowThreads / 64 : kRowThreads), ctx.n_batch);
  switch (op.n_in) {
    case 0: launch_row_u<T, 1>(splitk, grid, ctx, op, ubits, s); break;
    case 1: launch_row_u<T, 2>(splitk, grid, ctx, op, ubits, s); break;
    case 2: launch_row_u<T, 4>(splitk, grid, ctx, op, ubits, s); break;
    case 3: launch_row_u<T, 8>(splitk, grid, ctx, op, ubits, s); break;
    case 4: launch_row_u<T, 16>(splitk, grid, ctx, op, ubits, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

static RowOp with_runs(const RowOp& in) {
  RowOp op = in;
  prepare_row(op);
  return op;
}

hipError_t launch_row(const Ctx& ctx, const RowOp& in, bool f64, hipStream_t s) {
  const RowOp op = with_runs(in);
  return f64 ? launch_row_t<double>(ctx, op, s) : launch_row_t<float>(ctx, op, s);
}

hipError_t launch_reduce(const Ctx& ctx, const RowOp& in, bool f64, hipStream_t s) {
  const RowOp op = with_runs(in);
  const uint64_t n = uint64_t(1) << (op.n_rows + op.n_in);   // outputs, one wavefront each
  dim3 grid(blocks_for(n, kRowThreads / 64), ctx.n_batch);
  if (f64) hipLaunchKernelGGL(reduce_kernel<double>, grid, dim3(kRowThreads), 0, s, ctx, op);
  else hipLaunchKernelGGL(reduce_kernel<float>, grid, dim3(kRowThreads), 0, s, ctx, op);
  return hipGetLastError();
}

int gemm_tile_bits(int tile, int* bm, int* bn) {
  switch (tile) {
    case 0: *bm = 7; *bn = 7; return 0;     // 128 x 128, 4 waves of 64 x 64
    case 1: *bm = 6; *bn = 7; return 0;     // 64 x 128, 2 waves
    case 2: *bm = 7; *bn = 6; return 0;     // 128 x 64, 2 waves
    case 3: *bm = 6; *bn = 6; return 0;     // 64 x 64, 1 wave
    case 4: *bm = 6; *bn = 6; return 0;     // vector-ALU 64 x 64
    case 5: *bm = 8; *bn = 7; return 0;     // 256 x 128, 8 waves (4M only)
    case 6: *bm = 7; *bn = 7; return 0;     // 128 x 128 with raised matrix-core priority (4M only)
    case 7: *bm = 7; *bn = 7; return 0;     // 128 x 128 direct-to-LDS ring (4M / 3M, summed bits lowest)
    case 8: *bm = 8; *bn = 7; return 0;     // 256 x 128 direct-to-LDS ring, 8 waves
    case 9: *bm = 7; *bn = 7; return 0;     // 128 x 128 direct-to-LDS ring, 3 (4M) / 4 (3M) waves per SIMD
    case 10: *bm = 7; *bn = 7; return 0;    // 128 x 128 BF16x3 on pre-split operands (direct-to-LDS), 2 stages in flight
    case 11: *bm = 8; *bn = 7; return 0;    // 256 x 128 BF16x3 on pre-split operands, 8 waves
    case 12: *bm = 7; *bn = 7; return 0;    // 128 x 128 BF16x3 on pre-split operands, 3 stages in flight
    case 13: *bm = 8; *bn = 7; return 0;    // 256 x 128 BF16x3 on pre-split operands, next stage's fragments prefetched
    case 14: *bm = 7; *bn = 7; return 0;    // 128 x 128 direct-to-LDS 4M, 4-stage ring, next stage's fragments prefetched
    default: return -1;
  }
}

bool gemm_tile_ok(const GemmOp& op, int tile, int prec) {
  int bm, bn;
  if (gemm_tile_bits(tile, &bm, &bn)) return false;
  // pre-split operands run on their own kernel only
  const bool split_tile = tile >= kSplitTile && tile < kSplitTile + kNumSplitTiles;
  if (op.ab_split) return prec == TN_C64_BF16X3 && split_tile && op.n_k >= 3;
  if (split_tile) return false;
  if (prec == TN_C128) return tile == kValuTile;
  if (tile < kNumTilesShared || tile == kValuTile) return true;
  if (prec == TN_C64_3M ? (tile != 7 && tile != 8 && tile != 9) : prec != TN_C64_4M) return false;
  if (tile >= 7) {
    // the summed bits must be the lowest positions of both operands, in order
    if (op.n_k < 3) return false;
    for (int i = 0; i < op.n_k; i++)
      if (op.a_k[i] != i || op.b_k[i] != i) return false;
  }
  return true;
}

const char* gemm_kernel_name(const GemmOp& op, int prec) {
  if (prec == TN_C128) return "gemm_valu<double>";
  if (op.tile == kValuTile) return "gemm_valu<float>";
  if (prec == TN_C64_3M) {
    switch (op.tile) {
      case 0: return "gemm_mfma_3m<128,128,2,4>";
      case 1: return "gemm_mfma_3m<64,128,1,4>";
      case 2: return "gemm_mfma_3m<128,64,2,2>";
      case 3: return "gemm_mfma_3m<64,64,1,2>";
      case 7: return "gemm_mfma_3m_dl<128,128,2,2>";
      case 8: return "gemm_mfma_3m_dl<256,128,4,2>";
      case 9: return "gemm_mfma_3m_dl<128,128,2,4,4>";
      default: return "?";
    }
  }
  if (prec == TN_C64_BF16X3) {
    switch (op.tile) {
      case kSplitTile: return "gemm_mfma_bf16x3_dl<128,128,2,2,2,3>";
      case kSplitTile + 1: return "gemm_mfma_bf16x3_dl<256,128,4,2,2,3>";
      case kSplitTile + 2: return "gemm_mfma_bf16x3_dl<128,128,2,2,1,4>";
      case kSplitTile + 3: return "gemm_mfma_bf16x3_dlp<256,128,4,2,2>";
      case 0: return "gemm_mfma_bf16x3<128,128,8,2,2>";
      case 1: return "gemm_mfma_bf16x3<64,128,8,1,2,1>";
      case 2: return "gemm_mfma_bf16x3<128,64,8,2,1>";
      case 3: return "gemm_mfma_bf16x3<64,64,8,1,1,1>";
      default: return "?";
    }
  }
  switch (op.tile) {
    case 0: return "gemm_mfma_4m<128,128,2,2>";
    case 1: return "gemm_mfma_4m<64,128,1,2>";
    case 2: return "gemm_mfma_4m<128,64,2,1>";
    case 3: return "gemm_mfma_4m<64,64,1,1>";
    case 5: return "gemm_mfma_4m<256,128,4,2>";
    case 6: return "gemm_mfma_4m<128,128,2,2,1>";
    case 7: return "gemm_mfma_4m_dl<128,128,2,2>";
    case 8: return "gemm_mfma_4m_dl<256,128,4,2>";
    case 9: return "gemm_mfma_4m_dl<128,128,2,2,3>";
    case 14: return "gemm_mfma_4m_dlp<128,128,2,2,2>";
    default: return "?";
  }
}

static hipError_t launch_gemm_kernel(const Ctx& ctx, const GemmOp& op, int prec, dim3 grid, hipStream_t s);

hipError_t launch_gemm(const Ctx& ctx, const GemmOp& in, int prec, hipStream_t s) {
  GemmOp op = in;
  const int ks = op.k_split_bits > 0 ? op.k_split_bits : 0;
  const int e_bits = op.n_h + op.n_m + op.n_n;
  op.run_a_s.n = 0;
  op.run_b_s.n = 0;
  op.c_split_shift = 0;
  if (ks) {
    // the kernels sum the low n_k - ks summed bits; split z adds the top ks
    // bits' offsets and writes its tile to part[z][h][m][n]
    if (ks >= op.n_k || e_bits + ks > 40 || ks > 10) return hipErrorInvalidValue;
    op.n_k -= ks;
    make_runs(op.a_k + op.n_k, ks, op.run_a_s);
    make_runs(op.b_k + op.n_k, ks, op.run_b_s);
    op.c = op.part;
    op.accumulate = 0;
    for (int j = 0; j < op.n_n; j++) op.c_n[j] = (int8_t)j;
    for (int i = 0; i < op.n_m; i++) op.c_m[i] = (int8_t)(op.n_n + i);
    for (int i = 0; i < op.n_h; i++) op.c_h[i] = (int8_t)(op.n_n + op.n_m + i);
    op.c_split_shift = e_bits;
  }
  make_runs(op.a_h, op.n_h, op.run_a_h);
  make_runs(op.b_h, op.n_h, op.run_b_h);
  make_runs(op.c_h, op.n_h, op.run_c_h);
  make_runs(op.a_m, op.n_m, op.run_a_m);
  make_runs(op.c_m, op.n_m, op.run_c_m);
  make_runs(op.b_n, op.n_n, op.run_b_n);
  make_runs(op.c_n, op.n_n, op.run_c_n);
  int bm, bn;
  int tile = op.tile;
  if (prec == TN_C128) tile = 4;
  op.tile = tile;
  if (gemm_tile_bits(tile, &bm, &bn) || !gemm_tile_ok(op, tile, prec)) return hipErrorInvalidValue;
  const int tm = op.n_m < bm ? op.n_m : bm, tn = op.n_n < bn ? op.n_n : bn;
  const uint64_t tiles = uint64_t(1) << ((op.n_m - tm) + (op.n_n - tn));
  const uint64_t gy = uint64_t(ctx.n_batch) << op.n_h;
  if (tiles > 0x7fffffffULL || gy > 65535) return hipErrorInvalidConfiguration;
  hipError_t err = launch_gemm_kernel(ctx, op, prec, dim3((unsigned)tiles, (unsigned)gy, 1u << ks), s);
  if (err != hipSuccess || !ks) return err;
  SplitReduceOp r;
  r.part = in.part;
  r.c = in.c;
  r.n_e = e_bits;
  r.n_split = ks;
  r.accumulate = in.accumulate;
  int8_t pos[kMaxBits];
  for (int j = 0; j < in.n_n; j++) pos[j] = in.c_n[j];
  for (int i = 0; i < in.n_m; i++) pos[in.n_n + i] = in.c_m[i];
  for (int i = 0; i < in.n_h; i++) pos[in.n_n + in.n_m + i] = in.c_h[i];
  make_runs(pos, e_bits, r.run_c);
  dim3 rg(blocks_for(uint64_t(1) << e_bits, 256), ctx.n_batch);
  if (prec == TN_C128) hipLaunchKernelGGL(split_reduce_kernel<double>, rg, dim3(256), 0, s, ctx, r);
  else hipLaunchKernelGGL(split_reduce_kernel<float>, rg, dim3(256), 0, s, ctx, r);
  return hipGetLastError();
}

static hipError_t launch_gemm_kernel(const Ctx& ctx, const GemmOp& op, int prec, dim3 grid, hipStream_t s) {
  const int tile = op.tile;
  if (prec == TN_C128) {
    hipLaunchKernelGGL(gemm_valu<double>, grid, dim3(256), 0, s, ctx, op);
    return hipGetLastError();
  }
  if (tile == 4) {
    hipLaunchKernelGGL(gemm_valu<float>, grid, dim3(256), 0, s, ctx, op);
    return hipGetLastError();
  }
  if (prec == TN_C64_3M) {
    switch (tile) {
      // block tiles as in gemm_tile_bits; waves of 64 x 32
      case 0: hipLaunchKernelGGL((gemm_mfma_3m<128, 128, 2, 4>), grid, dim3(512), 0, s, ctx, op); break;
      case 1: hipLaunchKernelGGL((gemm_mfma_3m<64, 128, 1, 4>), grid, dim3(256), 0, s, ctx, op); break;
      case 2: hipLaunchKernelGGL((gemm_mfma_3m<128, 64, 2, 2>), grid, dim3(256), 0, s, ctx, op); break;
      case 3: hipLaunchKernelGGL((gemm_mfma_3m<64, 64, 1, 2>), grid, dim3(128), 0, s, ctx, op); break;
      // direct-to-LDS ring: waves of 64 x 64 (7, 8) or 64 x 32 (9)
      case 7: hipLaunchKernelGGL((gemm_mfma_3m_dl<128, 128, 2, 2>), grid, dim3(256), 0, s, ctx, op); break;
      case 8: hipLaunchKernelGGL((gemm_mfma_3m_dl<256, 128, 4, 2>), grid, dim3(512), 0, s, ctx, op); break;
      case 9: hipLaunchKernelGGL((gemm_mfma_3m_dl<128, 128, 2, 4, 4>), grid, dim3(512), 0, s, ctx, op); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  if (prec == TN_C64_BF16X3) {
    switch (tile) {
      case kSplitTile: hipLaunchKernelGGL((gemm_mfma_bf16x3_dl<128, 128, 2, 2, 2, 3>), grid, dim3(256), 0, s, ctx, op); break;
      case kSplitTile + 1: hipLaunchKernelGGL((gemm_mfma_bf16x3_dl<256, 128, 4, 2, 2, 3>), grid, dim3(512), 0, s, ctx, op); break;
      case kSplitTile + 2: hipLaunchKernelGGL((gemm_mfma_bf16x3_dl<128, 128, 2, 2, 1, 4>), grid, dim3(256), 0, s, ctx, op); break;
      case kSplitTile + 3: hipLaunchKernelGGL((gemm_mfma_bf16x3_dlp<256, 128, 4, 2, 2>), grid, dim3(512), 0, s, ctx, op); break;
      case 0: hipLaunchKernelGGL((gemm_mfma_bf16x3<128, 128, 8, 2, 2>), grid, dim3(256), 0, s, ctx, op); break;
      // the 64-row variants load twice as many elements per thread: one wave per SIMD
      case 1: hipLaunchKernelGGL((gemm_mfma_bf16x3<64, 128, 8, 1, 2, 1>), grid, dim3(128), 0, s, ctx, op); break;
      case 2: hipLaunchKernelGGL((gemm_mfma_bf16x3<128, 64, 8, 2, 1>), grid, dim3(128), 0, s, ctx, op); break;
      case 3: hipLaunchKernelGGL((gemm_mfma_bf16x3<64, 64, 8, 1, 1, 1>), grid, dim3(64), 0, s, ctx, op); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  switch (tile) {
    case 0: hipLaunchKernelGGL((gemm_mfma_4m<128, 128, 2, 2>), grid, dim3(256), 0, s, ctx, op); break;
    case 1: hipLaunchKernelGGL((gemm_mfma_4m<64, 128, 1, 2>), grid, dim3(128), 0, s, ctx, op); break;
    case 2: hipLaunchKernelGGL((gemm_mfma_4m<128, 64, 2, 1>), grid, dim3(128), 0, s, ctx, op); break;
    case 3: hipLaunchKernelGGL((gemm_mfma_4m<64, 64, 1, 1>), grid, dim3(64), 0, s, ctx, op); break;
    case 5: hipLaunchKernelGGL((gemm_mfma_4m<256, 128, 4, 2>), grid, dim3(512), 0, s, ctx, op); break;
    case 6: hipLaunchKernelGGL((gemm_mfma_4m<128, 128, 2, 2, 1>), grid, dim3(256), 0, s, ctx, op); break;
    case 7: hipLaunchKernelGGL((gemm_mfma_4m_dl<128, 128, 2, 2>), grid, dim3(256), 0, s, ctx, op); break;
    case 8: hipLaunchKernelGGL((gemm_mfma_4m_dl<256, 128, 4, 2>), grid, dim3(512), 0, s, ctx, op); break;
    case 9: hipLaunchKernelGGL((gemm_mfma_4m_dl<128, 128, 2, 2, 3>), grid, dim3(256), 0, s, ctx, op); break;
    case 14: hipLaunchKernelGGL((gemm_mfma_4m_dlp<128, 128, 2, 2, 2>), grid, dim3(256), 0, s, ctx, op); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_permute(const Ctx& ctx, const PermuteOp& in, bool f64, hipStream_t s) {
  PermuteOp op = in;
  make_runs(op.src_pos, op.n_bits, op.run_src);
  make_runs(op.dst_pos, op.n_bits, op.run_dst);
  const uint64_t n = uint64_t(1) << op.n_bits;
  dim3 grid(blocks_for(n, 256), op.per_slice_serial ? 1 : ctx.n_batch);
  const bool sd = op.src_c128 != 0, dd = op.dst_c128 != 0;
  (void)f64;
  if (sd && dd) hipLaunchKernelGGL((permute_kernel<double, double>), grid, dim3(256), 0, s, ctx, op);
  else if (sd) hipLaunchKernelGGL((permute_kernel<double, float>), grid, dim3(256), 0, s, ctx, op);
  else if (dd) hipLaunchKernelGGL((permute_kernel<float, double>), grid, dim3(256), 0, s, ctx, op);
  else hipLaunchKernelGGL((permute_kernel<float, float>), grid, dim3(256), 0, s, ctx, op);
  return hipGetLastError();
}

hipError_t launch_accum(const Ctx& ctx, const AccumOp& op, bool f64, hipStream_t s) {
  dim3 grid(blocks_for((uint64_t)op.n, 256));
  if (f64) hipLaunchKernelGGL(accum_kernel<double>, grid, dim3(256), 0, s, ctx, op);
  else hipLaunchKernelGGL(accum_kernel<float>, grid, dim3(256), 0, s, ctx, op);
  return hipGetLastError();
}

hipError_t launch_counter(const Ctx& ctx, int64_t value, int add, hipStream_t s) {
  hipLaunchKernelGGL(counter_kernel, dim3(1), dim3(64), 0, s, ctx, value, add);
  return hipGetLastError();
}

hipError_t launch_split(const Ctx& ctx, const SplitOp& in, hipStream_t s) {
  SplitOp op = in;
  if (op.n_k < 3 || op.n_rows + op.n_k > 40) return hipErrorInvalidValue;
  make_runs(op.row_pos, op.n_rows, op.run_row);
  make_runs(op.k_pos + 2, op.n_k - 2, op.run_khi);
  for (int j = 0; j < 4; j++)
    op.j_off[j] = ((j & 1) ? 1u << op.k_pos[0] : 0u) + ((j & 2) ? 1u << op.k_pos[1] : 0u);
  const uint64_t threads = uint64_t(1) << (op.n_rows + op.n_k - 2);
  dim3 grid(blocks_for(threads, 256), ctx.n_batch);
  hipLaunchKernelGGL(split_kernel, grid, dim3(256), 0, s, ctx, op);
  return hipGetLastError();
}

hipError_t launch_fill(uint64_t base, uint64_t bytes, hipStream_t s) {
  const uint64_t words = (bytes + 7) / 8;
  if (words == 0) return hipSuccess;
  const uint64_t blocks = blocks_for(words, 256);
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)(blocks < (1u << 23) ? blocks : (1u << 23))), dim3(256), 0, s, base,
                     words);
  return hipGetLastError();
}

}  // namespace tn
