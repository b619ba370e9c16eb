// Element helpers, operand addressing and the bandwidth-class contraction
// kernels (row, split-K, split-K reduction).  Included inside namespace tn by
// kernels.hip; written in plain C++ over a few HIP names (__global__,
// __device__, threadIdx / blockIdx / blockDim, __shfl_xor, the GMEM address
// space tag) so that the same source can also be compiled for the host with
// stand-ins for those names and run on the CPU in tests.
#pragma once

// ------------------------------------------------------------------ helpers

template <typename T> struct C2;
template <> struct C2<float> { using t = float2; };
template <> struct C2<double> { using t = double2; };

template <typename V> struct Scal;
template <> struct Scal<float2> { using t = float; };
template <> struct Scal<double2> { using t = double; };

// element load / store through the native two-lane vector type
template <typename V>
__device__ __forceinline__ V ld(GMEM const V* p) {
  typedef typename Scal<V>::t T;
  typedef T n2 __attribute__((ext_vector_type(2)));
  const n2 v = *reinterpret_cast<GMEM const n2*>(p);
  V r;
  r.x = v.x;
  r.y = v.y;
  return r;
}

// the same through the constant address space: a uniform address becomes a
// scalar load
template <typename V>
__device__ __forceinline__ V ldc(CMEM const V* p) {
  typedef typename Scal<V>::t T;
  typedef T n2 __attribute__((ext_vector_type(2)));
  const n2 v = *reinterpret_cast<CMEM const n2*>(p);
  V r;
  r.x = v.x;
  r.y = v.y;
  return r;
}

template <typename V>
__device__ __forceinline__ void st(GMEM V* p, V v) {
  typedef typename Scal<V>::t T;
  typedef T n2 __attribute__((ext_vector_type(2)));
  n2 w;
  w.x = v.x;
  w.y = v.y;
  *reinterpret_cast<GMEM n2*>(p) = w;
}

template <typename V>
__device__ __forceinline__ V cmul(V a, V b) {
  V r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}

template <typename V>
__device__ __forceinline__ V cfma(V acc, V a, V b) {
  acc.x = acc.x + a.x * b.x - a.y * b.y;
  acc.y = acc.y + a.x * b.y + a.y * b.x;
  return acc;
}

// Entry i of a bit-position list.  `base` is the start of an int8 list in a
// 4-byte aligned op struct of the kernel arguments; reading the containing
// dword keeps the load a uniform scalar load (there are no scalar byte loads).
__device__ __forceinline__ int pos_at(const int8_t* base, int i) {
  const uint32_t w = reinterpret_cast<const uint32_t*>(base)[i >> 2];
  return (int8_t)(w >> (8 * (i & 3)));
}

// The deposits are branch-free, so the position reads stay uniform even when
// v differs between lanes.
__device__ __forceinline__ uint64_t deposit(uint64_t v, const int8_t* pos, int first, int n) {
  uint64_t off = 0;
  for (int i = 0; i < n; i++) off |= ((v >> i) & 1) << pos_at(pos, first + i);
  return off;
}

// position list may hold -1 (bit absent from this operand)
__device__ __forceinline__ uint64_t deposit_opt(uint64_t v, const int8_t* pos, int first, int n) {
  uint64_t off = 0;
  for (int i = 0; i < n; i++) {
    const int p = pos_at(pos, first + i);
    off |= p >= 0 ? ((v >> i) & 1) << p : 0;
  }
  return off;
}

// The batch counter, the slice-id list and the pointer table are read at
// uniform addresses and do not change while a kernel runs: reading them
// through the constant address space (CMEM) makes these scalar loads instead
// of a chain of dependent vector loads at the start of every wavefront.
__device__ __forceinline__ int64_t slice_id(const Ctx& ctx, int z) {
  const int64_t cnt = *reinterpret_cast<CMEM const int64_t*>(ctx.ws + ctx.counter_off);
  CMEM const int64_t* sids = reinterpret_cast<CMEM const int64_t*>(ctx.ws + ctx.sid_off);
  return sids[cnt * ctx.n_batch + z];
}

// Base address of an operand for in-flight slice z with slice id sid.
__device__ __forceinline__ GMEM char* resolve(const Ctx& ctx, const Ref& r, int z, int64_t sid, int ebytes) {
  if (r.kind == 1)
    return reinterpret_cast<GMEM char*>(ctx.ws + ctx.arena_off + uint64_t(z) * ctx.arena_stride + r.off);
  const uint64_t p = reinterpret_cast<CMEM const uint64_t*>(ctx.ws + ctx.ptrtab_off)[r.slot];
  uint64_t off = 0;
  // the term lists are read as one batch; the work stops at n_slice
  const int ns = r.n_slice;
  uint32_t wb[kMaxSliceTerms / 4], wp[kMaxSliceTerms / 4];
#pragma unroll
  for (int i = 0; i < kMaxSliceTerms / 4; i++) {
    wb[i] = reinterpret_cast<const uint32_t*>(r.slice_bit)[i];
    wp[i] = reinterpret_cast<const uint32_t*>(r.slice_pos)[i];
  }
#pragma unroll
  for (int i = 0; i < kMaxSliceTerms; i++) {
    if (i >= ns) break;
    const int sh = 8 * (i & 3);
    off |= uint64_t((sid >> ((wb[i >> 2] >> sh) & 0xFF)) & 1) << ((wp[i >> 2] >> sh) & 0xFF);
  }
  return reinterpret_cast<GMEM char*>(p) + off * uint64_t(ebytes);
}

template <typename V>
__device__ __forceinline__ V conjv(V a, int c) {
  if (c) a.y = -a.y;
  return a;
}

// ------------------------------------------------------------------ row kernel

constexpr int kRowThreads = 256;

// Offsets below are 32-bit: the planner rejects tensors of 2^32 elements or more.

// Deposit of an index through the runs of its position list: one
// shift-and-mask per run (the run table is read at uniform addresses).
__device__ __forceinline__ uint64_t deposit_runs(uint64_t v, const BitRuns& R) {
  uint64_t off = 0;
  for (int i = 0; i < R.n; i++) {
    const uint32_t w = R.r[i];
    const uint32_t src = w & 0xFF, dst = (w >> 8) & 0xFF, len = w >> 16;
    off |= ((v >> src) & (~uint64_t(0) >> (64 - len))) << dst;
  }
  return off;
}
// The first eight entries are read as one batch of scalar loads; the
// per-lane work stops at the table's length (a uniform branch).
__device__ __forceinline__ uint32_t deposit_runs32(uint32_t v, const BitRuns& R) {
  uint32_t off = 0;
  auto piece = [&](uint32_t w) {
    const uint32_t src = w & 0xFF, dst = (w >> 8) & 0xFF, len = w >> 16;
    return ((v >> src) & (~0u >> (32 - len))) << dst;
  };
  const int n = R.n;
  uint32_t w[8];
#pragma unroll
  for (int i = 0; i < 8; i++) w[i] = R.r[i];
#pragma unroll
  for (int i = 0; i < 8; i++) {
    if (i >= n) return off;
    off |= piece(w[i]);
  }
  for (int i = 8; i < n; i++) off |= piece(R.r[i]);
  return off;
}

// The same for an index that is uniform over the wavefront, one run per pass
// of a loop that is kept rolled: the run table stays in memory (scalar loads
// at each use) instead of holding scalar registers across an enclosing loop.
__device__ __forceinline__ uint32_t deposit_runs_u(uint32_t v, const BitRuns& R) {
  uint32_t off = 0;
  const int n = R.n;
#pragma unroll 1
  for (int i = 0; i < n; i++) {
    const uint32_t w = R.r[i];
    const uint32_t src = w & 0xFF, dst = (w >> 8) & 0xFF, len = w >> 16;
    off |= ((v >> src) & (~0u >> (32 - len))) << dst;
  }
  return off;
}

// Offset change of a summed-bit walk from counter value c to c + 1, from the
// op's carry table (the carry bit is clamped to the walk's n bits, so the
// last step of a walk is harmless and needs no guard).
__device__ __forceinline__ uint32_t kstep(const uint32_t* tab, uint32_t c, int n) {
  int t = __builtin_ctz(~c);
  t = t < n ? t : n - 1;
  return t < 0 ? 0u : tab[t];
}

// Offset change of a counter going from c to c + 1 when its bit i sits at
// position pos[first + i] of an operand: the trailing ones of c clear and the
// next bit sets.  Two operands walked by the same counter may order their bits
// differently, so each takes its own delta; c is uniform, so this is scalar
// work (two iterations on average).  Call only while c + 1 is in range.
__device__ __forceinline__ uint64_t step_delta(uint64_t c, const int8_t* pos, int first) {
  const int t = __builtin_ctzll(~c);
  uint64_t d = uint64_t(1) << pos_at(pos, first + t);
  for (int b = 0; b < t; b++) d -= uint64_t(1) << pos_at(pos, first + b);
  return d;
}

// Steps of a summed-range walk whose loads are issued together (a template
// parameter chosen on the host: the range is a power of two, so no step is
// ever predicated and the compiler keeps all of a chunk's loads in flight).
constexpr int row_ku(int nin) { return nin <= 2 ? 8 : (nin <= 4 ? 4 : 2); }

// Stores of one row's in-thread outputs (C + oc + in_off_c[j]).  STAGE: the
// wavefront's 64 consecutive rows form one contiguous block of 64 * NIN values
// (prepare_row's stage_c); each lane puts its NIN values into the wavefront's
// LDS area (rows padded by 16 bytes against bank conflicts) and the wavefront
// then stores the block in 1 KiB pieces (16 bytes per lane), instead of
// 16-byte pieces at a row stride that touch 64 cache lines per store.
// blk_c: offset in C of the wavefront's first row (used by STAGE only).
template <typename T, int NIN, bool STAGE, typename V>
__device__ __forceinline__ void row_store(const RowOp& op, GMEM V* Cp, uint32_t oc, uint32_t blk_c, const V (&acc)[NIN],
                                          uint32_t tid) {
  typedef T t4 __attribute__((ext_vector_type(4)));
  if constexpr (STAGE && NIN >= 2) {
    constexpr int RS = NIN * 8 + 16;                        // bytes per staged row
    __shared__ __attribute__((aligned(16))) char stage[kRowThreads / 64][64 * RS];
    const int lane = tid & 63;
    char* S = &stage[tid >> 6][0];
#pragma unroll
    for (int j = 0; j < NIN; j += 2) {
      t4 w;
      w[0] = acc[j].x;
      w[1] = acc[j].y;
      w[2] = acc[j + 1].x;
      w[3] = acc[j + 1].y;
      *reinterpret_cast<t4*>(S + lane * RS + j * 8) = w;
    }
    // one wavefront's area only: its LDS accesses are performed in order
    TN_WAVE_SYNC();
    GMEM t4* D = reinterpret_cast<GMEM t4*>(Cp + blk_c);
#pragma unroll
    for (int t = 0; t < NIN / 2; t++) {
      const int c = lane + 64 * t;                           // 16-byte piece of the block
      D[c] = *reinterpret_cast<const t4*>(S + (c / (NIN / 2)) * RS + (c % (NIN / 2)) * 16);
    }
    // the next row's LDS writes follow this wavefront's reads
    TN_WAVE_SYNC();
  } else if (NIN >= 2 && op.pair_c) {
    // in-thread values j and j + 1 are adjacent in C
#pragma unroll
    for (int j = 0; j < NIN; j += 2) {
      t4 w;
      w[0] = acc[j].x;
      w[1] = acc[j].y;
      w[2] = acc[j + 1].x;
      w[3] = acc[j + 1].y;
      *reinterpret_cast<GMEM t4*>(Cp + oc + op.in_off_c[j]) = w;
    }
  } else {
#pragma unroll
    for (int j = 0; j < NIN; j++) st(Cp + oc + op.in_off_c[j], acc[j]);
  }
}

// One thread per row; the summed bits are walked in order with their A / B
// offsets advanced as masked counters, and a batch of A loads (and the B
// loads that go with them) is issued before any of it is used, so that each
// thread keeps several memory requests in flight.
template <typename T, int NIN, int U, bool STAGE = false>
__global__ __launch_bounds__(kRowThreads) void row_kernel(Ctx ctx, RowOp op) {
  using V = typename C2<T>::t;
  typedef T t4 __attribute__((ext_vector_type(4)));
  const int z = blockIdx.y;
  const int64_t sid = slice_id(ctx, z);
  if (sid < 0) return;
  const uint32_t tid = threadIdx.x;
  const uint64_t row = uint64_t(blockIdx.x) * blockDim.x + tid;
  if (row >> op.n_rows) return;
  const int eb = sizeof(V);
  GMEM const V* A = reinterpret_cast<GMEM const V*>(resolve(ctx, op.a, z, sid, eb));
  GMEM const V* B = reinterpret_cast<GMEM const V*>(resolve(ctx, op.b, z, sid, eb));
  GMEM V* Cp = reinterpret_cast<GMEM V*>(resolve(ctx, op.c, z, sid, eb));
  const uint32_t r32 = (uint32_t)row;
  const uint32_t oa = deposit_runs32(r32, op.run_a);
  const uint32_t ob = deposit_runs32(r32, op.run_b);
  const uint32_t oc = deposit_runs32(r32, op.run_c);
  uint32_t inb[NIN], inc[NIN];
#pragma unroll
  for (int j = 0; j < NIN; j++) { inb[j] = op.in_off_b[j]; inc[j] = op.in_off_c[j]; }
  V acc[NIN];
#pragma unroll
  for (int j = 0; j < NIN; j++) { acc[j].x = 0; acc[j].y = 0; }
  const uint32_t nk = 1u << op.n_k;
  // When no row bit reaches B (a gate or a small tensor applied to every row),
  // every B address is the same for all threads: B is then read with scalar
  // loads (once per wavefront) instead of per-lane vector loads.
  CMEM const V* Bc = reinterpret_cast<CMEM const V*>(reinterpret_cast<uintptr_t>(B));
  auto walk = [&](auto uniform_b) {
    constexpr bool UB = decltype(uniform_b)::value;
    auto ldb = [&](uint32_t off) -> V {
      if constexpr (UB) return conjv(ldc(Bc + off), op.conj_b);
      else return conjv(ld(B + off), op.conj_b);
    };
    if (op.pair_a) {
      // k and k + 1 are adjacent in A: one 16-byte load for both; the counter
      // c runs over the summed bits above the lowest
      const uint32_t b1 = 1u << pos_at(op.k_b, 0);
      uint32_t xa = 0, xb = 0;
      for (uint32_t i = 0; i < (nk >> 1); i += U) {
        t4 a2[U];
        uint32_t bo[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
          a2[u] = *reinterpret_cast<GMEM const t4*>(A + oa + xa);
          bo[u] = ob + xb;
          // i is a multiple of U: inside the chunk the carry position is static
          const uint32_t c = u + 1 < U ? uint32_t(u) : i + u;
          xa += kstep(op.kstep_a, c, op.n_k - 1);
          xb += kstep(op.kstep_b, c, op.n_k - 1);
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
          V a0, a1;
          a0.x = a2[u][0];
          a0.y = op.conj_a ? -a2[u][1] : a2[u][1];
          a1.x = a2[u][2];
          a1.y = op.conj_a ? -a2[u][3] : a2[u][3];
#pragma unroll
          for (int j = 0; j < NIN; j++) {
            acc[j] = cfma(acc[j], a0, ldb(bo[u] + inb[j]));
            acc[j] = cfma(acc[j], a1, ldb(bo[u] + b1 + inb[j]));
          }
        }
      }
    } else {
      uint32_t xa = 0, xb = 0;
      for (uint32_t i = 0; i < nk; i += U) {
        V a[U];
        uint32_t bo[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
          a[u] = conjv(ld(A + oa + xa), op.conj_a);
          bo[u] = ob + xb;
          const uint32_t c = u + 1 < U ? uint32_t(u) : i + u;
          xa += kstep(op.kstep_a, c, op.n_k);
          xb += kstep(op.kstep_b, c, op.n_k);
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
#pragma unroll
          for (int j = 0; j < NIN; j++) acc[j] = cfma(acc[j], a[u], ldb(bo[u] + inb[j]));
        }
      }
    }
  };
  if (op.run_b.n == 0) walk(std::true_type());
  else walk(std::false_type());
  if (op.accumulate) {
#pragma unroll
    for (int j = 0; j < NIN; j++) {
      V o = ld(Cp + oc + inc[j]);
      acc[j].x += o.x;
      acc[j].y += o.y;
    }
  }
  row_store<T, NIN, STAGE>(op, Cp, oc, STAGE ? deposit_runs32(r32 & ~63u, op.run_c) : 0u, acc, tid);
}

// Walk of a persistent wavefront over the units first, first + step, ... <
// count, with two register sets in turn so that no value is copied between
// them: the loads into one set are issued before the stores of the unit held
// by the other (past the last unit, a set reloads its own unit: in bounds,
// unused).  Vector memory operations complete in issue order, so a load
// issued after a batch of stores could only be consumed once those stores had
// completed; this way the stores stay in flight.  The first unit is peeled
// off so that every entry to the loop sees the same operations in flight (one
// set's loads, then the other set's stores): the wait count before each body
// is then the same on every pass.
template <typename S, typename L, typename Bd>
__device__ __forceinline__ void stream_walk(uint32_t first, uint32_t step, uint32_t count, S& s0, S& s1, L&& load,
                                            Bd&& body) {
  load(s0, first);
  uint32_t nx = first + step;                     // unit held in s1
  load(s1, nx < count ? nx : first);
  body(s0, first);
  while (nx < count) {
    const uint32_t n2 = nx + step;
    load(s0, n2 < count ? n2 : nx);
    body(s1, nx);
    if (n2 >= count) break;
    const uint32_t n3 = n2 + step;
    load(s1, n3 < count ? n3 : n2);
    body(s0, n2);
    nx = n3;
  }
}

// Streaming row kernel for ops whose B has no row bit (the same small tensor
// applied to every row) and whose summed range is at most four values: such
// ops write NIN outputs per value of A they read and are bound by the HBM
// write of C.  Persistent wavefronts walk units of RB blocks of 64
// consecutive rows (stream_walk: the next unit's A values are loaded before
// the current unit's stores).  Stores (MODE):
//   0: each lane takes one row of a block and stores its NIN values;
//   1 (complex64, the block one contiguous run of C with the in-thread
//      values lowest, prepare_row's stage_c): store t of a lane writes
//      16-byte piece lane + 64 t of the block, values 2 p and 2 p + 1
//      (p = lane mod NIN / 2) of row lane / (NIN / 2) + t * 128 / NIN, so
//      that every store covers 1 KiB of C with no exchange between lanes;
//      each lane loads the A values of its NIN / 2 rows and keeps its pair's
//      B values;
//   2 (the same layouts): one row per lane, the block staged through LDS
//      and stored in 1 KiB pieces (row_store).
// The sum over k runs in index order, as in row_kernel.
template <typename T, int NIN, int KN, int MODE, int RB>
__global__ __launch_bounds__(kRowThreads) void row_stream_kernel(Ctx ctx, RowOp op, RowKOffsets ko) {
  using V = typename C2<T>::t;
  typedef T t4 __attribute__((ext_vector_type(4)));
  constexpr int WPB = kRowThreads / 64;
  static_assert(MODE == 0 || (sizeof(T) == 4 && NIN >= 2), "coalesced pieces are complex64 pairs");
  const int z = blockIdx.y;
  const int64_t sid = slice_id(ctx, z);
  if (sid < 0) return;
  const uint32_t tid = threadIdx.x;
  const uint32_t lane = tid & 63;
  // uniform over the wavefront (the compiler cannot tell by itself): the
  // block offsets below are then scalar work
  const uint32_t wave = TN_UNIFORM(blockIdx.x * WPB + (tid >> 6));
  const uint32_t nwave = gridDim.x * WPB;
  const uint32_t units = 1u << (op.n_rows - 6) >> (RB == 2 ? 1 : 0);
  if (wave >= units) return;
  const int eb = sizeof(V);
  GMEM const V* A = reinterpret_cast<GMEM const V*>(resolve(ctx, op.a, z, sid, eb));
  GMEM const V* B = reinterpret_cast<GMEM const V*>(resolve(ctx, op.b, z, sid, eb));
  GMEM V* Cp = reinterpret_cast<GMEM V*>(resolve(ctx, op.c, z, sid, eb));
  if constexpr (MODE == 1) {
    constexpr int H = NIN / 2;                    // 16-byte pieces per row
    const uint32_t p = lane % H;
    V b0[KN], b1[KN];
#pragma unroll
    for (int k = 0; k < KN; k++) {
      b0[k] = conjv(ld(B + op.in_off_b[2 * p] + ko.b[k]), op.conj_b);
      b1[k] = conjv(ld(B + op.in_off_b[2 * p + 1] + ko.b[k]), op.conj_b);
    }
    // offsets in A of the lane's rows within a block
    uint32_t la[H];
#pragma unroll
    for (int t = 0; t < H; t++) la[t] = deposit_runs32(lane / H + t * (64 / H), op.run_a);
    struct Set {
      V a[RB][H][KN];
    };
    Set s0, s1;
    stream_walk(
        wave, nwave, units, s0, s1,
        [&](Set& s, uint32_t u) {
#pragma unroll
          for (int r = 0; r < RB; r++) {
            GMEM const V* Ab = A + deposit_runs_u((u * RB + r) << 6, op.run_a);
#pragma unroll
            for (int t = 0; t < H; t++)
#pragma unroll
              for (int k = 0; k < KN; k++) s.a[r][t][k] = ld(Ab + la[t] + ko.a[k]);
          }
        },
        [&](const Set& s, uint32_t u) {
#pragma unroll
          for (int r = 0; r < RB; r++) {
            GMEM t4* D = reinterpret_cast<GMEM t4*>(Cp + deposit_runs_u((u * RB + r) << 6, op.run_c));
#pragma unroll
            for (int t = 0; t < H; t++) {
              V u0, u1;
              u0.x = u0.y = u1.x = u1.y = 0;
#pragma unroll
              for (int k = 0; k < KN; k++) {
                const V a = conjv(s.a[r][t][k], op.conj_a);
                u0 = cfma(u0, a, b0[k]);
                u1 = cfma(u1, a, b1[k]);
              }
              t4 w;
              w[0] = u0.x;
              w[1] = u0.y;
              w[2] = u1.x;
              w[3] = u1.y;
              D[lane + 64 * t] = w;
            }
          }
        });
  } else {
    // B's values are the same for every lane: scalar loads, once
    CMEM const V* Bc = reinterpret_cast<CMEM const V*>(reinterpret_cast<uintptr_t>(B));
    V bv[NIN][KN];
#pragma unroll
    for (int j = 0; j < NIN; j++)
#pragma unroll
      for (int k = 0; k < KN; k++) bv[j][k] = conjv(ldc(Bc + op.in_off_b[j] + ko.b[k]), op.conj_b);
    // a row's offsets: deposit of its block's first row (uniform) + of its lane
    const uint32_t la = deposit_runs32(lane, op.run_a), lc = deposit_runs32(lane, op.run_c);
    struct Set {
      V a[RB][KN];
    };
    Set s0, s1;
    stream_walk(
        wave, nwave, units, s0, s1,
        [&](Set& s, uint32_t u) {
#pragma unroll
          for (int r = 0; r < RB; r++) {
            const uint32_t oa = deposit_runs_u((u * RB + r) << 6, op.run_a) + la;
#pragma unroll
            for (int k = 0; k < KN; k++) s.a[r][k] = ld(A + oa + ko.a[k]);
          }
        },
        [&](const Set& s, uint32_t u) {
#pragma unroll
          for (int r = 0; r < RB; r++) {
            V sum[NIN];
#pragma unroll
            for (int j = 0; j < NIN; j++) {
              sum[j].x = 0;
              sum[j].y = 0;
            }
#pragma unroll
            for (int k = 0; k < KN; k++) {
              const V a = conjv(s.a[r][k], op.conj_a);
#pragma unroll
              for (int j = 0; j < NIN; j++) sum[j] = cfma(sum[j], a, bv[j][k]);
            }
            const uint32_t bc = deposit_runs_u((u * RB + r) << 6, op.run_c);
            row_store<T, NIN, MODE == 2>(op, Cp, bc + lc, bc, sum, tid);
          }
        });
  }
}

// ------------------------------------------------------------------ split-K

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  // fixed butterfly order: identical result on every run
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// One wavefront per (chunk of the summed range, row): lane l takes
// k = chunk * 2^cbits + 64 t + l for t = 0, 1, ..., so every load of the
// wavefront covers 64 consecutive k; the lane bits of the offset are fixed
// and the bits above advance as a masked counter.  Partial sums of the lanes
// are combined by a fixed butterfly.
template <typename T, int NIN, int U>
__global__ __launch_bounds__(kRowThreads) void splitk_kernel(Ctx ctx, RowOp op) {
  using V = typename C2<T>::t;
  const int z = blockIdx.y;
  const int64_t sid = slice_id(ctx, z);
  if (sid < 0) return;
  const int lane = threadIdx.x & 63;
  const uint64_t wave = uint64_t(blockIdx.x) * (blockDim.x / 64) + (threadIdx.x >> 6);
  const int ks = op.k_split_bits > 0 ? op.k_split_bits : 0;
  // chunk-major order: the rows of one K chunk are adjacent wavefronts, so the
  // B values they share are read from HBM once and then hit in L2
  const uint32_t row = (uint32_t)(wave & ((uint64_t(1) << op.n_rows) - 1));
  const uint32_t chunk = (uint32_t)(wave >> op.n_rows);
  if (uint64_t(chunk) >> ks) return;
  const int eb = sizeof(V);
  GMEM const V* A = reinterpret_cast<GMEM const V*>(resolve(ctx, op.a, z, sid, eb));
  GMEM const V* B = reinterpret_cast<GMEM const V*>(resolve(ctx, op.b, z, sid, eb));
  const int cbits = op.n_k - ks;                  // >= 6
  const uint32_t ba = deposit_runs32(row, op.run_a) + deposit_runs32(chunk, op.run_ka_chunk) +
                      deposit_runs32(lane, op.run_ka_lane);
  const uint32_t bb = deposit_runs32(row, op.run_b) + deposit_runs32(chunk, op.run_kb_chunk) +
                      deposit_runs32(lane, op.run_kb_lane);
  uint32_t inb[NIN];
#pragma unroll
  for (int j = 0; j < NIN; j++) inb[j] = op.in_off_b[j];
  T ar[NIN], ai[NIN];
#pragma unroll
  for (int j = 0; j < NIN; j++) { ar[j] = 0; ai[j] = 0; }
  const uint32_t steps = 1u << (cbits - 6);
  uint32_t xa = 0, xb = 0;
  for (uint32_t i = 0; i < steps; i += U) {
    V a[U];
    uint32_t bo[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      a[u] = conjv(ld(A + ba + xa), op.conj_a);
      bo[u] = bb + xb;
      const uint32_t c = u + 1 < U ? uint32_t(u) : i + u;
      xa += kstep(op.kstep_a, c, cbits - 6);
      xb += kstep(op.kstep_b, c, cbits - 6);
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
#pragma unroll
      for (int j = 0; j < NIN; j++) {
        const V b = conjv(ld(B + bo[u] + inb[j]), op.conj_b);
        ar[j] += a[u].x * b.x - a[u].y * b.y;
        ai[j] += a[u].x * b.y + a[u].y * b.x;
      }
    }
  }
#pragma unroll
  for (int j = 0; j < NIN; j++) { ar[j] = wave_sum(ar[j]); ai[j] = wave_sum(ai[j]); }
  if (lane != 0) return;
  if (ks == 0) {
    GMEM V* Cp = reinterpret_cast<GMEM V*>(resolve(ctx, op.c, z, sid, eb));
    const uint32_t oc = deposit_runs32(row, op.run_c);
#pragma unroll
    for (int j = 0; j < NIN; j++) {
      const uint32_t c = oc + op.in_off_c[j];
      V o;
      o.x = ar[j];
      o.y = ai[j];
      if (op.accumulate) { V p = ld(Cp + c); o.x += p.x; o.y += p.y; }
      st(Cp + c, o);
    }
  } else {
    // partials [row][in][chunk]: the chunks of one output are contiguous
    GMEM V* P = reinterpret_cast<GMEM V*>(resolve(ctx, op.part, z, sid, eb));
#pragma unroll
    for (int j = 0; j < NIN; j++) {
      V o;
      o.x = ar[j];
      o.y = ai[j];
      st(P + ((uint64_t(row) * NIN + j) << ks) + chunk, o);
    }
  }
}

// Sum of the split-K partials of each output in a fixed order: one wavefront
// per output, lane l adds chunks l, l + 64, ... (contiguous in the partials
// buffer), then the fixed butterfly of wave_sum.  Deterministic.
template <typename T>
__global__ __launch_bounds__(kRowThreads) void reduce_kernel(Ctx ctx, RowOp op) {
  using V = typename C2<T>::t;
  const int z = blockIdx.y;
  const int64_t sid = slice_id(ctx, z);
  if (sid < 0) return;
  const int lane = threadIdx.x & 63;
  const uint64_t o = uint64_t(blockIdx.x) * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (o >> (op.n_rows + op.n_in)) return;
  const int eb = sizeof(V);
  GMEM const V* P = reinterpret_cast<GMEM const V*>(resolve(ctx, op.part, z, sid, eb)) + (o << op.k_split_bits);
  const uint32_t nch = 1u << op.k_split_bits;
  T sx = 0, sy = 0;
  for (uint32_t ch = lane; ch < nch; ch += 64) {
    const V p = ld(P + ch);
    sx += p.x;
    sy += p.y;
  }
  sx = wave_sum(sx);
  sy = wave_sum(sy);
  if (lane != 0) return;
  GMEM V* Cp = reinterpret_cast<GMEM V*>(resolve(ctx, op.c, z, sid, eb));
  const uint64_t row = o >> op.n_in;
  const uint32_t j = (uint32_t)(o & ((1u << op.n_in) - 1));
  const uint64_t c = deposit_runs(row, op.run_c) + op.in_off_c[j];
  V s;
  s.x = sx;
  s.y = sy;
  if (op.accumulate) { V q = ld(Cp + c); s.x += q.x; s.y += q.y; }
  st(Cp + c, s);
}
