// Internal types shared by the host planner (plan.cpp) and the device code
// (kernels.hip, exec.hip).  Not part of the public ABI.
//
// Every index of dimension 2^b is split into b binary "bit indices".  A tensor
// is then addressed by bit positions: the element offset of an assignment is
// the sum over its bit indices of (bit value << position), so any axis
// permutation, and any leaf with sliced axes removed, is described by the list
// of positions of its bits.  Kernels read operands straight from such layouts
// (the permutation is fused into the loads) and write outputs into the layout
// the consuming node asks for.
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace tn {

constexpr int kMaxBits = 48;      // bits per class list (rows, k)
constexpr int kMaxInThread = 4;   // in-thread free bits of the row kernels (16 outputs)
constexpr int kMaxSliceTerms = 8; // sliced bits on one leaf
constexpr int kMaxTileBits = 16;

// Where an operand lives.  kind: 0 = leaf (pointer table slot `slot`),
// 1 = per-slice arena (byte offset `off` + slice * arena_stride),
// 2 = external pointer table slot shared by all slices (outputs, grad_out).
struct Ref {
  int32_t kind;
  int32_t slot;
  int64_t off;
  int32_t n_slice;                       // sliced-bit terms (leaves only)
  uint8_t slice_bit[kMaxSliceTerms];     // bit of the slice id
  uint8_t slice_pos[kMaxSliceTerms];     // position in the leaf
};

// Common launch context of every op.
struct Ctx {
  uint64_t ws;            // workspace base (device address)
  uint64_t arena_stride;  // bytes between the arenas of consecutive in-flight slices
  int64_t ptrtab_off;     // byte offset of the device pointer table (uint64 per slot)
  int64_t sid_off;        // byte offset of the int64 slice-id list
  int64_t counter_off;    // byte offset of the int64 batch counter
  int64_t arena_off;      // byte offset of the first slice's arena
  int32_t n_batch;        // slices per batch (grid dimension)
  int32_t elem_bytes;     // 8 (complex64) or 16 (complex128)
};

// A position list as runs: bits src .. src+len-1 of an index land at
// positions dst .. dst+len-1 of an operand (absent bits are left out).  Kernels
// deposit an index with one shift-and-mask per run instead of one step per
// bit; layouts keep consecutive bits together, so there are few runs.
struct BitRuns {
  int32_t n;
  uint32_t r[kMaxBits];   // src | dst << 8 | len << 16
};

// Row kernel: out[c] = sum_k A[a] * opB(B[b]).  Threads enumerate `rows`
// (row index bit i has position row_c[i] in C, row_a[i] in A, row_b[i] in B;
// -1 = absent); each thread computes all 2^n_in outputs of its in-thread bits
// (positions in_c / in_b) and sums over 2^n_k values of the summed bits.
// With k_split_bits > 0 the summed range is cut into 2^k_split_bits chunks of
// 64-lane wavefronts (lanes stride over k) whose partial sums go to `part` and
// are reduced in a fixed order by the reduce kernel.
struct RowOp {
  Ref a, b, c;
  Ref part;                // split-K partials (arena), layout [chunk][row][in]
  int32_t n_rows, n_in, n_k;
  int32_t k_split_bits;    // log2 number of K chunks (split-K mode); -1 = row mode
  int32_t conj_a, conj_b;
  int32_t accumulate;      // add into C instead of overwriting
  int32_t pair_a;          // A's lowest summed bit sits at position 0 and A's base is pair-aligned: 16-byte loads over k
  int32_t pair_c;          // C's lowest in-thread bit sits at position 0: 16-byte stores over the in-thread values
  int32_t stage_c;         // a wavefront's 64 rows x in-thread values are one contiguous block of C (set at launch)
  int8_t row_c[kMaxBits], row_a[kMaxBits], row_b[kMaxBits];
  int8_t in_c[kMaxInThread], in_b[kMaxInThread];
  int8_t k_a[kMaxBits], k_b[kMaxBits];
  BitRuns run_a, run_b, run_c;   // row_a / row_b / row_c as runs
  // Launch-time tables (prepare_row): offset of in-thread value j in B and
  // in C, and the split-K lane bits (the six lowest summed bits) and chunk
  // bits (the top k_split_bits) as runs in A and B.
  uint32_t in_off_b[1 << kMaxInThread], in_off_c[1 << kMaxInThread];
  BitRuns run_ka_lane, run_kb_lane, run_ka_chunk, run_kb_chunk;
  // Offset change in A / B when the counter of the summed-bit walk carries
  // into its bit t (the walk covers summed bits from the lowest, from the
  // second for paired A loads, or from the seventh for split-K lanes).
  uint32_t kstep_a[kMaxBits], kstep_b[kMaxBits];
};

// Matrix-core / tiled GEMM: C[h, m, n] = sum_k A[h, m, k] * opB(B[h, k, n]).
// Logical bit i of m has position a_m[i] in A and c_m[i] in C, etc.  The tile
// covers the lowest tm_bits of m, tn_bits of n and tk_bits of k; the rest are
// enumerated by the grid (m, n, h) and by the k loop.
struct GemmOp {
  Ref a, b, c;
  int32_t n_h, n_m, n_n, n_k;
  int32_t conj_a, conj_b;
  int32_t accumulate;
  int32_t tile;            // tile variant id (autotuned)
  int8_t a_h[16], b_h[16], c_h[16];
  int8_t a_m[kMaxBits], c_m[kMaxBits];
  int8_t b_n[kMaxBits], c_n[kMaxBits];
  int8_t a_k[kMaxBits], b_k[kMaxBits];
  BitRuns run_a_h, run_b_h, run_c_h;     // a_h / b_h / c_h as runs
  BitRuns run_a_m, run_c_m, run_b_n, run_c_n;
  // Split-K: the top k_split_bits summed bits are enumerated by the grid's z
  // dimension; each split writes its partial product to `part`, laid out
  // [split][h][m][n] with n fastest, and a fixed-order sum over the splits
  // produces C.  Set at launch for the kernels: the positions of the split
  // bits in A and B as runs, and the element stride between splits of the
  // partial buffer (0 when the grid's z dimension is 1).
  Ref part;
  int32_t k_split_bits;
  int32_t c_split_shift;
  BitRuns run_a_s, run_b_s;
  // BF16x3 on pre-split operands: a and b point to SplitOp outputs (planes in
  // the canonical row layout, see SplitOp) instead of complex64 tensors, and
  // conj_a / conj_b were applied by the split; ab_k_bits = log2 of the whole
  // summed range (the row length of the planes, splits included)
  int32_t ab_split;
  int32_t ab_k_bits;
};

// A complex64 GEMM operand X[row][k] (rows = H then free bits, 2^n_rows of
// them; 2^n_k summed values, k in the order of the GEMM's summed bits) split
// into bf16 hi = RNE(x) and lo = RNE(x - hi) (re and im each; the source
// conjugated first when conj), stored for the BF16x3 matrix-core kernel:
// per row, per block of 8 summed values, 16-byte units of four (re, im)
// bf16 pairs.  A operand (patterns 1): units hi(k 0-3), lo(k 0-3),
// hi(k 4-7), lo(k 4-7).  B operand (patterns 2): those four units for the
// (re, -im) pattern that forms the real part of a product, then for the
// (im, re) pattern that forms the imaginary part.
struct SplitOp {
  Ref src, dst;
  int32_t n_rows, n_k;
  int32_t patterns;        // 1 (A operand) or 2 (B operand)
  int32_t conj;
  int8_t row_pos[kMaxBits];   // source position of row bit i (-1: absent)
  int8_t k_pos[kMaxBits];     // source position of summed bit i
  BitRuns run_row, run_khi;   // set at launch: row bits, summed bits from the third on
  uint32_t j_off[4];          // set at launch: source offset of summed values 0..3
};

// Fixed-order FP64 accumulation of each in-flight slice's root into dst.
struct AccumOp {
  Ref src;                 // root value (per slice, arena)
  Ref dst;                 // complex128 accumulator (pointer table slot)
  int64_t n;               // elements
};

// Copy a tensor between layouts (general bit permutation), with optional
// accumulation into the destination; used for leaf gradients and conversions.
struct PermuteOp {
  Ref src, dst;
  int32_t n_bits;
  int32_t src_c128;        // source stored as complex128 (grad_out)
  int32_t dst_c128;
  int32_t accumulate;
  int32_t per_slice_serial;// accumulate the in-flight slices one after another (deterministic)
  int8_t src_pos[kMaxBits], dst_pos[kMaxBits];
  BitRuns run_src, run_dst;      // src_pos / dst_pos as runs
};

// Runs of a position list (host side; positions < 0 are skipped).
inline void make_runs(const int8_t* pos, int n, BitRuns& R) {
  R.n = 0;
  int i = 0;
  while (i < n) {
    if (pos[i] < 0) { i++; continue; }
    int len = 1;
    while (i + len < n && pos[i + len] == pos[i] + len) len++;
    R.r[R.n++] = uint32_t(i) | uint32_t(pos[i]) << 8 | uint32_t(len) << 16;
    i += len;
  }
}

// Launch-time tables of a row op, filled on the host from its position lists
// (once per launch or graph capture): the row lists as runs, the in-thread
// offsets, the split-K lane and chunk runs, and whether a wavefront's 64 rows
// x in-thread values form one contiguous block of C (staged stores: no
// split, no accumulation, the in-thread values at C's lowest positions and
// the six lane bits of the row right above them).
inline void prepare_row(RowOp& op) {
  make_runs(op.row_a, op.n_rows, op.run_a);
  make_runs(op.row_b, op.n_rows, op.run_b);
  make_runs(op.row_c, op.n_rows, op.run_c);
  for (int j = 0; j < (1 << kMaxInThread); j++) {
    uint32_t ob = 0, oc = 0;
    for (int i = 0; i < op.n_in; i++)
      if ((j >> i) & 1) {
        if (op.in_b[i] >= 0) ob |= 1u << op.in_b[i];
        if (op.in_c[i] >= 0) oc |= 1u << op.in_c[i];
      }
    op.in_off_b[j] = ob;
    op.in_off_c[j] = oc;
  }
  const int ks = op.k_split_bits > 0 ? op.k_split_bits : 0;
  const int lane_bits = op.n_k < 6 ? op.n_k : 6;
  make_runs(op.k_a, lane_bits, op.run_ka_lane);
  make_runs(op.k_b, lane_bits, op.run_kb_lane);
  make_runs(op.k_a + (op.n_k - ks), ks, op.run_ka_chunk);
  make_runs(op.k_b + (op.n_k - ks), ks, op.run_kb_chunk);
  const int first = op.k_split_bits >= 0 ? 6 : (op.pair_a ? 1 : 0);
  const int walk = op.n_k - ks - first;
  for (int t = 0; t < kMaxBits; t++) {
    uint32_t da = 0, db = 0;
    if (t < walk) {
      da = 1u << op.k_a[first + t];
      db = 1u << op.k_b[first + t];
      for (int b = 0; b < t; b++) {
        da -= 1u << op.k_a[first + b];
        db -= 1u << op.k_b[first + b];
      }
    }
    op.kstep_a[t] = da;
    op.kstep_b[t] = db;
  }
  bool st = op.k_split_bits < 0 && op.pair_c && !op.accumulate && op.n_in >= 1 && op.n_rows >= 6;
  for (int i = 0; st && i < op.n_in; i++) st = op.in_c[i] == i;
  for (int i = 0; st && i < 6; i++) st = op.row_c[i] == op.n_in + i;
  op.stage_c = st ? 1 : 0;
}

// Whether a row op takes the streaming row kernel: row mode without
// accumulation, no row bit in B (the same small tensor for every row), at
// least one wavefront of rows, at most four summed values and at most 16 B
// values per row (run_b as set by prepare_row).
inline bool row_stream_ok(const RowOp& op) {
  return op.k_split_bits < 0 && !op.accumulate && op.run_b.n == 0 && op.n_rows >= 6 && op.n_k <= 2 &&
         (1 << (op.n_in + op.n_k)) <= 16;
}

// Offsets of the summed values k < 4 in A and in B (launch-time table of the
// streaming row kernel).
struct RowKOffsets {
  uint32_t a[4], b[4];
};

inline RowKOffsets row_k_offsets(const RowOp& op) {
  RowKOffsets ko{};
  for (int k = 0; k < (1 << op.n_k) && k < 4; k++)
    for (int i = 0; i < op.n_k; i++)
      if ((k >> i) & 1) {
        ko.a[k] += 1u << op.k_a[i];
        ko.b[k] += 1u << op.k_b[i];
      }
  return ko;
}

// Device code reads the int8 position lists a dword at a time: every op
// struct must be 4-byte aligned with a size that is a multiple of 4.
static_assert(offsetof(Ref, slice_bit) % 4 == 0 && offsetof(Ref, slice_pos) % 4 == 0, "Ref layout");
static_assert(alignof(RowOp) >= 4 && sizeof(RowOp) % 4 == 0, "RowOp layout");
static_assert(alignof(GemmOp) >= 4 && sizeof(GemmOp) % 4 == 0, "GemmOp layout");
static_assert(alignof(PermuteOp) >= 4 && sizeof(PermuteOp) % 4 == 0, "PermuteOp layout");
static_assert(alignof(AccumOp) >= 4 && sizeof(AccumOp) % 4 == 0, "AccumOp layout");
static_assert(alignof(SplitOp) >= 4 && sizeof(SplitOp) % 4 == 0, "SplitOp layout");

}  // namespace tn
