// tn_plan: host-side compilation of a contraction tree into a program of
// kernel launches (problem statement Sec. 2; slicing Sec. 4.7.1).
//
// Steps:
//   1. validate the network, tree and sliced set;
//   2. split every index of dimension 2^b into b bit indices; sliced bits are
//      removed from the tensors and become per-slice leaf offsets;
//   3. kept set of every node: index e is kept at v iff it occurs below v and
//      is an output or occurs outside v's subtree (eq. incidence, extended to
//      hyperedges and open indices); width W (eq. edgecon) and cost C (eq.
//      vertexcon) follow;
//   4. classes of every pairwise contraction: H (batch: both children, kept),
//      M (left only), N (right only), K (both, summed);
//   5. kernel class by shape: matrix-core GEMM when both free sides have at
//      least 32 elements, otherwise a vector-ALU row kernel whose small free
//      side stays inside each thread (split over K when rows are few);
//   6. layouts, top down from the root: each node asks its children to store
//      their values as [H][free][K] with K in the lowest bits, so that the
//      consumer's tile loads run along contiguous memory; the producer writes
//      that permuted layout directly (no separate transpose);
//   7. arena offsets from buffer lifetimes (first fit).
#include "plan.h"
#include "smallk_rule.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <numeric>
#include <set>

namespace tn {

static int log2_exact(int64_t d) {
  if (d < 1) return -1;
  int b = 0;
  while ((int64_t(1) << b) < d) b++;
  return (int64_t(1) << b) == d ? b : -1;
}

static bool contains(const std::vector<int>& v, int x) {
  return std::find(v.begin(), v.end(), x) != v.end();
}

// ---------------------------------------------------------------- validation

static int validate(tn_plan_s* p, std::string& err) {
  const int n = p->n_leaves;
  p->leaf_off.assign(n + 1, 0);
  std::vector<int> total(p->n_idx, 0);
  for (int i = 0; i < p->n_idx; i++)
    if (p->idx_dim[i] < 1) { err = "index " + std::to_string(i) + " has dimension < 1"; return TN_E_INVALID; }
  for (int v = 0; v < n; v++) {
    if (p->rank[v] < 0) { err = "negative rank"; return TN_E_INVALID; }
    p->leaf_off[v + 1] = p->leaf_off[v] + p->rank[v];
  }
  for (int v = 0; v < n; v++) {
    for (int a = 0; a < p->rank[v]; a++) {
      int64_t e = p->leaf_idx[p->leaf_off[v] + a];
      if (e < 0 || e >= p->n_idx) { err = "leaf " + std::to_string(v) + ": index id out of range"; return TN_E_INVALID; }
      for (int b = 0; b < a; b++)
        if (p->leaf_idx[p->leaf_off[v] + b] == e) {
          err = "leaf " + std::to_string(v) + " repeats index " + std::to_string(e) + " (self-loop)";
          return TN_E_INVALID;
        }
      total[e]++;
    }
  }
  std::vector<char> is_out(p->n_idx, 0), is_sl(p->n_idx, 0);
  for (int i = 0; i < p->n_out; i++) {
    int64_t e = p->out_idx[i];
    if (e < 0 || e >= p->n_idx) { err = "output index out of range"; return TN_E_INVALID; }
    if (is_out[e]) { err = "output index listed twice"; return TN_E_INVALID; }
    if (total[e] < 1) { err = "output index on no leaf"; return TN_E_INVALID; }
    is_out[e] = 1;
  }
  for (int e = 0; e < p->n_idx; e++)
    if (total[e] == 1 && !is_out[e]) {
      err = "index " + std::to_string(e) + " is on one leaf only and is not an output";
      return TN_E_INVALID;
    }
  for (int i = 0; i < p->n_sliced; i++) {
    int64_t e = p->sliced[i];
    if (e < 0 || e >= p->n_idx) { err = "sliced index out of range"; return TN_E_INVALID; }
    if (is_out[e]) { err = "sliced index " + std::to_string(e) + " is an output"; return TN_E_INVALID; }
    if (is_sl[e]) { err = "sliced index listed twice"; return TN_E_INVALID; }
    is_sl[e] = 1;
  }
  std::vector<char> used(2 * n - 1, 0);
  for (int k = 0; k < n - 1; k++) {
    int l = p->left[k], r = p->right[k], v = n + k;
    if (l < 0 || r < 0 || l >= v || r >= v || l == r || used[l] || used[r]) {
      err = "tree is not a full binary tree over the leaves (node " + std::to_string(v) + ")";
      return TN_E_INVALID;
    }
    used[l] = used[r] = 1;
  }
  // GPU path: every dimension a power of two
  for (int e = 0; e < p->n_idx; e++)
    if (log2_exact(p->idx_dim[e]) < 0) {
      err = "index " + std::to_string(e) + " has dimension " + std::to_string(p->idx_dim[e]) +
            ", not a power of two";
      return TN_E_UNSUPPORTED;
    }
  return TN_OK;
}

// ---------------------------------------------------------------- kept sets

static void kept_sets(tn_plan_s* p) {
  const int n = p->n_leaves, nn = 2 * n - 1;
  std::vector<int> total(p->n_idx, 0);
  std::vector<char> is_out(p->n_idx, 0);
  for (int64_t e : p->leaf_idx) total[e]++;
  for (int64_t e : p->out_idx) is_out[e] = 1;
  // per node: (index, leaf occurrences below) for kept indices, sorted by index
  std::vector<std::vector<std::pair<int64_t, int>>> cnt(nn);
  p->kept_idx.assign(nn, {});
  for (int v = 0; v < n; v++) {
    for (int a = 0; a < p->rank[v]; a++) cnt[v].push_back({p->leaf_idx[p->leaf_off[v] + a], 1});
    std::sort(cnt[v].begin(), cnt[v].end());
    for (auto& x : cnt[v]) p->kept_idx[v].push_back(x.first);
  }
  for (int k = 0; k < n - 1; k++) {
    int v = n + k;
    auto& A = cnt[p->left[k]];
    auto& B = cnt[p->right[k]];
    std::vector<std::pair<int64_t, int>> merged;
    size_t i = 0, j = 0;
    while (i < A.size() || j < B.size()) {
      if (j >= B.size() || (i < A.size() && A[i].first < B[j].first)) merged.push_back(A[i++]);
      else if (i >= A.size() || B[j].first < A[i].first) merged.push_back(B[j++]);
      else { merged.push_back({A[i].first, A[i].second + B[j].second}); i++; j++; }
    }
    for (auto& x : merged)
      if (is_out[x.first] || x.second < total[x.first]) {
        cnt[v].push_back(x);
        p->kept_idx[v].push_back(x.first);
      }
  }
}

// ---------------------------------------------------------------- bits

static void expand_bits(tn_plan_s* p) {
  p->bit_base.assign(p->n_idx, 0);
  p->bit_count.assign(p->n_idx, 0);
  int nb = 0;
  for (int e = 0; e < p->n_idx; e++) {
    p->bit_base[e] = nb;
    p->bit_count[e] = log2_exact(p->idx_dim[e]);
    nb += p->bit_count[e];
  }
  p->n_bits = nb;
  p->bit_index.assign(nb, 0);
  p->bit_sub.assign(nb, 0);
  p->bit_slice.assign(nb, -1);
  for (int e = 0; e < p->n_idx; e++)
    for (int s = 0; s < p->bit_count[e]; s++) {
      p->bit_index[p->bit_base[e] + s] = e;
      p->bit_sub[p->bit_base[e] + s] = s;
    }
  // slice id -> values: mixed radix, first sliced index most significant; with
  // power-of-two dims every value bit is one bit of the id
  int off = 0;
  p->d_sliced = 1;
  for (int i = p->n_sliced - 1; i >= 0; i--) {
    int64_t e = p->sliced[i];
    for (int s = 0; s < p->bit_count[e]; s++) p->bit_slice[p->bit_base[e] + s] = off + s;
    off += p->bit_count[e];
    p->d_sliced *= p->idx_dim[e];
  }
  p->slice_id_bits = off;
  const int n = p->n_leaves, nn = 2 * n - 1;
  p->kept_bits.assign(nn, {});
  for (int v = 0; v < nn; v++)
    for (int64_t e : p->kept_idx[v])
      for (int s = 0; s < p->bit_count[e]; s++) {
        int b = p->bit_base[e] + s;
        if (p->bit_slice[b] < 0) p->kept_bits[v].push_back(b);
      }
}

static void stats(tn_plan_s* p) {
  const int n = p->n_leaves, nn = 2 * n - 1;
  double W = 0, Ws = 0;
  std::vector<double> lw(p->n_idx);
  std::vector<char> sl(p->n_idx, 0);
  for (int e = 0; e < p->n_idx; e++) lw[e] = p->bit_count[e];
  for (int64_t e : p->sliced) sl[e] = 1;
  for (int v = 0; v < nn; v++) {
    double w = 0, ws = 0;
    for (int64_t e : p->kept_idx[v]) { w += lw[e]; if (!sl[e]) ws += lw[e]; }
    W = std::max(W, w);
    Ws = std::max(Ws, ws);
  }
  // log-sum-exp over internal nodes, in log2
  double mx = -1e300, mxs = -1e300;
  std::vector<double> lc, lcs;
  for (int k = 0; k < n - 1; k++) {
    std::set<int64_t> u(p->kept_idx[p->left[k]].begin(), p->kept_idx[p->left[k]].end());
    u.insert(p->kept_idx[p->right[k]].begin(), p->kept_idx[p->right[k]].end());
    double c = 0, cs = 0;
    for (int64_t e : u) { c += lw[e]; if (!sl[e]) cs += lw[e]; }
    lc.push_back(c);
    lcs.push_back(cs);
    mx = std::max(mx, c);
    mxs = std::max(mxs, cs);
  }
  double s = 0, ss = 0;
  for (size_t i = 0; i < lc.size(); i++) { s += std::exp2(lc[i] - mx); ss += std::exp2(lcs[i] - mxs); }
  p->W = (int)W;
  p->W_s = (int)Ws;
  p->log2_C = lc.empty() ? -INFINITY : mx + std::log2(s);
  p->flops_per_slice = lc.empty() ? 0.0 : 8.0 * std::exp2(mxs) * ss;
}

// ---------------------------------------------------------------- layouts

static Layout leaf_layout(const tn_plan_s* p, int v) {
  // row-major over t_v: the last axis is fastest; bit s of an axis value sits
  // at the axis base position + s
  Layout L;
  L.compact = false;
  int pos = 0;
  for (int a = p->rank[v] - 1; a >= 0; a--) {
    int64_t e = p->leaf_idx[p->leaf_off[v] + a];
    for (int s = 0; s < p->bit_count[e]; s++) {
      int b = p->bit_base[e] + s;
      if (p->bit_slice[b] < 0) { L.bits.push_back(b); L.pos.push_back(pos); }
      pos++;
    }
  }
  bool compact = true;
  for (size_t i = 0; i < L.pos.size(); i++) compact = compact && L.pos[i] == (int)i;
  L.compact = compact;
  return L;
}

static Layout compact_layout(const std::vector<int>& lowest_first) {
  Layout L;
  L.bits = lowest_first;
  L.pos.resize(lowest_first.size());
  std::iota(L.pos.begin(), L.pos.end(), 0);
  L.compact = true;
  return L;
}

static Ref leaf_ref(const tn_plan_s* p, int v) {
  Ref r;
  std::memset(&r, 0, sizeof r);
  r.kind = 0;
  r.slot = v;
  int pos = 0;
  for (int a = p->rank[v] - 1; a >= 0; a--) {
    int64_t e = p->leaf_idx[p->leaf_off[v] + a];
    for (int s = 0; s < p->bit_count[e]; s++) {
      int b = p->bit_base[e] + s;
      if (p->bit_slice[b] >= 0 && r.n_slice < kMaxSliceTerms) {
        r.slice_bit[r.n_slice] = (uint8_t)p->bit_slice[b];
        r.slice_pos[r.n_slice] = (uint8_t)pos;
        r.n_slice++;
      }
      pos++;
    }
  }
  return r;
}

static Ref buf_ref(int buf) {
  Ref r;
  std::memset(&r, 0, sizeof r);
  r.kind = 1;
  r.off = buf;   // buffer id until allocation
  return r;
}

static Ref slot_ref(int slot) {
  Ref r;
  std::memset(&r, 0, sizeof r);
  r.kind = 2;
  r.slot = slot;
  return r;
}

// Program under construction: ops plus symbolic buffers with lifetimes.
struct Buf {
  int64_t bytes = 0;
  int first = -1, last = -1;
  int64_t off = -1;
};

struct Prog {
  std::vector<Op> ops;
  std::vector<Buf> bufs;
  int new_buf(int64_t bytes) {
    bufs.push_back(Buf{std::max<int64_t>(bytes, 16), -1, -1, -1});
    return (int)bufs.size() - 1;
  }
  void touch(const Ref& r, int op) {
    if (r.kind != 1) return;
    Buf& b = bufs[(size_t)r.off];
    if (b.first < 0) b.first = op;
    b.last = std::max(b.last, op);
  }
  // keep a buffer alive until op index `op` (at least)
  void extend(int buf, int op) { bufs[buf].last = std::max(bufs[buf].last, op); }
};

// Operand as seen by one contraction.
struct Operand {
  Ref ref;
  Layout lay;
};

// Smallest GEMM-shaped contraction (log2 complex multiply-adds) that goes to
// the matrix-core or few-summed-values kernels.  A matrix-core launch of a
// small node costs about 20 us however little it computes (a one-block launch
// streams ~30 KB of unrolled kernel code through a cold instruction cache),
// against about 4 us for the row kernel; below ~2^25 multiply-adds the row
// kernel's lower throughput does not catch up (measured: cfg2 +17 %, cfg3 and
// cfg5h unchanged, QAOA terms -11 %).
constexpr int kMinGemmBits = 25;

static int kernel_class(const tn_plan_s* p, int m, int n, int k, int h) {
  const int min_bits = (p->opt.flags & TN_FLAG_GEMM_ALL_SIZES) ? 0 : kMinGemmBits;
  // two wide free sides: a GEMM op.  With many summed values a matrix-core
  // tile reuses each B value across its rows, where the row kernel would
  // reload it; with at most four (an outer product included) the product is
  // bound by the write of C and runs on the few-summed-values kernel, whose
  // threads keep their own operand values in registers across 16 rows
  if (m >= 5 && n >= 5 && h + m + n + k >= min_bits) return kGemm;
  return kRow;   // row or split-K, refined below
}

// Which operand supplies the in-thread (B) side of a node: for matrix-core
// nodes and row nodes with two wide free sides, the side holding the
// output's lowest axis (coalesced output tiles / contiguous row blocks);
// otherwise the smaller free side.
static bool pick_swap(int kc, const std::vector<int>& M, const std::vector<int>& N, const std::vector<int>& H,
                      const std::vector<int>& cbits) {
  const bool wide = kc == kGemm || ((int)M.size() > kMaxInThread && (int)N.size() > kMaxInThread);
  if (wide) return !cbits.empty() && contains(M, cbits[0]) && !contains(H, cbits[0]);
  return N.size() > M.size();
}

// Build one contraction op: C(out_bits in layout Cl) = sum A * op(B).
// Classes are derived from the operand and output bit sets.
// Longest summed range one matrix-core accumulator covers (log2).
constexpr int kMaxSplitSumBits = 13;
// Smallest BF16x3 matrix-core contraction (log2 complex multiply-adds) whose
// operands are split into bf16 planes once, before the GEMM, instead of in
// every block that loads a panel: the split pass reads each operand once and
// writes 8 (A) or 16 (B) bytes per element.
constexpr int kMinPresplitBits = 28;

static void push(Prog& prog, Op op);

// The split of one operand of a BF16x3 GEMM (see SplitOp): rows = the free
// bits (positions `fpos`), then the batch bits (`hpos`); summed bits `kpos`.
static Op split_op(const Ref& src, const int8_t* fpos, int nf, const int8_t* hpos, int nh, const int8_t* kpos,
                   int nk, int patterns, int conj, int dst_buf, int node, double bytes) {
  Op o;
  o.kind = OpKind::Split;
  o.node = node;
  SplitOp& t = o.split;
  t.src = src;
  t.dst = buf_ref(dst_buf);
  t.n_rows = nf + nh;
  t.n_k = nk;
  t.patterns = patterns;
  t.conj = conj;
  for (int i = 0; i < nf; i++) t.row_pos[i] = fpos[i];
  for (int i = 0; i < nh; i++) t.row_pos[nf + i] = hpos[i];
  for (int i = 0; i < nk; i++) t.k_pos[i] = kpos[i];
  o.flops = 0;
  o.bytes = bytes;
  return o;
}

static Op make_contract(const tn_plan_s* p, const Operand& A0, const Operand& B0, int conj_a,
                        int conj_b, const Ref& cref, const Layout& Cl, bool accumulate,
                        int forced_swap, int node, Prog& prog) {
  const std::vector<int>& cb = Cl.bits;
  auto inA0 = [&](int b) { return A0.lay.pos_of(b) >= 0; };
  auto inB0 = [&](int b) { return B0.lay.pos_of(b) >= 0; };
  std::vector<int> H, M, N, K;
  for (int b : cb) {
    bool a = inA0(b), bb = inB0(b);
    if (a && bb) H.push_back(b);
    else if (a) M.push_back(b);
    else if (bb) N.push_back(b);
  }
  for (int b : A0.lay.bits)
    if (!contains(cb, b)) K.push_back(b);
  // every summed bit must be in both operands
  for (int b : B0.lay.bits)
    if (!contains(cb, b) && !contains(K, b)) K.push_back(b);
  auto posC = [&](int b) { return Cl.pos_of(b); };
  auto byC = [&](std::vector<int>& v) {
    std::sort(v.begin(), v.end(), [&](int x, int y) { return posC(x) < posC(y); });
  };
  byC(H);
  byC(M);
  byC(N);
  const int h = (int)H.size(), m = (int)M.size(), n = (int)N.size(), k = (int)K.size();
  int kc = kernel_class(p, m, n, k, h);
  bool swap = false;
  if (forced_swap >= 0) swap = forced_swap != 0;
  else swap = pick_swap(kc, M, N, H, cb);
  const Operand& A = swap ? B0 : A0;
  const Operand& B = swap ? A0 : B0;
  int cA = swap ? conj_b : conj_a, cB = swap ? conj_a : conj_b;
  std::vector<int> FA = swap ? N : M, FB = swap ? M : N;
  // summed bits ordered by their position in A (contiguous loads along K)
  std::sort(K.begin(), K.end(), [&](int x, int y) { return A.lay.pos_of(x) < A.lay.pos_of(y); });

  Op op;
  std::memset(&op.row, 0, sizeof op.row);
  std::memset(&op.gemm, 0, sizeof op.gemm);
  op.node = node;
  int64_t out_elems = int64_t(1) << cb.size();
  double fl = 8.0 * std::exp2(h + m + n + k);
  double by = (double)p->elem_bytes *
              (std::exp2(A.lay.n()) + std::exp2(B.lay.n()) + (double)out_elems);
  op.flops = fl;
  op.bytes = by;
  int fa = (int)FA.size(), fb = (int)FB.size();
  if (kc == kGemm) {
    op.kind = OpKind::Gemm;
    GemmOp& g = op.gemm;
    g.a = A.ref; g.b = B.ref; g.c = cref;
    g.n_h = h; g.n_m = fa; g.n_n = fb; g.n_k = k;
    g.conj_a = cA;
    g.conj_b = cB;
    g.accumulate = accumulate ? 1 : 0;
    g.tile = 0;
    for (int i = 0; i < h; i++) { g.a_h[i] = (int8_t)A.lay.pos_of(H[i]); g.b_h[i] = (int8_t)B.lay.pos_of(H[i]); g.c_h[i] = (int8_t)posC(H[i]); }
    for (int i = 0; i < fa; i++) { g.a_m[i] = (int8_t)A.lay.pos_of(FA[i]); g.c_m[i] = (int8_t)posC(FA[i]); }
    for (int i = 0; i < fb; i++) { g.b_n[i] = (int8_t)B.lay.pos_of(FB[i]); g.c_n[i] = (int8_t)posC(FB[i]); }
    for (int i = 0; i < k; i++) { g.a_k[i] = (int8_t)A.lay.pos_of(K[i]); g.b_k[i] = (int8_t)B.lay.pos_of(K[i]); }
    op.grid_rows = int64_t(1) << (h + fa + fb);
    // few output tiles and a long sum: the top summed bits go to the grid
    // (about 2^9 blocks of 128 x 128 tiles, each summing at least 2^9 values),
    // the partial tiles to an arena buffer summed in a fixed order afterwards
    const int tiles_log = std::max(0, fa - 7) + std::max(0, fb - 7) + h;
    int ks = std::min(std::min(k - 9, 9 - tiles_log), 10);
    // a sum accumulated in one FP32 register loses accuracy as the square
    // root of its length (about 2^-24 * sqrt(K / 6) relative for terms of
    // random phase): sums longer than 2^kMaxSplitSumBits are split so that
    // no part is longer, with a partial buffer at most half the larger
    // operand; the parts are then added in a fixed order
    if (p->prec != TN_C128 && k > kMaxSplitSumBits) {
      const int acc = std::min(std::min(k - kMaxSplitSumBits, 10), k - 1 - std::min(fa, fb));
      ks = std::max(ks, acc);
    }
    g.k_split_bits = ks > 0 ? ks : 0;
    if (ks > 0) g.part = buf_ref(prog.new_buf((int64_t)p->elem_bytes << (h + fa + fb + ks)));
    // BF16x3: split both operands once into the planes the matrix-core kernel
    // streams (the GEMM then reads them instead of A and B)
    if (p->prec == TN_C64_BF16X3 && !gemm_smallk_ok(g) && k >= 3 && h + fa + fb + k >= kMinPresplitBits) {
      const int ba = prog.new_buf(int64_t(8) << (h + fa + k));
      const int bb = prog.new_buf(int64_t(16) << (h + fb + k));
      push(prog, split_op(g.a, g.a_m, fa, g.a_h, h, g.a_k, k, 1, g.conj_a, ba, node,
                          8.0 * (std::exp2(A.lay.n()) + std::exp2(h + fa + k))));
      push(prog, split_op(g.b, g.b_n, fb, g.b_h, h, g.b_k, k, 2, g.conj_b, bb, node,
                          8.0 * std::exp2(B.lay.n()) + 16.0 * std::exp2(h + fb + k)));
      g.a = buf_ref(ba);
      g.b = buf_ref(bb);
      g.conj_a = 0;
      g.conj_b = 0;
      g.ab_split = 1;
      g.ab_k_bits = k;
    }
  } else {
    op.kind = OpKind::Row;
    RowOp& r = op.row;
    r.a = A.ref; r.b = B.ref; r.c = cref;
    r.conj_a = cA;
    r.conj_b = cB;
    r.accumulate = accumulate ? 1 : 0;
    // at most kMaxInThread free bits of B in each thread (those at C's
    // lowest positions); the rest of B's free side joins the rows
    const int nin = std::min(fb, kMaxInThread);
    std::vector<int> rows = H;
    rows.insert(rows.end(), FA.begin(), FA.end());
    rows.insert(rows.end(), FB.begin() + nin, FB.end());
    byC(rows);
    r.n_rows = (int)rows.size();
    r.n_in = nin;
    r.n_k = k;
    for (int i = 0; i < r.n_rows; i++) {
      r.row_c[i] = (int8_t)posC(rows[i]);
      r.row_a[i] = (int8_t)A.lay.pos_of(rows[i]);
      r.row_b[i] = (int8_t)B.lay.pos_of(rows[i]);
    }
    for (int i = 0; i < nin; i++) { r.in_c[i] = (int8_t)posC(FB[i]); r.in_b[i] = (int8_t)B.lay.pos_of(FB[i]); }
    for (int i = 0; i < k; i++) { r.k_a[i] = (int8_t)A.lay.pos_of(K[i]); r.k_b[i] = (int8_t)B.lay.pos_of(K[i]); }
    // paired 16-byte accesses where the lowest bit of the run sits at
    // position 0 and no slice offset can make the base odd
    auto even_base = [](const Ref& rf) {
      for (int i = 0; i < rf.n_slice; i++)
        if (rf.slice_pos[i] == 0) return false;
      return true;
    };
    r.pair_a = (k >= 1 && r.k_a[0] == 0 && even_base(r.a) && p->elem_bytes == 8) ? 1 : 0;
    r.pair_c = (nin >= 1 && r.in_c[0] == 0 && even_base(r.c) && p->elem_bytes == 8) ? 1 : 0;
    // few rows and a long sum: lanes stride over K, chunks reduced in order
    int nrows = r.n_rows;
    if (nrows < 14 && k >= 6) {
      // about 2^15 wavefronts: several residency rounds, so the last one is a small tail
      int ks = std::min(k - 6, std::max(0, 15 - nrows));
      r.k_split_bits = ks;
      op.grid_rows = int64_t(1) << (nrows + ks);
      if (ks > 0) {
        int pb = prog.new_buf((int64_t)p->elem_bytes << (nrows + nin + ks));
        r.part = buf_ref(pb);
      }
    } else {
      r.k_split_bits = -1;   // row mode
      op.grid_rows = int64_t(1) << nrows;
    }
  }
  return op;
}

static void push(Prog& prog, Op op) {
  int idx = (int)prog.ops.size();
  if (op.kind == OpKind::Row) {
    prog.touch(op.row.a, idx); prog.touch(op.row.b, idx); prog.touch(op.row.c, idx);
    if (op.row.k_split_bits > 0) prog.touch(op.row.part, idx);
  } else if (op.kind == OpKind::Gemm) {
    prog.touch(op.gemm.a, idx); prog.touch(op.gemm.b, idx); prog.touch(op.gemm.c, idx);
    if (op.gemm.k_split_bits > 0) prog.touch(op.gemm.part, idx);
  } else if (op.kind == OpKind::Accum) {
    prog.touch(op.accum.src, idx); prog.touch(op.accum.dst, idx);
  } else if (op.kind == OpKind::Permute) {
    prog.touch(op.perm.src, idx); prog.touch(op.perm.dst, idx);
  } else if (op.kind == OpKind::Split) {
    prog.touch(op.split.src, idx); prog.touch(op.split.dst, idx);
  }
  prog.ops.push_back(op);
  if (prog.ops.back().kind == OpKind::Row && prog.ops.back().row.k_split_bits > 0) {
    // the reduce pass follows its row op
    Op red = prog.ops.back();
    red.kind = OpKind::RowReduce;
    red.flops = 0;
    red.bytes = 0;
    prog.touch(red.row.part, idx + 1);
    prog.touch(red.row.c, idx + 1);
    prog.ops.push_back(red);
  }
}

// K-bit order for a node whose children are both intermediates: group the
// summed bits by the class they have inside each child so that the lowest
// bits of each child's layout come from one side of that child's own product.
static int child_class(const tn_plan_s* p, int c, int b) {
  const int n = p->n_leaves;
  if (c < n) return 3;
  const NodeInfo& ci = p->nodes[c - n];
  if (contains(ci.M, b)) return 0;
  if (contains(ci.N, b)) return 1;
  return 2;
}

static void assign_layouts(tn_plan_s* p) {
  const int n = p->n_leaves, nn = 2 * n - 1;
  p->layout.assign(nn, Layout{});
  for (int v = 0; v < n; v++) p->layout[v] = leaf_layout(p, v);
  if (n == 1) return;
  // root: output order, last axis fastest
  std::vector<int> root;
  for (int i = p->n_out - 1; i >= 0; i--) {
    int64_t e = p->out_idx[i];
    for (int s = 0; s < p->bit_count[e]; s++) root.push_back(p->bit_base[e] + s);
  }
  p->layout[nn - 1] = compact_layout(root);
  for (int k = n - 2; k >= 0; k--) {
    int v = n + k;
    NodeInfo& ni = p->nodes[k];
    const Layout& Cl = p->layout[v];
    auto posC = [&](int b) { return Cl.pos_of(b); };
    auto byC = [&](std::vector<int>& x) {
      std::sort(x.begin(), x.end(), [&](int a, int b) { return posC(a) < posC(b); });
    };
    std::vector<int> H = ni.H, M = ni.M, N = ni.N, K = ni.K;
    byC(H); byC(M); byC(N);
    int kc = kernel_class(p, (int)M.size(), (int)N.size(), (int)K.size(), (int)H.size());
    const bool swap = pick_swap(kc, M, N, H, Cl.bits);
    ni.kclass = kc;
    ni.swap = swap;
    int A = swap ? ni.r : ni.l, B = swap ? ni.l : ni.r;
    std::vector<int> FA = swap ? N : M, FB = swap ? M : N;
    if (A >= n && B >= n) {
      std::sort(K.begin(), K.end(), [&](int x, int y) {
        int kx = child_class(p, A, x) * 4 + child_class(p, B, x);
        int ky = child_class(p, A, y) * 4 + child_class(p, B, y);
        return kx != ky ? kx < ky : x < y;
      });
    } else {
      int lf = A < n ? A : B;
      const Layout& L = p->layout[lf];
      std::sort(K.begin(), K.end(), [&](int x, int y) { return L.pos_of(x) < L.pos_of(y); });
    }
    if (A >= n) {
      std::vector<int> la = K;
      la.insert(la.end(), FA.begin(), FA.end());
      la.insert(la.end(), H.begin(), H.end());
      p->layout[A] = compact_layout(la);
    }
    if (B >= n) {
      std::vector<int> lb = K;
      lb.insert(lb.end(), FB.begin(), FB.end());
      lb.insert(lb.end(), H.begin(), H.end());
      p->layout[B] = compact_layout(lb);
    }
  }
}

static int classes(tn_plan_s* p, std::string& err) {
  const int n = p->n_leaves;
  p->nodes.assign(std::max(0, n - 1), NodeInfo{});
  for (int k = 0; k < n - 1; k++) {
    NodeInfo& ni = p->nodes[k];
    int v = n + k;
    ni.l = p->left[k];
    ni.r = p->right[k];
    const auto& KV = p->kept_bits[v];
    const auto& KL = p->kept_bits[ni.l];
    const auto& KR = p->kept_bits[ni.r];
    for (int b : KV) {
      bool a = contains(KL, b), c = contains(KR, b);
      if (a && c) ni.H.push_back(b);
      else if (a) ni.M.push_back(b);
      else if (c) ni.N.push_back(b);
      else { err = "internal: kept bit on neither child"; return TN_E_INVALID; }
    }
    for (int b : KL)
      if (!contains(KV, b)) {
        if (!contains(KR, b)) { err = "internal: summed bit on one child only"; return TN_E_INVALID; }
        ni.K.push_back(b);
      }
    for (int b : KR)
      if (!contains(KV, b) && !contains(KL, b)) { err = "internal: summed bit on one child only"; return TN_E_INVALID; }
    // 32-bit offsets in the bandwidth kernels, and at most 2^31 work-items
    // in the launches that take one per element
    if (KV.size() > 31 || KL.size() > 31 || KR.size() > 31) {
      err = "a tensor has 2^32 or more elements after slicing (slice more indices)";
      return TN_E_UNSUPPORTED;
    }
    if (ni.K.size() > (size_t)kMaxBits || (ni.H.size() + std::max(ni.M.size(), ni.N.size())) > (size_t)kMaxBits ||
        ni.H.size() > 16) {
      err = "contraction too large for the kernels' descriptors";
      return TN_E_UNSUPPORTED;
    }
  }
  return TN_OK;
}

// First-fit arena allocation from buffer lifetimes.
static uint64_t allocate(Prog& prog) {
  struct Ev { int t; int kind; int buf; };   // kind 0 = alloc, 1 = free
  std::vector<Ev> ev;
  for (size_t i = 0; i < prog.bufs.size(); i++) {
    if (prog.bufs[i].first < 0) continue;
    ev.push_back({prog.bufs[i].first, 0, (int)i});
    ev.push_back({prog.bufs[i].last, 1, (int)i});
  }
  // at one op: allocate everything first, free after
  std::sort(ev.begin(), ev.end(), [](const Ev& a, const Ev& b) {
    if (a.t != b.t) return a.t < b.t;
    if (a.kind != b.kind) return a.kind < b.kind;
    return a.buf < b.buf;
  });
  std::map<int64_t, int64_t> used;   // off -> size
  uint64_t peak = 0;
  const int64_t align = 256;
  for (const Ev& e : ev) {
    Buf& b = prog.bufs[e.buf];
    if (e.kind == 1) { used.erase(b.off); continue; }
    int64_t sz = (b.bytes + align - 1) / align * align;
    int64_t cur = 0;
    for (auto& u : used) {
      if (u.first - cur >= sz) break;
      cur = std::max(cur, u.first + u.second);
    }
    b.off = cur;
    used[cur] = sz;
    peak = std::max<uint64_t>(peak, (uint64_t)(cur + sz));
  }
  auto fix = [&](Ref& r) { if (r.kind == 1) r.off = prog.bufs[(size_t)r.off].off; };
  for (Op& op : prog.ops) {
    switch (op.kind) {
      case OpKind::Row:
      case OpKind::RowReduce:
        fix(op.row.a); fix(op.row.b); fix(op.row.c);
        if (op.row.k_split_bits > 0) fix(op.row.part);
        break;
      case OpKind::Gemm:
        fix(op.gemm.a); fix(op.gemm.b); fix(op.gemm.c);
        if (op.gemm.k_split_bits > 0) fix(op.gemm.part);
        break;
      case OpKind::Accum: fix(op.accum.src); fix(op.accum.dst); break;
      case OpKind::Permute: fix(op.perm.src); fix(op.perm.dst); break;
      case OpKind::Split: fix(op.split.src); fix(op.split.dst); break;
      default: break;
    }
  }
  return peak;
}

static Operand node_operand(const tn_plan_s* p, int v, const std::vector<int>& bufs) {
  Operand o;
  o.lay = p->layout[v];
  o.ref = v < p->n_leaves ? leaf_ref(p, v) : buf_ref(bufs[v]);
  return o;
}

static int64_t node_bytes(const tn_plan_s* p, int v) {
  return (int64_t)p->elem_bytes << p->kept_bits[v].size();
}

void layout_workspace(tn_plan_s* p, uint64_t arena_bytes, int n_batch, int64_t max_ids,
                      int extra_slots, uint64_t* ws_bytes) {
  auto up = [](int64_t x) { return (x + 255) / 256 * 256; };
  p->n_slots = p->n_leaves + extra_slots;
  p->counter_off = 0;
  p->ptrtab_off = 256;
  p->sid_off = p->ptrtab_off + up(8 * (int64_t)p->n_slots);
  p->max_ids = max_ids;
  p->arena_off = p->sid_off + up(8 * max_ids);
  *ws_bytes = (uint64_t)p->arena_off + arena_bytes * (uint64_t)n_batch;
}

int build_plan(tn_plan_s* p, std::string& err) {
  int rc = validate(p, err);
  if (rc) return rc;
  kept_sets(p);
  expand_bits(p);
  stats(p);
  rc = classes(p, err);
  if (rc) return rc;
  assign_layouts(p);
  const int n = p->n_leaves, nn = 2 * n - 1;
  // forward program: one contraction per internal node in tree order; the
  // root's value stays in the arena for the mode-specific tail
  Prog prog;
  std::vector<int> bufs(nn, -1);
  for (int v = n; v < nn; v++) bufs[v] = prog.new_buf(node_bytes(p, v));
  for (int k = 0; k < n - 1; k++) {
    int v = n + k;
    NodeInfo& ni = p->nodes[k];
    Operand A = node_operand(p, ni.l, bufs), B = node_operand(p, ni.r, bufs);
    Op op = make_contract(p, A, B, 0, 0, buf_ref(bufs[v]), p->layout[v], false, ni.swap ? 1 : 0, v, prog);
    ni.flops = op.flops;
    ni.bytes = op.bytes;
    ni.kclass = op.kind == OpKind::Gemm ? (op.gemm.k_split_bits > 0 ? kGemmSplitK : kGemm)
                                        : (op.row.k_split_bits >= 0 ? kSplitK : kRow);
    ni.k_split_bits = op.row.k_split_bits;
    push(prog, op);
  }
  if (nn - 1 >= n) prog.extend(bufs[nn - 1], (int)prog.ops.size());   // root read by the tail
  p->arena_bytes = std::max<uint64_t>(allocate(prog), 256);
  p->fwd = prog.ops;
  p->root_off = n > 1 ? prog.bufs[(size_t)bufs[nn - 1]].off : -1;
  // in-flight slices
  int nb = p->opt.max_inflight_slices;
  if (nb <= 0) {
    nb = 1;
    if (p->opt.workspace_cap > 0)
      nb = (int)std::max<uint64_t>(1, p->opt.workspace_cap / std::max<uint64_t>(p->arena_bytes, 1));
  }
  nb = (int)std::min<int64_t>(nb, std::max<int64_t>(1, p->d_sliced));
  nb = std::min(nb, 65535);
  p->n_batch = nb;
  int64_t max_ids = std::min<int64_t>(std::max<int64_t>(p->d_sliced, nb), int64_t(1) << 22);
  max_ids = (max_ids + nb - 1) / nb * nb;
  // slots: leaves, out, grad_out, then gradients (sized for every leaf)
  p->slot_out = n;
  p->slot_gout = n + 1;
  p->slot_grad0 = n + 2;
  layout_workspace(p, p->arena_bytes, p->n_batch, max_ids, 2 + n, &p->workspace_bytes);
  return TN_OK;
}

// ---------------------------------------------------------------- backward

// Reverse mode with recomputation.  Forward values needed by the backward pass
// are the siblings of children whose subtree holds a requested leaf.  Small
// ones (< 2^20 elements) are kept from the forward pass; large ones are kept
// only at every ceil(sqrt(#large))-th position in tree order and recomputed
// from the nearest kept descendants when first needed, caching the recomputed
// chain until its parent's step (segment checkpointing, about one extra
// forward pass of work and sqrt-many large tensors of memory).
int build_backward(tn_plan_s* p, const std::vector<int32_t>& wrt, std::string& err) {
  const int n = p->n_leaves, nn = 2 * n - 1;
  if (n < 2) { err = "backward needs at least two leaves"; return TN_E_INVALID; }
  std::vector<char> is_wrt(n, 0);
  for (int32_t t : wrt) {
    if (t < 0 || t >= n) { err = "wrt leaf out of range"; return TN_E_INVALID; }
    if (is_wrt[t]) { err = "wrt leaf listed twice"; return TN_E_INVALID; }
    is_wrt[t] = 1;
  }
  std::vector<char> need(nn, 0);
  for (int v = 0; v < n; v++) need[v] = is_wrt[v];
  for (int k = 0; k < n - 1; k++) need[n + k] = need[p->left[k]] || need[p->right[k]];
  std::vector<int> parent(nn, -1);
  for (int k = 0; k < n - 1; k++) { parent[p->left[k]] = n + k; parent[p->right[k]] = n + k; }
  // values needed as siblings
  std::vector<char> needed(nn, 0);
  for (int k = 0; k < n - 1; k++) {
    int l = p->left[k], r = p->right[k];
    if (!need[n + k]) continue;
    if (need[l]) needed[r] = 1;
    if (need[r]) needed[l] = 1;
  }
  const int small_bits = 20;
  std::vector<int> large;
  for (int v = n; v < nn; v++)
    if (needed[v] && (int)p->kept_bits[v].size() > small_bits) large.push_back(v);
  int stride = std::max(1, (int)std::ceil(std::sqrt((double)large.size())));
  std::vector<char> ckpt(nn, 0);
  for (int v = n; v < nn; v++)
    if (needed[v] && (int)p->kept_bits[v].size() <= small_bits) ckpt[v] = 1;
  for (size_t i = 0; i < large.size(); i++)
    if ((int)(i % stride) == stride - 1 || i + 1 == large.size()) ckpt[large[i]] = 1;

  Prog prog;
  std::vector<int> vbuf(nn, -1);   // current buffer holding the node value
  double flops = 0;
  auto emit_forward = [&](int v) {
    int k = v - n;
    NodeInfo& ni = p->nodes[k];
    vbuf[v] = prog.new_buf(node_bytes(p, v));
    Operand A = node_operand(p, ni.l, vbuf), B = node_operand(p, ni.r, vbuf);
    Op op = make_contract(p, A, B, 0, 0, buf_ref(vbuf[v]), p->layout[v], false, ni.swap ? 1 : 0, v, prog);
    flops += op.flops;
    push(prog, op);
  };
  // forward pass; values not kept die after their parent's forward op
  for (int v = n; v < nn; v++) emit_forward(v);
  for (int v = n; v < nn - 1; v++)
    if (!ckpt[v]) vbuf[v] = -1;   // lifetime ends at its last touch (the parent's op)
  // cotangent of the root: grad_out (complex128, out order) converted
  std::vector<int> gbuf(nn, -1);
  {
    gbuf[nn - 1] = prog.new_buf(node_bytes(p, nn - 1));
    Op op;
    op.kind = OpKind::Permute;
    std::memset(&op.perm, 0, sizeof op.perm);
    op.perm.src = slot_ref(p->slot_gout);
    op.perm.dst = buf_ref(gbuf[nn - 1]);
    op.perm.src_c128 = 1;
    op.perm.dst_c128 = p->prec == TN_C128;
    const Layout& R = p->layout[nn - 1];
    op.perm.n_bits = R.n();
    for (int i = 0; i < R.n(); i++) { op.perm.src_pos[i] = (int8_t)i; op.perm.dst_pos[i] = (int8_t)R.pos[i]; }
    op.node = nn - 1;
    push(prog, op);
  }
  // ensure a forward value is available, recomputing from kept descendants
  std::vector<int> cached;
  std::function<void(int)> ensure = [&](int v) {
    if (v < n || vbuf[v] >= 0) return;
    NodeInfo& ni = p->nodes[v - n];
    ensure(ni.l);
    ensure(ni.r);
    emit_forward(v);
    cached.push_back(v);
  };
  auto release = [&](int v) {
    if (v >= n && vbuf[v] >= 0) { prog.extend(vbuf[v], (int)prog.ops.size() - 1); vbuf[v] = -1; }
  };
  for (int v = nn - 1; v >= n; v--) {
    if (!need[v]) continue;
    NodeInfo& ni = p->nodes[v - n];
    int l = ni.l, r = ni.r;
    if (need[l]) ensure(r);
    if (need[r]) ensure(l);
    for (int side = 0; side < 2; side++) {
      int c = side == 0 ? l : r, s = side == 0 ? r : l;
      if (!need[c]) continue;
      Operand G;
      G.lay = p->layout[v];
      G.ref = buf_ref(gbuf[v]);
      Operand S = node_operand(p, s, vbuf);
      if (c >= n) {
        gbuf[c] = prog.new_buf(node_bytes(p, c));
        Op op = make_contract(p, G, S, 0, 1, buf_ref(gbuf[c]), p->layout[c], false, -1, v, prog);
        flops += op.flops;
        push(prog, op);
      } else {
        // leaf cotangent in a compact copy of the leaf's layout, then added
        // into the leaf gradient at this slice's block
        Layout Lc = p->layout[c];
        Layout tmp = compact_layout(Lc.bits);
        int tb = prog.new_buf(node_bytes(p, c));
        Op op = make_contract(p, G, S, 0, 1, buf_ref(tb), tmp, false, -1, v, prog);
        flops += op.flops;
        push(prog, op);
        int t = (int)(std::find(wrt.begin(), wrt.end(), c) - wrt.begin());
        Op sc;
        sc.kind = OpKind::Permute;
        std::memset(&sc.perm, 0, sizeof sc.perm);
        sc.perm.src = buf_ref(tb);
        Ref dst = leaf_ref(p, c);
        dst.kind = 2;
        dst.slot = p->slot_grad0 + t;
        sc.perm.dst = dst;
        sc.perm.src_c128 = p->prec == TN_C128;
        sc.perm.dst_c128 = p->prec == TN_C128;
        sc.perm.accumulate = 1;
        sc.perm.per_slice_serial = 1;
        sc.perm.n_bits = Lc.n();
        for (int i = 0; i < Lc.n(); i++) { sc.perm.src_pos[i] = (int8_t)i; sc.perm.dst_pos[i] = (int8_t)Lc.pos[i]; }
        sc.node = v;
        push(prog, sc);
      }
    }
    release(l);
    release(r);
    release(v);
    gbuf[v] = -1;
  }
  p->bwd_arena_bytes = std::max<uint64_t>(allocate(prog), 256);
  p->bwd = prog.ops;
  p->bwd_wrt = wrt;
  p->bwd_flops_per_slice = flops;
  uint64_t ws;
  layout_workspace(p, std::max(p->bwd_arena_bytes, p->arena_bytes), p->n_batch, p->max_ids, 2 + n, &ws);
  p->bwd_workspace_bytes = ws;
  // restore the forward workspace layout (same offsets below the arenas)
  layout_workspace(p, p->arena_bytes, p->n_batch, p->max_ids, 2 + n, &p->workspace_bytes);
  p->bwd_built = true;
  return TN_OK;
}

}  // namespace tn
