// Host-side plan: everything tn_plan fixes once per network structure and tree.
#pragma once

#include <array>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/tn.h"
#include "tn_internal.h"

namespace tn {

enum class OpKind { Row, RowReduce, Gemm, Accum, Permute, Fill, Counter, Split };

enum KernelClass { kRow = 0, kSplitK = 1, kGemm = 2, kGemmSplitK = 3 };

struct Op {
  Op() { std::memset(&row, 0, sizeof row); std::memset(&gemm, 0, sizeof gemm);
         std::memset(&accum, 0, sizeof accum); std::memset(&perm, 0, sizeof perm);
         std::memset(&split, 0, sizeof split); }
  OpKind kind = OpKind::Fill;
  int node = -1;          // tree node this op belongs to (reporting / tuning)
  RowOp row;
  GemmOp gemm;
  AccumOp accum;
  PermuteOp perm;
  SplitOp split;
  int64_t fill_off = 0, fill_bytes = 0;   // Fill: arena range to zero
  int32_t fill_slot = -1;                 // Fill: pointer-table slot (bytes = fill_bytes) instead
  double flops = 0, bytes = 0;            // algorithmic, per slice
  int64_t grid_rows = 0;                  // rows (row ops) or tiles (gemm) per slice
};

// Layout of one tensor: position of every present bit index; -1 = absent.
struct Layout {
  std::vector<int> bits;      // bit ids in increasing position order
  std::vector<int> pos;       // their positions
  bool compact = true;        // positions are 0..n-1
  int pos_of(int bit) const {
    for (size_t i = 0; i < bits.size(); i++)
      if (bits[i] == bit) return pos[i];
    return -1;
  }
  int n() const { return (int)bits.size(); }
};

struct NodeInfo {
  int l = -1, r = -1;
  std::vector<int> H, M, N, K;       // bit ids by class w.r.t. (l = M side, r = N side)
  int kclass = kRow;
  bool swap = false;                 // A operand = right child
  int tile = 0;                      // gemm tile variant
  int k_split_bits = 0;
  double flops = 0, bytes = 0;       // per slice, algorithmic
};

}  // namespace tn

struct tn_plan_s {
  // copies of the inputs
  int32_t n_leaves = 0, n_idx = 0, n_out = 0, n_sliced = 0;
  std::vector<int32_t> rank;
  std::vector<int64_t> leaf_idx, leaf_off, idx_dim, out_idx, sliced;
  std::vector<int32_t> left, right;
  tn_options opt{};
  int prec = TN_C64_4M;
  int elem_bytes = 8;

  // bit expansion
  std::vector<int> bit_base, bit_count;   // per index
  std::vector<int> bit_index, bit_sub;    // per bit id
  std::vector<int> bit_slice;             // slice-id bit for sliced bits, else -1
  int n_bits = 0;
  int slice_id_bits = 0;
  int64_t d_sliced = 1;

  // tree (internal node k = node n_leaves + k)
  std::vector<std::vector<int64_t>> kept_idx;   // per node, index ids (unsliced)
  std::vector<std::vector<int>> kept_bits;      // per node, bit ids with sliced bits removed
  std::vector<tn::NodeInfo> nodes;              // per internal node
  std::vector<tn::Layout> layout;               // per node
  std::vector<char> needs_grad;                 // per node: subtree holds a wrt leaf (backward plans)

  // statistics
  int W = 0, W_s = 0;
  double log2_C = 0, flops_per_slice = 0;

  // forward program
  std::vector<tn::Op> fwd;
  int64_t root_off = -1;     // arena offset of the root value (forward program)
  uint64_t arena_bytes = 0;
  int n_batch = 1;
  // workspace layout
  int64_t counter_off = 0, ptrtab_off = 0, sid_off = 0, arena_off = 0;
  int64_t max_ids = 0;
  int n_slots = 0;       // pointer table: leaves, then extra slots
  int slot_out = 0, slot_gout = 0, slot_grad0 = 0;
  uint64_t workspace_bytes = 0;

  // backward program, built on first use for a given wrt set
  std::vector<int32_t> bwd_wrt;
  std::vector<tn::Op> bwd;
  uint64_t bwd_arena_bytes = 0, bwd_workspace_bytes = 0;
  double bwd_flops_per_slice = 0;
  bool bwd_built = false;

  // Serialises every entry point that reads or changes the mutable state
  // below (graph cache, backward program, tile choices) or enqueues work.
  std::mutex mu;
  // cached HIP graphs, keyed by (mode, workspace address); at most
  // kMaxGraphs, least recently used evicted first.  `done` is an event
  // recorded after the entry's latest launch: an entry is destroyed only
  // after that event has completed, so no graph is freed while it runs.
  struct GraphEntry {
    void* exec = nullptr;   // hipGraphExec_t
    void* done = nullptr;   // hipEvent_t
    uint64_t last_use = 0;
  };
  static constexpr size_t kMaxGraphs = 8;
  std::map<std::pair<int, uint64_t>, GraphEntry> graphs;
  uint64_t graph_clock = 0;
  bool tuned = false;
  // autotune trials of the last tn_plan_tune: shape key (h, m, n, k, split
  // bits, direct-to-LDS eligible), tile, trial k bits, median ms
  struct TuneTrial {
    std::array<int, 6> key;
    int tile = 0, k_bits = 0;
    float ms = 0;
  };
  std::vector<TuneTrial> tune_trials;
  // matrix-core tile variants: autotuned choice per (h, m, n, k, split bits,
  // direct-to-LDS eligible), applied to the forward and backward programs;
  // a variant pinned by tn_plan_set_tile (-1: none) goes wherever it applies
  std::map<std::array<int, 6>, int> tile_choice;
  int pinned_tile = -1;
};

namespace tn {
int build_plan(tn_plan_s* p, std::string& err);
int build_backward(tn_plan_s* p, const std::vector<int32_t>& wrt, std::string& err);
void layout_workspace(tn_plan_s* p, uint64_t arena_bytes, int n_batch, int64_t max_ids,
                      int extra_slots, uint64_t* ws_bytes);
}  // namespace tn
