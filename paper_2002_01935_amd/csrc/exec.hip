// C-ABI entry points of libtn: plan creation, sliced/unsliced contraction,
// reverse mode, autotuning, and the launch machinery behind them.
//
// A call uploads the leaf/output pointer table and the slice-id list into the
// caller's workspace, then runs the plan's program once per batch of
// in-flight slices.  The per-batch program (every node contraction for all
// in-flight slices, the fixed-order FP64 accumulation of their roots and the
// advance of the device-side batch counter) is captured once into a HIP graph
// per (mode, workspace) and replayed for every batch, so the host issues one
// graph launch per batch and never waits on the GPU.  Kernels read the slice
// id of their in-flight slice from the workspace (slice list indexed by the
// batch counter), so the same graph serves every batch and every call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "exec.h"
#include "kernels.h"
#include "plan.h"
#include "smallk.h"

using namespace tn;

static thread_local std::string g_err;

static int set_err(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t _e = (expr);                                                            \
    if (_e != hipSuccess)                                                              \
      return set_err(TN_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

extern "C" const char* tn_last_error(void) { return g_err.c_str(); }

int tn::set_error(int code, const std::string& msg) { return set_err(code, msg); }

using PlanLock = std::lock_guard<std::mutex>;

// Wait for the last launch of a cached graph, then free it.
static void destroy_graph(tn_plan_s::GraphEntry& e) {
  if (e.done) {
    (void)hipEventSynchronize((hipEvent_t)e.done);
    (void)hipEventDestroy((hipEvent_t)e.done);
  }
  if (e.exec) (void)hipGraphExecDestroy((hipGraphExec_t)e.exec);
  e = tn_plan_s::GraphEntry{};
}

// Drop the cached graphs of one mode (-1: every mode).
static void drop_graphs(tn_plan_s* p, int mode) {
  for (auto it = p->graphs.begin(); it != p->graphs.end();) {
    if (mode < 0 || it->first.first == mode) {
      destroy_graph(it->second);
      it = p->graphs.erase(it);
    } else {
      ++it;
    }
  }
}

static void assign_tiles(tn_plan_s* p, std::vector<Op>& prog);

extern "C" int tn_plan(int32_t n_leaves, const int32_t* rank, const int64_t* leaf_idx, int32_t n_idx,
                       const int64_t* idx_dim, int32_t n_out, const int64_t* out_idx, const int32_t* left,
                       const int32_t* right, int32_t n_sliced, const int64_t* sliced_idx,
                       const tn_options* opt, tn_plan_t* plan) {
  g_err.clear();
  if (!plan) return set_err(TN_E_INVALID, "plan is null");
  *plan = nullptr;
  if (n_leaves < 1 || !rank || (n_idx > 0 && !idx_dim) || n_idx < 0 || n_out < 0 || n_sliced < 0)
    return set_err(TN_E_INVALID, "null or empty network");
  if (n_leaves > 1 && (!left || !right)) return set_err(TN_E_INVALID, "tree is null");
  if ((n_out > 0 && !out_idx) || (n_sliced > 0 && !sliced_idx)) return set_err(TN_E_INVALID, "null index list");
  int64_t tot = 0;
  for (int v = 0; v < n_leaves; v++) {
    if (rank[v] < 0 || rank[v] > 64) return set_err(TN_E_INVALID, "leaf rank out of range");
    tot += rank[v];
  }
  if (tot > 0 && !leaf_idx) return set_err(TN_E_INVALID, "leaf index list is null");
  tn_plan_s* p = new tn_plan_s();
  p->n_leaves = n_leaves;
  p->n_idx = n_idx;
  p->n_out = n_out;
  p->n_sliced = n_sliced;
  p->rank.assign(rank, rank + n_leaves);
  p->leaf_idx.assign(leaf_idx, leaf_idx + tot);
  p->idx_dim.assign(idx_dim, idx_dim + n_idx);
  if (n_out) p->out_idx.assign(out_idx, out_idx + n_out);
  if (n_sliced) p->sliced.assign(sliced_idx, sliced_idx + n_sliced);
  if (n_leaves > 1) {
    p->left.assign(left, left + n_leaves - 1);
    p->right.assign(right, right + n_leaves - 1);
  }
  if (opt) p->opt = *opt;
  p->prec = p->opt.prec;
  if (p->prec < TN_C64_4M || p->prec > TN_C128) {
    delete p;
    return set_err(TN_E_INVALID, "unknown precision");
  }
  p->elem_bytes = p->prec == TN_C128 ? 16 : 8;
  std::string err;
  int rc = build_plan(p, err);
  if (rc) {
    delete p;
    return set_err(rc, err);
  }
  assign_tiles(p, p->fwd);
  *plan = p;
  return TN_OK;
}

extern "C" int tn_plan_info(tn_plan_t p, int32_t* W, int32_t* W_s, double* log2_C, double* flops_8C_per_slice,
                            int64_t* d_sliced, uint64_t* workspace_bytes) {
  if (!p) return set_err(TN_E_INVALID, "plan is null");
  PlanLock lk(p->mu);
  if (W) *W = p->W;
  if (W_s) *W_s = p->W_s;
  if (log2_C) *log2_C = p->log2_C;
  if (flops_8C_per_slice) *flops_8C_per_slice = p->flops_per_slice;
  if (d_sliced) *d_sliced = p->d_sliced;
  if (workspace_bytes) *workspace_bytes = p->workspace_bytes;
  return TN_OK;
}

// Tile variant of every matrix-core contraction of a program: the pinned
// variant where it applies, else the autotuned one of its shape, else the
// direct-to-LDS variant where the operands allow it (4M at three waves per
// SIMD, 3M with 64 x 64 waves, BF16x3 on pre-split operands 256 x 128), else
// the register-staged 128 x 128 tile.
static std::array<int, 6> tile_key(const GemmOp& g, int prec) {
  return {g.n_h, g.n_m, g.n_n, g.n_k, g.k_split_bits, gemm_tile_ok(g, 7, prec) ? 1 : 0};
}

static int default_tile(const GemmOp& g, int prec) {
  if (prec == TN_C64_4M && gemm_tile_ok(g, 9, prec)) return 9;
  if (prec == TN_C64_3M && gemm_tile_ok(g, 7, prec)) return 7;
  if (g.ab_split && gemm_tile_ok(g, kSplitTile + 1, prec)) return kSplitTile + 1;
  return g.ab_split ? kSplitTile : 0;
}

static void assign_tiles(tn_plan_s* p, std::vector<Op>& prog) {
  for (Op& op : prog) {
    if (op.kind != OpKind::Gemm) continue;
    GemmOp& g = op.gemm;
    int t = default_tile(g, p->prec);
    auto it = p->tile_choice.find(tile_key(g, p->prec));
    if (p->pinned_tile >= 0 && gemm_tile_ok(g, p->pinned_tile, p->prec)) t = p->pinned_tile;
    else if (it != p->tile_choice.end()) t = it->second;
    g.tile = gemm_tile_ok(g, t, p->prec) ? t : (g.ab_split ? kSplitTile : 0);
  }
}

static int ensure_backward(tn_plan_s* p, int32_t n_wrt, const int32_t* wrt) {
  if (n_wrt < 0 || (n_wrt > 0 && !wrt)) return set_err(TN_E_INVALID, "null wrt list");
  std::vector<int32_t> w(wrt, wrt + n_wrt);
  if (p->bwd_built && w == p->bwd_wrt) return TN_OK;
  std::string err;
  int rc = build_backward(p, w, err);
  if (rc) return set_err(rc, err);
  assign_tiles(p, p->bwd);
  // the cached backward graphs belong to the previous wrt set
  drop_graphs(p, 2);
  return TN_OK;
}

extern "C" int tn_plan_backward_info(tn_plan_t p, int32_t n_wrt, const int32_t* wrt, uint64_t* workspace_bytes,
                                     double* flops_per_slice) {
  if (!p) return set_err(TN_E_INVALID, "plan is null");
  PlanLock lk(p->mu);
  int rc = ensure_backward(p, n_wrt, wrt);
  if (rc) return rc;
  if (workspace_bytes) *workspace_bytes = p->bwd_workspace_bytes;
  if (flops_per_slice) *flops_per_slice = p->bwd_flops_per_slice;
  return TN_OK;
}

extern "C" int tn_plan_num_nodes(tn_plan_t p, int32_t* n) {
  if (!p || !n) return set_err(TN_E_INVALID, "null pointer");
  PlanLock lk(p->mu);
  *n = (int32_t)p->nodes.size();
  return TN_OK;
}

extern "C" int tn_plan_node_info(tn_plan_t p, int32_t k, int32_t* kernel_class, int32_t* logH, int32_t* logM,
                                 int32_t* logN, int32_t* logK, double* flops, double* bytes) {
  if (!p) return set_err(TN_E_INVALID, "plan is null");
  PlanLock lk(p->mu);
  if (k < 0 || k >= (int32_t)p->nodes.size()) return set_err(TN_E_INVALID, "node out of range");
  const NodeInfo& ni = p->nodes[k];
  if (kernel_class) *kernel_class = ni.kclass;
  if (logH) *logH = (int32_t)ni.H.size();
  if (logM) *logM = (int32_t)ni.M.size();
  if (logN) *logN = (int32_t)ni.N.size();
  if (logK) *logK = (int32_t)ni.K.size();
  if (flops) *flops = ni.flops;
  if (bytes) *bytes = ni.bytes;
  return TN_OK;
}

// Kernel of a forward op, for reporting: symbol-like name and tile variant.
static const char* op_kernel_name(const tn_plan_s* p, const Op& op, int* tile) {
  *tile = -1;
  switch (op.kind) {
    case OpKind::Row: {
      if (op.row.k_split_bits >= 0) return "splitk_kernel";
      RowOp r = op.row;
      prepare_row(r);
      return row_stream_ok(r) ? "row_stream_kernel" : "row_kernel";
    }
    case OpKind::RowReduce: return "reduce_kernel";
    case OpKind::Gemm:
      if (gemm_smallk_ok(op.gemm)) return smallk_kernel_name(op.gemm, p->prec);
      *tile = p->prec == TN_C128 ? kValuTile : op.gemm.tile;
      return gemm_kernel_name(op.gemm, p->prec);
    case OpKind::Accum: return "accum_kernel";
    case OpKind::Permute: return "permute_kernel";
    case OpKind::Counter: return "counter_kernel";
    case OpKind::Split: return "split_kernel";
    default: return "";
  }
}

extern "C" int tn_plan_node_kernel(tn_plan_t p, int32_t k, int32_t* tile, char* name, int32_t name_cap) {
  if (!p) return set_err(TN_E_INVALID, "plan is null");
  PlanLock lk(p->mu);
  if (k < 0 || k >= (int32_t)p->nodes.size()) return set_err(TN_E_INVALID, "node out of range");
  const int node = p->n_leaves + k;
  const Op* main = nullptr;
  for (const Op& op : p->fwd)
    if (op.node == node && (op.kind == OpKind::Gemm || op.kind == OpKind::Row)) { main = &op; break; }
  if (!main) return set_err(TN_E_INVALID, "node has no contraction op");
  int t = -1;
  const char* nm = op_kernel_name(p, *main, &t);
  if (tile) *tile = t;
  if (name && name_cap > 0) {
    std::strncpy(name, nm, (size_t)name_cap - 1);
    name[name_cap - 1] = 0;
  }
  return TN_OK;
}

extern "C" int tn_plan_backward_kernels(tn_plan_t p, int32_t n_wrt, const int32_t* wrt, int32_t cap, int32_t* n,
                                        char* names, int32_t name_cap) {
  if (!p || !n) return set_err(TN_E_INVALID, "null pointer");
  PlanLock lk(p->mu);
  int rc = ensure_backward(p, n_wrt, wrt);
  if (rc) return rc;
  int32_t i = 0;
  for (const Op& op : p->bwd) {
    if (op.kind != OpKind::Gemm && op.kind != OpKind::Row) continue;
    if (names && name_cap > 0 && i < cap) {
      int t = -1;
      char* dst = names + (size_t)i * (size_t)name_cap;
      std::strncpy(dst, op_kernel_name(p, op, &t), (size_t)name_cap - 1);
      dst[name_cap - 1] = 0;
    }
    i++;
  }
  *n = i;
  return TN_OK;
}

extern "C" int tn_plan_tune_trials(tn_plan_t p, int32_t cap, int32_t* n, int32_t* keys, int32_t* tiles,
                                   int32_t* k_bits, float* ms) {
  if (!p || !n) return set_err(TN_E_INVALID, "null pointer");
  PlanLock lk(p->mu);
  *n = (int32_t)p->tune_trials.size();
  for (int32_t i = 0; i < *n && i < cap; i++) {
    const auto& t = p->tune_trials[(size_t)i];
    if (keys)
      for (int j = 0; j < 6; j++) keys[6 * i + j] = t.key[(size_t)j];
    if (tiles) tiles[i] = t.tile;
    if (k_bits) k_bits[i] = t.k_bits;
    if (ms) ms[i] = t.ms;
  }
  return TN_OK;
}

// ------------------------------------------------------------------ launching

Ctx tn::make_ctx(const tn_plan_s* p, void* ws, uint64_t arena_stride) {
  Ctx c;
  std::memset(&c, 0, sizeof c);
  c.ws = reinterpret_cast<uint64_t>(ws);
  c.arena_stride = arena_stride;
  c.ptrtab_off = p->ptrtab_off;
  c.sid_off = p->sid_off;
  c.counter_off = p->counter_off;
  c.arena_off = p->arena_off;
  c.n_batch = p->n_batch;
  c.elem_bytes = p->elem_bytes;
  return c;
}

hipError_t tn::launch_op(int prec, const Ctx& ctx, const Op& op, hipStream_t s) {
  const bool f64 = prec == TN_C128;
  switch (op.kind) {
    case OpKind::Row: return launch_row(ctx, op.row, f64, s);
    case OpKind::RowReduce: return launch_reduce(ctx, op.row, f64, s);
    case OpKind::Gemm:
      return gemm_smallk_ok(op.gemm) ? launch_gemm_smallk(ctx, op.gemm, prec, s) : launch_gemm(ctx, op.gemm, prec, s);
    case OpKind::Accum: return launch_accum(ctx, op.accum, f64, s);
    case OpKind::Permute: return launch_permute(ctx, op.perm, f64, s);
    case OpKind::Fill: return hipSuccess;
    case OpKind::Counter: return launch_counter(ctx, 1, 1, s);
    case OpKind::Split: return launch_split(ctx, op.split, s);
  }
  return hipErrorInvalidValue;
}

static hipError_t launch_op(const tn_plan_s* p, const Ctx& ctx, const Op& op, hipStream_t s) {
  return tn::launch_op(p->prec, ctx, op, s);
}

// Tail of the forward program: what happens to each in-flight slice's root.
// mode 0: copy to the output slot in the storage type (unsliced contraction)
// mode 1: FP64 accumulation into the complex128 output slot
std::vector<Op> tn::forward_program(const tn_plan_s* p, int mode) {
  std::vector<Op> prog = p->fwd;
  const int n = p->n_leaves;
  Ref root;
  std::memset(&root, 0, sizeof root);
  std::vector<int8_t> src_pos;
  int nb = 0;
  if (n > 1) {
    root.kind = 1;
    root.off = p->root_off;
    nb = (int)p->kept_bits[2 * n - 2].size();
    for (int i = 0; i < nb; i++) src_pos.push_back((int8_t)i);
  } else {
    // a single leaf: its axes are all outputs; read it in output order
    root.kind = 0;
    root.slot = 0;
    const Layout& L = p->layout[0];
    std::vector<int> outbits;
    for (int i = p->n_out - 1; i >= 0; i--) {
      int64_t e = p->out_idx[i];
      for (int s = 0; s < p->bit_count[e]; s++) outbits.push_back(p->bit_base[e] + s);
    }
    nb = (int)outbits.size();
    for (int b : outbits) src_pos.push_back((int8_t)L.pos_of(b));
  }
  // Unsliced contraction: the root's ops write the output buffer directly
  // (the root layout is already the output order and the storage type).
  if (mode == 0 && n > 1) {
    const int root_node = 2 * n - 2;
    bool direct = true;
    for (const Op& o : prog) {
      if (o.node != root_node) continue;
      if (o.kind == OpKind::Fill || (o.kind == OpKind::Row && o.row.accumulate) ||
          (o.kind == OpKind::Gemm && o.gemm.accumulate))
        direct = false;
    }
    if (direct) {
      auto redirect = [&](Ref& r) {
        if (r.kind == 1 && r.off == p->root_off) { r.kind = 2; r.slot = p->slot_out; r.off = 0; }
      };
      for (Op& o : prog) {
        if (o.node != root_node) continue;
        if (o.kind == OpKind::Row || o.kind == OpKind::RowReduce) redirect(o.row.c);
        else if (o.kind == OpKind::Gemm) redirect(o.gemm.c);
      }
      Op c;
      c.kind = OpKind::Counter;
      prog.push_back(c);
      return prog;
    }
  }
  Op t;
  std::memset(&t.perm, 0, sizeof t.perm);
  std::memset(&t.accum, 0, sizeof t.accum);
  if (mode == 0 || n == 1) {
    t.kind = OpKind::Permute;
    t.perm.src = root;
    t.perm.dst.kind = 2;
    t.perm.dst.slot = p->slot_out;
    t.perm.n_bits = nb;
    t.perm.src_c128 = p->prec == TN_C128;
    t.perm.dst_c128 = mode == 1 ? 1 : (p->prec == TN_C128);
    t.perm.accumulate = mode == 1 ? 1 : 0;
    t.perm.per_slice_serial = mode == 1 ? 1 : 0;
    for (int i = 0; i < nb; i++) { t.perm.src_pos[i] = src_pos[i]; t.perm.dst_pos[i] = (int8_t)i; }
  } else {
    t.kind = OpKind::Accum;
    t.accum.src = root;
    t.accum.dst.kind = 2;
    t.accum.dst.slot = p->slot_out;
    t.accum.n = int64_t(1) << nb;
  }
  prog.push_back(t);
  Op c;
  c.kind = OpKind::Counter;
  prog.push_back(c);
  return prog;
}

static std::vector<Op> backward_program(const tn_plan_s* p) {
  std::vector<Op> prog = p->bwd;
  Op c;
  c.kind = OpKind::Counter;
  prog.push_back(c);
  return prog;
}

static bool graphs_enabled() {
  const char* e = std::getenv("TN_NO_GRAPH");
  return !(e && e[0] == '1');
}

static hipStream_t capture_stream() {
  static thread_local hipStream_t s = nullptr;
  if (!s) {
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) s = nullptr;
  }
  return s;
}

// Run `prog` n_batches times on stream s: replays of the graph cached for
// (mode, workspace) when graphs are enabled and `use_graph` is set, else
// launch by launch.  Called with the plan's lock held.
static int run_batches(tn_plan_s* p, int mode, const std::vector<Op>& prog, const Ctx& ctx, int64_t n_batches,
                       hipStream_t s, bool use_graph = true) {
  if (n_batches <= 0) return TN_OK;
  if (use_graph && graphs_enabled()) {
    auto key = std::make_pair(mode, ctx.ws);
    auto it = p->graphs.find(key);
    if (it == p->graphs.end()) {
      if (p->graphs.size() >= tn_plan_s::kMaxGraphs) {
        auto lru = p->graphs.begin();
        for (auto j = p->graphs.begin(); j != p->graphs.end(); ++j)
          if (j->second.last_use < lru->second.last_use) lru = j;
        destroy_graph(lru->second);
        p->graphs.erase(lru);
      }
      hipStream_t cs = capture_stream();
      if (!cs) return set_err(TN_E_DEVICE, "could not create the capture stream");
      HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
      for (const Op& op : prog) {
        hipError_t e = launch_op(p, ctx, op, cs);
        if (e != hipSuccess) {
          hipGraph_t g = nullptr;
          (void)hipStreamEndCapture(cs, &g);
          if (g) (void)hipGraphDestroy(g);
          return set_err(TN_E_DEVICE, std::string("kernel launch during capture: ") + hipGetErrorString(e));
        }
      }
      hipGraph_t graph = nullptr;
      HIP_TRY(hipStreamEndCapture(cs, &graph));
      hipGraphExec_t exec = nullptr;
      hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (e != hipSuccess) return set_err(TN_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
      hipEvent_t done = nullptr;
      e = hipEventCreateWithFlags(&done, hipEventDisableTiming);
      if (e != hipSuccess) {
        (void)hipGraphExecDestroy(exec);
        return set_err(TN_E_DEVICE, std::string("hipEventCreateWithFlags: ") + hipGetErrorString(e));
      }
      tn_plan_s::GraphEntry entry;
      entry.exec = exec;
      entry.done = done;
      it = p->graphs.emplace(key, entry).first;
    }
    it->second.last_use = ++p->graph_clock;
    hipGraphExec_t exec = (hipGraphExec_t)it->second.exec;
    for (int64_t b = 0; b < n_batches; b++) HIP_TRY(hipGraphLaunch(exec, s));
    HIP_TRY(hipEventRecord((hipEvent_t)it->second.done, s));
    return TN_OK;
  }
  for (int64_t b = 0; b < n_batches; b++)
    for (const Op& op : prog) {
      hipError_t e = launch_op(p, ctx, op, s);
      if (e != hipSuccess) return set_err(TN_E_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
    }
  return TN_OK;
}

// Upload the pointer table and the (padded) slice ids; reset the batch counter.
static int upload(tn_plan_s* p, void* ws, const void* const* leaves, void* out, const void* gout,
                  void* const* grads, int n_grads, const std::vector<int64_t>& ids, hipStream_t s) {
  std::vector<uint64_t> tab(p->n_slots, 0);
  for (int v = 0; v < p->n_leaves; v++) tab[v] = reinterpret_cast<uint64_t>(leaves[v]);
  tab[p->slot_out] = reinterpret_cast<uint64_t>(out);
  tab[p->slot_gout] = reinterpret_cast<uint64_t>(gout);
  for (int i = 0; i < n_grads; i++) tab[p->slot_grad0 + i] = reinterpret_cast<uint64_t>(grads[i]);
  char* w = static_cast<char*>(ws);
  HIP_TRY(hipMemcpyAsync(w + p->ptrtab_off, tab.data(), tab.size() * 8, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(w + p->sid_off, ids.data(), ids.size() * 8, hipMemcpyHostToDevice, s));
  Ctx ctx = make_ctx(p, ws, 0);
  HIP_TRY(launch_counter(ctx, 0, 0, s));
  return TN_OK;
}

static int check_leaves(const tn_plan_s* p, const void* const* leaves) {
  if (!leaves) return set_err(TN_E_INVALID, "leaves is null");
  for (int v = 0; v < p->n_leaves; v++)
    if (!leaves[v]) return set_err(TN_E_INVALID, "leaf " + std::to_string(v) + " is null");
  return TN_OK;
}

static int make_ids(const tn_plan_s* p, int64_t n_ids, const int64_t* slice_ids, std::vector<int64_t>& ids) {
  if (slice_ids == nullptr) {
    if (p->d_sliced > p->max_ids)
      return set_err(TN_E_INVALID, "too many slices for one call; pass slice_ids in chunks");
    ids.resize(p->d_sliced);
    for (int64_t i = 0; i < p->d_sliced; i++) ids[i] = i;
  } else {
    if (n_ids < 0) return set_err(TN_E_INVALID, "negative n_ids");
    if (n_ids > p->max_ids) return set_err(TN_E_INVALID, "too many slice ids for one call (max " + std::to_string(p->max_ids) + ")");
    ids.assign(slice_ids, slice_ids + n_ids);
    for (int64_t x : ids)
      if (x < 0 || x >= p->d_sliced) return set_err(TN_E_INVALID, "slice id " + std::to_string(x) + " out of range");
  }
  const int64_t nb = p->n_batch;
  const int64_t padded = (int64_t)((ids.size() + nb - 1) / nb * nb);
  ids.resize(padded, -1);
  return TN_OK;
}

// Sliced contraction into out_c128 over `workspace`; with use_graph false
// every op is launched directly (no graph is captured or instantiated).
// Called with the plan's lock held.
static int contract_sliced_impl(tn_plan_s* p, const void* const* leaves, int64_t n_ids, const int64_t* slice_ids,
                                void* out_c128, void* workspace, uint64_t workspace_bytes, hipStream_t s,
                                bool use_graph) {
  if (!out_c128) return set_err(TN_E_INVALID, "output is null");
  int rc = check_leaves(p, leaves);
  if (rc) return rc;
  if (!workspace || workspace_bytes < p->workspace_bytes)
    return set_err(TN_E_WORKSPACE, "workspace of " + std::to_string(p->workspace_bytes) + " bytes required");
  std::vector<int64_t> ids;
  rc = make_ids(p, n_ids, slice_ids, ids);
  if (rc) return rc;
  rc = upload(p, workspace, leaves, out_c128, nullptr, nullptr, 0, ids, s);
  if (rc) return rc;
  const int64_t out_elems = int64_t(1) << (p->n_leaves > 1 ? p->kept_bits[2 * p->n_leaves - 2].size()
                                                           : p->layout[0].bits.size());
  HIP_TRY(launch_fill(reinterpret_cast<uint64_t>(out_c128), (uint64_t)out_elems * 16, s));
  Ctx ctx = make_ctx(p, workspace, p->arena_bytes);
  return run_batches(p, 1, forward_program(p, 1), ctx, (int64_t)ids.size() / p->n_batch, s, use_graph);
}

extern "C" int tn_contract_sliced(tn_plan_t p, const void* const* leaves, int64_t n_ids, const int64_t* slice_ids,
                                  void* out_c128, void* workspace, uint64_t workspace_bytes, void* stream) {
  g_err.clear();
  if (!p) return set_err(TN_E_INVALID, "plan is null");
  PlanLock lk(p->mu);
  return contract_sliced_impl(p, leaves, n_ids, slice_ids, out_c128, workspace, workspace_bytes,
                              static_cast<hipStream_t>(stream), true);
}

// ------------------------------------------------- allocation-free variant

// Workspace of tn_contract_sliced_noalloc: one array per device, loaded with
// the library's code object and held until the process ends.  In host code
// `scratch` names a host-side stand-in, so host code never passes it to a
// kernel or a copy; it uses the device address hipGetSymbolAddress returns
// for the current device, looked up once per device.
constexpr uint64_t kStaticScratchBytes = uint64_t(64) << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

static int static_scratch(void** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return set_err(TN_E_DEVICE, "device ordinal out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return set_err(TN_E_DEVICE, "hipGetSymbolAddress gave a null scratch address");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return TN_OK;
}

extern "C" int tn_contract_sliced_noalloc(tn_plan_t p, const void* const* leaves, int64_t n_ids,
                                          const int64_t* slice_ids, void* out_c128, void* stream) {
  g_err.clear();
  if (!p) return set_err(TN_E_INVALID, "plan is null");
  PlanLock lk(p->mu);
  if (p->workspace_bytes > kStaticScratchBytes)
    return set_err(TN_E_WORKSPACE, "plan needs a workspace of " + std::to_string(p->workspace_bytes) +
                                       " bytes; the static scratch holds " + std::to_string(kStaticScratchBytes));
  void* ws = nullptr;
  int rc = static_scratch(&ws);
  if (rc) return rc;
  return contract_sliced_impl(p, leaves, n_ids, slice_ids, out_c128, ws, kStaticScratchBytes,
                              static_cast<hipStream_t>(stream), false);
}

static int op_kind_code(const Op& op) {
  switch (op.kind) {
    case OpKind::Row: return op.row.k_split_bits >= 0 ? 1 : 0;
    case OpKind::RowReduce: return 2;
    case OpKind::Gemm: return 3;
    case OpKind::Accum: return 4;
    case OpKind::Permute: return 5;
    case OpKind::Counter: return 6;
    case OpKind::Split: return 7;
    default: return -1;
  }
}

extern "C" int tn_contract_sliced_timed(tn_plan_t p, const void* const* leaves, int64_t n_ids,
                                        const int64_t* slice_ids, void* out_c128, void* workspace,
                                        uint64_t workspace_bytes, void* stream, int32_t cap, float* op_ms,
                                        int32_t* op_kind, int32_t* op_node, double* op_flops, double* op_bytes,
                                        int32_t* n_ops) {
  g_err.clear();
  if (!p) return set_err(TN_E_INVALID, "plan is null");
  PlanLock lk(p->mu);
  if (!out_c128) return set_err(TN_E_INVALID, "output is null");
  int rc = check_leaves(p, leaves);
  if (rc) return rc;
  if (!workspace || workspace_bytes < p->workspace_bytes)
    return set_err(TN_E_WORKSPACE, "workspace of " + std::to_string(p->workspace_bytes) + " bytes required");
  std::vector<int64_t> ids;
  rc = make_ids(p, n_ids, slice_ids, ids);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  rc = upload(p, workspace, leaves, out_c128, nullptr, nullptr, 0, ids, s);
  if (rc) return rc;
  const int64_t out_elems = int64_t(1) << (p->n_leaves > 1 ? p->kept_bits[2 * p->n_leaves - 2].size()
                                                           : p->layout[0].bits.size());
  HIP_TRY(launch_fill(reinterpret_cast<uint64_t>(out_c128), (uint64_t)out_elems * 16, s));
  Ctx ctx = make_ctx(p, workspace, p->arena_bytes);
  std::vector<Op> prog = forward_program(p, 1);
  const size_t nop = prog.size();
  const int64_t nbatches = (int64_t)ids.size() / p->n_batch;
  std::vector<hipEvent_t> ev(nop + 1, nullptr);
  for (auto& e : ev) HIP_TRY(hipEventCreate(&e));
  std::vector<double> acc(nop, 0.0);
  int result = TN_OK;
  for (int64_t b = 0; b < nbatches && result == TN_OK; b++) {
    if (hipEventRecord(ev[0], s) != hipSuccess) { result = set_err(TN_E_DEVICE, "hipEventRecord"); break; }
    for (size_t i = 0; i < nop; i++) {
      hipError_t e = launch_op(p, ctx, prog[i], s);
      if (e == hipSuccess) e = hipEventRecord(ev[i + 1], s);
      if (e != hipSuccess) { result = set_err(TN_E_DEVICE, std::string("timed launch: ") + hipGetErrorString(e)); break; }
    }
    if (result != TN_OK) break;
    if (hipEventSynchronize(ev[nop]) != hipSuccess) { result = set_err(TN_E_DEVICE, "hipEventSynchronize"); break; }
    for (size_t i = 0; i < nop; i++) {
      float ms = 0;
      if (hipEventElapsedTime(&ms, ev[i], ev[i + 1]) == hipSuccess) acc[i] += ms;
    }
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  if (result != TN_OK) return result;
  if (n_ops) *n_ops = (int32_t)nop;
  for (size_t i = 0; i < nop && (int32_t)i < cap; i++) {
    if (op_ms) op_ms[i] = (float)acc[i];
    if (op_kind) op_kind[i] = op_kind_code(prog[i]);
    if (op_node) op_node[i] = prog[i].node;
    if (op_flops) op_flops[i] = prog[i].flops;
    if (op_bytes) op_bytes[i] = prog[i].bytes;
  }
  return TN_OK;
}

extern "C" int tn_contract(tn_plan_t p, const void* const* leaves, void* out, void* workspace,
                           uint64_t workspace_bytes, void* stream) {
  g_err.clear();
  if (!p) return set_err(TN_E_INVALID, "plan is null");
  PlanLock lk(p->mu);
  if (p->n_sliced > 0) return set_err(TN_E_INVALID, "plan has sliced indices; use tn_contract_sliced");
  if (!out) return set_err(TN_E_INVALID, "output is null");
  int rc = check_leaves(p, leaves);
  if (rc) return rc;
  if (!workspace || workspace_bytes < p->workspace_bytes)
    return set_err(TN_E_WORKSPACE, "workspace of " + std::to_string(p->workspace_bytes) + " bytes required");
  std::vector<int64_t> ids;
  rc = make_ids(p, 1, std::vector<int64_t>{0}.data(), ids);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  rc = upload(p, workspace, leaves, out, nullptr, nullptr, 0, ids, s);
  if (rc) return rc;
  Ctx ctx = make_ctx(p, workspace, p->arena_bytes);
  return run_batches(p, 0, forward_program(p, 0), ctx, (int64_t)ids.size() / p->n_batch, s);
}

extern "C" int tn_contract_backward(tn_plan_t p, const void* const* leaves, const void* grad_out_c128,
                                    int32_t n_wrt, const int32_t* wrt_leaf, void* const* grads, int64_t n_ids,
                                    const int64_t* slice_ids, void* workspace, uint64_t workspace_bytes,
                                    void* stream) {
  g_err.clear();
  if (!p) return set_err(TN_E_INVALID, "plan is null");
  PlanLock lk(p->mu);
  if (!grad_out_c128) return set_err(TN_E_INVALID, "grad_out is null");
  if (n_wrt > 0 && !grads) return set_err(TN_E_INVALID, "grads is null");
  int rc = check_leaves(p, leaves);
  if (rc) return rc;
  for (int i = 0; i < n_wrt; i++)
    if (!grads[i]) return set_err(TN_E_INVALID, "grads[" + std::to_string(i) + "] is null");
  rc = ensure_backward(p, n_wrt, wrt_leaf);
  if (rc) return rc;
  if (!workspace || workspace_bytes < p->bwd_workspace_bytes)
    return set_err(TN_E_WORKSPACE, "workspace of " + std::to_string(p->bwd_workspace_bytes) + " bytes required");
  std::vector<int64_t> ids;
  rc = make_ids(p, n_ids, slice_ids, ids);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  rc = upload(p, workspace, leaves, nullptr, grad_out_c128, grads, n_wrt, ids, s);
  if (rc) return rc;
  for (int i = 0; i < n_wrt; i++) {
    int v = wrt_leaf[i];
    int64_t elems = 1;
    for (int a = 0; a < p->rank[v]; a++) elems *= p->idx_dim[p->leaf_idx[p->leaf_off[v] + a]];
    HIP_TRY(launch_fill(reinterpret_cast<uint64_t>(grads[i]), (uint64_t)elems * p->elem_bytes, s));
  }
  if (n_wrt == 0) return TN_OK;
  Ctx ctx = make_ctx(p, workspace, p->bwd_arena_bytes);
  return run_batches(p, 2, backward_program(p), ctx, (int64_t)ids.size() / p->n_batch, s);
}

// ------------------------------------------------------------------ autotuning

// For every distinct matrix-core contraction shape, time each tile variant on
// the plan's own operands (zero-filled arena) and keep the fastest.  Each
// candidate runs once to warm up with the summed range cut to at most 2^12
// values per split, then in three separately timed launches, taken
// round-robin over the candidates, at the full summed range when all of
// them fit a budget of about 6 s, else at the cut range; the median decides.
extern "C" int tn_plan_tune(tn_plan_t p, void* workspace, uint64_t workspace_bytes, void* stream) {
  g_err.clear();
  if (!p) return set_err(TN_E_INVALID, "plan is null");
  PlanLock lk(p->mu);
  if (!workspace || workspace_bytes < p->workspace_bytes)
    return set_err(TN_E_WORKSPACE, "workspace of " + std::to_string(p->workspace_bytes) + " bytes required");
  if (p->prec == TN_C128) return TN_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::vector<int64_t> ids((size_t)std::max<int64_t>(p->n_batch, 1), -1);
  ids[0] = 0;   // one live slice
  std::vector<const void*> dummy(p->n_leaves, workspace);
  int rc = upload(p, workspace, dummy.data(), workspace, nullptr, nullptr, 0, ids, s);
  if (rc) return rc;
  HIP_TRY(launch_fill(reinterpret_cast<uint64_t>(workspace) + p->arena_off, p->arena_bytes, s));
  Ctx ctx = make_ctx(p, workspace, p->arena_bytes);
  constexpr int kReps = 3;
  constexpr double kTuneBudgetMs = 6000;   // trials of one shape at the full summed range
  hipEvent_t ev[kReps + 1] = {};
  for (auto& e : ev) HIP_TRY(hipEventCreate(&e));
  std::map<std::array<int, 6>, int> best;
  std::vector<tn_plan_s::TuneTrial> trials;
  int result = TN_OK;
  const bool verbose = std::getenv("TN_TUNE_VERBOSE") != nullptr;
  for (Op& op : p->fwd) {
    if (result != TN_OK) break;
    if (op.kind != OpKind::Gemm) continue;
    GemmOp& g = op.gemm;
    if (g.a.kind != 1 || g.b.kind != 1) continue;   // leaf operands: keep the default
    if (gemm_smallk_ok(g)) continue;                // few summed values: no tile to choose
    const std::array<int, 6> key = tile_key(g, p->prec);
    if (best.count(key)) continue;
    // candidates are timed round-robin, one launch each per round, so that a
    // drift of the clock (it falls under sustained matrix-core load) affects
    // every candidate alike; the median of three rounds decides
    std::vector<int> cand;
    for (int t = 0; t < kNumGemmTiles; t++)
      if (t != kValuTile && gemm_tile_ok(g, t, p->prec)) cand.push_back(t);
    std::vector<std::array<float, kReps>> t_ms(cand.size());
    hipError_t e = hipSuccess;
    // warm-up, each candidate once with the summed range cut to 2^12 per
    // split, timed: if every trial at the full range fits the budget, the
    // trials run at the full range (under sustained load the clock settles
    // lower than in a short launch, and a kernel's rank can change with it)
    const int cut_k = std::min(g.n_k, 12 + std::max(0, g.k_split_bits));
    float warm_max = 0;
    for (size_t c = 0; c < cand.size() && e == hipSuccess; c++) {
      GemmOp trial = g;
      trial.tile = cand[c];
      trial.n_k = cut_k;
      float ms = 0;
      e = hipEventRecord(ev[0], s);
      if (e == hipSuccess) e = launch_gemm(ctx, trial, p->prec, s);
      if (e == hipSuccess) e = hipEventRecord(ev[1], s);
      if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
      warm_max = std::max(warm_max, ms);
    }
    const double full_est = (double)warm_max * std::exp2((double)(g.n_k - cut_k)) * (double)cand.size() * kReps;
    const int trial_k = full_est <= kTuneBudgetMs ? g.n_k : cut_k;
    for (int r = 0; r < kReps && e == hipSuccess; r++)
      for (size_t c = 0; c < cand.size() && e == hipSuccess; c++) {
        GemmOp trial = g;
        trial.tile = cand[c];
        trial.n_k = trial_k;
        e = hipEventRecord(ev[0], s);
        if (e == hipSuccess) e = launch_gemm(ctx, trial, p->prec, s);
        if (e == hipSuccess) e = hipEventRecord(ev[1], s);
        if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
        if (e == hipSuccess) e = hipEventElapsedTime(&t_ms[c][(size_t)r], ev[0], ev[1]);
      }
    if (e != hipSuccess) {
      result = set_err(TN_E_DEVICE, std::string("autotune trial: ") + hipGetErrorString(e));
      break;
    }
    float best_ms = 1e30f, default_ms = 1e30f;
    int best_tile = 0;
    const int dflt = default_tile(g, p->prec);
    for (size_t c = 0; c < cand.size(); c++) {
      std::array<float, kReps> v = t_ms[c];
      std::sort(v.begin(), v.end());
      const float med = v[kReps / 2];
      tn_plan_s::TuneTrial tr;
      tr.key = key;
      tr.tile = cand[c];
      tr.k_bits = trial_k;
      tr.ms = med;
      trials.push_back(tr);
      if (verbose)
        fprintf(stderr, "tune (h,m,n,k)=(%d,%d,%d,%d) tile %d: median %.3f ms for k=2^%d\n", g.n_h, g.n_m, g.n_n,
                g.n_k, cand[c], med, tr.k_bits);
      if (med < best_ms) { best_ms = med; best_tile = cand[c]; }
      if (cand[c] == dflt) default_ms = med;
    }
    // the default variant unless another one is faster by more than 1 %: a
    // choice between near-equal variants would follow the timing noise of
    // one run, and repeated runs should execute the same kernels
    if (default_ms <= best_ms * 1.01f) best_tile = dflt;
    best[key] = best_tile;
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  if (result != TN_OK) return result;
  p->tile_choice = best;
  p->tune_trials = trials;
  p->pinned_tile = -1;
  assign_tiles(p, p->fwd);
  if (p->bwd_built) assign_tiles(p, p->bwd);
  drop_graphs(p, -1);
  p->tuned = true;
  return TN_OK;
}

extern "C" int tn_plan_set_tile(tn_plan_t p, int32_t tile, int32_t* n_set) {
  if (!p) return set_err(TN_E_INVALID, "plan is null");
  PlanLock lk(p->mu);
  int bm, bn;
  if (gemm_tile_bits(tile, &bm, &bn)) return set_err(TN_E_INVALID, "unknown tile variant");
  int32_t n = 0;
  p->pinned_tile = tile;                 // also for a backward program built later
  for (auto* prog : {&p->fwd, &p->bwd})
    for (Op& op : *prog)
      if (op.kind == OpKind::Gemm && op.gemm.tile != tile && gemm_tile_ok(op.gemm, tile, p->prec)) {
        op.gemm.tile = tile;
        n++;
      }
  if (n) drop_graphs(p, -1);
  if (n_set) *n_set = n;
  return TN_OK;
}

extern "C" void tn_plan_destroy(tn_plan_t p) {
  if (!p) return;
  {
    PlanLock lk(p->mu);
    drop_graphs(p, -1);
  }
  delete p;
}
