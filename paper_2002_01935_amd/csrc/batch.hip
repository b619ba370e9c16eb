// Many independent small networks in one graph launch.
//
// Workloads such as the QAOA energy (Sec. 4.5: one light-cone network per
// edge) or a batch of sampled bitstrings (Sec. 4.7.3) are many small networks
// whose contractions are mostly tiny: gate merges of a few dozen elements.
// Launched one kernel per pairwise contraction, such a network is bound by
// launch latency (about 190 launches per QAOA term).  Here each network's
// forward program (in its own order, so its arena stays valid) is cut into
// segments of tiny contractions separated by the contractions that are
// worth a launch of their own.  Segment L of every network runs in one launch
// of the interpreter kernel, one workgroup per network executing its tiny
// contractions one after another (a workgroup barrier between them); then the
// large contractions that follow segment L in each network are launched with
// the ordinary kernels; then segment L + 1.  The whole sequence is captured
// once per workspace into a HIP graph and replayed by tn_batch_contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "exec.h"
#include "kernels.h"
#include "plan.h"

namespace tn {

#define GMEM __attribute__((address_space(1)))
#define CMEM __attribute__((address_space(4)))
#define TN_WAVE_SYNC() __builtin_amdgcn_wave_barrier()
// A value the same in every lane of the wavefront, made known to the compiler as such.
#define TN_UNIFORM(x) __builtin_amdgcn_readfirstlane(x)

#include "rowops.h"

constexpr int kTinyBits = 16;       // bit-list capacity of a tiny contraction
constexpr int kTinyWorkBits = 16;   // log2 (outputs x summed values) of the largest one
constexpr int kTinyThreads = 256;
// parallel branches of a level's large contractions in the captured graph
// (one per hardware queue a process gets by default)
constexpr int kBranches = 4;

// One tiny pairwise contraction: for each of 2^n_out outputs,
//   C[o] (+)= sum over 2^n_k summed values of opA(A[o, k]) * opB(B[o, k])
// (opX = complex conjugate when conj_x), or C[o] (+)= opA(A[o]) without B.
// Output bit j sits at position oa[j] / ob[j] / oc[j] of A / B / C (-1:
// absent from that operand), summed bit j at ka[j] / kb[j].
struct TinyOp {
  Ref a, b, c;
  int32_t n_out, n_k;
  int32_t has_b, conj_a, conj_b, accumulate;
  int8_t oa[kTinyBits], ob[kTinyBits], oc[kTinyBits];
  int8_t ka[kTinyBits], kb[kTinyBits];
};
static_assert(offsetof(TinyOp, oa) % 4 == 0 && sizeof(TinyOp) % 8 == 0, "TinyOp layout");

__device__ __forceinline__ int tpos(CMEM const int8_t* list, int i) {
  const uint32_t w = reinterpret_cast<CMEM const uint32_t*>(list)[i >> 2];
  return (int8_t)(w >> (8 * (i & 3)));
}

// Offset of value v's bits in an operand (positions < 0: absent).
__device__ __forceinline__ uint32_t tdeposit(uint32_t v, CMEM const int8_t* list, int first, int n) {
  uint32_t off = 0;
  for (int i = 0; i < n; i++) {
    const int p = tpos(list, first + i);
    off |= p >= 0 ? ((v >> i) & 1u) << p : 0u;
  }
  return off;
}

// Copy of a uniform read-only struct (scalar loads, a dword at a time).
template <typename S>
__device__ __forceinline__ S cload(CMEM const S* p) {
  static_assert(sizeof(S) % 4 == 0, "dword copy");
  S out;
  CMEM const uint32_t* w = reinterpret_cast<CMEM const uint32_t*>(p);
  uint32_t* o = reinterpret_cast<uint32_t*>(&out);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(S) / 4); i++) o[i] = w[i];
  return out;
}

template <typename V>
__device__ __forceinline__ V conj_if(V v, int c) {
  if (c) v.y = -v.y;
  return v;
}

// Segment `level` of network blockIdx.x: its tiny contractions in program
// order.  An output is summed by 2^g threads (g = min(8 - n_out, n_k) when
// there are fewer than 256 outputs), each over a contiguous run of summed
// values walked with per-carry offset steps, and the 2^g partial sums are
// added in a fixed tree order (results do not depend on scheduling).
template <typename T>
__global__ __launch_bounds__(kTinyThreads) void tiny_kernel(CMEM const Ctx* ctxs, CMEM const TinyOp* ops,
                                                            CMEM const int32_t* seg) {
  using V = typename C2<T>::t;
  const int net = blockIdx.x;
  const int begin = seg[2 * net], end = seg[2 * net + 1];
  if (begin >= end) return;
  const Ctx ctx = cload(ctxs + net);
  const int tid = threadIdx.x;
  __shared__ uint32_t kd[2][kTinyBits];
  __shared__ V red[kTinyThreads];
  for (int i = begin; i < end; i++) {
    CMEM const TinyOp* op = ops + i;
    const int n_out = op->n_out, n_k = op->n_k, has_b = op->has_b;
    const int ca = op->conj_a, cb = op->conj_b, accum = op->accumulate;
    const int g = n_out < 8 ? min(8 - n_out, n_k) : 0;
    const int walk = n_k - g;
    const Ref ra = cload(&op->a), rb = cload(&op->b), rc = cload(&op->c);
    GMEM const V* A = reinterpret_cast<GMEM const V*>(resolve(ctx, ra, 0, 0, sizeof(V)));
    GMEM const V* B = has_b ? reinterpret_cast<GMEM const V*>(resolve(ctx, rb, 0, 0, sizeof(V))) : nullptr;
    GMEM V* C = reinterpret_cast<GMEM V*>(resolve(ctx, rc, 0, 0, sizeof(V)));
    // offset change in A / B when the walk's counter carries into its bit t
    if (tid < walk) {
      uint32_t da = 1u << tpos(op->ka, tid), db = has_b ? 1u << tpos(op->kb, tid) : 0u;
      for (int j = 0; j < tid; j++) {
        da -= 1u << tpos(op->ka, j);
        if (has_b) db -= 1u << tpos(op->kb, j);
      }
      kd[0][tid] = da;
      kd[1][tid] = db;
    }
    __syncthreads();
    const uint32_t n_outputs = 1u << n_out, steps = 1u << walk;
    const uint32_t per_pass = (uint32_t)kTinyThreads >> g;
    for (uint32_t o0 = 0; o0 < n_outputs; o0 += per_pass) {
      const uint32_t o = o0 + ((uint32_t)tid >> g);
      const uint32_t r = (uint32_t)tid & ((1u << g) - 1u);
      const bool active = o < n_outputs && ((uint32_t)tid >> g) < per_pass;
      V acc;
      acc.x = 0;
      acc.y = 0;
      if (active) {
        uint32_t xa = tdeposit(o, op->oa, 0, n_out) + tdeposit(r, op->ka, walk, g);
        uint32_t xb = has_b ? tdeposit(o, op->ob, 0, n_out) + tdeposit(r, op->kb, walk, g) : 0u;
        for (uint32_t s = 0; s < steps; s++) {
          const V a = conj_if(ld(A + xa), ca);
          if (has_b) {
            const V b = conj_if(ld(B + xb), cb);
            acc = cfma(acc, a, b);
          } else {
            acc.x += a.x;
            acc.y += a.y;
          }
          if (s + 1 < steps) {
            const int t = __builtin_ctz(~s);
            xa += kd[0][t];
            xb += kd[1][t];
          }
        }
      }
      if (g > 0) {
        red[tid] = acc;
        __syncthreads();
        for (int w = 1 << (g - 1); w >= 1; w >>= 1) {
          if ((int)r < w) {
            V u = red[tid], v = red[tid + w];
            u.x += v.x;
            u.y += v.y;
            red[tid] = u;
          }
          __syncthreads();
        }
        acc = red[tid];
      }
      if (active && r == 0) {
        GMEM V* dst = C + tdeposit(o, op->oc, 0, n_out);
        if (accum) {
          const V p = ld(dst);
          acc.x += p.x;
          acc.y += p.y;
        }
        st(dst, acc);
      }
      if (g > 0) __syncthreads();   // red[] is rewritten by the next pass
    }
    __syncthreads();   // this contraction's output is read by the next one
  }
}

// Whether op runs inside the interpreter, and its descriptor if so.
static bool as_tiny(const Op& op, int prec, TinyOp& t) {
  std::memset(&t, 0, sizeof t);
  for (int j = 0; j < kTinyBits; j++) t.oa[j] = t.ob[j] = t.oc[j] = t.ka[j] = t.kb[j] = -1;
  if (op.kind == OpKind::Row) {
    const RowOp& r = op.row;
    if (r.k_split_bits >= 0) return false;
    t.n_out = r.n_rows + r.n_in;
    t.n_k = r.n_k;
    if (t.n_out > kTinyBits || t.n_k > kTinyBits || t.n_out + t.n_k > kTinyWorkBits) return false;
    for (int j = 0; j < r.n_rows; j++) { t.oa[j] = r.row_a[j]; t.ob[j] = r.row_b[j]; t.oc[j] = r.row_c[j]; }
    for (int j = 0; j < r.n_in; j++) { t.ob[r.n_rows + j] = r.in_b[j]; t.oc[r.n_rows + j] = r.in_c[j]; }
    for (int j = 0; j < r.n_k; j++) { t.ka[j] = r.k_a[j]; t.kb[j] = r.k_b[j]; }
    t.a = r.a; t.b = r.b; t.c = r.c;
    t.has_b = 1;
    t.conj_a = r.conj_a; t.conj_b = r.conj_b; t.accumulate = r.accumulate;
    return true;
  }
  if (op.kind == OpKind::Gemm) {
    const GemmOp& g = op.gemm;
    if (g.k_split_bits > 0 || g.ab_split) return false;
    t.n_out = g.n_h + g.n_m + g.n_n;
    t.n_k = g.n_k;
    if (t.n_out > kTinyBits || t.n_k > kTinyBits || t.n_out + t.n_k > kTinyWorkBits) return false;
    int j = 0;
    for (int i = 0; i < g.n_h; i++, j++) { t.oa[j] = g.a_h[i]; t.ob[j] = g.b_h[i]; t.oc[j] = g.c_h[i]; }
    for (int i = 0; i < g.n_m; i++, j++) { t.oa[j] = g.a_m[i]; t.oc[j] = g.c_m[i]; }
    for (int i = 0; i < g.n_n; i++, j++) { t.ob[j] = g.b_n[i]; t.oc[j] = g.c_n[i]; }
    for (int i = 0; i < g.n_k; i++) { t.ka[i] = g.a_k[i]; t.kb[i] = g.b_k[i]; }
    t.a = g.a; t.b = g.b; t.c = g.c;
    t.has_b = 1;
    t.conj_a = g.conj_a; t.conj_b = g.conj_b; t.accumulate = g.accumulate;
    return true;
  }
  if (op.kind == OpKind::Permute) {
    const PermuteOp& pm = op.perm;
    const int c128 = prec == TN_C128;
    if (pm.n_bits > kTinyBits || pm.n_bits > kTinyWorkBits || pm.src_c128 != c128 || pm.dst_c128 != c128 ||
        pm.per_slice_serial)
      return false;
    t.n_out = pm.n_bits;
    t.n_k = 0;
    for (int j = 0; j < pm.n_bits; j++) { t.oa[j] = pm.src_pos[j]; t.oc[j] = pm.dst_pos[j]; }
    t.a = pm.src; t.c = pm.dst;
    t.has_b = 0;
    t.accumulate = pm.accumulate;
    return true;
  }
  return false;
}

}  // namespace tn

using namespace tn;

struct tn_batch_s {
  std::mutex mu;
  int prec = TN_C64_4M;
  int n_nets = 0, n_levels = 0;
  std::vector<int32_t> n_leaves;             // per network
  std::vector<uint64_t> region_off;          // per network: its plan workspace inside the batch workspace
  std::vector<Ctx> ctx_rel;                  // per network, ws relative to the batch workspace base
  std::vector<TinyOp> tiny;                  // ordered by level, then network
  std::vector<int32_t> seg;                  // [level][network] -> begin, end in `tiny`
  std::vector<std::vector<std::vector<Op>>> big;   // [level][network] -> ops launched after the segment
  uint64_t ctx_off = 0, ops_off = 0, seg_off = 0, ptr_off = 0, ws_bytes = 0;
  int ptr_stride = 0;                        // pointer-table slots per network
  int64_t n_launches = 0;
  // prepared workspaces: graph per workspace address, at most kMaxGraphs
  std::map<uint64_t, tn_plan_s::GraphEntry> graphs;
  uint64_t clock = 0;
};

static void batch_drop(tn_plan_s::GraphEntry& e) {
  if (e.done) {
    (void)hipEventSynchronize((hipEvent_t)e.done);
    (void)hipEventDestroy((hipEvent_t)e.done);
  }
  if (e.exec) (void)hipGraphExecDestroy((hipGraphExec_t)e.exec);
  e = tn_plan_s::GraphEntry{};
}

#define BATCH_TRY(expr)                                                                   \
  do {                                                                                    \
    hipError_t _e = (expr);                                                               \
    if (_e != hipSuccess)                                                                 \
      return set_error(TN_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(_e));   \
  } while (0)

extern "C" int tn_batch(int32_t n_plans, const tn_plan_t* plans, tn_batch_t* batch) {
  if (!batch) return set_error(TN_E_INVALID, "batch is null");
  *batch = nullptr;
  if (n_plans < 1 || !plans) return set_error(TN_E_INVALID, "no plans");
  for (int j = 0; j < n_plans; j++)
    if (!plans[j]) return set_error(TN_E_INVALID, "plan " + std::to_string(j) + " is null");
  const int prec = plans[0]->prec;
  for (int j = 0; j < n_plans; j++) {
    if (plans[j]->prec != prec) return set_error(TN_E_INVALID, "plans of a batch share one precision");
    if (plans[j]->d_sliced != 1 || plans[j]->n_batch != 1)
      return set_error(TN_E_UNSUPPORTED, "batched plans must be unsliced (plan " + std::to_string(j) + ")");
  }
  tn_batch_s* b = new tn_batch_s();
  b->prec = prec;
  b->n_nets = n_plans;
  // per network: the mode-0 program cut into (segment, following large ops) levels
  std::vector<std::vector<std::vector<TinyOp>>> segs(n_plans);
  std::vector<std::vector<std::vector<Op>>> bigs(n_plans);
  for (int j = 0; j < n_plans; j++) {
    tn_plan_s* p = plans[j];
    std::lock_guard<std::mutex> lk(p->mu);
    std::vector<Op> prog = forward_program(p, 0);
    segs[j].emplace_back();
    bigs[j].emplace_back();
    for (const Op& op : prog) {
      if (op.kind == OpKind::Counter || op.kind == OpKind::Fill) continue;
      TinyOp t;
      if (as_tiny(op, prec, t)) {
        if (!bigs[j].back().empty()) {   // a tiny op after large ones starts the next level
          segs[j].emplace_back();
          bigs[j].emplace_back();
        }
        segs[j].back().push_back(t);
      } else {
        bigs[j].back().push_back(op);
      }
    }
    b->n_levels = std::max(b->n_levels, (int)segs[j].size());
    b->n_leaves.push_back(p->n_leaves);
    b->ptr_stride = std::max(b->ptr_stride, p->n_leaves + 2);
  }
  const int L = b->n_levels, N = n_plans;
  b->seg.assign((size_t)L * N * 2, 0);
  b->big.assign(L, std::vector<std::vector<Op>>(N));
  for (int l = 0; l < L; l++)
    for (int j = 0; j < N; j++) {
      b->seg[((size_t)l * N + j) * 2] = (int32_t)b->tiny.size();
      if (l < (int)segs[j].size()) {
        b->tiny.insert(b->tiny.end(), segs[j][l].begin(), segs[j][l].end());
        b->big[l][j] = bigs[j][l];
      }
      b->seg[((size_t)l * N + j) * 2 + 1] = (int32_t)b->tiny.size();
    }
  // workspace: contexts | tiny ops | segments | pointer tables | per-network plan workspaces
  auto up = [](uint64_t x) { return (x + 255) / 256 * 256; };
  b->ctx_off = 0;
  b->ops_off = up(b->ctx_off + sizeof(Ctx) * (uint64_t)N);
  b->seg_off = up(b->ops_off + sizeof(TinyOp) * (uint64_t)std::max<size_t>(b->tiny.size(), 1));
  b->ptr_off = up(b->seg_off + sizeof(int32_t) * (uint64_t)b->seg.size());
  uint64_t off = up(b->ptr_off + 8 * (uint64_t)b->ptr_stride * N);
  for (int j = 0; j < N; j++) {
    tn_plan_s* p = plans[j];
    b->region_off.push_back(off);
    Ctx c = make_ctx(p, reinterpret_cast<void*>(off), p->arena_bytes);   // relative to the batch base
    c.ptrtab_off = (int64_t)(b->ptr_off + 8 * (uint64_t)b->ptr_stride * j) - (int64_t)off;
    b->ctx_rel.push_back(c);
    off = up(off + p->workspace_bytes);
  }
  b->ws_bytes = off;
  int64_t launches = 0;
  for (int l = 0; l < L; l++) {
    launches += 1;
    for (int j = 0; j < N; j++) launches += (int64_t)b->big[l][j].size();
  }
  b->n_launches = launches;
  *batch = b;
  return TN_OK;
}

extern "C" int tn_batch_info(tn_batch_t b, uint64_t* workspace_bytes, int32_t* n_levels, int64_t* n_tiny,
                             int64_t* n_launches) {
  if (!b) return set_error(TN_E_INVALID, "batch is null");
  std::lock_guard<std::mutex> lk(b->mu);
  if (workspace_bytes) *workspace_bytes = b->ws_bytes;
  if (n_levels) *n_levels = b->n_levels;
  if (n_tiny) *n_tiny = (int64_t)b->tiny.size();
  if (n_launches) *n_launches = b->n_launches;
  return TN_OK;
}

// Context of network j over the batch workspace at `base`.
static Ctx batch_ctx(const tn_batch_s* b, int j, uint64_t base) {
  Ctx c = b->ctx_rel[(size_t)j];
  c.ws += base;
  return c;
}

extern "C" int tn_batch_prepare(tn_batch_t b, void* workspace, uint64_t workspace_bytes, void* stream) {
  if (!b) return set_error(TN_E_INVALID, "batch is null");
  std::lock_guard<std::mutex> lk(b->mu);
  if (!workspace || workspace_bytes < b->ws_bytes)
    return set_error(TN_E_WORKSPACE, "workspace of " + std::to_string(b->ws_bytes) + " bytes required");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const uint64_t base = reinterpret_cast<uint64_t>(workspace);
  char* w = static_cast<char*>(workspace);
  std::vector<Ctx> ctxs;
  for (int j = 0; j < b->n_nets; j++) ctxs.push_back(batch_ctx(b, j, base));
  BATCH_TRY(hipMemcpyAsync(w + b->ctx_off, ctxs.data(), sizeof(Ctx) * ctxs.size(), hipMemcpyHostToDevice, s));
  if (!b->tiny.empty())
    BATCH_TRY(hipMemcpyAsync(w + b->ops_off, b->tiny.data(), sizeof(TinyOp) * b->tiny.size(), hipMemcpyHostToDevice, s));
  BATCH_TRY(hipMemcpyAsync(w + b->seg_off, b->seg.data(), sizeof(int32_t) * b->seg.size(), hipMemcpyHostToDevice, s));
  // each network's batch counter and slice-id list: 0 (one slice, id 0)
  for (int j = 0; j < b->n_nets; j++) {
    const Ctx c = ctxs[(size_t)j];
    BATCH_TRY(launch_fill(c.ws + c.counter_off, 8, s));
    BATCH_TRY(launch_fill(c.ws + c.sid_off, 8, s));
  }
  auto it = b->graphs.find(base);
  if (it != b->graphs.end()) {
    batch_drop(it->second);
    b->graphs.erase(it);
  }
  if (b->graphs.size() >= tn_plan_s::kMaxGraphs) {
    auto lru = b->graphs.begin();
    for (auto j = b->graphs.begin(); j != b->graphs.end(); ++j)
      if (j->second.last_use < lru->second.last_use) lru = j;
    batch_drop(lru->second);
    b->graphs.erase(lru);
  }
  // capture: level by level, the interpreter launch, then the large ops of
  // the networks on kBranches parallel branches (networks are independent;
  // the graph may run the branches concurrently), joined before the next level
  hipStream_t cs[kBranches] = {};
  hipEvent_t fork[kBranches] = {}, join[kBranches] = {};
  hipError_t e = hipSuccess;
  for (int i = 0; i < kBranches && e == hipSuccess; i++) {
    e = hipStreamCreateWithFlags(&cs[i], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&fork[i], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&join[i], hipEventDisableTiming);
  }
  if (e == hipSuccess) e = hipStreamBeginCapture(cs[0], hipStreamCaptureModeThreadLocal);
  const int N = b->n_nets;
  for (int l = 0; l < b->n_levels && e == hipSuccess; l++) {
    CMEM const Ctx* dctx = reinterpret_cast<CMEM const Ctx*>(base + b->ctx_off);
    CMEM const TinyOp* dops = reinterpret_cast<CMEM const TinyOp*>(base + b->ops_off);
    CMEM const int32_t* dseg = reinterpret_cast<CMEM const int32_t*>(base + b->seg_off + sizeof(int32_t) * 2 * (uint64_t)l * N);
    if (b->prec == TN_C128) hipLaunchKernelGGL(tiny_kernel<double>, dim3(N), dim3(kTinyThreads), 0, cs[0], dctx, dops, dseg);
    else hipLaunchKernelGGL(tiny_kernel<float>, dim3(N), dim3(kTinyThreads), 0, cs[0], dctx, dops, dseg);
    e = hipGetLastError();
    for (int i = 1; i < kBranches && e == hipSuccess; i++) {
      e = hipEventRecord(fork[i], cs[0]);
      if (e == hipSuccess) e = hipStreamWaitEvent(cs[i], fork[i], 0);
    }
    for (int j = 0; j < N && e == hipSuccess; j++)
      for (const Op& op : b->big[(size_t)l][(size_t)j]) {
        e = launch_op(b->prec, ctxs[(size_t)j], op, cs[j % kBranches]);
        if (e != hipSuccess) break;
      }
    for (int i = 1; i < kBranches && e == hipSuccess; i++) {
      e = hipEventRecord(join[i], cs[i]);
      if (e == hipSuccess) e = hipStreamWaitEvent(cs[0], join[i], 0);
    }
  }
  hipGraph_t graph = nullptr;
  hipError_t e2 = cs[0] ? hipStreamEndCapture(cs[0], &graph) : hipErrorInvalidValue;
  for (int i = 0; i < kBranches; i++) {
    if (cs[i]) (void)hipStreamDestroy(cs[i]);
    if (fork[i]) (void)hipEventDestroy(fork[i]);
    if (join[i]) (void)hipEventDestroy(join[i]);
  }
  if (e != hipSuccess || e2 != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return set_error(TN_E_DEVICE, std::string("batch capture: ") + hipGetErrorString(e != hipSuccess ? e : e2));
  }
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return set_error(TN_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  hipEvent_t done = nullptr;
  e = hipEventCreateWithFlags(&done, hipEventDisableTiming);
  if (e != hipSuccess) {
    (void)hipGraphExecDestroy(exec);
    return set_error(TN_E_DEVICE, std::string("hipEventCreateWithFlags: ") + hipGetErrorString(e));
  }
  tn_plan_s::GraphEntry ent;
  ent.exec = exec;
  ent.done = done;
  ent.last_use = ++b->clock;
  b->graphs[base] = ent;
  return TN_OK;
}

extern "C" int tn_batch_contract(tn_batch_t b, const void* const* leaves, void* const* outs, void* workspace,
                                 uint64_t workspace_bytes, void* stream) {
  if (!b) return set_error(TN_E_INVALID, "batch is null");
  std::lock_guard<std::mutex> lk(b->mu);
  if (!leaves || !outs) return set_error(TN_E_INVALID, "leaves or outs is null");
  if (!workspace || workspace_bytes < b->ws_bytes)
    return set_error(TN_E_WORKSPACE, "workspace of " + std::to_string(b->ws_bytes) + " bytes required");
  const uint64_t base = reinterpret_cast<uint64_t>(workspace);
  auto it = b->graphs.find(base);
  if (it == b->graphs.end()) return set_error(TN_E_WORKSPACE, "workspace not prepared (tn_batch_prepare)");
  std::vector<uint64_t> tab((size_t)b->ptr_stride * b->n_nets, 0);
  size_t li = 0;
  for (int j = 0; j < b->n_nets; j++) {
    uint64_t* t = &tab[(size_t)b->ptr_stride * j];
    for (int v = 0; v < b->n_leaves[(size_t)j]; v++, li++) {
      if (!leaves[li]) return set_error(TN_E_INVALID, "leaf pointer " + std::to_string(li) + " is null");
      t[v] = reinterpret_cast<uint64_t>(leaves[li]);
    }
    if (!outs[j]) return set_error(TN_E_INVALID, "output " + std::to_string(j) + " is null");
    t[b->n_leaves[(size_t)j]] = reinterpret_cast<uint64_t>(outs[j]);
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  BATCH_TRY(hipMemcpyAsync(static_cast<char*>(workspace) + b->ptr_off, tab.data(), tab.size() * 8,
                           hipMemcpyHostToDevice, s));
  it->second.last_use = ++b->clock;
  BATCH_TRY(hipGraphLaunch((hipGraphExec_t)it->second.exec, s));
  BATCH_TRY(hipEventRecord((hipEvent_t)it->second.done, s));
  return TN_OK;
}

extern "C" void tn_batch_destroy(tn_batch_t b) {
  if (!b) return;
  {
    std::lock_guard<std::mutex> lk(b->mu);
    for (auto& kv : b->graphs) batch_drop(kv.second);
    b->graphs.clear();
  }
  delete b;
}
