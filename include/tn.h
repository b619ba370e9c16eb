/*
 * libtn: execution of a fixed tensor-network contraction tree on one AMD
 * Instinct MI355X (gfx950).
 *
 * The problem statement follows Sec. 2 of Gray & Kourtis, "Hyper-optimized
 * tensor network contraction" (arXiv:2002.01935): leaf tensors T_v with
 * ordered index tuples t_v over indices e of dimension |D(e)|, an optional
 * list of open output indices, and a rooted binary contraction tree given by
 * the child tuples l(v), r(v) with the leaves numbered first.  Each internal
 * node is a pairwise contraction (Sec. 2): the product of its two children,
 * summed over the indices that no longer occur outside its subtree.  Sliced
 * indices (Sec. 4.7.1) are summed last, as an exterior sum over independent
 * copies of the network, each with the sliced indices fixed.
 *
 * Conventions shared by every entry point:
 *   - Return value: TN_OK (0) or a negative tn_status; tn_last_error() gives
 *     a thread-local message.  No exception or abort crosses this ABI.
 *   - Complex data is interleaved (re, im): complex64 = 2 x float,
 *     complex128 = 2 x double.  Leaves are dense, row-major in t_v order
 *     (last index fastest).  Outputs are row-major in out_idx order.
 *   - Device pointers: leaves, outputs, gradients and the workspace live in
 *     device memory owned by the caller.  Index lists, the tree, slice ids and
 *     the pointer arrays themselves are host memory owned by the caller and
 *     are not retained after the call returns (the plan copies what it needs).
 *   - The library allocates no device memory of its own beyond the HIP graphs
 *     cached inside a plan and the static scratch array of
 *     tn_contract_sliced_noalloc (64 MiB per GPU, part of its code object).
 *     All work is enqueued on
 *     the caller's stream (a hipStream_t passed as void*; NULL = default
 *     stream); calls return without waiting for the GPU.
 *   - Threads: every entry point that takes a plan holds that plan's lock
 *     while it reads or changes the plan's mutable state (cached graphs, the
 *     reverse program, tile choices) and enqueues its work, so several host
 *     threads may call into one plan at once.  Calls that run at the same
 *     time on the GPU must use distinct workspaces (and, for the
 *     allocation-free variant, distinct GPUs); calls that share a workspace
 *     must be ordered, e.g. on one stream.  A plan caches at most 8 graphs,
 *     one per (call kind, workspace address); the least recently used one is
 *     freed, after its last launch has finished, when a ninth is needed.
 *     tn_plan_destroy must not race with other calls on the same plan.
 */
#ifndef TN_H
#define TN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TN_OK = 0,
    TN_E_INVALID = -1,     /* malformed network, tree, ids or null pointer */
    TN_E_UNSUPPORTED = -2, /* valid input the GPU path does not run (non power-of-two dim, rank > 64) */
    TN_E_DEVICE = -3,      /* a HIP call failed */
    TN_E_WORKSPACE = -4    /* workspace missing or smaller than required */
} tn_status;

/* Arithmetic of the contraction.  C64 modes store complex64 tensors; the
   pairwise products on matrix cores use:
     TN_C64_4M     four real products per complex product, FP32 MFMA, FP32 accumulation
     TN_C64_3M     three real products (Gauss/Karatsuba), FP32 MFMA, FP32 accumulation
     TN_C64_BF16X3 4M with each FP32 operand split into bf16 hi + lo parts and the
                   product formed as hi*hi + hi*lo + lo*hi on BF16 MFMA, FP32 accumulation
     TN_C128       complex128 storage and FP64 arithmetic throughout
   Small (non-matrix) contractions run on the vector ALU in the storage precision.
   Slice sums and norm checks are always FP64. */
typedef enum {
    TN_C64_4M = 0,
    TN_C64_3M = 1,
    TN_C64_BF16X3 = 2,
    TN_C128 = 3
} tn_precision;

/* tn_options.flags */
enum {
    /* GEMM-shaped contractions (both free sides of at least 32 values) go to
       the matrix-core or few-summed-values kernels whatever their size.  By
       default those under 2^25 complex multiply-adds run on the row kernel,
       whose launches cost a fraction of a matrix-core launch at that size. */
    TN_FLAG_GEMM_ALL_SIZES = 1
};

typedef struct {
    int32_t prec;                /* tn_precision */
    int32_t autotune;            /* nonzero: tn_plan_tune may retune tile shapes */
    int32_t max_inflight_slices; /* slices contracted together per launch; 0 = choose from workspace_cap */
    int32_t flags;               /* TN_FLAG_* */
    uint64_t workspace_cap;      /* bytes; 0 = no cap (in-flight slices default to 1) */
} tn_options;

typedef struct tn_plan_s* tn_plan_t;

/*
 * Compile a plan for one network structure and tree (Sec. 2; slicing Sec. 4.7.1).
 *
 * n_leaves          number of leaf tensors |V| (>= 1)
 * rank[v]           number of axes of leaf v (d_v)
 * leaf_idx          concatenation of the tuples t_v (index ids in [0, n_idx))
 * idx_dim[e]        |D(e)|; the GPU path needs powers of two (else TN_E_UNSUPPORTED)
 * n_out, out_idx    open output indices, in output axis order (may be 0 / NULL)
 * left, right       n_leaves - 1 child pairs; internal node n_leaves + k has
 *                   children left[k], right[k], each an earlier node id; every
 *                   node except the last is used exactly once (a full binary tree)
 * n_sliced, sliced_idx  indices summed last; slice id -> index values is mixed
 *                   radix over this list, first index most significant
 * opt               options (NULL = defaults: TN_C64_4M, no autotune)
 * plan              receives the opaque plan
 *
 * Index e is kept at node v iff it occurs on a leaf below v and it is an open
 * output or occurs on a leaf outside the subtree of v; with plain two-ended
 * edges this is the symmetric-difference rule of eq. (incidence).
 *
 * Errors (TN_E_INVALID): null pointers; an index repeated within one leaf (a
 * self-loop); a non-output index on only one leaf; a tree that is not a full
 * binary tree over all leaves; a sliced index that is also an output, or
 * listed twice; an output listed twice.  TN_E_UNSUPPORTED: a tensor of the
 * tree (leaf, intermediate or root) holds 2^32 or more elements once the
 * sliced indices are removed (slice more indices).  Host-only: enqueues no
 * GPU work.
 */
int tn_plan(int32_t n_leaves, const int32_t* rank, const int64_t* leaf_idx,
            int32_t n_idx, const int64_t* idx_dim,
            int32_t n_out, const int64_t* out_idx,
            const int32_t* left, const int32_t* right,
            int32_t n_sliced, const int64_t* sliced_idx,
            const tn_options* opt, tn_plan_t* plan);

/*
 * Plan summary (any pointer may be NULL):
 *   W        contraction width of the unsliced tree, log2 of the largest tensor (eq. edgecon)
 *   W_s      width with the sliced indices removed
 *   log2_C   log2 of the unsliced cost C (eq. vertexcon, internal nodes)
 *   flops_8C_per_slice  8 * C of one slice: complex FLOPs as counted in Sec. 2
 *   d_sliced number of slices, prod over sliced indices of |D(e)|
 *   workspace_bytes  device workspace needed by tn_contract / tn_contract_sliced
 */
int tn_plan_info(tn_plan_t plan, int32_t* W, int32_t* W_s, double* log2_C,
                 double* flops_8C_per_slice, int64_t* d_sliced, uint64_t* workspace_bytes);

/* Device workspace needed by tn_contract_backward for the leaves wrt_leaf[0..n_wrt),
   and the FLOPs (8C convention) of one slice of the backward pass including the
   forward pass and recomputation.  Builds (and caches in the plan) the reverse
   program for that leaf set; host-only. */
int tn_plan_backward_info(tn_plan_t plan, int32_t n_wrt, const int32_t* wrt_leaf,
                          uint64_t* workspace_bytes, double* flops_per_slice);

/* Number of internal nodes, and per-node details for reporting: kernel class
   (0 = vector ALU row kernel, 1 = vector ALU split-K, 2 = GEMM: on the matrix
   cores, or, with at most three summed bits, on the write-bound vector ALU kernel,
   3 = matrix-core GEMM with its summed range split across the grid and the
   partial tiles summed in a fixed order),
   log2 of the batch (H), free-left (M), free-right (N) and summed (K) sizes,
   complex FLOPs (8 * 2^{H+M+N+K}) and algorithmic bytes (operands read once,
   output written once) per slice. */
int tn_plan_num_nodes(tn_plan_t plan, int32_t* n);
int tn_plan_node_info(tn_plan_t plan, int32_t k, int32_t* kernel_class, int32_t* logH,
                      int32_t* logM, int32_t* logN, int32_t* logK, double* flops, double* bytes);

/*
 * Optional autotune pass: times the candidate tile shapes of every distinct
 * matrix-core contraction shape of the forward program on synthetic data in
 * `workspace` (one warm-up launch with the summed range cut to at most 2^12
 * values per split, then the median of three timed launches taken
 * round-robin over the candidates, at the full summed range when the trials
 * of a shape fit about 6 s, else at the cut range; tn_plan_tune_trials
 * reports the table) and keeps the fastest in the plan, for the forward and the
 * backward program (contractions of the same shape, split and operand
 * layout class); the default variant stays unless another is faster by more
 * than 1 %, so that repeated runs execute the same kernels.  Without it, a
 * contraction takes the default: the direct-to-LDS variant where its
 * operands allow (tile 9 for TN_C64_4M, 7 for TN_C64_3M, 11 on pre-split
 * BF16x3 operands), else tile 0 (10 on pre-split operands).  Clears a tile
 * pinned by tn_plan_set_tile.  Overwrites the workspace; synchronises the
 * stream.
 */
int tn_plan_tune(tn_plan_t plan, void* workspace, uint64_t workspace_bytes, void* stream);

/*
 * Pin the tile variant of every matrix-core contraction of the plan (forward
 * and backward programs, also one built later) that variant `tile` can run,
 * in place of the default or autotuned choice; the others keep theirs.  Variants: 0 = 128x128,
 * 1 = 64x128, 2 = 128x64, 3 = 64x64 (every precision); 4 = vector ALU; for
 * TN_C64_4M also 5 = 256x128 and 6 = 128x128 with raised matrix-core
 * priority; for TN_C64_4M and TN_C64_3M 7 = 128x128, 8 = 256x128 and
 * 9 = 128x128 at more waves per SIMD, all direct-to-LDS (operands whose
 * summed indices are their lowest axes), and for TN_C64_4M 14 = 128x128
 * direct-to-LDS with the next stage's fragments read during the current
 * stage's matrix-core work; for TN_C64_BF16X3, on operands
 * split into bf16 planes beforehand, all direct-to-LDS: 10 = 128x128,
 * 11 = 256x128 (the default), 12 = 128x128 with three stages in flight,
 * 13 = 256x128 with the next stage's fragments read during the current
 * stage's matrix-core work (the planner splits the operands of contractions
 * of at least 2^28 multiply-adds, which then run on variants 10-13 only; the
 * others take 0-4).  *n_set (may be NULL) receives the
 * number of contractions changed.  TN_E_INVALID for an unknown variant.  Used to test
 * every variant and to reproduce a tuned plan.
 */
int tn_plan_set_tile(tn_plan_t plan, int32_t tile, int32_t* n_set);

/*
 * Contract an unsliced plan (n_sliced == 0).
 * leaves[v]   device pointer to leaf v (complex64, or complex128 for TN_C128)
 * out         device pointer, output in the plan's storage type, out_idx order
 *             (one element for a scalar)
 */
int tn_contract(tn_plan_t plan, const void* const* leaves, void* out,
                void* workspace, uint64_t workspace_bytes, void* stream);

/*
 * Sliced contraction (Sec. 4.7.1): the sum over the given slice ids of the
 * contraction with the sliced indices fixed to each id's values.
 * n_ids, slice_ids  host array of ids in [0, d_sliced); NULL = every id in
 *                   ascending order.  Ids are summed in the order given.  The
 *                   workspace holds the id list: one call takes at most
 *                   max(d_sliced, slices per graph replay) ids, capped at 2^22
 *                   (NULL with d_sliced above the cap is refused too); longer
 *                   lists return TN_E_INVALID; sum them over several calls.
 * out_c128          device pointer, complex128, out_idx order; overwritten with
 *                   the FP64 sum (each slice's root is promoted to FP64 and added
 *                   in a fixed order, so repeated calls are bitwise identical)
 * An unsliced plan is accepted (d_sliced = 1, id 0).
 */
int tn_contract_sliced(tn_plan_t plan, const void* const* leaves, int64_t n_ids,
                       const int64_t* slice_ids, void* out_c128,
                       void* workspace, uint64_t workspace_bytes, void* stream);

/*
 * Reverse mode.  grad_out_c128 (device, complex128, out_idx order) is
 * dL/d conj(R) for the contraction value R summed over the given slice ids.
 * For each requested leaf t = wrt_leaf[i], grads[i] (device, the leaf's storage
 * type and shape) is overwritten with
 *   grads[i][k] = sum_o conj(dR_o / dT_t[k]) * grad_out[o],
 * PyTorch's convention for complex gradients.  The pass recomputes forward
 * intermediates from checkpoints instead of storing every node value; the
 * cotangent of a child is the parent's cotangent contracted with the complex
 * conjugate of its sibling.  Each leaf may be listed once.
 */
int tn_contract_backward(tn_plan_t plan, const void* const* leaves,
                         const void* grad_out_c128, int32_t n_wrt,
                         const int32_t* wrt_leaf, void* const* grads,
                         int64_t n_ids, const int64_t* slice_ids,
                         void* workspace, uint64_t workspace_bytes, void* stream);

/*
 * Same result as tn_contract_sliced, but the program runs op by op (no
 * graph) with a HIP event recorded on `stream` before and after every kernel
 * launch, and the call waits for the GPU.  For measurement: on return,
 * n_ops receives the number of ops of one batch's program and, for i <
 * min(n_ops, cap), op_ms[i] the summed duration of op i over all batches,
 * op_kind[i] its kernel (0 row, 1 split-K, 2 split-K reduce, 3 GEMM,
 * 4 FP64 accumulation, 5 permute, 6 batch counter, 7 BF16x3 operand split),
 * op_node[i] its tree node
 * (-1 if none), op_flops[i] / op_bytes[i] its algorithmic complex FLOPs and
 * bytes per in-flight slice.  Any output array may be NULL.
 */
int tn_contract_sliced_timed(tn_plan_t plan, const void* const* leaves, int64_t n_ids,
                             const int64_t* slice_ids, void* out_c128, void* workspace,
                             uint64_t workspace_bytes, void* stream, int32_t cap, float* op_ms,
                             int32_t* op_kind, int32_t* op_node, double* op_flops,
                             double* op_bytes, int32_t* n_ops);

/*
 * Kernel of internal node k's contraction in the forward program, for
 * reporting: *tile receives the matrix-core tile variant (-1 for vector-ALU
 * kernels; 4 for complex128 products), `name` (capacity name_cap bytes, NUL
 * terminated, truncated if short) the kernel's name with its template
 * arguments, e.g. "gemm_mfma_4m_dl<128,128,2,2,3>".  Either may be NULL.
 * TN_E_INVALID for k outside [0, number of internal nodes).  Host-only.
 */
int tn_plan_node_kernel(tn_plan_t plan, int32_t k, int32_t* tile, char* name, int32_t name_cap);

/*
 * Kernels of the contractions of the reverse program for the leaves
 * wrt_leaf[0..n_wrt) (Sec. 2 pairwise products applied to cotangents), in
 * program order, for reporting: *n receives their number; for i < min(*n,
 * cap), names[i * name_cap ..] the i-th kernel's name as tn_plan_node_kernel
 * writes it (NUL terminated, truncated if short).  Builds (and caches) the
 * reverse program like tn_plan_backward_info.  names may be NULL.  Host-only.
 */
int tn_plan_backward_kernels(tn_plan_t plan, int32_t n_wrt, const int32_t* wrt_leaf, int32_t cap, int32_t* n,
                             char* names, int32_t name_cap);

/*
 * Trials of the last tn_plan_tune: *n receives their number; for i < min(*n,
 * cap): keys[6i .. 6i+5] the contraction shape (log2 H, M, N, K, split bits,
 * 1 if both operands hold the summed indices lowest), tiles[i] the variant,
 * k_bits[i] log2 of the summed range it ran with, ms[i] its median time.
 * Output arrays may be NULL.  Host-only.
 */
int tn_plan_tune_trials(tn_plan_t plan, int32_t cap, int32_t* n, int32_t* keys, int32_t* tiles,
                        int32_t* k_bits, float* ms);

/*
 * For callers that cannot allocate device memory (code that must not call
 * hipMalloc, e.g. a serving loop with a fixed memory budget): the same
 * contraction and result as tn_contract_sliced, with the workspace replaced
 * by a static array of 64 MiB that the library holds on each GPU it runs on
 * (loaded with its code object, kept until the process ends).  The call
 * allocates no device memory and captures no graph: every kernel is launched
 * on `stream`, which must belong to the calling thread's current device.
 * Plans whose workspace (tn_plan_info) exceeds 64 MiB get TN_E_WORKSPACE.
 * The array keeps the last call's contents; the call resets what must start
 * from zero (the batch counter and out_c128).  All calls on one GPU share the
 * array: calls that overlap on one GPU, from any plan or thread, race and
 * must be ordered by the caller (e.g. on one stream).
 */
int tn_contract_sliced_noalloc(tn_plan_t plan, const void* const* leaves, int64_t n_ids,
                               const int64_t* slice_ids, void* out_c128, void* stream);

/*
 * Many independent small networks in one graph launch (Sec. 4.5: the QAOA
 * energy is a sum of one light-cone network per edge; Sec. 4.7.3: sampling
 * needs many contractions).  A batch takes n_plans compiled, unsliced plans
 * of one precision (TN_E_UNSUPPORTED for a sliced plan, TN_E_INVALID for
 * mixed precisions); it copies their programs (with their tile choices at
 * this time), so the plans may be destroyed afterwards.  Each network's
 * contractions with at most 2^14 (outputs x summed values) run inside one
 * interpreter kernel, one workgroup per network, in the network's own order;
 * the others with the ordinary kernels between the interpreter's launches.
 * The result of network j is its tn_contract result.
 *
 * tn_batch_info: workspace bytes, number of interpreter launches (levels),
 * number of contractions the interpreter runs, and launches per call.
 *
 * tn_batch_prepare: writes the batch's tables (contraction descriptors and
 * per-network launch contexts) into `workspace` and captures the graph for
 * that workspace address (at most 8 workspaces per batch; the least recently
 * used is dropped, after its last launch has finished).  The caller must not
 * modify a prepared workspace between calls.
 *
 * tn_batch_contract: leaves = the leaf pointers of network 0 (in leaf
 * order), then of network 1, ...; outs[j] = network j's output, in its plan's
 * storage type and out_idx order.  `workspace` must have been prepared
 * (TN_E_WORKSPACE otherwise).  Uploads the pointer tables and replays the
 * graph on `stream`.  Calls on one workspace must be ordered.
 */
typedef struct tn_batch_s* tn_batch_t;
int tn_batch(int32_t n_plans, const tn_plan_t* plans, tn_batch_t* batch);
int tn_batch_info(tn_batch_t batch, uint64_t* workspace_bytes, int32_t* n_levels, int64_t* n_tiny,
                  int64_t* n_launches);
int tn_batch_prepare(tn_batch_t batch, void* workspace, uint64_t workspace_bytes, void* stream);
int tn_batch_contract(tn_batch_t batch, const void* const* leaves, void* const* outs, void* workspace,
                      uint64_t workspace_bytes, void* stream);
void tn_batch_destroy(tn_batch_t batch);

void tn_plan_destroy(tn_plan_t plan);

/* Message for the last failing call on this thread ("" if none). */
const char* tn_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TN_H */
