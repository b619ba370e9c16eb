/*
 * Oracle: plain CPU complex128 tensor-network contractor.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the GPU library and never touches a GPU.
 *
 * What it computes (Sec. 4.7.1, Slicing; Sec. 2, Problem statement):
 *   R[o] = sum over every non-output index value of prod_v T_v(x restricted to t_v),
 * evaluated pairwise along the given contraction tree (any tree gives the same
 * result, up to rounding, because the tree only re-brackets the nested sums),
 * with the sliced indices summed last as an exterior sum over fixed values:
 *   R = sum_{sigma} R_sigma,  R_sigma = the same network with the sliced
 *   indices fixed to sigma (each leaf carrying them replaced by its slice).
 *
 * Pairwise contraction (Sec. 2): the product of the two tensors, summed over
 * every index that is not kept.  Index e is kept at tree node v iff e occurs on
 * a leaf below v and (e is an open output index or e occurs on a leaf outside
 * the subtree of v).  With plain two-ended edges and no outputs this is the
 * symmetric-difference rule of eq. (incidence); the general rule also covers
 * hyperedges and open indices.
 *
 * Kept-index order of a node: the left child's kept indices in the left
 * child's order, then the right child's kept indices not already listed.
 * Slice id -> index values: mixed radix over the sliced list, first index most
 * significant.  Slices are summed in the order given.
 *
 * Reverse mode (oracle_grad): with g_out = dL/d conj(R), the cotangent of a
 * child is the contraction of the parent's cotangent with the complex
 * conjugate of the sibling, onto the child's index set:
 *   g_l[x_l] = sum_{indices of v and r not in l} g_v[x_v] * conj(T_r[x_r]),
 * and the leaf gradients are the cotangents that reach the leaves
 * (grad_t[k] = sum_o conj(dR_o / dT_t[k]) g_out[o]).  For a sliced leaf the
 * slice's cotangent lands in that slice's block of the full leaf gradient.
 *
 * Arithmetic: every multiply-add is an explicit complex128 operation
 * (re = ar*br - ai*bi, im = ar*bi + ai*br); OpenMP splits only over output
 * elements, so results do not depend on the thread count.
 *
 * ORACLE_PLANT_* macros plant one deliberate mistake each.  They exist only so
 * that the test suite can show its pins catch such mistakes; the normal build
 * defines none of them.
 */

#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <stdarg.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static char g_err[512];

static int fail(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return -1;
}

const char* oracle_last_error(void) { return g_err; }

typedef struct {
    int rank;
    int64_t* idx;      /* index ids, axis order (outermost first) */
    int64_t* dim;      /* dims per axis */
    int64_t size;
    double* data;      /* complex128 interleaved */
} otensor;

static void ot_free(otensor* t) {
    free(t->idx);
    free(t->dim);
    free(t->data);
    memset(t, 0, sizeof *t);
}

static int64_t pos_in(const int64_t* list, int n, int64_t e) {
    for (int i = 0; i < n; i++)
        if (list[i] == e) return i;
    return -1;
}

/* Strides (in elements) of a row-major tensor with the given dims. */
static void row_major_strides(int rank, const int64_t* dim, int64_t* stride) {
    int64_t s = 1;
    for (int i = rank - 1; i >= 0; i--) {
        stride[i] = s;
        s *= dim[i];
    }
}

/*
 * Generic pairwise product:  out[x_out] = sum_{x_sum} A[x_A] * opB(B[x_B])
 * where x_out ranges over the `out` index list, x_sum over `sum` list, and
 * every index of A and B is in out or sum.  conjB selects conj(B).
 */
static int contract_pair(const otensor* A, const otensor* B, int conjB,
                         int n_out, const int64_t* out_idx, const int64_t* out_dim,
                         int n_sum, const int64_t* sum_idx, const int64_t* sum_dim,
                         otensor* C, int n_threads) {
    int64_t sA[64], sB[64];
    if (A->rank > 64 || B->rank > 64 || n_out > 64 || n_sum > 64) return fail("rank too large");
    row_major_strides(A->rank, A->dim, sA);
    row_major_strides(B->rank, B->dim, sB);
    /* stride contributions of each out / sum index to A and B addresses */
    int64_t oA[64], oB[64], uA[64], uB[64];
    for (int i = 0; i < n_out; i++) {
        int64_t pa = pos_in(A->idx, A->rank, out_idx[i]);
        int64_t pb = pos_in(B->idx, B->rank, out_idx[i]);
        oA[i] = pa >= 0 ? sA[pa] : 0;
        oB[i] = pb >= 0 ? sB[pb] : 0;
    }
    for (int i = 0; i < n_sum; i++) {
        int64_t pa = pos_in(A->idx, A->rank, sum_idx[i]);
        int64_t pb = pos_in(B->idx, B->rank, sum_idx[i]);
        uA[i] = pa >= 0 ? sA[pa] : 0;
        uB[i] = pb >= 0 ? sB[pb] : 0;
    }
    /* every axis of A and B must be covered by out or sum */
    for (int i = 0; i < A->rank; i++)
        if (pos_in(out_idx, n_out, A->idx[i]) < 0 && pos_in(sum_idx, n_sum, A->idx[i]) < 0)
            return fail("index %lld of left operand neither kept nor summed", (long long)A->idx[i]);
    for (int i = 0; i < B->rank; i++)
        if (pos_in(out_idx, n_out, B->idx[i]) < 0 && pos_in(sum_idx, n_sum, B->idx[i]) < 0)
            return fail("index %lld of right operand neither kept nor summed", (long long)B->idx[i]);

    int64_t out_size = 1, sum_size = 1;
    for (int i = 0; i < n_out; i++) out_size *= out_dim[i];
    for (int i = 0; i < n_sum; i++) sum_size *= sum_dim[i];

    /* offsets of every summed assignment, summed indices in lexicographic order
       (last index fastest) */
    int64_t* offA = (int64_t*)malloc(sizeof(int64_t) * (size_t)sum_size);
    int64_t* offB = (int64_t*)malloc(sizeof(int64_t) * (size_t)sum_size);
    if (!offA || !offB) { free(offA); free(offB); return fail("out of host memory"); }
    {
        int64_t val[64] = {0};
        for (int64_t s = 0; s < sum_size; s++) {
            int64_t a = 0, b = 0;
            for (int i = 0; i < n_sum; i++) { a += val[i] * uA[i]; b += val[i] * uB[i]; }
            offA[s] = a;
            offB[s] = b;
            for (int i = n_sum - 1; i >= 0; i--) {   /* odometer */
                if (++val[i] < sum_dim[i]) break;
                val[i] = 0;
            }
        }
    }

    C->rank = n_out;
    C->idx = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_out > 0 ? n_out : 1));
    C->dim = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_out > 0 ? n_out : 1));
    C->size = out_size;
    C->data = (double*)malloc(sizeof(double) * 2 * (size_t)out_size);
    if (!C->idx || !C->dim || !C->data) { free(offA); free(offB); ot_free(C); return fail("out of host memory"); }
    memcpy(C->idx, out_idx, sizeof(int64_t) * (size_t)n_out);
    memcpy(C->dim, out_dim, sizeof(int64_t) * (size_t)n_out);

    const double* a = A->data;
    const double* b = B->data;
    double* c = C->data;
    const double sgn = conjB ? -1.0 : 1.0;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(n_threads > 0 ? n_threads : 1)
#endif
    for (int64_t o = 0; o < out_size; o++) {
        /* decode the output assignment (last index fastest) */
        int64_t rem = o, baseA = 0, baseB = 0;
        for (int i = n_out - 1; i >= 0; i--) {
            int64_t v = rem % out_dim[i];
            rem /= out_dim[i];
            baseA += v * oA[i];
            baseB += v * oB[i];
        }
        double re = 0.0, im = 0.0;
#ifdef ORACLE_PLANT_DROP
        for (int64_t s = 0; s < (sum_size > 1 ? sum_size - 1 : sum_size); s++) {
#else
        for (int64_t s = 0; s < sum_size; s++) {
#endif
            const double ar = a[2 * (baseA + offA[s])], ai = a[2 * (baseA + offA[s]) + 1];
            const double br = b[2 * (baseB + offB[s])], bi = sgn * b[2 * (baseB + offB[s]) + 1];
            re += ar * br - ai * bi;
#ifdef ORACLE_PLANT_SIGN
            im += ar * bi - ai * br;
#else
            im += ar * bi + ai * br;
#endif
        }
        c[2 * o] = re;
        c[2 * o + 1] = im;
    }
    (void)n_threads;
    free(offA);
    free(offB);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Network description, validation and per-node kept sets                   */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t n_leaves, n_idx, n_out, n_sliced;
    const int32_t* rank;
    const int64_t* leaf_idx;
    int64_t* leaf_off;       /* start of each leaf's index list in leaf_idx */
    const int64_t* idx_dim;
    const int64_t* out_idx;
    const int32_t* left;
    const int32_t* right;
    const int64_t* sliced;
    int32_t* total;          /* number of leaves carrying each index */
    char* is_out;
    char* is_sliced;
    /* per tree node: leaf-occurrence count of each index below the node */
    int32_t* below;          /* (2n-1) x n_idx, built lazily: row per node */
    int64_t** kept;          /* per node: kept index list (ordered) */
    int32_t* n_kept;
} onet;

static void onet_free(onet* g) {
    free(g->leaf_off);
    free(g->total);
    free(g->is_out);
    free(g->is_sliced);
    free(g->below);
    if (g->kept) {
        for (int v = 0; v < 2 * g->n_leaves - 1; v++) free(g->kept[v]);
        free(g->kept);
    }
    free(g->n_kept);
    memset(g, 0, sizeof *g);
}

static int onet_build(onet* g, int32_t n_leaves, const int32_t* rank, const int64_t* leaf_idx,
                      int32_t n_idx, const int64_t* idx_dim, int32_t n_out, const int64_t* out_idx,
                      const int32_t* left, const int32_t* right, int32_t n_sliced,
                      const int64_t* sliced) {
    memset(g, 0, sizeof *g);
    if (n_leaves < 1 || !rank || (n_idx > 0 && !idx_dim) || (n_leaves > 1 && (!left || !right)))
        return fail("null or empty network");
    g->n_leaves = n_leaves; g->n_idx = n_idx; g->n_out = n_out; g->n_sliced = n_sliced;
    g->rank = rank; g->leaf_idx = leaf_idx; g->idx_dim = idx_dim; g->out_idx = out_idx;
    g->left = left; g->right = right; g->sliced = sliced;
    int nn = 2 * n_leaves - 1;
    g->leaf_off = (int64_t*)calloc((size_t)n_leaves + 1, sizeof(int64_t));
    g->total = (int32_t*)calloc((size_t)n_idx + 1, sizeof(int32_t));
    g->is_out = (char*)calloc((size_t)n_idx + 1, 1);
    g->is_sliced = (char*)calloc((size_t)n_idx + 1, 1);
    g->below = (int32_t*)calloc((size_t)nn * (size_t)(n_idx + 1), sizeof(int32_t));
    g->kept = (int64_t**)calloc((size_t)nn, sizeof(int64_t*));
    g->n_kept = (int32_t*)calloc((size_t)nn, sizeof(int32_t));
    if (!g->leaf_off || !g->total || !g->is_out || !g->is_sliced || !g->below || !g->kept || !g->n_kept)
        return fail("out of host memory");
    for (int i = 0; i < n_idx; i++)
        if (idx_dim[i] < 1) return fail("index %d has dimension < 1", i);
    for (int v = 0; v < n_leaves; v++) {
        g->leaf_off[v + 1] = g->leaf_off[v] + rank[v];
        for (int a = 0; a < rank[v]; a++) {
            int64_t e = leaf_idx[g->leaf_off[v] + a];
            if (e < 0 || e >= n_idx) return fail("leaf %d: index id %lld out of range", v, (long long)e);
            for (int b = 0; b < a; b++)
                if (leaf_idx[g->leaf_off[v] + b] == e)
                    return fail("leaf %d repeats index %lld (self-loop)", v, (long long)e);
            g->total[e]++;
            g->below[(size_t)v * (n_idx + 1) + e] = 1;
        }
    }
    for (int i = 0; i < n_out; i++) {
        int64_t e = out_idx[i];
        if (e < 0 || e >= n_idx) return fail("output index %lld out of range", (long long)e);
        if (g->is_out[e]) return fail("output index %lld listed twice", (long long)e);
        if (g->total[e] < 1) return fail("output index %lld is on no leaf", (long long)e);
        g->is_out[e] = 1;
    }
    for (int i = 0; i < n_idx; i++)
        if (g->total[i] == 1 && !g->is_out[i])
            return fail("index %d is on one leaf only and is not an output", i);
    for (int i = 0; i < n_sliced; i++) {
        int64_t e = sliced[i];
        if (e < 0 || e >= n_idx) return fail("sliced index %lld out of range", (long long)e);
        if (g->is_out[e]) return fail("sliced index %lld is an output", (long long)e);
        if (g->is_sliced[e]) return fail("sliced index %lld listed twice", (long long)e);
        g->is_sliced[e] = 1;
    }
    /* tree: every id used exactly once as a child, children created earlier */
    char* used = (char*)calloc((size_t)nn, 1);
    if (!used) return fail("out of host memory");
    for (int k = 0; k < n_leaves - 1; k++) {
        int32_t l = left[k], r = right[k], v = n_leaves + k;
        if (l < 0 || r < 0 || l >= v || r >= v || l == r || used[l] || used[r]) {
            free(used);
            return fail("tree is not a full binary tree over the leaves (node %d)", v);
        }
        used[l] = used[r] = 1;
        int32_t* bv = g->below + (size_t)v * (n_idx + 1);
        const int32_t* bl = g->below + (size_t)l * (n_idx + 1);
        const int32_t* br = g->below + (size_t)r * (n_idx + 1);
        for (int e = 0; e < n_idx; e++) bv[e] = bl[e] + br[e];
    }
    free(used);
    /* kept sets, with the sliced indices removed from the network */
    for (int v = 0; v < nn; v++) {
        const int32_t* bv = g->below + (size_t)v * (n_idx + 1);
        int64_t* list = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_idx + 1));
        int n = 0;
        if (!list) return fail("out of host memory");
        if (v < n_leaves) {
            for (int a = 0; a < rank[v]; a++) {
                int64_t e = leaf_idx[g->leaf_off[v] + a];
                if (!g->is_sliced[e]) list[n++] = e;
            }
        } else {
            int32_t l = left[v - n_leaves], r = right[v - n_leaves];
            /* left's kept in left's order, then right's kept not yet present */
            for (int pass = 0; pass < 2; pass++) {
                int32_t c = pass == 0 ? l : r;
                for (int a = 0; a < g->n_kept[c]; a++) {
                    int64_t e = g->kept[c][a];
                    if (pos_in(list, n, e) >= 0) continue;
#ifdef ORACLE_PLANT_KEPT
                    if (bv[e] < g->total[e]) list[n++] = e;
#else
                    if (g->is_out[e] || bv[e] < g->total[e]) list[n++] = e;
#endif
                }
            }
        }
        g->kept[v] = list;
        g->n_kept[v] = n;
    }
    return 0;
}

/* Sub-block of leaf v with its sliced indices fixed to the slice's values. */
static int leaf_slice(const onet* g, int v, const double* data, const int64_t* slice_val, otensor* t) {
    int r = g->rank[v];
    const int64_t* ix = g->leaf_idx + g->leaf_off[v];
    int64_t dim[64], stride[64];
    if (r > 64) return fail("leaf rank too large");
    for (int a = 0; a < r; a++) dim[a] = g->idx_dim[ix[a]];
    row_major_strides(r, dim, stride);
    int64_t base = 0;
    int nr = 0;
    int64_t nidx[64], ndim[64], nstride[64];
    for (int a = 0; a < r; a++) {
        if (g->is_sliced[ix[a]]) {
            base += slice_val[ix[a]] * stride[a];
        } else {
            nidx[nr] = ix[a];
            ndim[nr] = dim[a];
            nstride[nr] = stride[a];
            nr++;
        }
    }
    int64_t size = 1;
    for (int a = 0; a < nr; a++) size *= ndim[a];
    t->rank = nr;
    t->idx = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nr > 0 ? nr : 1));
    t->dim = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nr > 0 ? nr : 1));
    t->size = size;
    t->data = (double*)malloc(sizeof(double) * 2 * (size_t)size);
    if (!t->idx || !t->dim || !t->data) return fail("out of host memory");
    memcpy(t->idx, nidx, sizeof(int64_t) * (size_t)nr);
    memcpy(t->dim, ndim, sizeof(int64_t) * (size_t)nr);
    int64_t val[64] = {0};
    for (int64_t o = 0; o < size; o++) {
        int64_t src = base;
        for (int a = 0; a < nr; a++) src += val[a] * nstride[a];
        t->data[2 * o] = data[2 * src];
        t->data[2 * o + 1] = data[2 * src + 1];
        for (int a = nr - 1; a >= 0; a--) {
            if (++val[a] < ndim[a]) break;
            val[a] = 0;
        }
    }
    return 0;
}

static int64_t n_slices_of(const onet* g) {
    int64_t d = 1;
    for (int i = 0; i < g->n_sliced; i++) d *= g->idx_dim[g->sliced[i]];
    return d;
}

/* Mixed radix, first sliced index most significant. */
static void slice_values(const onet* g, int64_t sid, int64_t* val) {
#ifdef ORACLE_PLANT_SLICE
    for (int i = 0; i < g->n_sliced; i++) {
#else
    for (int i = g->n_sliced - 1; i >= 0; i--) {
#endif
        int64_t e = g->sliced[i];
        val[e] = sid % g->idx_dim[e];
        sid /= g->idx_dim[e];
    }
}

/* Contract node v: its own kept set, summing every other index of the two
   children. */
static int contract_node(const onet* g, int v, const otensor* L, const otensor* R, otensor* out,
                         int n_threads) {
    int64_t sum_idx[128], sum_dim[128], out_dim[128];
    int ns = 0;
    const int64_t* keep = g->kept[v];
    int nk = g->n_kept[v];
    if (nk > 128) return fail("node rank too large");
    for (int i = 0; i < nk; i++) out_dim[i] = g->idx_dim[keep[i]];
    for (int pass = 0; pass < 2; pass++) {
        const otensor* T = pass == 0 ? L : R;
        for (int a = 0; a < T->rank; a++) {
            int64_t e = T->idx[a];
            if (pos_in(keep, nk, e) >= 0 || pos_in(sum_idx, ns, e) >= 0) continue;
            if (ns >= 128) return fail("too many summed indices");
            sum_idx[ns] = e;
            sum_dim[ns] = g->idx_dim[e];
            ns++;
        }
    }
    return contract_pair(L, R, 0, nk, keep, out_dim, ns, sum_idx, sum_dim, out, n_threads);
}

/* Forward pass of one slice; keeps every node value when `keep_all`. */
static int forward_slice(const onet* g, const double* const* leaves, const int64_t* sval,
                         otensor* vals, int keep_all, int n_threads) {
    int n = g->n_leaves;
    for (int v = 0; v < n; v++) {
        if (!leaves[v]) return fail("leaf %d data is null", v);
        if (leaf_slice(g, v, leaves[v], sval, &vals[v])) return -1;
    }
    for (int k = 0; k < n - 1; k++) {
        int v = n + k, l = g->left[k], r = g->right[k];
        if (contract_node(g, v, &vals[l], &vals[r], &vals[v], n_threads)) return -1;
        if (!keep_all) {
            ot_free(&vals[l]);
            ot_free(&vals[r]);
        }
    }
    return 0;
}

/* Add the root value, permuted to out_idx order, into out (complex128). */
static int add_root(const onet* g, const otensor* root, double* out) {
    int64_t pos[128], st[128];
    if (root->rank != g->n_out) return fail("root rank %d != number of outputs %d", root->rank, g->n_out);
    row_major_strides(root->rank, root->dim, st);
    for (int i = 0; i < g->n_out; i++) {
#ifdef ORACLE_PLANT_ROOT
        pos[i] = pos_in(root->idx, root->rank, g->out_idx[g->n_out - 1 - i]);
#else
        pos[i] = pos_in(root->idx, root->rank, g->out_idx[i]);
#endif
        if (pos[i] < 0) return fail("output index %lld missing at the root", (long long)g->out_idx[i]);
    }
    int64_t size = root->size;
    int64_t val[128] = {0};
    for (int64_t o = 0; o < size; o++) {   /* o enumerates out_idx order */
        int64_t src = 0;
        for (int i = 0; i < g->n_out; i++) src += val[i] * st[pos[i]];
        out[2 * o] += root->data[2 * src];
        out[2 * o + 1] += root->data[2 * src + 1];
        for (int i = g->n_out - 1; i >= 0; i--) {
            if (++val[i] < g->idx_dim[g->out_idx[i]]) break;
            val[i] = 0;
        }
    }
    return 0;
}

int oracle_contract(int32_t n_leaves, const int32_t* rank, const int64_t* leaf_idx,
                    int32_t n_idx, const int64_t* idx_dim, int32_t n_out, const int64_t* out_idx,
                    const int32_t* left, const int32_t* right, int32_t n_sliced,
                    const int64_t* sliced_idx, const double* const* leaves, int64_t n_ids,
                    const int64_t* slice_ids, double* out, int32_t n_threads) {
    onet g;
    if (!out || !leaves) return fail("null pointer");
    if (onet_build(&g, n_leaves, rank, leaf_idx, n_idx, idx_dim, n_out, out_idx, left, right,
                   n_sliced, sliced_idx)) {
        onet_free(&g);
        return -1;
    }
    int64_t out_size = 1;
    for (int i = 0; i < n_out; i++) out_size *= idx_dim[out_idx[i]];
    memset(out, 0, sizeof(double) * 2 * (size_t)out_size);
    int64_t d = n_slices_of(&g);
    int64_t ns = slice_ids ? n_ids : d;
    int nn = 2 * n_leaves - 1;
    otensor* vals = (otensor*)calloc((size_t)nn, sizeof(otensor));
    int64_t* sval = (int64_t*)calloc((size_t)n_idx + 1, sizeof(int64_t));
    int rc = (vals && sval) ? 0 : fail("out of host memory");
    for (int64_t s = 0; s < ns && rc == 0; s++) {
        int64_t sid = slice_ids ? slice_ids[s] : s;
        if (sid < 0 || sid >= d) { rc = fail("slice id %lld out of range", (long long)sid); break; }
        slice_values(&g, sid, sval);
        rc = forward_slice(&g, leaves, sval, vals, 0, n_threads);
        if (rc == 0) rc = add_root(&g, &vals[nn - 1], out);
        for (int v = 0; v < nn; v++) ot_free(&vals[v]);
    }
    free(vals);
    free(sval);
    onet_free(&g);
    return rc;
}

/*
 * Reverse mode.  grad_out: complex128 in out_idx order (dL/d conj(R)).
 * grads[t]: complex128 buffer of the full (unsliced) leaf wrt[t], overwritten.
 */
int oracle_grad(int32_t n_leaves, const int32_t* rank, const int64_t* leaf_idx,
                int32_t n_idx, const int64_t* idx_dim, int32_t n_out, const int64_t* out_idx,
                const int32_t* left, const int32_t* right, int32_t n_sliced,
                const int64_t* sliced_idx, const double* const* leaves, const double* grad_out,
                int32_t n_wrt, const int32_t* wrt, double* const* grads, int64_t n_ids,
                const int64_t* slice_ids, int32_t n_threads) {
    onet g;
    if (!leaves || !grad_out || (n_wrt > 0 && (!wrt || !grads))) return fail("null pointer");
    if (onet_build(&g, n_leaves, rank, leaf_idx, n_idx, idx_dim, n_out, out_idx, left, right,
                   n_sliced, sliced_idx)) {
        onet_free(&g);
        return -1;
    }
    int rc = 0;
    int nn = 2 * n_leaves - 1;
    /* zero the requested gradients */
    for (int t = 0; t < n_wrt && rc == 0; t++) {
        int v = wrt[t];
        if (v < 0 || v >= n_leaves) { rc = fail("wrt leaf %d out of range", v); break; }
        int64_t sz = 1;
        for (int a = 0; a < rank[v]; a++) sz *= idx_dim[leaf_idx[g.leaf_off[v] + a]];
        memset(grads[t], 0, sizeof(double) * 2 * (size_t)sz);
    }
    int64_t d = n_slices_of(&g);
    int64_t ns = slice_ids ? n_ids : d;
    otensor* vals = (otensor*)calloc((size_t)nn, sizeof(otensor));
    otensor* cot = (otensor*)calloc((size_t)nn, sizeof(otensor));
    int64_t* sval = (int64_t*)calloc((size_t)n_idx + 1, sizeof(int64_t));
    if (!vals || !cot || !sval) rc = fail("out of host memory");
    for (int64_t s = 0; s < ns && rc == 0; s++) {
        int64_t sid = slice_ids ? slice_ids[s] : s;
        if (sid < 0 || sid >= d) { rc = fail("slice id %lld out of range", (long long)sid); break; }
        slice_values(&g, sid, sval);
        rc = forward_slice(&g, leaves, sval, vals, 1, n_threads);
        if (rc) break;
        /* root cotangent: grad_out permuted from out_idx order to the root's order */
        {
            const otensor* root = &vals[nn - 1];
            otensor* c = &cot[nn - 1];
            c->rank = root->rank;
            c->size = root->size;
            c->idx = (int64_t*)malloc(sizeof(int64_t) * (size_t)(root->rank > 0 ? root->rank : 1));
            c->dim = (int64_t*)malloc(sizeof(int64_t) * (size_t)(root->rank > 0 ? root->rank : 1));
            c->data = (double*)malloc(sizeof(double) * 2 * (size_t)root->size);
            if (!c->idx || !c->dim || !c->data) { rc = fail("out of host memory"); break; }
            memcpy(c->idx, root->idx, sizeof(int64_t) * (size_t)root->rank);
            memcpy(c->dim, root->dim, sizeof(int64_t) * (size_t)root->rank);
            int64_t ost[128];
            int64_t odim[128];
            for (int i = 0; i < n_out; i++) odim[i] = idx_dim[out_idx[i]];
            row_major_strides(n_out, odim, ost);
            int64_t val[128] = {0};
            for (int64_t o = 0; o < root->size; o++) {   /* o in root order */
                int64_t src = 0;
                for (int i = 0; i < root->rank; i++) src += val[i] * ost[pos_in(out_idx, n_out, root->idx[i])];
                c->data[2 * o] = grad_out[2 * src];
                c->data[2 * o + 1] = grad_out[2 * src + 1];
                for (int i = root->rank - 1; i >= 0; i--) {
                    if (++val[i] < root->dim[i]) break;
                    val[i] = 0;
                }
            }
        }
        /* top-down: children cotangents */
        for (int k = n_leaves - 2; k >= 0 && rc == 0; k--) {
            int v = n_leaves + k, l = g.left[k], r = g.right[k];
            for (int side = 0; side < 2 && rc == 0; side++) {
                int child = side == 0 ? l : r, sib = side == 0 ? r : l;
                const otensor* T = &vals[child];
                int64_t sum_idx[128], sum_dim[128], cdim[128];
                int nsu = 0;
                for (int i = 0; i < T->rank; i++) cdim[i] = T->dim[i];
                for (int pass = 0; pass < 2; pass++) {
                    const otensor* X = pass == 0 ? &cot[v] : &vals[sib];
                    for (int a = 0; a < X->rank; a++) {
                        int64_t e = X->idx[a];
                        if (pos_in(T->idx, T->rank, e) >= 0 || pos_in(sum_idx, nsu, e) >= 0) continue;
                        sum_idx[nsu] = e;
                        sum_dim[nsu] = idx_dim[e];
                        nsu++;
                    }
                }
#ifdef ORACLE_PLANT_CONJ
                rc = contract_pair(&cot[v], &vals[sib], 0, T->rank, T->idx, cdim, nsu, sum_idx, sum_dim,
                                   &cot[child], n_threads);
#else
                rc = contract_pair(&cot[v], &vals[sib], 1, T->rank, T->idx, cdim, nsu, sum_idx, sum_dim,
                                   &cot[child], n_threads);
#endif
            }
            ot_free(&cot[v]);
        }
        /* scatter leaf cotangents into the sliced block of each requested leaf */
        for (int t = 0; t < n_wrt && rc == 0; t++) {
            int v = wrt[t];
            int r = rank[v];
            const int64_t* ix = leaf_idx + g.leaf_off[v];
            int64_t dim[64], st[64];
            for (int a = 0; a < r; a++) dim[a] = idx_dim[ix[a]];
            row_major_strides(r, dim, st);
            int64_t base = 0;
            int64_t nst[64];
            int nr = 0;
            for (int a = 0; a < r; a++) {
                if (g.is_sliced[ix[a]]) base += sval[ix[a]] * st[a];
                else nst[nr++] = st[a];
            }
            const otensor* c = &cot[v];
            int64_t val[64] = {0};
            for (int64_t o = 0; o < c->size; o++) {
                int64_t dst = base;
                for (int a = 0; a < nr; a++) dst += val[a] * nst[a];
                grads[t][2 * dst] += c->data[2 * o];
                grads[t][2 * dst + 1] += c->data[2 * o + 1];
                for (int a = nr - 1; a >= 0; a--) {
                    if (++val[a] < c->dim[a]) break;
                    val[a] = 0;
                }
            }
        }
        for (int v = 0; v < nn; v++) {
            ot_free(&vals[v]);
            ot_free(&cot[v]);
        }
    }
    if (vals) for (int v = 0; v < nn; v++) ot_free(&vals[v]);
    if (cot) for (int v = 0; v < nn; v++) ot_free(&cot[v]);
    free(vals);
    free(cot);
    free(sval);
    onet_free(&g);
    return rc;
}

/*
 * Width and cost of the tree with the sliced indices removed (eqs. edgecon
 * and vertexcon): W = max over all nodes of sum_{e in s_v} log2 |D(e)|,
 * log2 C with C = sum over internal nodes of prod_{e in s_l U s_r} |D(e)|.
 */
int oracle_width_cost(int32_t n_leaves, const int32_t* rank, const int64_t* leaf_idx,
                      int32_t n_idx, const int64_t* idx_dim, int32_t n_out, const int64_t* out_idx,
                      const int32_t* left, const int32_t* right, int32_t n_sliced,
                      const int64_t* sliced_idx, double* W, double* C) {
    onet g;
    if (onet_build(&g, n_leaves, rank, leaf_idx, n_idx, idx_dim, n_out, out_idx, left, right,
                   n_sliced, sliced_idx)) {
        onet_free(&g);
        return -1;
    }
    double w = 0.0, c = 0.0;
    for (int v = 0; v < 2 * n_leaves - 1; v++) {
        double sz = 1.0;
        for (int a = 0; a < g.n_kept[v]; a++) sz *= (double)idx_dim[g.kept[v][a]];
        if (sz > w) w = sz;
        if (v >= n_leaves) {
            int l = left[v - n_leaves], r = right[v - n_leaves];
            double u = 1.0;
            int64_t seen[256];
            int nseen = 0;
            if (g.n_kept[l] + g.n_kept[r] > 256) { onet_free(&g); return fail("node rank too large"); }
            for (int pass = 0; pass < 2; pass++) {
                int ch = pass == 0 ? l : r;
                for (int a = 0; a < g.n_kept[ch]; a++) {
                    int64_t e = g.kept[ch][a];
                    if (pos_in(seen, nseen, e) >= 0) continue;
                    seen[nseen++] = e;
                    u *= (double)idx_dim[e];
                }
            }
            c += u;
        }
    }
    *W = w;   /* as a size: 2^W for |D| = 2 */
    *C = c;
    onet_free(&g);
    return 0;
}
