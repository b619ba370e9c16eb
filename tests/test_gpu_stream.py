"""The bandwidth kernels of write-bound nodes on the GPU (row_stream_kernel:
no row bit in B, at most four summed values; gemm_smallk_stream: a GEMM with
at most eight summed values whose fast side spans a wavefront, with eight
summed values, an operand larger than the L2 or fewer than 2^25 outputs;
gemm_smallk_wide: the same with at most four summed values and a small
fast-side operand, one-shot) at sizes where every persistent wavefront walks several
units (a ragged last pass included), against the oracle: complex64 within
1e-5 of the exact value of the same complex64 leaves (normwise and
max-componentwise), complex128 within 1e-10.  Each case asserts the kernel
that ran."""

import numpy as np
import pytest

from tests.gpu_util import TOL_C64, TOL_C128, c64_leaves, check, gpu_sliced, note
from tn_inputs.graphs import pairwise_network
from tn_inputs.network import Network, Tree

pytestmark = pytest.mark.gpu

TWO = Tree(np.array([0], np.int32), np.array([1], np.int32))


def _rows(m, n, k, seed):
    """A(M, K) x B(N, K) -> C(M, N), output in index order: the in-thread
    bits N lowest in C, the row bits M above them (contiguous row blocks)."""
    M, K, N = list(range(m)), list(range(m, m + k)), list(range(m + k, m + k + n))
    rng = np.random.default_rng(seed)
    a = rng.normal(size=(2,) * (m + k)) + 1j * rng.normal(size=(2,) * (m + k))
    b = rng.normal(size=(2,) * (n + k)) + 1j * rng.normal(size=(2,) * (n + k))
    return Network([a, b], [M + K, N + K], [2] * (m + n + k), M + N)


def _run(net, prec, kernel, oracle_lib, sliced=(), inflight=0):
    from paper_2002_01935_amd.binding import Plan
    plan = Plan(net, TWO, sliced=list(sliced), precision=prec, max_inflight_slices=inflight)
    names = [nd["kernel"] for nd in plan.nodes()]
    note("stream", prec, kernel, names, "sliced", list(sliced), "in flight", inflight)
    assert names == [kernel], names
    ref = oracle_lib.contract(net if prec == "c128" else c64_leaves(net), TWO)
    got = gpu_sliced(net, TWO, sliced=list(sliced), precision=prec, plan=plan)
    check(got.ravel(), ref.ravel(), TOL_C128 if prec == "c128" else TOL_C64, "stream", prec, kernel)


# (m, n, k): 2^m rows, 2^n in-thread values, 2^k summed values; 2^(m - 7)
# units of two 64-row blocks against 4096 wavefronts (16 per compute unit)
ROWS = [(20, 4, 0), (21, 2, 2), (21, 3, 1), (22, 0, 1), (19, 1, 2), (13, 4, 0)]


@pytest.mark.parametrize("prec", ["c64_4m", "c128"])
@pytest.mark.parametrize("shape", ROWS)
def test_row_stream(oracle_lib, shape, prec):
    _run(_rows(*shape, seed=sum(shape)), prec, "row_stream_kernel", oracle_lib)


@pytest.mark.parametrize("prec", ["c64_4m", "c128"])
def test_row_stream_sliced(oracle_lib, prec):
    """A summed index sliced: several slices in flight on the grid's second
    dimension, each walked by the persistent wavefronts."""
    net = _rows(20, 2, 2, seed=5)
    _run(net, prec, "row_stream_kernel", oracle_lib, sliced=[20], inflight=2)


# (h, m, n, k): GEMM class by default (h + m + n + k >= 25), random axis
# orders; fast-side operands of at most 2^(13 + 2) values and at least 2^25
# outputs per batch index: one-shot variant
SMALLK = [(0, 13, 12, 0), (0, 12, 13, 2), (1, 13, 12, 1), (0, 13, 13, 1), (2, 12, 13, 2)]


@pytest.mark.parametrize("prec", ["c64_4m", "c128"])
@pytest.mark.parametrize("shape", SMALLK)
def test_smallk_wide(oracle_lib, shape, prec):
    net = pairwise_network(*shape, seed=7 * sum(shape) + 1, dims=(2,))
    _run(net, prec, "gemm_smallk_wide", oracle_lib)


# fewer outputs than the one-shot variant's threshold: streaming variant
SMALLK_SMALL = [(0, 12, 12, 1), (1, 11, 11, 2), (2, 10, 12, 1), (0, 12, 12, 3)]


@pytest.mark.parametrize("prec", ["c64_4m", "c128"])
@pytest.mark.parametrize("shape", SMALLK_SMALL)
def test_smallk_stream_small(oracle_lib, shape, prec):
    net = pairwise_network(*shape, seed=7 * sum(shape) + 1, dims=(2,))
    _run(net, prec, "gemm_smallk_stream", oracle_lib)


# eight summed values (the streaming variant whatever the operand size)
SMALLK_EIGHT = [(0, 13, 12, 3), (1, 12, 13, 3), (2, 11, 12, 3)]


@pytest.mark.parametrize("prec", ["c64_4m", "c128"])
@pytest.mark.parametrize("shape", SMALLK_EIGHT)
def test_smallk_stream_eight(oracle_lib, shape, prec):
    net = pairwise_network(*shape, seed=7 * sum(shape) + 3, dims=(2,))
    _run(net, prec, "gemm_smallk_stream", oracle_lib)


# (m, n, k) of A(M, K) x B(N, K) -> C(M, N) with N lowest in C: the fast side
# N's operand holds 2^(n + k) >= 2^20 values (at least 8 MiB), more than the
# one-shot variant takes, so the streaming variant runs (one to eight summed
# values)
SMALLK_BIG = [(6, 20, 0), (5, 19, 2), (7, 18, 2), (6, 18, 3)]


@pytest.mark.parametrize("prec", ["c64_4m", "c128"])
@pytest.mark.parametrize("shape", SMALLK_BIG)
def test_smallk_stream(oracle_lib, shape, prec):
    _run(_rows(*shape, seed=11 + sum(shape)), prec, "gemm_smallk_stream", oracle_lib)


@pytest.mark.parametrize("prec", ["c64_4m", "c128"])
def test_smallk_wide_sliced(oracle_lib, prec):
    """One of two summed indices sliced, both slices in flight on the grid's
    second dimension: each slice is a (2^13, 2^13, 2) node on the one-shot
    kernel, the slices' roots summed in FP64."""
    net = _rows(13, 13, 2, seed=9)
    _run(net, prec, "gemm_smallk_wide", oracle_lib, sliced=[14], inflight=2)


@pytest.mark.parametrize("prec", ["c64_3m", "c64_bf16x3"])
@pytest.mark.parametrize("shape,kernel", [((0, 13, 12, 1), "gemm_smallk_wide"), ((0, 13, 12, 3), "gemm_smallk_stream")])
def test_smallk_other_precisions(oracle_lib, shape, kernel, prec):
    """3M and BF16x3 plans send the same nodes to the few-summed-values
    kernels, which form plain FP32 products there: held to the complex64
    bound, not to the looser bounds of those precisions' GEMMs."""
    from paper_2002_01935_amd.binding import Plan
    net = pairwise_network(*shape, seed=7 * sum(shape) + 5, dims=(2,))
    plan = Plan(net, TWO, precision=prec)
    names = [nd["kernel"] for nd in plan.nodes()]
    note("smallk", prec, shape, names)
    assert names == [kernel], names
    ref = oracle_lib.contract(c64_leaves(net), TWO)
    got = gpu_sliced(net, TWO, precision=prec, plan=plan)
    check(got.ravel(), ref.ravel(), TOL_C64, "smallk", prec, kernel)
