"""The largest tensors a plan accepts (2^31 elements after slicing; 2^32 is
rejected at plan time, tests/test_libtn_host.py) through the GPU path: a
pairwise contraction whose output holds 2^31 complex64 values (16 GiB in the
arena, 32 GiB as the complex128 sum) on each kernel class that can produce
it: the one-shot few-summed-values kernel, the streaming row kernel and the
matrix-core GEMM.  The output stays on the GPU; a seeded block of it is
compared with the oracle's contraction of the leaves restricted to that
block's rows and columns (complex64 within 1e-5 of the exact value of the same
complex64 leaves, normwise and max-componentwise)."""

import numpy as np
import pytest

from tests.gpu_util import TOL_C64, check, note
from tn_inputs.network import Network, Tree

pytestmark = pytest.mark.gpu

TWO = Tree(np.array([0], np.int32), np.array([1], np.int32))


def _c64(rng, n):
    return rng.standard_normal(2 * n, dtype=np.float32).view(np.complex64)


# (m, n, k, kernel class): A(M, K) x B(N, K) -> C(M, N), m + n = 31
CASES = [(15, 16, 1, "gemm_smallk_wide"), (27, 4, 0, "row_stream_kernel"), (15, 16, 5, None)]


@pytest.mark.parametrize("m,n,k,kernel", CASES)
def test_output_of_2_31_elements(oracle_lib, m, n, k, kernel):
    import torch

    from paper_2002_01935_amd.binding import Plan
    rng = np.random.default_rng(31 + m + n + k)
    a = _c64(rng, 2 ** (m + k))
    b = _c64(rng, 2 ** (n + k))
    M, K, N = list(range(m)), list(range(m, m + k)), list(range(m + k, m + k + n))
    # leaves as zero-stride views of the right shape for the planner (it reads
    # shapes only); the data goes to the GPU from the flat arrays
    net = Network([np.broadcast_to(np.zeros(1, np.complex64), (2,) * (m + k)),
                   np.broadcast_to(np.zeros(1, np.complex64), (2,) * (n + k))],
                  [M + K, N + K], [2] * (m + n + k), M + N)
    plan = Plan(net, TWO, precision="c64_4m")
    nodes = plan.nodes()
    note("maxsize", m, n, k, [nd["kernel"] for nd in nodes])
    if kernel is not None:
        assert [nd["kernel"] for nd in nodes] == [kernel]
    else:
        assert nodes[0]["kclass"].startswith("gemm") and nodes[0]["kernel"].startswith("gemm_mfma")
    assert plan.info()["W"] == 31
    leaves = [torch.from_numpy(a).to("cuda"), torch.from_numpy(b).to("cuda")]
    ws = plan.workspace()
    out = torch.empty(plan.out_shape, dtype=torch.complex128, device="cuda")
    plan.contract_sliced(leaves, out=out, workspace=ws)
    torch.cuda.synchronize()
    # a seeded block: 64 rows (all columns when there are at most 64) x 64 columns
    rows = np.sort(rng.choice(2 ** m, 64, replace=False))
    cols = np.arange(2 ** n) if n <= 6 else np.sort(rng.choice(2 ** n, 64, replace=False))
    got = out.view(2 ** m, 2 ** n)[torch.from_numpy(rows).to("cuda")][:, torch.from_numpy(cols).to("cuda")]
    got = got.cpu().numpy()
    del out, ws, leaves
    torch.cuda.empty_cache()
    a_blk = a.reshape(2 ** m, 2 ** k)[rows].astype(np.complex128)
    b_blk = b.reshape(2 ** n, 2 ** k)[cols].astype(np.complex128)
    # the block as its own network: C_blk[r][c] = sum_k A[r][k] B[c][k]
    if k:
        blk = Network([a_blk, b_blk], [[0, 1], [2, 1]], [len(rows), 2 ** k, len(cols)], [0, 2])
    else:
        blk = Network([a_blk[:, 0], b_blk[:, 0]], [[0], [1]], [len(rows), len(cols)], [0, 1])
    ref = oracle_lib.contract(blk, TWO)
    check(got.ravel(), np.asarray(ref).ravel(), TOL_C64, "maxsize", m, n, k)
