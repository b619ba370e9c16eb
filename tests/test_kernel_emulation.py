"""The bandwidth-class kernels (row, split-K and its reduction: csrc/rowops.h;
the few-summed-values GEMM: csrc/smallk_kernel.h) compiled for the host with stand-ins for the HIP names they use and run on
the CPU by tests/emu/emu_rowops.cpp, driven by the real planner, against the
oracle.  This checks their operand addressing (bit-permuted layouts, paired
accesses, summed-index walks whose order differs between the operands,
split-K chunking, slice offsets) without a GPU; the build uses
AddressSanitizer, so an out-of-bounds leaf access fails the test."""

import os
import shutil
import subprocess

import numpy as np
import pytest

from tn_inputs.graphs import pairwise_network
from tn_inputs.network import Tree

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang++"
TWO = Tree(np.array([0], np.int32), np.array([1], np.int32))
PREC = {"c64_4m": 0, "c128": 3}
TOL = {"c64_4m": 1e-5, "c128": 1e-12}


@pytest.fixture(scope="module")
def emu(tmp_path_factory):
    if not os.path.exists(CLANG) and shutil.which("clang++") is None:
        pytest.skip("no clang++ for the host build")
    cxx = CLANG if os.path.exists(CLANG) else shutil.which("clang++")
    out = str(tmp_path_factory.mktemp("emu") / "emu_rowops")
    csrc = os.path.join(ROOT, "paper_2002_01935_amd", "csrc")
    cmd = [cxx, "-O2", "-g", "-std=c++20", "-fsanitize=address", "-I", csrc, "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "emu", "emu_rowops.cpp"), os.path.join(csrc, "plan.cpp"), "-o", out,
           "-lpthread"]
    subprocess.run(cmd, check=True, capture_output=True)
    return out


def run(emu, net, prec, sliced=(), ids=(0,), tmp=None, streams=None, gemm_all_sizes=False, wides=None,
        no_wide=False, wide_any_size=False):
    """Root values of the emulated plan; `streams`, a list, receives the
    number of launches that took a streaming (persistent) kernel, `wides`
    the number that took the one-shot few-summed-values kernel.
    gemm_all_sizes: GEMM-shaped contractions of any size take the GEMM class
    (the plan flag TN_FLAG_GEMM_ALL_SIZES), so that small test networks reach
    the few-summed-values kernel.  no_wide: that kernel's streaming variant
    runs where the one-shot one would; wide_any_size: the one-shot variant
    runs on outputs under its size threshold too."""
    d = tmp
    with open(os.path.join(d, "net.txt"), "w") as f:
        f.write(f"{net.n_leaves} {len(net.idx_dim)} {len(net.out_idx)} {PREC[prec]}\n")
        f.write(" ".join(str(len(t)) for t in net.leaf_idx) + "\n")
        f.write(" ".join(str(i) for t in net.leaf_idx for i in t) + "\n")
        f.write(" ".join(str(x) for x in net.idx_dim) + "\n")
        f.write(" ".join(str(x) for x in net.out_idx) + "\n0\n1\n")
        f.write(f"{len(sliced)} " + " ".join(str(x) for x in sliced) + "\n")
        f.write(f"{len(ids)} " + " ".join(str(x) for x in ids) + "\n")
    with open(os.path.join(d, "leaves.bin"), "wb") as f:
        for t in net.leaves:
            np.ascontiguousarray(t, dtype=np.complex128).tofile(f)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    args = [emu, os.path.join(d, "net.txt"), os.path.join(d, "leaves.bin"), os.path.join(d, "out.bin")]
    flags = (1 if gemm_all_sizes else 0) | (0x10000 if no_wide else 0) | (0x20000 if wide_any_size else 0)
    if flags:
        args.append(str(flags))
    r = subprocess.run(args, capture_output=True, text=True, env=env)
    if r.returncode == 3:
        return None
    assert r.returncode == 0, r.stderr[-2000:]
    if streams is not None:
        streams.append(int(r.stderr.split("streaming launches:")[1].split()[0]))
    if wides is not None:
        wides.append(int(r.stderr.split("one-shot launches:")[1].split()[0]))
    return np.fromfile(os.path.join(d, "out.bin"), dtype=np.complex128)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# (h, m, n, k): row kernel with 1..16 in-thread outputs, summed walks of 0..5
# bits (paired and unpaired A accesses), batch bits; split-K with short and
# long chunks
ROW = [(0, 3, 2, 0), (0, 10, 2, 3), (0, 10, 1, 3), (0, 10, 0, 3), (0, 9, 4, 2), (3, 2, 2, 2), (0, 10, 3, 5),
       (2, 8, 4, 5), (1, 8, 0, 1), (0, 7, 2, 4)]
SPLITK = [(0, 0, 0, 10), (0, 2, 2, 8), (0, 4, 2, 7), (3, 0, 0, 8), (1, 4, 2, 9), (0, 1, 1, 13), (0, 8, 0, 6)]


@pytest.mark.parametrize("prec", ["c64_4m", "c128"])
@pytest.mark.parametrize("shape", ROW + SPLITK)
def test_pairwise_emulated(emu, oracle_lib, tmp_path, shape, prec):
    for seed in range(2):
        net = pairwise_network(*shape, seed=1000 + 17 * seed + sum(shape), dims=(2, 4))
        got = run(emu, net, prec, tmp=str(tmp_path))
        assert got is not None, "plan uses a matrix-core GEMM; pick a smaller free side"
        ref = oracle_lib.contract(net, TWO).ravel()
        assert rel(got, ref) < TOL[prec], (shape, prec, seed)


# (h, m, n, k): GEMM-class contractions with at most three summed bits (outer
# products included), which take the few-summed-values kernel
SMALLK = [(0, 5, 5, 1), (2, 6, 5, 2), (1, 5, 7, 0), (0, 7, 5, 2), (3, 5, 5, 1), (0, 6, 6, 0), (0, 5, 6, 3), (1, 5, 5, 3)]


@pytest.mark.parametrize("prec", ["c64_4m", "c128"])
@pytest.mark.parametrize("shape", SMALLK)
def test_smallk_emulated(emu, oracle_lib, tmp_path, shape, prec):
    """gemm_smallk on the host (csrc/smallk_kernel.h) with random axis orders:
    either free side may hold C's lowest bit, with and without the paired
    16-byte stores, batch bits and conjugation-free operands."""
    for seed in range(3):
        net = pairwise_network(*shape, seed=2000 + 31 * seed + sum(shape), dims=(2, 4))
        got = run(emu, net, prec, tmp=str(tmp_path), gemm_all_sizes=True)
        assert got is not None, "plan uses a matrix-core GEMM"
        ref = oracle_lib.contract(net, TWO).ravel()
        assert rel(got, ref) < TOL[prec], (shape, prec, seed)


def _canonical_rows(m, n, k, seed):
    """A(M, K) x B(N, K) -> C(M, N) with C's free-right bits lowest and the
    row bits right above them (the row kernel's staged-store layout)."""
    M, K, N = list(range(m)), list(range(m, m + k)), list(range(m + k, m + k + n))
    rng = np.random.default_rng(seed)
    a = rng.normal(size=(2,) * (m + k)) + 1j * rng.normal(size=(2,) * (m + k))
    b = rng.normal(size=(2,) * (n + k)) + 1j * rng.normal(size=(2,) * (n + k))
    from tn_inputs.network import Network
    return Network([a, b], [M + K, N + K], [2] * (m + n + k), M + N)


@pytest.mark.parametrize("shape", [(9, 1, 2), (10, 2, 1), (8, 3, 0), (8, 4, 2), (6, 2, 3)])
def test_staged_rows_emulated(emu, oracle_lib, tmp_path, shape):
    """Row kernel with the output transposed through LDS (64 rows of a
    wavefront stored as one block)."""
    net = _canonical_rows(*shape, seed=sum(shape))
    got = run(emu, net, "c64_4m", tmp=str(tmp_path))
    assert got is not None
    assert rel(got, oracle_lib.contract(net, TWO).ravel()) < TOL["c64_4m"]


@pytest.mark.parametrize("prec", ["c64_4m", "c128"])
def test_sliced_emulated(emu, oracle_lib, tmp_path, prec):
    """Slices fixed by the per-leaf slice offsets: the sum of the per-slice
    roots equals the unsliced contraction."""
    for shape in ((0, 9, 2, 4), (0, 2, 1, 12)):
        net = pairwise_network(*shape, seed=77 + sum(shape), dims=(2, 4))
        summed = [e for e in range(len(net.idx_dim)) if e not in net.out_idx]
        sliced = summed[:2]
        d = int(np.prod([net.idx_dim[e] for e in sliced]))
        got = run(emu, net, prec, sliced=sliced, ids=list(range(d)), tmp=str(tmp_path))
        assert got is not None
        got = got.reshape(d, -1)
        ref = oracle_lib.contract(net, TWO).ravel()
        assert rel(got.sum(axis=0), ref) < TOL[prec]
        for s in (0, d - 1):
            assert rel(got[s], oracle_lib.contract(net, TWO, sliced=sliced, slice_ids=[s]).ravel()) < TOL[prec]


@pytest.mark.parametrize("shape", [(9, 1, 2), (10, 4, 0), (8, 2, 1), (11, 0, 2), (8, 3, 1), (6, 2, 0)])
def test_stream_rows_emulated(emu, oracle_lib, tmp_path, shape):
    """The streaming row kernel (no row bit in B, at most four summed values):
    four persistent wavefronts walk every block of 64 rows, the next block's
    A values loaded before the current stores; staged and plain stores."""
    net = _canonical_rows(*shape, seed=3 + sum(shape))
    streams = []
    got = run(emu, net, "c64_4m", tmp=str(tmp_path), streams=streams)
    assert streams[0] >= 1
    assert rel(got, oracle_lib.contract(net, TWO).ravel()) < TOL["c64_4m"]
    got = run(emu, net, "c128", tmp=str(tmp_path))
    assert rel(got, oracle_lib.contract(net, TWO).ravel()) < TOL["c128"]


# (h, m, n, k): few-summed-values GEMMs whose fast side spans a wavefront,
# which take the streaming variant
SMALLK_STREAM = [(0, 8, 7, 2), (0, 7, 9, 0), (1, 8, 6, 1), (2, 7, 7, 2), (0, 9, 5, 1), (0, 8, 7, 3)]


@pytest.mark.parametrize("prec", ["c64_4m", "c128"])
@pytest.mark.parametrize("shape", SMALLK_STREAM)
def test_smallk_stream_emulated(emu, oracle_lib, tmp_path, shape, prec):
    """gemm_smallk_stream on the host: persistent wavefronts over units of 64
    fast-side lanes x 32 rows, the shared operand's values broadcast through
    LDS, random axis orders (either side fast, paired and single stores)."""
    n_stream = 0
    for seed in range(3):
        net = pairwise_network(*shape, seed=4000 + 31 * seed + sum(shape), dims=(2,))
        streams = []
        got = run(emu, net, prec, tmp=str(tmp_path), streams=streams, gemm_all_sizes=True, no_wide=True)
        assert got is not None, "plan uses a matrix-core GEMM"
        n_stream += streams[0]
        ref = oracle_lib.contract(net, TWO).ravel()
        assert rel(got, ref) < TOL[prec], (shape, prec, seed)
    assert n_stream >= 1


# (h, m, n, k): few-summed-values GEMMs whose fast side spans the one-shot
# variant's pieces (small operands)
SMALLK_WIDE = [(0, 9, 9, 2), (0, 10, 5, 1), (1, 9, 6, 0), (0, 5, 10, 2), (2, 9, 9, 1)]


@pytest.mark.parametrize("prec", ["c64_4m", "c128"])
@pytest.mark.parametrize("shape", SMALLK_WIDE)
def test_smallk_wide_emulated(emu, oracle_lib, tmp_path, shape, prec):
    """gemm_smallk_wide on the host (below its output-size threshold): each
    wavefront writes a few consecutive 64-lane pieces of one to four rows of
    the shared index; random axis orders (either side fast, paired and single
    stores), batch bits, one, two and four summed values."""
    n_wide = 0
    for seed in range(3):
        net = pairwise_network(*shape, seed=5000 + 31 * seed + sum(shape), dims=(2,))
        wides = []
        got = run(emu, net, prec, tmp=str(tmp_path), wides=wides, gemm_all_sizes=True, wide_any_size=True)
        assert got is not None, "plan uses a matrix-core GEMM"
        n_wide += wides[0]
        ref = oracle_lib.contract(net, TWO).ravel()
        assert rel(got, ref) < TOL[prec], (shape, prec, seed)
    assert n_wide >= 1
