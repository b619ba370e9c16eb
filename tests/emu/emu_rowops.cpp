// Host build of the row / split-K / reduce kernels (csrc/rowops.h) and of the
// few-summed-values GEMM kernel (csrc/smallk_kernel.h) with
// stand-ins for the HIP names they use, driven by the real planner
// (csrc/plan.cpp): plans a network read from a text file, runs the forward
// program's ops on the CPU (one host thread per lane for split-K wavefronts,
// whose lane sums need the cross-lane shuffle), and writes the root of each
// requested slice.  Test infrastructure: used by tests/test_kernel_emulation.py.
//
// usage: emu_rowops NET.txt LEAVES.bin OUT.bin [FLAGS]
//   NET.txt: n_leaves n_idx n_out prec / ranks / leaf indices / dims / out / left / right /
//            n_sliced sliced... / n_ids ids...
//   LEAVES.bin: complex128 leaves, row-major; OUT.bin: complex128 roots (out order), one per id
//   FLAGS: tn_options.flags of the plan (default 0), plus 0x10000: no one-shot
//          few-summed-values variant (the streaming one runs instead), 0x20000:
//          that variant whatever the output size
// exit code 3: the plan holds an op kind the emulator does not run (matrix-core GEMM)
// exit code 4: a few-summed-values GEMM op its launch preparation refused
#include <algorithm>
#include <barrier>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <complex>
#include <string>
#include <thread>
#include <type_traits>
#include <utility>
#include <vector>

#include "plan.h"
#include "smallk_rule.h"

struct float2 { float x, y; };
struct double2 { double x, y; };
struct Dim3 { unsigned x, y, z; };
static thread_local Dim3 threadIdx, blockIdx, blockDim, gridDim;
#define __global__
#define __device__
#define __forceinline__ inline
#define __launch_bounds__(x)
#define GMEM
#define __shared__ static
#define CMEM

static std::barrier<>* g_wave_barrier = nullptr;
// lanes of a wavefront run as host threads in lockstep at this point
#define TN_WAVE_SYNC() g_wave_barrier->arrive_and_wait()
// every lane holds the same value already
#define TN_UNIFORM(x) (x)
static double g_lane_value[64];
template <typename T>
static T __shfl_xor(T v, int mask, int) {
  const int l = threadIdx.x & 63;
  g_lane_value[l] = (double)v;
  g_wave_barrier->arrive_and_wait();
  const T r = (T)g_lane_value[l ^ mask];
  g_wave_barrier->arrive_and_wait();
  return r;
}

namespace tn {
#include "rowops.h"
#include "smallk_kernel.h"
}
using namespace tn;

// Steps per batch of loads, as the library's launcher picks them.
static int chunk_bits(const RowOp& op) {
  const int nin = 1 << op.n_in;
  const int kb = row_ku(nin) == 8 ? 3 : (row_ku(nin) == 4 ? 2 : 1);
  int ub;
  if (op.k_split_bits >= 0) ub = op.n_k - (op.k_split_bits > 0 ? op.k_split_bits : 0) - 6;
  else ub = op.pair_a ? op.n_k - 1 : op.n_k;
  return ub < kb ? ub : kb;
}

// the library's launcher picks the staged-store variant for complex64 ops
// that prepare_row marks
static bool staged(const RowOp& op, int eb) { return eb == 8 && op.stage_c; }

template <typename T, int NIN, int U>
static void call_row(bool stage, const Ctx& ctx, const RowOp& op) {
  if (stage) row_kernel<T, NIN, U, true>(ctx, op);
  else row_kernel<T, NIN, U>(ctx, op);
}

template <typename T, int NIN>
static void call_lane(bool splitk, int ub, const Ctx& ctx, const RowOp& op, bool stage = false) {
  constexpr int KU = row_ku(NIN);
  switch (ub) {
    case 0: if (splitk) splitk_kernel<T, NIN, 1>(ctx, op); else call_row<T, NIN, 1>(stage, ctx, op); break;
    case 1: if (splitk) splitk_kernel<T, NIN, 2>(ctx, op); else call_row<T, NIN, 2>(stage, ctx, op); break;
    case 2: if constexpr (KU >= 4) { if (splitk) splitk_kernel<T, NIN, 4>(ctx, op); else call_row<T, NIN, 4>(stage, ctx, op); } break;
    default: if constexpr (KU >= 8) { if (splitk) splitk_kernel<T, NIN, 8>(ctx, op); else call_row<T, NIN, 8>(stage, ctx, op); } break;
  }
}

template <typename T>
static void call_any(bool splitk, const Ctx& ctx, const RowOp& op, bool stage = false) {
  const int ub = chunk_bits(op);
  switch (op.n_in) {
    case 0: call_lane<T, 1>(splitk, ub, ctx, op, stage); break;
    case 1: call_lane<T, 2>(splitk, ub, ctx, op, stage); break;
    case 2: call_lane<T, 4>(splitk, ub, ctx, op, stage); break;
    case 3: call_lane<T, 8>(splitk, ub, ctx, op, stage); break;
    default: call_lane<T, 16>(splitk, ub, ctx, op, stage); break;
  }
}

// Runs fn() for every wavefront of a grid of `blocks` x `gy` workgroups of
// 256 threads, one wavefront at a time, its 64 lanes as host threads in
// lockstep (the kernels' wavefront syncs are barriers among them).
template <class Fn>
static void run_waves(unsigned blocks, unsigned gy, Fn fn) {
  std::barrier<> bar(64);
  g_wave_barrier = &bar;
  std::vector<std::thread> lanes;
  for (int l = 0; l < 64; l++)
    lanes.emplace_back([&, l] {
      for (unsigned y = 0; y < gy; y++)
        for (unsigned b = 0; b < blocks; b++)
          for (unsigned w = 0; w < 4; w++) {
            blockDim = {256, 1, 1};
            gridDim = {blocks, gy, 1};
            blockIdx = {b, y, 0};
            threadIdx = {w * 64 + l, 0, 0};
            fn();
            bar.arrive_and_wait();
          }
    });
  for (auto& t : lanes) t.join();
}

// The streaming row kernel in each of its store modes and unit sizes that
// apply, on one workgroup (four persistent wavefronts walk all row blocks).
template <typename T, int NIN>
static void run_row_stream_n(const Ctx& ctx, const RowOp& op, int z) {
  const RowKOffsets ko = row_k_offsets(op);
  const bool contiguous = op.stage_c && sizeof(T) == 4 && NIN >= 2;
  // every variant writes all of C: each one's result is checked against the
  // first one's (a variant that misplaced a value would otherwise be hidden
  // by the next one overwriting it)
  const size_t n_c = (size_t(1) << (op.n_rows + op.n_in)) * 2;
  const int64_t sid = slice_id(ctx, z);
  T* Cv = reinterpret_cast<T*>(resolve(ctx, op.c, z, sid, sizeof(T) * 2));
  std::vector<T> first;
  auto go = [&](auto kn) {
    constexpr int KN = decltype(kn)::value;
    auto one = [&](auto mode, auto rb) {
      constexpr int M = decltype(mode)::value, RB = decltype(rb)::value;
      std::fill(Cv, Cv + n_c, T(12345));
      run_waves(1, 1, [&] {
        blockIdx.y = z;
        row_stream_kernel<T, NIN, KN, M, RB>(ctx, op, ko);
      });
      if (first.empty()) {
        first.assign(Cv, Cv + n_c);
        return;
      }
      double scale = 0;
      for (size_t i = 0; i < n_c; i++) scale = std::max(scale, std::abs((double)first[i]));
      for (size_t i = 0; i < n_c; i++)
        if (std::abs((double)Cv[i] - (double)first[i]) > 1e-6 * scale) {
          fprintf(stderr, "streaming row variant mode %d rb %d differs at %zu\n", M, RB, i);
          exit(5);
        }
    };
    auto modes = [&](auto rb) {
      if constexpr (sizeof(T) == 4 && NIN >= 2)
        if (contiguous) {
          one(std::integral_constant<int, 1>(), rb);
          one(std::integral_constant<int, 2>(), rb);
        }
      one(std::integral_constant<int, 0>(), rb);
    };
    modes(std::integral_constant<int, 1>());
    if (op.n_rows >= 7) modes(std::integral_constant<int, 2>());
  };
  if (op.n_k == 0) go(std::integral_constant<int, 1>());
  else if constexpr (NIN <= 8) {
    if (op.n_k == 1) go(std::integral_constant<int, 2>());
    else if constexpr (NIN <= 4) go(std::integral_constant<int, 4>());
  }
}

template <typename T>
static void run_row_stream(const Ctx& ctx, const RowOp& op, int z) {
  switch (op.n_in) {
    case 0: run_row_stream_n<T, 1>(ctx, op, z); break;
    case 1: run_row_stream_n<T, 2>(ctx, op, z); break;
    case 2: run_row_stream_n<T, 4>(ctx, op, z); break;
    case 3: run_row_stream_n<T, 8>(ctx, op, z); break;
    default: run_row_stream_n<T, 16>(ctx, op, z); break;
  }
}

static int g_stream_ops = 0;   // streaming launches run (reported on stderr)
static int g_wide_ops = 0;     // one-shot few-summed-values launches run (reported on stderr)
// FLAGS bits of the emulator itself (not plan flags): leave out the one-shot
// few-summed-values variant, so that small test operands reach the streaming
// one; or run it whatever the output size
constexpr uint32_t kEmuNoWide = 0x10000, kEmuWideAnySize = 0x20000;
static int g_wide_rule = kWideDefault;

template <typename T>
static void run_row(const Ctx& ctx, const RowOp& op, int z) {
  if (row_stream_ok(op)) {
    g_stream_ops++;
    run_row_stream<T>(ctx, op, z);
    return;
  }
  const uint64_t rows = 1ull << op.n_rows;
  const unsigned nblk = (unsigned)((rows + kRowThreads - 1) / kRowThreads);
  if (staged(op, sizeof(T) * 2)) {
    // lanes exchange values through LDS: run each wavefront's lanes together
    const int64_t waves = (int64_t)nblk * (kRowThreads / 64);
    std::barrier<> bar(64);
    g_wave_barrier = &bar;
    std::vector<std::thread> lanes;
    for (int l = 0; l < 64; l++)
      lanes.emplace_back([&, l] {
        for (int64_t w = 0; w < waves; w++) {
          blockDim = {(unsigned)kRowThreads, 1, 1};
          blockIdx = {(unsigned)(w / (kRowThreads / 64)), (unsigned)z, 0};
          threadIdx = {(unsigned)((w % (kRowThreads / 64)) * 64 + l), 0, 0};
          call_any<T>(false, ctx, op, true);
          bar.arrive_and_wait();
        }
      });
    for (auto& t : lanes) t.join();
    return;
  }
  for (unsigned b = 0; b < nblk; b++)
    for (unsigned t = 0; t < (unsigned)kRowThreads; t++) {
      blockDim = {(unsigned)kRowThreads, 1, 1};
      blockIdx = {b, (unsigned)z, 0};
      threadIdx = {t, 0, 0};
      call_any<T>(false, ctx, op);
    }
}

// 64 host threads play the lanes of one wavefront at a time; the shuffles
// and the end of each wavefront synchronise them.
template <typename T>
static void run_splitk(const Ctx& ctx, const RowOp& op, int64_t waves, int z) {
  const int wpb = kRowThreads / 64;
  std::barrier<> bar(64);
  g_wave_barrier = &bar;
  std::vector<std::thread> lanes;
  for (int l = 0; l < 64; l++)
    lanes.emplace_back([&, l] {
      for (int64_t w = 0; w < waves; w++) {
        blockDim = {(unsigned)kRowThreads, 1, 1};
        blockIdx = {(unsigned)(w / wpb), (unsigned)z, 0};
        threadIdx = {(unsigned)((w % wpb) * 64 + l), 0, 0};
        call_any<T>(true, ctx, op);
        bar.arrive_and_wait();
      }
    });
  for (auto& t : lanes) t.join();
}

template <typename T>
static void run_reduce(const Ctx& ctx, const RowOp& op, int z) {
  const int64_t waves = int64_t(1) << (op.n_rows + op.n_in);
  const int wpb = kRowThreads / 64;
  std::barrier<> bar(64);
  g_wave_barrier = &bar;
  std::vector<std::thread> lanes;
  for (int l = 0; l < 64; l++)
    lanes.emplace_back([&, l] {
      for (int64_t w = 0; w < waves; w++) {
        blockDim = {(unsigned)kRowThreads, 1, 1};
        blockIdx = {(unsigned)(w / wpb), (unsigned)z, 0};
        threadIdx = {(unsigned)((w % wpb) * 64 + l), 0, 0};
        reduce_kernel<T>(ctx, op);
        bar.arrive_and_wait();
      }
    });
  for (auto& t : lanes) t.join();
}

// One launch of the few-summed-values GEMM kernel, in the variant the
// library's launcher picks: the plain and one-shot kernels thread by thread
// (they have no cross-lane step), the streaming one on one workgroup per grid
// row (four persistent wavefronts walk all units).
static bool run_smallk(const Ctx& ctx, const GemmOp& in, int prec) {
  GemmOp op = in;
  SmallkTables kt;
  SmallkLaunch L;
  if (!smallk_prepare(op, prec, ctx.n_batch, kt, L, g_wide_rule)) return false;
  smallk_dispatch(L, prec, [&](auto t, auto fastn, auto p, auto kn, auto variant) {
    using T = decltype(t);
    constexpr bool FN = decltype(fastn)::value;
    constexpr int P = decltype(p)::value, KN = decltype(kn)::value, VAR = decltype(variant)::value;
    if constexpr (VAR == kSmallkStream) {
      g_stream_ops++;
      run_waves(1, (unsigned)L.gy, [&] { gemm_smallk_stream<T, FN, P, KN>(ctx, op, kt); });
    } else if constexpr (VAR == kSmallkWide) {
      // no cross-lane step: thread by thread, over the launcher's grid
      if constexpr (KN <= kWideMaxSummed) {
        g_wide_ops++;
        blockDim = {256, 1, 1};
        gridDim = {(unsigned)((L.units + 3) / 4), (unsigned)L.gy, 1};
        for (uint64_t y = 0; y < L.gy; y++)
          for (uint64_t x = 0; x < gridDim.x; x++)
            for (unsigned th = 0; th < 256; th++) {
              blockIdx = {(unsigned)x, (unsigned)y, 0};
              threadIdx = {th, 0, 0};
              gemm_smallk_wide<T, FN, P, KN>(ctx, op, kt);
            }
      }
    } else {
      blockDim = {256, 1, 1};
      gridDim = {(unsigned)L.blocks, (unsigned)L.gy, 1};
      for (uint64_t y = 0; y < L.gy; y++)
        for (uint64_t x = 0; x < L.blocks; x++)
          for (unsigned th = 0; th < 256; th++) {
            blockIdx = {(unsigned)x, (unsigned)y, 0};
            threadIdx = {th, 0, 0};
            gemm_smallk<T, FN, P, kSmallkRows, KN>(ctx, op, kt);
          }
    }
  });
  return true;
}

int main(int argc, char** argv) {
  if (argc != 4 && argc != 5) return 1;
  FILE* f = fopen(argv[1], "r");
  if (!f) return 1;
  int nl, nidx, nout, prec;
  if (fscanf(f, "%d %d %d %d", &nl, &nidx, &nout, &prec) != 4) return 1;
  tn_plan_s* p = new tn_plan_s();
  p->n_leaves = nl;
  p->n_idx = nidx;
  p->n_out = nout;
  int tot = 0;
  for (int v = 0; v < nl; v++) { int r; fscanf(f, "%d", &r); p->rank.push_back(r); tot += r; }
  for (int i = 0; i < tot; i++) { long x; fscanf(f, "%ld", &x); p->leaf_idx.push_back(x); }
  for (int i = 0; i < nidx; i++) { long x; fscanf(f, "%ld", &x); p->idx_dim.push_back(x); }
  for (int i = 0; i < nout; i++) { long x; fscanf(f, "%ld", &x); p->out_idx.push_back(x); }
  for (int i = 0; i < nl - 1; i++) { int x; fscanf(f, "%d", &x); p->left.push_back(x); }
  for (int i = 0; i < nl - 1; i++) { int x; fscanf(f, "%d", &x); p->right.push_back(x); }
  int ns;
  fscanf(f, "%d", &ns);
  p->n_sliced = ns;
  for (int i = 0; i < ns; i++) { long x; fscanf(f, "%ld", &x); p->sliced.push_back(x); }
  int nids;
  fscanf(f, "%d", &nids);
  std::vector<int64_t> ids(nids);
  for (int i = 0; i < nids; i++) { long x; fscanf(f, "%ld", &x); ids[i] = x; }
  fclose(f);
  p->opt.prec = (tn_precision)prec;
  const uint32_t flags = argc == 5 ? (uint32_t)strtoul(argv[4], nullptr, 0) : 0u;
  g_wide_rule = (flags & kEmuNoWide) ? kWideNever : ((flags & kEmuWideAnySize) ? kWideAnySize : kWideDefault);
  p->opt.flags = flags & ~(kEmuNoWide | kEmuWideAnySize);
  p->prec = p->opt.prec;
  p->elem_bytes = prec == TN_C128 ? 16 : 8;
  std::string err;
  if (build_plan(p, err)) { fprintf(stderr, "plan: %s\n", err.c_str()); return 2; }
  for (const Op& op : p->fwd)
    if (op.kind != OpKind::Row && op.kind != OpKind::RowReduce && !(op.kind == OpKind::Gemm && gemm_smallk_ok(op.gemm)))
      return 3;
  const int eb = p->elem_bytes;
  // leaves, each in its own exactly sized buffer
  std::vector<std::vector<char>> leaves(nl);
  FILE* fb = fopen(argv[2], "rb");
  int off = 0;
  for (int v = 0; v < nl; v++) {
    size_t n = 1;
    for (int i = 0; i < p->rank[v]; i++) n *= p->idx_dim[p->leaf_idx[off + i]];
    off += p->rank[v];
    std::vector<std::complex<double>> buf(n);
    if (fread(buf.data(), 16, n, fb) != n) return 1;
    leaves[v].resize(n * eb);
    for (size_t i = 0; i < n; i++) {
      if (eb == 8) {
        float* q = reinterpret_cast<float*>(leaves[v].data());
        q[2 * i] = (float)buf[i].real();
        q[2 * i + 1] = (float)buf[i].imag();
      } else {
        double* q = reinterpret_cast<double*>(leaves[v].data());
        q[2 * i] = buf[i].real();
        q[2 * i + 1] = buf[i].imag();
      }
    }
  }
  fclose(fb);
  std::vector<char> ws(p->arena_off + p->arena_bytes + 512);
  char* base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(ws.data()) + 255) & ~uintptr_t(255));
  uint64_t* tab = reinterpret_cast<uint64_t*>(base + p->ptrtab_off);
  for (int v = 0; v < nl; v++) tab[v] = reinterpret_cast<uint64_t>(leaves[v].data());
  Ctx ctx;
  std::memset(&ctx, 0, sizeof ctx);
  ctx.ws = reinterpret_cast<uint64_t>(base);
  ctx.arena_stride = p->arena_bytes;
  ctx.ptrtab_off = p->ptrtab_off;
  ctx.sid_off = p->sid_off;
  ctx.counter_off = p->counter_off;
  ctx.arena_off = p->arena_off;
  ctx.n_batch = 1;
  ctx.elem_bytes = eb;
  size_t nout_el = 1;
  for (int i = 0; i < nout; i++) nout_el *= p->idx_dim[p->out_idx[i]];
  FILE* fo = fopen(argv[3], "wb");
  for (int64_t sid : ids) {
    *reinterpret_cast<int64_t*>(base + p->counter_off) = 0;
    *reinterpret_cast<int64_t*>(base + p->sid_off) = sid;
    for (const Op& op : p->fwd) {
      if (op.kind == OpKind::Gemm) {
        if (!run_smallk(ctx, op.gemm, prec)) return 4;
        continue;
      }
      RowOp r = op.row;                       // launch-time tables, as the library's launchers fill them
      prepare_row(r);
      if (op.kind == OpKind::RowReduce) {
        if (eb == 8) run_reduce<float>(ctx, r, 0); else run_reduce<double>(ctx, r, 0);
      } else if (r.k_split_bits >= 0) {
        if (eb == 8) run_splitk<float>(ctx, r, op.grid_rows, 0); else run_splitk<double>(ctx, r, op.grid_rows, 0);
      } else {
        if (eb == 8) run_row<float>(ctx, r, 0); else run_row<double>(ctx, r, 0);
      }
    }
    const char* root = base + p->arena_off + p->root_off;
    for (size_t i = 0; i < nout_el; i++) {
      double re, im;
      if (eb == 8) { re = reinterpret_cast<const float*>(root)[2 * i]; im = reinterpret_cast<const float*>(root)[2 * i + 1]; }
      else { re = reinterpret_cast<const double*>(root)[2 * i]; im = reinterpret_cast<const double*>(root)[2 * i + 1]; }
      fwrite(&re, 8, 1, fo);
      fwrite(&im, 8, 1, fo);
    }
  }
  fclose(fo);
  delete p;
  fprintf(stderr, "streaming launches: %d\n", g_stream_ops);
  fprintf(stderr, "one-shot launches: %d\n", g_wide_ops);
  return 0;
}
