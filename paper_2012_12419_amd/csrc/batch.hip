// batch.hip -- many independent instances of the occupancy MDP in one call
// (a parameter sweep over arrival rates and fleet sizes).
//
// Two execution forms share the Bellman backup of the single-instance sweep:
//
// * LDS-resident instances (two FP32 copies of V fit the workgroup's LDS):
//   one workgroup owns one instance for its whole solve.  It stages V^0 in
//   LDS, runs every Jacobi sweep LDS to LDS with a workgroup barrier between
//   sweeps and a workgroup max-reduction for the residual, and writes the
//   final iterate back once.  No sweep touches HBM, and the only
//   synchronisation is within the workgroup.  The grid is one persistent
//   launch over all such instances, ordered largest first so the hardware
//   dispatcher balances the tail.
//
// * Larger instances: a round kernel applies one sweep to every unfinished
//   large instance at once, 1024-occupancy tiles of all of them in one grid.
//   Each instance has its own stopping test, residual words and done flag;
//   the values of a sweep become visible to the next at the kernel boundary
//   (the L2 caches of the 8 XCDs are not coherent with each other inside a
//   kernel).  Rounds are enqueued in chunks; the host reads one counter of
//   unfinished instances per chunk.
//
// Fixed-policy evaluation (FP64) and the adjoint sweeps of every instance run
// in the round form; extraction, the greedy heuristic, the policy check and
// the gradient pass are one kernel over the tiles of all instances.
#include "batch.hpp"
#include "device.hpp"
#include "kernels.hpp"
#include "adjoint_impl.hpp"
#include "tile_eval.hpp"
#include "tile_vi.hpp"
#include "policy_impl.hpp"
#include "sweep_impl.hpp"

#include <type_traits>

namespace mdpvi {

// ---------------------------------------------------------------- LDS form

// The LDS-resident solve of one instance by the calling workgroup, with the
// backup of bounds KMAX, JMAX (KMAX = K and JMAX = J: exact loops).
template <int KMAX, int JMAX>
__device__ __forceinline__ void lds_solve(const BatchInst& I, int i, float* lds, double* part, float* V,
                                          double tol, long long max_iter, BatchOut* out) {
  const Model& M = I.M;
  const uint32_t N = static_cast<uint32_t>(M.n_states);
  const uint32_t nocc = static_cast<uint32_t>(M.n_occ);
  float* A = lds;
  float* B = lds + N;
  float* Vg = V + I.offset;
  for (uint32_t s = threadIdx.x; s < N; s += kLdsBlock) A[s] = Vg[s];
  __syncthreads();
  long long it = 0;
  double res = 0.0;
  while (it < max_iter) {
    double dmax = 0.0;
    for (uint32_t o = threadIdx.x; o < nocc; o += kLdsBlock) {
      const double d = backup_occupancy<KMAX, JMAX, uint32_t>(M, A, B, o);
      dmax = (d > dmax || d != d) ? d : dmax;
    }
    dmax = wave_max(dmax);
    if (threadIdx.x % kWave == 0) part[threadIdx.x / kWave] = dmax;
    __syncthreads();
    double m = part[0];
#pragma unroll
    for (int w = 1; w < kLdsBlock / kWave; ++w) m = (part[w] > m || part[w] != part[w]) ? part[w] : m;
    ++it;
    res = m;
    float* t = A;
    A = B;
    B = t;
    __syncthreads();  // every thread has read part[] and finished writing the new A
    if (!(res >= tol)) break;
  }
  for (uint32_t s = threadIdx.x; s < N; s += kLdsBlock) Vg[s] = A[s];
  if (threadIdx.x == 0) {
    out[i].iterations = it;
    out[i].residual = res;
  }
}

// One workgroup per instance of `list`.  Instances of up to 5 hosts and 3
// classes run the backup instantiated for their own (K, J) (a uniform switch
// per workgroup); the others the one of bounds KMAX, JMAX.  Same arithmetic
// either way (the bounds only remove guards): bit-identical iterates.
template <int KMAX, int JMAX>
__global__ __launch_bounds__(kLdsBlock) void batch_lds_vi_kernel(const BatchInst* __restrict__ insts,
                                                                  const int32_t* __restrict__ list,
                                                                  float* __restrict__ V, double tol,
                                                                  long long max_iter,
                                                                  BatchOut* __restrict__ out) {
  extern __shared__ float lds[];
  __shared__ double part[kLdsBlock / kWave];
  const int i = __builtin_amdgcn_readfirstlane(list[blockIdx.x]);
  const BatchInst& I = insts[i];
  switch (I.M.J <= 3 ? I.M.K * 4 + I.M.J : 0) {
#define MDPVI_LDS_CASE(K_, J_) \
  case K_ * 4 + J_: lds_solve<K_, J_>(I, i, lds, part, V, tol, max_iter, out); return;
    MDPVI_LDS_CASE(1, 1) MDPVI_LDS_CASE(1, 2) MDPVI_LDS_CASE(1, 3)
    MDPVI_LDS_CASE(2, 1) MDPVI_LDS_CASE(2, 2) MDPVI_LDS_CASE(2, 3)
    MDPVI_LDS_CASE(3, 1) MDPVI_LDS_CASE(3, 2) MDPVI_LDS_CASE(3, 3)
    MDPVI_LDS_CASE(4, 1) MDPVI_LDS_CASE(4, 2) MDPVI_LDS_CASE(4, 3)
    MDPVI_LDS_CASE(5, 1) MDPVI_LDS_CASE(5, 2) MDPVI_LDS_CASE(5, 3)
#undef MDPVI_LDS_CASE
    default: lds_solve<KMAX, JMAX>(I, i, lds, part, V, tol, max_iter, out);
  }
}

// ---------------------------------------------------------------- round form

// Sweep operations of the round form: run is the generic backup (bounds
// KM, JM), run_exact the exact-shape one (K hosts and J classes known at
// compile time, every load issued before the first use), which gives the
// same bits; exact_ok tells whether an instance meets run_exact's terms.
// side() picks the exact backup's side arrays from the launch's A0 / A1 for
// round j and returns false when the launch brings none it needs (the
// generic backup then runs).  Value iteration's exact backup reads the FP64
// arrival terms of the previous round from the instance's side array (ain:
// n_occ entries and a -inf entry for placements without room) and writes
// this round's (aout); the adjoint's reads the reset-line sums of its input
// (ain, A0 = the line table; batch_line_sum_kernel).
struct VIOp {
  using T = float;
  static constexpr ResKind RK = ResKind::kMax;
  template <int KM, int JM>
  __device__ static double run(const Model& M, const uint8_t*, const T* in, T* out, uint32_t o) {
    return backup_occupancy<KM, JM, uint32_t>(M, in, out, o);
  }
  __device__ static bool exact_ok(const BatchInst& I) {
    const Model& M = I.M;
    return I.aoff >= 0 && M.n_states < (int64_t{1} << 29) && M.J <= 3 && M.n_sizes == M.J;
  }
  __device__ static bool side(const BatchInst& I, long long j, double* A0, double* A1, const double** ain,
                              double** aout) {
    if (A0 == nullptr) return false;
    *ain = ((j & 1) ? A1 : A0) + I.aoff;
    *aout = ((j & 1) ? A0 : A1) + I.aoff;
    return true;
  }
  template <int K, int J>
  __device__ static double run_exact(const Model& M, const uint8_t*, const T* in, T* out, const double* ain,
                                     double* aout, uint32_t o) {
    return backup_arrival<K, J>(M, make_view(in, static_cast<uint32_t>(M.n_states) * 4u),
                                make_view(ain, static_cast<uint32_t>(M.n_occ + 1) * 8u), out, aout, o);
  }
};
struct EvalOp {
  using T = double;
  static constexpr ResKind RK = ResKind::kMax;
  __device__ static bool side(const BatchInst&, long long, double*, double*, const double**, double**) {
    return true;
  }
  template <int KM, int JM>
  __device__ static double run(const Model& M, const uint8_t* pi, const T* in, T* out, uint32_t o) {
    return eval_occupancy<KM, JM, uint32_t>(M, pi, in, out, o);
  }
  __device__ static bool exact_ok(const BatchInst& I) { return I.M.n_states < (int64_t{1} << 28) && I.M.J <= 3; }
  template <int K, int J>
  __device__ static double run_exact(const Model& M, const uint8_t* pi, const T* in, T* out, const double*,
                                     double*, uint32_t o) {
    return eval_exact<K, J>(M, make_view(pi, static_cast<uint32_t>(M.n_states)),
                            make_view(in, static_cast<uint32_t>(M.n_states) * 8u), out, o);
  }
};
struct AdjOp {
  using T = float;
  static constexpr ResKind RK = ResKind::kSum;
  template <int KM, int JM>
  __device__ static double run(const Model& M, const uint8_t* pi, const T* in, T* out, uint32_t o) {
    return adjoint_occupancy<KM, JM, uint32_t>(M, pi, in, out, o);
  }
  __device__ static bool exact_ok(const BatchInst& I) { return I.M.J <= 3 && I.loff >= 0; }
  __device__ static bool side(const BatchInst& I, long long, double* A0, double*, const double** ain,
                              double**) {
    if (A0 == nullptr) return false;
    *ain = A0 + I.loff;
    return true;
  }
  template <int K, int J>
  __device__ static double run_exact(const Model& M, const uint8_t* pi, const T* in, T* out, const double* lines,
                                     double*, uint32_t o) {
    return adjoint_occupancy_exact<K, J, true>(M, pi, in, out, o, lines);
  }
};

// Sum of the N weights win[base + x st], x = 0..N-1, from zero in that order
// (all N loads issued before the first add).
template <int N>
__device__ __forceinline__ double line_sum(const float* __restrict__ win, uint32_t base, uint32_t st) {
  float v[N];
#pragma unroll
  for (int x = 0; x < N; ++x) v[x] = win[base + static_cast<uint32_t>(x) * st];
  double line = 0.0;
#pragma unroll
  for (int x = 0; x < N; ++x) line += static_cast<double>(v[x]);
  return line;
}

// The reset-line sums of the adjoint's input for round j (the table the
// exact adjoint backup reads, layout in adjoint_occupancy_exact): for the
// tile's instance, every digit k, class e and line i in [ceil(first / R),
// ceil(end / R)) with R = C+1 -- the tiles of an instance partition
// [0, n_occ), so these ranges partition its n_occ / R lines -- the sum of
// w along the line, from zero in the order x = 0..C.  Consecutive threads
// take consecutive lines of one (k, e): along a high digit their loads are
// consecutive addresses.  A line's base (n_k = 0) is i with a zero digit
// inserted at k.
__global__ __launch_bounds__(kBlock) void batch_line_sum_kernel(const BatchInst* __restrict__ insts,
                                                                 const Tile* __restrict__ tiles,
                                                                 const float* __restrict__ w,
                                                                 const float* __restrict__ W,
                                                                 BatchCtl* __restrict__ ctl, long long j,
                                                                 double* __restrict__ lines, int opt) {
  const Tile tile = tiles[blockIdx.x];
  const BatchInst& I = insts[tile.inst];
  if (I.loff < 0) return;
  // an instance that already stopped (done_iter only changes in round
  // kernels, never while this one runs: the same answer for every lane)
  if (load_agent(&ctl[tile.inst].done_iter) >= 0) return;
  const Model& M = I.M;
  const float* win = ((j & 1) ? W : w) + I.offset;
  double* L = lines + I.loff;
  const uint32_t R = static_cast<uint32_t>(M.R), C = static_cast<uint32_t>(M.C);
  const uint32_t nocc = static_cast<uint32_t>(M.n_occ);
  const uint32_t end = min(tile.first + static_cast<uint32_t>(kBlock * opt), nocc);
  const uint32_t i0 = fast_div(tile.first + R - 1, M.divR);
  const uint32_t cnt = fast_div(end + R - 1, M.divR) - i0;
  const uint32_t nl = fast_div(nocc, M.divR);
  const uint32_t total = cnt * static_cast<uint32_t>(M.K * M.J);
  for (uint32_t u = threadIdx.x; u < total; u += kBlock) {
    const uint32_t ke = u / cnt;
    const uint32_t i = i0 + (u - ke * cnt);
    const uint32_t k = ke / static_cast<uint32_t>(M.J);
    const uint32_t e = ke - k * static_cast<uint32_t>(M.J);
    uint32_t hi = i;
    for (uint32_t h = 0; h < k; ++h) hi = fast_div(hi, M.divR);
    const uint32_t st = static_cast<uint32_t>(M.stride[k]);
    const uint32_t base = hi * st * R + (i - hi * st) + e * nocc;
    double line;
    switch (C) {
#define MDPVI_LINE_CASE(C_) \
  case C_: line = line_sum<C_ + 1>(win, base, st); break;
      MDPVI_LINE_CASE(1) MDPVI_LINE_CASE(2) MDPVI_LINE_CASE(3) MDPVI_LINE_CASE(4) MDPVI_LINE_CASE(5)
      MDPVI_LINE_CASE(6) MDPVI_LINE_CASE(7) MDPVI_LINE_CASE(8) MDPVI_LINE_CASE(9) MDPVI_LINE_CASE(10)
      MDPVI_LINE_CASE(11) MDPVI_LINE_CASE(12) MDPVI_LINE_CASE(13) MDPVI_LINE_CASE(14) MDPVI_LINE_CASE(15)
#undef MDPVI_LINE_CASE
      default:
        line = 0.0;
        for (uint32_t x = 0; x <= C; ++x) line += static_cast<double>(win[base + x * st]);
    }
    L[ke * nl + i] = line;
  }
}


// Per-instance control of the round form: true (for the whole workgroup) when
// the instance already stopped.  The leader workgroup of the instance (its
// first tile) records done_iter, counts the instance off and clears the
// residual words of the next round.
template <ResKind RK>
__device__ __forceinline__ bool inst_stopped(BatchCtl* c, long long j, double tol, int* remaining,
                                             bool leader) {
  __shared__ int stop;
  if (threadIdx.x < kWave) {
    bool s = load_agent(&c->done_iter) >= 0;
    if (!s && j > 0) {
      double v = 0.0;
      if (threadIdx.x < kBatchLanes)
        v = __longlong_as_double(static_cast<long long>(
            load_agent(&c->res[(j - 1) % kResSlots][threadIdx.x][0])));
      if constexpr (RK == ResKind::kMax) {
        v = wave_max(v);
      } else {
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
      }
      if (!(v >= tol)) {
        s = true;
        if (leader && threadIdx.x == 0) {
          store_agent(&c->done_iter, j);
          atomicSub(remaining, 1);
        }
      }
    }
    if (threadIdx.x == 0) stop = s ? 1 : 0;
  }
  __syncthreads();
  if (stop) return true;
  if (leader && threadIdx.x < kBatchLanes) store_agent(&c->res[(j + 1) % kResSlots][threadIdx.x][0], 0ull);
  return false;
}

// The workgroup's part of round j's residual of its instance: the largest
// (kMax, a NaN wins) or the sum (kSum) of the lanes' acc, added to residual
// word `lane` of the instance's control block.
template <ResKind RK>
__device__ __forceinline__ void round_residual(double acc, BatchCtl* c, long long j, uint32_t lane) {
  __shared__ double part[kBlock / kWave];
  if constexpr (RK == ResKind::kMax) {
    acc = wave_max(acc);
  } else {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kWave);
  }
  if (threadIdx.x % kWave == 0) part[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = part[0];
#pragma unroll
    for (int w = 1; w < kBlock / kWave; ++w) {
      if constexpr (RK == ResKind::kMax) m = (part[w] > m || part[w] != part[w]) ? part[w] : m;
      else m += part[w];
    }
    unsigned long long* word = &c->res[j % kResSlots][lane][0];
    if (m != 0.0) {
      if constexpr (RK == ResKind::kMax)
        atomicMax(word, static_cast<unsigned long long>(__double_as_longlong(m)));
      else
        atomicAdd(reinterpret_cast<double*>(word), m);
    }
  }
}

// The tile's occupancies through the exact-shape backup of (K, J), reduced
// as the round kernel reduces them.
template <class Op, int K, int J>
__device__ __forceinline__ double round_tile_exact(const Model& M, const uint8_t* p,
                                                   const typename Op::T* Vin, typename Op::T* Vout,
                                                   const double* Ain, double* Aout, uint32_t first, int opt) {
  double acc = 0.0;
  for (int k = 0; k < opt; ++k) {
    const uint32_t o = first + threadIdx.x + k * kBlock;
    if (o < static_cast<uint32_t>(M.n_occ)) {
      const double d = Op::template run_exact<K, J>(M, p, Vin, Vout, Ain, Aout, o);
      if constexpr (Op::RK == ResKind::kMax) acc = (d > acc || d != d) ? d : acc;
      else acc += d;
    }
  }
  return acc;
}

// FORM kRoundExact: instances of up to kBatchExactK hosts and 3 classes
// that meet Op::exact_ok take the exact-shape backup of their own (K, J) (a
// uniform branch per workgroup: a tile belongs to one instance), others the
// generic one; kRoundGeneric: every instance the generic one;
// kRoundExactOnly: the exact-shape backups alone (the host launches it when
// every instance qualifies; without the generic body the kernel needs far
// fewer registers), an instance that does not qualify reporting a NaN
// residual.  A tile holds kBlock * opt occupancies, opt per thread (opt in
// 1..kOccPerThread).
constexpr int kRoundGeneric = 0, kRoundExact = 1, kRoundExactOnly = 2;

template <class Op, int KMAX, int JMAX, int FORM>
__device__ __forceinline__ void round_body(const BatchInst* __restrict__ insts, const Tile tile,
                                           typename Op::T* __restrict__ V, typename Op::T* __restrict__ W,
                                           const uint8_t* __restrict__ pi, BatchCtl* __restrict__ ctl,
                                           int* remaining, long long j, double tol, int opt, double* A0,
                                           double* A1) {
  using T = typename Op::T;
  const BatchInst& I = insts[tile.inst];
  const Model& M = I.M;
  BatchCtl* c = ctl + tile.inst;
  if (inst_stopped<Op::RK>(c, j, tol, remaining, tile.first == 0)) return;
  const T* Vin = ((j & 1) ? W : V) + I.offset;
  T* Vout = ((j & 1) ? V : W) + I.offset;
  const uint8_t* p = pi ? pi + I.offset : nullptr;
  double acc = 0.0;
  bool done = false;
  if constexpr (FORM != kRoundGeneric) {
    const double* Ain = nullptr;
    double* Aout = nullptr;
    if (Op::exact_ok(I) && Op::side(I, j, A0, A1, &Ain, &Aout)) {
      done = true;
      switch (M.K * 4 + M.J) {
#define MDPVI_ROUND_CASE(K_, J_) \
  case K_ * 4 + J_: acc = round_tile_exact<Op, K_, J_>(M, p, Vin, Vout, Ain, Aout, tile.first, opt); break;
        MDPVI_ROUND_CASE(1, 1) MDPVI_ROUND_CASE(1, 2) MDPVI_ROUND_CASE(1, 3)
        MDPVI_ROUND_CASE(2, 1) MDPVI_ROUND_CASE(2, 2) MDPVI_ROUND_CASE(2, 3)
        MDPVI_ROUND_CASE(3, 1) MDPVI_ROUND_CASE(3, 2) MDPVI_ROUND_CASE(3, 3)
        MDPVI_ROUND_CASE(4, 1) MDPVI_ROUND_CASE(4, 2) MDPVI_ROUND_CASE(4, 3)
        MDPVI_ROUND_CASE(5, 1) MDPVI_ROUND_CASE(5, 2) MDPVI_ROUND_CASE(5, 3)
#undef MDPVI_ROUND_CASE
        default: done = false;
      }
      static_assert(kBatchExactK == 5, "the cases above cover K = 1..kBatchExactK");
    }
  }
  if constexpr (FORM == kRoundExactOnly) {
    if (!done) acc = NAN;
  } else {
    if (!done) {
      for (int k = 0; k < opt; ++k) {
        const uint32_t o = tile.first + threadIdx.x + k * kBlock;
        if (o < static_cast<uint32_t>(M.n_occ)) {
          const double d = Op::template run<KMAX, JMAX>(M, p, Vin, Vout, o);
          if constexpr (Op::RK == ResKind::kMax) acc = (d > acc || d != d) ? d : acc;
          else acc += d;
        }
      }
    }
  }
  round_residual<Op::RK>(acc, c, j, (tile.first / kBlock) % kBatchLanes);
}

template <class Op, int KMAX, int JMAX, int FORM>
__global__ __launch_bounds__(kBlock) void batch_round_kernel(const BatchInst* __restrict__ insts,
                                                              const Tile* __restrict__ tiles,
                                                              typename Op::T* __restrict__ V,
                                                              typename Op::T* __restrict__ W,
                                                              const uint8_t* __restrict__ pi,
                                                              BatchCtl* __restrict__ ctl,
                                                              int* remaining, long long j, double tol,
                                                              int opt, double* A0, double* A1) {
  round_body<Op, KMAX, JMAX, FORM>(insts, tiles[blockIdx.x], V, W, pi, ctl, remaining, j, tol, opt, A0, A1);
}

// Value-iteration round in the tile form (tile_vi.hpp) for the instances
// with I.tocc > 0 (K in 4..5, J <= 3 distinct sizes, tiles of T = 3 low
// digits): tile.first is the index of one of the instance's (C+1)^(K-3)
// tiles.  The workgroup stages the tile's values in LDS (dynamic: Vl
// [J][tocc]) and backs up its occupancies with the low-digit neighbours from
// LDS, the high-digit ones and every arrival term from global memory
// (tile_backup's AGlobal form: the staged image stays small, so more
// workgroups share a CU): the per-state arithmetic of the direct round
// backup, so the same bits.  Placements without room read the -inf block
// that ends the instance's side arrays.
template <int K, int J>
__device__ __forceinline__ double batch_vi_tile_body(const BatchInst& I, uint32_t tb, const float* Vin,
                                                     float* Vout, const double* Ain, double* Aout,
                                                     double* Al, float* Vl) {
  constexpr int T = 3;
  const Model& M = I.M;
  const uint32_t occ = static_cast<uint32_t>(I.tocc);
  const uint32_t nocc = static_cast<uint32_t>(M.n_occ);
  const uint32_t ns = static_cast<uint32_t>(M.n_states);
  const uint32_t cls = nocc * 4u;
  const BufView vin = make_view(Vin, ns * 4u);
  const BufView vout = make_view(Vout, ns * 4u);
  const BufView ain = make_view(Ain, (nocc + occ) * 8u);
  const BufView aout = make_view(Aout, nocc * 8u);
  TileHigh<K, J, T> H;
  tile_high_setup<K, J, T>(M, tb, H);
  tile_stage_values<J, kBlock>(M, occ, H.o0, vin, Vl);
  __syncthreads();
  double acc = 0.0;
  for (uint32_t i = threadIdx.x; i < occ; i += kBlock) {
    float vs[J], vn[J];
    double anew;
    tile_backup<K, J, T, false, true>(M, H, occ, Vl, Al, vin, ain, i, vs, vn, anew);
#pragma unroll
    for (int e = 0; e < J; ++e) {
      st_f32(vout, vn[e], i * 4u, H.o0 * 4u + e * cls);
      const double d = fabs(static_cast<double>(vn[e]) - static_cast<double>(vs[e]));
      acc = (d > acc || d != d) ? d : acc;
    }
    st_f64(aout, anew, i * 8u, H.o0 * 8u);
  }
  return acc;
}

__global__ __launch_bounds__(kBlock) void batch_vi_tile_kernel(const BatchInst* __restrict__ insts,
                                                                const Tile* __restrict__ tiles,
                                                                float* __restrict__ V, float* __restrict__ W,
                                                                BatchCtl* __restrict__ ctl, int* remaining,
                                                                long long j, double tol, double* A0, double* A1) {
  extern __shared__ double tile_lds[];
  const Tile tile = tiles[blockIdx.x];
  const BatchInst& I = insts[tile.inst];
  const Model& M = I.M;
  BatchCtl* c = ctl + tile.inst;
  if (inst_stopped<ResKind::kMax>(c, j, tol, remaining, tile.first == 0)) return;
  const float* Vin = ((j & 1) ? W : V) + I.offset;
  float* Vout = ((j & 1) ? V : W) + I.offset;
  const double* Ain = ((j & 1) ? A1 : A0) + I.aoff;
  double* Aout = ((j & 1) ? A0 : A1) + I.aoff;
  float* Vl = reinterpret_cast<float*>(tile_lds);   // [J][tocc]; the arrival terms stay in global memory
  double acc = 0.0;
  switch (M.K * 4 + M.J) {
#define MDPVI_TILE_CASE(K_, J_) \
  case K_ * 4 + J_: acc = batch_vi_tile_body<K_, J_>(I, tile.first, Vin, Vout, Ain, Aout, nullptr, Vl); break;
    MDPVI_TILE_CASE(4, 1) MDPVI_TILE_CASE(4, 2) MDPVI_TILE_CASE(4, 3)
    MDPVI_TILE_CASE(5, 1) MDPVI_TILE_CASE(5, 2) MDPVI_TILE_CASE(5, 3)
#undef MDPVI_TILE_CASE
    default: acc = NAN;   // not a tile-form shape: the host never lists such a tile
  }
  round_residual<ResKind::kMax>(acc, c, j, tile.first % kBatchLanes);
}

// FP64 evaluation round in the tile form (tile_eval.hpp) for the instances
// with I.eocc > 0 (K in 4..5, J <= 3 distinct sizes, tiles of T = 3 low
// digits): tile.first is the index of one of the instance's tiles.  The
// arrival terms of the policy's actions come from the instance's FP64 side
// arrays (E0/E1 + eoff, ping-pong with the values), written by the previous
// round or by batch_eval_arrival_init_kernel: the same bits as the direct
// round backup.
__device__ __forceinline__ void eval_tile_round(const BatchInst* __restrict__ insts, const Tile tile,
                                                const uint8_t* __restrict__ pi, double* __restrict__ V,
                                                double* __restrict__ W, BatchCtl* __restrict__ ctl, int* remaining,
                                                long long j, double tol, double* E0, double* E1,
                                                double* tile_lds) {
  const BatchInst& I = insts[tile.inst];
  const Model& M = I.M;
  BatchCtl* c = ctl + tile.inst;
  if (inst_stopped<ResKind::kMax>(c, j, tol, remaining, tile.first == 0)) return;
  const uint32_t nocc = static_cast<uint32_t>(M.n_occ);
  const uint32_t ns = static_cast<uint32_t>(M.n_states);
  const BufView pv = make_view(pi + I.offset, ns);
  const BufView vin = make_view(((j & 1) ? W : V) + I.offset, ns * 8u);
  const BufView vout = make_view(((j & 1) ? V : W) + I.offset, ns * 8u);
  const BufView ain = make_view(((j & 1) ? E1 : E0) + I.eoff, nocc * 8u);
  const BufView aout = make_view(((j & 1) ? E0 : E1) + I.eoff, nocc * 8u);
  const uint32_t occ = static_cast<uint32_t>(I.eocc);
  double acc = 0.0;
  switch (M.K * 4 + M.J) {
#define MDPVI_TILE_CASE(K_, J_) \
  case K_ * 4 + J_: acc = eval_tile_block<K_, J_, 3, kBlock>(M, tile.first, occ, pv, vin, vout, ain, aout, tile_lds, 0.0); break;
    MDPVI_TILE_CASE(4, 1) MDPVI_TILE_CASE(4, 2) MDPVI_TILE_CASE(4, 3)
    MDPVI_TILE_CASE(5, 1) MDPVI_TILE_CASE(5, 2) MDPVI_TILE_CASE(5, 3)
#undef MDPVI_TILE_CASE
    default: acc = NAN;   // not a tile-form shape: the host never lists such a tile
  }
  round_residual<ResKind::kMax>(acc, c, j, tile.first % kBatchLanes);
}

__global__ __launch_bounds__(kBlock) void batch_eval_tile_kernel(const BatchInst* __restrict__ insts,
                                                                  const Tile* __restrict__ tiles,
                                                                  const uint8_t* __restrict__ pi,
                                                                  double* __restrict__ V, double* __restrict__ W,
                                                                  BatchCtl* __restrict__ ctl, int* remaining,
                                                                  long long j, double tol, double* E0, double* E1) {
  extern __shared__ double tile_lds[];
  eval_tile_round(insts, tiles[blockIdx.x], pi, V, W, ctl, remaining, j, tol, E0, E1, tile_lds);
}

// One evaluation round over both kinds of tile in one launch (one tail per
// round): workgroups 0..n_tile-1 take the tile-form tiles, the rest the
// direct-form ones (the exact-shape round backup; every instance of the
// batch has at most kBatchExactK hosts and 3 classes).
__global__ __launch_bounds__(kBlock) void batch_eval_mixed_kernel(const BatchInst* __restrict__ insts,
                                                                   const Tile* __restrict__ dtiles,
                                                                   const Tile* __restrict__ ttiles, int n_tile,
                                                                   const uint8_t* __restrict__ pi,
                                                                   double* __restrict__ V, double* __restrict__ W,
                                                                   BatchCtl* __restrict__ ctl, int* remaining,
                                                                   long long j, double tol, int opt, double* E0,
                                                                   double* E1) {
  extern __shared__ double tile_lds[];
  if (static_cast<int>(blockIdx.x) < n_tile)
    eval_tile_round(insts, ttiles[blockIdx.x], pi, V, W, ctl, remaining, j, tol, E0, E1, tile_lds);
  else
    round_body<EvalOp, 8, 4, kRoundExact>(insts, dtiles[blockIdx.x - n_tile], V, W, pi, ctl, remaining, j, tol,
                                          opt, nullptr, nullptr);
}

// A(o) = sum_e lambda_e/Lam V(o, e) (the FMA chain of the evaluation
// backups) of the FP64 iterate V into E0, for the occupancies of the
// evaluation tiles {inst, tile index} (eocc each).
__global__ __launch_bounds__(kBlock) void batch_eval_arrival_init_kernel(const BatchInst* __restrict__ insts,
                                                                          const Tile* __restrict__ tiles,
                                                                          const double* __restrict__ V,
                                                                          double* __restrict__ E0) {
  const Tile tile = tiles[blockIdx.x];
  const BatchInst& I = insts[tile.inst];
  if (I.eoff < 0 || I.eocc <= 0) return;
  const Model& M = I.M;
  const uint64_t nocc = static_cast<uint64_t>(M.n_occ);
  const uint64_t o0 = static_cast<uint64_t>(tile.first) * static_cast<uint64_t>(I.eocc);
  for (uint32_t i = threadIdx.x; i < static_cast<uint32_t>(I.eocc); i += kBlock) {
    const uint64_t o = o0 + i;
    double a = 0.0;
    for (int e = 0; e < M.J; ++e) a = fma(M.p[e], V[I.offset + o + static_cast<uint64_t>(e) * nocc], a);
    E0[I.eoff + o] = a;
  }
}

// Copies the final iterate of instances that stopped after an odd number of
// sweeps (it lives in W) back to V, and reports iterations and residuals.
template <typename T, ResKind RK>
__global__ void batch_round_finish_kernel(const BatchInst* __restrict__ insts,
                                          const int32_t* __restrict__ list, int n_list,
                                          T* __restrict__ V, const T* __restrict__ W,
                                          BatchCtl* __restrict__ ctl, long long issued,
                                          BatchOut* __restrict__ out) {
  const int li = blockIdx.y;
  if (li >= n_list) return;
  const int i = list[li];
  const BatchInst& I = insts[i];
  BatchCtl* c = ctl + i;
  const long long d = load_agent(&c->done_iter);
  const long long fin = d >= 0 ? d : issued;
  if (fin & 1) {
    const uint64_t N = static_cast<uint64_t>(I.M.n_states);
    for (uint64_t s = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; s < N;
         s += static_cast<uint64_t>(gridDim.x) * blockDim.x)
      V[I.offset + s] = W[I.offset + s];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double r = 0.0;
    for (int l = 0; l < kBatchLanes && fin > 0; ++l) {   // fin = 0: an instance that was not run
      const double v =
          __longlong_as_double(static_cast<long long>(load_agent(&c->res[(fin - 1) % kResSlots][l][0])));
      if constexpr (RK == ResKind::kMax) r = (v > r || v != v) ? v : r;
      else r += v;
    }
    out[i].iterations = fin;
    out[i].residual = r;
  }
}

// Arrival terms A(o) = sum_e lambda_e/Lam V(o, e) of the initial iterate
// (backup_arrival's FMA chain) into A0 for the instances with side arrays,
// and the -inf entry A[n_occ] into both arrays.
__global__ __launch_bounds__(kBlock) void batch_arrival_init_kernel(const BatchInst* __restrict__ insts,
                                                                     const Tile* __restrict__ tiles,
                                                                     const float* __restrict__ V,
                                                                     double* __restrict__ A0,
                                                                     double* __restrict__ A1, int opt) {
  const Tile tile = tiles[blockIdx.x];
  const BatchInst& I = insts[tile.inst];
  if (I.aoff < 0) return;
  const Model& M = I.M;
  const uint64_t nocc = static_cast<uint64_t>(M.n_occ);
  if (tile.first == 0) {   // the -inf block: one entry, or tocc for the tile form
    const uint32_t ns = I.tocc > 0 ? static_cast<uint32_t>(I.tocc) : 1u;
    for (uint32_t t = threadIdx.x; t < ns; t += kBlock) {
      A0[I.aoff + nocc + t] = -INFINITY;
      A1[I.aoff + nocc + t] = -INFINITY;
    }
  }
  for (int k = 0; k < opt; ++k) {
    const uint64_t o = tile.first + threadIdx.x + static_cast<uint64_t>(k) * kBlock;
    if (o >= nocc) break;
    double a = 0.0;
    for (int e = 0; e < M.J; ++e)
      a = fma(M.p[e], static_cast<double>(V[I.offset + o + static_cast<uint64_t>(e) * nocc]), a);
    A0[I.aoff + o] = a;
  }
}

// Writes the tiles of `in` whose instance has not stopped to `out` (in no
// particular order: every tile's work and residual word depend on the tile
// alone) and their number to *n_out, which must be zero on entry.  One
// atomic per wavefront.
__global__ void batch_compact_kernel(const Tile* __restrict__ in, int n_in, const BatchCtl* __restrict__ ctl,
                                     Tile* __restrict__ out, int* n_out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  Tile tile{};
  bool keep = false;
  if (t < n_in) {
    tile = in[t];
    keep = load_agent(&ctl[tile.inst].done_iter) < 0;
  }
  const unsigned long long mask = __ballot(keep);
  const int lane = threadIdx.x % kWave;
  const int before = __popcll(mask & ((1ull << lane) - 1ull));
  int base = 0;
  if (lane == 0 && mask != 0ull) base = atomicAdd(n_out, __popcll(mask));
  base = __shfl(base, 0, kWave);
  if (keep) out[base + before] = tile;
}

__global__ void batch_zero_kernel(int* p) { *p = 0; }

// Control blocks of instances 0..n-1 for a round loop over the active ones
// (active[i] != 0): done_iter -1 for those and 0 (already stopped, no sweep)
// for the others, residual words cleared; *remaining = n_active.
__global__ void batch_ctl_activate_kernel(BatchCtl* ctl, const int* __restrict__ active, int n,
                                          int* remaining, int n_active) {
  const int i = blockIdx.x;
  if (i < n) {
    BatchCtl* c = ctl + i;
    if (threadIdx.x == 0) c->done_iter = active[i] ? -1 : 0;
    for (int w = threadIdx.x; w < kResSlots * kBatchLanes; w += blockDim.x)
      c->res[w / kBatchLanes][w % kBatchLanes][0] = 0ull;
  }
  if (i == 0 && threadIdx.x == 0) *remaining = n_active;
}

// Policy improvement (improve_occupancy, in place) of the tiles' instances
// with active[inst] != 0; changed[inst] := 1 where some action changed
// (changed must be cleared).  Tiles of kBlock * kOccPerThread occupancies.
template <int KMAX, int JMAX>
__global__ __launch_bounds__(kBlock) void batch_improve_kernel(const BatchInst* __restrict__ insts,
                                                                const Tile* __restrict__ tiles,
                                                                const double* __restrict__ V, uint8_t* pi,
                                                                double tol, const int* __restrict__ active,
                                                                int* __restrict__ changed) {
  const Tile tile = tiles[blockIdx.x];
  if (!active[tile.inst]) return;
  const BatchInst& I = insts[tile.inst];
  bool ch = false;
  for (int k = 0; k < kOccPerThread; ++k) {
    const uint32_t o = tile.first + threadIdx.x + k * kBlock;
    if (o < static_cast<uint32_t>(I.M.n_occ))
      ch |= improve_occupancy<KMAX, JMAX, uint32_t>(I.M, V + I.offset, pi + I.offset, pi + I.offset, tol, o);
  }
  if (__ballot(ch) != 0ull && threadIdx.x % kWave == 0) changed[tile.inst] = 1;
}

__global__ void batch_ctl_init_kernel(BatchCtl* ctl, const int32_t* __restrict__ list, int n_list,
                                      int* remaining, int* flags, int n_flags) {
  const int li = blockIdx.x;
  if (li < n_list) {
    BatchCtl* c = ctl + list[li];
    if (threadIdx.x == 0) c->done_iter = -1;
    for (int w = threadIdx.x; w < kResSlots * kBatchLanes; w += blockDim.x)
      c->res[w / kBatchLanes][w % kBatchLanes][0] = 0ull;
  }
  if (li == 0) {
    if (threadIdx.x == 0) *remaining = n_list;
    for (int f = threadIdx.x; f < n_flags; f += blockDim.x) flags[f] = 0;
  }
}

// ---------------------------------------------------------------- one-pass tile kernels

template <int KMAX, int JMAX, typename T>
__global__ __launch_bounds__(kBlock) void batch_extract_kernel(const BatchInst* __restrict__ insts,
                                                                const Tile* __restrict__ tiles,
                                                                const T* __restrict__ V,
                                                                uint8_t* __restrict__ pi,
                                                                float* __restrict__ gap) {
  const Tile tile = tiles[blockIdx.x];
  const BatchInst& I = insts[tile.inst];
#pragma unroll
  for (int k = 0; k < kOccPerThread; ++k) {
    const uint32_t o = tile.first + threadIdx.x + k * kBlock;
    if (o < static_cast<uint32_t>(I.M.n_occ))
      extract_occupancy<KMAX, JMAX, T, uint32_t>(I.M, V + I.offset, pi + I.offset,
                                                 gap ? gap + I.offset : nullptr, o);
  }
}

template <int KMAX, int JMAX>
__global__ __launch_bounds__(kBlock) void batch_greedy_kernel(const BatchInst* __restrict__ insts,
                                                               const Tile* __restrict__ tiles, int kind,
                                                               uint8_t* __restrict__ pi) {
  const Tile tile = tiles[blockIdx.x];
  const BatchInst& I = insts[tile.inst];
#pragma unroll
  for (int k = 0; k < kOccPerThread; ++k) {
    const uint32_t o = tile.first + threadIdx.x + k * kBlock;
    if (o < static_cast<uint32_t>(I.M.n_occ)) greedy_occupancy<KMAX, JMAX, uint32_t>(I.M, kind, pi + I.offset, o);
  }
}

template <int KMAX, int JMAX>
__global__ __launch_bounds__(kBlock) void batch_check_kernel(const BatchInst* __restrict__ insts,
                                                              const Tile* __restrict__ tiles,
                                                              const uint8_t* __restrict__ pi,
                                                              int* __restrict__ flags) {
  const Tile tile = tiles[blockIdx.x];
  const BatchInst& I = insts[tile.inst];
  bool bad = false;
#pragma unroll
  for (int k = 0; k < kOccPerThread; ++k) {
    const uint32_t o = tile.first + threadIdx.x + k * kBlock;
    if (o < static_cast<uint32_t>(I.M.n_occ)) bad |= check_occupancy<KMAX, JMAX, uint32_t>(I.M, pi + I.offset, o);
  }
  if (bad) flags[tile.inst] = 1;
}

template <int KMAX, int JMAX>
__global__ __launch_bounds__(kBlock) void batch_grad_partial_kernel(const BatchInst* __restrict__ insts,
                                                                     const Tile* __restrict__ tiles,
                                                                     const uint8_t* __restrict__ pi,
                                                                     const double* __restrict__ V,
                                                                     const float* __restrict__ w,
                                                                     double* __restrict__ partial) {
  constexpr int TMAX = 2 * JMAX + 2;
  const Tile tile = tiles[blockIdx.x];
  const BatchInst& I = insts[tile.inst];
  double g[TMAX];
#pragma unroll
  for (int t = 0; t < TMAX; ++t) g[t] = 0.0;
  for (int k = 0; k < kOccPerThread; ++k) {
    const uint32_t o = tile.first + threadIdx.x + k * kBlock;
    if (o >= static_cast<uint32_t>(I.M.n_occ)) break;
    grad_occupancy<KMAX, JMAX, uint32_t>(I.M, pi + I.offset, V + I.offset, w + I.offset, o, g);
  }
  __shared__ double part[kBlock / kWave][TMAX];
  const int lane = threadIdx.x % kWave;
  const int wid = threadIdx.x / kWave;
#pragma unroll
  for (int t = 0; t < TMAX; ++t) {
    double v = g[t];
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    if (lane == 0) part[wid][t] = v;
  }
  __syncthreads();
  if (threadIdx.x < TMAX) {
    double v = 0.0;
#pragma unroll
    for (int wv = 0; wv < kBlock / kWave; ++wv) v += part[wv][threadIdx.x];
    partial[static_cast<size_t>(blockIdx.x) * TMAX + threadIdx.x] = v;
  }
}

// One workgroup per instance: sums its tiles' partials in tile order and adds
// the objective-weight terms; out rows hold 2*kMaxJ+3 doubles (gradient in
// the packed order lambda_1..J, mu, nu, r_1..J, then J at index 2J+2).
template <int JMAX>
__global__ void batch_grad_final_kernel(const BatchInst* __restrict__ insts,
                                        const int32_t* __restrict__ tile_begin,
                                        const double* __restrict__ partial, const double* __restrict__ V,
                                        double* __restrict__ out) {
  constexpr int TMAX = 2 * JMAX + 2;
  const int i = blockIdx.x;
  const BatchInst& I = insts[i];
  const Model& M = I.M;
  const int t = threadIdx.x;
  const size_t nocc = static_cast<size_t>(M.n_occ);
  const double* Vi = V + I.offset;
  double* o = out + static_cast<size_t>(i) * (2 * kMaxJ + 3);
  if (t < TMAX) {
    double v = 0.0;
    for (int b = tile_begin[i]; b < tile_begin[i + 1]; ++b) v += partial[static_cast<size_t>(b) * TMAX + t];
    int dst = -1;
    if (t < JMAX) {
      if (t < M.J) {
        dst = t;
        const double lt = M.lam_tot;
        for (int e = 0; e < M.J; ++e)
          v += ((e == t ? lt : 0.0) - M.lam[e]) / (lt * lt) * Vi[static_cast<size_t>(e) * nocc];
      }
    } else if (t == JMAX) {
      dst = M.J;
    } else if (t == JMAX + 1) {
      dst = M.J + 1;
    } else if (t - JMAX - 2 < M.J) {
      dst = M.J + 2 + (t - JMAX - 2);
    }
    if (dst >= 0) o[dst] = v;
  }
  if (t == 0) {
    double Jv = 0.0;
    for (int e = 0; e < M.J; ++e) Jv = fma(M.c_obj[e], Vi[static_cast<size_t>(e) * nocc], Jv);
    o[2 * M.J + 2] = Jv;
  }
}

// ---------------------------------------------------------------- launchers

template <typename F>
static hipError_t dispatch_kj_b(int K, int J, F&& f) {
  using I4 = std::integral_constant<int, 4>;
  using I8 = std::integral_constant<int, 8>;
  using I16 = std::integral_constant<int, 16>;
  if (J <= 4) {
    if (K <= 4) return f(I4{}, I4{});
    if (K <= 8) return f(I8{}, I4{});
    return f(I16{}, I4{});
  }
  if (K <= 4) return f(I4{}, I8{});
  if (K <= 8) return f(I8{}, I8{});
  return f(I16{}, I8{});
}

hipError_t launch_batch_lds_vi(const BatchInst* insts, const int32_t* list, int n_list, int maxK,
                               int maxJ, size_t lds_bytes, float* V, double tol, long long max_iter,
                               BatchOut* out, hipStream_t s) {
  if (n_list == 0) return hipSuccess;
  return dispatch_kj_b(maxK, maxJ, [&](auto km, auto jm) {
    constexpr int KM = decltype(km)::value, JM = decltype(jm)::value;
    auto kern = batch_lds_vi_kernel<KM, JM>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(lds_bytes));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(n_list), dim3(kLdsBlock), lds_bytes, s, insts, list, V, tol,
                       max_iter, out);
    return hipGetLastError();
  });
}

hipError_t launch_batch_arrival_init(const BatchInst* insts, const Tile* tiles, int n_tiles, const float* V,
                                     double* A0, double* A1, int opt, hipStream_t s) {
  if (n_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(batch_arrival_init_kernel, dim3(n_tiles), dim3(kBlock), 0, s, insts, tiles, V, A0, A1, opt);
  return hipGetLastError();
}

hipError_t launch_batch_ctl_activate(BatchCtl* ctl, const int* active, int n, int* remaining, int n_active,
                                     hipStream_t s) {
  hipLaunchKernelGGL(batch_ctl_activate_kernel, dim3(n > 0 ? n : 1), dim3(64), 0, s, ctl, active, n, remaining,
                     n_active);
  return hipGetLastError();
}

hipError_t launch_batch_improve_active(const BatchInst* insts, const Tile* tiles, int n_tiles, int maxK, int maxJ,
                                       const double* V, uint8_t* pi, double tol, const int* active, int* changed,
                                       hipStream_t s) {
  if (n_tiles == 0) return hipSuccess;
  return dispatch_kj_b(maxK, maxJ, [&](auto km, auto jm) {
    constexpr int KM = decltype(km)::value, JM = decltype(jm)::value;
    hipLaunchKernelGGL((batch_improve_kernel<KM, JM>), dim3(n_tiles), dim3(kBlock), 0, s, insts, tiles, V, pi,
                       tol, active, changed);
    return hipGetLastError();
  });
}

hipError_t launch_batch_compact(const Tile* in, int n_in, const BatchCtl* ctl, Tile* out, int* n_out,
                                hipStream_t s) {
  hipLaunchKernelGGL(batch_zero_kernel, dim3(1), dim3(1), 0, s, n_out);
  if (n_in > 0)
    hipLaunchKernelGGL(batch_compact_kernel, dim3((n_in + 255) / 256), dim3(256), 0, s, in, n_in, ctl, out, n_out);
  return hipGetLastError();
}

hipError_t launch_batch_ctl_init(BatchCtl* ctl, const int32_t* list, int n_list, int* remaining,
                                 int* flags, int n_flags, hipStream_t s) {
  hipLaunchKernelGGL(batch_ctl_init_kernel, dim3(n_list > 0 ? n_list : 1), dim3(64), 0, s, ctl, list,
                     n_list, remaining, flags, n_flags);
  return hipGetLastError();
}

template <class Op>
static hipError_t launch_round_t(const BatchInst* insts, const Tile* tiles, int n_tiles, int maxK,
                                 int maxJ, typename Op::T* V, typename Op::T* W, const uint8_t* pi,
                                 BatchCtl* ctl, int* remaining, long long j, double tol, int opt,
                                 double* A0, double* A1, bool all_exact, hipStream_t s) {
  if (n_tiles == 0) return hipSuccess;
  if (opt < 1 || opt > kOccPerThread) return hipErrorInvalidValue;
  if (maxK <= kBatchExactK && maxJ <= 3) {
    if (all_exact)
      hipLaunchKernelGGL((batch_round_kernel<Op, 8, 4, kRoundExactOnly>), dim3(n_tiles), dim3(kBlock), 0, s, insts,
                         tiles, V, W, pi, ctl, remaining, j, tol, opt, A0, A1);
    else
      hipLaunchKernelGGL((batch_round_kernel<Op, 8, 4, kRoundExact>), dim3(n_tiles), dim3(kBlock), 0, s, insts,
                         tiles, V, W, pi, ctl, remaining, j, tol, opt, A0, A1);
    return hipGetLastError();
  }
  return dispatch_kj_b(maxK, maxJ, [&](auto km, auto jm) {
    constexpr int KM = decltype(km)::value, JM = decltype(jm)::value;
    hipLaunchKernelGGL((batch_round_kernel<Op, KM, JM, kRoundGeneric>), dim3(n_tiles), dim3(kBlock), 0, s, insts,
                       tiles, V, W, pi, ctl, remaining, j, tol, opt, A0, A1);
    return hipGetLastError();
  });
}

hipError_t launch_batch_round(const BatchInst* insts, const Tile* tiles, int n_tiles, int maxK,
                              int maxJ, float* V, float* W, BatchCtl* ctl, int* remaining,
                              long long j, double tol, int opt, double* A0, double* A1, bool all_exact,
                              hipStream_t s) {
  return launch_round_t<VIOp>(insts, tiles, n_tiles, maxK, maxJ, V, W, nullptr, ctl, remaining, j, tol, opt,
                              A0, A1, all_exact && A0 != nullptr, s);
}

hipError_t launch_batch_vi_tile(const BatchInst* insts, const Tile* tiles, int n_tiles, size_t lds, float* V,
                                float* W, BatchCtl* ctl, int* remaining, long long j, double tol, double* A0,
                                double* A1, hipStream_t s) {
  if (n_tiles == 0) return hipSuccess;
  if (A0 == nullptr || A1 == nullptr || lds == 0 || lds > kBatchTileLds) return hipErrorInvalidValue;
  hipLaunchKernelGGL(batch_vi_tile_kernel, dim3(n_tiles), dim3(kBlock), lds, s, insts, tiles, V, W, ctl,
                     remaining, j, tol, A0, A1);
  return hipGetLastError();
}

hipError_t launch_batch_eval_tile(const BatchInst* insts, const Tile* tiles, int n_tiles, size_t lds,
                                  const uint8_t* pi, double* V, double* W, BatchCtl* ctl, int* remaining,
                                  long long j, double tol, double* E0, double* E1, hipStream_t s) {
  if (n_tiles == 0) return hipSuccess;
  if (E0 == nullptr || E1 == nullptr || lds == 0 || lds > kBatchTileLds) return hipErrorInvalidValue;
  hipLaunchKernelGGL(batch_eval_tile_kernel, dim3(n_tiles), dim3(kBlock), lds, s, insts, tiles, pi, V, W, ctl,
                     remaining, j, tol, E0, E1);
  return hipGetLastError();
}

hipError_t launch_batch_eval_mixed(const BatchInst* insts, const Tile* dtiles, int n_direct, const Tile* ttiles,
                                   int n_tile, size_t lds, int maxK, int maxJ, const uint8_t* pi, double* V,
                                   double* W, BatchCtl* ctl, int* remaining, long long j, double tol, int opt,
                                   double* E0, double* E1, bool all_exact, hipStream_t s) {
  if (n_tile == 0)
    return launch_batch_eval_round(insts, dtiles, n_direct, maxK, maxJ, pi, V, W, ctl, remaining, j, tol, opt,
                                   all_exact, s);
  if (n_direct == 0 || !(maxK <= kBatchExactK && maxJ <= 3)) {
    const hipError_t e = launch_batch_eval_tile(insts, ttiles, n_tile, lds, pi, V, W, ctl, remaining, j, tol, E0,
                                                E1, s);
    if (e != hipSuccess) return e;
    return launch_batch_eval_round(insts, dtiles, n_direct, maxK, maxJ, pi, V, W, ctl, remaining, j, tol, opt,
                                   all_exact, s);
  }
  if (opt < 1 || opt > kOccPerThread || E0 == nullptr || E1 == nullptr || lds == 0 || lds > kBatchTileLds)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(batch_eval_mixed_kernel, dim3(n_tile + n_direct), dim3(kBlock), lds, s, insts, dtiles, ttiles,
                     n_tile, pi, V, W, ctl, remaining, j, tol, opt, E0, E1);
  return hipGetLastError();
}

hipError_t launch_batch_eval_arrival_init(const BatchInst* insts, const Tile* tiles, int n_tiles, const double* V,
                                          double* E0, hipStream_t s) {
  if (n_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(batch_eval_arrival_init_kernel, dim3(n_tiles), dim3(kBlock), 0, s, insts, tiles, V, E0);
  return hipGetLastError();
}

hipError_t launch_batch_eval_round(const BatchInst* insts, const Tile* tiles, int n_tiles, int maxK,
                                   int maxJ, const uint8_t* pi, double* V, double* W, BatchCtl* ctl,
                                   int* remaining, long long j, double tol, int opt, bool all_exact,
                                   hipStream_t s) {
  return launch_round_t<EvalOp>(insts, tiles, n_tiles, maxK, maxJ, V, W, pi, ctl, remaining, j, tol, opt,
                                nullptr, nullptr, all_exact, s);
}

hipError_t launch_batch_adjoint_round(const BatchInst* insts, const Tile* tiles, int n_tiles, int maxK,
                                      int maxJ, const uint8_t* pi, float* w, float* W, BatchCtl* ctl,
                                      int* remaining, long long j, double tol, int opt, double* lines,
                                      bool all_exact, hipStream_t s) {
  if (n_tiles == 0) return hipSuccess;
  if (opt < 1 || opt > kOccPerThread) return hipErrorInvalidValue;
  // the table is read only by the exact backups of the kernel below
  if (!(maxK <= kBatchExactK && maxJ <= 3)) lines = nullptr;
  if (lines) {
    hipLaunchKernelGGL(batch_line_sum_kernel, dim3(n_tiles), dim3(kBlock), 0, s, insts, tiles, w, W, ctl, j,
                       lines, opt);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return launch_round_t<AdjOp>(insts, tiles, n_tiles, maxK, maxJ, w, W, pi, ctl, remaining, j, tol, opt, lines,
                               nullptr, all_exact && lines != nullptr, s);
}

template <typename T, ResKind RK>
static hipError_t launch_finish_t(const BatchInst* insts, const int32_t* list, int n_list, T* V,
                                  const T* W, BatchCtl* ctl, long long issued, BatchOut* out,
                                  hipStream_t s) {
  if (n_list == 0) return hipSuccess;
  hipLaunchKernelGGL((batch_round_finish_kernel<T, RK>), dim3(64, n_list), dim3(256), 0, s, insts, list,
                     n_list, V, W, ctl, issued, out);
  return hipGetLastError();
}

hipError_t launch_batch_round_finish(const BatchInst* insts, const int32_t* list, int n_list,
                                     float* V, const float* W, BatchCtl* ctl, long long issued,
                                     BatchOut* out, hipStream_t s) {
  return launch_finish_t<float, ResKind::kMax>(insts, list, n_list, V, W, ctl, issued, out, s);
}

hipError_t launch_batch_eval_finish(const BatchInst* insts, const int32_t* list, int n_list,
                                    double* V, const double* W, BatchCtl* ctl, long long issued,
                                    BatchOut* out, hipStream_t s) {
  return launch_finish_t<double, ResKind::kMax>(insts, list, n_list, V, W, ctl, issued, out, s);
}

hipError_t launch_batch_adjoint_finish(const BatchInst* insts, const int32_t* list, int n_list,
                                       float* w, const float* W, BatchCtl* ctl, long long issued,
                                       BatchOut* out, hipStream_t s) {
  return launch_finish_t<float, ResKind::kSum>(insts, list, n_list, w, W, ctl, issued, out, s);
}

hipError_t launch_batch_extract(const BatchInst* insts, const Tile* tiles, int n_tiles, int maxK,
                                int maxJ, const void* V, bool f64, uint8_t* pi, float* gap,
                                hipStream_t s) {
  if (n_tiles == 0) return hipSuccess;
  return dispatch_kj_b(maxK, maxJ, [&](auto km, auto jm) {
    constexpr int KM = decltype(km)::value, JM = decltype(jm)::value;
    if (f64)
      hipLaunchKernelGGL((batch_extract_kernel<KM, JM, double>), dim3(n_tiles), dim3(kBlock), 0, s, insts,
                         tiles, static_cast<const double*>(V), pi, gap);
    else
      hipLaunchKernelGGL((batch_extract_kernel<KM, JM, float>), dim3(n_tiles), dim3(kBlock), 0, s, insts,
                         tiles, static_cast<const float*>(V), pi, gap);
    return hipGetLastError();
  });
}

hipError_t launch_batch_greedy(const BatchInst* insts, const Tile* tiles, int n_tiles, int maxK, int maxJ,
                               int kind, uint8_t* pi, hipStream_t s) {
  if (n_tiles == 0) return hipSuccess;
  return dispatch_kj_b(maxK, maxJ, [&](auto km, auto jm) {
    constexpr int KM = decltype(km)::value, JM = decltype(jm)::value;
    hipLaunchKernelGGL((batch_greedy_kernel<KM, JM>), dim3(n_tiles), dim3(kBlock), 0, s, insts, tiles,
                       kind, pi);
    return hipGetLastError();
  });
}

hipError_t launch_batch_check(const BatchInst* insts, const Tile* tiles, int n_tiles, int maxK, int maxJ,
                              const uint8_t* pi, int* flags, hipStream_t s) {
  if (n_tiles == 0) return hipSuccess;
  return dispatch_kj_b(maxK, maxJ, [&](auto km, auto jm) {
    constexpr int KM = decltype(km)::value, JM = decltype(jm)::value;
    hipLaunchKernelGGL((batch_check_kernel<KM, JM>), dim3(n_tiles), dim3(kBlock), 0, s, insts, tiles, pi,
                       flags);
    return hipGetLastError();
  });
}

size_t batch_grad_partial_doubles(int n_tiles, int maxJ) {
  return static_cast<size_t>(n_tiles) * (2 * (maxJ <= 4 ? 4 : 8) + 2);
}

hipError_t launch_batch_grad(const BatchInst* insts, const Tile* tiles, int n_tiles, const int32_t* tile_begin,
                             int n, int maxK, int maxJ, const uint8_t* pi, const double* V, const float* w,
                             double* partial, double* out, hipStream_t s) {
  if (n_tiles == 0) return hipSuccess;
  return dispatch_kj_b(maxK, maxJ, [&](auto km, auto jm) {
    constexpr int KM = decltype(km)::value, JM = decltype(jm)::value;
    hipLaunchKernelGGL((batch_grad_partial_kernel<KM, JM>), dim3(n_tiles), dim3(kBlock), 0, s, insts, tiles,
                       pi, V, w, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((batch_grad_final_kernel<JM>), dim3(n), dim3(64), 0, s, insts, tile_begin, partial, V,
                       out);
    return hipGetLastError();
  });
}

}  // namespace mdpvi
