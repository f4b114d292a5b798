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
#include "batch.hpp"
#include "device.hpp"
#include "kernels.hpp"
#include "sweep_impl.hpp"

#include <type_traits>

namespace mdpvi {

// ---------------------------------------------------------------- LDS form

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

// ---------------------------------------------------------------- round form

// Per-instance control of the round form.
__device__ __forceinline__ bool inst_stopped(BatchCtl* c, long long j, double tol, int* remaining,
                                             bool leader) {
  __shared__ int stop;
  if (threadIdx.x < kWave) {
    bool s = load_agent(&c->done_iter) >= 0;
    if (!s && j > 0) {
      double v = __longlong_as_double(static_cast<long long>(
          load_agent(&c->res[(j - 1) % kResSlots][threadIdx.x % kBatchLanes][0])));
      v = wave_max(v);
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

template <int KMAX, int JMAX>
__global__ __launch_bounds__(kBlock) void batch_round_kernel(const BatchInst* __restrict__ insts,
                                                              const Tile* __restrict__ tiles,
                                                              float* __restrict__ V,
                                                              float* __restrict__ W,
                                                              BatchCtl* __restrict__ ctl,
                                                              int* remaining, long long j, double tol) {
  const Tile T = tiles[blockIdx.x];
  const int i = T.inst;
  const BatchInst& I = insts[i];
  const Model& M = I.M;
  BatchCtl* c = ctl + I.ctl;
  if (inst_stopped(c, j, tol, remaining, T.first != 0 ? false : true)) return;
  const float* Vin = ((j & 1) ? W : V) + I.offset;
  float* Vout = ((j & 1) ? V : W) + I.offset;
  double dmax = 0.0;
#pragma unroll
  for (int k = 0; k < kOccPerThread; ++k) {
    const uint32_t o = T.first + threadIdx.x + k * kBlock;
    if (o < static_cast<uint32_t>(M.n_occ)) {
      const double d = backup_occupancy<KMAX, JMAX, uint32_t>(M, Vin, Vout, o);
      dmax = (d > dmax || d != d) ? d : dmax;
    }
  }
  __shared__ double part[kBlock / kWave];
  dmax = wave_max(dmax);
  if (threadIdx.x % kWave == 0) part[threadIdx.x / kWave] = dmax;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = part[0];
#pragma unroll
    for (int w = 1; w < kBlock / kWave; ++w) m = (part[w] > m || part[w] != part[w]) ? part[w] : m;
    if (m != 0.0)
      atomicMax(&c->res[j % kResSlots][(T.first / (kBlock * kOccPerThread)) % kBatchLanes][0],
                static_cast<unsigned long long>(__double_as_longlong(m)));
  }
}

// Copies the final iterate of instances that stopped after an odd number of
// sweeps (it lives in W) back to V, and reports iterations and residuals.
__global__ void batch_round_finish_kernel(const BatchInst* __restrict__ insts,
                                          const int32_t* __restrict__ list, int n_list,
                                          float* __restrict__ V, const float* __restrict__ W,
                                          BatchCtl* __restrict__ ctl, long long issued,
                                          BatchOut* __restrict__ out) {
  const int li = blockIdx.y;
  if (li >= n_list) return;
  const int i = list[li];
  const BatchInst& I = insts[i];
  BatchCtl* c = ctl + I.ctl;
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
    for (int l = 0; l < kBatchLanes; ++l) {
      const double v =
          __longlong_as_double(static_cast<long long>(load_agent(&c->res[(fin - 1) % kResSlots][l][0])));
      r = (v > r || v != v) ? v : r;
    }
    out[i].iterations = fin;
    out[i].residual = r;
  }
}

__global__ void batch_ctl_init_kernel(BatchCtl* ctl, int n, int* remaining) {
  const int i = blockIdx.x;
  if (i < n) {
    if (threadIdx.x == 0) ctl[i].done_iter = -1;
    for (int w = threadIdx.x; w < kResSlots * kBatchLanes; w += blockDim.x)
      ctl[i].res[w / kBatchLanes][w % kBatchLanes][0] = 0ull;
  }
  if (i == 0 && threadIdx.x == 0) *remaining = n;
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

hipError_t launch_batch_ctl_init(BatchCtl* ctl, int n, int* remaining, hipStream_t s) {
  hipLaunchKernelGGL(batch_ctl_init_kernel, dim3(n > 0 ? n : 1), dim3(64), 0, s, ctl, n, remaining);
  return hipGetLastError();
}

hipError_t launch_batch_round(const BatchInst* insts, const Tile* tiles, int n_tiles, int maxK,
                              int maxJ, float* V, float* W, BatchCtl* ctl, int* remaining,
                              long long j, double tol, hipStream_t s) {
  if (n_tiles == 0) return hipSuccess;
  return dispatch_kj_b(maxK, maxJ, [&](auto km, auto jm) {
    constexpr int KM = decltype(km)::value, JM = decltype(jm)::value;
    hipLaunchKernelGGL((batch_round_kernel<KM, JM>), dim3(n_tiles), dim3(kBlock), 0, s, insts, tiles,
                       V, W, ctl, remaining, j, tol);
    return hipGetLastError();
  });
}

hipError_t launch_batch_round_finish(const BatchInst* insts, const int32_t* list, int n_list,
                                     float* V, const float* W, BatchCtl* ctl, long long issued,
                                     BatchOut* out, hipStream_t s) {
  if (n_list == 0) return hipSuccess;
  hipLaunchKernelGGL(batch_round_finish_kernel, dim3(64, n_list), dim3(256), 0, s, insts, list, n_list,
                     V, W, ctl, issued, out);
  return hipGetLastError();
}

}  // namespace mdpvi
