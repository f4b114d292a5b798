// device.hpp -- device helpers shared by the kernels: digit decoding of the
// mixed-radix occupancy index, the XCD-aware block order, the wavefront /
// workgroup max-reduction of the residual, and the sweep-loop control test.
#pragma once

#include "model.hpp"

namespace mdpvi {


// Digits n_0..n_{K-1} of occupancy index o (host 0 fastest).
template <int KMAX, typename Idx>
__device__ __forceinline__ void decode(const Model& M, Idx o, int (&n)[KMAX]) {
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    if (k < M.K) {
      if constexpr (sizeof(Idx) == 4) {
        uint32_t q = fast_div(static_cast<uint32_t>(o), M.divR);
        n[k] = static_cast<int>(static_cast<uint32_t>(o) - q * static_cast<uint32_t>(M.R));
        o = static_cast<Idx>(q);
      } else {
        n[k] = static_cast<int>(o % static_cast<Idx>(M.R));
        o /= static_cast<Idx>(M.R);
      }
    } else {
      n[k] = 0;
    }
  }
}

// Workgroups are handed to the 8 XCDs round-robin by their id.  Remap so that
// XCD x works on one contiguous range of occupancies: neighbouring tiles then
// share that XCD's L2.  Bijective: the first 8*floor(G/8) ids are permuted,
// the tail keeps its ids.
__device__ __forceinline__ uint32_t xcd_block(uint32_t bid, uint32_t grid) {
  uint32_t per = grid / kNumXcd;
  uint32_t full = per * kNumXcd;
  if (bid >= full) return bid;
  return (bid % kNumXcd) * per + bid / kNumXcd;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    double o = __shfl_xor(v, off, kWave);
    v = (o > v || o != o) ? o : v;   // a NaN wins so that it is reported
  }
  return v;
}

// Max of v over the workgroup, then one atomicMax of its bit pattern into the
// residual word of this workgroup (v >= 0 or NaN).
__device__ __forceinline__ void block_max_to(double v, Ctl* ctl, long long j) {
  __shared__ double part[kBlock / kWave];
  v = wave_max(v);
  const int lane = threadIdx.x % kWave;
  const int wid = threadIdx.x / kWave;
  if (lane == 0) part[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = part[0];
#pragma unroll
    for (int w = 1; w < kBlock / kWave; ++w) m = (part[w] > m || part[w] != part[w]) ? part[w] : m;
    if (m != 0.0)
      atomicMax(res_word(ctl, j, blockIdx.x % kResLanes),
                static_cast<unsigned long long>(__double_as_longlong(m)));
  }
}

// Sum of v over the workgroup, then one FP64 atomicAdd into the residual
// word of this workgroup (for 1-norm residuals).
__device__ __forceinline__ void block_sum_to(double v, Ctl* ctl, long long j) {
  __shared__ double part[kBlock / kWave];
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  const int lane = threadIdx.x % kWave;
  const int wid = threadIdx.x / kWave;
  if (lane == 0) part[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0.0;
#pragma unroll
    for (int w = 0; w < kBlock / kWave; ++w) m += part[w];
    if (m != 0.0) atomicAdd(reinterpret_cast<double*>(res_word(ctl, j, blockIdx.x % kResLanes)), m);
  }
}

enum class ResKind { kMax, kSum };

// Residual of sweep j from its kResLanes words, computed by the first
// wavefront of the workgroup.
// Control words are read and written with agent-scope atomics: the L2 of
// each XCD is not coherent with the others, and the residual words are
// updated by atomics performed beyond the L2.
__device__ __forceinline__ long long load_agent(const long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long load_agent(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void store_agent(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <ResKind RK>
__device__ __forceinline__ double read_residual(Ctl* ctl, long long j) {
  double v = __longlong_as_double(
      static_cast<long long>(load_agent(res_word(ctl, j, threadIdx.x % kResLanes))));
  if constexpr (RK == ResKind::kMax) {
    return wave_max(v);
  } else {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
  }
}

// Sweep-loop control, run at the top of the sweep with index j (computing
// V^{j+1} from V^j).  Returns true (for the whole workgroup) when the loop
// has already stopped: a previous sweep met the test, or the residual of
// sweep j-1 is below tol (or NaN), in which case workgroup 0 records
// done_iter = j.  Otherwise workgroup 0 clears the residual words of sweep
// j+1 (nobody reads or writes them during sweep j).
template <ResKind RK>
__device__ __forceinline__ bool sweep_stopped(Ctl* ctl, long long j, double tol) {
  __shared__ int stop;
  if (threadIdx.x < kWave) {
    bool s = load_agent(&ctl->done_iter) >= 0;
    if (!s && j > 0) {
      const double prev = read_residual<RK>(ctl, j - 1);
      if (!(prev >= tol)) {
        s = true;
        if (blockIdx.x == 0 && threadIdx.x == 0) store_agent(&ctl->done_iter, j);
      }
    }
    if (threadIdx.x == 0) stop = s ? 1 : 0;
  }
  __syncthreads();
  if (stop) return true;
  if (blockIdx.x == 0 && threadIdx.x < kResLanes) store_agent(res_word(ctl, j + 1, threadIdx.x), 0ull);
  return false;
}

}  // namespace mdpvi
