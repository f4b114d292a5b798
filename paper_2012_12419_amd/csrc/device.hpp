// device.hpp -- device helpers shared by the kernels: digit decoding of the
// mixed-radix occupancy index, the XCD-aware block order, the wavefront /
// workgroup max-reduction of the residual, and the sweep-loop control test.
#pragma once

#include "model.hpp"

namespace mdpvi {


// Raw buffer views of value arrays for the exact-shape kernels: a load takes
// a 32-bit per-lane byte offset plus a wavefront-uniform byte offset (held in
// a scalar register), so a gather costs no 64-bit address arithmetic.  The
// per-lane offset always stays inside the array (stand-in addresses replace
// the neighbours that do not exist) and the uniform offset only selects the
// class block, so every access is in bounds.  Arrays must stay below 2 GiB.
struct BufView {
  __amdgpu_buffer_rsrc_t r;
};

__device__ __forceinline__ BufView make_view(const void* p, uint32_t bytes) {
  return BufView{__builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), static_cast<short>(0),
                                                   static_cast<int>(bytes), 0x00020000)};
}

__device__ __forceinline__ float ld_f32(BufView v, uint32_t lane_off, uint32_t uni_off) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(v.r, lane_off, uni_off, 0));
}

__device__ __forceinline__ double ld_f64(BufView v, uint32_t lane_off, uint32_t uni_off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(v.r, lane_off, uni_off, 0));
}

__device__ __forceinline__ int ld_u8(BufView v, uint32_t lane_off, uint32_t uni_off) {
  return static_cast<int>(__builtin_amdgcn_raw_buffer_load_b8(v.r, lane_off, uni_off, 0));
}

typedef unsigned int U32x2 __attribute__((__vector_size__(8)));

__device__ __forceinline__ void st_f32(BufView v, float x, uint32_t lane_off, uint32_t uni_off) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(x), v.r, lane_off, uni_off, 0);
}

__device__ __forceinline__ void st_f64(BufView v, double x, uint32_t lane_off, uint32_t uni_off) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U32x2, x), v.r, lane_off, uni_off, 0);
}

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

// Control words are read and written with agent-scope atomics: the L2 of
// each XCD is not coherent with the others inside a kernel.
__device__ __forceinline__ long long load_agent(const long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long load_agent(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned int load_agent(const unsigned int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double load_agent(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void store_agent(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

enum class ResKind { kMax, kSum };

// End of a max-norm sweep: the workgroup's largest |V' - V| is stored to
// res[r * grid + b]; if it is not below tol the workgroup raises go[r]
// (and nan[r] for a NaN).  No atomics.
template <int NB = kBlock>
__device__ __forceinline__ void block_max_to(double v, Ctl* ctl, double* res, long long j, double tol) {
  __shared__ double part[NB / kWave];
  v = wave_max(v);
  const int lane = threadIdx.x % kWave;
  const int wid = threadIdx.x / kWave;
  if (lane == 0) part[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = part[0];
#pragma unroll
    for (int w = 1; w < NB / kWave; ++w) m = (part[w] > m || part[w] != part[w]) ? part[w] : m;
    const int r = static_cast<int>(j % kResSlots);
    const int x = blockIdx.x % kNumXcd;
    res[static_cast<size_t>(r) * gridDim.x + blockIdx.x] = m;
    volatile unsigned int* go = &ctl->go[r][x][0];
    if (!(m < tol) && *go == 0u) *go = 1u;
    volatile unsigned int* nn = &ctl->nan[r][x][0];
    if (m != m && *nn == 0u) *nn = 1u;
  }
}

// End of a 1-norm sweep: the workgroup's sum of |w' - w| is added to its
// residual word.
__device__ __forceinline__ void block_sum_to(double v, double* res, long long j) {
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
    if (m != 0.0) atomicAdd(res + sum_word(j, blockIdx.x % kResLanes), m);
  }
}

// Sweep-loop control, run at the top of the sweep with index j (computing
// V^{j+1} from V^j).  Returns true (for the whole workgroup) when the loop
// has already stopped: a previous sweep met the test, or sweep j-1 met it
// (max norm: nobody raised go; 1-norm: the sum of its words is below tol) or
// produced a NaN, in which case workgroup 0 records done_iter = j.
// Otherwise workgroup 0 clears the words of sweep j+1 (nobody reads or
// writes them during sweep j).
template <ResKind RK>
__device__ __forceinline__ bool sweep_stopped(Ctl* ctl, double* res, long long j, double tol) {
  __shared__ int stop;
  if (threadIdx.x < kWave) {
    bool s = load_agent(&ctl->done_iter) >= 0;
    if (!s && j > 0) {
      const int r = static_cast<int>((j - 1) % kResSlots);
      if constexpr (RK == ResKind::kMax) {
        const int x = threadIdx.x % kNumXcd;
        const bool up = load_agent(&ctl->go[r][x][0]) != 0u;
        const bool bad = load_agent(&ctl->nan[r][x][0]) != 0u;
        s = __ballot(bad) != 0 || __ballot(up) == 0;
      } else {
        double v = load_agent(res + sum_word(j - 1, threadIdx.x % kResLanes));
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
        s = !(v >= tol);
      }
      if (s && blockIdx.x == 0 && threadIdx.x == 0) store_agent(&ctl->done_iter, j);
    }
    if (threadIdx.x == 0) stop = s ? 1 : 0;
  }
  __syncthreads();
  if (stop) return true;
  if (blockIdx.x == 0 && threadIdx.x < kResLanes) {
    const int r = static_cast<int>((j + 1) % kResSlots);
    if constexpr (RK == ResKind::kMax) {
      if (threadIdx.x < kNumXcd) {
        store_agent(&ctl->go[r][threadIdx.x][0], 0u);
        store_agent(&ctl->nan[r][threadIdx.x][0], 0u);
      }
    } else {
      store_agent(res + sum_word(j + 1, threadIdx.x), 0.0);
    }
  }
  return false;
}

}  // namespace mdpvi
