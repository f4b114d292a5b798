// device.hpp -- device helpers shared by the kernels: digit decoding of the
// mixed-radix occupancy index, the XCD-aware block order, the wavefront /
// workgroup max-reduction of the residual, and the sweep-loop control test.
#pragma once

#include "model.hpp"

namespace mdpvi {

constexpr int kBlock = 256;     // 4 wavefronts of 64
constexpr int kWave = 64;
constexpr int kNumXcd = 8;      // MI355X: 8 accelerator complex dies, 32 CUs each

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

// Max of v over the workgroup, then one atomicMax of its bit pattern into dst
// (v >= 0 or NaN; NaN bit patterns order above +inf).
__device__ __forceinline__ void block_max_to(double v, unsigned long long* dst) {
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
    if (m != 0.0) atomicMax(dst, static_cast<unsigned long long>(__double_as_longlong(m)));
  }
}

// Sweep-loop control, run at the top of the sweep with index j (computing
// V^{j+1} from V^j).  Returns true when the loop has already stopped: a
// previous sweep met the test, or the residual of sweep j-1 is below tol (or
// NaN), in which case workgroup 0 records done_iter = j.  Otherwise workgroup
// 0 clears the residual slot of sweep j+1 (nobody reads or writes it during
// sweep j).
__device__ __forceinline__ bool sweep_stopped(Ctl* ctl, long long j, double tol) {
  if (__atomic_load_n(&ctl->done_iter, __ATOMIC_RELAXED) >= 0) return true;
  if (j > 0) {
    double prev = __longlong_as_double(static_cast<long long>(
        __atomic_load_n(&ctl->res[(j - 1) % kResSlots], __ATOMIC_RELAXED)));
    if (!(prev >= tol)) {
      if (blockIdx.x == 0 && threadIdx.x == 0) ctl->done_iter = j;
      return true;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) ctl->res[(j + 1) % kResSlots] = 0ull;
  return false;
}

}  // namespace mdpvi
