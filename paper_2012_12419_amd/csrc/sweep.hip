// sweep.hip -- the synchronous (Jacobi) value-iteration sweep.
//
// One sweep applies the Bellman operator of Eq. (18) to every state from the
// previous iterate (Alg. 3, step 2) and measures ||V^{j+1} - V^j||_inf
// (Alg. 3, step 3).  The backup is matrix-free: from state (n, e) a
// uniformised step reaches only
//   (m_a, j)        arrival of the next class j, after the pending class-e
//                   task was placed on host a (m_a = n + size_e 1_a) or sent
//                   to the paid cloud (m = n),
//   (n - 1_k, e)    one occupied unit of host k released,
//   (n^{k<-0}, e)   host k left and was replaced empty,
//   (n, e)          idle,
// so the sweep is a K-dimensional stencil on the (C+1)^K occupancy grid.
//
// Work split: one thread per occupancy vector n, computing all J classes of
// it.  The arrival term A(m) = sum_j lambda_j/Lam V(m, j) is shared by every
// class with the same task size, and the release / reset / idle term
//   D(n, e) = sum_k mu n_k/Lam V(n - 1_k, e) + nu/Lam sum_k V(n^{k<-0}, e)
//           + mu (KC - |n|)/Lam V(n, e)
// (the idle probability 1 - P_arr - (mu|n| + K nu)/Lam written as the
// non-negative mu (KC - |n|)/Lam) does not depend on the action, so
//   V'(n, e) = gamma D(n, e) + max( P_arr r_e + gamma max_a A(m_a),
//                                  -P_arr c_e + gamma A(n) ).
// Consecutive threads own consecutive occupancies (host 0 digit), so every
// neighbour read of a wavefront is a contiguous run of the value array.
//
// Precision: values are stored in FP32; every sum is formed in FP64 with
// non-negative weights and rounded once.  All operations are monotone in V,
// so from a sub-solution the iterates increase to an exact FP32 fixed point.
#include "device.hpp"
#include "kernels.hpp"
#include "sweep_impl.hpp"

namespace mdpvi {

// Each workgroup owns kOccPerThread * kBlock consecutive occupancies
// (XCD-aware order), each thread kOccPerThread of them strided by kBlock so
// that every load of a wavefront stays contiguous.
template <int KMAX, int JMAX, typename Idx>
__global__ __launch_bounds__(kBlock) void vi_sweep_kernel(Model M, const float* __restrict__ Vin,
                                                           float* __restrict__ Vout, Ctl* ctl,
                                                           long long j, double tol) {
  if (sweep_stopped<ResKind::kMax>(ctl, j, tol)) return;
  const uint32_t b = xcd_block(blockIdx.x, gridDim.x);
  const Idx base = static_cast<Idx>(b) * (kBlock * kOccPerThread) + threadIdx.x;
  double dmax = 0.0;
#pragma unroll
  for (int i = 0; i < kOccPerThread; ++i) {
    const Idx o = base + static_cast<Idx>(i * kBlock);
    if (o < static_cast<Idx>(M.n_occ)) {
      const double d = backup_occupancy<KMAX, JMAX>(M, Vin, Vout, o);
      dmax = (d > dmax || d != d) ? d : dmax;
    }
  }
  block_max_to(dmax, ctl, j);
}

__global__ void ctl_init_kernel(Ctl* ctl) {
  if (threadIdx.x == 0) {
    ctl->done_iter = -1;
    ctl->flag = 0;
  }
  for (int w = threadIdx.x; w < kResSlots * kResLanes; w += blockDim.x)
    ctl->res[w / kResLanes][w % kResLanes][0] = 0ull;
}

hipError_t launch_ctl_init(Ctl* ctl, hipStream_t s) {
  hipLaunchKernelGGL(ctl_init_kernel, dim3(1), dim3(256), 0, s, ctl);
  return hipGetLastError();
}

template <int KMAX, int JMAX, typename Idx>
static hipError_t launch_sweep_t(const Model& M, const float* Vin, float* Vout, Ctl* ctl,
                                 long long j, double tol, hipStream_t s) {
  const uint64_t per = static_cast<uint64_t>(kBlock) * kOccPerThread;
  const uint64_t grid = (static_cast<uint64_t>(M.n_occ) + per - 1) / per;
  hipLaunchKernelGGL((vi_sweep_kernel<KMAX, JMAX, Idx>), dim3(static_cast<uint32_t>(grid)),
                     dim3(kBlock), 0, s, M, Vin, Vout, ctl, j, tol);
  return hipGetLastError();
}

template <typename Idx>
static hipError_t launch_sweep_idx(const Model& M, const float* Vin, float* Vout, Ctl* ctl,
                                   long long j, double tol, hipStream_t s) {
  if (M.J <= 4) {
    if (M.K <= 4) return launch_sweep_t<4, 4, Idx>(M, Vin, Vout, ctl, j, tol, s);
    if (M.K <= 8) return launch_sweep_t<8, 4, Idx>(M, Vin, Vout, ctl, j, tol, s);
    return launch_sweep_t<16, 4, Idx>(M, Vin, Vout, ctl, j, tol, s);
  }
  if (M.K <= 4) return launch_sweep_t<4, 8, Idx>(M, Vin, Vout, ctl, j, tol, s);
  if (M.K <= 8) return launch_sweep_t<8, 8, Idx>(M, Vin, Vout, ctl, j, tol, s);
  return launch_sweep_t<16, 8, Idx>(M, Vin, Vout, ctl, j, tol, s);
}

hipError_t launch_vi_sweep(const Model& M, const float* Vin, float* Vout, Ctl* ctl, long long j,
                           double tol, hipStream_t s) {
  if (use_32bit_index(M)) return launch_sweep_idx<uint32_t>(M, Vin, Vout, ctl, j, tol, s);
  return launch_sweep_idx<uint64_t>(M, Vin, Vout, ctl, j, tol, s);
}

}  // namespace mdpvi
