// policy.hip -- greedy extraction (Alg. 3, step 4), fixed-policy evaluation
// (the Bellman equation of Eq. (18) without the max) and the fast greedy
// heuristic of Alg. 2 as a fixed policy.
//
// Same stencil and work split as the value-iteration sweep: one thread per
// occupancy vector, all J classes of it, neighbour reads contiguous along
// the host-0 digit.
#include "device.hpp"
#include "kernels.hpp"
#include "policy_impl.hpp"

#include <type_traits>

namespace mdpvi {

template <int KMAX, int JMAX, typename T, typename Idx>
__global__ __launch_bounds__(kBlock) void extract_kernel(Model M, const T* __restrict__ V,
                                                          uint8_t* __restrict__ pi,
                                                          float* __restrict__ gap) {
  const Idx o = static_cast<Idx>(blockIdx.x) * kBlock + threadIdx.x;
  if (o < static_cast<Idx>(M.n_occ)) extract_occupancy<KMAX, JMAX>(M, V, pi, gap, o);
}

template <int KMAX, int JMAX, typename Idx>
__global__ __launch_bounds__(kBlock) void policy_check_kernel(Model M, const uint8_t* __restrict__ pi,
                                                               Ctl* ctl) {
  const Idx o = static_cast<Idx>(blockIdx.x) * kBlock + threadIdx.x;
  if (o < static_cast<Idx>(M.n_occ) && check_occupancy<KMAX, JMAX>(M, pi, o)) ctl->flag = 1;
}

template <int KMAX, int JMAX, typename Idx>
__global__ __launch_bounds__(kBlock) void eval_sweep_kernel(Model M, const uint8_t* __restrict__ pi,
                                                             const double* __restrict__ Vin,
                                                             double* __restrict__ Vout, Ctl* ctl,
                                                             double* res, long long j, double tol) {
  if (sweep_stopped<ResKind::kMax>(ctl, res, j, tol)) return;
  const uint32_t b = xcd_block(blockIdx.x, gridDim.x);
  double dmax = 0.0;
#pragma unroll
  for (int i = 0; i < kOccPerThread; ++i) {
    const Idx o = static_cast<Idx>(b) * (kBlock * kOccPerThread) + threadIdx.x +
                  static_cast<Idx>(i * kBlock);
    if (o < static_cast<Idx>(M.n_occ)) {
      const double d = eval_occupancy<KMAX, JMAX>(M, pi, Vin, Vout, o);
      dmax = (d > dmax || d != d) ? d : dmax;
    }
  }
  block_max_to(dmax, ctl, res, j, tol);
}

template <int KMAX, int JMAX, typename Idx>
__global__ __launch_bounds__(kBlock) void greedy_kernel(Model M, int kind, uint8_t* __restrict__ pi) {
  const Idx o = static_cast<Idx>(blockIdx.x) * kBlock + threadIdx.x;
  if (o < static_cast<Idx>(M.n_occ)) greedy_occupancy<KMAX, JMAX>(M, kind, pi, o);
}

template <int K, int J>
__global__ __launch_bounds__(kBlock) void eval_exact_kernel(Model M, const uint8_t* __restrict__ pi,
                                                             const double* __restrict__ Vin,
                                                             double* __restrict__ Vout, Ctl* ctl,
                                                             double* res, long long j, double tol) {
  if (sweep_stopped<ResKind::kMax>(ctl, res, j, tol)) return;
  const uint32_t b = xcd_block(blockIdx.x, gridDim.x);
  const uint32_t o = b * kBlock + threadIdx.x;
  double dmax = 0.0;
  const BufView pv = make_view(pi, static_cast<uint32_t>(M.n_states));
  const BufView vin = make_view(Vin, static_cast<uint32_t>(M.n_states) * 8u);
  if (o < static_cast<uint32_t>(M.n_occ)) dmax = eval_exact<K, J>(M, pv, vin, Vout, o);
  block_max_to(dmax, ctl, res, j, tol);
}

// ---------------------------------------------------------------- launchers

static inline dim3 occ_grid(const Model& M) {
  return dim3(static_cast<uint32_t>((static_cast<uint64_t>(M.n_occ) + kBlock - 1) / kBlock));
}

static bool eval_exact_shape(const Model& M) {
  return M.n_states < (int64_t{1} << 28) && M.K >= 1 && M.K <= 8 && M.J >= 1 && M.J <= 3;
}

template <int K, int J>
static hipError_t launch_eval_exact_t(const Model& M, const uint8_t* pi, const double* Vin, double* Vout,
                                      Ctl* ctl, double* res, long long j, double tol, hipStream_t s) {
  const uint32_t grid = static_cast<uint32_t>((static_cast<uint64_t>(M.n_occ) + kBlock - 1) / kBlock);
  hipLaunchKernelGGL((eval_exact_kernel<K, J>), dim3(grid), dim3(kBlock), 0, s, M, pi, Vin, Vout, ctl, res,
                     j, tol);
  return hipGetLastError();
}

static hipError_t launch_eval_exact(const Model& M, const uint8_t* pi, const double* Vin, double* Vout,
                                    Ctl* ctl, double* res, long long j, double tol, hipStream_t s) {
  switch (M.K * 4 + M.J) {
    case 5: return launch_eval_exact_t<1, 1>(M, pi, Vin, Vout, ctl, res, j, tol, s);
    case 6: return launch_eval_exact_t<1, 2>(M, pi, Vin, Vout, ctl, res, j, tol, s);
    case 7: return launch_eval_exact_t<1, 3>(M, pi, Vin, Vout, ctl, res, j, tol, s);
    case 9: return launch_eval_exact_t<2, 1>(M, pi, Vin, Vout, ctl, res, j, tol, s);
    case 10: return launch_eval_exact_t<2, 2>(M, pi, Vin, Vout, ctl, res, j, tol, s);
    case 11: return launch_eval_exact_t<2, 3>(M, pi, Vin, Vout, ctl, res, j, tol, s);
    case 13: return launch_eval_exact_t<3, 1>(M, pi, Vin, Vout, ctl, res, j, tol, s);
    case 14: return launch_eval_exact_t<3, 2>(M, pi, Vin, Vout, ctl, res, j, tol, s);
    case 15: return launch_eval_exact_t<3, 3>(M, pi, Vin, Vout, ctl, res, j, tol, s);
    case 17: return launch_eval_exact_t<4, 1>(M, pi, Vin, Vout, ctl, res, j, tol, s);
    case 18: return launch_eval_exact_t<4, 2>(M, pi, Vin, Vout, ctl, res, j, tol, s);
    case 19: return launch_eval_exact_t<4, 3>(M, pi, Vin, Vout, ctl, res, j, tol, s);
    case 21: return launch_eval_exact_t<5, 1>(M, pi, Vin, Vout, ctl, res, j, tol, s);
    case 22: return launch_eval_exact_t<5, 2>(M, pi, Vin, Vout, ctl, res, j, tol, s);
    case 23: return launch_eval_exact_t<5, 3>(M, pi, Vin, Vout, ctl, res, j, tol, s);
    case 25: return launch_eval_exact_t<6, 1>(M, pi, Vin, Vout, ctl, res, j, tol, s);
    case 26: return launch_eval_exact_t<6, 2>(M, pi, Vin, Vout, ctl, res, j, tol, s);
    case 27: return launch_eval_exact_t<6, 3>(M, pi, Vin, Vout, ctl, res, j, tol, s);
    case 29: return launch_eval_exact_t<7, 1>(M, pi, Vin, Vout, ctl, res, j, tol, s);
    case 30: return launch_eval_exact_t<7, 2>(M, pi, Vin, Vout, ctl, res, j, tol, s);
    case 31: return launch_eval_exact_t<7, 3>(M, pi, Vin, Vout, ctl, res, j, tol, s);
    case 33: return launch_eval_exact_t<8, 1>(M, pi, Vin, Vout, ctl, res, j, tol, s);
    case 34: return launch_eval_exact_t<8, 2>(M, pi, Vin, Vout, ctl, res, j, tol, s);
    case 35: return launch_eval_exact_t<8, 3>(M, pi, Vin, Vout, ctl, res, j, tol, s);
    default:
      return hipErrorInvalidValue;
  }
}

uint32_t eval_sweep_grid(const Model& M) {
  if (eval_exact_shape(M))
    return static_cast<uint32_t>((static_cast<uint64_t>(M.n_occ) + kBlock - 1) / kBlock);
  const uint64_t per = static_cast<uint64_t>(kBlock) * kOccPerThread;
  return static_cast<uint32_t>((static_cast<uint64_t>(M.n_occ) + per - 1) / per);
}

uint32_t occ_sweep_grid(const Model& M) {
  const uint64_t per = static_cast<uint64_t>(kBlock) * kOccPerThread;
  return static_cast<uint32_t>((static_cast<uint64_t>(M.n_occ) + per - 1) / per);
}

static inline dim3 sweep_grid(const Model& M) {
  const uint64_t per = static_cast<uint64_t>(kBlock) * kOccPerThread;
  return dim3(static_cast<uint32_t>((static_cast<uint64_t>(M.n_occ) + per - 1) / per));
}

// Calls f(KMAX, JMAX) with the smallest compiled bounds that fit M.
template <typename F>
static hipError_t dispatch_kj(const Model& M, F&& f) {
  using I4 = std::integral_constant<int, 4>;
  using I8 = std::integral_constant<int, 8>;
  using I16 = std::integral_constant<int, 16>;
  if (M.J <= 4) {
    if (M.K <= 4) return f(I4{}, I4{});
    if (M.K <= 8) return f(I8{}, I4{});
    return f(I16{}, I4{});
  }
  if (M.K <= 4) return f(I4{}, I8{});
  if (M.K <= 8) return f(I8{}, I8{});
  return f(I16{}, I8{});
}

template <typename T>
static hipError_t launch_extract_t(const Model& M, const T* V, uint8_t* pi, float* gap,
                                   hipStream_t s) {
  if (use_32bit_index(M)) {
    return dispatch_kj(M, [&](auto km, auto jm) {
      constexpr int KM = decltype(km)::value, JM = decltype(jm)::value;
      hipLaunchKernelGGL((extract_kernel<KM, JM, T, uint32_t>), occ_grid(M),
                                           dim3(kBlock), 0, s, M, V, pi, gap);
      return hipGetLastError();
    });
  } else {
    return dispatch_kj(M, [&](auto km, auto jm) {
      constexpr int KM = decltype(km)::value, JM = decltype(jm)::value;
      hipLaunchKernelGGL((extract_kernel<KM, JM, T, uint64_t>), occ_grid(M),
                                           dim3(kBlock), 0, s, M, V, pi, gap);
      return hipGetLastError();
    });
  }
  return hipGetLastError();
}

hipError_t launch_extract_f32(const Model& M, const float* V, uint8_t* pi, float* gap,
                              hipStream_t s) {
  return launch_extract_t<float>(M, V, pi, gap, s);
}

hipError_t launch_extract_f64(const Model& M, const double* V, uint8_t* pi, float* gap,
                              hipStream_t s) {
  return launch_extract_t<double>(M, V, pi, gap, s);
}

hipError_t launch_policy_check(const Model& M, const uint8_t* pi, Ctl* ctl, hipStream_t s) {
  if (use_32bit_index(M)) {
    return dispatch_kj(M, [&](auto km, auto jm) {
      constexpr int KM = decltype(km)::value, JM = decltype(jm)::value;
      hipLaunchKernelGGL((policy_check_kernel<KM, JM, uint32_t>), occ_grid(M),
                                           dim3(kBlock), 0, s, M, pi, ctl);
      return hipGetLastError();
    });
  } else {
    return dispatch_kj(M, [&](auto km, auto jm) {
      constexpr int KM = decltype(km)::value, JM = decltype(jm)::value;
      hipLaunchKernelGGL((policy_check_kernel<KM, JM, uint64_t>), occ_grid(M),
                                           dim3(kBlock), 0, s, M, pi, ctl);
      return hipGetLastError();
    });
  }
  return hipGetLastError();
}

template <int KMAX, int JMAX, typename Idx>
__global__ __launch_bounds__(kBlock) void improve_kernel(Model M, const double* __restrict__ V,
                                                          const uint8_t* __restrict__ pi_in,
                                                          uint8_t* __restrict__ pi_out, double tol) {
  const Idx o = static_cast<Idx>(blockIdx.x) * kBlock + threadIdx.x;
  if (o < static_cast<Idx>(M.n_occ)) improve_occupancy<KMAX, JMAX>(M, V, pi_in, pi_out, tol, o);
}

hipError_t launch_improve(const Model& M, const double* V, const uint8_t* pi_in, uint8_t* pi_out, double tol,
                          hipStream_t s) {
  return dispatch_kj(M, [&](auto km, auto jm) {
    constexpr int KM = decltype(km)::value, JM = decltype(jm)::value;
    if (use_32bit_index(M))
      hipLaunchKernelGGL((improve_kernel<KM, JM, uint32_t>), occ_grid(M), dim3(kBlock), 0, s, M, V, pi_in,
                         pi_out, tol);
    else
      hipLaunchKernelGGL((improve_kernel<KM, JM, uint64_t>), occ_grid(M), dim3(kBlock), 0, s, M, V, pi_in,
                         pi_out, tol);
    return hipGetLastError();
  });
}

// ctl->flag := 1 if the byte arrays a and b (n bytes) differ anywhere.
// Sixteen bytes per thread (one 16-byte load each when both arrays are
// 16-byte aligned); one store per wavefront that found a difference.
__global__ __launch_bounds__(kBlock) void policy_diff_kernel(uint64_t n, const uint8_t* __restrict__ a,
                                                              const uint8_t* __restrict__ b, Ctl* ctl) {
  const uint64_t i = (static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x) * 16u;
  bool diff = false;
  const bool aligned = ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b)) & 15u) == 0;
  if (aligned && i + 16u <= n) {
    const uint4 x = *reinterpret_cast<const uint4*>(a + i);
    const uint4 y = *reinterpret_cast<const uint4*>(b + i);
    diff = (x.x != y.x) || (x.y != y.y) || (x.z != y.z) || (x.w != y.w);
  } else {
    for (uint64_t k = i; k < n && k < i + 16u; ++k) diff = diff || (a[k] != b[k]);
  }
  if (__ballot(diff) != 0 && threadIdx.x % kWave == 0) ctl->flag = 1;
}

hipError_t launch_policy_diff(uint64_t n, const uint8_t* a, const uint8_t* b, Ctl* ctl, hipStream_t s) {
  const uint64_t threads = (n + 15) / 16;
  const uint32_t grid = static_cast<uint32_t>((threads + kBlock - 1) / kBlock);
  if (grid == 0) return hipSuccess;
  hipLaunchKernelGGL(policy_diff_kernel, dim3(grid), dim3(kBlock), 0, s, n, a, b, ctl);
  return hipGetLastError();
}

hipError_t launch_eval_sweep(const Model& M, const uint8_t* pi, const double* Vin, double* Vout,
                             Ctl* ctl, double* res, long long j, double tol, hipStream_t s) {
  if (eval_exact_shape(M)) return launch_eval_exact(M, pi, Vin, Vout, ctl, res, j, tol, s);
  if (use_32bit_index(M)) {
    return dispatch_kj(M, [&](auto km, auto jm) {
      constexpr int KM = decltype(km)::value, JM = decltype(jm)::value;
      hipLaunchKernelGGL((eval_sweep_kernel<KM, JM, uint32_t>), sweep_grid(M),
                                           dim3(kBlock), 0, s, M, pi, Vin, Vout, ctl, res, j, tol);
      return hipGetLastError();
    });
  } else {
    return dispatch_kj(M, [&](auto km, auto jm) {
      constexpr int KM = decltype(km)::value, JM = decltype(jm)::value;
      hipLaunchKernelGGL((eval_sweep_kernel<KM, JM, uint64_t>), sweep_grid(M),
                                           dim3(kBlock), 0, s, M, pi, Vin, Vout, ctl, res, j, tol);
      return hipGetLastError();
    });
  }
  return hipGetLastError();
}

hipError_t launch_greedy(const Model& M, int kind, uint8_t* pi, hipStream_t s) {
  if (use_32bit_index(M)) {
    return dispatch_kj(M, [&](auto km, auto jm) {
      constexpr int KM = decltype(km)::value, JM = decltype(jm)::value;
      hipLaunchKernelGGL((greedy_kernel<KM, JM, uint32_t>), occ_grid(M),
                                           dim3(kBlock), 0, s, M, kind, pi);
      return hipGetLastError();
    });
  } else {
    return dispatch_kj(M, [&](auto km, auto jm) {
      constexpr int KM = decltype(km)::value, JM = decltype(jm)::value;
      hipLaunchKernelGGL((greedy_kernel<KM, JM, uint64_t>), occ_grid(M),
                                           dim3(kBlock), 0, s, M, kind, pi);
      return hipGetLastError();
    });
  }
  return hipGetLastError();
}

}  // namespace mdpvi
