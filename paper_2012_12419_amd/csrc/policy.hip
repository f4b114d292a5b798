// policy.hip -- greedy extraction (Alg. 3, step 4), fixed-policy evaluation
// (the Bellman equation of Eq. (18) without the max) and the fast greedy
// heuristic of Alg. 2 as a fixed policy.
//
// Same stencil and work split as the value-iteration sweep: one thread per
// occupancy vector, all J classes of it, neighbour reads contiguous along
// the host-0 digit.
#include "device.hpp"
#include "kernels.hpp"

#include <type_traits>

namespace mdpvi {

// Arrival term A(m) = sum_j lambda_j/Lam V(m, j), FP64.
template <int JMAX, typename T, typename Idx>
__device__ __forceinline__ double arrival(const Model& M, const T* __restrict__ V, Idx m, Idx nocc) {
  double A = 0.0;
#pragma unroll
  for (int jj = 0; jj < JMAX; ++jj)
    if (jj < M.J) A = fma(M.p[jj], static_cast<double>(V[m + jj * nocc]), A);
  return A;
}

// Release / reset / idle term D(n, e) (action independent), FP64.
template <int KMAX, typename T, typename Idx>
__device__ __forceinline__ double no_arrival(const Model& M, const T* __restrict__ V, Idx base,
                                             const int (&n)[KMAX], int load) {
  double D = M.mu_L * static_cast<double>(M.KC - load) * static_cast<double>(V[base]);
  double rs = 0.0;
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    if (k < M.K) {
      const Idx st = static_cast<Idx>(M.stride[k]);
      if (n[k] > 0) D = fma(M.mu_L * n[k], static_cast<double>(V[base - st]), D);
      rs += static_cast<double>(V[base - static_cast<Idx>(n[k]) * st]);
    }
  }
  return fma(M.nu_L, rs, D);
}

template <int KMAX, int JMAX, typename T, typename Idx>
__global__ __launch_bounds__(kBlock) void extract_kernel(Model M, const T* __restrict__ V,
                                                          uint8_t* __restrict__ pi,
                                                          float* __restrict__ gap) {
  const Idx o = static_cast<Idx>(blockIdx.x) * kBlock + threadIdx.x;
  if (o >= static_cast<Idx>(M.n_occ)) return;
  const Idx nocc = static_cast<Idx>(M.n_occ);
  int n[KMAX];
  decode<KMAX>(M, o, n);
  int load = 0;
#pragma unroll
  for (int k = 0; k < KMAX; ++k) load += n[k];
  const double a_rej = arrival<JMAX>(M, V, o, nocc);
#pragma unroll
  for (int e = 0; e < JMAX; ++e) {
    if (e < M.J) {
      const Idx base = o + e * nocc;
      const double D = no_arrival<KMAX>(M, V, base, n, load);
      const int se = M.size[e];
      double best = 0.0, second = 0.0;
      int arg = -1;
      bool have_second = false;
#pragma unroll
      for (int a = 0; a <= KMAX; ++a) {
        if (a <= M.K) {
          double q;
          if (a < M.K) {
            if (n[a] + se > M.C) continue;
            const Idx m = o + static_cast<Idx>(se) * static_cast<Idx>(M.stride[a]);
            q = fma(M.gamma, arrival<JMAX>(M, V, m, nocc) + D, M.r_place[e]);
          } else {
            q = fma(M.gamma, a_rej + D, M.r_reject[e]);
          }
          if (arg < 0) {
            best = q;
            arg = a;
          } else if (q > best) {
            second = best;
            have_second = true;
            best = q;
            arg = a;
          } else if (!have_second || q > second) {
            second = q;
            have_second = true;
          }
        }
      }
      pi[base] = static_cast<uint8_t>(arg);
      if (gap) gap[base] = have_second ? static_cast<float>(best - second) : INFINITY;
    }
  }
}

template <int KMAX, int JMAX, typename Idx>
__global__ __launch_bounds__(kBlock) void policy_check_kernel(Model M, const uint8_t* __restrict__ pi,
                                                               Ctl* ctl) {
  const Idx o = static_cast<Idx>(blockIdx.x) * kBlock + threadIdx.x;
  if (o >= static_cast<Idx>(M.n_occ)) return;
  const Idx nocc = static_cast<Idx>(M.n_occ);
  int n[KMAX];
  decode<KMAX>(M, o, n);
  bool bad = false;
#pragma unroll
  for (int e = 0; e < JMAX; ++e) {
    if (e < M.J) {
      const int a = pi[o + e * nocc];
      if (a > M.K) {
        bad = true;
      } else if (a < M.K) {
        int na = 0;
#pragma unroll
        for (int k = 0; k < KMAX; ++k)
          if (k == a) na = n[k];
        if (na + M.size[e] > M.C) bad = true;
      }
    }
  }
  if (bad) ctl->flag = 1;
}

template <int KMAX, int JMAX, typename Idx>
__global__ __launch_bounds__(kBlock) void eval_sweep_kernel(Model M, const uint8_t* __restrict__ pi,
                                                             const double* __restrict__ Vin,
                                                             double* __restrict__ Vout, Ctl* ctl,
                                                             long long j, double tol) {
  if (sweep_stopped<ResKind::kMax>(ctl, j, tol)) return;
  const uint32_t b = xcd_block(blockIdx.x, gridDim.x);
  double dmax = 0.0;
  for (int i = 0; i < kOccPerThread; ++i) {
    const Idx o = static_cast<Idx>(b) * (kBlock * kOccPerThread) + threadIdx.x +
                  static_cast<Idx>(i * kBlock);
    if (o >= static_cast<Idx>(M.n_occ)) break;
    const Idx nocc = static_cast<Idx>(M.n_occ);
    int n[KMAX];
    decode<KMAX>(M, o, n);
    int load = 0;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) load += n[k];
#pragma unroll
    for (int e = 0; e < JMAX; ++e) {
      if (e < M.J) {
        const Idx base = o + e * nocc;
        const int a = pi[base];
        Idx m = o;
        double r = M.r_reject[e];
        if (a < M.K) {
          Idx st = 0;
#pragma unroll
          for (int k = 0; k < KMAX; ++k)
            if (k == a) st = static_cast<Idx>(M.stride[k]);
          m = o + static_cast<Idx>(M.size[e]) * st;
          r = M.r_place[e];
        }
        const double D = no_arrival<KMAX>(M, Vin, base, n, load);
        const double A = arrival<JMAX>(M, Vin, m, nocc);
        const double vn = fma(M.gamma, D, fma(M.gamma, A, r));
        const double old = Vin[base];
        Vout[base] = vn;
        const double d = fabs(vn - old);
        dmax = (d > dmax || d != d) ? d : dmax;
      }
    }
  }
  block_max_to(dmax, ctl, j);
}

template <int KMAX, int JMAX, typename Idx>
__global__ __launch_bounds__(kBlock) void greedy_kernel(Model M, int kind, uint8_t* __restrict__ pi) {
  const Idx o = static_cast<Idx>(blockIdx.x) * kBlock + threadIdx.x;
  if (o >= static_cast<Idx>(M.n_occ)) return;
  const Idx nocc = static_cast<Idx>(M.n_occ);
  int n[KMAX];
  decode<KMAX>(M, o, n);
#pragma unroll
  for (int e = 0; e < JMAX; ++e) {
    if (e < M.J) {
      int choice = M.K;
      int least = M.C + 1;
#pragma unroll
      for (int a = 0; a < KMAX; ++a) {
        if (a < M.K && n[a] + M.size[e] <= M.C) {
          if (kind == 0) {
            if (n[a] < least) {
              least = n[a];
              choice = a;
            }
          } else if (choice == M.K) {
            choice = a;
          }
        }
      }
      pi[o + e * nocc] = static_cast<uint8_t>(choice);
    }
  }
}

// ---------------------------------------------------------------- launchers

static inline dim3 occ_grid(const Model& M) {
  return dim3(static_cast<uint32_t>((static_cast<uint64_t>(M.n_occ) + kBlock - 1) / kBlock));
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

hipError_t launch_eval_sweep(const Model& M, const uint8_t* pi, const double* Vin, double* Vout,
                             Ctl* ctl, long long j, double tol, hipStream_t s) {
  if (use_32bit_index(M)) {
    return dispatch_kj(M, [&](auto km, auto jm) {
      constexpr int KM = decltype(km)::value, JM = decltype(jm)::value;
      hipLaunchKernelGGL((eval_sweep_kernel<KM, JM, uint32_t>), sweep_grid(M),
                                           dim3(kBlock), 0, s, M, pi, Vin, Vout, ctl, j, tol);
      return hipGetLastError();
    });
  } else {
    return dispatch_kj(M, [&](auto km, auto jm) {
      constexpr int KM = decltype(km)::value, JM = decltype(jm)::value;
      hipLaunchKernelGGL((eval_sweep_kernel<KM, JM, uint64_t>), sweep_grid(M),
                                           dim3(kBlock), 0, s, M, pi, Vin, Vout, ctl, j, tol);
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
