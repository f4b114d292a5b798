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
#include "tile.hpp"

namespace mdpvi {

// Each workgroup owns kOccPerThread * kBlock consecutive occupancies
// (XCD-aware order), each thread kOccPerThread of them strided by kBlock so
// that every load of a wavefront stays contiguous.
template <int KMAX, int JMAX, typename Idx>
__global__ __launch_bounds__(kBlock) void vi_sweep_kernel(Model M, const float* __restrict__ Vin,
                                                           float* __restrict__ Vout, Ctl* ctl,
                                                           double* res, long long j, double tol) {
  if (sweep_stopped<ResKind::kMax>(ctl, res, j, tol)) return;
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
  block_max_to(dmax, ctl, res, j, tol);
}


// ---------------------------------------------------------------- slab form
//
// The occupancy grid is cut into slabs: all occupancies that share the high
// digits n_t..n_{K-1}.  A workgroup stages its slab's values (all J classes)
// in LDS together with the arrival term A(o) = sum_j lambda_j/Lam V(o, j) of
// every slab occupancy (FP64), so that every neighbour along the t low
// digits (placements, releases, resets) is an LDS read; only neighbours along
// the high digits are read from global memory, still contiguous per
// wavefront.  The high digits are the same for the whole workgroup, so every
// feasibility test along them is uniform.  The arithmetic and its order are
// those of backup_occupancy: the two forms give bit-identical iterates.
template <int KMAX, int JMAX>
__global__ __launch_bounds__(kBlock) void vi_slab_kernel(Model M, int t, uint32_t slab_occ,
                                                          const float* __restrict__ Vin,
                                                          float* __restrict__ Vout, Ctl* ctl,
                                                          double* res, long long j, double tol) {
  if (sweep_stopped<ResKind::kMax>(ctl, res, j, tol)) return;
  extern __shared__ double slab_lds[];
  double* Al = slab_lds;                                     // [slab_occ]
  float* Vl = reinterpret_cast<float*>(slab_lds + slab_occ);  // [J][slab_occ]
  const uint32_t nocc = static_cast<uint32_t>(M.n_occ);
  const uint32_t slab = xcd_block(blockIdx.x, gridDim.x);
  const uint32_t o0 = slab * slab_occ;
  int nh[KMAX];
  {
    uint32_t q = slab;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      nh[k] = 0;
      if (k >= t && k < M.K) {
        const uint32_t q2 = fast_div(q, M.divR);
        nh[k] = static_cast<int>(q - q2 * static_cast<uint32_t>(M.R));
        q = q2;
      }
    }
  }
  for (uint32_t x = threadIdx.x; x < static_cast<uint32_t>(M.J) * slab_occ; x += kBlock) {
    const uint32_t e = x / slab_occ;
    const uint32_t ol = x - e * slab_occ;
    Vl[x] = Vin[o0 + ol + e * nocc];
  }
  __syncthreads();
  for (uint32_t ol = threadIdx.x; ol < slab_occ; ol += kBlock) {
    double A = 0.0;
#pragma unroll
    for (int e = 0; e < JMAX; ++e)
      if (e < M.J) A = fma(M.p[e], static_cast<double>(Vl[e * slab_occ + ol]), A);
    Al[ol] = A;
  }
  __syncthreads();

  double dmax = 0.0;
  for (uint32_t ol = threadIdx.x; ol < slab_occ; ol += kBlock) {
    const uint32_t o = o0 + ol;
    int n[KMAX];
    {
      uint32_t q = ol;
#pragma unroll
      for (int k = 0; k < KMAX; ++k) {
        if (k < t) {
          const uint32_t q2 = fast_div(q, M.divR);
          n[k] = static_cast<int>(q - q2 * static_cast<uint32_t>(M.R));
          q = q2;
        } else {
          n[k] = nh[k];
        }
      }
    }
    int load = 0;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) load += n[k];
    const double a_rej = Al[ol];
    double a_best[JMAX];
    bool any[JMAX];
#pragma unroll
    for (int u = 0; u < JMAX; ++u) {
      a_best[u] = 0.0;
      any[u] = false;
    }
#pragma unroll
    for (int a = 0; a < KMAX; ++a) {
      if (a < M.K) {
#pragma unroll
        for (int u = 0; u < JMAX; ++u) {
          if (u < M.n_sizes && n[a] + M.size_u[u] <= M.C) {
            const uint32_t off = static_cast<uint32_t>(M.size_u[u]) * static_cast<uint32_t>(M.stride[a]);
            double A;
            if (a < t) {
              A = Al[ol + off];
            } else {
              A = 0.0;
              const uint32_t m = o + off;
#pragma unroll
              for (int jj = 0; jj < JMAX; ++jj)
                if (jj < M.J) A = fma(M.p[jj], static_cast<double>(Vin[m + jj * nocc]), A);
            }
            if (!any[u] || A > a_best[u]) a_best[u] = A;
            any[u] = true;
          }
        }
      }
    }
    const double idle = M.mu_L * static_cast<double>(M.KC - load);
#pragma unroll
    for (int e = 0; e < JMAX; ++e) {
      if (e < M.J) {
        const uint32_t gbase = o + e * nocc;
        const uint32_t lbase = ol + e * slab_occ;
        const float vse = Vl[lbase];
        double D = idle * static_cast<double>(vse);
        double rs = 0.0;
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
          if (k < M.K) {
            const uint32_t st = static_cast<uint32_t>(M.stride[k]);
            if (k < t) {
              if (n[k] > 0) D = fma(M.mu_L * n[k], static_cast<double>(Vl[lbase - st]), D);
              rs += static_cast<double>(Vl[lbase - static_cast<uint32_t>(n[k]) * st]);
            } else {
              if (n[k] > 0) D = fma(M.mu_L * n[k], static_cast<double>(Vin[gbase - st]), D);
              float v = vse;
              if (n[k] > 0) v = Vin[gbase - static_cast<uint32_t>(n[k]) * st];
              rs += static_cast<double>(v);
            }
          }
        }
        D = fma(M.nu_L, rs, D);
        const double fu = static_cast<double>(M.KC - load);   // free units (under-utilisation penalty)
        double best = fma(M.gamma, a_rej, fma(-M.hold, fu, M.r_reject[e]));
        const int u = M.size_idx[e];
        double ab = 0.0;
        bool an = false;
#pragma unroll
        for (int uu = 0; uu < JMAX; ++uu)
          if (uu == u) {
            ab = a_best[uu];
            an = any[uu];
          }
        if (an) {
          const double q = fma(M.gamma, ab, fma(-M.hold, fu, M.r_place[e]));
          if (q > best) best = q;
        }
        const float vn = static_cast<float>(fma(M.gamma, D, best));
        Vout[gbase] = vn;
        const double d = fabs(static_cast<double>(vn) - static_cast<double>(vse));
        dmax = (d > dmax || d != d) ? d : dmax;
      }
    }
  }
  block_max_to(dmax, ctl, res, j, tol);
}


// ---------------------------------------------------------------- exact-shape direct form
//
// One occupancy per thread with the branch-free backup of a compile-time
// (K, J) whose arrival terms come from the FP64 side array written by the
// previous sweep (backup_arrival): every gather of the thread is issued
// before the first use.
template <int K, int J>
__global__ __launch_bounds__(kBlock) void vi_exact_kernel(Model M, const float* __restrict__ Vin,
                                                           float* __restrict__ Vout,
                                                           const double* __restrict__ Ain,
                                                           double* __restrict__ Aout, Ctl* ctl,
                                                           double* res, long long j, double tol) {
  if (sweep_stopped<ResKind::kMax>(ctl, res, j, tol)) return;
  const uint32_t b = xcd_block(blockIdx.x, gridDim.x);
  const uint32_t o = b * kBlock + threadIdx.x;
  const BufView vin = make_view(Vin, static_cast<uint32_t>(M.n_states) * 4u);
  const BufView ain = make_view(Ain, static_cast<uint32_t>(M.n_occ + 1) * 8u);
  double dmax = 0.0;
  if (o < static_cast<uint32_t>(M.n_occ)) dmax = backup_arrival<K, J>(M, vin, ain, Vout, Aout, o);
  block_max_to(dmax, ctl, res, j, tol);
}

// A(o) = sum_e lambda_e/Lam V(o, e) of the initial iterate (the FMA chain of
// backup_arrival) into A0, and the -inf sentinel block A[n_occ .. n_occ +
// kSentinel) into both arrays.
__global__ void arrival_init_kernel(Model M, const float* __restrict__ V, double* __restrict__ A0,
                                    double* __restrict__ A1) {
  const uint64_t o = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (o >= static_cast<uint64_t>(M.n_occ) && o < static_cast<uint64_t>(M.n_occ) + kSentinel) {
    A0[o] = -INFINITY;   // read by placements without room
    A1[o] = -INFINITY;
  }
  if (o >= static_cast<uint64_t>(M.n_occ)) return;
  double* A = A0;
  double a = 0.0;
  for (int e = 0; e < M.J; ++e)
    a = fma(M.p[e], static_cast<double>(V[o + static_cast<uint64_t>(e) * M.n_occ]), a);
  A[o] = a;
}

hipError_t launch_arrival_init(const Model& M, const float* V, double* A0, double* A1, hipStream_t s) {
  const uint32_t grid = static_cast<uint32_t>((static_cast<uint64_t>(M.n_occ) + kSentinel + 255) / 256);
  hipLaunchKernelGGL(arrival_init_kernel, dim3(grid), dim3(256), 0, s, M, V, A0, A1);
  return hipGetLastError();
}

// Every byte offset of the exact-shape forms fits 31 bits: values (FP32,
// n_states) and arrival terms (FP64, n_occ + kSentinel).
bool exact_shape(const Model& M) {
  return M.n_states < (int64_t{1} << 29) && M.n_occ + kSentinel < (int64_t{1} << 28) && M.K >= 1 &&
         M.K <= 8 && M.J >= 1 && M.J <= 3 && M.n_sizes == M.J;
}

template <int K, int J>
static hipError_t launch_exact_t(const Model& M, const float* Vin, float* Vout, const double* Ain,
                                 double* Aout, Ctl* ctl, double* res, long long j, double tol,
                                 hipStream_t s) {
  const uint32_t grid = static_cast<uint32_t>((static_cast<uint64_t>(M.n_occ) + kBlock - 1) / kBlock);
  hipLaunchKernelGGL((vi_exact_kernel<K, J>), dim3(grid), dim3(kBlock), 0, s, M, Vin, Vout, Ain, Aout, ctl,
                     res, j, tol);
  return hipGetLastError();
}

static hipError_t launch_exact(const Model& M, const float* Vin, float* Vout, const double* Ain,
                               double* Aout, Ctl* ctl, double* res, long long j, double tol,
                               hipStream_t s) {
  switch (M.K * 4 + M.J) {
    case 5: return launch_exact_t<1, 1>(M, Vin, Vout, Ain, Aout, ctl, res, j, tol, s);
    case 6: return launch_exact_t<1, 2>(M, Vin, Vout, Ain, Aout, ctl, res, j, tol, s);
    case 7: return launch_exact_t<1, 3>(M, Vin, Vout, Ain, Aout, ctl, res, j, tol, s);
    case 9: return launch_exact_t<2, 1>(M, Vin, Vout, Ain, Aout, ctl, res, j, tol, s);
    case 10: return launch_exact_t<2, 2>(M, Vin, Vout, Ain, Aout, ctl, res, j, tol, s);
    case 11: return launch_exact_t<2, 3>(M, Vin, Vout, Ain, Aout, ctl, res, j, tol, s);
    case 13: return launch_exact_t<3, 1>(M, Vin, Vout, Ain, Aout, ctl, res, j, tol, s);
    case 14: return launch_exact_t<3, 2>(M, Vin, Vout, Ain, Aout, ctl, res, j, tol, s);
    case 15: return launch_exact_t<3, 3>(M, Vin, Vout, Ain, Aout, ctl, res, j, tol, s);
    case 17: return launch_exact_t<4, 1>(M, Vin, Vout, Ain, Aout, ctl, res, j, tol, s);
    case 18: return launch_exact_t<4, 2>(M, Vin, Vout, Ain, Aout, ctl, res, j, tol, s);
    case 19: return launch_exact_t<4, 3>(M, Vin, Vout, Ain, Aout, ctl, res, j, tol, s);
    case 21: return launch_exact_t<5, 1>(M, Vin, Vout, Ain, Aout, ctl, res, j, tol, s);
    case 22: return launch_exact_t<5, 2>(M, Vin, Vout, Ain, Aout, ctl, res, j, tol, s);
    case 23: return launch_exact_t<5, 3>(M, Vin, Vout, Ain, Aout, ctl, res, j, tol, s);
    case 25: return launch_exact_t<6, 1>(M, Vin, Vout, Ain, Aout, ctl, res, j, tol, s);
    case 26: return launch_exact_t<6, 2>(M, Vin, Vout, Ain, Aout, ctl, res, j, tol, s);
    case 27: return launch_exact_t<6, 3>(M, Vin, Vout, Ain, Aout, ctl, res, j, tol, s);
    case 29: return launch_exact_t<7, 1>(M, Vin, Vout, Ain, Aout, ctl, res, j, tol, s);
    case 30: return launch_exact_t<7, 2>(M, Vin, Vout, Ain, Aout, ctl, res, j, tol, s);
    case 31: return launch_exact_t<7, 3>(M, Vin, Vout, Ain, Aout, ctl, res, j, tol, s);
    case 33: return launch_exact_t<8, 1>(M, Vin, Vout, Ain, Aout, ctl, res, j, tol, s);
    case 34: return launch_exact_t<8, 2>(M, Vin, Vout, Ain, Aout, ctl, res, j, tol, s);
    case 35: return launch_exact_t<8, 3>(M, Vin, Vout, Ain, Aout, ctl, res, j, tol, s);
    default:
      return hipErrorInvalidValue;
  }
}

// Slab depth for M: the most low digits t whose slab (values of all classes
// in FP32 plus the FP64 arrival term) fits kSlabLds bytes while leaving at
// least kMinSlabs workgroups; 0 when no t >= 1 qualifies (use the direct form).
bool exact_shape(const Model& M);

uint32_t vi_sweep_grid(const Model& M, int slab_t) {
  if (slab_t > 0) {
    uint64_t occ = 1;
    for (int k = 0; k < slab_t; ++k) occ *= static_cast<uint64_t>(M.R);
    return static_cast<uint32_t>(static_cast<uint64_t>(M.n_occ) / occ);
  }
  if (exact_shape(M))
    return static_cast<uint32_t>((static_cast<uint64_t>(M.n_occ) + kBlock - 1) / kBlock);
  const uint64_t per = static_cast<uint64_t>(kBlock) * kOccPerThread;
  return static_cast<uint32_t>((static_cast<uint64_t>(M.n_occ) + per - 1) / per);
}

int slab_digits(const Model& M) {
  if (!use_32bit_index(M)) return 0;
  int best = 0;
  uint64_t occ = 1;
  for (int t = 1; t < M.K; ++t) {
    occ *= static_cast<uint64_t>(M.R);
    const uint64_t bytes = occ * (8 + 4 * static_cast<uint64_t>(M.J));
    const uint64_t slabs = static_cast<uint64_t>(M.n_occ) / occ;
    if (bytes <= kSlabLds && slabs >= kMinSlabs) best = t;
  }
  return best;
}

__global__ void ctl_init_kernel(Ctl* ctl, double* res) {
  if (threadIdx.x == 0) {
    ctl->done_iter = -1;
    ctl->flag = 0;
  }
  if (threadIdx.x < kResSlots * kNumXcd) {
    ctl->go[threadIdx.x / kNumXcd][threadIdx.x % kNumXcd][0] = 0u;
    ctl->nan[threadIdx.x / kNumXcd][threadIdx.x % kNumXcd][0] = 0u;
  }
  if (res)
    for (int w = threadIdx.x; w < kResSlots * kResLanes; w += blockDim.x)
      res[static_cast<size_t>(w) * kSumStride] = 0.0;
}

hipError_t launch_ctl_init(Ctl* ctl, double* res, hipStream_t s) {
  hipLaunchKernelGGL(ctl_init_kernel, dim3(1), dim3(256), 0, s, ctl, res);
  return hipGetLastError();
}

template <int KMAX, int JMAX, typename Idx>
static hipError_t launch_sweep_t(const Model& M, const float* Vin, float* Vout, Ctl* ctl,
                                 double* res, long long j, double tol, hipStream_t s) {
  const uint64_t per = static_cast<uint64_t>(kBlock) * kOccPerThread;
  const uint64_t grid = (static_cast<uint64_t>(M.n_occ) + per - 1) / per;
  hipLaunchKernelGGL((vi_sweep_kernel<KMAX, JMAX, Idx>), dim3(static_cast<uint32_t>(grid)),
                     dim3(kBlock), 0, s, M, Vin, Vout, ctl, res, j, tol);
  return hipGetLastError();
}

template <int KMAX, int JMAX>
static hipError_t launch_slab_t(const Model& M, int t, const float* Vin, float* Vout, Ctl* ctl,
                                double* res, long long j, double tol, hipStream_t s) {
  uint32_t slab_occ = 1;
  for (int k = 0; k < t; ++k) slab_occ *= static_cast<uint32_t>(M.R);
  const uint32_t grid = static_cast<uint32_t>(M.n_occ / slab_occ);
  const size_t lds = static_cast<size_t>(slab_occ) * (8 + 4 * M.J);
  hipLaunchKernelGGL((vi_slab_kernel<KMAX, JMAX>), dim3(grid), dim3(kBlock), lds, s, M, t, slab_occ,
                     Vin, Vout, ctl, res, j, tol);
  return hipGetLastError();
}

template <typename Idx>
static hipError_t launch_sweep_idx(const Model& M, const float* Vin, float* Vout, Ctl* ctl,
                                   double* res, long long j, double tol, hipStream_t s) {
  if (M.J <= 4) {
    if (M.K <= 4) return launch_sweep_t<4, 4, Idx>(M, Vin, Vout, ctl, res, j, tol, s);
    if (M.K <= 8) return launch_sweep_t<8, 4, Idx>(M, Vin, Vout, ctl, res, j, tol, s);
    return launch_sweep_t<16, 4, Idx>(M, Vin, Vout, ctl, res, j, tol, s);
  }
  if (M.K <= 4) return launch_sweep_t<4, 8, Idx>(M, Vin, Vout, ctl, res, j, tol, s);
  if (M.K <= 8) return launch_sweep_t<8, 8, Idx>(M, Vin, Vout, ctl, res, j, tol, s);
  return launch_sweep_t<16, 8, Idx>(M, Vin, Vout, ctl, res, j, tol, s);
}

hipError_t launch_vi_sweep(const Model& M, const float* Vin, float* Vout, Ctl* ctl, double* res,
                           long long j, double tol, hipStream_t s, int slab_t, double* const* A) {
  if (slab_t > 0) {
    if (M.J <= 4) {
      if (M.K <= 4) return launch_slab_t<4, 4>(M, slab_t, Vin, Vout, ctl, res, j, tol, s);
      if (M.K <= 8) return launch_slab_t<8, 4>(M, slab_t, Vin, Vout, ctl, res, j, tol, s);
      return launch_slab_t<16, 4>(M, slab_t, Vin, Vout, ctl, res, j, tol, s);
    }
    if (M.K <= 4) return launch_slab_t<4, 8>(M, slab_t, Vin, Vout, ctl, res, j, tol, s);
    if (M.K <= 8) return launch_slab_t<8, 8>(M, slab_t, Vin, Vout, ctl, res, j, tol, s);
    return launch_slab_t<16, 8>(M, slab_t, Vin, Vout, ctl, res, j, tol, s);
  }
  if (exact_shape(M) && A)
    return launch_exact(M, Vin, Vout, A[j & 1], A[(j + 1) & 1], ctl, res, j, tol, s);
  if (use_32bit_index(M)) return launch_sweep_idx<uint32_t>(M, Vin, Vout, ctl, res, j, tol, s);
  return launch_sweep_idx<uint64_t>(M, Vin, Vout, ctl, res, j, tol, s);
}

}  // namespace mdpvi
