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

namespace mdpvi {

template <int KMAX, int JMAX, typename Idx>
__global__ __launch_bounds__(kBlock) void vi_sweep_kernel(Model M, const float* __restrict__ Vin,
                                                           float* __restrict__ Vout, Ctl* ctl,
                                                           long long j, double tol) {
  if (sweep_stopped(ctl, j, tol)) return;
  const uint32_t b = xcd_block(blockIdx.x, gridDim.x);
  const Idx o = static_cast<Idx>(b) * kBlock + threadIdx.x;
  double dmax = 0.0;
  if (o < static_cast<Idx>(M.n_occ)) {
    const Idx nocc = static_cast<Idx>(M.n_occ);
    int n[KMAX];
    decode<KMAX>(M, o, n);
    int load = 0;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) load += n[k];

    float vs[JMAX];
#pragma unroll
    for (int e = 0; e < JMAX; ++e) vs[e] = (e < M.J) ? Vin[o + e * nocc] : 0.0f;

    // arrival term at the current occupancy (paid-cloud action)
    double a_rej = 0.0;
#pragma unroll
    for (int e = 0; e < JMAX; ++e)
      if (e < M.J) a_rej = fma(M.p[e], static_cast<double>(vs[e]), a_rej);

    // best arrival term over the hosts with room, per distinct task size
    double a_best[JMAX];
#pragma unroll
    for (int u = 0; u < JMAX; ++u) a_best[u] = -1.0;   // A >= 0 never holds for "none"
    bool any[JMAX];
#pragma unroll
    for (int u = 0; u < JMAX; ++u) any[u] = false;
#pragma unroll
    for (int a = 0; a < KMAX; ++a) {
      if (a < M.K) {
#pragma unroll
        for (int u = 0; u < JMAX; ++u) {
          if (u < M.n_sizes && n[a] + M.size_u[u] <= M.C) {
            const Idx m = o + static_cast<Idx>(M.size_u[u]) * static_cast<Idx>(M.stride[a]);
            double A = 0.0;
#pragma unroll
            for (int jj = 0; jj < JMAX; ++jj)
              if (jj < M.J) A = fma(M.p[jj], static_cast<double>(Vin[m + jj * nocc]), A);
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
        const Idx base = o + e * nocc;
        double D = idle * static_cast<double>(vs[e]);
        double rs = 0.0;
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
          if (k < M.K) {
            const Idx st = static_cast<Idx>(M.stride[k]);
            if (n[k] > 0) D = fma(M.mu_L * n[k], static_cast<double>(Vin[base - st]), D);
            rs += static_cast<double>(Vin[base - static_cast<Idx>(n[k]) * st]);
          }
        }
        D = fma(M.nu_L, rs, D);
        double best = fma(M.gamma, a_rej, M.r_reject[e]);
        const int u = M.size_idx[e];
        if (any[u]) {
          const double q = fma(M.gamma, a_best[u], M.r_place[e]);
          if (q > best) best = q;
        }
        const float vn = static_cast<float>(fma(M.gamma, D, best));
        Vout[base] = vn;
        const double d = fabs(static_cast<double>(vn) - static_cast<double>(vs[e]));
        dmax = (d > dmax || d != d) ? d : dmax;
      }
    }
  }
  block_max_to(dmax, &ctl->res[j % kResSlots]);
}

__global__ void ctl_init_kernel(Ctl* ctl) {
  if (threadIdx.x == 0) {
    ctl->done_iter = -1;
    ctl->flag = 0;
#pragma unroll
    for (int r = 0; r < kResSlots; ++r) ctl->res[r] = 0ull;
  }
}

hipError_t launch_ctl_init(Ctl* ctl, hipStream_t s) {
  hipLaunchKernelGGL(ctl_init_kernel, dim3(1), dim3(64), 0, s, ctl);
  return hipGetLastError();
}

template <int KMAX, int JMAX, typename Idx>
static hipError_t launch_sweep_t(const Model& M, const float* Vin, float* Vout, Ctl* ctl,
                                 long long j, double tol, hipStream_t s) {
  const uint64_t grid = (static_cast<uint64_t>(M.n_occ) + kBlock - 1) / kBlock;
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
