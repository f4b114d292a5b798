// adjoint.hip -- gradient of the expected discounted reward from the empty
// system with respect to the model rates and rewards.
//
// Objective: J = sum_e c_e V_pi(0, e), c_e = lambda_e / sum_j lambda_j, with pi
// the optimal policy of Eq. (18) held fixed.  With w the solution of
//   (I - gamma P_pi)^T w = c          (c supported on the empty states),
// the derivative of J with respect to theta = (lambda_1..lambda_J, mu, nu,
// r_1..r_J) is
//   dJ/dtheta = sum_s w(s) (d r_pi(s) + gamma d(P_pi V_pi)(s)) + sum_e d c_e V_pi(0, e).
//
// Transposed sweep: w' = c + gamma P_pi^T w, one thread per occupancy n', all
// classes e'.  The predecessors of (n', e') are
//   arrivals   (n, e) whose post-decision occupancy m(n, e, pi) equals n', with
//              probability lambda_e'/Lam: the inflow B(n') = sum of those w,
//              shared by every e' (the paid cloud at n', or a placement of a
//              class-e task on host k from n' - size_e 1_k);
//   releases   (n' + 1_k, e') with probability mu (n'_k + 1)/Lam;
//   resets     when n'_k = 0, every (n' with digit k = x, e'), x = 0..C, with
//              probability nu/Lam each (a line sum along digit k);
//   idle       (n', e') itself with probability mu (KC - |n'|)/Lam.
// All weights are non-negative: w is FP32, sums are FP64, one rounding per
// state, and the residual is the 1-norm ||w' - w||_1 (the norm in which
// P_pi^T is a contraction).
#include "adjoint_impl.hpp"
#include "device.hpp"
#include "kernels.hpp"
#include "tile.hpp"

#include <type_traits>

namespace mdpvi {

// OPT occupancies per thread: 1 below kAdjointWideOcc occupancies, so that a
// small instance still spreads over every CU; kOccPerThread above.
template <int KMAX, int JMAX, typename Idx, int OPT, bool EXACT>
__global__ __launch_bounds__(kBlock) void adjoint_sweep_kernel(Model M, const uint8_t* __restrict__ pi,
                                                                const float* __restrict__ win,
                                                                float* __restrict__ wout, Ctl* ctl,
                                                                double* res, long long j, double tol) {
  if (sweep_stopped<ResKind::kSum>(ctl, res, j, tol)) return;
  const uint32_t b = xcd_block(blockIdx.x, gridDim.x);
  const Idx base = static_cast<Idx>(b) * (kBlock * OPT) + threadIdx.x;
  double dsum = 0.0;
#pragma unroll
  for (int i = 0; i < OPT; ++i) {
    const Idx o = base + static_cast<Idx>(i * kBlock);
    if (o < static_cast<Idx>(M.n_occ)) {
      if constexpr (EXACT)
        dsum += adjoint_occupancy_exact<KMAX, JMAX>(M, pi, win, wout, static_cast<uint32_t>(o));
      else
        dsum += adjoint_occupancy<KMAX, JMAX, Idx>(M, pi, win, wout, o);
    }
  }
  block_sum_to(dsum, res, j);
}

// Number of gradient entries: lambda_1..J, mu, nu, r_1..J.
__host__ __device__ inline int n_theta(const Model& M) { return 2 * M.J + 2; }

// Per-workgroup partial sums of sum_s w(s) (d r_pi(s) + gamma d(P_pi V)(s)),
// with P_pi V = V_s + G/Lam written in differences from V_s:
//   G = sum_j lambda_j (V(m,j) - V_s) + mu sum_k n_k (V(n-1_k,e) - V_s)
//       + nu sum_k (V(n^{k<-0},e) - V_s),
//   d/dlambda_j = (V(m,j) - V_s)/Lam - G/Lam^2,
//   d/dmu       = sum_k n_k (V(n-1_k,e) - V_s)/Lam - KC G/Lam^2,
//   d/dnu       = sum_k (V(n^{k<-0},e) - V_s)/Lam - K G/Lam^2,
// and r_pi = (sum lambda / Lam) R(e, a): d/dlambda_j = R (Lam - sum lambda)/Lam^2,
// d/dmu = -sum lambda R KC / Lam^2, d/dnu = -sum lambda R K / Lam^2,
// d/dr_j = sum lambda / Lam when e = j and a places the task.
template <int KMAX, int JMAX, typename Idx>
__global__ __launch_bounds__(kBlock) void grad_partial_kernel(Model M, const uint8_t* __restrict__ pi,
                                                               const double* __restrict__ V,
                                                               const float* __restrict__ w,
                                                               double* __restrict__ partial) {
  constexpr int TMAX = 2 * JMAX + 2;
  double g[TMAX];
#pragma unroll
  for (int t = 0; t < TMAX; ++t) g[t] = 0.0;
  const Idx base0 = static_cast<Idx>(blockIdx.x) * (kBlock * kOccPerThread) + threadIdx.x;
  for (int i = 0; i < kOccPerThread; ++i) {
    const Idx o = base0 + static_cast<Idx>(i * kBlock);
    if (o >= static_cast<Idx>(M.n_occ)) break;
    grad_occupancy<KMAX, JMAX>(M, pi, V, w, o, g);
  }
  // workgroup reduction in a fixed order: wavefront shuffles, then the
  // wavefront partials summed by thread t for entry t
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

// Sums the workgroup partials in block order, adds the objective-weight terms
// d c_e / d lambda_j V(0, e) = (delta_ej sum lambda - lambda_e)/(sum lambda)^2
// V(0, e), and writes out[0..2J+1] = dJ/dtheta (lambda_1..J, mu, nu, r_1..J)
// and out[2J+2] = J.
template <int JMAX>
__global__ void grad_final_kernel(Model M, const double* __restrict__ partial, int nblocks,
                                  const double* __restrict__ V, double* __restrict__ out) {
  constexpr int TMAX = 2 * JMAX + 2;
  const int t = threadIdx.x;
  const size_t nocc = static_cast<size_t>(M.n_occ);
  if (t < TMAX) {
    double v = 0.0;
    for (int b = 0; b < nblocks; ++b) v += partial[static_cast<size_t>(b) * TMAX + t];
    // map the compiled layout (lambda at 0..JMAX-1, mu at JMAX, nu at JMAX+1,
    // r at JMAX+2..) onto the packed output
    int dst = -1;
    if (t < JMAX) {
      if (t < M.J) {
        dst = t;
        const double lt = M.lam_tot;
        for (int e = 0; e < M.J; ++e)
          v += ((e == t ? lt : 0.0) - M.lam[e]) / (lt * lt) * V[static_cast<size_t>(e) * nocc];
      }
    } else if (t == JMAX) {
      dst = M.J;
    } else if (t == JMAX + 1) {
      dst = M.J + 1;
    } else if (t - JMAX - 2 < M.J) {
      dst = M.J + 2 + (t - JMAX - 2);
    }
    if (dst >= 0) out[dst] = v;
  }
  if (t == 0) {
    double Jv = 0.0;
    for (int e = 0; e < M.J; ++e) Jv = fma(M.c_obj[e], V[static_cast<size_t>(e) * nocc], Jv);
    out[2 * M.J + 2] = Jv;
  }
}

// ---------------------------------------------------------------- launchers

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

static inline uint32_t sweep_blocks(const Model& M) {
  const uint64_t per = static_cast<uint64_t>(kBlock) * kOccPerThread;
  return static_cast<uint32_t>((static_cast<uint64_t>(M.n_occ) + per - 1) / per);
}

// Below this many occupancies the adjoint sweep takes one occupancy per
// thread (at 161,051 occupancies four per thread leave 158 workgroups for
// 256 CUs).
constexpr int64_t kAdjointWideOcc = int64_t{2} << 20;

static inline uint32_t adjoint_blocks(const Model& M, int opt) {
  const uint64_t per = static_cast<uint64_t>(kBlock) * static_cast<uint64_t>(opt);
  return static_cast<uint32_t>((static_cast<uint64_t>(M.n_occ) + per - 1) / per);
}

size_t grad_partial_doubles(const Model& M) {
  return static_cast<size_t>(sweep_blocks(M)) * (2 * (M.J <= 4 ? 4 : 8) + 2);
}

// Adjoint sweep forms: kAdjointGroup (adjoint_group.hip), kAdjointExact +
// OPT (exact-shape kernels, K in 3..8, J <= 3, OPT occupancies per thread)
// or OPT alone (the generic kernels); 0 picks the group form where it
// applies, else the exact form, with one occupancy per thread below
// kAdjointWideOcc occupancies and kOccPerThread above.
bool adjoint_exact_shape(const Model& M) {
  return M.K >= 3 && M.K <= 8 && M.J >= 1 && M.J <= 3 && use_32bit_index(M);
}

int adjoint_auto_form(const Model& M) {
  if (adjoint_group_shape(M)) return kAdjointGroup;
  const int opt = M.n_occ < kAdjointWideOcc ? 1 : kOccPerThread;
  return adjoint_exact_shape(M) ? kAdjointExact + opt : opt;
}

bool adjoint_form_valid(const Model& M, int form) {
  if (form == kAdjointGroup) return adjoint_group_shape(M);
  const int opt = form & (kAdjointExact - 1);
  if (opt != 1 && opt != 2 && opt != 4) return false;
  return (form & kAdjointExact) ? adjoint_exact_shape(M) : (form == opt);
}

template <int OPT>
static hipError_t launch_adjoint_opt(const Model& M, bool exact, const uint8_t* pi, const float* win,
                                     float* wout, Ctl* ctl, double* res, long long j, double tol, hipStream_t s) {
  const dim3 grid(adjoint_blocks(M, OPT));
  if (exact) {
    return tile_dispatch(M.K, M.J, 2, [&](auto kc, auto jc, auto) {
      constexpr int Kc = decltype(kc)::value, Jc = decltype(jc)::value;
      hipLaunchKernelGGL((adjoint_sweep_kernel<Kc, Jc, uint32_t, OPT, true>), grid, dim3(kBlock), 0, s, M, pi, win,
                         wout, ctl, res, j, tol);
      return hipGetLastError();
    });
  }
  return dispatch_kj(M, [&](auto km, auto jm) {
    constexpr int KM = decltype(km)::value, JM = decltype(jm)::value;
    if (use_32bit_index(M))
      hipLaunchKernelGGL((adjoint_sweep_kernel<KM, JM, uint32_t, OPT, false>), grid, dim3(kBlock), 0, s, M, pi,
                         win, wout, ctl, res, j, tol);
    else
      hipLaunchKernelGGL((adjoint_sweep_kernel<KM, JM, uint64_t, OPT, false>), grid, dim3(kBlock), 0, s, M, pi,
                         win, wout, ctl, res, j, tol);
    return hipGetLastError();
  });
}

hipError_t launch_adjoint_sweep(const Model& M, int form, const uint8_t* pi, const float* win, float* wout,
                                Ctl* ctl, double* res, long long j, double tol, hipStream_t s) {
  if (form == 0) form = adjoint_auto_form(M);
  if (!adjoint_form_valid(M, form)) return hipErrorInvalidValue;
  if (form == kAdjointGroup) return launch_adjoint_group(M, pi, win, wout, ctl, res, j, tol, s);
  const bool exact = (form & kAdjointExact) != 0;
  switch (form & (kAdjointExact - 1)) {
    case 1: return launch_adjoint_opt<1>(M, exact, pi, win, wout, ctl, res, j, tol, s);
    case 2: return launch_adjoint_opt<2>(M, exact, pi, win, wout, ctl, res, j, tol, s);
    default: return launch_adjoint_opt<4>(M, exact, pi, win, wout, ctl, res, j, tol, s);
  }
}

hipError_t launch_grad(const Model& M, const uint8_t* pi, const double* V, const float* w,
                       double* partial, double* out, hipStream_t s) {
  return dispatch_kj(M, [&](auto km, auto jm) {
    constexpr int KM = decltype(km)::value, JM = decltype(jm)::value;
    const uint32_t nb = sweep_blocks(M);
    if (use_32bit_index(M)) {
      hipLaunchKernelGGL((grad_partial_kernel<KM, JM, uint32_t>), dim3(nb), dim3(kBlock), 0, s, M, pi,
                         V, w, partial);
    } else {
      hipLaunchKernelGGL((grad_partial_kernel<KM, JM, uint64_t>), dim3(nb), dim3(kBlock), 0, s, M, pi,
                         V, w, partial);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((grad_final_kernel<JM>), dim3(1), dim3(64), 0, s, M, partial,
                       static_cast<int>(nb), V, out);
    return hipGetLastError();
  });
}

// J = sum_e c_e V(0, e) alone.
__global__ void objective_kernel(Model M, const double* __restrict__ V, double* __restrict__ out) {
  if (threadIdx.x == 0) {
    double Jv = 0.0;
    for (int e = 0; e < M.J; ++e)
      Jv = fma(M.c_obj[e], V[static_cast<size_t>(e) * static_cast<size_t>(M.n_occ)], Jv);
    out[0] = Jv;
  }
}

hipError_t launch_objective(const Model& M, const double* V, double* out, hipStream_t s) {
  hipLaunchKernelGGL(objective_kernel, dim3(1), dim3(64), 0, s, M, V, out);
  return hipGetLastError();
}

}  // namespace mdpvi
