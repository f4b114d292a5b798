// policy_impl.hpp -- per-occupancy device functions of extraction, fixed-policy
// evaluation, the greedy heuristic and the policy check, shared by the
// single-instance kernels and the batched forms.
#pragma once

#include "device.hpp"

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

// Greedy extraction at occupancy o (all classes): lowest-index argmax of Q
// formed in FP64 from V, and the best-minus-second gap.
template <int KMAX, int JMAX, typename T, typename Idx>
__device__ __forceinline__ void extract_occupancy(const Model& M, const T* __restrict__ V,
                                                  uint8_t* __restrict__ pi, float* __restrict__ gap,
                                                  Idx o) {
  const Idx nocc = static_cast<Idx>(M.n_occ);
  int n[KMAX];
  decode<KMAX>(M, o, n);
  int load = 0;
#pragma unroll
  for (int k = 0; k < KMAX; ++k) load += n[k];
  const double a_rej = arrival<JMAX>(M, V, o, nocc);
  const double fu = static_cast<double>(M.KC - load);   // free units (under-utilisation penalty)
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
            q = fma(M.gamma, arrival<JMAX>(M, V, m, nocc) + D, fma(-M.hold, fu, M.r_place[e]));
          } else {
            q = fma(M.gamma, a_rej + D, fma(-M.hold, fu, M.r_reject[e]));
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

// Policy improvement at occupancy o (all classes), Q formed in FP64 from V
// as in extract_occupancy: the current action pi_in stays unless some action
// beats its Q by more than tol; then the lowest-index argmax.  Returns true
// when some class's action changed.  pi_in may equal pi_out (each state
// reads and writes only its own entry).
template <int KMAX, int JMAX, typename Idx>
__device__ __forceinline__ bool improve_occupancy(const Model& M, const double* __restrict__ V,
                                                  const uint8_t* pi_in, uint8_t* pi_out, double tol, Idx o) {
  bool changed = false;
  const Idx nocc = static_cast<Idx>(M.n_occ);
  int n[KMAX];
  decode<KMAX>(M, o, n);
  int load = 0;
#pragma unroll
  for (int k = 0; k < KMAX; ++k) load += n[k];
  const double a_rej = arrival<JMAX>(M, V, o, nocc);
  const double fu = static_cast<double>(M.KC - load);   // free units (under-utilisation penalty)
#pragma unroll
  for (int e = 0; e < JMAX; ++e) {
    if (e < M.J) {
      const Idx base = o + e * nocc;
      const double D = no_arrival<KMAX>(M, V, base, n, load);
      const int se = M.size[e];
      const int cur = pi_in[base];
      double best = 0.0, q_cur = 0.0;
      int arg = -1;
#pragma unroll
      for (int a = 0; a <= KMAX; ++a) {
        if (a <= M.K) {
          double q;
          if (a < M.K) {
            if (n[a] + se > M.C) continue;
            const Idx m = o + static_cast<Idx>(se) * static_cast<Idx>(M.stride[a]);
            q = fma(M.gamma, arrival<JMAX>(M, V, m, nocc) + D, fma(-M.hold, fu, M.r_place[e]));
          } else {
            q = fma(M.gamma, a_rej + D, fma(-M.hold, fu, M.r_reject[e]));
          }
          if (a == cur) q_cur = q;
          if (arg < 0 || q > best) {
            best = q;
            arg = a;
          }
        }
      }
      const int chosen = q_cur >= best - tol ? cur : arg;
      changed |= chosen != cur;
      pi_out[base] = static_cast<uint8_t>(chosen);
    }
  }
  return changed;
}

// True if some class at occupancy o has an action that is not feasible.
template <int KMAX, int JMAX, typename Idx>
__device__ __forceinline__ bool check_occupancy(const Model& M, const uint8_t* __restrict__ pi, Idx o) {
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
  return bad;
}

// Fixed-policy backup V'(s) = r_pi(s) + gamma (A(m_pi) + D(s)) in FP64 for the
// classes of occupancy o; returns the largest |V' - V|.
template <int KMAX, int JMAX, typename Idx>
__device__ __forceinline__ double eval_occupancy(const Model& M, const uint8_t* __restrict__ pi,
                                                 const double* __restrict__ Vin,
                                                 double* __restrict__ Vout, Idx o) {
  const Idx nocc = static_cast<Idx>(M.n_occ);
  int n[KMAX];
  decode<KMAX>(M, o, n);
  int load = 0;
#pragma unroll
  for (int k = 0; k < KMAX; ++k) load += n[k];
  double dmax = 0.0;
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
      const double vn = fma(M.gamma, D, fma(M.gamma, A, fma(-M.hold, static_cast<double>(M.KC - load), r)));
      const double old = Vin[base];
      Vout[base] = vn;
      const double d = fabs(vn - old);
      dmax = (d > dmax || d != d) ? d : dmax;
    }
  }
  return dmax;
}

// Greedy heuristic at occupancy o: kind 0 least-loaded, 1 first-fit.
template <int KMAX, int JMAX, typename Idx>
__device__ __forceinline__ void greedy_occupancy(const Model& M, int kind, uint8_t* __restrict__ pi, Idx o) {
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

// Fixed-policy backup for a compile-time (K, J), without a branch around any
// load (stand-in addresses with zero weights, raw buffer loads, as
// backup_exact).  Same operations in the same order as eval_occupancy:
// bit-identical results.
template <int K, int J>
__device__ __forceinline__ double eval_exact(const Model& M, BufView pv, BufView vin,
                                             double* __restrict__ Vout, uint32_t o) {
  const uint32_t nocc = static_cast<uint32_t>(M.n_occ);
  int n[K];
  {
    uint32_t q = o;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const uint32_t q2 = fast_div(q, M.divR);
      n[k] = static_cast<int>(q - q2 * static_cast<uint32_t>(M.R));
      q = q2;
    }
  }
  int load = 0;
#pragma unroll
  for (int k = 0; k < K; ++k) load += n[k];
  const uint32_t o8 = o * 8u;
  const uint32_t cls8 = nocc * 8u;
  int a[J];
  double vs[J], va[J][J], vd[K][J], vr[K][J];
#pragma unroll
  for (int e = 0; e < J; ++e) {
    a[e] = ld_u8(pv, o, e * nocc);
    vs[e] = ld_f64(vin, o8, e * cls8);
  }
#pragma unroll
  for (int e = 0; e < J; ++e) {
    uint32_t st8 = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) st8 = (k == a[e]) ? static_cast<uint32_t>(M.stride[k]) * 8u : st8;
    const uint32_t m8 = o8 + static_cast<uint32_t>(M.size[e]) * st8;   // st8 = 0 for the paid cloud
#pragma unroll
    for (int jj = 0; jj < J; ++jj) va[e][jj] = ld_f64(vin, m8, jj * cls8);
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const uint32_t st8 = static_cast<uint32_t>(M.stride[k]) * 8u;
    const uint32_t d8 = n[k] > 0 ? o8 - st8 : o8;
    const uint32_t r8 = o8 - static_cast<uint32_t>(n[k]) * st8;
#pragma unroll
    for (int e = 0; e < J; ++e) {
      vd[k][e] = ld_f64(vin, d8, e * cls8);
      vr[k][e] = ld_f64(vin, r8, e * cls8);
    }
  }
  double dmax = 0.0;
#pragma unroll
  for (int e = 0; e < J; ++e) {
    const double r = fma(-M.hold, static_cast<double>(M.KC - load), a[e] < M.K ? M.r_place[e] : M.r_reject[e]);
    double D = M.mu_L * static_cast<double>(M.KC - load) * vs[e];
    double rs = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (n[k] > 0) D = fma(M.mu_L * n[k], vd[k][e], D);
      rs += vr[k][e];
    }
    D = fma(M.nu_L, rs, D);
    double A = 0.0;
#pragma unroll
    for (int jj = 0; jj < J; ++jj) A = fma(M.p[jj], va[e][jj], A);
    const double vn = fma(M.gamma, D, fma(M.gamma, A, r));
    Vout[o + e * nocc] = vn;
    const double d = fabs(vn - vs[e]);
    dmax = (d > dmax || d != d) ? d : dmax;
  }
  return dmax;
}

}  // namespace mdpvi
