// sweep_impl.hpp -- the Bellman backup of one occupancy vector (all classes),
// shared by the single-instance sweep and the batched forms.  The value
// arrays may live in global memory or in LDS.
#pragma once

#include "device.hpp"

namespace mdpvi {

// Bellman backup of every class of occupancy o (V^j -> V^{j+1}); returns the
// largest |V^{j+1} - V^j| over those states.
template <int KMAX, int JMAX, typename Idx>
__device__ __forceinline__ double backup_occupancy(const Model& M, const float* __restrict__ Vin,
                                                   float* __restrict__ Vout, Idx o) {
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
  double dmax = 0.0;
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
      double ab = 0.0;
      bool an = false;
#pragma unroll
      for (int uu = 0; uu < JMAX; ++uu)
        if (uu == u) {
          ab = a_best[uu];
          an = any[uu];
        }
      if (an) {
        const double q = fma(M.gamma, ab, M.r_place[e]);
        if (q > best) best = q;
      }
      const float vn = static_cast<float>(fma(M.gamma, D, best));
      Vout[base] = vn;
      const double d = fabs(static_cast<double>(vn) - static_cast<double>(vs[e]));
      dmax = (d > dmax || d != d) ? d : dmax;
    }
  }
  return dmax;
}

}  // namespace mdpvi
