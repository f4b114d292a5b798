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
      Vout[base] = vn;
      const double d = fabs(static_cast<double>(vn) - static_cast<double>(vs[e]));
      dmax = (d > dmax || d != d) ? d : dmax;
    }
  }
  return dmax;
}

// Digits of occupancy o for a compile-time host count K.
template <int K, typename Idx>
__device__ __forceinline__ void decode_exact(const Model& M, Idx o, int (&n)[K]) {
#pragma unroll
  for (int k = 0; k < K; ++k) {
    if constexpr (sizeof(Idx) == 4) {
      const uint32_t q = fast_div(static_cast<uint32_t>(o), M.divR);
      n[k] = static_cast<int>(static_cast<uint32_t>(o) - q * static_cast<uint32_t>(M.R));
      o = static_cast<Idx>(q);
    } else {
      n[k] = static_cast<int>(o % static_cast<Idx>(M.R));
      o /= static_cast<Idx>(M.R);
    }
  }
}

// The same backup as backup_occupancy for a compile-time host count K and
// class count J whose task sizes are all distinct, written without a branch
// around any load: an infeasible placement or an absent release reads a
// valid stand-in address (the state itself) whose value is then ignored by a
// select or multiplied by a zero weight.  Every gather of the occupancy can
// therefore be in flight at once, and each one is a raw buffer load whose
// per-lane byte offset is shared by the J classes.  Same operations in the
// same order as backup_occupancy, so the iterates are bit-identical.
template <int K, int J>
__device__ __forceinline__ double backup_exact(const Model& M, BufView vin, float* __restrict__ Vout,
                                               uint32_t o) {
  const uint32_t nocc = static_cast<uint32_t>(M.n_occ);
  const uint32_t cls = nocc * 4u;  // bytes between class blocks
  int n[K];
  decode_exact<K>(M, o, n);
  int load = 0;
#pragma unroll
  for (int k = 0; k < K; ++k) load += n[k];
  const uint32_t o4 = o * 4u;

  float vs[J], va[K][J][J], vd[K][J], vr[K][J];
  bool fa[K][J];
#pragma unroll
  for (int e = 0; e < J; ++e) vs[e] = ld_f32(vin, o4, e * cls);
#pragma unroll
  for (int a = 0; a < K; ++a) {
    const uint32_t st4 = static_cast<uint32_t>(M.stride[a]) * 4u;
#pragma unroll
    for (int e = 0; e < J; ++e) {
      fa[a][e] = n[a] + M.size[e] <= M.C;
      const uint32_t m4 = fa[a][e] ? o4 + static_cast<uint32_t>(M.size[e]) * st4 : o4;
#pragma unroll
      for (int jj = 0; jj < J; ++jj) va[a][e][jj] = ld_f32(vin, m4, jj * cls);
    }
    const uint32_t d4 = n[a] > 0 ? o4 - st4 : o4;
    const uint32_t r4 = o4 - static_cast<uint32_t>(n[a]) * st4;
#pragma unroll
    for (int e = 0; e < J; ++e) {
      vd[a][e] = ld_f32(vin, d4, e * cls);
      vr[a][e] = ld_f32(vin, r4, e * cls);
    }
  }

  double a_rej = 0.0;
#pragma unroll
  for (int e = 0; e < J; ++e) a_rej = fma(M.p[e], static_cast<double>(vs[e]), a_rej);
  double a_best[J];
  bool any[J];
#pragma unroll
  for (int e = 0; e < J; ++e) {
    a_best[e] = 0.0;
    any[e] = false;
  }
#pragma unroll
  for (int a = 0; a < K; ++a) {
#pragma unroll
    for (int e = 0; e < J; ++e) {
      double A = 0.0;
#pragma unroll
      for (int jj = 0; jj < J; ++jj) A = fma(M.p[jj], static_cast<double>(va[a][e][jj]), A);
      const bool take = fa[a][e] && (!any[e] || A > a_best[e]);
      a_best[e] = take ? A : a_best[e];
      any[e] = any[e] || fa[a][e];
    }
  }
  const double idle = M.mu_L * static_cast<double>(M.KC - load);
  double dmax = 0.0;
#pragma unroll
  for (int e = 0; e < J; ++e) {
    double D = idle * static_cast<double>(vs[e]);
    double rs = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (n[k] > 0) D = fma(M.mu_L * n[k], static_cast<double>(vd[k][e]), D);
      rs += static_cast<double>(vr[k][e]);
    }
    D = fma(M.nu_L, rs, D);
    const double fu = static_cast<double>(M.KC - load);   // free units (under-utilisation penalty)
    double best = fma(M.gamma, a_rej, fma(-M.hold, fu, M.r_reject[e]));
    const double q = fma(M.gamma, a_best[e], fma(-M.hold, fu, M.r_place[e]));
    best = (any[e] && q > best) ? q : best;
    const float vn = static_cast<float>(fma(M.gamma, D, best));
    Vout[o + e * nocc] = vn;
    const double d = fabs(static_cast<double>(vn) - static_cast<double>(vs[e]));
    dmax = (d > dmax || d != d) ? d : dmax;
  }
  return dmax;
}

// Arrival-term form of backup_exact: A^j(o) = sum_j lambda_j/Lam V^j(o, j) of
// every occupancy comes from an FP64 array written by the previous sweep
// (the same FMA chain backup_exact evaluates per neighbour), so a placement
// neighbour costs one FP64 load instead of J loads, conversions and FMAs.
// The new A^{j+1}(o) is formed from the freshly rounded FP32 values and
// stored.  A placement without room reads the sentinel A[n_occ] = -inf, so
// the maximum over hosts needs no select; an absent release is an FMA with a
// zero weight.  Same values as backup_occupancy (max() equals its
// compare-and-select on non-NaN operands, and adding a zero product leaves a
// sum unchanged): bit-identical iterates.  A NaN anywhere in the state's
// classes is reported as a NaN residual.
template <int K, int J>
__device__ __forceinline__ double backup_arrival(const Model& M, BufView vin, BufView ain,
                                                 float* __restrict__ Vout, double* __restrict__ Aout,
                                                 uint32_t o) {
  const uint32_t nocc = static_cast<uint32_t>(M.n_occ);
  const uint32_t cls = nocc * 4u;
  const uint32_t none8 = nocc * 8u;   // A[n_occ] holds -inf: the stand-in of a placement without room
  int n[K];
  decode_exact<K>(M, o, n);
  int load = 0;
#pragma unroll
  for (int k = 0; k < K; ++k) load += n[k];
  const uint32_t o4 = o * 4u, o8 = o * 8u;

  float vs[J], vd[K][J], vr[K][J];
  double aa[K][J];
#pragma unroll
  for (int e = 0; e < J; ++e) vs[e] = ld_f32(vin, o4, e * cls);
  const double a_rej = ld_f64(ain, o8, 0);
#pragma unroll
  for (int a = 0; a < K; ++a) {
    const uint32_t st = static_cast<uint32_t>(M.stride[a]);
#pragma unroll
    for (int e = 0; e < J; ++e) {
      const bool room = n[a] + M.size[e] <= M.C;
      aa[a][e] = ld_f64(ain, room ? o8 + static_cast<uint32_t>(M.size[e]) * st * 8u : none8, 0);
    }
    const uint32_t d4 = n[a] > 0 ? o4 - st * 4u : o4;
    const uint32_t r4 = o4 - static_cast<uint32_t>(n[a]) * st * 4u;
#pragma unroll
    for (int e = 0; e < J; ++e) {
      vd[a][e] = ld_f32(vin, d4, e * cls);
      vr[a][e] = ld_f32(vin, r4, e * cls);
    }
  }
  const double idle = M.mu_L * static_cast<double>(M.KC - load);
  double dmax = 0.0, anew = 0.0;
  bool bad = false;
#pragma unroll
  for (int e = 0; e < J; ++e) {
    double ab = aa[0][e];
#pragma unroll
    for (int a = 1; a < K; ++a) ab = fmax(ab, aa[a][e]);
    double D = idle * static_cast<double>(vs[e]);
    double rs = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      // a host with n_k = 0 has weight 0 (its stand-in read is the state itself)
      D = fma(M.mu_L * n[k], static_cast<double>(vd[k][e]), D);
      rs += static_cast<double>(vr[k][e]);
    }
    D = fma(M.nu_L, rs, D);
    const double fu = static_cast<double>(M.KC - load);   // free units (under-utilisation penalty)
    const double best = fmax(fma(M.gamma, a_rej, fma(-M.hold, fu, M.r_reject[e])), fma(M.gamma, ab, fma(-M.hold, fu, M.r_place[e])));
    const float vn = static_cast<float>(fma(M.gamma, D, best));
    Vout[o + e * nocc] = vn;
    anew = fma(M.p[e], static_cast<double>(vn), anew);
    const double d = fabs(static_cast<double>(vn) - static_cast<double>(vs[e]));
    dmax = fmax(dmax, d);
    bad = bad || (d != d);
  }
  Aout[o] = anew;
  return bad ? NAN : dmax;
}

}  // namespace mdpvi
