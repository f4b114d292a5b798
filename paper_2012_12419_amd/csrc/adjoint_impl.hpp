// adjoint_impl.hpp -- per-occupancy device functions of the transposed
// (adjoint) sweep and of the gradient accumulation, shared by the
// single-instance kernels and the batched forms.
#pragma once

#include "device.hpp"

namespace mdpvi {

// Transposed backup of every class of occupancy o (the sweep's arithmetic,
// in this order, for every form).  EXACT: KMAX = K and JMAX = J, so the
// host and class loops need no run-time bounds.
template <int KMAX, int JMAX, typename Idx, bool EXACT = false>
__device__ __forceinline__ double adjoint_occupancy(const Model& M, const uint8_t* __restrict__ pi,
                                                    const float* __restrict__ win,
                                                    float* __restrict__ wout, Idx o) {
  const Idx nocc = static_cast<Idx>(M.n_occ);
  int n[KMAX];
  decode<KMAX>(M, o, n);
  int load = 0;
#pragma unroll
  for (int k = 0; k < KMAX; ++k) load += n[k];

  // arrival inflow into occupancy n'
  double B = 0.0;
#pragma unroll
  for (int e = 0; e < JMAX; ++e) {
    if (EXACT || e < M.J) {
      const Idx s = o + e * nocc;
      if (pi[s] == M.K) B += static_cast<double>(win[s]);
    }
  }
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    if (EXACT || k < M.K) {
      const Idx st = static_cast<Idx>(M.stride[k]);
#pragma unroll
      for (int e = 0; e < JMAX; ++e) {
        if ((EXACT || e < M.J) && n[k] >= M.size[e]) {
          const Idx src = o - static_cast<Idx>(M.size[e]) * st + e * nocc;
          if (pi[src] == k) B += static_cast<double>(win[src]);
        }
      }
    }
  }

  const double idle = M.mu_L * static_cast<double>(M.KC - load);
  double dsum = 0.0;
#pragma unroll
  for (int e = 0; e < JMAX; ++e) {
    if (EXACT || e < M.J) {
      const Idx base = o + e * nocc;
      const float wold = win[base];
      double acc = fma(M.p[e], B, idle * static_cast<double>(wold));
      double rs = 0.0;
#pragma unroll
      for (int k = 0; k < KMAX; ++k) {
        if (EXACT || k < M.K) {
          const Idx st = static_cast<Idx>(M.stride[k]);
          if (n[k] < M.C) acc = fma(M.mu_L * (n[k] + 1), static_cast<double>(win[base + st]), acc);
          if (n[k] == 0) {
            double line = 0.0;
            for (int x = 0; x <= M.C; ++x) line += static_cast<double>(win[base + static_cast<Idx>(x) * st]);
            rs += line;
          }
        }
      }
      acc = fma(M.nu_L, rs, acc);
      const double c = (o == 0) ? M.c_obj[e] : 0.0;
      const float wn = static_cast<float>(fma(M.gamma, acc, c));
      wout[base] = wn;
      dsum += fabs(static_cast<double>(wn) - static_cast<double>(wold));
    }
  }
  return dsum;
}

// The same transposed backup for an exact shape (K hosts, J classes known
// at compile time), with every load issued before the first use: the
// predecessors' actions and weights are loaded unconditionally (a missing
// predecessor reads the state itself) and selected afterwards, so a thread
// waits for one round trip instead of one per predecessor.  Adding the
// weight of a predecessor that does not apply is adding +0.0 to a sum of
// non-negative terms and a release from a full host multiplies by 0.0: the
// sums are those of adjoint_occupancy, term by term and in the same order.
//
// ls (LINES = true): the reset lines' sums are taken from a table instead of
// being summed here.  ls[(k J + e) nl + i], nl = n_occ / (C+1), holds the sum
// of class e's weights along the line i of digit k, summed from zero in the
// order x = 0..C (the order used here).  Line i of digit k has the
// occupancies whose other digits give i as a number with digit k removed:
// i = sum_{h<k} n_h (C+1)^h + sum_{h>k} n_h (C+1)^(h-1).
constexpr int kLineLoads = 16;

template <int K, int J, bool LINES = false>
__device__ __forceinline__ double adjoint_occupancy_exact(const Model& M, const uint8_t* __restrict__ pi,
                                                          const float* __restrict__ win,
                                                          float* __restrict__ wout, uint32_t o,
                                                          const double* __restrict__ ls = nullptr) {
  const uint32_t nocc = static_cast<uint32_t>(M.n_occ);
  int n[K];
  decode<K>(M, o, n);
  int load = 0;
#pragma unroll
  for (int k = 0; k < K; ++k) load += n[k];
  uint32_t st[K];
#pragma unroll
  for (int k = 0; k < K; ++k) st[k] = static_cast<uint32_t>(M.stride[k]);
  // arrival predecessors: (n', e) itself and (n' - size_e 1_k, e)
  int p_own[J], p_k[K][J];
  float w_own[J], w_k[K][J], w_rel[K][J];
  bool has[K][J];
#pragma unroll
  for (int e = 0; e < J; ++e) {
    const uint32_t s0 = o + e * nocc;
    p_own[e] = pi[s0];
    w_own[e] = win[s0];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      has[k][e] = n[k] >= M.size[e];
      const uint32_t src = has[k][e] ? s0 - static_cast<uint32_t>(M.size[e]) * st[k] : s0;
      p_k[k][e] = pi[src];
      w_k[k][e] = win[src];
      w_rel[k][e] = win[n[k] < M.C ? s0 + st[k] : s0];
    }
  }
  // the line sums of the digits with n_k = 0 (a load under a branch that
  // waits nowhere: the sums are used after every load is issued)
  double lsum[K][J];
  if constexpr (LINES) {
    const uint32_t nl = fast_div(nocc, M.divR);
    uint32_t idx[K];
    uint32_t below = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      idx[k] = below;
      below += static_cast<uint32_t>(n[k]) * st[k];
    }
    uint32_t above = 0;
#pragma unroll
    for (int k = K - 1; k >= 0; --k) {
      idx[k] += above;
      if (k > 0) above += static_cast<uint32_t>(n[k]) * st[k - 1];
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
#pragma unroll
      for (int e = 0; e < J; ++e) {
        lsum[k][e] = 0.0;
        if (n[k] == 0) lsum[k][e] = ls[static_cast<uint32_t>(k * J + e) * nl + idx[k]];
      }
    }
  }
  double B = 0.0;
#pragma unroll
  for (int e = 0; e < J; ++e) B += p_own[e] == M.K ? static_cast<double>(w_own[e]) : 0.0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
#pragma unroll
    for (int e = 0; e < J; ++e) B += (has[k][e] && p_k[k][e] == k) ? static_cast<double>(w_k[k][e]) : 0.0;
  }
  const double idle = M.mu_L * static_cast<double>(M.KC - load);
  double dsum = 0.0;
#pragma unroll
  for (int e = 0; e < J; ++e) {
    const uint32_t base = o + e * nocc;
    const float wold = w_own[e];
    double acc = fma(M.p[e], B, idle * static_cast<double>(wold));
    double rs = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      acc = fma(n[k] < M.C ? M.mu_L * (n[k] + 1) : 0.0, static_cast<double>(w_rel[k][e]), acc);
      if (n[k] == 0) {
        // the line sum along digit k, in order x = 0..C; lines of up to
        // kLineLoads values are loaded all at once
        if constexpr (LINES) {
          rs += lsum[k][e];
        } else if (M.C < kLineLoads) {
          float v[kLineLoads];
#pragma unroll
          for (int x = 0; x < kLineLoads; ++x) v[x] = win[base + (x <= M.C ? static_cast<uint32_t>(x) * st[k] : 0u)];
          double line = 0.0;
#pragma unroll
          for (int x = 0; x < kLineLoads; ++x)
            if (x <= M.C) line += static_cast<double>(v[x]);
          rs += line;
        } else {
          double line = 0.0;
          for (int x = 0; x <= M.C; ++x) line += static_cast<double>(win[base + static_cast<uint32_t>(x) * st[k]]);
          rs += line;
        }
      }
    }
    acc = fma(M.nu_L, rs, acc);
    const double c = (o == 0) ? M.c_obj[e] : 0.0;
    const float wn = static_cast<float>(fma(M.gamma, acc, c));
    wout[base] = wn;
    dsum += fabs(static_cast<double>(wn) - static_cast<double>(wold));
  }
  return dsum;
}

// Adds the gradient terms of the classes of occupancy o to g[] (layout:
// lambda at 0..JMAX-1, mu at JMAX, nu at JMAX+1, r at JMAX+2..).
template <int KMAX, int JMAX, typename Idx>
__device__ __forceinline__ void grad_occupancy(const Model& M, const uint8_t* __restrict__ pi,
                                               const double* __restrict__ V,
                                               const float* __restrict__ w, Idx o,
                                               double (&g)[2 * JMAX + 2]) {
  const Idx nocc = static_cast<Idx>(M.n_occ);
  const double Lam = M.Lam, L2 = M.Lam * M.Lam, lt = M.lam_tot;
  int n[KMAX];
  decode<KMAX>(M, o, n);
#pragma unroll
  for (int e = 0; e < JMAX; ++e) {
    if (e < M.J) {
      const Idx s = o + e * nocc;
      const double ws = static_cast<double>(w[s]);
      const int a = pi[s];
      Idx m = o;
      double R = -M.cost[e];
      if (a < M.K) {
        Idx st = 0;
#pragma unroll
        for (int k = 0; k < KMAX; ++k)
          if (k == a) st = static_cast<Idx>(M.stride[k]);
        m = o + static_cast<Idx>(M.size[e]) * st;
        R = M.reward[e];
      }
      const double Vs = V[s];
      double darr[JMAX];
      double G = 0.0;
#pragma unroll
      for (int jj = 0; jj < JMAX; ++jj) {
        darr[jj] = 0.0;
        if (jj < M.J) {
          darr[jj] = V[m + jj * nocc] - Vs;
          G = fma(M.lam[jj], darr[jj], G);
        }
      }
      double sdep = 0.0, sres = 0.0;
#pragma unroll
      for (int k = 0; k < KMAX; ++k) {
        if (k < M.K) {
          const Idx st = static_cast<Idx>(M.stride[k]);
          if (n[k] > 0) sdep = fma(static_cast<double>(n[k]), V[s - st] - Vs, sdep);
          sres += V[s - static_cast<Idx>(n[k]) * st] - Vs;
        }
      }
      G = fma(M.mu, sdep, fma(M.nu, sres, G));
      const double gw = M.gamma * ws;
#pragma unroll
      for (int jj = 0; jj < JMAX; ++jj) {
        if (jj < M.J) {
          const double dP = darr[jj] / Lam - G / L2;
          const double dr = R * (Lam - lt) / L2;
          g[jj] = fma(ws, dr, fma(gw, dP, g[jj]));
        }
      }
      const double KC = static_cast<double>(M.KC), K = static_cast<double>(M.K);
      g[JMAX] = fma(ws, -lt * R * KC / L2, fma(gw, sdep / Lam - KC * G / L2, g[JMAX]));
      g[JMAX + 1] = fma(ws, -lt * R * K / L2, fma(gw, sres / Lam - K * G / L2, g[JMAX + 1]));
      if (a < M.K) {
#pragma unroll
        for (int jj = 0; jj < JMAX; ++jj)
          if (jj == e) g[JMAX + 2 + jj] = fma(ws, lt / Lam, g[JMAX + 2 + jj]);
      }
    }
  }
}

}  // namespace mdpvi
