// adjoint_group.hpp -- the group form of the transposed (adjoint) backup as
// a workgroup-level device function, shared by the single-instance group
// kernel (adjoint_group.hip) and the batched round kernel (batch.hip).
//
// A group is the (C+1)^2 occupancies that share digits 2..K-1.  The calling
// workgroup (kBlock lanes) takes groups first_group .. first_group +
// per_block - 1 of the instance's n_groups, one occupancy per lane.  Each
// lane loads the actions and weights of its own states and its neighbours
// along the high digits, and publishes its own to LDS; every neighbour along
// digits 0 and 1 -- arrival and release predecessors and the two reset lines
// -- is then an LDS read.  A line along a high digit is needed by a whole
// group (n_k is the same for all its occupancies): the first such line is
// loaded right after the rest, further ones (groups with two or more zero
// high digits) later.  Terms are added in the order of adjoint_occupancy, so
// w is bit-identical to the other adjoint forms.
#pragma once

#include "adjoint_impl.hpp"
#include "device.hpp"

namespace mdpvi {

// stop(): called by every lane once its loads are issued; true makes the
// function return false at once (before any LDS write or barrier: the answer
// must be the same for the whole workgroup).  Otherwise the new weights are
// stored and *dsum_out receives the lane's sum of |w' - w|; returns true.
template <int K, int J, typename Stop>
__device__ __forceinline__ bool adjoint_group_block(const Model& M, const uint8_t* __restrict__ pi,
                                                    const float* __restrict__ win, float* __restrict__ wout,
                                                    uint32_t first_group, uint32_t per_block, uint32_t n_groups,
                                                    Stop&& stop, double* dsum_out) {
  __shared__ float ws[J][kBlock];
  __shared__ int ps[J][kBlock];
  const uint32_t R = static_cast<uint32_t>(M.R), G = R * R;
  const uint32_t C = static_cast<uint32_t>(M.C);
  const uint32_t nocc = static_cast<uint32_t>(M.n_occ);
  const uint32_t l = threadIdx.x;
  // lanes past the last whole group stand in for the group's last occupancy
  // and lanes of a group past n_groups for group n_groups - 1: both compute
  // from data that exists and store nothing
  uint32_t gi = l / G, r = l - gi * G;
  bool active = gi < per_block;
  if (!active) {
    gi = per_block - 1;
    r = G - 1;
  }
  uint32_t g = first_group + gi;
  if (g >= n_groups) {
    active = false;
    g = n_groups - 1;
  }
  const uint32_t o = g * G + r;
  const uint32_t pos = gi * G + r;   // this occupancy's LDS slot (= l for an active lane)

  int n[K];
  n[0] = static_cast<int>(r % R);
  n[1] = static_cast<int>(r / R);
  {
    uint32_t q = g;
#pragma unroll
    for (int k = 2; k < K; ++k) {
      const uint32_t d = fast_div(q, M.divR);
      n[k] = static_cast<int>(q - d * R);
      q = d;
    }
  }
  int load = 0;
#pragma unroll
  for (int k = 0; k < K; ++k) load += n[k];

  const BufView vp = make_view(pi, static_cast<uint32_t>(M.n_states));
  const BufView vw = make_view(win, static_cast<uint32_t>(M.n_states) * 4u);
  const BufView vo = make_view(wout, static_cast<uint32_t>(M.n_states) * 4u);

  // own states, and the neighbours along the high digits
  int p_own[J];
  float w_own[J];
  int p_k[K][J];
  float w_k[K][J], w_rel[K][J];
#pragma unroll
  for (int e = 0; e < J; ++e) {
    const uint32_t eo = static_cast<uint32_t>(e) * nocc;
    p_own[e] = ld_u8(vp, o, eo);
    w_own[e] = ld_f32(vw, 4u * o, 4u * eo);
#pragma unroll
    for (int k = 2; k < K; ++k) {
      const uint32_t st = static_cast<uint32_t>(M.stride[k]);
      const uint32_t src = n[k] >= M.size[e] ? o - static_cast<uint32_t>(M.size[e]) * st : o;
      p_k[k][e] = ld_u8(vp, src, eo);
      w_k[k][e] = ld_f32(vw, 4u * src, 4u * eo);
      w_rel[k][e] = ld_f32(vw, 4u * (n[k] < M.C ? o + st : o), 4u * eo);
    }
  }
  // the line along the first high digit with n_k = 0 (positions x > C read
  // the occupancy itself: a guard per load would make each one a branch
  // that waits for its load)
  int k1 = K;
  uint32_t st1 = 0;
#pragma unroll
  for (int k = K - 1; k >= 2; --k) {
    if (n[k] == 0) {
      k1 = k;
      st1 = static_cast<uint32_t>(M.stride[k]);
    }
  }
  float h1[J][kLineLoads];
  if (k1 < K) {
#pragma unroll
    for (int e = 0; e < J; ++e) {
#pragma unroll
      for (int x = 0; x < kLineLoads; ++x) {
        const uint32_t s = static_cast<uint32_t>(x) <= C ? o + static_cast<uint32_t>(x) * st1 : o;
        h1[e][x] = ld_f32(vw, 4u * s, 4u * static_cast<uint32_t>(e) * nocc);
      }
    }
  }

  // the caller's stop test, with the loads above in flight
  if (stop()) return false;

#pragma unroll
  for (int e = 0; e < J; ++e) {
    ws[e][l] = w_own[e];
    ps[e][l] = p_own[e];
  }
  __syncthreads();

  // arrival inflow: the paid cloud at n', then placements on host k from
  // n' - size_e 1_k, k = 0..K-1, e = 0..J-1
  double B = 0.0;
#pragma unroll
  for (int e = 0; e < J; ++e) B += p_own[e] == M.K ? static_cast<double>(w_own[e]) : 0.0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
#pragma unroll
    for (int e = 0; e < J; ++e) {
      if (k < 2) {
        if (n[k] >= M.size[e]) {
          const uint32_t q = pos - static_cast<uint32_t>(M.size[e]) * (k == 0 ? 1u : R);
          if (ps[e][q] == k) B += static_cast<double>(ws[e][q]);
        }
      } else {
        B += (n[k] >= M.size[e] && p_k[k][e] == k) ? static_cast<double>(w_k[k][e]) : 0.0;
      }
    }
  }

  // reset term, per class: each line summed from zero in the order x =
  // 0..C, the lines added in the order k = 0..K-1; the lines of further
  // zero high digits are loaded for every class at once
  double rs[J];
#pragma unroll
  for (int e = 0; e < J; ++e) rs[e] = 0.0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    if (n[k] != 0) continue;
    if (k < 2) {
      const uint32_t st = k == 0 ? 1u : R;
#pragma unroll
      for (int e = 0; e < J; ++e) {
        float v[kLineLoads];
#pragma unroll
        for (int x = 0; x < kLineLoads; ++x) v[x] = ws[e][static_cast<uint32_t>(x) <= C ? pos + x * st : pos];
        double line = 0.0;
#pragma unroll
        for (int x = 0; x < kLineLoads; ++x)
          if (static_cast<uint32_t>(x) <= C) line += static_cast<double>(v[x]);
        rs[e] += line;
      }
    } else if (k == k1) {
#pragma unroll
      for (int e = 0; e < J; ++e) {
        double line = 0.0;
#pragma unroll
        for (int x = 0; x < kLineLoads; ++x)
          if (static_cast<uint32_t>(x) <= C) line += static_cast<double>(h1[e][x]);
        rs[e] += line;
      }
    } else {
      const uint32_t st = static_cast<uint32_t>(M.stride[k]);
      float v[J][kLineLoads];
#pragma unroll
      for (int e = 0; e < J; ++e) {
#pragma unroll
        for (int x = 0; x < kLineLoads; ++x)
          v[e][x] = ld_f32(vw, 4u * (static_cast<uint32_t>(x) <= C ? o + x * st : o),
                           4u * static_cast<uint32_t>(e) * nocc);
      }
#pragma unroll
      for (int e = 0; e < J; ++e) {
        double line = 0.0;
#pragma unroll
        for (int x = 0; x < kLineLoads; ++x)
          if (static_cast<uint32_t>(x) <= C) line += static_cast<double>(v[e][x]);
        rs[e] += line;
      }
    }
  }

  const double idle = M.mu_L * static_cast<double>(M.KC - load);
  double dsum = 0.0;
#pragma unroll
  for (int e = 0; e < J; ++e) {
    const uint32_t eo = static_cast<uint32_t>(e) * nocc;
    const float wold = w_own[e];
    double acc = fma(M.p[e], B, idle * static_cast<double>(wold));
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (k < 2) {
        const uint32_t st = k == 0 ? 1u : R;
        if (n[k] < M.C) acc = fma(M.mu_L * (n[k] + 1), static_cast<double>(ws[e][pos + st]), acc);
      } else {
        acc = fma(n[k] < M.C ? M.mu_L * (n[k] + 1) : 0.0, static_cast<double>(w_rel[k][e]), acc);
      }
    }
    acc = fma(M.nu_L, rs[e], acc);
    const double c = (o == 0) ? M.c_obj[e] : 0.0;
    const float wn = static_cast<float>(fma(M.gamma, acc, c));
    if (active) {
      st_f32(vo, wn, 4u * o, 4u * eo);
      dsum += fabs(static_cast<double>(wn) - static_cast<double>(wold));
    }
  }
  *dsum_out = dsum;
  return true;
}


}  // namespace mdpvi
