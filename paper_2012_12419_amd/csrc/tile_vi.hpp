// tile_vi.hpp -- the per-occupancy backup and the staging of the tile form
// of value iteration, shared by the single-instance tile and
// block-asynchronous kernels (tile_vi.hip) and the batched tile rounds
// (batch.hip).
#pragma once

#include "device.hpp"
#include "tile.hpp"

namespace mdpvi {

// Backup of tile occupancy i: own values, low-digit neighbours and in-tile
// arrival terms from the LDS image (Vl [J][occ], Al [occ + 1] with -inf at
// occ), high-digit neighbours from global memory.  With SelfLatest the reset
// of an empty high-digit host, which is the state itself, takes the state's
// LDS value (the block-asynchronous form; in a Jacobi sweep both are the
// same).  Returns the new values vn, the new arrival term anew = sum_e
// lambda_e/Lam vn_e and the values vs the backup read at the state itself.
//
// AGlobal: the arrival terms inside the tile too are read from ain (global
// memory) instead of Al, which is then not used: the own term at o0 + i, a
// placement along a low digit at o0 + i + size_e (C+1)^k, one without room
// from the -inf block that follows the n_occ terms (occ entries).  The
// workgroup then stages only the values (a smaller LDS image); the
// arithmetic is the same.
template <int K, int J, int T, bool SelfLatest, bool AGlobal = false>
__device__ __forceinline__ void tile_backup(const Model& M, const TileHigh<K, J, T>& H, uint32_t occ,
                                            const float* Vl, const double* Al, BufView vin, BufView ain,
                                            uint32_t i, float (&vs)[J], float (&vn)[J], double& anew) {
  constexpr int NH = K - T;
  const uint32_t cls = static_cast<uint32_t>(M.n_occ) * 4u;
  float vd[K][J], vr[K][J];
  double aa[K][J];
  const uint32_t i4 = i * 4u, i8 = i * 8u;
#pragma unroll
  for (int h = 0; h < NH; ++h) {
#pragma unroll
    for (int e = 0; e < J; ++e) {
      vd[T + h][e] = ld_f32(vin, i4, H.hd4[h] + e * cls);
      vr[T + h][e] = ld_f32(vin, i4, H.hr4[h] + e * cls);
      aa[T + h][e] = ld_f64(ain, i8, H.ha8[h][e]);
    }
  }
  int n[K];
  tile_low<T>(M, i, n);
#pragma unroll
  for (int h = 0; h < NH; ++h) n[T + h] = H.nh[h];
  int load = H.load_high;
#pragma unroll
  for (int k = 0; k < T; ++k) load += n[k];
#pragma unroll
  for (int e = 0; e < J; ++e) vs[e] = Vl[e * occ + i];
  if constexpr (SelfLatest) {
#pragma unroll
    for (int h = 0; h < NH; ++h) {
#pragma unroll
      for (int e = 0; e < J; ++e) vr[T + h][e] = H.nh[h] == 0 ? vs[e] : vr[T + h][e];
    }
  }
  double a_rej;
  if constexpr (AGlobal) {
    a_rej = ld_f64(ain, i8, H.o0 * 8u);
  } else {
    a_rej = Al[i];
  }
#pragma unroll
  for (int k = 0; k < T; ++k) {
    const uint32_t st = static_cast<uint32_t>(M.stride[k]);
    const uint32_t d = n[k] > 0 ? i - st : i;   // n_k = 0: the state itself, weight 0
    const uint32_t r = i - static_cast<uint32_t>(n[k]) * st;
#pragma unroll
    for (int e = 0; e < J; ++e) {
      vd[k][e] = Vl[e * occ + d];
      vr[k][e] = Vl[e * occ + r];
      const int s = M.size[e];
      if constexpr (AGlobal) {
        const uint32_t nocc8 = static_cast<uint32_t>(M.n_occ) * 8u;
        aa[k][e] = ld_f64(ain, n[k] + s <= M.C ? i8 + static_cast<uint32_t>(s) * st * 8u : nocc8 - H.o0 * 8u + i8,
                          H.o0 * 8u);
      } else {
        aa[k][e] = Al[n[k] + s <= M.C ? i + static_cast<uint32_t>(s) * st : occ];
      }
    }
  }
  const double idle = M.mu_L * static_cast<double>(M.KC - load);
  anew = 0.0;
#pragma unroll
  for (int e = 0; e < J; ++e) {
    double ab = aa[0][e];
#pragma unroll
    for (int a = 1; a < K; ++a) ab = fmax(ab, aa[a][e]);
    double D = idle * static_cast<double>(vs[e]);
    double rs = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      D = fma(M.mu_L * n[k], static_cast<double>(vd[k][e]), D);
      rs += static_cast<double>(vr[k][e]);
    }
    D = fma(M.nu_L, rs, D);
    const double fu = static_cast<double>(M.KC - load);   // free units (under-utilisation penalty)
    const double best = fmax(fma(M.gamma, a_rej, fma(-M.hold, fu, M.r_reject[e])), fma(M.gamma, ab, fma(-M.hold, fu, M.r_place[e])));
    vn[e] = static_cast<float>(fma(M.gamma, D, best));
    anew = fma(M.p[e], static_cast<double>(vn[e]), anew);
  }
}

// Stages only the tile's FP32 values into Vl [J][occ] (for AGlobal
// backups), NB threads, kStageRounds loads per thread in flight.
template <int J, int NB>
__device__ __forceinline__ void tile_stage_values(const Model& M, uint32_t occ, uint32_t o0, BufView vin,
                                                  float* Vl) {
  const uint32_t cls = static_cast<uint32_t>(M.n_occ) * 4u;
  for (uint32_t base = 0; base < occ; base += kStageRounds * NB) {
    float v[kStageRounds][J];
#pragma unroll
    for (int r = 0; r < kStageRounds; ++r) {
      uint32_t i = base + r * NB + threadIdx.x;
      i = i < occ ? i : occ - 1;
#pragma unroll
      for (int e = 0; e < J; ++e) v[r][e] = ld_f32(vin, i * 4u, o0 * 4u + e * cls);
    }
#pragma unroll
    for (int r = 0; r < kStageRounds; ++r) {
      const uint32_t i = base + r * NB + threadIdx.x;
      if (i < occ) {
#pragma unroll
        for (int e = 0; e < J; ++e) Vl[e * occ + i] = v[r][e];
      }
    }
  }
}

// Stages the tile's values and arrival terms into (Vl, Al) and sets the
// sentinel Al[occ] = -inf.
template <int J, int NB>
__device__ __forceinline__ void tile_stage(const Model& M, uint32_t occ, uint32_t o0, BufView vin, BufView ain,
                                           float* Vl, double* Al) {
  stage_tile<J, NB, float>(occ, o0, static_cast<uint32_t>(M.n_occ) * 4u, vin, ain, Vl, Al);
  if (threadIdx.x == 0) Al[occ] = -INFINITY;
}

}  // namespace mdpvi
