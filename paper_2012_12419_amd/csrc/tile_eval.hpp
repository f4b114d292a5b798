// tile_eval.hpp -- one tile of the fixed-policy FP64 evaluation sweep in the
// tile form, shared by the single-instance tile kernel (tile_eval.hip) and
// the batched tile rounds (batch.hip).
//
// The workgroup (NB lanes) stages the values of tile tb ((C+1)^T
// occupancies, J classes) in LDS (Vl [J][occ]) and backs up every state of
// the tile: low-digit neighbours from LDS, high-digit ones from global
// memory at workgroup-uniform offsets, the arrival term of the state's
// action from the FP64 side array (ain) of the previous sweep; it writes the
// new values and the new arrival terms (aout).  dmax: the running largest
// |V' - V| (a NaN wins), returned updated.  The caller synchronises the
// workgroup before the LDS image is overwritten.
#pragma once

#include "device.hpp"
#include "tile.hpp"

namespace mdpvi {

template <int K, int J, int T, int NB>
__device__ __forceinline__ double eval_tile_block(const Model& M, uint32_t tb, uint32_t occ, BufView pv,
                                                  BufView vin, BufView vout, BufView ain, BufView aout,
                                                  double* Vl, double dmax) {
  constexpr int H = K - T;
  const uint32_t nocc = static_cast<uint32_t>(M.n_occ);
  const uint32_t cls = nocc * 8u;
  int nh[H];
  const uint32_t o0 = tile_high<K, T>(M, tb, nh);

  stage_values<J, NB>(occ, o0, cls, vin, Vl);
  __syncthreads();

  uint32_t hd8[H], hr8[H];
  int load_high = 0;
#pragma unroll
  for (int h = 0; h < H; ++h) {
    const uint32_t st = static_cast<uint32_t>(M.stride[T + h]);
    hd8[h] = (nh[h] > 0 ? o0 - st : o0) * 8u;   // n_k = 0: the state itself, weight 0
    hr8[h] = (o0 - static_cast<uint32_t>(nh[h]) * st) * 8u;
    load_high += nh[h];
  }
  // lane a < K: size_e (C+1)^a, the index offset of a class-e placement on host a
  const uint32_t lane = threadIdx.x % kWave;
  int off_tab[J];
#pragma unroll
  for (int e = 0; e < J; ++e) {
    int v = 0;
#pragma unroll
    for (int a = 0; a < K; ++a)
      if (lane == static_cast<uint32_t>(a)) v = M.size[e] * static_cast<int>(M.stride[a]);
    off_tab[e] = v;
  }

  for (uint32_t i0 = 0; i0 < occ; i0 += NB) {
    // every lane takes part in the cross-lane reads; lanes past the tile
    // work on its last occupancy and store nothing
    const bool valid = i0 + threadIdx.x < occ;
    const uint32_t i = valid ? i0 + threadIdx.x : occ - 1;
    const uint32_t i8 = i * 8u;
    double vd[K][J], vr[K][J];
    int a[J];
#pragma unroll
    for (int e = 0; e < J; ++e) a[e] = ld_u8(pv, i, o0 + e * nocc);
#pragma unroll
    for (int h = 0; h < H; ++h) {
#pragma unroll
      for (int e = 0; e < J; ++e) {
        vd[T + h][e] = ld_f64(vin, i8, hd8[h] + e * cls);
        vr[T + h][e] = ld_f64(vin, i8, hr8[h] + e * cls);
      }
    }
    // arrival terms: placements along a high digit from global memory (the
    // other lanes load their own entry and use the LDS value)
    double ag[J];
#pragma unroll
    for (int e = 0; e < J; ++e) {
      const uint32_t off = static_cast<uint32_t>(__shfl(off_tab[e], a[e], kWave));
      ag[e] = ld_f64(ain, a[e] < K ? i8 + off * 8u : i8, o0 * 8u);
    }
    int n[K];
    tile_low<T>(M, i, n);
#pragma unroll
    for (int h = 0; h < H; ++h) n[T + h] = nh[h];
    int load = load_high;
#pragma unroll
    for (int k = 0; k < T; ++k) load += n[k];
    double vs[J];
#pragma unroll
    for (int e = 0; e < J; ++e) vs[e] = Vl[e * occ + i];
#pragma unroll
    for (int k = 0; k < T; ++k) {
      const uint32_t st = static_cast<uint32_t>(M.stride[k]);
      const uint32_t d = n[k] > 0 ? i - st : i;
      const uint32_t r = i - static_cast<uint32_t>(n[k]) * st;
#pragma unroll
      for (int e = 0; e < J; ++e) {
        vd[k][e] = Vl[e * occ + d];
        vr[k][e] = Vl[e * occ + r];
      }
    }
    const double idle = M.mu_L * static_cast<double>(M.KC - load);
    double anew = 0.0;
#pragma unroll
    for (int e = 0; e < J; ++e) {
      const double r = fma(-M.hold, static_cast<double>(M.KC - load), a[e] < K ? M.r_place[e] : M.r_reject[e]);
      double D = idle * vs[e];
      double rs = 0.0;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        D = fma(M.mu_L * n[k], vd[k][e], D);
        rs += vr[k][e];
      }
      D = fma(M.nu_L, rs, D);
      const double A = ag[e];
      const double vn = fma(M.gamma, D, fma(M.gamma, A, r));
      anew = fma(M.p[e], vn, anew);
      if (valid) {
        st_f64(vout, vn, i8, o0 * 8u + e * cls);
        const double d = fabs(vn - vs[e]);
        dmax = (d > dmax || d != d) ? d : dmax;
      }
    }
    if (valid) st_f64(aout, anew, i8, o0 * 8u);
  }
  return dmax;
}

}  // namespace mdpvi
