// tile_vi.hip -- the value-iteration sweep (Eq. (18), Alg. 3 step 2) in the
// tile form, and the block-asynchronous variant (the paper's BSDI, Alg. 4)
// built on the same tiles.
//
// Tile form: a workgroup stages the values and FP64 arrival terms of its
// (C+1)^T-occupancy tile in LDS, reads low-digit neighbours from LDS and
// high-digit neighbours from global memory at workgroup-uniform offsets.
// Per state the backup is that of the exact-shape direct form (arrival terms
// from the FP64 side array of the previous sweep, zero-weight stand-ins for
// missing release neighbours, -inf for placements without room), in the same
// order: bit-identical iterates.
//
// Block-asynchronous form: a pass stages the tile, runs `inner` episodes of
// the same backup on it, each episode reading the tile's latest values from
// LDS (its previous episode's results, a double-buffered synchronous update
// inside the tile) and every successor outside the tile from the previous
// pass in global memory, and writes the last episode's values back.  A
// successor stays inside the tile when it moves along a low digit, when it is
// the state itself (idle, paid cloud) and when it is the reset of a high-digit
// host that is already empty.  The pass residual is the largest change
// against the previous pass.  With inner = 1 a pass is one Jacobi sweep.
#include "kernels.hpp"
#include "tile.hpp"
#include "tile_vi.hpp"

namespace mdpvi {

template <int K, int J, int T>
__global__ __launch_bounds__(kTileBlock, kTileMinWaves) void vi_tile_kernel(Model M, TileShape S, const float* __restrict__ Vin,
                                                          float* __restrict__ Vout,
                                                          const double* __restrict__ Ain,
                                                          double* __restrict__ Aout, Ctl* ctl, double* res,
                                                          long long j, double tol) {
  if (sweep_stopped<ResKind::kMax>(ctl, res, j, tol)) return;
  extern __shared__ double tile_lds[];
  const uint32_t occ = S.occ;
  double* Al = tile_lds;                                       // [occ + 1], -inf at occ
  float* Vl = reinterpret_cast<float*>(tile_lds + occ + 1);     // [J][occ]
  const uint32_t nocc = static_cast<uint32_t>(M.n_occ);
  const uint32_t ns = static_cast<uint32_t>(M.n_states);
  const uint32_t cls = nocc * 4u;
  const BufView vin = make_view(Vin, ns * 4u);
  const BufView vout = make_view(Vout, ns * 4u);
  const BufView ain = make_view(Ain, (nocc + kSentinel) * 8u);
  const BufView aout = make_view(Aout, nocc * 8u);
  double dmax = 0.0;
  bool bad = false;
  const TileWalk tw = tile_walk(S);
  for (uint32_t tp = tw.first; tp < tw.end; tp += tw.step) {
    const uint32_t tb = tile_at(S, tp);
    TileHigh<K, J, T> H;
    tile_high_setup<K, J, T>(M, tb, H);
    tile_stage<J, kTileBlock>(M, occ, H.o0, vin, ain, Vl, Al);
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < occ; i += kTileBlock) {
      float vs[J], vn[J];
      double anew;
      tile_backup<K, J, T, false>(M, H, occ, Vl, Al, vin, ain, i, vs, vn, anew);
#pragma unroll
      for (int e = 0; e < J; ++e) {
        st_f32(vout, vn[e], i * 4u, H.o0 * 4u + e * cls);
        const double dd = fabs(static_cast<double>(vn[e]) - static_cast<double>(vs[e]));
        dmax = fmax(dmax, dd);
        bad = bad || (dd != dd);
      }
      st_f64(aout, anew, i * 8u, H.o0 * 8u);
    }
    __syncthreads();   // the next tile overwrites the LDS image
  }
  block_max_to<kTileBlock>(bad ? NAN : dmax, ctl, res, j, tol);
}

template <int K, int J, int T>
__global__ __launch_bounds__(kBlock) void vi_bsdi_kernel(Model M, TileShape S, int inner,
                                                          const float* __restrict__ Vin, float* __restrict__ Vout,
                                                          const double* __restrict__ Ain,
                                                          double* __restrict__ Aout, Ctl* ctl, double* res,
                                                          long long j, double tol) {
  if (sweep_stopped<ResKind::kMax>(ctl, res, j, tol)) return;
  extern __shared__ double tile_lds[];
  const uint32_t occ = S.occ;
  // two LDS images: episode k reads image k % 2 and writes the other
  const uint32_t img = occ + 1 + (occ * J + 1) / 2;   // doubles per image
  double* Al[2] = {tile_lds, tile_lds + img};
  float* Vl[2] = {reinterpret_cast<float*>(Al[0] + occ + 1), reinterpret_cast<float*>(Al[1] + occ + 1)};
  const uint32_t nocc = static_cast<uint32_t>(M.n_occ);
  const uint32_t ns = static_cast<uint32_t>(M.n_states);
  const uint32_t cls = nocc * 4u;
  const BufView vin = make_view(Vin, ns * 4u);
  const BufView vout = make_view(Vout, ns * 4u);
  const BufView ain = make_view(Ain, (nocc + kSentinel) * 8u);
  const BufView aout = make_view(Aout, nocc * 8u);
  double dmax = 0.0;
  bool bad = false;
  const TileWalk tw = tile_walk(S);
  for (uint32_t tp = tw.first; tp < tw.end; tp += tw.step) {
    const uint32_t tb = tile_at(S, tp);
    TileHigh<K, J, T> H;
    tile_high_setup<K, J, T>(M, tb, H);
    tile_stage<J, kBlock>(M, occ, H.o0, vin, ain, Vl[0], Al[0]);
    if (threadIdx.x == 0) Al[1][occ] = -INFINITY;
    __syncthreads();
    for (int k = 0; k < inner; ++k) {
      const int src = k & 1;
      const bool last = k + 1 == inner;
      for (uint32_t i = threadIdx.x; i < occ; i += kBlock) {
        float vs[J], vn[J];
        double anew;
        tile_backup<K, J, T, true>(M, H, occ, Vl[src], Al[src], vin, ain, i, vs, vn, anew);
        if (!last) {
#pragma unroll
          for (int e = 0; e < J; ++e) Vl[src ^ 1][e * occ + i] = vn[e];
          Al[src ^ 1][i] = anew;
        } else {
#pragma unroll
          for (int e = 0; e < J; ++e) {
            st_f32(vout, vn[e], i * 4u, H.o0 * 4u + e * cls);
            // change against the previous pass, whose value was staged
            const float v0 = k == 0 ? vs[e] : ld_f32(vin, i * 4u, H.o0 * 4u + e * cls);
            const double dd = fabs(static_cast<double>(vn[e]) - static_cast<double>(v0));
            dmax = fmax(dmax, dd);
            bad = bad || (dd != dd);
          }
          st_f64(aout, anew, i * 8u, H.o0 * 8u);
        }
      }
      __syncthreads();   // episode k's image is complete before episode k+1 reads it
    }
  }
  block_max_to(bad ? NAN : dmax, ctl, res, j, tol);
}

bool vi_tile_shape(const Model& M, TileShape* S) { return tile_shape(M, 4u * M.J + 8u, kTileLds, S); }

bool vi_bsdi_shape(const Model& M, TileShape* S) {
  return tile_shape(M, 2u * (4u * M.J + 8u), kBsdiLds, S);
}

hipError_t launch_vi_tile(const Model& M, const TileShape& S, const float* Vin, float* Vout, const double* Ain,
                          double* Aout, Ctl* ctl, double* res, long long j, double tol, hipStream_t s) {
  const size_t lds = static_cast<size_t>(S.occ + 1) * 8 + static_cast<size_t>(S.occ) * 4 * M.J;
  return tile_dispatch(M.K, M.J, S.T, [&](auto kc, auto jc, auto tc) {
    constexpr int Kc = decltype(kc)::value, Jc = decltype(jc)::value, Tc = decltype(tc)::value;
    hipLaunchKernelGGL((vi_tile_kernel<Kc, Jc, Tc>), dim3(S.grid), dim3(kTileBlock), lds, s, M, S, Vin, Vout, Ain,
                       Aout, ctl, res, j, tol);
    return hipGetLastError();
  });
}

hipError_t launch_vi_bsdi(const Model& M, const TileShape& S, int inner, const float* Vin, float* Vout,
                          const double* Ain, double* Aout, Ctl* ctl, double* res, long long j, double tol,
                          hipStream_t s) {
  const size_t img = static_cast<size_t>(S.occ) + 1 + (static_cast<size_t>(S.occ) * M.J + 1) / 2;
  const size_t lds = 2 * img * 8;
  return tile_dispatch(M.K, M.J, S.T, [&](auto kc, auto jc, auto tc) {
    constexpr int Kc = decltype(kc)::value, Jc = decltype(jc)::value, Tc = decltype(tc)::value;
    hipLaunchKernelGGL((vi_bsdi_kernel<Kc, Jc, Tc>), dim3(S.grid), dim3(kBlock), lds, s, M, S, inner, Vin,
                       Vout, Ain, Aout, ctl, res, j, tol);
    return hipGetLastError();
  });
}

}  // namespace mdpvi
