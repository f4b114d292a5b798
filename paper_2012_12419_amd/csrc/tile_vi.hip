// tile_vi.hip -- the value-iteration sweep (Eq. (18), Alg. 3 step 2) in the
// tile form: a workgroup stages the values and FP64 arrival terms of its
// (C+1)^T-occupancy tile in LDS, reads low-digit neighbours from LDS and
// high-digit neighbours from global memory at workgroup-uniform offsets.
//
// Per state the backup is that of the exact-shape direct form (arrival terms
// from the FP64 side array of the previous sweep, zero-weight stand-ins for
// missing release neighbours, -inf for placements without room), in the same
// order: bit-identical iterates.
#include "kernels.hpp"
#include "tile.hpp"

namespace mdpvi {

template <int K, int J, int T>
__global__ __launch_bounds__(kBlock) void vi_tile_kernel(Model M, TileShape S, const float* __restrict__ Vin,
                                                          float* __restrict__ Vout,
                                                          const double* __restrict__ Ain,
                                                          double* __restrict__ Aout, Ctl* ctl, double* res,
                                                          long long j, double tol) {
  if (sweep_stopped<ResKind::kMax>(ctl, res, j, tol)) return;
  constexpr int H = K - T;
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
  for (uint32_t tb = tw.first; tb < tw.end; tb += tw.step) {
  int nh[H];
  const uint32_t o0 = tile_high<K, T>(M, tb, nh);

  for (uint32_t i = threadIdx.x; i < occ; i += kBlock) {
#pragma unroll
    for (int e = 0; e < J; ++e) Vl[e * occ + i] = ld_f32(vin, i * 4u, o0 * 4u + e * cls);
    Al[i] = ld_f64(ain, i * 8u, o0 * 8u);
  }
  if (threadIdx.x == 0) Al[occ] = -INFINITY;
  __syncthreads();

  // high-digit neighbours: workgroup-uniform byte offsets of the tile base
  uint32_t hd4[H], hr4[H], ha8[H][J];
  int load_high = 0;
#pragma unroll
  for (int h = 0; h < H; ++h) {
    const uint32_t st = static_cast<uint32_t>(M.stride[T + h]);
    hd4[h] = (nh[h] > 0 ? o0 - st : o0) * 4u;   // n_k = 0: the state itself, weight 0
    hr4[h] = (o0 - static_cast<uint32_t>(nh[h]) * st) * 4u;
#pragma unroll
    for (int e = 0; e < J; ++e) {
      const int s = M.size[e];
      ha8[h][e] = nh[h] + s <= M.C ? (o0 + static_cast<uint32_t>(s) * st) * 8u : nocc * 8u;
    }
    load_high += nh[h];
  }

  for (uint32_t i = threadIdx.x; i < occ; i += kBlock) {
    float vd[K][J], vr[K][J];
    double aa[K][J];
    const uint32_t i4 = i * 4u, i8 = i * 8u;
#pragma unroll
    for (int h = 0; h < H; ++h) {
#pragma unroll
      for (int e = 0; e < J; ++e) {
        vd[T + h][e] = ld_f32(vin, i4, hd4[h] + e * cls);
        vr[T + h][e] = ld_f32(vin, i4, hr4[h] + e * cls);
        aa[T + h][e] = ld_f64(ain, i8, ha8[h][e]);
      }
    }
    int n[K];
    tile_low<T>(M, i, n);
#pragma unroll
    for (int h = 0; h < H; ++h) n[T + h] = nh[h];
    int load = load_high;
#pragma unroll
    for (int k = 0; k < T; ++k) load += n[k];
    float vs[J];
#pragma unroll
    for (int e = 0; e < J; ++e) vs[e] = Vl[e * occ + i];
    const double a_rej = Al[i];
#pragma unroll
    for (int k = 0; k < T; ++k) {
      const uint32_t st = static_cast<uint32_t>(M.stride[k]);
      const uint32_t d = n[k] > 0 ? i - st : i;
      const uint32_t r = i - static_cast<uint32_t>(n[k]) * st;
#pragma unroll
      for (int e = 0; e < J; ++e) {
        vd[k][e] = Vl[e * occ + d];
        vr[k][e] = Vl[e * occ + r];
        const int s = M.size[e];
        aa[k][e] = Al[n[k] + s <= M.C ? i + static_cast<uint32_t>(s) * st : occ];
      }
    }
    const double idle = M.mu_L * static_cast<double>(M.KC - load);
    double anew = 0.0;
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
      const double best = fmax(fma(M.gamma, a_rej, M.r_reject[e]), fma(M.gamma, ab, M.r_place[e]));
      const float vn = static_cast<float>(fma(M.gamma, D, best));
      st_f32(vout, vn, i4, o0 * 4u + e * cls);
      anew = fma(M.p[e], static_cast<double>(vn), anew);
      const double dd = fabs(static_cast<double>(vn) - static_cast<double>(vs[e]));
      dmax = fmax(dmax, dd);
      bad = bad || (dd != dd);
    }
    st_f64(aout, anew, i8, o0 * 8u);
  }
  __syncthreads();   // the next tile overwrites the LDS image
  }
  block_max_to(bad ? NAN : dmax, ctl, res, j, tol);
}

bool vi_tile_shape(const Model& M, TileShape* S) { return tile_shape(M, 4u * M.J + 8u, S); }

hipError_t launch_vi_tile(const Model& M, const TileShape& S, const float* Vin, float* Vout, const double* Ain,
                          double* Aout, Ctl* ctl, double* res, long long j, double tol, hipStream_t s) {
  const size_t lds = static_cast<size_t>(S.occ + 1) * 8 + static_cast<size_t>(S.occ) * 4 * M.J;
  return tile_dispatch(M.K, M.J, S.T, [&](auto kc, auto jc, auto tc) {
    constexpr int Kc = decltype(kc)::value, Jc = decltype(jc)::value, Tc = decltype(tc)::value;
    hipLaunchKernelGGL((vi_tile_kernel<Kc, Jc, Tc>), dim3(S.grid), dim3(kBlock), lds, s, M, S, Vin, Vout, Ain,
                       Aout, ctl, res, j, tol);
    return hipGetLastError();
  });
}

}  // namespace mdpvi
