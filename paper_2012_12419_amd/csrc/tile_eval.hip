// tile_eval.hip -- the fixed-policy FP64 evaluation sweep
// V'(n, e) = r(e, pi) + gamma (A(m_pi) + D(n, e)) (Eq. (18) without the max)
// in the tile form.
//
// The arrival term A(m) = sum_j lambda_j/Lam V(m, j) is kept in an FP64 side
// array written at the end of every sweep (the FMA chain the direct form
// evaluates at m, in the same order, so the value is the same).  A state
// reads the one arrival term its action needs straight from global memory
// (one double; the tile's own block and its neighbours' are L2 hits): only
// the values are staged in LDS, which keeps the image at 8J bytes per
// occupancy and four workgroups per CU.  The placement offset size_e
// (C+1)^a of action a comes from lane a of a per-class register table (one
// cross-lane read).
#include "kernels.hpp"
#include "tile.hpp"

namespace mdpvi {

template <int K, int J, int T>
__global__ __launch_bounds__(kTileBlock, kTileMinWaves) void eval_tile_kernel(Model M, TileShape S, const uint8_t* __restrict__ pi,
                                                            const double* __restrict__ Vin,
                                                            double* __restrict__ Vout,
                                                            const double* __restrict__ Ain,
                                                            double* __restrict__ Aout, Ctl* ctl, double* res,
                                                            long long j, double tol) {
  if (sweep_stopped<ResKind::kMax>(ctl, res, j, tol)) return;
  constexpr int H = K - T;
  extern __shared__ double tile_lds[];
  const uint32_t occ = S.occ;
  double* Vl = tile_lds;            // [J][occ]
  const uint32_t nocc = static_cast<uint32_t>(M.n_occ);
  const uint32_t ns = static_cast<uint32_t>(M.n_states);
  const uint32_t cls = nocc * 8u;
  const BufView pv = make_view(pi, ns);
  const BufView vin = make_view(Vin, ns * 8u);
  const BufView vout = make_view(Vout, ns * 8u);
  const BufView ain = make_view(Ain, nocc * 8u);
  const BufView aout = make_view(Aout, nocc * 8u);
  double dmax = 0.0;
  const TileWalk tw = tile_walk(S);
  for (uint32_t tp = tw.first; tp < tw.end; tp += tw.step) {
    const uint32_t tb = tile_at(S, tp);
  int nh[H];
  const uint32_t o0 = tile_high<K, T>(M, tb, nh);

  stage_values<J, kTileBlock>(occ, o0, cls, vin, Vl);
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

  for (uint32_t i0 = 0; i0 < occ; i0 += kTileBlock) {
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
  __syncthreads();   // the next tile overwrites the LDS image
  }
  block_max_to<kTileBlock>(dmax, ctl, res, j, tol);
}

// A(o) = sum_e lambda_e/Lam V(o, e) of an FP64 iterate (the FMA chain the
// evaluation sweeps use).
__global__ void eval_arrival_init_kernel(Model M, const double* __restrict__ V, double* __restrict__ A) {
  const uint64_t o = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (o >= static_cast<uint64_t>(M.n_occ)) return;
  double a = 0.0;
  for (int e = 0; e < M.J; ++e) a = fma(M.p[e], V[o + static_cast<uint64_t>(e) * M.n_occ], a);
  A[o] = a;
}

bool eval_tile_shape(const Model& M, TileShape* S) {
  return M.n_states < (int64_t{1} << 28) && tile_shape(M, 8u * M.J, kTileLds, S);
}

hipError_t launch_eval_arrival_init(const Model& M, const double* V, double* A, hipStream_t s) {
  const uint32_t grid = static_cast<uint32_t>((static_cast<uint64_t>(M.n_occ) + 255) / 256);
  hipLaunchKernelGGL(eval_arrival_init_kernel, dim3(grid), dim3(256), 0, s, M, V, A);
  return hipGetLastError();
}

hipError_t launch_eval_tile(const Model& M, const TileShape& S, const uint8_t* pi, const double* Vin,
                            double* Vout, const double* Ain, double* Aout, Ctl* ctl, double* res, long long j,
                            double tol, hipStream_t s) {
  const size_t lds = static_cast<size_t>(S.occ) * 8 * M.J;
  return tile_dispatch(M.K, M.J, S.T, [&](auto kc, auto jc, auto tc) {
    constexpr int Kc = decltype(kc)::value, Jc = decltype(jc)::value, Tc = decltype(tc)::value;
    hipLaunchKernelGGL((eval_tile_kernel<Kc, Jc, Tc>), dim3(S.grid), dim3(kTileBlock), lds, s, M, S, pi, Vin, Vout,
                       Ain, Aout, ctl, res, j, tol);
    return hipGetLastError();
  });
}

}  // namespace mdpvi
