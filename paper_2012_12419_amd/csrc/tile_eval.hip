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
#include "tile_eval.hpp"

namespace mdpvi {

template <int K, int J, int T>
__global__ __launch_bounds__(kTileBlock, kTileMinWaves) void eval_tile_kernel(Model M, TileShape S, const uint8_t* __restrict__ pi,
                                                            const double* __restrict__ Vin,
                                                            double* __restrict__ Vout,
                                                            const double* __restrict__ Ain,
                                                            double* __restrict__ Aout, Ctl* ctl, double* res,
                                                            long long j, double tol) {
  if (sweep_stopped<ResKind::kMax>(ctl, res, j, tol)) return;
  extern __shared__ double tile_lds[];
  const uint32_t occ = S.occ;
  double* Vl = tile_lds;            // [J][occ]
  const uint32_t nocc = static_cast<uint32_t>(M.n_occ);
  const uint32_t ns = static_cast<uint32_t>(M.n_states);
  const BufView pv = make_view(pi, ns);
  const BufView vin = make_view(Vin, ns * 8u);
  const BufView vout = make_view(Vout, ns * 8u);
  const BufView ain = make_view(Ain, nocc * 8u);
  const BufView aout = make_view(Aout, nocc * 8u);
  double dmax = 0.0;
  const TileWalk tw = tile_walk(S);
  for (uint32_t tp = tw.first; tp < tw.end; tp += tw.step) {
    const uint32_t tb = tile_at(S, tp);
    dmax = eval_tile_block<K, J, T, kTileBlock>(M, tb, occ, pv, vin, vout, ain, aout, Vl, dmax);
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
