// adjoint_group.hip -- single-instance launches of the group form of the
// transposed (adjoint) sweep (adjoint_group.hpp), with the stop test's
// control words loaded together with the weights.
//
// The transposed backup of adjoint.hip (w' = c + gamma P_pi^T w, predecessors
// by arrival, release, reset and idling) reads, for a target occupancy n',
// the actions and weights of its arrival predecessors n' - size_e 1_k, the
// weights of n' + 1_k, and for every digit k with n'_k = 0 the C+1 weights
// of the line along digit k.  Done one occupancy per thread straight from
// global memory this is a chain of memory round trips: a wavefront takes as
// many as the lines any of its lanes sums; the group form reads every
// neighbour along the two lowest digits from LDS instead.
#include "adjoint_group.hpp"
#include "adjoint_impl.hpp"
#include "device.hpp"
#include "kernels.hpp"
#include "tile.hpp"

namespace mdpvi {

template <int K, int J>
__global__ __launch_bounds__(kBlock) void adjoint_group_kernel(Model M, const uint8_t* __restrict__ pi,
                                                               const float* __restrict__ win,
                                                               float* __restrict__ wout, Ctl* ctl, double* res,
                                                               long long j, double tol, uint32_t per_block,
                                                               uint32_t n_groups) {
  // the stop test's words, loaded first so that their round trip overlaps
  // the weights' (the test itself runs once the weights' loads are issued)
  const long long done = load_agent(&ctl->done_iter);
  const double rv = j > 0 ? load_agent(res + sum_word(j - 1, threadIdx.x % kResLanes)) : 0.0;
  // the result is the same in every wavefront of the launch: the residual
  // words of sweep j-1 are final, and done_iter only changes here to j when
  // that test has failed
  auto stop = [&]() -> bool {
    double v = rv;
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    const bool by_res = done < 0 && j > 0 && !(v >= tol);
    if (done >= 0 || by_res) {
      if (by_res && blockIdx.x == 0 && threadIdx.x == 0) store_agent(&ctl->done_iter, j);
      return true;
    }
    if (blockIdx.x == 0 && threadIdx.x < kResLanes) store_agent(res + sum_word(j + 1, threadIdx.x), 0.0);
    return false;
  };
  double dsum = 0.0;
  if (!adjoint_group_block<K, J>(M, pi, win, wout, xcd_block(blockIdx.x, gridDim.x) * per_block, per_block,
                                 n_groups, stop, &dsum))
    return;
  block_sum_to(dsum, res, j);
}

bool adjoint_group_shape(const Model& M) {
  return M.K >= 3 && M.K <= 8 && M.J >= 1 && M.J <= 3 && M.R * M.R <= kBlock && M.C < kLineLoads &&
         M.n_states < (int64_t{1} << 29);
}

hipError_t launch_adjoint_group(const Model& M, const uint8_t* pi, const float* win, float* wout, Ctl* ctl,
                                double* res, long long j, double tol, hipStream_t s) {
  if (!adjoint_group_shape(M)) return hipErrorInvalidValue;
  const uint32_t G = static_cast<uint32_t>(M.R * M.R);
  const uint32_t per_block = kBlock / G;
  const uint32_t n_groups = static_cast<uint32_t>(M.n_occ / G);
  const dim3 grid((n_groups + per_block - 1) / per_block);
  return tile_dispatch(M.K, M.J, 2, [&](auto kc, auto jc, auto) {
    constexpr int Kc = decltype(kc)::value, Jc = decltype(jc)::value;
    hipLaunchKernelGGL((adjoint_group_kernel<Kc, Jc>), grid, dim3(kBlock), 0, s, M, pi, win, wout, ctl, res, j,
                       tol, per_block, n_groups);
    return hipGetLastError();
  });
}

}  // namespace mdpvi
