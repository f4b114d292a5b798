// tile.hpp -- the tile form of the exact-shape sweeps (value iteration and
// fixed-policy evaluation).
//
// A tile is the set of (C+1)^T occupancies that share the high digits
// n_T..n_{K-1}; one workgroup per tile, tiles in index order (XCD-aware), so
// the traversal of the occupancy grid is the linear one of the direct form
// and neighbouring tiles share an XCD's L2.  The workgroup stages its tile's
// values (all classes) and FP64 arrival terms in LDS; then every neighbour
// along a low digit (release, reset, placement) is an LDS read, and every
// neighbour along a high digit is a global load at the thread's own offset
// plus a workgroup-uniform offset (a scalar register of the buffer load),
// with a workgroup-uniform feasibility test.  Against the direct form this
// moves 3T of the 3K neighbour groups of a state from the vector memory
// pipeline to LDS and the high-digit address arithmetic to the scalar unit.
//
// Per state the arithmetic and its order are those of the direct exact-shape
// forms: every form computes bit-identical iterates.
#pragma once

#include "device.hpp"

#include <type_traits>

namespace mdpvi {

// Entries of -inf after the n_occ arrival terms of each value-iteration
// arrival array: a placement without room along a high digit reads entry
// n_occ + i (i < tile size <= kSentinel).
constexpr uint32_t kSentinel = 4096;
// LDS bytes a tile image may take (the block-asynchronous form holds two).
constexpr uint32_t kTileLds = 48 * 1024;
constexpr uint32_t kBsdiLds = 64 * 1024;

struct TileShape {
  uint32_t occ;    // (C+1)^T occupancies per tile
  uint32_t n;      // (C+1)^(K-T) tiles
  int32_t T;       // low digits of a tile
  uint32_t grid;   // workgroups launched: n (one tile each), or a multiple of 8
                   // that walk the tiles of their XCD's range in order
};

// Tiles of workgroup blockIdx.x: with one workgroup per tile, the XCD-aware
// order of the direct form; otherwise XCD x (workgroups b with b % 8 = x)
// owns tiles [x n / 8, (x+1) n / 8), which its grid / 8 workgroups take in
// index order, so that the tiles in flight on an XCD form a sliding window.
struct TileWalk {
  uint32_t first, end, step;
};

__device__ __forceinline__ TileWalk tile_walk(const TileShape& S) {
  if (S.grid == S.n) {
    const uint32_t t = xcd_block(blockIdx.x, gridDim.x);
    return TileWalk{t, t + 1, 1};
  }
  const uint32_t x = blockIdx.x % kNumXcd;
  const uint32_t w = blockIdx.x / kNumXcd;
  const uint32_t lo = static_cast<uint32_t>(static_cast<uint64_t>(S.n) * x / kNumXcd);
  const uint32_t hi = static_cast<uint32_t>(static_cast<uint64_t>(S.n) * (x + 1) / kNumXcd);
  return TileWalk{lo + w, hi, gridDim.x / kNumXcd};
}

// The deepest tile (T in 2..min(4, K-1)) whose LDS footprint of
// bytes_per_occ bytes per occupancy fits lds_limit (and, for the -inf
// sentinel block, at most kSentinel occupancies); false if none, or if the
// shape is not an exact one (K in 3..8, J <= 3 distinct sizes).
inline bool tile_shape(const Model& M, uint32_t bytes_per_occ, uint32_t lds_limit, TileShape* S) {
  if (M.K < 3 || M.K > 8 || M.J < 1 || M.J > 3 || M.n_sizes != M.J) return false;
  if (M.n_occ + kSentinel >= (int64_t{1} << 28)) return false;
  for (int T = (M.K - 1 < 4 ? M.K - 1 : 4); T >= 2; --T) {
    uint64_t occ = 1;
    for (int i = 0; i < T; ++i) occ *= static_cast<uint64_t>(M.R);
    if (occ * bytes_per_occ + 16 <= lds_limit && occ <= kSentinel) {
      S->occ = static_cast<uint32_t>(occ);
      S->n = static_cast<uint32_t>(static_cast<uint64_t>(M.n_occ) / occ);
      S->T = T;
      S->grid = S->n;
      return true;
    }
  }
  return false;
}

// The automatic choice takes the tile form only when every thread of a
// workgroup has an occupancy and there are enough tiles to fill the GPU.
inline bool tile_worthwhile(const TileShape& S) { return S.occ >= kBlock && S.n >= 256; }

// Form codes MDPVI_FORM_TILE + w, w = 1..8: w workgroups per CU walking
// their XCD's tiles (grid = w * CUs, rounded to a multiple of 8, at most
// one workgroup per tile); w = 0: one workgroup per tile.
inline void tile_set_walkers(TileShape* S, int w, int cus) {
  if (w <= 0) {
    S->grid = S->n;
    return;
  }
  uint32_t g = static_cast<uint32_t>(w) * static_cast<uint32_t>(cus);
  g = g / kNumXcd * kNumXcd;
  if (g < kNumXcd) g = kNumXcd;
  if (g >= S->n) g = S->n;   // one tile each (the direct order)
  S->grid = g;
}

template <int N>
using IC = std::integral_constant<int, N>;

// f(K, J, T) for the compiled (K, J, T): K 3..8, J 1..3, T 2..min(4, K-1).
template <typename F>
hipError_t tile_dispatch(int K, int J, int T, F&& f) {
  auto on_k = [&](auto kc) -> hipError_t {
    constexpr int Kc = decltype(kc)::value;
    auto on_j = [&](auto jc) -> hipError_t {
      if (T == 2) return f(kc, jc, IC<2>{});
      if constexpr (Kc >= 4) {
        if (T == 3) return f(kc, jc, IC<3>{});
      }
      if constexpr (Kc >= 5) {
        if (T == 4) return f(kc, jc, IC<4>{});
      }
      return hipErrorInvalidValue;
    };
    switch (J) {
      case 1: return on_j(IC<1>{});
      case 2: return on_j(IC<2>{});
      case 3: return on_j(IC<3>{});
      default: return hipErrorInvalidValue;
    }
  };
  switch (K) {
    case 3: return on_k(IC<3>{});
    case 4: return on_k(IC<4>{});
    case 5: return on_k(IC<5>{});
    case 6: return on_k(IC<6>{});
    case 7: return on_k(IC<7>{});
    case 8: return on_k(IC<8>{});
    default: return hipErrorInvalidValue;
  }
}

// High digits n_T..n_{K-1} of tile b (workgroup-uniform), and the tile's
// first occupancy.
template <int K, int T>
__device__ __forceinline__ uint32_t tile_high(const Model& M, uint32_t b, int (&nh)[K - T]) {
  uint32_t q = b;
#pragma unroll
  for (int k = 0; k < K - T; ++k) {
    const uint32_t q2 = fast_div(q, M.divR);
    nh[k] = static_cast<int>(q - q2 * static_cast<uint32_t>(M.R));
    q = q2;
  }
  return b * static_cast<uint32_t>(M.stride[T]);
}

// Low digits n_0..n_{T-1} of tile index i into n[0..T-1].
template <int T, int N>
__device__ __forceinline__ void tile_low(const Model& M, uint32_t i, int (&n)[N]) {
  static_assert(T <= N, "digit array too short");
#pragma unroll
  for (int k = 0; k < T; ++k) {
    const uint32_t q2 = fast_div(i, M.divR);
    n[k] = static_cast<int>(i - q2 * static_cast<uint32_t>(M.R));
    i = q2;
  }
}

}  // namespace mdpvi
