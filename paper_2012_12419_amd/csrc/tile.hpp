// tile.hpp -- the tile form of the exact-shape sweeps (value iteration and
// fixed-policy evaluation).
//
// A tile is the set of (C+1)^T occupancies that share the high digits
// n_T..n_{K-1}; one workgroup per tile, in a host-computed order that gives
// each XCD a compact block of tiles (or, for sweeps beyond the last-level
// cache, keeps all XCDs on one region).  The workgroup stages its tile's
// values (all classes; value iteration also its FP64 arrival terms) in LDS;
// then every neighbour
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

#include <algorithm>
#include <functional>
#include <type_traits>
#include <vector>

namespace mdpvi {

// Entries of -inf after the n_occ arrival terms of each value-iteration
// arrival array: a placement without room along a high digit reads entry
// n_occ + i (i < tile size <= kSentinel).
constexpr uint32_t kSentinel = 4096;
// Threads of a tile workgroup and the waves per SIMD the register budget of
// the tile kernels must allow (the compiler caps VGPRs at 512 / that).
#ifndef MDPVI_TILE_BLOCK
#define MDPVI_TILE_BLOCK 256
#endif
#ifndef MDPVI_TILE_MIN_WAVES
#define MDPVI_TILE_MIN_WAVES 1
#endif
constexpr int kTileBlock = MDPVI_TILE_BLOCK;
constexpr int kTileMinWaves = MDPVI_TILE_MIN_WAVES;
// LDS bytes a tile image may take (the block-asynchronous form holds two).
constexpr uint32_t kTileLds = 48 * 1024;
constexpr uint32_t kBsdiLds = 64 * 1024;

struct TileShape {
  uint32_t occ;    // (C+1)^T occupancies per tile
  uint32_t n;      // (C+1)^(K-T) tiles
  int32_t T;       // low digits of a tile
  uint32_t grid;   // workgroups launched: n (one tile each), or a multiple of 8
                   // that walk the tiles of their XCD's range in order
  const uint32_t* order;   // device [n]: the tiles of XCD 0, then of XCD 1, ...
                           // (tile_partition); nullptr: index order
};

// Positions of workgroup blockIdx.x in the tile order.  Workgroups are
// handed to the 8 XCDs round-robin by their id, so XCD x runs the
// workgroups b = x (mod 8): with one workgroup per tile it runs
// count_x = ceil((n - x) / 8) of them, and owns positions [start_x,
// start_x + count_x) of the order; its walkers (grid < n) take those
// positions in turn, so that the tiles in flight on an XCD stay close.
// Without an order table the positions are tile indices (contiguous ranges
// per XCD, as in the direct form).
struct TileWalk {
  uint32_t first, end, step;
};

__host__ __device__ inline uint32_t tile_xcd_count(uint32_t n, uint32_t x) {
  return (n + kNumXcd - 1 - x) / kNumXcd;
}

__host__ __device__ inline uint32_t tile_xcd_start(uint32_t n, uint32_t x) {
  const uint32_t rem = n % kNumXcd;
  return x * (n / kNumXcd) + (x < rem ? x : rem);
}

__device__ __forceinline__ TileWalk tile_walk(const TileShape& S) {
  const uint32_t x = blockIdx.x % kNumXcd;
  const uint32_t w = blockIdx.x / kNumXcd;
  if (S.order) {
    const uint32_t lo = tile_xcd_start(S.n, x);
    if (S.grid == S.n) return TileWalk{lo + w, lo + w + 1, 1};
    return TileWalk{lo + w, lo + tile_xcd_count(S.n, x), gridDim.x / kNumXcd};
  }
  if (S.grid == S.n) {
    const uint32_t t = xcd_block(blockIdx.x, gridDim.x);
    return TileWalk{t, t + 1, 1};
  }
  const uint32_t lo = static_cast<uint32_t>(static_cast<uint64_t>(S.n) * x / kNumXcd);
  const uint32_t hi = static_cast<uint32_t>(static_cast<uint64_t>(S.n) * (x + 1) / kNumXcd);
  return TileWalk{lo + w, hi, gridDim.x / kNumXcd};
}

// The tile at walk position p (a workgroup-uniform scalar load).
__device__ __forceinline__ uint32_t tile_at(const TileShape& S, uint32_t p) {
  return S.order ? S.order[p] : p;
}

// Host: the tile order of a shape.  The n tiles are points of the
// (C+1)^(K-T) grid of high digits; recursive coordinate bisection splits
// them into 8 parts of count_x tiles, each split cutting the current set
// across its widest digit (the higher digit on ties) at the rank that gives
// each side its count, ties on that digit broken by tile index.  Every XCD
// then owns a compact block of tiles instead of a slab one or two values
// thick along the top digit: the neighbours it fetches from other XCDs'
// tiles (the halo of release, reset and placement reads along the high
// digits) shrink with the block's surface.  Within a part, tiles keep index
// order.
inline void tile_partition(int K, int R, const TileShape& S, std::vector<uint32_t>* order) {
  const int H = K - S.T;
  const uint32_t n = S.n;
  std::vector<uint32_t> ids(n);
  for (uint32_t i = 0; i < n; ++i) ids[i] = i;
  std::vector<uint32_t> pw(H);
  for (int h = 0; h < H; ++h) pw[h] = h == 0 ? 1u : pw[h - 1] * static_cast<uint32_t>(R);
  auto digit = [&](uint32_t t, int h) { return static_cast<int>((t / pw[h]) % static_cast<uint32_t>(R)); };
  order->assign(n, 0u);
  // split ids[lo, hi) among XCDs [x0, x1)
  std::function<void(uint32_t, uint32_t, int, int)> split = [&](uint32_t lo, uint32_t hi, int x0, int x1) {
    if (x1 - x0 == 1) {
      std::sort(ids.begin() + lo, ids.begin() + hi);
      std::copy(ids.begin() + lo, ids.begin() + hi, order->begin() + tile_xcd_start(n, x0));
      return;
    }
    const int xm = (x0 + x1) / 2;
    uint32_t left = 0;
    for (int x = x0; x < xm; ++x) left += tile_xcd_count(n, static_cast<uint32_t>(x));
    int axis = H - 1, widest = -1;
    for (int h = H - 1; h >= 0; --h) {
      int mn = R, mx = -1;
      for (uint32_t i = lo; i < hi; ++i) {
        const int d = digit(ids[i], h);
        mn = d < mn ? d : mn;
        mx = d > mx ? d : mx;
      }
      if (mx - mn > widest) {
        widest = mx - mn;
        axis = h;
      }
    }
    std::sort(ids.begin() + lo, ids.begin() + hi, [&](uint32_t a, uint32_t b) {
      const int da = digit(a, axis), db = digit(b, axis);
      return da != db ? da < db : a < b;
    });
    split(lo, lo + left, x0, xm);
    split(lo + left, hi, xm, x1);
  };
  split(0, n, 0, kNumXcd);
}

// The deepest tile (T in 2..min(4, K-1)) whose LDS footprint of
// bytes_per_occ bytes per occupancy fits lds_limit (and, for the -inf
// sentinel block, at most kSentinel occupancies); false if none, if the
// shape is not an exact one (K in 3..8, J <= 3 distinct sizes), or if the
// value array reaches 2 GiB (2^29 FP32 states).
inline bool tile_shape(const Model& M, uint32_t bytes_per_occ, uint32_t lds_limit, TileShape* S) {
  if (M.K < 3 || M.K > 8 || M.J < 1 || M.J > 3 || M.n_sizes != M.J) return false;
  // buffer views hold byte offsets below 2^31: the FP32 values (n_states
  // words) and the FP64 arrival terms with their sentinel block
  if (M.n_states >= (int64_t{1} << 29) || M.n_occ + kSentinel >= (int64_t{1} << 28)) return false;
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

// Stages a tile's values (J classes of TV, class c at byte offset
// o0 * sizeof(TV) + c * cls) and arrival terms into Vl [J][occ] and Al [occ]
// with NB threads.  Loads are issued in batches of kStageRounds rounds per
// thread before the first LDS write, so that a thread waits for one round
// trip per batch instead of one per round; lanes past the tile load the last
// occupancy again (in bounds) and write nothing.
constexpr int kStageRounds = 8;

template <int J, int NB, typename TV>
__device__ __forceinline__ void stage_tile(uint32_t occ, uint32_t o0, uint32_t cls, BufView vin, BufView ain,
                                           TV* Vl, double* Al) {
  constexpr uint32_t tv = sizeof(TV);
  for (uint32_t base = 0; base < occ; base += kStageRounds * NB) {
    TV v[kStageRounds][J];
    double a[kStageRounds];
#pragma unroll
    for (int r = 0; r < kStageRounds; ++r) {
      uint32_t i = base + r * NB + threadIdx.x;
      i = i < occ ? i : occ - 1;
#pragma unroll
      for (int e = 0; e < J; ++e) {
        if constexpr (tv == 4)
          v[r][e] = ld_f32(vin, i * 4u, o0 * 4u + e * cls);
        else
          v[r][e] = ld_f64(vin, i * 8u, o0 * 8u + e * cls);
      }
      a[r] = ld_f64(ain, i * 8u, o0 * 8u);
    }
#pragma unroll
    for (int r = 0; r < kStageRounds; ++r) {
      const uint32_t i = base + r * NB + threadIdx.x;
      if (i < occ) {
#pragma unroll
        for (int e = 0; e < J; ++e) Vl[e * occ + i] = v[r][e];
        Al[i] = a[r];
      }
    }
  }
}

// Stages only the tile's values (FP64, J classes) into Vl [J][occ], in the
// batches of stage_tile.
template <int J, int NB>
__device__ __forceinline__ void stage_values(uint32_t occ, uint32_t o0, uint32_t cls, BufView vin, double* Vl) {
  for (uint32_t base = 0; base < occ; base += kStageRounds * NB) {
    double v[kStageRounds][J];
#pragma unroll
    for (int r = 0; r < kStageRounds; ++r) {
      uint32_t i = base + r * NB + threadIdx.x;
      i = i < occ ? i : occ - 1;
#pragma unroll
      for (int e = 0; e < J; ++e) v[r][e] = ld_f64(vin, i * 8u, o0 * 8u + e * cls);
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

// Host: runs of `run` consecutive tiles dealt to the XCDs in turn (an XCD
// whose share is full passes its run to the next), so that all XCDs sweep
// the same region of the grid at the same time: for sweeps whose working set
// exceeds the last-level cache, the neighbour planes of that region are then
// read from it by every XCD instead of from HBM.
inline void tile_deal(const TileShape& S, uint32_t run, std::vector<uint32_t>* order) {
  const uint32_t n = S.n;
  std::vector<uint32_t> fill(kNumXcd, 0u);
  order->assign(n, 0u);
  for (uint32_t t = 0; t < n; ++t) {
    uint32_t x = (t / run) % kNumXcd;
    while (fill[x] == tile_xcd_count(n, x)) x = (x + 1) % kNumXcd;
    (*order)[tile_xcd_start(n, x) + fill[x]++] = t;
  }
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

// Workgroup-uniform data of one tile: its first occupancy, its high digits
// and the byte offsets (relative to the tile base, in the scalar operand of a
// buffer load) of its high-digit neighbours.
template <int K, int J, int T>
struct TileHigh {
  uint32_t o0;
  int nh[K - T];
  int load_high;
  uint32_t hd4[K - T];      // release neighbour (the tile itself when n_k = 0: weight 0)
  uint32_t hr4[K - T];      // reset neighbour
  uint32_t ha8[K - T][J];   // placement, or the -inf sentinel block
};

template <int K, int J, int T>
__device__ __forceinline__ void tile_high_setup(const Model& M, uint32_t tb, TileHigh<K, J, T>& H) {
  constexpr int NH = K - T;
  const uint32_t nocc = static_cast<uint32_t>(M.n_occ);
  H.o0 = tile_high<K, T>(M, tb, H.nh);
  H.load_high = 0;
#pragma unroll
  for (int h = 0; h < NH; ++h) {
    const uint32_t st = static_cast<uint32_t>(M.stride[T + h]);
    H.hd4[h] = (H.nh[h] > 0 ? H.o0 - st : H.o0) * 4u;
    H.hr4[h] = (H.o0 - static_cast<uint32_t>(H.nh[h]) * st) * 4u;
#pragma unroll
    for (int e = 0; e < J; ++e) {
      const int s = M.size[e];
      H.ha8[h][e] = H.nh[h] + s <= M.C ? (H.o0 + static_cast<uint32_t>(s) * st) * 8u : nocc * 8u;
    }
    H.load_high += H.nh[h];
  }
}

}  // namespace mdpvi
