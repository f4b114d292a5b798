// row.hpp -- shared pieces of the row form of the tile sweeps (row_vi.hip,
// row_eval.hip): 16-byte buffer loads and stores, the FP64 max without
// canonicalisation, the geometry of a tile's rows and chunks, and the
// dispatch over the compiled shapes.
//
// A tile holds the R^3 occupancies (R = C + 1) that share the high digits
// n_3..n_{K-1}.  It is staged in LDS row by row along digit 0, each row
// padded to a multiple of P slots; a lane owns a chunk of P consecutive
// occupancies of one row, so its digits are fixed by its row and chunk and
// every neighbour along a high digit is a 16-byte load at the lane's offset
// plus a workgroup-uniform one.
#pragma once

#include "tile.hpp"

namespace mdpvi {

typedef unsigned int U32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int U32x3 __attribute__((ext_vector_type(3)));
typedef unsigned int U32x2v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ void ld4f(BufView v, uint32_t lo, uint32_t uo, float (&x)[4]) {
  const U32x4 r = __builtin_amdgcn_raw_buffer_load_b128(v.r, lo, uo, 0);
  x[0] = __uint_as_float(r.x);
  x[1] = __uint_as_float(r.y);
  x[2] = __uint_as_float(r.z);
  x[3] = __uint_as_float(r.w);
}

// Three values (the last chunk of the last row of an array), the fourth 0.
__device__ __forceinline__ void ld3f(BufView v, uint32_t lo, uint32_t uo, float (&x)[4]) {
  const U32x3 r = __builtin_amdgcn_raw_buffer_load_b96(v.r, lo, uo, 0);
  x[0] = __uint_as_float(r.x);
  x[1] = __uint_as_float(r.y);
  x[2] = __uint_as_float(r.z);
  x[3] = 0.0f;
}

__device__ __forceinline__ double u2d(unsigned int lo, unsigned int hi) {
  return __builtin_bit_cast(double, (static_cast<unsigned long long>(hi) << 32) | lo);
}

__device__ __forceinline__ void ld4d(BufView v, uint32_t lo, uint32_t uo, double (&x)[4]) {
  const U32x4 a = __builtin_amdgcn_raw_buffer_load_b128(v.r, lo, uo, 0);
  const U32x4 b = __builtin_amdgcn_raw_buffer_load_b128(v.r, lo + 16u, uo, 0);
  x[0] = u2d(a.x, a.y);
  x[1] = u2d(a.z, a.w);
  x[2] = u2d(b.x, b.y);
  x[3] = u2d(b.z, b.w);
}

__device__ __forceinline__ unsigned int lo32(double d) {
  return static_cast<unsigned int>(__builtin_bit_cast(unsigned long long, d));
}
__device__ __forceinline__ unsigned int hi32(double d) {
  return static_cast<unsigned int>(__builtin_bit_cast(unsigned long long, d) >> 32);
}

// The larger of two FP64 numbers (v_max_f64 without the canonicalisation
// the compiler adds for fmax: no operand is ever a signalling NaN).
__device__ __forceinline__ double max_f64(double a, double b) {
  double r;
  asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

// Waves per SIMD the register budget of the row kernels must allow.
#ifndef MDPVI_ROW_WAVES
#define MDPVI_ROW_WAVES 1
#endif

// Geometry of the row form for radix R and P occupancies per lane.
template <int R, int P>
struct RowGeo {
  static constexpr int RP = (R + P - 1) / P * P;       // LDS value slots per row
  static constexpr int RPA = (R + 3 + 1) / 2 * 2;      // LDS arrival slots per row: R, then >= 3 of -inf
  static constexpr int NC = RP / P;                    // chunks per row
  static constexpr int ROWS = R * R;                   // rows of a tile (digits 1 and 2)
  static constexpr int OCC = R * R * R;                // occupancies of a tile
  static constexpr int LANES = ROWS * NC;              // lanes with a chunk
  static constexpr int BLOCK = (LANES + kWave - 1) / kWave * kWave;
  static constexpr int TAIL = R - (NC - 1) * P;        // occupancies of a row's last chunk (1..P)
  static constexpr int MAXS = 3;                       // largest task size the padding covers
};

// Radixes and host counts with a compiled row form.
template <typename F>
hipError_t row_dispatch(int K, int J, int R, F&& f) {
  auto on_r = [&](auto rc) -> hipError_t {
    auto on_j = [&](auto jc) -> hipError_t {
      switch (K) {
        case 5: return f(IC<5>{}, jc, rc);
        case 6: return f(IC<6>{}, jc, rc);
        case 7: return f(IC<7>{}, jc, rc);
        default: return hipErrorInvalidValue;
      }
    };
    switch (J) {
      case 1: return on_j(IC<1>{});
      case 2: return on_j(IC<2>{});
      case 3: return on_j(IC<3>{});
      default: return hipErrorInvalidValue;
    }
  };
  switch (R) {
    case 11: return on_r(IC<11>{});
    default: return hipErrorInvalidValue;
  }
}

}  // namespace mdpvi
