// model.hpp -- device-side description of one occupancy MDP instance and the
// small host/device helpers shared by every kernel.
//
// The model is the uniformised occupancy chain of paper Sec. V-B..V-E with
// the Bellman backup of Eq. (18); the public header mdpvi.h states it in
// full.  Everything a kernel needs is folded into one trivially-copyable
// struct passed by value as a kernel argument (about 0.5 KB), so no device
// parameter block has to be allocated or kept coherent.
#pragma once

#include <stdint.h>

#include <hip/hip_runtime.h>

namespace mdpvi {

constexpr int kBlock = 256;       // threads of a sweep workgroup: 4 wavefronts of 64
constexpr int kWave = 64;
constexpr int kNumXcd = 8;        // MI355X: 8 accelerator complex dies, 32 CUs each
constexpr int kOccPerThread = 4;  // occupancies per thread in the sweep kernels
constexpr int kMaxK = 16;
constexpr int kMaxJ = 8;
constexpr int kResSlots = 4;    // ring of per-sweep residuals
constexpr int kResLanes = 64;   // words per residual: workgroup b reduces into word b % 64
constexpr int kResStride = 16;  // one word per 128-byte line (64-bit words)

// Unsigned 32-bit division by a run-time constant d >= 2 with one high
// multiply, a subtract, an add and two shifts (Granlund & Montgomery, "Division
// by invariant integers using multiplication", PLDI 1994, the round-up
// variant with a 33-bit multiplier split as m + 2^32).
struct FastDiv {
  uint32_t d;
  uint32_t m;
  uint32_t s;
};

__host__ __device__ inline uint32_t mulhi_u32(uint32_t a, uint32_t b) {
  return static_cast<uint32_t>((static_cast<uint64_t>(a) * b) >> 32);
}

__host__ __device__ inline uint32_t fast_div(uint32_t n, FastDiv f) {
  uint32_t t = mulhi_u32(n, f.m);
  return (t + ((n - t) >> 1)) >> f.s;
}

inline FastDiv make_fast_div(uint32_t d) {
  // l = ceil(log2 d), m = floor(2^32 (2^l - d) / d) + 1, shift = l - 1
  uint32_t l = 0;
  while ((uint64_t{1} << l) < d) ++l;
  uint64_t m = ((uint64_t{1} << 32) * ((uint64_t{1} << l) - d)) / d + 1;
  return FastDiv{d, static_cast<uint32_t>(m), l - 1};
}

// One MDP instance as the kernels see it.  Probabilities are pre-divided by
// the uniformisation rate Lam; rewards are pre-multiplied by P_arr.
struct Model {
  int32_t K;           // hosts
  int32_t C;           // units per host
  int32_t J;           // task classes
  int32_t R;           // radix C + 1
  int32_t KC;          // K * C
  int32_t n_sizes;     // distinct task sizes
  int64_t n_occ;       // (C+1)^K occupancy vectors
  int64_t n_states;    // J (C+1)^K
  int64_t stride[kMaxK];        // (C+1)^k
  FastDiv divR;                 // division by R (32-bit indices only)
  int32_t size[kMaxJ];          // units of a class-j task
  int32_t size_u[kMaxJ];        // the distinct sizes
  int32_t size_idx[kMaxJ];      // class -> position in size_u
  double p[kMaxJ];              // lambda_j / Lam
  double mu_L;                  // mu / Lam
  double nu_L;                  // nu / Lam
  double r_place[kMaxJ];        // P_arr * reward_j
  double r_reject[kMaxJ];       // -P_arr * reject_cost_j
  double gamma;
  // raw parameters, for the gradient with respect to them
  double lam[kMaxJ];            // lambda_j
  double reward[kMaxJ];         // r_j
  double cost[kMaxJ];           // c_j (paid-cloud cost)
  double c_obj[kMaxJ];          // lambda_j / sum lambda: weights of the empty states in J
  double mu, nu, Lam, lam_tot;
};

// Control words of one iterative solve, in device memory.
//   done_iter: -1 while running; else the index k of the first iterate V^k
//              whose residual ||V^k - V^{k-1}|| passed the test (or was NaN).
//   flag:      set by validation kernels (an infeasible policy entry).
//   res:       the residual of the sweep with index j lives in ring slot
//              r = j mod kResSlots as kResLanes partial words, one per
//              128-byte line so that concurrent atomics from different
//              workgroups do not queue on one address; the residual is the
//              max (or, for 1-norm residuals, the sum) of the lanes.  A word
//              holds the bit pattern of a non-negative double: such doubles
//              order like their bit patterns, so atomicMax on the bits is a
//              max, and NaN patterns order above +inf.
struct Ctl {
  long long done_iter;
  long long flag;
  long long pad[kResStride - 2];
  unsigned long long res[kResSlots][kResLanes][kResStride];
};

__host__ __device__ inline unsigned long long* res_word(Ctl* c, long long j, int lane) {
  return &c->res[j % kResSlots][lane][0];
}

}  // namespace mdpvi
