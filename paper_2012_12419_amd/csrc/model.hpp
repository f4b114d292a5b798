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
constexpr int kResLanes = 64;   // words of a 1-norm residual: workgroup b adds into word b % 64
constexpr int kResStride = 16;  // 64-bit words per 128-byte line (batched control blocks)
constexpr int kSumStride = 544; // doubles between 1-norm words (17 x 256 bytes: distinct channels)

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
  double hold;                  // under-utilisation penalty per free unit and step
  double gamma;
  // raw parameters, for the gradient with respect to them
  double lam[kMaxJ];            // lambda_j
  double reward[kMaxJ];         // r_j
  double cost[kMaxJ];           // c_j (paid-cloud cost)
  double c_obj[kMaxJ];          // lambda_j / sum lambda: weights of the empty states in J
  double mu, nu, Lam, lam_tot;
};

// Control words of one iterative solve, in device memory (copied to the host
// once per chunk of sweeps).
//   done_iter: -1 while running; else the index k of the first iterate V^k
//              whose residual ||V^k - V^{k-1}|| passed the test (or was NaN).
//   flag:      set by validation kernels (an infeasible policy entry).
//   go[r][x]:  the sweep with index j (r = j mod kResSlots) failed the test in
//              some workgroup b with b mod 8 = x: that workgroup's largest
//              |V' - V| is not below tol.  Workgroups raise it with a plain
//              store only after reading it still clear, so a word sees a few
//              stores per sweep instead of one per workgroup (stores to one
//              address from thousands of workgroups serialise in the memory
//              system).  Workgroups b and b + 8 normally share an XCD and
//              hence its L2.  The sweep converged iff every go[r][x] is clear.
//   nan[r][x]: likewise for a NaN.  Every word sits on its own 128-byte line.
// The residual values themselves live in a separate buffer.
struct Ctl {
  long long done_iter;
  long long flag;
  long long pad[14];
  unsigned int go[kResSlots][kNumXcd][32];
  unsigned int nan[kResSlots][kNumXcd][32];
};

// Layout of the residual buffer of one solve:
//   max-norm sweeps: res[r * grid + b] = largest |V' - V| of workgroup b in
//                    the sweep of ring slot r (plain stores, no atomics);
//   1-norm sweeps:   res[(r * kResLanes + l) * kSumStride] = sum of the
//                    workgroups b with b % kResLanes = l (FP64 atomicAdd; the
//                    words are kSumStride doubles apart so that concurrent
//                    atomics from different workgroups reach different memory
//                    channels instead of queueing on one).
__host__ __device__ inline size_t sum_word(long long j, int lane) {
  return (static_cast<size_t>(j % kResSlots) * kResLanes + lane) * kSumStride;
}
__host__ __device__ inline size_t res_doubles(uint32_t grid) {
  const size_t a = static_cast<size_t>(kResSlots) * grid;
  const size_t b = static_cast<size_t>(kResSlots) * kResLanes * kSumStride;
  return a > b ? a : b;
}

}  // namespace mdpvi
