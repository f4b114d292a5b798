// kernels.hpp -- host-side launchers of the HIP kernels (internal to the
// library; the public surface is the C ABI in mdpvi.h).
#pragma once

#include "model.hpp"

namespace mdpvi {

// 32-bit index arithmetic is used while every state index and every
// neighbour offset fits in 31 bits.
inline bool use_32bit_index(const Model& M) { return M.n_states < (int64_t{1} << 31); }

hipError_t launch_ctl_init(Ctl* ctl, hipStream_t s);

// V^{j+1} = T V^j (Vin -> Vout), residual into ctl->res[j % kResSlots];
// a no-op once the stopping test has passed.
hipError_t launch_vi_sweep(const Model& M, const float* Vin, float* Vout, Ctl* ctl, long long j,
                           double tol, hipStream_t s);

// Greedy extraction from FP32 or FP64 values.
hipError_t launch_extract_f32(const Model& M, const float* V, uint8_t* pi, float* gap,
                              hipStream_t s);
hipError_t launch_extract_f64(const Model& M, const double* V, uint8_t* pi, float* gap,
                              hipStream_t s);

// ctl->flag := 1 if some pi entry is not a feasible action.
hipError_t launch_policy_check(const Model& M, const uint8_t* pi, Ctl* ctl, hipStream_t s);

// One fixed-policy FP64 sweep V^{j+1} = r_pi + gamma P_pi V^j.
hipError_t launch_eval_sweep(const Model& M, const uint8_t* pi, const double* Vin, double* Vout,
                             Ctl* ctl, long long j, double tol, hipStream_t s);

// Greedy heuristic policies (0 least-loaded, 1 first-fit).
hipError_t launch_greedy(const Model& M, int kind, uint8_t* pi, hipStream_t s);

}  // namespace mdpvi
