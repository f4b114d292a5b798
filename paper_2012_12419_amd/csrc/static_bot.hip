// static_bot.hip -- the fast greedy heuristic (Alg. 2) on a static set of
// bags of tasks, and the cloud-wide reward of a placement (Eqs. (14)-(16)
// summed: beta_vc per VM used in a VC, minus beta_tc per VM bought in the
// paid cloud, minus gamma_vc per VM left idle in a VC; the example of
// Sec. VII).
//
// One wavefront per scenario, one lane per vehicular cloud (K <= 64).  A
// task's VC is the lowest lane of the ballot "free >= need": the first VC in
// the cloud's order with room, found in one instruction instead of Alg. 2's
// scan.  Tasks are read 64 at a time (one coalesced load), broadcast from
// their lane with readlane, and their placements written back by the lane
// that read them.  The tasks of one scenario are placed in order (each
// depends on the VMs the earlier ones took); scenarios run in parallel.
#include "device.hpp"
#include "kernels.hpp"

namespace mdpvi {

namespace {

constexpr int kStaticWaves = 4;                   // scenarios per workgroup
constexpr int32_t kStaticMaxUnits = 1 << 30;      // largest capacity or task need
constexpr int32_t kPlacePaid = -1;
constexpr int32_t kPlaceEmpty = -2;

__device__ __forceinline__ long long wave_sum(long long v) {
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Reward of the totals, products rounded before the subtractions (no
// contraction), left to right.
__device__ __forceinline__ double cloud_reward(long long vc, long long paid, long long idle,
                                               double bvc, double btc, double gvc) {
  const double a = __dmul_rn(bvc, static_cast<double>(vc));
  const double b = __dmul_rn(btc, static_cast<double>(paid));
  const double c = __dmul_rn(gvc, static_cast<double>(idle));
  return __dsub_rn(__dsub_rn(a, b), c);
}

__device__ __forceinline__ void write_totals(long long b, long long vc, long long paid, long long idle,
                                             double bvc, double btc, double gvc,
                                             long long* totals, double* reward, int32_t* status) {
  totals[3 * b + 0] = vc;
  totals[3 * b + 1] = paid;
  totals[3 * b + 2] = idle;
  reward[b] = cloud_reward(vc, paid, idle, bvc, btc, gvc);
  status[b] = 0;
}

// 0, or 1 if a capacity of the scenario is out of [0, 2^30], or 2 if a task
// need is out of [0, 2^30] (checked before any output is written).
__device__ __forceinline__ int32_t check_inputs(int lane, int K, long long T, const int32_t* cb,
                                                const int32_t* nb) {
  const int32_t c = lane < K ? cb[lane] : 0;
  if (__ballot(c < 0 || c > kStaticMaxUnits)) return 1;
  for (long long t0 = 0; t0 < T; t0 += kWave) {
    const long long t = t0 + lane;
    const int32_t n = t < T ? nb[t] : 0;
    if (__ballot(n < 0 || n > kStaticMaxUnits)) return 2;
  }
  return 0;
}

__global__ __launch_bounds__(kWave* kStaticWaves) void static_first_fit_kernel(
    long long B, int K, long long T, const int32_t* __restrict__ caps, const int32_t* __restrict__ need,
    double bvc, double btc, double gvc, int32_t* __restrict__ place, int32_t* __restrict__ used,
    long long* __restrict__ totals, double* __restrict__ reward, int32_t* __restrict__ status) {
  const int lane = threadIdx.x % kWave;
  const long long b = static_cast<long long>(blockIdx.x) * kStaticWaves + threadIdx.x / kWave;
  if (b >= B) return;  // the whole wavefront leaves together
  const int32_t* cb = caps + b * K;
  const int32_t* nb = need + b * T;
  const int32_t bad = check_inputs(lane, K, T, cb, nb);
  if (bad) {
    if (lane == 0) status[b] = bad;
    return;
  }
  const int32_t cap = lane < K ? cb[lane] : 0;
  int32_t free = lane < K ? cap : -1;  // lanes past the last VC never have room
  long long paid = 0;                  // wavefront-uniform
  for (long long t0 = 0; t0 < T; t0 += kWave) {
    const long long t = t0 + lane;
    const int32_t mine = t < T ? nb[t] : 0;
    int32_t my_place = kPlaceEmpty;
    const int cnt = static_cast<int>(T - t0 < kWave ? T - t0 : kWave);
    for (int i = 0; i < cnt; ++i) {
      const int32_t n = __builtin_amdgcn_readlane(mine, i);
      if (n > 0) {
        const unsigned long long fits = __ballot(free >= n);
        int32_t where = kPlacePaid;
        if (fits) {
          where = static_cast<int32_t>(__builtin_ctzll(fits));
          if (lane == where) free -= n;
        } else {
          paid += n;
        }
        if (lane == i) my_place = where;
      }
    }
    if (t < T) place[b * T + t] = my_place;
  }
  const long long u = lane < K ? cap - free : 0;
  const long long f = lane < K ? free : 0;
  if (lane < K) used[b * K + lane] = static_cast<int32_t>(u);
  const long long vc = wave_sum(u), idle = wave_sum(f);
  if (lane == 0) write_totals(b, vc, paid, idle, bvc, btc, gvc, totals, reward, status);
}

// Score a given placement: place[t] = VC index, kPlacePaid, or anything for
// an empty slot (need 0).  Status 3: a VC over its capacity; 4: a place code
// out of [-1, K) on a task; nothing but the status is written then.
__global__ __launch_bounds__(kWave* kStaticWaves) void static_score_kernel(
    long long B, int K, long long T, const int32_t* __restrict__ caps, const int32_t* __restrict__ need,
    const int32_t* __restrict__ place, double bvc, double btc, double gvc, int32_t* __restrict__ used,
    long long* __restrict__ totals, double* __restrict__ reward, int32_t* __restrict__ status) {
  const int lane = threadIdx.x % kWave;
  const long long b = static_cast<long long>(blockIdx.x) * kStaticWaves + threadIdx.x / kWave;
  if (b >= B) return;
  const int32_t* cb = caps + b * K;
  const int32_t* nb = need + b * T;
  const int32_t* pb = place + b * T;
  int32_t bad = check_inputs(lane, K, T, cb, nb);
  if (bad) {
    if (lane == 0) status[b] = bad;
    return;
  }
  const int32_t cap = lane < K ? cb[lane] : 0;
  long long u = 0, paid = 0;
  bool range_bad = false;
  for (long long t0 = 0; t0 < T; t0 += kWave) {
    const long long t = t0 + lane;
    const int32_t n = t < T ? nb[t] : 0;
    const int32_t p = t < T && n > 0 ? pb[t] : kPlaceEmpty;
    range_bad = range_bad || (n > 0 && (p < kPlacePaid || p >= K));
    if (n > 0 && p == kPlacePaid) paid += n;
    const int cnt = static_cast<int>(T - t0 < kWave ? T - t0 : kWave);
    for (int i = 0; i < cnt; ++i) {
      const int32_t ni = __builtin_amdgcn_readlane(n, i);
      const int32_t pi = __builtin_amdgcn_readlane(p, i);
      if (ni > 0 && lane == pi) u += ni;
    }
  }
  paid = wave_sum(paid);
  if (__ballot(range_bad)) bad = 4;
  else if (__ballot(lane < K && u > cap)) bad = 3;
  if (bad) {
    if (lane == 0) status[b] = bad;
    return;
  }
  if (lane < K) used[b * K + lane] = static_cast<int32_t>(u);
  const long long vc = wave_sum(u), idle = wave_sum(lane < K ? cap - u : 0);
  if (lane == 0) write_totals(b, vc, paid, idle, bvc, btc, gvc, totals, reward, status);
}

dim3 static_grid(long long B) { return dim3(static_cast<uint32_t>((B + kStaticWaves - 1) / kStaticWaves)); }

}  // namespace

hipError_t launch_static_first_fit(long long B, int K, long long T, const int32_t* caps, const int32_t* need,
                                   double bvc, double btc, double gvc, int32_t* place, int32_t* used,
                                   long long* totals, double* reward, int32_t* status, hipStream_t s) {
  if (B == 0) return hipSuccess;
  hipLaunchKernelGGL(static_first_fit_kernel, static_grid(B), dim3(kWave * kStaticWaves), 0, s, B, K, T,
                     caps, need, bvc, btc, gvc, place, used, totals, reward, status);
  return hipGetLastError();
}

hipError_t launch_static_score(long long B, int K, long long T, const int32_t* caps, const int32_t* need,
                               const int32_t* place, double bvc, double btc, double gvc, int32_t* used,
                               long long* totals, double* reward, int32_t* status, hipStream_t s) {
  if (B == 0) return hipSuccess;
  hipLaunchKernelGGL(static_score_kernel, static_grid(B), dim3(kWave * kStaticWaves), 0, s, B, K, T,
                     caps, need, place, bvc, btc, gvc, used, totals, reward, status);
  return hipGetLastError();
}

}  // namespace mdpvi
