// api.hip -- the C ABI declared in include/mdpvi.h: parameter validation,
// handle and scratch ownership, and the host side of the sweep loops.
//
// The sweep loop (Alg. 3 steps 2-3) runs on the device without per-sweep
// host synchronisation: sweeps are enqueued in chunks, each sweep first checks
// on the device whether an earlier sweep already met the stopping test (and
// then does nothing), and the host reads the control words once per chunk.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "../../include/mdpvi.h"
#include "kernels.hpp"
#include "model.hpp"

using mdpvi::Ctl;
using mdpvi::Model;

struct mdpvi_mdp {
  Model M;
  int64_t feasible_pairs = 0;
  int device = -1;              // device of the scratch below (-1: none yet)
  void* vbuf = nullptr;         // second value buffer (ping-pong partner)
  size_t vbuf_bytes = 0;
  Ctl* ctl = nullptr;           // device control words
  Ctl* ctl_host = nullptr;      // pinned mirror
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int fail_hip(hipError_t e, const char* what) {
  return fail(MDPVI_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr)                                          \
  do {                                                         \
    hipError_t _e = (expr);                                    \
    if (_e != hipSuccess) return fail_hip(_e, #expr);          \
  } while (0)

bool is_finite(double x) { return std::isfinite(x); }

// Device scratch of a handle: control words, pinned mirror, events and a
// ping-pong partner of at least `bytes`.  Bound to the device current at
// first use.
int ensure_scratch(mdpvi_mdp* h, size_t bytes) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (h->device >= 0 && h->device != dev)
    return fail(MDPVI_EINVAL, "handle scratch lives on device %d, current device is %d", h->device,
                dev);
  if (!h->ctl) {
    if (hipMalloc(&h->ctl, sizeof(Ctl)) != hipSuccess) {
      h->ctl = nullptr;
      return fail(MDPVI_ENOMEM, "hipMalloc of %zu control bytes failed", sizeof(Ctl));
    }
    if (hipHostMalloc(reinterpret_cast<void**>(&h->ctl_host), sizeof(Ctl), hipHostMallocDefault) !=
        hipSuccess) {
      h->ctl_host = nullptr;
      return fail(MDPVI_ENOMEM, "hipHostMalloc of the control mirror failed");
    }
    HIP_TRY(hipEventCreate(&h->ev0));
    HIP_TRY(hipEventCreate(&h->ev1));
    h->device = dev;
  }
  if (bytes > h->vbuf_bytes) {
    if (h->vbuf) {
      HIP_TRY(hipDeviceSynchronize());
      HIP_TRY(hipFree(h->vbuf));
      h->vbuf = nullptr;
      h->vbuf_bytes = 0;
    }
    if (hipMalloc(&h->vbuf, bytes) != hipSuccess) {
      h->vbuf = nullptr;
      return fail(MDPVI_ENOMEM, "hipMalloc of a %zu-byte value buffer failed", bytes);
    }
    h->vbuf_bytes = bytes;
  }
  return MDPVI_OK;
}

double bits_to_double(unsigned long long b) {
  double d;
  std::memcpy(&d, &b, sizeof d);
  return d;
}

// Enqueue sweeps j = 0, 1, ... in chunks until the device reports the test
// met or max_iter sweeps were issued; leaves the final iterate in buf0.
// `sweep(j, in, out)` enqueues sweep j.
template <typename T, typename Sweep>
int run_loop(mdpvi_mdp* h, T* buf0, double tol, int64_t max_iter, hipStream_t s,
             mdpvi_stats* st, double bytes_per_sweep, double backups_per_sweep, Sweep sweep) {
  T* buf[2] = {buf0, static_cast<T*>(h->vbuf)};
  HIP_TRY(mdpvi::launch_ctl_init(h->ctl, s));
  HIP_TRY(hipEventRecord(h->ev0, s));
  int64_t issued = 0;
  int64_t chunk = 8;
  long long done = -1;
  while (issued < max_iter) {
    const int64_t n = std::min<int64_t>(chunk, max_iter - issued);
    for (int64_t i = 0; i < n; ++i) {
      const int64_t j = issued + i;
      HIP_TRY(sweep(static_cast<long long>(j), buf[j & 1], buf[(j + 1) & 1]));
    }
    issued += n;
    HIP_TRY(hipMemcpyAsync(h->ctl_host, h->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    done = h->ctl_host->done_iter;
    if (done >= 0) break;
    if (chunk < 256) chunk *= 2;
  }
  int64_t final_iter;
  double res;
  bool converged;
  if (done >= 0) {
    final_iter = done;
    res = bits_to_double(h->ctl_host->res[(final_iter - 1) % mdpvi::kResSlots]);
    converged = res < tol;
  } else {
    final_iter = issued;
    res = bits_to_double(h->ctl_host->res[(final_iter - 1) % mdpvi::kResSlots]);
    converged = res < tol;
  }
  if (final_iter & 1) {
    HIP_TRY(hipMemcpyAsync(buf0, buf[1], static_cast<size_t>(h->M.n_states) * sizeof(T),
                           hipMemcpyDeviceToDevice, s));
  }
  HIP_TRY(hipEventRecord(h->ev1, s));
  HIP_TRY(hipEventSynchronize(h->ev1));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, h->ev0, h->ev1));
  if (st) {
    st->iterations = final_iter;
    st->residual_inf = res;
    st->bound_inf = h->M.gamma / (1.0 - h->M.gamma) * res;
    st->seconds = ms * 1e-3;
    st->backups = backups_per_sweep * static_cast<double>(final_iter);
    st->bytes = bytes_per_sweep * static_cast<double>(final_iter);
  }
  if (std::isnan(res) || std::isinf(res))
    return fail(MDPVI_ENAN, "non-finite residual after %lld sweeps", (long long)final_iter);
  if (!converged)
    return fail(MDPVI_ENOCONV, "residual %.3e >= tol %.3e after %lld sweeps (max_iter)", res, tol,
                (long long)final_iter);
  return MDPVI_OK;
}

}  // namespace

extern "C" {

const char* mdpvi_last_error(void) { return g_err.c_str(); }

int mdp_build(const mdpvi_params* p, mdpvi_mdp_t* out) {
  if (!p || !out) return fail(MDPVI_EINVAL, "NULL argument");
  *out = nullptr;
  if (p->K < 1 || p->K > MDPVI_MAX_K) return fail(MDPVI_EINVAL, "K=%d outside [1, %d]", p->K, MDPVI_MAX_K);
  if (p->J < 1 || p->J > MDPVI_MAX_J) return fail(MDPVI_EINVAL, "J=%d outside [1, %d]", p->J, MDPVI_MAX_J);
  if (p->C < 1) return fail(MDPVI_EINVAL, "C=%d must be >= 1", p->C);
  if (!p->size || !p->lambda || !p->reward) return fail(MDPVI_EINVAL, "NULL size/lambda/reward");
  if (!(p->gamma >= 0.0 && p->gamma < 1.0)) return fail(MDPVI_EINVAL, "gamma=%g outside [0, 1)", p->gamma);
  if (!is_finite(p->mu) || p->mu < 0) return fail(MDPVI_EINVAL, "mu=%g must be finite and >= 0", p->mu);
  if (!is_finite(p->nu) || p->nu < 0) return fail(MDPVI_EINVAL, "nu=%g must be finite and >= 0", p->nu);
  double lam_tot = 0.0;
  for (int j = 0; j < p->J; ++j) {
    if (p->size[j] < 1 || p->size[j] > p->C)
      return fail(MDPVI_EINVAL, "size[%d]=%d outside [1, C=%d]", j, p->size[j], p->C);
    if (!is_finite(p->lambda[j]) || p->lambda[j] < 0)
      return fail(MDPVI_EINVAL, "lambda[%d]=%g must be finite and >= 0", j, p->lambda[j]);
    if (!is_finite(p->reward[j])) return fail(MDPVI_EINVAL, "reward[%d] is not finite", j);
    if (p->reject_cost && !is_finite(p->reject_cost[j]))
      return fail(MDPVI_EINVAL, "reject_cost[%d] is not finite", j);
    lam_tot += p->lambda[j];
  }
  if (!(lam_tot > 0)) return fail(MDPVI_EINVAL, "sum of lambda must be > 0");
  // N = J (C+1)^K, refused above 2^62; every occupancy index must fit the
  // 32-bit thread grid of one launch.
  const double logN = std::log2(static_cast<double>(p->J)) + p->K * std::log2(p->C + 1.0);
  if (logN > 62.0) return fail(MDPVI_ERANGE, "J (C+1)^K = 2^%.1f states exceeds 2^62", logN);
  int64_t n_occ = 1;
  for (int k = 0; k < p->K; ++k) n_occ *= (p->C + 1);
  if (n_occ > (int64_t{1} << 32) - 1024)
    return fail(MDPVI_ERANGE, "(C+1)^K = %lld occupancies exceed one launch grid",
                (long long)n_occ);

  mdpvi_mdp* h = new (std::nothrow) mdpvi_mdp();
  if (!h) return fail(MDPVI_ENOMEM, "host allocation failed");
  Model& M = h->M;
  std::memset(&M, 0, sizeof M);
  M.K = p->K;
  M.C = p->C;
  M.J = p->J;
  M.R = p->C + 1;
  M.KC = p->K * p->C;
  M.n_occ = n_occ;
  M.n_states = n_occ * p->J;
  int64_t st = 1;
  for (int k = 0; k < p->K; ++k) {
    M.stride[k] = st;
    st *= M.R;
  }
  M.divR = mdpvi::make_fast_div(static_cast<uint32_t>(M.R));
  const double Lam = lam_tot + p->K * p->C * p->mu + p->K * p->nu;
  const double P_arr = lam_tot / Lam;
  M.n_sizes = 0;
  for (int j = 0; j < p->J; ++j) {
    M.size[j] = p->size[j];
    int u = 0;
    while (u < M.n_sizes && M.size_u[u] != p->size[j]) ++u;
    if (u == M.n_sizes) M.size_u[M.n_sizes++] = p->size[j];
    M.size_idx[j] = u;
    M.p[j] = p->lambda[j] / Lam;
    M.r_place[j] = P_arr * p->reward[j];
    M.r_reject[j] = -P_arr * (p->reject_cost ? p->reject_cost[j] : 0.0);
  }
  M.mu_L = p->mu / Lam;
  M.nu_L = p->nu / Lam;
  M.gamma = p->gamma;
  // feasible pairs: the paid cloud everywhere plus, per class e and host a,
  // the (C+1-size_e)/(C+1) share of occupancies with room on a
  int64_t pairs = 0;
  for (int j = 0; j < p->J; ++j)
    pairs += n_occ + static_cast<int64_t>(p->K) * (n_occ / M.R) * (M.R - p->size[j]);
  h->feasible_pairs = pairs;
  *out = h;
  return MDPVI_OK;
}

void mdp_free(mdpvi_mdp_t h) {
  if (!h) return;
  if (h->vbuf) (void)hipFree(h->vbuf);
  if (h->ctl) (void)hipFree(h->ctl);
  if (h->ctl_host) (void)hipHostFree(h->ctl_host);
  if (h->ev0) (void)hipEventDestroy(h->ev0);
  if (h->ev1) (void)hipEventDestroy(h->ev1);
  delete h;
}

int64_t mdp_num_states(mdpvi_mdp_t h) { return h ? h->M.n_states : -1; }
int32_t mdp_num_actions(mdpvi_mdp_t h) { return h ? h->M.K + 1 : -1; }
int64_t mdp_feasible_pairs(mdpvi_mdp_t h) { return h ? h->feasible_pairs : -1; }

int vi_solve(mdpvi_mdp_t h, float* V, double tol, int64_t max_iter, void* hip_stream,
             mdpvi_stats* st) {
  if (!h || !V) return fail(MDPVI_EINVAL, "NULL handle or value array");
  if (!(tol > 0)) return fail(MDPVI_EINVAL, "tol=%g must be > 0", tol);
  if (max_iter < 1) return fail(MDPVI_EINVAL, "max_iter=%lld must be >= 1", (long long)max_iter);
  int rc = ensure_scratch(h, static_cast<size_t>(h->M.n_states) * sizeof(float));
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const Model& M = h->M;
  return run_loop<float>(h, V, tol, max_iter, s, st, 8.0 * M.n_states,
                         static_cast<double>(h->feasible_pairs),
                         [&](long long j, float* in, float* out) {
                           return mdpvi::launch_vi_sweep(M, in, out, h->ctl, j, tol, s);
                         });
}

int policy_extract(mdpvi_mdp_t h, const float* V, uint8_t* pi, float* gap, void* hip_stream) {
  if (!h || !V || !pi) return fail(MDPVI_EINVAL, "NULL handle, value or policy array");
  HIP_TRY(mdpvi::launch_extract_f32(h->M, V, pi, gap, static_cast<hipStream_t>(hip_stream)));
  return MDPVI_OK;
}

int policy_extract_f64(mdpvi_mdp_t h, const double* V, uint8_t* pi, float* gap, void* hip_stream) {
  if (!h || !V || !pi) return fail(MDPVI_EINVAL, "NULL handle, value or policy array");
  HIP_TRY(mdpvi::launch_extract_f64(h->M, V, pi, gap, static_cast<hipStream_t>(hip_stream)));
  return MDPVI_OK;
}

int policy_eval(mdpvi_mdp_t h, const uint8_t* pi, double* V, double tol, int64_t max_iter,
                void* hip_stream, mdpvi_stats* st) {
  if (!h || !V || !pi) return fail(MDPVI_EINVAL, "NULL handle, policy or value array");
  if (!(tol > 0)) return fail(MDPVI_EINVAL, "tol=%g must be > 0", tol);
  if (max_iter < 1) return fail(MDPVI_EINVAL, "max_iter=%lld must be >= 1", (long long)max_iter);
  int rc = ensure_scratch(h, static_cast<size_t>(h->M.n_states) * sizeof(double));
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const Model& M = h->M;
  HIP_TRY(mdpvi::launch_ctl_init(h->ctl, s));
  HIP_TRY(mdpvi::launch_policy_check(M, pi, h->ctl, s));
  HIP_TRY(hipMemcpyAsync(h->ctl_host, h->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (h->ctl_host->flag)
    return fail(MDPVI_EINVAL, "policy has an action that is not feasible in its state");
  return run_loop<double>(h, V, tol, max_iter, s, st, 17.0 * M.n_states,
                          static_cast<double>(M.n_states),
                          [&](long long j, double* in, double* out) {
                            return mdpvi::launch_eval_sweep(M, pi, in, out, h->ctl, j, tol, s);
                          });
}

int policy_greedy(mdpvi_mdp_t h, int32_t kind, uint8_t* pi, void* hip_stream) {
  if (!h || !pi) return fail(MDPVI_EINVAL, "NULL handle or policy array");
  if (kind != 0 && kind != 1) return fail(MDPVI_EINVAL, "kind=%d must be 0 or 1", kind);
  HIP_TRY(mdpvi::launch_greedy(h->M, kind, pi, static_cast<hipStream_t>(hip_stream)));
  return MDPVI_OK;
}

}  // extern "C"
