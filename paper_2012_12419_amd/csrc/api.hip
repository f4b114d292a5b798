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
#include <algorithm>
#include <cstdlib>
#include <fstream>
#include <map>
#include <chrono>
#include <mutex>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/mdpvi.h"
#include "kernels.hpp"
#include "model.hpp"
#include "tile.hpp"

using mdpvi::Ctl;
using mdpvi::Model;

struct mdpvi_mdp {
  Model M;
  int64_t feasible_pairs = 0;
  int device = -1;              // device of the scratch below (-1: none yet)
  void* vbuf = nullptr;         // second value buffer (ping-pong partner)
  size_t vbuf_bytes = 0;
  uint8_t* pbuf = nullptr;      // policy scratch (policy iteration), N + 16 bytes
  double* abuf = nullptr;       // two FP64 arrival-term arrays of n_occ + kSentinel doubles
                                // (exact-shape direct and tile forms)
  Ctl* ctl = nullptr;           // device control words
  Ctl* ctl_host = nullptr;      // pinned mirror
  double* res = nullptr;        // residual words / per-workgroup partials
  double* res_host = nullptr;   // pinned, res_n doubles
  size_t res_n = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  double* aux = nullptr;        // gradient partials and outputs
  size_t aux_bytes = 0;
  double* out_host = nullptr;   // pinned, 2 * kMaxJ + 3 doubles
  bool timing = false;          // bracket every sweep with events
  int adjoint_form = 0;         // adjoint sweep form: 0 automatic, else a valid form
  int slab_t = -1;              // sweep form: -1 automatic, 0 direct, t > 0 slab of t digits,
                                // MDPVI_FORM_TILE the tile form
  hipEvent_t* sweep_ev = nullptr;   // 2 * kMaxChunk events (created on demand)
  uint32_t* tile_order[3][2] = {};   // device tile orders of T = 2, 3, 4: bisection, dealt runs
  uint32_t tile_order_run[3] = {};   // run length of the dealt orders
};

namespace {
constexpr int64_t kMaxChunk = 256;
}

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
    // the largest grid of any sweep form: the direct form, or the slab form
    // with one low digit (n_occ / (C+1) workgroups)
    const uint64_t g1 = static_cast<uint64_t>(h->M.n_occ) / static_cast<uint64_t>(h->M.R);
    const uint32_t gmax = std::max<uint32_t>(
        std::max(std::max(mdpvi::occ_sweep_grid(h->M), mdpvi::eval_sweep_grid(h->M)), mdpvi::vi_sweep_grid(h->M, 0)),
        static_cast<uint32_t>(g1));
    h->res_n = mdpvi::res_doubles(gmax);
    if (hipMalloc(reinterpret_cast<void**>(&h->res), h->res_n * sizeof(double)) != hipSuccess) {
      h->res = nullptr;
      return fail(MDPVI_ENOMEM, "hipMalloc of %zu residual words failed", h->res_n);
    }
    if (hipHostMalloc(reinterpret_cast<void**>(&h->res_host), h->res_n * sizeof(double),
                      hipHostMallocDefault) != hipSuccess) {
      h->res_host = nullptr;
      return fail(MDPVI_ENOMEM, "hipHostMalloc of the residual mirror failed");
    }
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

// Auxiliary device doubles (gradient partials + outputs) and the pinned
// host words the outputs are copied to.
int ensure_aux(mdpvi_mdp* h, size_t doubles) {
  if (!h->out_host) {
    if (hipHostMalloc(reinterpret_cast<void**>(&h->out_host), (2 * MDPVI_MAX_J + 3) * sizeof(double),
                      hipHostMallocDefault) != hipSuccess) {
      h->out_host = nullptr;
      return fail(MDPVI_ENOMEM, "hipHostMalloc of the output words failed");
    }
  }
  const size_t bytes = doubles * sizeof(double);
  if (bytes > h->aux_bytes) {
    if (h->aux) {
      HIP_TRY(hipDeviceSynchronize());
      HIP_TRY(hipFree(h->aux));
      h->aux = nullptr;
      h->aux_bytes = 0;
    }
    if (hipMalloc(reinterpret_cast<void**>(&h->aux), bytes) != hipSuccess) {
      h->aux = nullptr;
      return fail(MDPVI_ENOMEM, "hipMalloc of %zu auxiliary bytes failed", bytes);
    }
    h->aux_bytes = bytes;
  }
  return MDPVI_OK;
}

int tune_lookup(const Model& M, const char* op);

// The two FP64 arrival-term arrays (n_occ + kSentinel doubles each),
// allocated on first use, initialised from V: A[0] = sum_e lambda_e/Lam
// V(., e), and the -inf sentinel block of both.
int arrival_arrays(mdpvi_mdp* h, const float* V, hipStream_t s, double* A[2]) {
  const Model& M = h->M;
  const size_t per = static_cast<size_t>(M.n_occ) + mdpvi::kSentinel;
  if (!h->abuf && hipMalloc(reinterpret_cast<void**>(&h->abuf), 2 * per * sizeof(double)) != hipSuccess) {
    h->abuf = nullptr;
    return fail(MDPVI_ENOMEM, "hipMalloc of the arrival-term arrays failed");
  }
  A[0] = h->abuf;
  A[1] = h->abuf + per;
  HIP_TRY(mdpvi::launch_arrival_init(M, V, A[0], A[1], s));
  return MDPVI_OK;
}

int cu_count() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    return 1;
  return cus;
}

static_assert(MDPVI_ADJOINT_GROUP == mdpvi::kAdjointGroup, "adjoint group form code");
static_assert(mdpvi::kAdjointGroup > mdpvi::kAdjointExact + 4, "adjoint form codes overlap");
bool is_tile_form(int f) { return f >= MDPVI_FORM_TILE && f <= MDPVI_FORM_TILE + 8; }
bool is_row_form(int f) { return f >= MDPVI_FORM_ROW && f <= MDPVI_FORM_ROW + 8; }
// Workgroups of the column walk with w per CU: a multiple of 8.
// The tile or row form of a form code: its walkers per CU.
int form_walkers(int f) { return is_row_form(f) ? f - MDPVI_FORM_ROW : f - MDPVI_FORM_TILE; }

// Workgroups per CU of the automatic tile form (0: one workgroup per tile).
// With fewer tiles than two per walker, w persistent walkers per CU (4 for
// value iteration, 5 for evaluation) beat one workgroup per tile: 7% and 5%
// at 1,331 tiles (K = 6, C = 10); at 14,641 tiles (K = 7) one workgroup per
// tile is 10-14% faster.
constexpr int kTileWalkersVi = 4;
constexpr int kTileWalkersEval = 5;
// The row form's automatic choice: one persistent workgroup (384 lanes) per
// CU; it is taken where a sweep's working set exceeds the last-level cache
// (K = 7, C = 10: 8% faster than the tile form; within the cache the two
// are equal to within 3%).
constexpr int kRowWalkersVi = 1;
constexpr double kLlcBytes = 256.0 * 1024 * 1024;
// Bytes a sweep reads and writes once: values in and out, arrival terms in
// and out, and for evaluation the policy.
double vi_working_set(const Model& M) { return 8.0 * M.n_states + 16.0 * M.n_occ; }
double eval_working_set(const Model& M) { return 17.0 * M.n_states + 16.0 * M.n_occ; }

int auto_walkers(const mdpvi::TileShape& S, int w) {
  return S.n < 2u * static_cast<uint32_t>(w) * static_cast<uint32_t>(cu_count()) ? w : 0;
}

// The value-iteration form to run: the handle's choice, else the tuned one
// for the shape, else the row form or the tile form when it applies and is
// worthwhile, else the exact-shape direct form, else the slab form.  S is
// filled for the tile and row forms.
int vi_form(mdpvi_mdp* h, mdpvi::TileShape* S) {
  const Model& M = h->M;
  const int fallback = mdpvi::exact_shape(M) ? 0 : mdpvi::slab_digits(M);
  int f = h->slab_t;
  if (f < 0) {
    const int cached = tune_lookup(M, "vi");
    if (cached >= 0)
      f = cached;
    else if (vi_working_set(M) > kLlcBytes && mdpvi::vi_row_shape(M, S) && mdpvi::tile_worthwhile(*S))
      f = MDPVI_FORM_ROW + kRowWalkersVi;
    else if (mdpvi::vi_tile_shape(M, S) && mdpvi::tile_worthwhile(*S))
      f = MDPVI_FORM_TILE + auto_walkers(*S, kTileWalkersVi);
    else
      f = fallback;
  }
  if (is_row_form(f) && !mdpvi::vi_row_shape(M, S)) f = MDPVI_FORM_TILE + form_walkers(f);
  if (is_tile_form(f) && !mdpvi::vi_tile_shape(M, S)) return fallback;
  if (is_tile_form(f) || is_row_form(f)) mdpvi::tile_set_walkers(S, form_walkers(f), cu_count());
  return f;
}

// The evaluation form to run: the tile form where it applies and is
// worthwhile (or where the handle asks for the tile or row form of value
// iteration), else the direct form (0).
int eval_form(mdpvi_mdp* h, mdpvi::TileShape* S) {
  if (h->slab_t == -1) {   // a form mdp_autotune recorded for the shape
    const int cached = tune_lookup(h->M, "eval");
    if (cached == 0) return 0;
    if (is_tile_form(cached) && mdpvi::eval_tile_shape(h->M, S)) {
      mdpvi::tile_set_walkers(S, form_walkers(cached), cu_count());
      return cached;
    }
  }
  const bool forced = is_tile_form(h->slab_t) || is_row_form(h->slab_t);
  if (!(h->slab_t == -1 || forced) || !mdpvi::eval_tile_shape(h->M, S) || !(forced || mdpvi::tile_worthwhile(*S)))
    return 0;
  const int w = forced ? form_walkers(h->slab_t) : auto_walkers(*S, kTileWalkersEval);
  mdpvi::tile_set_walkers(S, w, cu_count());
  return MDPVI_FORM_TILE + w;
}

int eval_run(mdpvi_mdp* h, const uint8_t* pi, double* V, double tol, int64_t max_iter, hipStream_t s,
             mdpvi_stats* st);

// The adjoint sweep form to run: the one set on the handle, else the one
// mdp_autotune recorded for the shape, else the automatic one.
int adjoint_form(mdpvi_mdp* h) {
  if (h->adjoint_form > 0) return h->adjoint_form;
  const int cached = tune_lookup(h->M, "adjoint");
  if (cached > 0 && mdpvi::adjoint_form_valid(h->M, cached)) return cached;
  return mdpvi::adjoint_auto_form(h->M);
}

// Tile orders: for a sweep whose working set (values and arrival terms read
// and written) fits the last-level cache, recursive coordinate bisection
// (each XCD a compact block: fewest halo lines through its L2); beyond it,
// runs of kDealRun tiles dealt round-robin (all XCDs on one region, whose
// neighbour planes then stay in the last-level cache).
constexpr uint32_t kDealRun = 16;

// Tile-order codes (the tuning cache's "vi-order" and "eval-order"
// entries): kOrderRcb recursive coordinate bisection, kOrderIndex contiguous
// eighths of the index order, N >= 2 runs of N tiles dealt round-robin.
constexpr int kOrderRcb = 0;
constexpr int kOrderIndex = 1;

// Points S->order at the handle's device copy of the tile order for S's tile
// depth, built and uploaded on first use.  The order is `force` when it is a
// code (>= 0); else the one the environment variable MDPVI_TILE_ORDER names
// (a measurement aid: "index", "rcb" or "dealN"); else the one mdp_autotune
// recorded for operation op ("vi" or "eval") and this shape; else bisection
// for a sweep working set of ws bytes within the last-level cache and dealt
// runs of kDealRun tiles beyond it.
int set_tile_order(mdpvi_mdp* h, mdpvi::TileShape* S, double ws, const char* op, int force = -1) {
  int code = ws <= kLlcBytes ? kOrderRcb : static_cast<int>(kDealRun);
  if (force >= 0) {
    code = force;
  } else {
    const char* env = std::getenv("MDPVI_TILE_ORDER");
    const std::string forced(env ? env : "");
    if (forced == "index") code = kOrderIndex;
    else if (forced == "rcb") code = kOrderRcb;
    else if (forced.rfind("deal", 0) == 0) code = std::max(2, std::atoi(forced.c_str() + 4));
    else {
      const int cached = tune_lookup(h->M, (std::string(op) + "-order").c_str());
      if (cached >= 0) code = cached;
    }
  }
  S->order = nullptr;
  if (code == kOrderIndex) return MDPVI_OK;
  if (S->T < 2 || S->T > 4) return fail(MDPVI_EINVAL, "tile depth %d outside [2, 4]", S->T);
  const uint32_t run = code == kOrderRcb ? 0u : static_cast<uint32_t>(code);   // 0: bisection
  uint32_t*& d = h->tile_order[S->T - 2][run ? 1 : 0];
  uint32_t& d_run = h->tile_order_run[S->T - 2];
  if (d && run && d_run != run) {   // another dealt run length was forced
    (void)hipFree(d);
    d = nullptr;
  }
  if (!d) {
    std::vector<uint32_t> order;
    if (run)
      mdpvi::tile_deal(*S, run, &order);
    else
      mdpvi::tile_partition(h->M.K, h->M.R, *S, &order);
    if (hipMalloc(reinterpret_cast<void**>(&d), order.size() * sizeof(uint32_t)) != hipSuccess) {
      d = nullptr;
      return fail(MDPVI_ENOMEM, "hipMalloc of the tile order failed");
    }
    const hipError_t e = hipMemcpy(d, order.data(), order.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(d);
      d = nullptr;
      return fail_hip(e, "hipMemcpy(tile order)");
    }
    if (run) d_run = run;
  }
  S->order = d;
  return MDPVI_OK;
}

double bits_to_double(unsigned long long b) {
  double d;
  std::memcpy(&d, &b, sizeof d);
  return d;
}

// Final residual of sweep j, read from the device: the max over the grid
// workgroup maxima (max norm) or the sum of the kResLanes words (1-norm); a
// NaN anywhere makes the result NaN.
int final_residual(mdpvi_mdp* h, long long j, bool sum, uint32_t grid, hipStream_t s, double* out) {
  double r = 0.0;
  if (sum) {
    HIP_TRY(hipMemcpy2DAsync(h->res_host, sizeof(double), h->res + mdpvi::sum_word(j, 0),
                             mdpvi::kSumStride * sizeof(double), sizeof(double), mdpvi::kResLanes,
                             hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int l = 0; l < mdpvi::kResLanes; ++l) r += h->res_host[l];
  } else {
    HIP_TRY(hipMemcpyAsync(h->res_host, h->res + static_cast<size_t>(j % mdpvi::kResSlots) * grid,
                           grid * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (uint32_t b = 0; b < grid; ++b) {
      const double v = h->res_host[b];
      if (std::isnan(v)) {
        r = v;
        break;
      }
      r = std::max(r, v);
    }
  }
  *out = r;
  return MDPVI_OK;
}

// Enqueue sweeps j = 0, 1, ... in chunks until the device reports the test
// met or max_iter sweeps were issued; leaves the final iterate in buf0.
// `sweep(j, in, out)` enqueues sweep j.
template <typename T, typename Sweep>
int run_loop(mdpvi_mdp* h, T* buf0, double tol, int64_t max_iter, hipStream_t s,
             mdpvi_stats* st, double bytes_per_sweep, double backups_per_sweep, Sweep sweep,
             bool sum_residual, uint32_t grid) {
  T* buf[2] = {buf0, static_cast<T*>(h->vbuf)};
  HIP_TRY(mdpvi::launch_ctl_init(h->ctl, h->res, s));
  HIP_TRY(hipEventRecord(h->ev0, s));
  if (h->timing && !h->sweep_ev) {
    h->sweep_ev = new (std::nothrow) hipEvent_t[2 * kMaxChunk]();
    if (!h->sweep_ev) return fail(MDPVI_ENOMEM, "host allocation of timing events failed");
    for (int64_t i = 0; i < 2 * kMaxChunk; ++i) HIP_TRY(hipEventCreate(&h->sweep_ev[i]));
  }
  int64_t issued = 0;
  int64_t chunk = 8;
  long long done = -1;
  double sweep_ms = 0.0;
  while (issued < max_iter) {
    const int64_t n = std::min<int64_t>(chunk, max_iter - issued);
    for (int64_t i = 0; i < n; ++i) {
      const int64_t j = issued + i;
      if (h->timing) HIP_TRY(hipEventRecord(h->sweep_ev[2 * i], s));
      HIP_TRY(sweep(static_cast<long long>(j), buf[j & 1], buf[(j + 1) & 1]));
      if (h->timing) HIP_TRY(hipEventRecord(h->sweep_ev[2 * i + 1], s));
    }
    HIP_TRY(hipMemcpyAsync(h->ctl_host, h->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    done = h->ctl_host->done_iter;
    if (h->timing) {
      for (int64_t i = 0; i < n; ++i) {
        if (done >= 0 && issued + i >= done) break;   // sweeps from `done` on did no work
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, h->sweep_ev[2 * i], h->sweep_ev[2 * i + 1]));
        sweep_ms += ms;
      }
    }
    issued += n;
    if (done >= 0) break;
    if (chunk < kMaxChunk) chunk *= 2;
  }
  int64_t final_iter;
  double res;
  bool converged;
  final_iter = done >= 0 ? done : issued;
  {
    int rc = final_residual(h, final_iter - 1, sum_residual, grid, s, &res);
    if (rc) return rc;
  }
  converged = res < tol;
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
    st->sweep_seconds = sweep_ms * 1e-3;
  }
  if (std::isnan(res) || std::isinf(res))
    return fail(MDPVI_ENAN, "non-finite residual after %lld sweeps", (long long)final_iter);
  if (!converged)
    return fail(MDPVI_ENOCONV, "residual %.3e >= tol %.3e after %lld sweeps (max_iter)", res, tol,
                (long long)final_iter);
  return MDPVI_OK;
}

// ---------------------------------------------------------------- tuning cache
//
// Best sweep form per operation and problem shape, kept in memory and, when
// the environment variable MDPVI_AUTOTUNE_CACHE names a file, in that JSON
// file:
//   {"vi|gfx950|K=6|C=10|J=3|S=1,2,3": [20, 31.2], "eval|gfx950|...": [21, 44.0],
//    "adjoint|gfx950|...": [17, 9.1], ...}   (form, microseconds per sweep)
// A key without an operation (an older cache file) is value iteration's.
std::mutex g_tune_mu;
std::map<std::string, std::pair<int, double>> g_tune;
bool g_tune_loaded = false;

std::string tune_arch() {
  int dev = 0;
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
  }
  return arch;
}

std::string tune_key(const Model& M, const char* op) {
  std::ostringstream k;
  k << op << "|" << tune_arch() << "|K=" << M.K << "|C=" << M.C << "|J=" << M.J << "|S=";
  for (int j = 0; j < M.J; ++j) k << (j ? "," : "") << M.size[j];
  return k.str();
}

void tune_load_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = std::getenv("MDPVI_AUTOTUNE_CACHE");
  if (!path) return;
  std::ifstream f(path);
  if (!f) return;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  // entries of the form "key": [form, us]
  size_t pos = 0;
  while ((pos = s.find('"', pos)) != std::string::npos) {
    const size_t end = s.find('"', pos + 1);
    if (end == std::string::npos) break;
    const std::string key = s.substr(pos + 1, end - pos - 1);
    const size_t lb = s.find('[', end), rb = s.find(']', end);
    if (lb == std::string::npos || rb == std::string::npos || lb > rb) break;
    int form = 0;
    double us = 0.0;
    if (std::sscanf(s.c_str() + lb + 1, "%d , %lf", &form, &us) == 2)
      g_tune[key.rfind("gfx", 0) == 0 ? "vi|" + key : key] = {form, us};
    pos = rb + 1;
  }
}

void tune_store_locked() {
  const char* path = std::getenv("MDPVI_AUTOTUNE_CACHE");
  if (!path) return;
  std::ofstream f(path);
  f << "{\n";
  size_t i = 0;
  for (const auto& kv : g_tune) {
    char buf[64];
    std::snprintf(buf, sizeof buf, "[%d, %.4f]", kv.second.first, kv.second.second);
    f << "  \"" << kv.first << "\": " << buf << (++i < g_tune.size() ? ",\n" : "\n");
  }
  f << "}\n";
}

// Cached form of operation op ("vi", "eval", "adjoint") for M, or -2 when
// none is known.
int tune_lookup(const Model& M, const char* op) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_load_locked();
  auto it = g_tune.find(tune_key(M, op));
  return it == g_tune.end() ? -2 : it->second.first;
}

int tune_lookup_key(const std::string& key) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_load_locked();
  auto it = g_tune.find(key);
  return it == g_tune.end() ? -2 : it->second.first;
}

void tune_record_key(const std::string& key, int form, double us) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_load_locked();
  g_tune[key] = {form, us};
  tune_store_locked();
}

void tune_record(const Model& M, const char* op, int form, double us) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_load_locked();
  g_tune[tune_key(M, op)] = {form, us};
  tune_store_locked();
}

// Fill a Model from validated parameters (shared by single and batched builds).
int fill_model(const mdpvi_params* p, Model& M, int64_t& pairs_out) {
  if (!p) return fail(MDPVI_EINVAL, "NULL argument");
  if (p->K < 1 || p->K > MDPVI_MAX_K) return fail(MDPVI_EINVAL, "K=%d outside [1, %d]", p->K, MDPVI_MAX_K);
  if (p->J < 1 || p->J > MDPVI_MAX_J) return fail(MDPVI_EINVAL, "J=%d outside [1, %d]", p->J, MDPVI_MAX_J);
  if (p->C < 1) return fail(MDPVI_EINVAL, "C=%d must be >= 1", p->C);
  if (!p->size || !p->lambda || !p->reward) return fail(MDPVI_EINVAL, "NULL size/lambda/reward");
  if (!(p->gamma >= 0.0 && p->gamma < 1.0)) return fail(MDPVI_EINVAL, "gamma=%g outside [0, 1)", p->gamma);
  if (!is_finite(p->mu) || p->mu < 0) return fail(MDPVI_EINVAL, "mu=%g must be finite and >= 0", p->mu);
  if (!is_finite(p->nu) || p->nu < 0) return fail(MDPVI_EINVAL, "nu=%g must be finite and >= 0", p->nu);
  if (!is_finite(p->idle_unit_cost) || p->idle_unit_cost < 0)
    return fail(MDPVI_EINVAL, "idle_unit_cost=%g must be finite and >= 0", p->idle_unit_cost);
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
  M.hold = p->idle_unit_cost;
  M.gamma = p->gamma;
  for (int j = 0; j < p->J; ++j) {
    M.lam[j] = p->lambda[j];
    M.reward[j] = p->reward[j];
    M.cost[j] = p->reject_cost ? p->reject_cost[j] : 0.0;
    M.c_obj[j] = p->lambda[j] / lam_tot;
  }
  M.mu = p->mu;
  M.nu = p->nu;
  M.Lam = Lam;
  M.lam_tot = lam_tot;
  // feasible pairs: the paid cloud everywhere plus, per class e and host a,
  // the (C+1-size_e)/(C+1) share of occupancies with room on a
  int64_t pairs = 0;
  for (int j = 0; j < p->J; ++j)
    pairs += n_occ + static_cast<int64_t>(p->K) * (n_occ / M.R) * (M.R - p->size[j]);
  pairs_out = pairs;
  return MDPVI_OK;
}


}  // namespace

struct mdpvi_batch {
  int n = 0;
  std::vector<Model> models;
  std::vector<int64_t> offsets;      // n + 1 state offsets
  std::vector<int64_t> pairs;        // feasible pairs per sweep, per instance
  std::vector<int32_t> lds_list, round_list, all_list;
  std::vector<mdpvi::Tile> tiles;        // round-form instances (value iteration)
  std::vector<mdpvi::Tile> tiles_all;    // every instance (other passes)
  std::vector<int32_t> tile_begin;       // n+1 offsets of each instance in tiles_all
  // tiles of the round loops with 1, 2 and 4 occupancies per thread (index
  // log2 of that count): round-form instances, and every instance
  std::vector<mdpvi::Tile> rtiles[3], rtiles_all[3];
  mdpvi::Tile* d_rtiles[3] = {nullptr, nullptr, nullptr};
  mdpvi::Tile* d_rtiles_all[3] = {nullptr, nullptr, nullptr};
  // value iteration's tile form: tiles {inst, tile index} of the round-form
  // instances it covers (tocc > 0), and the direct tiles of the others
  std::vector<int32_t> tocc;             // per instance: (C+1)^3, or 0
  std::vector<mdpvi::Tile> vt_tiles, rtiles_nt[3];
  mdpvi::Tile* d_vt_tiles = nullptr;
  mdpvi::Tile* d_rtiles_nt[3] = {nullptr, nullptr, nullptr};
  mdpvi::Tile* d_vact[2] = {nullptr, nullptr};   // active-tile lists of the tile form
  size_t vt_lds = 0;                     // dynamic LDS of the tile-form rounds
  // FP64 evaluation's tile form: tiles of the instances it covers (eocc > 0),
  // the direct tiles of the others, and its arrival side arrays
  std::vector<int32_t> eocc;             // per instance: (C+1)^3, or 0
  std::vector<mdpvi::Tile> et_tiles, rtiles_all_nt[3];
  mdpvi::Tile* d_et_tiles = nullptr;
  mdpvi::Tile* d_rtiles_all_nt[3] = {nullptr, nullptr, nullptr};
  mdpvi::Tile* d_eact[2] = {nullptr, nullptr};
  size_t et_lds = 0;
  double* d_E[2] = {nullptr, nullptr};
  int64_t e_total = 0;                   // their length: sum of n_occ
  int tile_mode[2] = {-1, -1};           // tile form of value iteration and evaluation:
                                         // -1 automatic, 0 off, 1 on
  bool exact_all[3] = {false, false, false};   // per operation: every instance it rounds over meets
                                               // the exact-shape round backup's terms
  int round_opt[3] = {0, 0, 0};          // per operation (value iteration, evaluation, adjoint):
                                         // occupancies per thread, 0 automatic
  int lds_maxK = 1, lds_maxJ = 1, rnd_maxK = 1, rnd_maxJ = 1, maxK = 1, maxJ = 1;
  size_t lds_bytes = 0;
  int device = -1;
  mdpvi::BatchInst* d_inst = nullptr;
  int32_t* d_lds = nullptr;
  int32_t* d_round = nullptr;
  mdpvi::Tile* d_tiles = nullptr;
  mdpvi::Tile* d_tiles_all = nullptr;
  int32_t* d_all = nullptr;
  int32_t* d_tile_begin = nullptr;
  int* d_flags = nullptr;
  int* h_flags = nullptr;           // pinned
  double* d_gpart = nullptr;        // gradient partials per tile
  double* d_gout = nullptr;         // n rows of 2*kMaxJ+3
  double* h_gout = nullptr;         // pinned
  void* W2 = nullptr;               // FP64 ping-pong partner (evaluation), on first use
  mdpvi::BatchCtl* d_ctl = nullptr;
  int* d_remaining = nullptr;       // [0] unfinished instances, [1] active tiles after a compaction,
                                    // [2] active tile-form tiles
  mdpvi::Tile* d_act[2] = {nullptr, nullptr};   // active-tile lists of the round loops
  double* d_A[2] = {nullptr, nullptr};          // FP64 arrival terms of the round-form instances (VI)
  int* d_active[2] = {nullptr, nullptr};        // per-instance flags of batched policy iteration
  int* h_active = nullptr;                      // pinned
  uint8_t* d_pbuf = nullptr;                    // policy scratch (round check), on first use
  int64_t a_total = 0;                          // their length: sum of n_occ + max(1, tocc)
  double* d_lines = nullptr;                    // the adjoint's reset-line sums (BatchInst::loff)
  int64_t l_total = 0;                          // their length: sum of K J n_occ / (C+1)
  mdpvi::BatchOut* d_out = nullptr;
  float* W = nullptr;               // ping-pong partner of the concatenated values
  int* h_remaining = nullptr;       // pinned
  mdpvi::BatchOut* h_out = nullptr; // pinned
  hipStream_t side = nullptr;       // second stream for the LDS-resident solves
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev0 = nullptr, ev1 = nullptr;
};

extern "C" {

const char* mdpvi_last_error(void) { return g_err.c_str(); }

int mdp_build(const mdpvi_params* p, mdpvi_mdp_t* out) {
  if (!p || !out) return fail(MDPVI_EINVAL, "NULL argument");
  *out = nullptr;
  Model M;
  int64_t pairs = 0;
  int rc = fill_model(p, M, pairs);
  if (rc) return rc;
  mdpvi_mdp* h = new (std::nothrow) mdpvi_mdp();
  if (!h) return fail(MDPVI_ENOMEM, "host allocation failed");
  h->M = M;
  h->feasible_pairs = pairs;
  *out = h;
  return MDPVI_OK;
}

void mdp_free(mdpvi_mdp_t h) {
  if (!h) return;
  if (h->vbuf) (void)hipFree(h->vbuf);
  if (h->abuf) (void)hipFree(h->abuf);
  if (h->pbuf) (void)hipFree(h->pbuf);
  if (h->ctl) (void)hipFree(h->ctl);
  if (h->ctl_host) (void)hipHostFree(h->ctl_host);
  if (h->res) (void)hipFree(h->res);
  if (h->res_host) (void)hipHostFree(h->res_host);
  if (h->ev0) (void)hipEventDestroy(h->ev0);
  if (h->ev1) (void)hipEventDestroy(h->ev1);
  if (h->aux) (void)hipFree(h->aux);
  for (auto& per_t : h->tile_order)
    for (uint32_t* o : per_t)
      if (o) (void)hipFree(o);
  if (h->out_host) (void)hipHostFree(h->out_host);
  if (h->sweep_ev) {
    for (int64_t i = 0; i < 2 * kMaxChunk; ++i)
      if (h->sweep_ev[i]) (void)hipEventDestroy(h->sweep_ev[i]);
    delete[] h->sweep_ev;
  }
  delete h;
}

int mdp_sweep_forms(mdpvi_mdp_t h, int32_t* vi, int32_t* eval) {
  if (!h) return fail(MDPVI_EINVAL, "NULL handle");
  mdpvi::TileShape S{};
  if (vi) *vi = vi_form(h, &S);
  if (eval) *eval = eval_form(h, &S);
  return MDPVI_OK;
}

int mdp_set_timing(mdpvi_mdp_t h, int32_t per_sweep_events) {
  if (!h) return fail(MDPVI_EINVAL, "NULL handle");
  h->timing = per_sweep_events != 0;
  return MDPVI_OK;
}

int mdp_set_sweep_form(mdpvi_mdp_t h, int32_t slab_digits) {
  if (!h) return fail(MDPVI_EINVAL, "NULL handle");
  if (is_tile_form(slab_digits)) {
    mdpvi::TileShape S{};
    if (!mdpvi::vi_tile_shape(h->M, &S))
      return fail(MDPVI_EINVAL, "the tile form does not apply to this instance");
    h->slab_t = slab_digits;
    return MDPVI_OK;
  }
  if (is_row_form(slab_digits)) {
    mdpvi::TileShape S{};
    if (!mdpvi::vi_row_shape(h->M, &S))
      return fail(MDPVI_EINVAL, "the row form does not apply to this instance");
    h->slab_t = slab_digits;
    return MDPVI_OK;
  }
  if (slab_digits < -1 || slab_digits >= h->M.K)
    return fail(MDPVI_EINVAL, "slab_digits=%d outside [-1, K-1=%d]", slab_digits, h->M.K - 1);
  if (slab_digits > 0) {
    uint64_t occ = 1;
    for (int k = 0; k < slab_digits; ++k) occ *= static_cast<uint64_t>(h->M.R);
    if (occ * (8 + 4 * static_cast<uint64_t>(h->M.J)) > 64 * 1024 || !mdpvi::use_32bit_index(h->M))
      return fail(MDPVI_EINVAL, "a slab of %d digits does not fit the LDS budget", slab_digits);
  }
  h->slab_t = slab_digits;
  return MDPVI_OK;
}

int mdp_autotune(mdpvi_mdp_t h, const float* V, int32_t trials, void* hip_stream,
                 int32_t* best_form, double* best_us) {
  if (!h || !V) return fail(MDPVI_EINVAL, "NULL handle or value array");
  if (trials < 1) return fail(MDPVI_EINVAL, "trials=%d must be >= 1", trials);
  int rc = ensure_scratch(h, static_cast<size_t>(h->M.n_states) * sizeof(float));
  if (rc) return rc;
  const Model& M = h->M;
  const size_t N = static_cast<size_t>(M.n_states);
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  // median of `trials` timed launches of one sweep (after one untimed)
  auto time_form = [&](auto&& sweep, double* us) -> int {
    HIP_TRY(mdpvi::launch_ctl_init(h->ctl, h->res, s));
    HIP_TRY(sweep());
    std::vector<float> ms(trials);
    for (int r = 0; r < trials; ++r) {
      HIP_TRY(mdpvi::launch_ctl_init(h->ctl, h->res, s));
      HIP_TRY(hipEventRecord(h->ev0, s));
      HIP_TRY(sweep());
      HIP_TRY(hipEventRecord(h->ev1, s));
      HIP_TRY(hipEventSynchronize(h->ev1));
      HIP_TRY(hipEventElapsedTime(&ms[r], h->ev0, h->ev1));
    }
    std::sort(ms.begin(), ms.end());
    *us = ms[trials / 2] * 1e3;
    return MDPVI_OK;
  };

  // ---- value iteration: direct, slab, tile and row forms
  std::vector<int> forms = {0};
  if (mdpvi::use_32bit_index(M)) {
    uint64_t occ = 1;
    for (int t = 1; t < M.K; ++t) {
      occ *= static_cast<uint64_t>(M.R);
      if (occ * (8 + 4 * static_cast<uint64_t>(M.J)) <= 64 * 1024 &&
          static_cast<uint64_t>(M.n_occ) / occ >= 64)
        forms.push_back(t);
    }
  }
  mdpvi::TileShape S{};
  if (mdpvi::vi_tile_shape(M, &S)) {
    for (int w = 0; w <= 4; ++w) forms.push_back(MDPVI_FORM_TILE + w);
    mdpvi::TileShape Sr{};
    if (mdpvi::vi_row_shape(M, &Sr))
      for (int w = 0; w <= 4; ++w) forms.push_back(MDPVI_FORM_ROW + w);
    rc = set_tile_order(h, &S, vi_working_set(M), "vi");
    if (rc) return rc;
  }
  float* out = static_cast<float*>(h->vbuf);
  double* A[2] = {nullptr, nullptr};
  if (mdpvi::exact_shape(M) || is_tile_form(forms.back()) || is_row_form(forms.back())) {
    int arc = arrival_arrays(h, V, s, A);
    if (arc) return arc;
  }
  int best = 0;
  double best_t = 1e300;
  for (int form : forms) {
    // sweep 0 (no stopping test) from V into the scratch buffer
    auto sweep = [&]() -> hipError_t {
      if (is_tile_form(form)) {
        mdpvi::tile_set_walkers(&S, form - MDPVI_FORM_TILE, cu_count());
        return mdpvi::launch_vi_tile(M, S, V, out, A[0], A[1], h->ctl, h->res, 0, 1.0, s);
      }
      if (is_row_form(form)) {
        mdpvi::tile_set_walkers(&S, form - MDPVI_FORM_ROW, cu_count());
        return mdpvi::launch_vi_row(M, S, V, out, A[0], A[1], h->ctl, h->res, 0, 1.0, s);
      }
      return mdpvi::launch_vi_sweep(M, V, out, h->ctl, h->res, 0, 1.0, s, form,
                                    (form == 0 && A[0] && mdpvi::exact_shape(M)) ? A : nullptr);
    };
    double us = 0.0;
    if ((rc = time_form(sweep, &us))) return rc;
    if (us < best_t) {
      best_t = us;
      best = form;
    }
  }
  tune_record(M, "vi", best, best_t);
  if (best_form) *best_form = best;
  if (best_us) *best_us = best_t;
  // the tile order (the assignment of tiles to XCDs) of the best tile or row
  // form: bisection, index order, dealt runs of 16 and of (C+1)^2 tiles
  if (is_tile_form(best) || is_row_form(best)) {
    const bool row = is_row_form(best);
    mdpvi::tile_set_walkers(&S, form_walkers(best), cu_count());
    int obest = -1;
    double obest_t = 1e300;
    for (int code : {kOrderRcb, kOrderIndex, 16, M.R * M.R}) {
      if ((rc = set_tile_order(h, &S, vi_working_set(M), "vi", code))) return rc;
      auto sweep = [&]() -> hipError_t {
        return row ? mdpvi::launch_vi_row(M, S, V, out, A[0], A[1], h->ctl, h->res, 0, 1.0, s)
                   : mdpvi::launch_vi_tile(M, S, V, out, A[0], A[1], h->ctl, h->res, 0, 1.0, s);
      };
      double us = 0.0;
      if ((rc = time_form(sweep, &us))) return rc;
      if (us < obest_t) {
        obest_t = us;
        obest = code;
      }
    }
    tune_record(M, "vi-order", obest, obest_t);
  }

  // ---- FP64 evaluation (direct form, tile form with 0..5 workgroups per CU)
  // and the adjoint sweep (generic and exact-shape kernels, 1, 2 or 4
  // occupancies per thread), both on the least-loaded policy; temporary
  // buffers only
  uint8_t* pol = nullptr;
  double* ev[2] = {nullptr, nullptr};
  if (hipMalloc(reinterpret_cast<void**>(&pol), N + 16) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&ev[0]), 2 * N * sizeof(double)) != hipSuccess) {
    if (pol) (void)hipFree(pol);
    return fail(MDPVI_ENOMEM, "hipMalloc of the tuning buffers failed");
  }
  ev[1] = ev[0] + N;
  auto release = [&]() {
    (void)hipStreamSynchronize(s);
    (void)hipFree(pol);
    (void)hipFree(ev[0]);
  };
  auto tune_rest = [&]() -> int {
    HIP_TRY(mdpvi::launch_greedy(M, 0, pol, s));
    HIP_TRY(hipMemsetAsync(ev[0], 0, 2 * N * sizeof(double), s));
    std::vector<int> eforms = {0};
    mdpvi::TileShape Se{};
    double* Ae[2] = {nullptr, nullptr};
    if (mdpvi::eval_tile_shape(M, &Se)) {
      for (int w = 0; w <= 5; ++w) eforms.push_back(MDPVI_FORM_TILE + w);
      const size_t per = static_cast<size_t>(M.n_occ) + mdpvi::kSentinel;
      if (!h->abuf && hipMalloc(reinterpret_cast<void**>(&h->abuf), 2 * per * sizeof(double)) != hipSuccess) {
        h->abuf = nullptr;
        return fail(MDPVI_ENOMEM, "hipMalloc of the arrival-term arrays failed");
      }
      Ae[0] = h->abuf;
      Ae[1] = h->abuf + per;
      int orc = set_tile_order(h, &Se, eval_working_set(M), "eval");
      if (orc) return orc;
      HIP_TRY(mdpvi::launch_eval_arrival_init(M, ev[0], Ae[0], s));
    }
    int ebest = 0;
    double ebest_t = 1e300;
    for (int form : eforms) {
      auto sweep = [&]() -> hipError_t {
        if (is_tile_form(form)) {
          mdpvi::tile_set_walkers(&Se, form - MDPVI_FORM_TILE, cu_count());
          return mdpvi::launch_eval_tile(M, Se, pol, ev[0], ev[1], Ae[0], Ae[1], h->ctl, h->res, 0, 1.0, s);
        }
        return mdpvi::launch_eval_sweep(M, pol, ev[0], ev[1], h->ctl, h->res, 0, 1.0, s);
      };
      double us = 0.0;
      int trc = time_form(sweep, &us);
      if (trc) return trc;
      if (us < ebest_t) {
        ebest_t = us;
        ebest = form;
      }
    }
    tune_record(M, "eval", ebest, ebest_t);
    if (is_tile_form(ebest)) {
      mdpvi::tile_set_walkers(&Se, ebest - MDPVI_FORM_TILE, cu_count());
      int obest = -1;
      double obest_t = 1e300;
      for (int code : {kOrderRcb, kOrderIndex, 16, M.R * M.R}) {
        int orc = set_tile_order(h, &Se, eval_working_set(M), "eval", code);
        if (orc) return orc;
        auto sweep = [&]() -> hipError_t {
          return mdpvi::launch_eval_tile(M, Se, pol, ev[0], ev[1], Ae[0], Ae[1], h->ctl, h->res, 0, 1.0, s);
        };
        double us = 0.0;
        int trc = time_form(sweep, &us);
        if (trc) return trc;
        if (us < obest_t) {
          obest_t = us;
          obest = code;
        }
      }
      tune_record(M, "eval-order", obest, obest_t);
    }
    std::vector<int> aforms;
    if (mdpvi::adjoint_form_valid(M, mdpvi::kAdjointGroup)) aforms.push_back(mdpvi::kAdjointGroup);
    for (int opt : {1, 2, 4}) {
      if (mdpvi::adjoint_form_valid(M, opt)) aforms.push_back(opt);
      if (mdpvi::adjoint_form_valid(M, mdpvi::kAdjointExact + opt)) aforms.push_back(mdpvi::kAdjointExact + opt);
    }
    int abest = mdpvi::adjoint_auto_form(M);
    double abest_t = 1e300;
    for (int form : aforms) {
      auto sweep = [&]() -> hipError_t {
        return mdpvi::launch_adjoint_sweep(M, form, pol, V, out, h->ctl, h->res, 0, 1.0, s);
      };
      double us = 0.0;
      int trc = time_form(sweep, &us);
      if (trc) return trc;
      if (us < abest_t) {
        abest_t = us;
        abest = form;
      }
    }
    tune_record(M, "adjoint", abest, abest_t);
    return MDPVI_OK;
  };
  rc = tune_rest();
  release();
  return rc;
}

int32_t mdp_adjoint_form(mdpvi_mdp_t h) { return h ? adjoint_form(h) : -1; }

int mdp_set_adjoint_form(mdpvi_mdp_t h, int32_t form) {
  if (!h) return fail(MDPVI_EINVAL, "NULL handle");
  if (form != 0 && !mdpvi::adjoint_form_valid(h->M, form))
    return fail(MDPVI_EINVAL, "adjoint form %d does not apply to this instance", form);
  h->adjoint_form = form;
  return MDPVI_OK;
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
  mdpvi::TileShape S{};
  const int form = vi_form(h, &S);
  const bool tiled = is_tile_form(form) || is_row_form(form);
  double* A[2] = {nullptr, nullptr};
  if ((form == 0 && mdpvi::exact_shape(M)) || tiled) {
    int arc = arrival_arrays(h, V, s, A);
    if (arc) return arc;
  }
  if (tiled) {
    int orc = set_tile_order(h, &S, vi_working_set(M), "vi");
    if (orc) return orc;
  }
  if (is_row_form(form))
    return run_loop<float>(h, V, tol, max_iter, s, st, 8.0 * M.n_states,
                           static_cast<double>(h->feasible_pairs),
                           [&](long long j, float* in, float* out) {
                             return mdpvi::launch_vi_row(M, S, in, out, A[j & 1], A[(j + 1) & 1], h->ctl, h->res,
                                                         j, tol, s);
                           },
                           false, S.grid);
  if (is_tile_form(form))
    return run_loop<float>(h, V, tol, max_iter, s, st, 8.0 * M.n_states,
                           static_cast<double>(h->feasible_pairs),
                           [&](long long j, float* in, float* out) {
                             return mdpvi::launch_vi_tile(M, S, in, out, A[j & 1], A[(j + 1) & 1], h->ctl,
                                                          h->res, j, tol, s);
                           },
                           false, S.grid);
  return run_loop<float>(h, V, tol, max_iter, s, st, 8.0 * M.n_states,
                         static_cast<double>(h->feasible_pairs),
                         [&](long long j, float* in, float* out) {
                           return mdpvi::launch_vi_sweep(M, in, out, h->ctl, h->res, j, tol, s, form,
                                                         A[0] ? A : nullptr);
                         },
                         false, mdpvi::vi_sweep_grid(M, form));
}

}  // extern "C"

// ---------------------------------------------------------------- allocation-free value iteration
//
// vi_solve_noalloc runs the sweeps of vi_solve with every piece of device
// scratch (control words, residual words, the two FP64 arrival-term arrays,
// the ping-pong value buffer) carved out of one file-scope device array.
// Each device that runs it holds its own copy of the array until the process
// ends; the host reaches a device's copy only through the address
// hipGetSymbolAddress returns with that device current (the array's name in
// host code is a host-side stand-in, not a device address).

namespace {
constexpr size_t kNoAllocBytes = size_t{64} << 20;
constexpr int kNoAllocDevices = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

std::mutex g_scratch_mu;
unsigned char* g_scratch_dev[kNoAllocDevices] = {};

// The current device's copy of the scratch array (looked up once per device).
int noalloc_scratch(unsigned char** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kNoAllocDevices)
    return fail(MDPVI_EINVAL, "device %d is beyond the %d the allocation-free form supports", dev,
                kNoAllocDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return fail_hip(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(MDPVI_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_dev[dev] = static_cast<unsigned char*>(p);
  }
  *out = g_scratch_dev[dev];
  return MDPVI_OK;
}

size_t round256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

extern "C" {

int vi_solve_noalloc(mdpvi_mdp_t h, float* V, double tol, int64_t max_iter, void* hip_stream,
                     mdpvi_stats* st) {
  if (!h || !V) return fail(MDPVI_EINVAL, "NULL handle or value array");
  if (!(tol > 0)) return fail(MDPVI_EINVAL, "tol=%g must be > 0", tol);
  if (max_iter < 1) return fail(MDPVI_EINVAL, "max_iter=%lld must be >= 1", (long long)max_iter);
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const Model& M = h->M;
  // the form of vi_solve without the tuning cache: the handle's explicit
  // choice, else the tile form where worthwhile, else the direct forms; the
  // tiles run in index order (every order gives the same iterates)
  mdpvi::TileShape S{};
  const int fallback = mdpvi::exact_shape(M) ? 0 : mdpvi::slab_digits(M);
  int form = h->slab_t;
  if (form < 0) {
    if (vi_working_set(M) > kLlcBytes && mdpvi::vi_row_shape(M, &S) && mdpvi::tile_worthwhile(S))
      form = MDPVI_FORM_ROW + kRowWalkersVi;
    else if (mdpvi::vi_tile_shape(M, &S) && mdpvi::tile_worthwhile(S))
      form = MDPVI_FORM_TILE + auto_walkers(S, kTileWalkersVi);
    else
      form = fallback;
  }
  if (is_row_form(form) && !mdpvi::vi_row_shape(M, &S)) form = MDPVI_FORM_TILE + form_walkers(form);
  if (is_tile_form(form) && !mdpvi::vi_tile_shape(M, &S)) form = fallback;
  const bool row = is_row_form(form);
  if (is_tile_form(form) || row) {
    mdpvi::tile_set_walkers(&S, form_walkers(form), cu_count());
    S.order = nullptr;
  }
  const bool tile = is_tile_form(form) || row;
  const bool arrival = tile || (form == 0 && mdpvi::exact_shape(M));
  const uint32_t grid = tile ? S.grid : mdpvi::vi_sweep_grid(M, form);
  // scratch layout: control words | residual words | A0 | A1 | second values
  const size_t a_doubles = static_cast<size_t>(M.n_occ) + mdpvi::kSentinel;
  const size_t o_res = round256(sizeof(Ctl));
  const size_t o_a0 = o_res + round256(mdpvi::res_doubles(grid) * sizeof(double));
  const size_t o_a1 = o_a0 + (arrival ? round256(a_doubles * sizeof(double)) : 0);
  const size_t o_v = o_a1 + (arrival ? round256(a_doubles * sizeof(double)) : 0);
  const size_t need = o_v + round256(static_cast<size_t>(M.n_states) * sizeof(float));
  if (need > kNoAllocBytes)
    return fail(MDPVI_ERANGE,
                "%lld states need %zu bytes of scratch; the allocation-free form holds %zu (use vi_solve)",
                (long long)M.n_states, need, kNoAllocBytes);
  unsigned char* base = nullptr;
  int rc = noalloc_scratch(&base);
  if (rc) return rc;
  Ctl* ctl = reinterpret_cast<Ctl*>(base);
  double* res = reinterpret_cast<double*>(base + o_res);
  double* A[2] = {arrival ? reinterpret_cast<double*>(base + o_a0) : nullptr,
                  arrival ? reinterpret_cast<double*>(base + o_a1) : nullptr};
  float* buf[2] = {V, reinterpret_cast<float*>(base + o_v)};

  // control and residual words start cleared (a kernel, not a memset)
  HIP_TRY(mdpvi::launch_ctl_init(ctl, res, s));
  if (arrival) HIP_TRY(mdpvi::launch_arrival_init(M, V, A[0], A[1], s));
  int64_t issued = 0, chunk = 8;
  long long done = -1;
  while (issued < max_iter) {
    const int64_t n = std::min<int64_t>(chunk, max_iter - issued);
    for (int64_t i = 0; i < n; ++i) {
      const long long j = static_cast<long long>(issued + i);
      if (row)
        HIP_TRY(mdpvi::launch_vi_row(M, S, buf[j & 1], buf[(j + 1) & 1], A[j & 1], A[(j + 1) & 1], ctl, res, j,
                                     tol, s));
      else if (tile)
        HIP_TRY(mdpvi::launch_vi_tile(M, S, buf[j & 1], buf[(j + 1) & 1], A[j & 1], A[(j + 1) & 1], ctl, res, j,
                                      tol, s));
      else
        HIP_TRY(mdpvi::launch_vi_sweep(M, buf[j & 1], buf[(j + 1) & 1], ctl, res, j, tol, s, form,
                                       arrival ? A : nullptr));
    }
    HIP_TRY(hipMemcpyAsync(&done, &ctl->done_iter, sizeof done, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    issued += n;
    if (done >= 0) break;
    if (chunk < kMaxChunk) chunk *= 2;
  }
  const int64_t final_iter = done >= 0 ? done : issued;
  // largest workgroup residual of the last sweep, read in pieces
  double r = 0.0;
  {
    const double* words = res + static_cast<size_t>((final_iter - 1) % mdpvi::kResSlots) * grid;
    double part[512];
    for (uint32_t b0 = 0; b0 < grid && !std::isnan(r); b0 += 512) {
      const uint32_t m = std::min<uint32_t>(512, grid - b0);
      HIP_TRY(hipMemcpyAsync(part, words + b0, m * sizeof(double), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      for (uint32_t b = 0; b < m; ++b) {
        if (std::isnan(part[b])) {
          r = part[b];
          break;
        }
        r = std::max(r, part[b]);
      }
    }
  }
  if (final_iter & 1)
    HIP_TRY(hipMemcpyAsync(V, buf[1], static_cast<size_t>(M.n_states) * sizeof(float), hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (st) {
    st->iterations = final_iter;
    st->residual_inf = r;
    st->bound_inf = M.gamma / (1.0 - M.gamma) * r;
    st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    st->backups = static_cast<double>(h->feasible_pairs) * static_cast<double>(final_iter);
    st->bytes = 8.0 * static_cast<double>(M.n_states) * static_cast<double>(final_iter);
    st->sweep_seconds = 0.0;
  }
  if (std::isnan(r) || std::isinf(r))
    return fail(MDPVI_ENAN, "non-finite residual after %lld sweeps", (long long)final_iter);
  if (!(r < tol))
    return fail(MDPVI_ENOCONV, "residual %.3e >= tol %.3e after %lld sweeps (max_iter)", r, tol,
                (long long)final_iter);
  return MDPVI_OK;
}

int vi_solve_bsdi(mdpvi_mdp_t h, float* V, double tol, int64_t max_iter, int32_t inner, void* hip_stream,
                  mdpvi_stats* st) {
  if (!h || !V) return fail(MDPVI_EINVAL, "NULL handle or value array");
  if (!(tol > 0)) return fail(MDPVI_EINVAL, "tol=%g must be > 0", tol);
  if (max_iter < 1) return fail(MDPVI_EINVAL, "max_iter=%lld must be >= 1", (long long)max_iter);
  if (inner < 1 || inner > 1024) return fail(MDPVI_EINVAL, "inner=%d outside [1, 1024]", inner);
  const Model& M = h->M;
  mdpvi::TileShape S{};
  if (!mdpvi::vi_bsdi_shape(M, &S))
    return fail(MDPVI_EINVAL, "the block-asynchronous form needs an exact shape (K in 3..8, J <= 3 distinct "
                              "sizes) whose tile fits the LDS budget");
  int rc = ensure_scratch(h, static_cast<size_t>(M.n_states) * sizeof(float));
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  double* A[2] = {nullptr, nullptr};
  rc = arrival_arrays(h, V, s, A);
  if (rc) return rc;
  rc = set_tile_order(h, &S, vi_working_set(M), "vi");
  if (rc) return rc;
  return run_loop<float>(h, V, tol, max_iter, s, st, 8.0 * M.n_states,
                         static_cast<double>(h->feasible_pairs) * inner,
                         [&](long long j, float* in, float* out) {
                           return mdpvi::launch_vi_bsdi(M, S, inner, in, out, A[j & 1], A[(j + 1) & 1], h->ctl,
                                                        h->res, j, tol, s);
                         },
                         false, S.grid);
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
  HIP_TRY(mdpvi::launch_ctl_init(h->ctl, h->res, s));
  HIP_TRY(mdpvi::launch_policy_check(M, pi, h->ctl, s));
  HIP_TRY(hipMemcpyAsync(h->ctl_host, h->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (h->ctl_host->flag)
    return fail(MDPVI_EINVAL, "policy has an action that is not feasible in its state");
  return eval_run(h, pi, V, tol, max_iter, s, st);
}

}  // extern "C"

namespace {

// Evaluation sweeps of a policy known to be feasible (policy_eval after its
// check; policy_iteration).  The scratch must hold N doubles.
int eval_run(mdpvi_mdp* h, const uint8_t* pi, double* V, double tol, int64_t max_iter, hipStream_t s,
             mdpvi_stats* st) {
  const Model& M = h->M;
  // the tile form where it applies and is worthwhile, or where the handle
  // asks for it; the direct form otherwise
  mdpvi::TileShape S{};
  if (eval_form(h, &S) != 0) {
    const size_t per = static_cast<size_t>(M.n_occ) + mdpvi::kSentinel;
    if (!h->abuf && hipMalloc(reinterpret_cast<void**>(&h->abuf), 2 * per * sizeof(double)) != hipSuccess) {
      h->abuf = nullptr;
      return fail(MDPVI_ENOMEM, "hipMalloc of the arrival-term arrays failed");
    }
    double* A[2] = {h->abuf, h->abuf + per};
    int orc = set_tile_order(h, &S, eval_working_set(M), "eval");
    if (orc) return orc;
    HIP_TRY(mdpvi::launch_eval_arrival_init(M, V, A[0], s));
    return run_loop<double>(h, V, tol, max_iter, s, st, 17.0 * M.n_states,
                            static_cast<double>(M.n_states),
                            [&](long long j, double* in, double* out) {
                              return mdpvi::launch_eval_tile(M, S, pi, in, out, A[j & 1], A[(j + 1) & 1],
                                                             h->ctl, h->res, j, tol, s);
                            },
                            false, S.grid);
  }
  return run_loop<double>(h, V, tol, max_iter, s, st, 17.0 * M.n_states,
                          static_cast<double>(M.n_states),
                          [&](long long j, double* in, double* out) {
                            return mdpvi::launch_eval_sweep(M, pi, in, out, h->ctl, h->res, j, tol, s);
                          },
                          false, mdpvi::eval_sweep_grid(M));
}

}  // namespace

extern "C" {

int policy_iteration(mdpvi_mdp_t h, uint8_t* pi, double* V, double eval_tol, int64_t eval_max_iter,
                     double improve_tol, int64_t max_rounds, void* hip_stream, mdpvi_stats* st,
                     int64_t* rounds) {
  if (!h || !V || !pi) return fail(MDPVI_EINVAL, "NULL handle, policy or value array");
  if (!(eval_tol > 0)) return fail(MDPVI_EINVAL, "eval_tol=%g must be > 0", eval_tol);
  if (!(improve_tol >= 0) || std::isinf(improve_tol))
    return fail(MDPVI_EINVAL, "improve_tol=%g must be finite and >= 0", improve_tol);
  if (eval_max_iter < 1 || max_rounds < 1)
    return fail(MDPVI_EINVAL, "eval_max_iter=%lld and max_rounds=%lld must be >= 1", (long long)eval_max_iter,
                (long long)max_rounds);
  const Model& M = h->M;
  const size_t N = static_cast<size_t>(M.n_states);
  int rc = ensure_scratch(h, N * sizeof(double));
  if (rc) return rc;
  if (!h->pbuf) {
    if (hipMalloc(reinterpret_cast<void**>(&h->pbuf), N + 16) != hipSuccess) {
      h->pbuf = nullptr;
      return fail(MDPVI_ENOMEM, "hipMalloc of the policy scratch failed");
    }
  }
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  HIP_TRY(mdpvi::launch_ctl_init(h->ctl, h->res, s));
  HIP_TRY(mdpvi::launch_policy_check(M, pi, h->ctl, s));
  HIP_TRY(hipMemcpyAsync(h->ctl_host, h->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (h->ctl_host->flag)
    return fail(MDPVI_EINVAL, "policy has an action that is not feasible in its state");
  const auto t0 = std::chrono::steady_clock::now();
  mdpvi_stats tot{};
  int64_t r = 0;
  bool stable = false;
  while (r < max_rounds && !stable) {
    ++r;
    mdpvi_stats e{};
    rc = eval_run(h, pi, V, eval_tol, eval_max_iter, s, &e);
    tot.iterations += e.iterations;
    tot.residual_inf = e.residual_inf;
    tot.bound_inf = e.bound_inf;
    tot.backups += e.backups;
    tot.bytes += e.bytes;
    tot.sweep_seconds += e.sweep_seconds;
    if (rc != MDPVI_OK) break;
    // improvement: keep the current action unless another beats its Q by
    // more than improve_tol (lowest-index argmax then), FP64
    HIP_TRY(mdpvi::launch_improve(M, V, pi, h->pbuf, improve_tol, s));
    HIP_TRY(mdpvi::launch_ctl_init(h->ctl, nullptr, s));
    HIP_TRY(mdpvi::launch_policy_diff(N, pi, h->pbuf, h->ctl, s));
    HIP_TRY(hipMemcpyAsync(h->ctl_host, h->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    stable = h->ctl_host->flag == 0;
    if (!stable) HIP_TRY(hipMemcpyAsync(pi, h->pbuf, N, hipMemcpyDeviceToDevice, s));
  }
  HIP_TRY(hipStreamSynchronize(s));
  tot.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (st) *st = tot;
  if (rounds) *rounds = r;
  if (rc != MDPVI_OK) return rc;
  if (!stable)
    return fail(MDPVI_ENOCONV, "policy still changing after %lld rounds (max_rounds)", (long long)r);
  return MDPVI_OK;
}

int vi_adjoint(mdpvi_mdp_t h, const uint8_t* pi, const double* V_pi, float* w, double* grad,
               double* objective, double tol, int64_t max_iter, void* hip_stream,
               mdpvi_stats* st) {
  if (!h || !pi || !V_pi || !w || !grad)
    return fail(MDPVI_EINVAL, "NULL handle, policy, value, adjoint or gradient array");
  if (!(tol > 0)) return fail(MDPVI_EINVAL, "tol=%g must be > 0", tol);
  if (max_iter < 1) return fail(MDPVI_EINVAL, "max_iter=%lld must be >= 1", (long long)max_iter);
  int rc = ensure_scratch(h, static_cast<size_t>(h->M.n_states) * sizeof(float));
  if (rc) return rc;
  const size_t npart = mdpvi::grad_partial_doubles(h->M);
  rc = ensure_aux(h, npart + 2 * MDPVI_MAX_J + 3);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const Model& M = h->M;
  HIP_TRY(mdpvi::launch_ctl_init(h->ctl, h->res, s));
  HIP_TRY(mdpvi::launch_policy_check(M, pi, h->ctl, s));
  HIP_TRY(hipMemcpyAsync(h->ctl_host, h->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (h->ctl_host->flag)
    return fail(MDPVI_EINVAL, "policy has an action that is not feasible in its state");
  const int aform = adjoint_form(h);
  rc = run_loop<float>(
      h, w, tol, max_iter, s, st, 9.0 * M.n_states, static_cast<double>(M.n_states),
      [&](long long j, float* in, float* out) {
        return mdpvi::launch_adjoint_sweep(M, aform, pi, in, out, h->ctl, h->res, j, tol, s);
      },
      /*sum_residual=*/true, mdpvi::occ_sweep_grid(M));
  if (rc != MDPVI_OK && rc != MDPVI_ENOCONV) return rc;
  double* out_dev = h->aux + npart;
  HIP_TRY(mdpvi::launch_grad(M, pi, V_pi, w, h->aux, out_dev, s));
  const int nt = 2 * M.J + 2;
  HIP_TRY(hipMemcpyAsync(h->out_host, out_dev, (nt + 1) * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  std::memcpy(grad, h->out_host, nt * sizeof(double));
  if (objective) *objective = h->out_host[nt];
  return rc;
}

int policy_objective(mdpvi_mdp_t h, const double* V, double* out, void* hip_stream) {
  if (!h || !V || !out) return fail(MDPVI_EINVAL, "NULL handle, value array or output");
  int rc = ensure_aux(h, 1);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  HIP_TRY(mdpvi::launch_objective(h->M, V, h->aux, s));
  HIP_TRY(hipMemcpyAsync(h->out_host, h->aux, sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  *out = h->out_host[0];
  return MDPVI_OK;
}

int policy_greedy(mdpvi_mdp_t h, int32_t kind, uint8_t* pi, void* hip_stream) {
  if (!h || !pi) return fail(MDPVI_EINVAL, "NULL handle or policy array");
  if (kind != 0 && kind != 1) return fail(MDPVI_EINVAL, "kind=%d must be 0 or 1", kind);
  HIP_TRY(mdpvi::launch_greedy(h->M, kind, pi, static_cast<hipStream_t>(hip_stream)));
  return MDPVI_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- batches

namespace {

// Tuning-cache key of a batch's round kernels for operation op (0 value
// iteration, 1 evaluation, 2 adjoint): the architecture, the instance count
// and an FNV-1a digest of every instance's (K, C, J, sizes).
std::string batch_tune_key(const mdpvi_batch* b, int op) {
  static const char* const names[3] = {"batch-vi", "batch-eval", "batch-adjoint"};
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](int64_t v) {
    for (int byte = 0; byte < 8; ++byte) {
      h ^= static_cast<uint64_t>(v >> (8 * byte)) & 0xffu;
      h *= 1099511628211ull;
    }
  };
  for (const Model& M : b->models) {
    mix(M.K);
    mix(M.C);
    mix(M.J);
    for (int j = 0; j < M.J; ++j) mix(M.size[j]);
  }
  char buf[32];
  std::snprintf(buf, sizeof buf, "%016llx", static_cast<unsigned long long>(h));
  std::ostringstream k;
  k << names[op] << "|" << tune_arch() << "|n=" << b->n << "|shapes=" << buf;
  return k.str();
}

// Occupancies per thread of the round kernels of operation op: the one set
// on the batch, else the one batch_autotune recorded for its shapes, else
// kOccPerThread.
int batch_opt(const mdpvi_batch* b, int op) {
  if (b->round_opt[op] > 0) return b->round_opt[op];
  const int cached = tune_lookup_key(batch_tune_key(b, op));
  if (cached == 1 || cached == 2 || cached == 4) return cached;
  return mdpvi::kOccPerThread;
}

int opt_index(int opt) { return opt == 1 ? 0 : opt == 2 ? 1 : 2; }

// Whether the rounds of operation op (0 value iteration, 1 evaluation) run
// the tile form for the instances it covers: the mode set on the batch,
// else the choice batch_autotune recorded for its shapes, else on for value
// iteration and off for evaluation (on the 256-instance gradient batch the
// tile form takes value iteration from 76 to 49 ms, while evaluation to
// tolerance stays at 123 ms with or without it).
bool batch_tile_on(const mdpvi_batch* b, int op) {
  if ((op == 0 ? b->vt_tiles : b->et_tiles).empty()) return false;
  if (b->tile_mode[op] >= 0) return b->tile_mode[op] == 1;
  const int cached = tune_lookup_key(batch_tune_key(b, op) + "|tile");
  return cached == -2 ? op == 0 : cached != 0;
}

// The evaluation rounds' tile lists: direct tiles with opt occupancies per
// thread (t, n) and tile-form tiles (t2, n2; none when the form is off).
struct EvalLists {
  const mdpvi::Tile* t;
  int n;
  const mdpvi::Tile* t2;
  int n2;
};

EvalLists eval_lists(const mdpvi_batch* b, int opt) {
  const int oi = opt_index(opt);
  if (batch_tile_on(b, 1))
    return {b->d_rtiles_all_nt[oi], static_cast<int>(b->rtiles_all_nt[oi].size()), b->d_et_tiles,
            static_cast<int>(b->et_tiles.size())};
  return {b->d_rtiles_all[oi], static_cast<int>(b->rtiles_all[oi].size()), nullptr, 0};
}

int ensure_batch_device(mdpvi_batch* b) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (b->device >= 0) {
    if (b->device != dev)
      return fail(MDPVI_EINVAL, "batch lives on device %d, current device is %d", b->device, dev);
    return MDPVI_OK;
  }
  const int n = b->n;
  std::vector<mdpvi::BatchInst> inst(n);
  int n_ctl = 0;
  for (int i = 0; i < n; ++i) {
    inst[i].M = b->models[i];
    inst[i].offset = b->offsets[i];
    inst[i].aoff = -1;
    inst[i].loff = -1;
    inst[i].lds = 0;
    inst[i].tocc = b->tocc[i];
    inst[i].eocc = b->eocc[i];
    inst[i].eoff = -1;
    inst[i].ctl = -1;
  }
  for (int32_t i : b->lds_list) inst[i].lds = 1;
  b->a_total = 0;
  for (int32_t i : b->round_list) {
    inst[i].aoff = b->a_total;
    b->a_total += b->models[i].n_occ + std::max<int64_t>(1, b->tocc[i]);
  }
  b->e_total = 0;
  for (int i = 0; i < n; ++i) {
    if (b->eocc[i] > 0) {
      inst[i].eoff = b->e_total;
      b->e_total += b->models[i].n_occ;
    }
  }
  // line tables for the instances whose adjoint rounds take the exact backup
  b->l_total = 0;
  for (int i = 0; i < n; ++i) {
    const mdpvi::Model& M = b->models[i];
    if (M.K <= mdpvi::kBatchExactK && M.J <= 3) {
      inst[i].loff = b->l_total;
      b->l_total += static_cast<int64_t>(M.K) * M.J * (M.n_occ / M.R);
    }
  }
  for (int i = 0; i < n; ++i) inst[i].ctl = i;
  n_ctl = n;
  auto dalloc = [&](void** p, size_t bytes) -> int {
    if (bytes == 0) bytes = 16;
    if (hipMalloc(p, bytes) != hipSuccess) {
      *p = nullptr;
      return fail(MDPVI_ENOMEM, "hipMalloc of %zu bytes failed", bytes);
    }
    return MDPVI_OK;
  };
  int rc;
  if ((rc = dalloc(reinterpret_cast<void**>(&b->d_inst), n * sizeof(mdpvi::BatchInst)))) return rc;
  if ((rc = dalloc(reinterpret_cast<void**>(&b->d_lds), b->lds_list.size() * sizeof(int32_t)))) return rc;
  if ((rc = dalloc(reinterpret_cast<void**>(&b->d_round), b->round_list.size() * sizeof(int32_t)))) return rc;
  if ((rc = dalloc(reinterpret_cast<void**>(&b->d_tiles), b->tiles.size() * sizeof(mdpvi::Tile)))) return rc;
  if ((rc = dalloc(reinterpret_cast<void**>(&b->d_tiles_all), b->tiles_all.size() * sizeof(mdpvi::Tile)))) return rc;
  if ((rc = dalloc(reinterpret_cast<void**>(&b->d_all), n * sizeof(int32_t)))) return rc;
  if ((rc = dalloc(reinterpret_cast<void**>(&b->d_tile_begin), (n + 1) * sizeof(int32_t)))) return rc;
  if ((rc = dalloc(reinterpret_cast<void**>(&b->d_flags), n * sizeof(int)))) return rc;
  if ((rc = dalloc(reinterpret_cast<void**>(&b->d_gpart),
                   mdpvi::batch_grad_partial_doubles(static_cast<int>(b->tiles_all.size()), b->maxJ) * sizeof(double))))
    return rc;
  if ((rc = dalloc(reinterpret_cast<void**>(&b->d_gout), static_cast<size_t>(n) * (2 * MDPVI_MAX_J + 3) * sizeof(double))))
    return rc;
  if ((rc = dalloc(reinterpret_cast<void**>(&b->d_ctl), std::max(n_ctl, 1) * sizeof(mdpvi::BatchCtl)))) return rc;
  if ((rc = dalloc(reinterpret_cast<void**>(&b->d_remaining), 3 * sizeof(int)))) return rc;
  if ((rc = dalloc(reinterpret_cast<void**>(&b->d_vt_tiles), b->vt_tiles.size() * sizeof(mdpvi::Tile)))) return rc;
  if ((rc = dalloc(reinterpret_cast<void**>(&b->d_et_tiles), b->et_tiles.size() * sizeof(mdpvi::Tile)))) return rc;
  for (int a = 0; a < 2; ++a) {
    if ((rc = dalloc(reinterpret_cast<void**>(&b->d_eact[a]), std::max<size_t>(b->et_tiles.size(), 1) * sizeof(mdpvi::Tile))))
      return rc;
    if ((rc = dalloc(reinterpret_cast<void**>(&b->d_E[a]), b->e_total * sizeof(double)))) return rc;
  }
  for (int oi = 0; oi < 3; ++oi)
    if ((rc = dalloc(reinterpret_cast<void**>(&b->d_rtiles_all_nt[oi]),
                     b->rtiles_all_nt[oi].size() * sizeof(mdpvi::Tile))))
      return rc;
  for (int a = 0; a < 2; ++a)
    if ((rc = dalloc(reinterpret_cast<void**>(&b->d_vact[a]), std::max<size_t>(b->vt_tiles.size(), 1) * sizeof(mdpvi::Tile))))
      return rc;
  for (int oi = 0; oi < 3; ++oi)
    if ((rc = dalloc(reinterpret_cast<void**>(&b->d_rtiles_nt[oi]), b->rtiles_nt[oi].size() * sizeof(mdpvi::Tile))))
      return rc;
  for (int a = 0; a < 2; ++a)
    if ((rc = dalloc(reinterpret_cast<void**>(&b->d_act[a]),
                     std::max<size_t>(b->rtiles_all[0].size(), 1) * sizeof(mdpvi::Tile))))
      return rc;
  if ((rc = dalloc(reinterpret_cast<void**>(&b->d_lines), b->l_total * sizeof(double)))) return rc;
  for (int a = 0; a < 2; ++a) {
    if ((rc = dalloc(reinterpret_cast<void**>(&b->d_A[a]), b->a_total * sizeof(double)))) return rc;
    if ((rc = dalloc(reinterpret_cast<void**>(&b->d_active[a]), n * sizeof(int)))) return rc;
  }
  if (hipHostMalloc(reinterpret_cast<void**>(&b->h_active), std::max(n, 1) * sizeof(int), hipHostMallocDefault) !=
      hipSuccess) {
    b->h_active = nullptr;
    return fail(MDPVI_ENOMEM, "hipHostMalloc of the batch flags failed");
  }
  for (int oi = 0; oi < 3; ++oi) {
    if ((rc = dalloc(reinterpret_cast<void**>(&b->d_rtiles[oi]), b->rtiles[oi].size() * sizeof(mdpvi::Tile))))
      return rc;
    if ((rc = dalloc(reinterpret_cast<void**>(&b->d_rtiles_all[oi]), b->rtiles_all[oi].size() * sizeof(mdpvi::Tile))))
      return rc;
  }
  if ((rc = dalloc(reinterpret_cast<void**>(&b->d_out), n * sizeof(mdpvi::BatchOut)))) return rc;
  if ((rc = dalloc(reinterpret_cast<void**>(&b->W), std::max<int64_t>(b->offsets[n], 1) * sizeof(float)))) return rc;
  if (hipHostMalloc(reinterpret_cast<void**>(&b->h_remaining), 3 * sizeof(int), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&b->h_out), n * sizeof(mdpvi::BatchOut), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&b->h_flags), n * sizeof(int), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&b->h_gout), static_cast<size_t>(n) * (2 * MDPVI_MAX_J + 3) * sizeof(double),
                    hipHostMallocDefault) != hipSuccess)
    return fail(MDPVI_ENOMEM, "hipHostMalloc of batch outputs failed");
  HIP_TRY(hipMemcpy(b->d_inst, inst.data(), n * sizeof(mdpvi::BatchInst), hipMemcpyHostToDevice));
  if (!b->lds_list.empty())
    HIP_TRY(hipMemcpy(b->d_lds, b->lds_list.data(), b->lds_list.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  if (!b->round_list.empty())
    HIP_TRY(hipMemcpy(b->d_round, b->round_list.data(), b->round_list.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  if (!b->tiles.empty())
    HIP_TRY(hipMemcpy(b->d_tiles, b->tiles.data(), b->tiles.size() * sizeof(mdpvi::Tile), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(b->d_tiles_all, b->tiles_all.data(), b->tiles_all.size() * sizeof(mdpvi::Tile),
                    hipMemcpyHostToDevice));
  for (int oi = 0; oi < 3; ++oi) {
    if (!b->rtiles[oi].empty())
      HIP_TRY(hipMemcpy(b->d_rtiles[oi], b->rtiles[oi].data(), b->rtiles[oi].size() * sizeof(mdpvi::Tile),
                        hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(b->d_rtiles_all[oi], b->rtiles_all[oi].data(), b->rtiles_all[oi].size() * sizeof(mdpvi::Tile),
                      hipMemcpyHostToDevice));
    if (!b->rtiles_nt[oi].empty())
      HIP_TRY(hipMemcpy(b->d_rtiles_nt[oi], b->rtiles_nt[oi].data(), b->rtiles_nt[oi].size() * sizeof(mdpvi::Tile),
                        hipMemcpyHostToDevice));
  }
  if (!b->vt_tiles.empty())
    HIP_TRY(hipMemcpy(b->d_vt_tiles, b->vt_tiles.data(), b->vt_tiles.size() * sizeof(mdpvi::Tile),
                      hipMemcpyHostToDevice));
  if (!b->et_tiles.empty())
    HIP_TRY(hipMemcpy(b->d_et_tiles, b->et_tiles.data(), b->et_tiles.size() * sizeof(mdpvi::Tile),
                      hipMemcpyHostToDevice));
  for (int oi = 0; oi < 3; ++oi)
    if (!b->rtiles_all_nt[oi].empty())
      HIP_TRY(hipMemcpy(b->d_rtiles_all_nt[oi], b->rtiles_all_nt[oi].data(),
                        b->rtiles_all_nt[oi].size() * sizeof(mdpvi::Tile), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(b->d_all, b->all_list.data(), n * sizeof(int32_t), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(b->d_tile_begin, b->tile_begin.data(), (n + 1) * sizeof(int32_t), hipMemcpyHostToDevice));
  HIP_TRY(hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking));
  HIP_TRY(hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming));
  HIP_TRY(hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming));
  HIP_TRY(hipEventCreate(&b->ev0));
  HIP_TRY(hipEventCreate(&b->ev1));
  b->device = dev;
  return MDPVI_OK;
}

}  // namespace

extern "C" {

int mdp_build_batch(const mdpvi_params* p, int32_t n, mdpvi_batch_t* out) {
  if (!p || !out) return fail(MDPVI_EINVAL, "NULL argument");
  *out = nullptr;
  if (n < 1) return fail(MDPVI_EINVAL, "n=%d must be >= 1", n);
  mdpvi_batch* b = new (std::nothrow) mdpvi_batch();
  if (!b) return fail(MDPVI_ENOMEM, "host allocation failed");
  b->n = n;
  b->models.resize(n);
  b->offsets.resize(n + 1);
  b->pairs.resize(n);
  b->offsets[0] = 0;
  for (int i = 0; i < n; ++i) {
    int rc = fill_model(&p[i], b->models[i], b->pairs[i]);
    if (rc) {
      std::string msg = g_err;
      delete b;
      return fail(rc, "instance %d: %s", i, msg.c_str());
    }
    if (b->models[i].n_states >= (int64_t{1} << 31)) {
      delete b;
      return fail(MDPVI_ERANGE, "instance %d has %lld states; batched instances must stay below 2^31", i,
                  (long long)b->models[i].n_states);
    }
    b->offsets[i + 1] = b->offsets[i] + b->models[i].n_states;
  }
  if (b->offsets[n] >= (int64_t{1} << 40)) {
    delete b;
    return fail(MDPVI_ERANGE, "batch holds too many states");
  }
  // LDS-resident when two FP32 copies fit the workgroup's LDS budget; the
  // rest are tiled for the round form.
  const int64_t lds_states = static_cast<int64_t>(mdpvi::kLdsBudget / (2 * sizeof(float)));
  std::vector<std::pair<double, int32_t>> cost;
  int64_t max_lds_n = 0;
  for (int i = 0; i < n; ++i) {
    const Model& M = b->models[i];
    if (M.n_states <= lds_states) {
      // sweeps to convergence grow like 1/(1 - gamma)
      cost.push_back({static_cast<double>(M.n_states) / (1.0 - M.gamma + 1e-3), i});
      max_lds_n = std::max(max_lds_n, M.n_states);
      b->lds_maxK = std::max(b->lds_maxK, M.K);
      b->lds_maxJ = std::max(b->lds_maxJ, M.J);
    } else {
      b->round_list.push_back(i);
      b->rnd_maxK = std::max(b->rnd_maxK, M.K);
      b->rnd_maxJ = std::max(b->rnd_maxJ, M.J);
      const uint32_t per = mdpvi::kBlock * mdpvi::kOccPerThread;
      for (uint32_t t = 0; t < static_cast<uint32_t>(M.n_occ); t += per) b->tiles.push_back({i, t});
    }
  }
  b->tile_begin.push_back(0);
  for (int i = 0; i < n; ++i) {
    const Model& M = b->models[i];
    b->all_list.push_back(i);
    b->maxK = std::max(b->maxK, M.K);
    b->maxJ = std::max(b->maxJ, M.J);
    const uint32_t per = mdpvi::kBlock * mdpvi::kOccPerThread;
    for (uint32_t t = 0; t < static_cast<uint32_t>(M.n_occ); t += per) b->tiles_all.push_back({i, t});
    b->tile_begin.push_back(static_cast<int32_t>(b->tiles_all.size()));
  }
  for (int oi = 0; oi < 3; ++oi) {
    const uint32_t per = static_cast<uint32_t>(mdpvi::kBlock) << oi;
    for (int i = 0; i < n; ++i) {
      const uint32_t n_occ = static_cast<uint32_t>(b->models[i].n_occ);
      const bool in_round = b->models[i].n_states > lds_states;
      for (uint32_t t = 0; t < n_occ; t += per) {
        if (in_round) b->rtiles[oi].push_back({i, t});
        b->rtiles_all[oi].push_back({i, t});
      }
    }
  }
  // value iteration's tile form: round-form instances of 4 or 5 hosts and
  // up to 3 classes of distinct sizes whose tile of (C+1)^3 occupancies
  // (values and arrival terms) fits the workgroup's LDS
  b->tocc.assign(n, 0);
  for (int32_t i : b->round_list) {
    const Model& M = b->models[i];
    const int64_t occ = static_cast<int64_t>(M.R) * M.R * M.R;
    const int64_t lds = (occ + 1) * 8 + occ * 4 * M.J;
    // buffer views hold byte offsets below 2^31
    const bool views = M.n_states < (int64_t{1} << 29) && M.n_occ + occ < (int64_t{1} << 28);
    if ((M.K == 4 || M.K == 5) && M.J <= 3 && M.n_sizes == M.J && views &&
        lds <= static_cast<int64_t>(mdpvi::kBatchTileLds))
      b->tocc[i] = static_cast<int32_t>(occ);
  }
  for (int32_t i : b->round_list) {
    const Model& M = b->models[i];
    if (b->tocc[i] > 0) {
      const uint32_t nt = static_cast<uint32_t>(M.n_occ / b->tocc[i]);
      for (uint32_t t = 0; t < nt; ++t) b->vt_tiles.push_back({i, t});
      b->vt_lds = std::max(b->vt_lds, static_cast<size_t>(b->tocc[i]) * 4 * M.J);
    } else {
      for (int oi = 0; oi < 3; ++oi) {
        const uint32_t per = static_cast<uint32_t>(mdpvi::kBlock) << oi;
        for (uint32_t t = 0; t < static_cast<uint32_t>(M.n_occ); t += per) b->rtiles_nt[oi].push_back({i, t});
      }
    }
  }
  // FP64 evaluation's tile form: instances of 4 or 5 hosts and up to 3
  // classes of distinct sizes whose (C+1)^3-occupancy tile has at least
  // 1,000 occupancies and whose FP64 values fit 32 KB of LDS (measured per
  // round against the direct form on batches of 4- and 5-host instances:
  // 16% faster at C+1 = 10..11; no faster at C+1 <= 9, whose tiles leave
  // lanes idle, nor at C+1 = 12..13 with 3 classes, whose 41-52 KB of LDS
  // allow three workgroups per CU)
  b->eocc.assign(n, 0);
  for (int i = 0; i < n; ++i) {
    const Model& M = b->models[i];
    const int64_t occ = static_cast<int64_t>(M.R) * M.R * M.R;
    const bool views = M.n_states < (int64_t{1} << 28);
    if ((M.K == 4 || M.K == 5) && M.J <= 3 && M.n_sizes == M.J && views && occ >= 1000 &&
        occ * 8 * M.J <= static_cast<int64_t>(mdpvi::kBatchEvalTileLds))
      b->eocc[i] = static_cast<int32_t>(occ);
  }
  for (int i = 0; i < n; ++i) {
    const Model& M = b->models[i];
    if (b->eocc[i] > 0) {
      const uint32_t nt = static_cast<uint32_t>(M.n_occ / b->eocc[i]);
      for (uint32_t t = 0; t < nt; ++t) b->et_tiles.push_back({i, t});
      b->et_lds = std::max(b->et_lds, static_cast<size_t>(b->eocc[i]) * 8 * M.J);
    } else {
      for (int oi = 0; oi < 3; ++oi) {
        const uint32_t per = static_cast<uint32_t>(mdpvi::kBlock) << oi;
        for (uint32_t t = 0; t < static_cast<uint32_t>(M.n_occ); t += per) b->rtiles_all_nt[oi].push_back({i, t});
      }
    }
  }
  // the exact-shape round backups' terms (the device-side exact_ok of each
  // operation): value iteration over the round-form instances, evaluation
  // and the adjoint over all
  b->exact_all[0] = b->exact_all[1] = b->exact_all[2] = true;
  for (int i = 0; i < n; ++i) {
    const Model& M = b->models[i];
    const bool shape = M.K <= mdpvi::kBatchExactK && M.J <= 3;
    if (M.n_states > lds_states && !(shape && M.n_sizes == M.J && M.n_states < (int64_t{1} << 29)))
      b->exact_all[0] = false;
    if (!(shape && M.n_states < (int64_t{1} << 28))) b->exact_all[1] = false;
    if (!shape) b->exact_all[2] = false;
  }
  std::sort(cost.begin(), cost.end(), [](auto& x, auto& y) { return x.first > y.first; });
  for (auto& c : cost) b->lds_list.push_back(c.second);
  b->lds_bytes = static_cast<size_t>(2 * max_lds_n) * sizeof(float);
  *out = b;
  return MDPVI_OK;
}

void mdp_free_batch(mdpvi_batch_t b) {
  if (!b) return;
  if (b->side) (void)hipStreamSynchronize(b->side);
  (void)hipFree(b->d_inst);
  (void)hipFree(b->d_lds);
  (void)hipFree(b->d_round);
  (void)hipFree(b->d_tiles);
  (void)hipFree(b->d_tiles_all);
  (void)hipFree(b->d_all);
  (void)hipFree(b->d_tile_begin);
  (void)hipFree(b->d_flags);
  (void)hipFree(b->d_gpart);
  (void)hipFree(b->d_gout);
  (void)hipFree(b->W2);
  if (b->h_flags) (void)hipHostFree(b->h_flags);
  if (b->h_gout) (void)hipHostFree(b->h_gout);
  (void)hipFree(b->d_ctl);
  (void)hipFree(b->d_remaining);
  (void)hipFree(b->d_act[0]);
  (void)hipFree(b->d_act[1]);
  (void)hipFree(b->d_A[0]);
  (void)hipFree(b->d_A[1]);
  (void)hipFree(b->d_lines);
  (void)hipFree(b->d_vt_tiles);
  (void)hipFree(b->d_et_tiles);
  for (int a = 0; a < 2; ++a) {
    (void)hipFree(b->d_eact[a]);
    (void)hipFree(b->d_E[a]);
  }
  for (int oi = 0; oi < 3; ++oi) (void)hipFree(b->d_rtiles_all_nt[oi]);
  (void)hipFree(b->d_vact[0]);
  (void)hipFree(b->d_vact[1]);
  for (int oi = 0; oi < 3; ++oi) (void)hipFree(b->d_rtiles_nt[oi]);
  (void)hipFree(b->d_active[0]);
  (void)hipFree(b->d_active[1]);
  if (b->h_active) (void)hipHostFree(b->h_active);
  for (int oi = 0; oi < 3; ++oi) {
    (void)hipFree(b->d_rtiles[oi]);
    (void)hipFree(b->d_rtiles_all[oi]);
  }
  (void)hipFree(b->d_out);
  (void)hipFree(b->W);
  if (b->h_remaining) (void)hipHostFree(b->h_remaining);
  if (b->h_out) (void)hipHostFree(b->h_out);
  if (b->side) (void)hipStreamDestroy(b->side);
  for (hipEvent_t e : {b->ev_fork, b->ev_join, b->ev0, b->ev1})
    if (e) (void)hipEventDestroy(e);
  delete b;
}

int32_t batch_num_instances(mdpvi_batch_t b) { return b ? b->n : -1; }

int64_t batch_num_states(mdpvi_batch_t b, int32_t i) {
  if (!b || i < -1 || i >= b->n) return -1;
  return i < 0 ? b->offsets[b->n] : b->models[i].n_states;
}

int64_t batch_feasible_pairs(mdpvi_batch_t b, int32_t i) {
  if (!b || i < -1 || i >= b->n) return -1;
  if (i >= 0) return b->pairs[i];
  int64_t t = 0;
  for (int64_t x : b->pairs) t += x;
  return t;
}

int batch_offsets(mdpvi_batch_t b, int64_t* offsets) {
  if (!b || !offsets) return fail(MDPVI_EINVAL, "NULL batch or offsets");
  std::memcpy(offsets, b->offsets.data(), (b->n + 1) * sizeof(int64_t));
  return MDPVI_OK;
}

int vi_solve_batch(mdpvi_batch_t b, float* V, double tol, int64_t max_iter, void* hip_stream,
                   mdpvi_stats* st, int64_t* iterations, double* residuals) {
  if (!b || !V) return fail(MDPVI_EINVAL, "NULL batch or value array");
  if (!(tol > 0)) return fail(MDPVI_EINVAL, "tol=%g must be > 0", tol);
  if (max_iter < 1) return fail(MDPVI_EINVAL, "max_iter=%lld must be >= 1", (long long)max_iter);
  int rc = ensure_batch_device(b);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const int n_round = static_cast<int>(b->round_list.size());
  const int n_lds = static_cast<int>(b->lds_list.size());
  HIP_TRY(mdpvi::launch_batch_ctl_init(b->d_ctl, b->d_round, n_round, b->d_remaining, b->d_flags, 0, s));
  HIP_TRY(hipEventRecord(b->ev0, s));
  HIP_TRY(hipEventRecord(b->ev_fork, s));
  HIP_TRY(hipStreamWaitEvent(b->side, b->ev_fork, 0));
  HIP_TRY(mdpvi::launch_batch_lds_vi(b->d_inst, b->d_lds, n_lds, b->lds_maxK, b->lds_maxJ, b->lds_bytes,
                                     V, tol, max_iter, b->d_out, b->side));
  HIP_TRY(hipEventRecord(b->ev_join, b->side));
  int64_t issued = 0;
  if (n_round > 0) {
    int64_t chunk = 8;
    const int opt = batch_opt(b, 0);
    const int oi = opt_index(opt);
    // every round-form instance's arrival terms (and -inf blocks)
    HIP_TRY(mdpvi::launch_batch_arrival_init(b->d_inst, b->d_rtiles[oi], static_cast<int>(b->rtiles[oi].size()), V,
                                             b->d_A[0], b->d_A[1], opt, s));
    // the tile form's instances, and the direct form's (the others, or all)
    const bool tile = batch_tile_on(b, 0);
    const mdpvi::Tile* vtiles = tile ? b->d_vt_tiles : nullptr;
    int nvt = tile ? static_cast<int>(b->vt_tiles.size()) : 0;
    const mdpvi::Tile* tiles = tile ? b->d_rtiles_nt[oi] : b->d_rtiles[oi];
    int nt = static_cast<int>(tile ? b->rtiles_nt[oi].size() : b->rtiles[oi].size()), cur = 0;
    while (issued < max_iter) {
      const int64_t m = std::min<int64_t>(chunk, max_iter - issued);
      for (int64_t k = 0; k < m; ++k) {
        HIP_TRY(mdpvi::launch_batch_vi_tile(b->d_inst, vtiles, nvt, b->vt_lds, V, b->W, b->d_ctl, b->d_remaining,
                                            issued + k, tol, b->d_A[0], b->d_A[1], s));
        HIP_TRY(mdpvi::launch_batch_round(b->d_inst, tiles, nt, b->rnd_maxK, b->rnd_maxJ, V, b->W, b->d_ctl,
                                          b->d_remaining, issued + k, tol, opt, b->d_A[0], b->d_A[1],
                                          b->exact_all[0], s));
      }
      issued += m;
      // drop the tiles of instances that have stopped from the next chunk
      HIP_TRY(mdpvi::launch_batch_compact(tiles, nt, b->d_ctl, b->d_act[cur], b->d_remaining + 1, s));
      HIP_TRY(mdpvi::launch_batch_compact(vtiles, nvt, b->d_ctl, b->d_vact[cur], b->d_remaining + 2, s));
      HIP_TRY(hipMemcpyAsync(b->h_remaining, b->d_remaining, 3 * sizeof(int), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      if (b->h_remaining[0] <= 0) break;
      tiles = b->d_act[cur];
      nt = b->h_remaining[1];
      vtiles = b->d_vact[cur];
      nvt = b->h_remaining[2];
      cur ^= 1;
      if (chunk < kMaxChunk) chunk *= 2;
    }
    HIP_TRY(mdpvi::launch_batch_round_finish(b->d_inst, b->d_round, n_round, V, b->W, b->d_ctl, issued,
                                             b->d_out, s));
  }
  HIP_TRY(hipStreamWaitEvent(s, b->ev_join, 0));
  HIP_TRY(hipMemcpyAsync(b->h_out, b->d_out, b->n * sizeof(mdpvi::BatchOut), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipEventRecord(b->ev1, s));
  HIP_TRY(hipEventSynchronize(b->ev1));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, b->ev0, b->ev1));
  int64_t max_it = 0, not_conv = 0, nan = 0;
  double backups = 0, bytes = 0, max_res = 0;
  for (int i = 0; i < b->n; ++i) {
    const mdpvi::BatchOut& o = b->h_out[i];
    if (iterations) iterations[i] = o.iterations;
    if (residuals) residuals[i] = o.residual;
    max_it = std::max<int64_t>(max_it, o.iterations);
    backups += static_cast<double>(b->pairs[i]) * o.iterations;
    bytes += 8.0 * b->models[i].n_states * o.iterations;
    if (std::isnan(o.residual)) ++nan;
    else if (!(o.residual < tol)) ++not_conv;
    if (!std::isnan(o.residual)) max_res = std::max(max_res, o.residual);
  }
  if (st) {
    st->iterations = max_it;
    st->residual_inf = max_res;
    st->bound_inf = 0.0;
    for (int i = 0; i < b->n; ++i)
      st->bound_inf = std::max(st->bound_inf, b->models[i].gamma / (1.0 - b->models[i].gamma) * b->h_out[i].residual);
    st->seconds = ms * 1e-3;
    st->backups = backups;
    st->bytes = bytes;
    st->sweep_seconds = 0.0;
  }
  if (nan) return fail(MDPVI_ENAN, "%lld instances produced a non-finite residual", (long long)nan);
  if (not_conv)
    return fail(MDPVI_ENOCONV, "%lld instances did not meet tol within max_iter", (long long)not_conv);
  return MDPVI_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- batch passes

namespace {

// Flags every instance whose policy has an infeasible action; returns the
// first such instance or -1.
int batch_check_policy(mdpvi_batch* b, const uint8_t* pi, hipStream_t s, int* bad_inst) {
  *bad_inst = -1;
  HIP_TRY(mdpvi::launch_batch_ctl_init(b->d_ctl, b->d_all, 0, b->d_remaining, b->d_flags, b->n, s));
  HIP_TRY(mdpvi::launch_batch_check(b->d_inst, b->d_tiles_all, static_cast<int>(b->tiles_all.size()), b->maxK,
                                    b->maxJ, pi, b->d_flags, s));
  HIP_TRY(hipMemcpyAsync(b->h_flags, b->d_flags, b->n * sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int i = 0; i < b->n; ++i)
    if (b->h_flags[i]) {
      *bad_inst = i;
      break;
    }
  return MDPVI_OK;
}

// Round-form loop over every instance: `round(j, tiles, n)` enqueues round j
// over the n tiles of the instances still running, `finish(issued)`
// writes back odd finals and the per-instance outputs.  Fills stats from them.
// With `active` (device int[n], nullable), only the instances with
// active[i] != 0 (n_active of them) are swept; the others keep their values
// and report 0 sweeps.
// The round loop over every instance (or the active ones): round(j, tiles,
// n, tiles2, n2) issues round j over the direct-form tiles and the
// tile-form tiles (tiles2: the evaluation's, or none), which are compacted
// to the instances still running after each chunk.
template <typename Round, typename Finish>
int batch_all_rounds(mdpvi_batch* b, const mdpvi::Tile* tiles, int nt, const mdpvi::Tile* tiles2, int nt2,
                     double tol, int64_t max_iter, hipStream_t s, mdpvi_stats* st, int64_t* iterations,
                     double* residuals, double bytes_per_state, Round round, Finish finish,
                     const int* active = nullptr, int n_active = 0) {
  int64_t issued = 0, chunk = 8;
  int cur = 0;
  if (active) {
    HIP_TRY(mdpvi::launch_batch_ctl_activate(b->d_ctl, active, b->n, b->d_remaining, n_active, s));
    HIP_TRY(mdpvi::launch_batch_compact(tiles, nt, b->d_ctl, b->d_act[cur], b->d_remaining + 1, s));
    HIP_TRY(mdpvi::launch_batch_compact(tiles2, nt2, b->d_ctl, b->d_eact[cur], b->d_remaining + 2, s));
    HIP_TRY(hipMemcpyAsync(b->h_remaining, b->d_remaining, 3 * sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    tiles = b->d_act[cur];
    nt = b->h_remaining[1];
    tiles2 = b->d_eact[cur];
    nt2 = b->h_remaining[2];
    cur ^= 1;
  } else {
    HIP_TRY(mdpvi::launch_batch_ctl_init(b->d_ctl, b->d_all, b->n, b->d_remaining, b->d_flags, 0, s));
  }
  HIP_TRY(hipEventRecord(b->ev0, s));
  while (issued < max_iter && nt + nt2 > 0) {
    const int64_t m = std::min<int64_t>(chunk, max_iter - issued);
    for (int64_t k = 0; k < m; ++k) HIP_TRY(round(issued + k, tiles, nt, tiles2, nt2));
    issued += m;
    // drop the tiles of instances that have stopped from the next chunk
    HIP_TRY(mdpvi::launch_batch_compact(tiles, nt, b->d_ctl, b->d_act[cur], b->d_remaining + 1, s));
    HIP_TRY(mdpvi::launch_batch_compact(tiles2, nt2, b->d_ctl, b->d_eact[cur], b->d_remaining + 2, s));
    HIP_TRY(hipMemcpyAsync(b->h_remaining, b->d_remaining, 3 * sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (b->h_remaining[0] <= 0) break;
    tiles = b->d_act[cur];
    nt = b->h_remaining[1];
    tiles2 = b->d_eact[cur];
    nt2 = b->h_remaining[2];
    cur ^= 1;
    if (chunk < kMaxChunk) chunk *= 2;
  }
  HIP_TRY(finish(issued));
  HIP_TRY(hipMemcpyAsync(b->h_out, b->d_out, b->n * sizeof(mdpvi::BatchOut), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipEventRecord(b->ev1, s));
  HIP_TRY(hipEventSynchronize(b->ev1));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, b->ev0, b->ev1));
  int64_t max_it = 0, not_conv = 0, nan = 0;
  double backups = 0, bytes = 0, max_res = 0, bound = 0;
  for (int i = 0; i < b->n; ++i) {
    const mdpvi::BatchOut& o = b->h_out[i];
    if (iterations) iterations[i] = o.iterations;
    if (residuals) residuals[i] = o.residual;
    max_it = std::max<int64_t>(max_it, o.iterations);
    backups += static_cast<double>(b->models[i].n_states) * o.iterations;
    bytes += bytes_per_state * b->models[i].n_states * o.iterations;
    if (std::isnan(o.residual)) {
      ++nan;
    } else {
      if (!(o.residual < tol)) ++not_conv;
      max_res = std::max(max_res, o.residual);
      bound = std::max(bound, b->models[i].gamma / (1.0 - b->models[i].gamma) * o.residual);
    }
  }
  if (st) {
    st->iterations = max_it;
    st->residual_inf = max_res;
    st->bound_inf = bound;
    st->seconds = ms * 1e-3;
    st->backups = backups;
    st->bytes = bytes;
    st->sweep_seconds = 0.0;
  }
  if (nan) return fail(MDPVI_ENAN, "%lld instances produced a non-finite residual", (long long)nan);
  if (not_conv) return fail(MDPVI_ENOCONV, "%lld instances did not meet tol within max_iter", (long long)not_conv);
  return MDPVI_OK;
}

int batch_args(mdpvi_batch* b, double tol, int64_t max_iter) {
  if (!(tol > 0)) return fail(MDPVI_EINVAL, "tol=%g must be > 0", tol);
  if (max_iter < 1) return fail(MDPVI_EINVAL, "max_iter=%lld must be >= 1", (long long)max_iter);
  return ensure_batch_device(b);
}

}  // namespace

extern "C" {

int policy_extract_batch(mdpvi_batch_t b, const float* V, uint8_t* pi, float* gap, void* hip_stream) {
  if (!b || !V || !pi) return fail(MDPVI_EINVAL, "NULL batch, value or policy array");
  int rc = ensure_batch_device(b);
  if (rc) return rc;
  HIP_TRY(mdpvi::launch_batch_extract(b->d_inst, b->d_tiles_all, static_cast<int>(b->tiles_all.size()), b->maxK,
                                      b->maxJ, V, false, pi, gap, static_cast<hipStream_t>(hip_stream)));
  return MDPVI_OK;
}

int policy_extract_batch_f64(mdpvi_batch_t b, const double* V, uint8_t* pi, float* gap, void* hip_stream) {
  if (!b || !V || !pi) return fail(MDPVI_EINVAL, "NULL batch, value or policy array");
  int rc = ensure_batch_device(b);
  if (rc) return rc;
  HIP_TRY(mdpvi::launch_batch_extract(b->d_inst, b->d_tiles_all, static_cast<int>(b->tiles_all.size()), b->maxK,
                                      b->maxJ, V, true, pi, gap, static_cast<hipStream_t>(hip_stream)));
  return MDPVI_OK;
}

int policy_greedy_batch(mdpvi_batch_t b, int32_t kind, uint8_t* pi, void* hip_stream) {
  if (!b || !pi) return fail(MDPVI_EINVAL, "NULL batch or policy array");
  if (kind != 0 && kind != 1) return fail(MDPVI_EINVAL, "kind=%d must be 0 or 1", kind);
  int rc = ensure_batch_device(b);
  if (rc) return rc;
  HIP_TRY(mdpvi::launch_batch_greedy(b->d_inst, b->d_tiles_all, static_cast<int>(b->tiles_all.size()), b->maxK,
                                     b->maxJ, kind, pi, static_cast<hipStream_t>(hip_stream)));
  return MDPVI_OK;
}

int policy_eval_batch(mdpvi_batch_t b, const uint8_t* pi, double* V, double tol, int64_t max_iter,
                      void* hip_stream, mdpvi_stats* st, int64_t* iterations, double* residuals) {
  if (!b || !pi || !V) return fail(MDPVI_EINVAL, "NULL batch, policy or value array");
  int rc = batch_args(b, tol, max_iter);
  if (rc) return rc;
  if (!b->W2) {
    if (hipMalloc(&b->W2, std::max<int64_t>(b->offsets[b->n], 1) * sizeof(double)) != hipSuccess) {
      b->W2 = nullptr;
      return fail(MDPVI_ENOMEM, "hipMalloc of the FP64 batch scratch failed");
    }
  }
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  int bad = -1;
  if ((rc = batch_check_policy(b, pi, s, &bad))) return rc;
  if (bad >= 0) return fail(MDPVI_EINVAL, "instance %d: policy has an infeasible action", bad);
  double* W = static_cast<double*>(b->W2);
  const int opt = batch_opt(b, 1);
  EvalLists L = eval_lists(b, opt);
  if (L.n2) HIP_TRY(mdpvi::launch_batch_eval_arrival_init(b->d_inst, L.t2, L.n2, V, b->d_E[0], s));
  return batch_all_rounds(
      b, L.t, L.n, L.t2, L.n2, tol, max_iter, s, st, iterations, residuals, 17.0,
      [&](long long j, const mdpvi::Tile* tiles, int n, const mdpvi::Tile* tiles2, int n2) {
        return mdpvi::launch_batch_eval_mixed(b->d_inst, tiles, n, tiles2, n2, b->et_lds, b->maxK, b->maxJ, pi, V, W,
                                              b->d_ctl, b->d_remaining, j, tol, opt, b->d_E[0], b->d_E[1],
                                              b->exact_all[1], s);
      },
      [&](int64_t issued) {
        return mdpvi::launch_batch_eval_finish(b->d_inst, b->d_all, b->n, V, W, b->d_ctl, issued, b->d_out, s);
      });
}

int policy_iteration_batch(mdpvi_batch_t b, uint8_t* pi, double* V, double eval_tol, int64_t eval_max_iter,
                           double improve_tol, int64_t max_rounds, void* hip_stream, mdpvi_stats* st,
                           int64_t* rounds) {
  if (!b || !pi || !V) return fail(MDPVI_EINVAL, "NULL batch, policy or value array");
  if (!(improve_tol >= 0) || std::isinf(improve_tol))
    return fail(MDPVI_EINVAL, "improve_tol=%g must be finite and >= 0", improve_tol);
  if (max_rounds < 1) return fail(MDPVI_EINVAL, "max_rounds=%lld must be >= 1", (long long)max_rounds);
  int rc = batch_args(b, eval_tol, eval_max_iter);
  if (rc) return rc;
  if (!b->W2) {
    if (hipMalloc(&b->W2, std::max<int64_t>(b->offsets[b->n], 1) * sizeof(double)) != hipSuccess) {
      b->W2 = nullptr;
      return fail(MDPVI_ENOMEM, "hipMalloc of the FP64 batch scratch failed");
    }
  }
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  int bad = -1;
  if ((rc = batch_check_policy(b, pi, s, &bad))) return rc;
  if (bad >= 0) return fail(MDPVI_EINVAL, "instance %d: policy has an infeasible action", bad);
  double* W = static_cast<double*>(b->W2);
  const int opt = batch_opt(b, 1);
  const EvalLists L = eval_lists(b, opt);
  const int n = b->n;
  const auto t0 = std::chrono::steady_clock::now();
  std::vector<int64_t> rr(n, 0);
  for (int i = 0; i < n; ++i) b->h_active[i] = 1;
  HIP_TRY(hipMemcpyAsync(b->d_active[0], b->h_active, n * sizeof(int), hipMemcpyHostToDevice, s));
  int n_active = n, a = 0;
  int64_t r = 0;
  mdpvi_stats tot{};
  while (n_active > 0 && r < max_rounds) {
    ++r;
    for (int i = 0; i < n; ++i)
      if (b->h_active[i]) ++rr[i];
    mdpvi_stats e{};
    if (L.n2) HIP_TRY(mdpvi::launch_batch_eval_arrival_init(b->d_inst, L.t2, L.n2, V, b->d_E[0], s));
    rc = batch_all_rounds(
        b, L.t, L.n, L.t2, L.n2, eval_tol, eval_max_iter, s, &e, nullptr, nullptr, 17.0,
        [&](long long j, const mdpvi::Tile* tiles, int nt, const mdpvi::Tile* tiles2, int nt2) {
          return mdpvi::launch_batch_eval_mixed(b->d_inst, tiles, nt, tiles2, nt2, b->et_lds, b->maxK, b->maxJ, pi, V,
                                                W, b->d_ctl, b->d_remaining, j, eval_tol, opt, b->d_E[0], b->d_E[1],
                                                b->exact_all[1], s);
        },
        [&](int64_t issued) {
          return mdpvi::launch_batch_eval_finish(b->d_inst, b->d_all, n, V, W, b->d_ctl, issued, b->d_out, s);
        },
        b->d_active[a], n_active);
    tot.iterations += e.iterations;
    tot.residual_inf = std::max(tot.residual_inf, e.residual_inf);
    tot.bound_inf = std::max(tot.bound_inf, e.bound_inf);
    tot.backups += e.backups;
    tot.bytes += e.bytes;
    if (rc != MDPVI_OK) break;
    // improvement of the instances just evaluated: an instance whose policy
    // does not change is done (its V is the value of its final policy)
    HIP_TRY(hipMemsetAsync(b->d_active[a ^ 1], 0, n * sizeof(int), s));
    HIP_TRY(mdpvi::launch_batch_improve_active(b->d_inst, b->d_tiles_all, static_cast<int>(b->tiles_all.size()),
                                               b->maxK, b->maxJ, V, pi, improve_tol, b->d_active[a],
                                               b->d_active[a ^ 1], s));
    HIP_TRY(hipMemcpyAsync(b->h_active, b->d_active[a ^ 1], n * sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    a ^= 1;
    n_active = 0;
    for (int i = 0; i < n; ++i) n_active += b->h_active[i] ? 1 : 0;
  }
  HIP_TRY(hipStreamSynchronize(s));
  tot.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (st) *st = tot;
  if (rounds) std::memcpy(rounds, rr.data(), n * sizeof(int64_t));
  if (rc != MDPVI_OK) return rc;
  if (n_active > 0)
    return fail(MDPVI_ENOCONV, "%d instances still change their policy after %lld rounds (max_rounds)", n_active,
                (long long)r);
  return MDPVI_OK;
}

int vi_adjoint_batch(mdpvi_batch_t b, const uint8_t* pi, const double* V_pi, float* w, double* grad,
                     double* objective, double tol, int64_t max_iter, void* hip_stream, mdpvi_stats* st,
                     int64_t* iterations) {
  if (!b || !pi || !V_pi || !w || !grad) return fail(MDPVI_EINVAL, "NULL batch, policy, value, adjoint or gradient");
  int rc = batch_args(b, tol, max_iter);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  int bad = -1;
  if ((rc = batch_check_policy(b, pi, s, &bad))) return rc;
  if (bad >= 0) return fail(MDPVI_EINVAL, "instance %d: policy has an infeasible action", bad);
  const int nt = static_cast<int>(b->tiles_all.size());
  const int opt = batch_opt(b, 2);
  rc = batch_all_rounds(
      b, b->d_rtiles_all[opt_index(opt)], static_cast<int>(b->rtiles_all[opt_index(opt)].size()), nullptr, 0, tol,
      max_iter, s, st, iterations, nullptr, 9.0,
      [&](long long j, const mdpvi::Tile* tiles, int n, const mdpvi::Tile*, int) {
        return mdpvi::launch_batch_adjoint_round(b->d_inst, tiles, n, b->maxK, b->maxJ, pi, w, b->W,
                                                 b->d_ctl, b->d_remaining, j, tol, opt, b->d_lines,
                                                 b->exact_all[2], s);
      },
      [&](int64_t issued) {
        return mdpvi::launch_batch_adjoint_finish(b->d_inst, b->d_all, b->n, w, b->W, b->d_ctl, issued, b->d_out,
                                                  s);
      });
  if (rc != MDPVI_OK && rc != MDPVI_ENOCONV) return rc;
  HIP_TRY(mdpvi::launch_batch_grad(b->d_inst, b->d_tiles_all, nt, b->d_tile_begin, b->n, b->maxK, b->maxJ, pi, V_pi,
                                   w, b->d_gpart, b->d_gout, s));
  const size_t row = 2 * MDPVI_MAX_J + 3;
  HIP_TRY(hipMemcpyAsync(b->h_gout, b->d_gout, b->n * row * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  size_t at = 0;
  for (int i = 0; i < b->n; ++i) {
    const int nth = 2 * b->models[i].J + 2;
    std::memcpy(grad + at, b->h_gout + i * row, nth * sizeof(double));
    at += nth;
    if (objective) objective[i] = b->h_gout[i * row + nth];
  }
  return rc;
}

int batch_set_round_form(mdpvi_batch_t b, int32_t op, int32_t opt) {
  if (!b) return fail(MDPVI_EINVAL, "NULL batch");
  if (op < 0 || op > 2) return fail(MDPVI_EINVAL, "operation %d outside 0..2", op);
  if (opt != 0 && opt != 1 && opt != 2 && opt != 4)
    return fail(MDPVI_EINVAL, "occupancies per thread %d not in {0, 1, 2, 4}", opt);
  b->round_opt[op] = opt;
  return MDPVI_OK;
}

int batch_round_forms(mdpvi_batch_t b, int32_t* opt) {
  if (!b || !opt) return fail(MDPVI_EINVAL, "NULL batch or output");
  for (int op = 0; op < 3; ++op) opt[op] = batch_opt(b, op);
  return MDPVI_OK;
}

int batch_set_tile_form(mdpvi_batch_t b, int32_t op, int32_t mode) {
  if (!b) return fail(MDPVI_EINVAL, "NULL batch");
  if (op < 0 || op > 1) return fail(MDPVI_EINVAL, "operation %d outside 0..1", op);
  if (mode < -1 || mode > 1) return fail(MDPVI_EINVAL, "mode=%d not in {-1, 0, 1}", mode);
  b->tile_mode[op] = mode;
  return MDPVI_OK;
}

int32_t batch_tile_form_instances(mdpvi_batch_t b, int32_t op) {
  if (!b || op < 0 || op > 1) return -1;
  if (!batch_tile_on(b, op)) return 0;
  int32_t c = 0;
  for (int32_t t : (op == 0 ? b->tocc : b->eocc)) c += t > 0 ? 1 : 0;
  return c;
}

int batch_autotune(mdpvi_batch_t b, int32_t trials, void* hip_stream, int32_t* opt, double* us) {
  if (!b) return fail(MDPVI_EINVAL, "NULL batch");
  if (trials < 1 || trials > 1000) return fail(MDPVI_EINVAL, "trials=%d outside [1, 1000]", trials);
  int rc = ensure_batch_device(b);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const int64_t N = std::max<int64_t>(b->offsets[b->n], 1);
  // inputs of the timed rounds: zero values and weights, the least-loaded
  // policy (feasible everywhere)
  float* v32 = nullptr;
  double* v64 = nullptr;
  double* w64 = nullptr;
  uint8_t* pol = nullptr;
  auto release = [&]() {
    (void)hipFree(v32);
    (void)hipFree(v64);
    (void)hipFree(w64);
    (void)hipFree(pol);
  };
  if (hipMalloc(&v32, N * sizeof(float)) != hipSuccess || hipMalloc(&v64, N * sizeof(double)) != hipSuccess ||
      hipMalloc(&w64, N * sizeof(double)) != hipSuccess || hipMalloc(&pol, N) != hipSuccess) {
    release();
    return fail(MDPVI_ENOMEM, "hipMalloc of the tuning buffers failed");
  }
  auto run = [&]() -> int {
    HIP_TRY(hipMemsetAsync(v32, 0, N * sizeof(float), s));
    HIP_TRY(hipMemsetAsync(v64, 0, N * sizeof(double), s));
    HIP_TRY(mdpvi::launch_batch_greedy(b->d_inst, b->d_tiles_all, static_cast<int>(b->tiles_all.size()), b->maxK,
                                       b->maxJ, 0, pol, s));
    for (int op = 0; op < 3; ++op) {
      const bool vi = op == 0;
      if (vi && b->rtiles[0].empty()) continue;   // every instance is solved in LDS
      int best = mdpvi::kOccPerThread;
      double best_us = 1e300;
      for (int oi = 0; oi < 3; ++oi) {
        const int o = 1 << oi;
        const mdpvi::Tile* tiles = vi ? b->d_rtiles[oi] : b->d_rtiles_all[oi];
        const int nt = static_cast<int>(vi ? b->rtiles[oi].size() : b->rtiles_all[oi].size());
        if (vi) HIP_TRY(mdpvi::launch_batch_arrival_init(b->d_inst, tiles, nt, v32, b->d_A[0], b->d_A[1], o, s));
        auto round = [&]() -> hipError_t {
          if (op == 0)
            return mdpvi::launch_batch_round(b->d_inst, tiles, nt, b->rnd_maxK, b->rnd_maxJ, v32, b->W, b->d_ctl,
                                             b->d_remaining, 0, 1.0, o, b->d_A[0], b->d_A[1], b->exact_all[0], s);
          if (op == 1)
            return mdpvi::launch_batch_eval_round(b->d_inst, tiles, nt, b->maxK, b->maxJ, pol, v64, w64, b->d_ctl,
                                                  b->d_remaining, 0, 1.0, o, b->exact_all[1], s);
          return mdpvi::launch_batch_adjoint_round(b->d_inst, tiles, nt, b->maxK, b->maxJ, pol, v32, b->W,
                                                   b->d_ctl, b->d_remaining, 0, 1.0, o, b->d_lines,
                                                   b->exact_all[2], s);
        };
        std::vector<float> ms(trials);
        for (int r = -1; r < trials; ++r) {   // r = -1: untimed first launch
          HIP_TRY(mdpvi::launch_batch_ctl_init(b->d_ctl, b->d_all, b->n, b->d_remaining, b->d_flags, 0, s));
          HIP_TRY(hipEventRecord(b->ev0, s));
          HIP_TRY(round());
          HIP_TRY(hipEventRecord(b->ev1, s));
          HIP_TRY(hipEventSynchronize(b->ev1));
          if (r >= 0) HIP_TRY(hipEventElapsedTime(&ms[r], b->ev0, b->ev1));
        }
        std::sort(ms.begin(), ms.end());
        const double t = ms[trials / 2] * 1e3;
        if (t < best_us) {
          best_us = t;
          best = o;
        }
      }
      tune_record_key(batch_tune_key(b, op), best, best_us);
      if (opt) opt[op] = best;
      if (us) us[op] = best_us;
      if (vi && !b->vt_tiles.empty()) {
        // the tile form for the instances it covers, the direct form with the
        // chosen occupancies per thread for the others
        const int oi = opt_index(best);
        const int nt = static_cast<int>(b->rtiles_nt[oi].size());
        const int nvt = static_cast<int>(b->vt_tiles.size());
        HIP_TRY(mdpvi::launch_batch_arrival_init(b->d_inst, b->d_rtiles[oi], static_cast<int>(b->rtiles[oi].size()),
                                                 v32, b->d_A[0], b->d_A[1], best, s));
        std::vector<float> ms(trials);
        for (int r = -1; r < trials; ++r) {
          HIP_TRY(mdpvi::launch_batch_ctl_init(b->d_ctl, b->d_all, b->n, b->d_remaining, b->d_flags, 0, s));
          HIP_TRY(hipEventRecord(b->ev0, s));
          HIP_TRY(mdpvi::launch_batch_vi_tile(b->d_inst, b->d_vt_tiles, nvt, b->vt_lds, v32, b->W, b->d_ctl,
                                              b->d_remaining, 0, 1.0, b->d_A[0], b->d_A[1], s));
          HIP_TRY(mdpvi::launch_batch_round(b->d_inst, b->d_rtiles_nt[oi], nt, b->rnd_maxK, b->rnd_maxJ, v32, b->W,
                                            b->d_ctl, b->d_remaining, 0, 1.0, best, b->d_A[0], b->d_A[1],
                                            b->exact_all[0], s));
          HIP_TRY(hipEventRecord(b->ev1, s));
          HIP_TRY(hipEventSynchronize(b->ev1));
          if (r >= 0) HIP_TRY(hipEventElapsedTime(&ms[r], b->ev0, b->ev1));
        }
        std::sort(ms.begin(), ms.end());
        const double t = ms[trials / 2] * 1e3;
        tune_record_key(batch_tune_key(b, 0) + "|tile", t < best_us ? 1 : 0, t);
        if (us && t < best_us) us[0] = t;
      }
      if (op == 1 && !b->et_tiles.empty()) {
        // the evaluation's tile form beside the winner's direct tiles
        const int oi = opt_index(best);
        const int nt = static_cast<int>(b->rtiles_all_nt[oi].size());
        const int net = static_cast<int>(b->et_tiles.size());
        HIP_TRY(mdpvi::launch_batch_eval_arrival_init(b->d_inst, b->d_et_tiles, net, v64, b->d_E[0], s));
        std::vector<float> ms(trials);
        for (int r = -1; r < trials; ++r) {
          HIP_TRY(mdpvi::launch_batch_ctl_init(b->d_ctl, b->d_all, b->n, b->d_remaining, b->d_flags, 0, s));
          HIP_TRY(hipEventRecord(b->ev0, s));
          HIP_TRY(mdpvi::launch_batch_eval_mixed(b->d_inst, b->d_rtiles_all_nt[oi], nt, b->d_et_tiles, net, b->et_lds,
                                                 b->maxK, b->maxJ, pol, v64, w64, b->d_ctl, b->d_remaining, 0, 1.0,
                                                 best, b->d_E[0], b->d_E[1], b->exact_all[1], s));
          HIP_TRY(hipEventRecord(b->ev1, s));
          HIP_TRY(hipEventSynchronize(b->ev1));
          if (r >= 0) HIP_TRY(hipEventElapsedTime(&ms[r], b->ev0, b->ev1));
        }
        std::sort(ms.begin(), ms.end());
        const double t = ms[trials / 2] * 1e3;
        tune_record_key(batch_tune_key(b, 1) + "|tile", t < best_us ? 1 : 0, t);
        if (us && t < best_us) us[1] = t;
      }
    }
    return MDPVI_OK;
  };
  rc = run();
  release();
  return rc;
}

}  // extern "C"

// ---------------------------------------------------------------- static bags of tasks

namespace {

int check_static(const int32_t* caps, const int32_t* need, const void* place, int64_t B, int32_t K, int64_t T,
                 double bvc, double btc, double gvc, const void* used, const void* totals,
                 const void* reward, const void* status) {
  if (B < 0 || T < 0) return fail(MDPVI_EINVAL, "B=%lld and T=%lld must be >= 0", (long long)B, (long long)T);
  if (K < 1 || K > MDPVI_STATIC_MAX_K) return fail(MDPVI_EINVAL, "K=%d must be in [1, %d]", K, MDPVI_STATIC_MAX_K);
  if (B > 4LL * 0x7fffffffLL) return fail(MDPVI_ERANGE, "B=%lld scenarios exceed the grid", (long long)B);
  if (T > 0 && B > (int64_t(1) << 62) / T) return fail(MDPVI_ERANGE, "B*T overflows");
  if (!is_finite(bvc) || !is_finite(btc) || !is_finite(gvc))
    return fail(MDPVI_EINVAL, "beta_vc, beta_tc and gamma_vc must be finite");
  if (B == 0) return MDPVI_OK;
  if (!caps || !used || !totals || !reward || !status) return fail(MDPVI_EINVAL, "NULL array");
  if (T > 0 && (!need || !place)) return fail(MDPVI_EINVAL, "NULL task array with T > 0");
  return MDPVI_OK;
}

}  // namespace

extern "C" {

int static_first_fit(const int32_t* caps, const int32_t* need, int64_t B, int32_t K, int64_t T,
                     double beta_vc, double beta_tc, double gamma_vc, int32_t* place, int32_t* used,
                     int64_t* totals, double* reward, int32_t* status, void* hip_stream) {
  const int rc = check_static(caps, need, place, B, K, T, beta_vc, beta_tc, gamma_vc, used, totals, reward,
                              status);
  if (rc != MDPVI_OK) return rc;
  HIP_TRY(mdpvi::launch_static_first_fit(B, K, T, caps, need, beta_vc, beta_tc, gamma_vc, place, used,
                                         reinterpret_cast<long long*>(totals), reward, status,
                                         static_cast<hipStream_t>(hip_stream)));
  return MDPVI_OK;
}

int static_score(const int32_t* caps, const int32_t* need, const int32_t* place, int64_t B, int32_t K,
                 int64_t T, double beta_vc, double beta_tc, double gamma_vc, int32_t* used, int64_t* totals,
                 double* reward, int32_t* status, void* hip_stream) {
  const int rc = check_static(caps, need, place, B, K, T, beta_vc, beta_tc, gamma_vc, used, totals, reward,
                              status);
  if (rc != MDPVI_OK) return rc;
  HIP_TRY(mdpvi::launch_static_score(B, K, T, caps, need, place, beta_vc, beta_tc, gamma_vc, used,
                                     reinterpret_cast<long long*>(totals), reward, status,
                                     static_cast<hipStream_t>(hip_stream)));
  return MDPVI_OK;
}

}  // extern "C"
