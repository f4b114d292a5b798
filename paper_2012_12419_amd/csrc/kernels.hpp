// kernels.hpp -- host-side launchers of the HIP kernels (internal to the
// library; the public surface is the C ABI in mdpvi.h).
#pragma once

#include "batch.hpp"
#include "model.hpp"

namespace mdpvi {

// 32-bit index arithmetic is used while every state index and every
// neighbour offset fits in 31 bits.
inline bool use_32bit_index(const Model& M) { return M.n_states < (int64_t{1} << 31); }

hipError_t launch_ctl_init(Ctl* ctl, double* res, hipStream_t s);

// V^{j+1} = T V^j (Vin -> Vout), residual into the words of sweep j; a
// no-op once the stopping test has passed.  slab_t > 0 selects the LDS slab
// form with that many low digits per slab (see slab_digits), 0 the direct form.
// A: the two FP64 arrival-term arrays (n_occ + kSentinel doubles each) of the
// exact-shape direct form (sweep j reads A[j % 2], writes A[(j + 1) % 2]);
// NULL uses the forms without them.
hipError_t launch_vi_sweep(const Model& M, const float* Vin, float* Vout, Ctl* ctl, double* res,
                           long long j, double tol, hipStream_t s, int slab_t, double* const* A);
// True when the exact-shape direct form (with arrival-term arrays) applies.
bool exact_shape(const Model& M);
// A0(o) = sum_e lambda_e/Lam V(o, e) for every occupancy; entries n_occ ..
// n_occ + kSentinel - 1 of A0 and A1 = -inf (each array holds n_occ +
// kSentinel doubles).
hipError_t launch_arrival_init(const Model& M, const float* V, double* A0, double* A1, hipStream_t s);
// Workgroups of one value-iteration sweep in the given form.
uint32_t vi_sweep_grid(const Model& M, int slab_t);

// LDS bytes per slab and the fewest slabs (workgroups) a slab depth may leave.
constexpr uint64_t kSlabLds = 40 * 1024;
constexpr uint64_t kMinSlabs = 512;
int slab_digits(const Model& M);

// Tile form (tile_vi.hip, tile_eval.hip).  *_shape fills S and returns
// false when the form does not apply to M.  The value-iteration tile reads
// and writes the FP64 arrival-term arrays like the exact-shape direct form
// (n_occ + kSentinel doubles each); the evaluation tile uses two FP64
// arrival-term arrays of n_occ doubles, the first set from the initial
// iterate by launch_eval_arrival_init.
struct TileShape;
bool vi_tile_shape(const Model& M, TileShape* S);
hipError_t launch_vi_tile(const Model& M, const TileShape& S, const float* Vin, float* Vout, const double* Ain,
                          double* Aout, Ctl* ctl, double* res, long long j, double tol, hipStream_t s);
// Block-asynchronous passes on tiles (two LDS images each): `inner`
// episodes per pass, successors outside the tile from the previous pass.
bool vi_bsdi_shape(const Model& M, TileShape* S);
hipError_t launch_vi_bsdi(const Model& M, const TileShape& S, int inner, const float* Vin, float* Vout,
                          const double* Ain, double* Aout, Ctl* ctl, double* res, long long j, double tol,
                          hipStream_t s);
// Row form of the value-iteration tile sweep (row_vi.hip): the tiles of T = 3,
// four consecutive occupancies along digit 0 per lane; same arrival-term
// arrays as the tile form.
bool vi_row_shape(const Model& M, TileShape* S);
hipError_t launch_vi_row(const Model& M, const TileShape& S, const float* Vin, float* Vout, const double* Ain,
                         double* Aout, Ctl* ctl, double* res, long long j, double tol, hipStream_t s);
bool eval_tile_shape(const Model& M, TileShape* S);
hipError_t launch_eval_arrival_init(const Model& M, const double* V, double* A, hipStream_t s);
hipError_t launch_eval_tile(const Model& M, const TileShape& S, const uint8_t* pi, const double* Vin,
                            double* Vout, const double* Ain, double* Aout, Ctl* ctl, double* res, long long j,
                            double tol, hipStream_t s);

// Greedy extraction from FP32 or FP64 values.
hipError_t launch_extract_f32(const Model& M, const float* V, uint8_t* pi, float* gap,
                              hipStream_t s);
hipError_t launch_extract_f64(const Model& M, const double* V, uint8_t* pi, float* gap,
                              hipStream_t s);

// ctl->flag := 1 if some pi entry is not a feasible action.
hipError_t launch_policy_check(const Model& M, const uint8_t* pi, Ctl* ctl, hipStream_t s);
// Policy improvement: pi_out = pi_in where no action beats the current one's
// FP64 Q (from V) by more than tol, the lowest-index argmax elsewhere.
hipError_t launch_improve(const Model& M, const double* V, const uint8_t* pi_in, uint8_t* pi_out, double tol,
                          hipStream_t s);
// ctl->flag := 1 if the n-byte arrays a and b differ.
hipError_t launch_policy_diff(uint64_t n, const uint8_t* a, const uint8_t* b, Ctl* ctl, hipStream_t s);

// One fixed-policy FP64 sweep V^{j+1} = r_pi + gamma P_pi V^j.
hipError_t launch_eval_sweep(const Model& M, const uint8_t* pi, const double* Vin, double* Vout,
                             Ctl* ctl, double* res, long long j, double tol, hipStream_t s);
// Workgroups of one generic-form evaluation or adjoint sweep (4 occupancies
// per thread), and of the evaluation sweep actually launched.
uint32_t occ_sweep_grid(const Model& M);
uint32_t eval_sweep_grid(const Model& M);

// Greedy heuristic policies (0 least-loaded, 1 first-fit).
hipError_t launch_greedy(const Model& M, int kind, uint8_t* pi, hipStream_t s);

// One transposed (adjoint) sweep w^{j+1} = c + gamma P_pi^T w^j, 1-norm
// residual.  form: kAdjointGroup (group form: whole (C+1)^2-occupancy groups
// per workgroup, low-digit neighbours through LDS), kAdjointExact + OPT
// (exact-shape kernels) or OPT (generic kernels), OPT in {1, 2, 4}
// occupancies per thread; 0 automatic.
constexpr int kAdjointExact = 16;
constexpr int kAdjointGroup = 32;
bool adjoint_exact_shape(const Model& M);
bool adjoint_group_shape(const Model& M);
hipError_t launch_adjoint_group(const Model& M, const uint8_t* pi, const float* win, float* wout, Ctl* ctl,
                                double* res, long long j, double tol, hipStream_t s);

int adjoint_auto_form(const Model& M);
bool adjoint_form_valid(const Model& M, int form);
hipError_t launch_adjoint_sweep(const Model& M, int form, const uint8_t* pi, const float* win, float* wout,
                                Ctl* ctl, double* res, long long j, double tol, hipStream_t s);

// Doubles of workgroup partials needed by launch_grad.
size_t grad_partial_doubles(const Model& M);

// out[0..2J+1] = dJ/dtheta, out[2J+2] = J (device pointers).
hipError_t launch_grad(const Model& M, const uint8_t* pi, const double* V, const float* w,
                       double* partial, double* out, hipStream_t s);

// out[0] = J = sum_e c_e V(0, e) (device pointer).
hipError_t launch_objective(const Model& M, const double* V, double* out, hipStream_t s);

// Batched forms (batch.hip).
hipError_t launch_batch_lds_vi(const BatchInst* insts, const int32_t* list, int n_list, int maxK,
                               int maxJ, size_t lds_bytes, float* V, double tol, long long max_iter,
                               BatchOut* out, hipStream_t s);
// Control blocks for a round loop over the instances with active[i] != 0
// (the others count as stopped before their first sweep).
hipError_t launch_batch_ctl_activate(BatchCtl* ctl, const int* active, int n, int* remaining, int n_active,
                                     hipStream_t s);
// In-place FP64 policy improvement (tolerance tol) of the tiles' instances
// with active[inst] != 0 (tiles of kBlock * kOccPerThread occupancies);
// changed[inst] := 1 where an action changed.
hipError_t launch_batch_improve_active(const BatchInst* insts, const Tile* tiles, int n_tiles, int maxK, int maxJ,
                                       const double* V, uint8_t* pi, double tol, const int* active, int* changed,
                                       hipStream_t s);
// The tiles of `in` whose instance has not stopped, into `out`; their count
// into *n_out.
hipError_t launch_batch_compact(const Tile* in, int n_in, const BatchCtl* ctl, Tile* out, int* n_out,
                                hipStream_t s);
hipError_t launch_batch_ctl_init(BatchCtl* ctl, const int32_t* list, int n_list, int* remaining,
                                 int* flags, int n_flags, hipStream_t s);
// One round of value iteration, FP64 evaluation or the adjoint over the
// given tiles (kBlock * opt occupancies each, opt in 1..kOccPerThread).
// Value iteration's round reads and writes the FP64 arrival terms of the
// instances with side arrays in A0/A1 (ping-pong like V/W; nullptr: every
// instance takes the backup without them).  all_exact (every round
// launcher): every instance of the tiles meets the exact-shape backup's
// terms (at most kBatchExactK hosts, 3 classes; value iteration: distinct
// sizes and side arrays; the adjoint: a line table), which selects a kernel
// without the generic backup (fewer registers).
hipError_t launch_batch_round(const BatchInst* insts, const Tile* tiles, int n_tiles, int maxK,
                              int maxJ, float* V, float* W, BatchCtl* ctl, int* remaining,
                              long long j, double tol, int opt, double* A0, double* A1, bool all_exact,
                              hipStream_t s);
// Value iteration's round in the tile form over tiles {inst, tile index} of
// instances with tocc > 0 (K in 4..5, J <= 3 distinct sizes); lds: bytes of
// dynamic LDS, at least J * tocc * 4 for every listed instance and at most
// kBatchTileLds.
hipError_t launch_batch_vi_tile(const BatchInst* insts, const Tile* tiles, int n_tiles, size_t lds, float* V,
                                float* W, BatchCtl* ctl, int* remaining, long long j, double tol, double* A0,
                                double* A1, hipStream_t s);
// FP64 evaluation's round in the tile form over tiles {inst, tile index} of
// instances with eocc > 0; E0/E1: the evaluation's arrival side arrays
// (ping-pong like V/W, E0 initialised by launch_batch_eval_arrival_init);
// lds: bytes of dynamic LDS, at least J * eocc * 8 for every listed
// instance and at most kBatchTileLds.
hipError_t launch_batch_eval_tile(const BatchInst* insts, const Tile* tiles, int n_tiles, size_t lds,
                                  const uint8_t* pi, double* V, double* W, BatchCtl* ctl, int* remaining,
                                  long long j, double tol, double* E0, double* E1, hipStream_t s);
hipError_t launch_batch_eval_arrival_init(const BatchInst* insts, const Tile* tiles, int n_tiles, const double* V,
                                          double* E0, hipStream_t s);
// One evaluation round over direct-form tiles and tile-form tiles: a single
// launch carrying both kinds of workgroup when the batch's instances all
// have at most kBatchExactK hosts and 3 classes, else the two launches.
hipError_t launch_batch_eval_mixed(const BatchInst* insts, const Tile* dtiles, int n_direct, const Tile* ttiles,
                                   int n_tile, size_t lds, int maxK, int maxJ, const uint8_t* pi, double* V,
                                   double* W, BatchCtl* ctl, int* remaining, long long j, double tol, int opt,
                                   double* E0, double* E1, bool all_exact, hipStream_t s);
// The arrival terms of V (the initial iterate) into A0, the -inf entries
// into A0 and A1, for the instances of the tiles that have side arrays.
hipError_t launch_batch_arrival_init(const BatchInst* insts, const Tile* tiles, int n_tiles, const float* V,
                                     double* A0, double* A1, int opt, hipStream_t s);
hipError_t launch_batch_eval_round(const BatchInst* insts, const Tile* tiles, int n_tiles, int maxK,
                                   int maxJ, const uint8_t* pi, double* V, double* W, BatchCtl* ctl,
                                   int* remaining, long long j, double tol, int opt, bool all_exact,
                                   hipStream_t s);
// The adjoint's round: with a line table (lines != nullptr; the instances'
// loff entries) the reset-line sums of the round's input are written to it
// first and the exact backups read them; nullptr: every instance sums its
// lines itself (the generic backup).
hipError_t launch_batch_adjoint_round(const BatchInst* insts, const Tile* tiles, int n_tiles, int maxK,
                                      int maxJ, const uint8_t* pi, float* w, float* W, BatchCtl* ctl,
                                      int* remaining, long long j, double tol, int opt, double* lines,
                                      bool all_exact, hipStream_t s);
hipError_t launch_batch_round_finish(const BatchInst* insts, const int32_t* list, int n_list,
                                     float* V, const float* W, BatchCtl* ctl, long long issued,
                                     BatchOut* out, hipStream_t s);
hipError_t launch_batch_eval_finish(const BatchInst* insts, const int32_t* list, int n_list,
                                    double* V, const double* W, BatchCtl* ctl, long long issued,
                                    BatchOut* out, hipStream_t s);
hipError_t launch_batch_adjoint_finish(const BatchInst* insts, const int32_t* list, int n_list,
                                       float* w, const float* W, BatchCtl* ctl, long long issued,
                                       BatchOut* out, hipStream_t s);
hipError_t launch_batch_extract(const BatchInst* insts, const Tile* tiles, int n_tiles, int maxK,
                                int maxJ, const void* V, bool f64, uint8_t* pi, float* gap,
                                hipStream_t s);
hipError_t launch_batch_greedy(const BatchInst* insts, const Tile* tiles, int n_tiles, int maxK, int maxJ,
                               int kind, uint8_t* pi, hipStream_t s);
hipError_t launch_batch_check(const BatchInst* insts, const Tile* tiles, int n_tiles, int maxK, int maxJ,
                              const uint8_t* pi, int* flags, hipStream_t s);
size_t batch_grad_partial_doubles(int n_tiles, int maxJ);
hipError_t launch_batch_grad(const BatchInst* insts, const Tile* tiles, int n_tiles, const int32_t* tile_begin,
                             int n, int maxK, int maxJ, const uint8_t* pi, const double* V, const float* w,
                             double* partial, double* out, hipStream_t s);

// Static bag-of-task placement (static_bot.hip): B scenarios of K <= 64 VCs
// and T task slots, one wavefront per scenario.
hipError_t launch_static_first_fit(long long B, int K, long long T, const int32_t* caps, const int32_t* need,
                                   double bvc, double btc, double gvc, int32_t* place, int32_t* used,
                                   long long* totals, double* reward, int32_t* status, hipStream_t s);
hipError_t launch_static_score(long long B, int K, long long T, const int32_t* caps, const int32_t* need,
                               const int32_t* place, double bvc, double btc, double gvc, int32_t* used,
                               long long* totals, double* reward, int32_t* status, hipStream_t s);

}  // namespace mdpvi
