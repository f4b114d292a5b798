// batch.hpp -- device descriptors of the batched forms.
#pragma once

#include "model.hpp"

namespace mdpvi {

constexpr int kLdsBlock = 1024;       // threads of an LDS-resident instance solve
constexpr int kBatchLanes = 8;        // residual words per instance (round form)
constexpr size_t kLdsBudget = 160 * 1024 - 1024;  // dynamic LDS per workgroup
constexpr int kBatchExactK = 5;       // host counts up to which the round kernels
                                      // carry exact-shape backups
constexpr size_t kBatchTileLds = 60 * 1024;   // dynamic LDS of a tile-form round workgroup
constexpr size_t kBatchEvalTileLds = 32 * 1024;   // ... of the evaluation's tile form

struct BatchInst {
  Model M;
  int64_t offset;   // first state of this instance in the concatenated arrays
  int64_t aoff;     // first entry of its arrival terms (n_occ + 1 doubles) in the
                    // value-iteration side arrays; -1 when it has none
  int64_t loff;     // first entry of its reset-line sums (K J n_occ / (C+1)
                    // doubles) in the adjoint's line table; -1 when none
  int64_t eoff;     // first entry of its FP64 arrival terms (n_occ doubles) in
                    // the evaluation's side arrays; -1 when none
  int32_t lds;      // 1: solved LDS-resident by one workgroup
  int32_t ctl;      // index of its round-form control block (-1 if none)
  int32_t tocc;     // > 0: its value-iteration rounds run in the tile form, with
                    // tiles of tocc = (C+1)^3 occupancies (its arrival side
                    // arrays then end in tocc -inf entries); 0: direct form
  int32_t eocc;     // > 0: its evaluation rounds run in the tile form, tiles of
                    // eocc = (C+1)^3 occupancies; 0: direct form
};

struct Tile {
  int32_t inst;
  uint32_t first;   // first occupancy of the tile (tile form: the tile's index)
};

struct BatchCtl {
  long long done_iter;
  long long pad[kResStride - 1];
  unsigned long long res[kResSlots][kBatchLanes][kResStride];
};

struct BatchOut {
  long long iterations;
  double residual;
};

}  // namespace mdpvi
