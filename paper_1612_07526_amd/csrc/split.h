// Split-precision update (split.hip).
#pragma once
#include "phdc_internal.h"

namespace phdc {

struct SplitBufs {
  __bf16* aslice;  // per merge at nsl * x_off: [slice][row][kd rounded to 8] for each half
  __bf16* bslice;  // per merge at nsl * x_off: [slice][grouped row][K rounded to 8]
  int32_t* erow;   // n_total: row exponents
  int32_t* fcol;   // n_total: column exponents
  int32_t kgroups; // k-group stride of the A slicer
  int32_t rgroups; // row stride of the B slicer
};

constexpr int kSplitKGroups = 32;
constexpr int kSplitRGroups = 64;

// Row of element r held by lane group lg in a 16x16 FP32 MFMA result block.
__host__ __device__ constexpr int kSplitRow(int lg, int r) { return 4 * lg + r; }

void launch_split_update(const MergeDesc* descs, int nm, const LevelMaps& maps, const Scratch& S,
                         const SplitBufs& B, int nsl, hipStream_t s);

}  // namespace phdc
