// Storage of each spectra form in input sample order (the layouts hcg_grid
// takes): element bytes, whether the form carries one scale per channel, and
// whether a low plane follows the high one.
#pragma once

#include <cstddef>

#include "hcg.h"

namespace hcg {

inline size_t form_elem(int dtype) {
  return dtype == HCG_F32 ? 4 : (dtype == HCG_FP8E4M3_SCALED || dtype == HCG_FP8E4M3_SPLIT) ? 1 : 2;
}
inline bool form_scaled(int dtype) {
  return dtype == HCG_F16_SCALED || dtype == HCG_FP8E4M3_SCALED || dtype == HCG_FP8E4M3_SPLIT;
}
inline bool form_split(int dtype) { return dtype == HCG_BF16_SPLIT || dtype == HCG_FP8E4M3_SPLIT; }

}  // namespace hcg
