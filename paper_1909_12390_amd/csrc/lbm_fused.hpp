// Fused one-launch schedule of the step (filled in below the two-pass path).
#pragma once
#include "lbm_kernels.hpp"

namespace lbmk {

struct FusedShape {
  int tx, ty, chunk;   // cross-section tile and marching chunk length
  int ntiles, nchunks;
};

inline bool fused_supported(int) { return false; }

inline FusedShape fused_shape(int, int, int, int) { return FusedShape{0, 0, 0, 0, 0}; }

template <int LAT, int NC, int ST>
void launch_fused(const KParams&, const Pops<ST>&, const Pops<ST>&, const FusedShape&, hipStream_t) {}

}  // namespace lbmk
