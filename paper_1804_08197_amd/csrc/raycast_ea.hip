// raycast_ea.hip -- ray-casting kernel instances of the emission-absorption model
// (every voxel type, channel count, kernel flavour and statistics mode).
#include "raycast_kernels.h"

namespace sg {

const void* raycast_kernel_absorption(int bpv, int channels, bool stats, bool gather,
                                      bool loop, bool mb) {
  return model_kernel<kModelAbsorption>(bpv, channels, stats, gather, loop, mb);
}

}  // namespace sg
