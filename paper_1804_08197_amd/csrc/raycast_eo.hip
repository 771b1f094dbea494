// raycast_eo.hip -- ray-casting kernel instances of the emission only model
// (every voxel type, channel count, kernel flavour and statistics mode).
#include "raycast_kernels.h"

namespace sg {

sg_status launch_raycast_emission(int bpv, int channels, const RenderArgs& a, bool stats,
                                  hipStream_t s) {
  return launch_model<kModelEmission>(bpv, channels, a, stats, s);
}

}  // namespace sg
