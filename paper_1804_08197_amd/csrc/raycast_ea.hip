// raycast_ea.hip -- ray-casting kernel instances of the emission absorption model
// (every voxel type, channel count, kernel flavour and statistics mode).
#include "raycast_kernels.h"

namespace sg {

sg_status launch_raycast_absorption(int bpv, int channels, const RenderArgs& a, bool stats,
                                    hipStream_t s) {
  return launch_model<kModelAbsorption>(bpv, channels, a, stats, s);
}

}  // namespace sg
