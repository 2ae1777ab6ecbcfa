// pf_tiled.hip -- face-sharing z-marching variant of the sweeps (in progress).
#include <hip/hip_runtime.h>

#include "pf_kernels_common.h"
#include "pf_launch.h"

namespace pfk {

hipError_t launch_phi_tiled(const LaunchSet&, int, bool, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_mu_tiled(const LaunchSet&, int, hipStream_t) { return hipErrorNotSupported; }

}  // namespace pfk
