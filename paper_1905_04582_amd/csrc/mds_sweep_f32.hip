// FP32 instantiations of the pair sweep (Y stored in FP32, pair arithmetic in
// FP32, pair differences formed and all cross-lane sums finished in FP64).
#include "mds_sweep.inc.h"

namespace mds {
hipError_t launch_sweep_f32(int d, bool grad, const Tiling& t, const SweepArgs& a, hipStream_t s)
{
    return launch_sweep_t<float>(d, grad, t, a, s);
}
}  // namespace mds
