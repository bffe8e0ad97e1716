// FP64 instantiations of the pair sweep (Y stored and processed in FP64).
#include "mds_sweep.inc.h"

namespace mds {
hipError_t launch_sweep_f64(int d, bool grad, const Tiling& t, const SweepArgs& a, hipStream_t s)
{
    return launch_sweep_t<double>(d, grad, t, a, s);
}
}  // namespace mds
