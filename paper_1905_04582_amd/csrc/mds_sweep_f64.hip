// FP64 instantiations of the pair sweep (Y stored and processed in FP64).
#include "mds_sweep.inc.h"

namespace mds {
hipError_t launch_sweep_f64(int d, bool grad, const Tiling& t, const SweepArgs& a, hipStream_t s,
                            hipEvent_t start, hipEvent_t stop)
{
    return launch_sweep_t<double>(d, grad, t, a, s, start, stop);
}

hipError_t launch_batch_sweep_f64(bool grad, int maxd, const BatchProblem* probs, int32_t count,
                                 int64_t total_tiles, unsigned long long* cursor, int waves,
                                 size_t lds, int grid, hipStream_t s)
{
    return launch_batch_sweep_t<double>(grad, maxd, probs, count, total_tiles, cursor, waves, lds,
                                     grid, s);
}

int batch_sweep_blocks_per_cu_f64(bool grad, int maxd, int waves, size_t lds)
{
    return batch_sweep_blocks_per_cu<double>(grad, maxd, waves, lds);
}
}  // namespace mds
