// pm_staged_ilv_f64.hip -- launchers of the per-stage migration kernels with
// double velocities on node-interleaved fields (both stages, every launch shape,
// halo and drag law).
#include "pm_device.h"

namespace pm {

#define PM_STAGE_CASE(W, I)                                                            \
    if (sh.wg == W && sh.items == I)                                                   \
        return stage == 1 ? Kern<W, I>::stage_ft<double, 1, kFieldIlv>(a, grid, st)      \
                          : Kern<W, I>::stage_ft<double, 2, kFieldIlv>(a, grid, st);

hipError_t launch_stage_ilv_f64(const KArgs &a, Shape sh, int stage, int grid, hipStream_t st)
{
    PM_STAGE_SHAPES(PM_STAGE_CASE)
    return hipErrorInvalidValue;
}

#define PM_STAGE_OCC_CASE(W, I)                                                        \
    if (sh.wg == W && sh.items == I)                                                   \
        return stage == 1 ? Kern<W, I>::stage_occ_ft<double, 1, kFieldIlv>(halo, nonlinear) \
                          : Kern<W, I>::stage_occ_ft<double, 2, kFieldIlv>(halo, nonlinear);

int stage_occupancy_ilv_f64(Shape sh, bool halo, bool nonlinear, int stage)
{
    PM_STAGE_SHAPES(PM_STAGE_OCC_CASE)
    return 1;
}

}  // namespace pm
