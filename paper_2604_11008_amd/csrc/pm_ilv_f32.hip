// pm_ilv_f32.hip -- launchers of the fused and advance kernels with float
// velocities on collocated fields whose three components are interleaved node by
// node (every launch shape, halo and drag-law variant).
#include "pm_device.h"

namespace pm {

#define PM_STEP_CASE(W, I)                                                             \
    if (sh.wg == W && sh.items == I)                                                   \
        return Kern<W, I>::step_ft<float, kFieldIlv>(a, grid, st);

hipError_t launch_step_ilv_f32(const KArgs &a, Shape sh, int grid, hipStream_t st)
{
    PM_SHAPES(PM_STEP_CASE)
    return hipErrorInvalidValue;
}

#define PM_ADV_CASE(W, I)                                                              \
    if (sh.wg == W && sh.items == I)                                                   \
        return Kern<W, I>::advance_ft<float, kFieldIlv>(a, grid, st);

hipError_t launch_advance_ilv_f32(const KArgs &a, Shape sh, int grid, hipStream_t st)
{
    PM_SHAPES(PM_ADV_CASE)
    return hipErrorInvalidValue;
}

#define PM_OCC_CASE(W, I)                                                              \
    if (sh.wg == W && sh.items == I)                                                   \
        return Kern<W, I>::occupancy_ft<float, kFieldIlv>(halo, nonlinear);

int step_occupancy_ilv_f32(Shape sh, bool halo, bool nonlinear)
{
    PM_SHAPES(PM_OCC_CASE)
    return 1;
}

}  // namespace pm
