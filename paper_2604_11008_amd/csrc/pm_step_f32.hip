// pm_step_f32.hip -- launchers of the fused and advance kernels with float
// velocities on collocated fields stored as one array per component (every
// launch shape, halo and drag-law variant).
#include "pm_device.h"

namespace pm {

#define PM_STEP_CASE(W, I)                                                             \
    if (sh.wg == W && sh.items == I)                                                   \
        return Kern<W, I>::step_ft<float, kFieldSplit>(a, grid, st);

hipError_t launch_step_f32(const KArgs &a, Shape sh, int grid, hipStream_t st)
{
    if (a.f.stagger)
        return launch_step_mac_f32(a, sh, grid, st);
    if (a.f.layout)
        return launch_step_ilv_f32(a, sh, grid, st);
    PM_SHAPES(PM_STEP_CASE)
    return hipErrorInvalidValue;
}

#define PM_ADV_CASE(W, I)                                                              \
    if (sh.wg == W && sh.items == I)                                                   \
        return Kern<W, I>::advance_ft<float, kFieldSplit>(a, grid, st);

hipError_t launch_advance_f32(const KArgs &a, Shape sh, int grid, hipStream_t st)
{
    if (a.f.stagger)
        return launch_advance_mac_f32(a, sh, grid, st);
    if (a.f.layout)
        return launch_advance_ilv_f32(a, sh, grid, st);
    PM_SHAPES(PM_ADV_CASE)
    return hipErrorInvalidValue;
}

#define PM_OCC_CASE(W, I)                                                              \
    if (sh.wg == W && sh.items == I)                                                   \
        return Kern<W, I>::occupancy_ft<float, kFieldSplit>(halo, nonlinear);

int step_occupancy_f32(Shape sh, bool halo, bool nonlinear, int arr)
{
    if (arr == kFieldMac)
        return step_occupancy_mac_f32(sh, halo, nonlinear);
    if (arr == kFieldIlv)
        return step_occupancy_ilv_f32(sh, halo, nonlinear);
    PM_SHAPES(PM_OCC_CASE)
    return 1;
}

}  // namespace pm
