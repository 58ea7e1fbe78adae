// pm_staged_f32.hip -- launchers of the per-stage migration kernels with
// float velocities on fields stored as one array per component (both stages,
// every launch shape, halo and drag law).
#include "pm_device.h"

namespace pm {

#define PM_STAGE_CASE(W, I)                                                            \
    if (sh.wg == W && sh.items == I)                                                   \
        return stage == 1 ? Kern<W, I>::stage_ft<float, 1, kFieldSplit>(a, grid, st)                 \
                          : Kern<W, I>::stage_ft<float, 2, kFieldSplit>(a, grid, st);

hipError_t launch_stage_f32(const KArgs &a, Shape sh, int stage, int grid, hipStream_t st)
{
    if (a.f.layout)
        return launch_stage_ilv_f32(a, sh, stage, grid, st);
    PM_STAGE_SHAPES(PM_STAGE_CASE)
    return hipErrorInvalidValue;
}

#define PM_STAGE_OCC_CASE(W, I)                                                        \
    if (sh.wg == W && sh.items == I)                                                   \
        return stage == 1 ? Kern<W, I>::stage_occ_ft<float, 1, kFieldSplit>(halo, nonlinear)         \
                          : Kern<W, I>::stage_occ_ft<float, 2, kFieldSplit>(halo, nonlinear);

int stage_occupancy_f32(Shape sh, bool halo, bool nonlinear, int stage, bool ilv)
{
    if (ilv)
        return stage_occupancy_ilv_f32(sh, halo, nonlinear, stage);
    PM_STAGE_SHAPES(PM_STAGE_OCC_CASE)
    return 1;
}

}  // namespace pm
