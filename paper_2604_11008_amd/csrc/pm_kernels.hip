// pm_kernels.hip -- launchers of the particle step's kernels (all but the
// fused and advance kernels, whose variants live in pm_step_f64.hip and
// pm_step_f32.hip).
#include "pm_device.h"

namespace pm {
bool stage_shape_supported(Shape sh)
{
#define PM_ONE(W, I) if (sh.wg == W && sh.items == I) return true;
    PM_STAGE_SHAPES(PM_ONE)
#undef PM_ONE
    return false;
}

bool shape_supported(Shape sh)
{
#define PM_ONE(W, I) if (sh.wg == W && sh.items == I) return true;
    PM_SHAPES(PM_ONE)
#undef PM_ONE
    return false;
}

hipError_t launch_prep(const KArgs &a, int mode, hipStream_t st)
{
    int64_t work = 1;
    if (mode & kPrepZeroLb)
        work = (int64_t)a.ws.pool_extent / a.tile + a.sub_count + 2;
    if (mode & (kPrepZeroCounts | kPrepCheckSend))
        work = work > (int64_t)a.dc.nsub * 27 ? work : (int64_t)a.dc.nsub * 27;
    if (mode & kPrepZeroCounts)
        work = work > (int64_t)a.sub_count * 27 ? work : (int64_t)a.sub_count * 27;
    int64_t g = (work + 1023) / 1024;
    const int grid = (int)(g < 1 ? 1 : (g > 1024 ? 1024 : g));
    hipLaunchKernelGGL(k_prep, dim3(grid), dim3(256), 0, st, a, mode);
    return hipGetLastError();
}

#define PM_CLS_CASE(W, I)                                                              \
    if (sh.wg == W && sh.items == I) {                                                 \
        if (mixed)                                                                     \
            hipLaunchKernelGGL((k_classify<W, I, float>), dim3(grid), dim3(W), 0, st, a); \
        else                                                                           \
            hipLaunchKernelGGL((k_classify<W, I, double>), dim3(grid), dim3(W), 0, st, a); \
        return hipGetLastError();                                                      \
    }

hipError_t launch_classify(const KArgs &a, Shape sh, bool mixed, int grid, hipStream_t st)
{
    PM_SHAPES(PM_CLS_CASE)
    return hipErrorInvalidValue;
}

#define PM_CMP_CASE(W, I)                                                              \
    if (sh.wg == W && sh.items == I) {                                                 \
        if (mixed)                                                                     \
            hipLaunchKernelGGL((k_compact<W, I, float>), dim3(grid), dim3(W), 0, st, a); \
        else                                                                           \
            hipLaunchKernelGGL((k_compact<W, I, double>), dim3(grid), dim3(W), 0, st, a); \
        return hipGetLastError();                                                      \
    }

hipError_t launch_compact(const KArgs &a, Shape sh, bool mixed, int grid, hipStream_t st)
{
    PM_SHAPES(PM_CMP_CASE)
    return hipErrorInvalidValue;
}

hipError_t launch_append(const KArgs &a, bool mixed, int grid, hipStream_t st)
{
    if (mixed)
        hipLaunchKernelGGL((k_append<float>), dim3(grid), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL((k_append<double>), dim3(grid), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_route(const KArgs &a, bool mixed, bool append, hipStream_t st, bool ext)
{
    const int64_t jobs = (int64_t)a.sub_count * 27;
    const int grid = (int)(jobs < 4096 ? jobs : 4096);
    if (ext) {  // mid-step records of per-stage migration (always appended)
        if (mixed)
            hipLaunchKernelGGL((k_route<float, true, true>), dim3(grid), dim3(256), 0, st, a);
        else
            hipLaunchKernelGGL((k_route<double, true, true>), dim3(grid), dim3(256), 0, st, a);
        return hipGetLastError();
    }
    if (mixed) {
        if (append)
            hipLaunchKernelGGL((k_route<float, true, false>), dim3(grid), dim3(256), 0, st, a);
        else
            hipLaunchKernelGGL((k_route<float, false, false>), dim3(grid), dim3(256), 0, st, a);
    } else {
        if (append)
            hipLaunchKernelGGL((k_route<double, true, false>), dim3(grid), dim3(256), 0, st, a);
        else
            hipLaunchKernelGGL((k_route<double, false, false>), dim3(grid), dim3(256), 0, st, a);
    }
    return hipGetLastError();
}

template <typename FT, bool H, int FA>
hipError_t interp_t(const KArgs &a, int grid, int64_t n, const double *x, const double *y,
                    const double *z, void *ux, void *uy, void *uz, hipStream_t st)
{
    hipLaunchKernelGGL((k_interp<FT, H, FA>), dim3(grid), dim3(256), 0, st, a, n, x, y, z,
                       (FT *)ux, (FT *)uy, (FT *)uz);
    return hipGetLastError();
}

template <typename FT, bool H>
hipError_t interp_h(const KArgs &a, int grid, int64_t n, const double *x, const double *y,
                    const double *z, void *ux, void *uy, void *uz, hipStream_t st)
{
    switch (field_arr(a.f)) {
    case kFieldMac:
        return interp_t<FT, H, kFieldMac>(a, grid, n, x, y, z, ux, uy, uz, st);
    case kFieldIlv:
        return interp_t<FT, H, kFieldIlv>(a, grid, n, x, y, z, ux, uy, uz, st);
    default:
        return interp_t<FT, H, kFieldSplit>(a, grid, n, x, y, z, ux, uy, uz, st);
    }
}

template <typename FT>
hipError_t interp_ft(const KArgs &a, int grid, int64_t n, const double *x, const double *y,
                     const double *z, void *ux, void *uy, void *uz, hipStream_t st)
{
    return a.f.halo != 0 ? interp_h<FT, true>(a, grid, n, x, y, z, ux, uy, uz, st)
                         : interp_h<FT, false>(a, grid, n, x, y, z, ux, uy, uz, st);
}

hipError_t launch_interp(const KArgs &a, bool mixed, int64_t n, const double *x,
                         const double *y, const double *z, void *ux, void *uy, void *uz,
                         hipStream_t st)
{
    int64_t g = (n + 255) / 256;
    const int grid = (int)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
    return mixed ? interp_ft<float>(a, grid, n, x, y, z, ux, uy, uz, st)
                 : interp_ft<double>(a, grid, n, x, y, z, ux, uy, uz, st);
}

hipError_t launch_touch(const KArgs &a, bool mixed, uint64_t *bits, hipStream_t st)
{
    const int grid = 4096;
    if (mixed) {
        if (a.f.halo)
            hipLaunchKernelGGL((k_touch<float, true>), dim3(grid), dim3(256), 0, st, a, bits);
        else
            hipLaunchKernelGGL((k_touch<float, false>), dim3(grid), dim3(256), 0, st, a, bits);
    } else {
        if (a.f.halo)
            hipLaunchKernelGGL((k_touch<double, true>), dim3(grid), dim3(256), 0, st, a, bits);
        else
            hipLaunchKernelGGL((k_touch<double, false>), dim3(grid), dim3(256), 0, st, a, bits);
    }
    return hipGetLastError();
}

hipError_t launch_popcount(const uint64_t *bits, int64_t words, unsigned long long *out,
                           hipStream_t st)
{
    hipLaunchKernelGGL(k_popcount, dim3(2048), dim3(256), 0, st, bits, words, out);
    return hipGetLastError();
}

hipError_t launch_fill(uint64_t *p, int64_t words, hipStream_t st)
{
    int64_t g = (words + 255) / 256;
    const int grid = (int)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
    hipLaunchKernelGGL(k_fill, dim3(grid), dim3(256), 0, st, p, words);
    return hipGetLastError();
}

hipError_t launch_flags_move(uint32_t *hdr, uint32_t *dst, hipStream_t st)
{
    hipLaunchKernelGGL(k_flags_move, dim3(1), dim3(64), 0, st, hdr, dst);
    return hipGetLastError();
}

hipError_t launch_step(const KArgs &a, Shape sh, bool mixed, int grid, hipStream_t st)
{
    return mixed ? launch_step_f32(a, sh, grid, st) : launch_step_f64(a, sh, grid, st);
}

hipError_t launch_advance(const KArgs &a, Shape sh, bool mixed, int grid, hipStream_t st)
{
    return mixed ? launch_advance_f32(a, sh, grid, st) : launch_advance_f64(a, sh, grid, st);
}

hipError_t launch_stage(const KArgs &a, Shape sh, bool mixed, int stage, int grid,
                        hipStream_t st)
{
    return mixed ? launch_stage_f32(a, sh, stage, grid, st)
                 : launch_stage_f64(a, sh, stage, grid, st);
}

int stage_occupancy(Shape sh, bool mixed, bool halo, bool nonlinear, int stage, bool ilv)
{
    const int nb = mixed ? stage_occupancy_f32(sh, halo, nonlinear, stage, ilv)
                         : stage_occupancy_f64(sh, halo, nonlinear, stage, ilv);
    return nb < 1 ? 1 : nb;
}

int step_occupancy(Shape sh, bool mixed, bool halo, bool nonlinear, int arr)
{
    const int nb = mixed ? step_occupancy_f32(sh, halo, nonlinear, arr)
                         : step_occupancy_f64(sh, halo, nonlinear, arr);
    return nb < 1 ? 1 : nb;
}

}  // namespace pm
