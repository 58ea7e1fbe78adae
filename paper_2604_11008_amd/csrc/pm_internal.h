// pm_internal.h -- shared declarations of the HIP kernels and their host
// launchers (library-internal; the public interface is include/pm.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pm.h"

namespace pm {

// Look-back status word of a tile: the tile's count of stayers (bits 0-30)
// and of leavers (bits 31-61), and a 2-bit state (bits 62-63).
constexpr uint64_t kLbA = 1ull << 62;     // tile aggregate published
constexpr uint64_t kLbP = 2ull << 62;     // inclusive prefix published
constexpr uint64_t kLbMask = (1ull << 62) - 1;
constexpr uint64_t kM31 = 0x7fffffffull;
constexpr uint32_t kMigrantSlot = 0xffffffffu;

// Smallest tile any launch shape uses; sizes the look-back workspace.
constexpr int kMinTile = 256;

// Header words of the workspace.
enum { kHdrFlags = 0, kHdrTicket = 1, kHdrTiles = 2, kHdrGroupTicket = 32, kHdrWords = 64 };

// Ticket groups of the tile kernels: one per XCD (workgroups are dispatched
// to the XCDs round-robin, so workgroup b runs on XCD b mod 8).
enum { kMaxGroups = 8 };

struct DField {
    const void *u[3];  // interleaved: u[0] only
    int32_t n[3];
    int32_t halo;
    int32_t stagger; // 0 collocated, 1 MAC (component c face-centred along axis c)
    int32_t layout;  // 0 one array per component, 1 node-interleaved (collocated only)
    double r[3];     // n / L per axis
    int64_t sx;      // stored row length (n0 + 2 halo)
    int64_t sxy;     // stored plane size
};

// Field arrangements of the interpolating kernels (their template parameter
// FA): collocated with one array per component, MAC, collocated with the
// three components of a node interleaved.
enum { kFieldSplit = 0, kFieldMac = 1, kFieldIlv = 2 };

inline int field_arr(const DField &f)
{
    return f.stagger ? kFieldMac : (f.layout ? kFieldIlv : kFieldSplit);
}

struct DDecomp {
    int32_t p[3];
    int32_t nsub;
    double b[3][PM_MAX_P + 1];
    double L[3];
    double predL[3]; // largest double below L
};

struct DPool {
    const int64_t *base;
    const int64_t *cap;
    int64_t *count;
    double *x[3];
    void *v[3];
    void *tau;
    uint64_t *id;
    // mid-step records of per-stage migration only (else null): the stage-1
    // position and velocity and the stage-1 acceleration
    double *xs[3];
    void *vs[3];
    void *a[3];
};

struct DWS {
    uint32_t *hdr;
    int64_t *tile_start;   // [PM_MAX_NSUB + 1] first ticket of each segment of the range
    int64_t *stay;         // [nsub] stayers per segment
    int64_t *migtot;       // [nsub] leavers per segment
    int64_t *stg_start;    // [PM_MAX_NSUB + 1] staging offset of each segment of the range
    uint64_t *lb;          // [max_tiles] look-back status words
    uint32_t *slot;        // [pool_extent] stayer slots (plain path)
    // staging of the leavers, in scan order per segment: [stg_extent]
    double *stg_x[3];
    double *stg_v[3];      // read as float in the mixed mode
    double *stg_tau;
    uint64_t *stg_id;
    double *stg_xs[3];     // per-stage migration's extra fields
    double *stg_vs[3];
    double *stg_a[3];
    uint8_t *stg_d;
    int64_t max_tiles;
    int64_t pool_extent;
    int64_t send_extent;
    int64_t stg_extent;
};

struct KArgs {
    DField f;
    DDecomp dc;
    DPool in, out, send;
    DWS ws;
    double dt, half_dt, g[3];
    float dtf, half_dtf, gf[3];
    int32_t drag;        // pm_drag
    double kappa;        // nonlinear drag: Re_p = kappa sqrt(tau) |V - U|
    float kappaf;
    int32_t sub_first, sub_count;
    int32_t tile;        // records per tile of this launch shape
    int32_t xg, xb;      // ticket groups (<= 1: one global ticket), tiles per block
    int32_t cpt;         // append: workgroups per destination
};

// Work arrays of the cell re-sort (a caller-owned workspace of its own):
// (key, pool position) pairs in two buffers ping-ponged by the radix passes,
// and per tile the digit counts and the pool positions they start at.
struct DSort {
    uint64_t *keys[2];   // [pool_extent]
    uint32_t *vals[2];   // [pool_extent]
    uint32_t *hist;      // [tiles * 256]
    int64_t *off;        // [tiles * 256]
    int64_t tiles;       // capacity of hist and off, in tiles
};

// Prep kernel modes.
enum {
    kPrepTiles = 1,       // tile_start/ticket for the segment range
    kPrepZeroLb = 2,      // clear the look-back words
    kPrepZeroCounts = 4,  // clear send counts and stay counts of the range
    kPrepCheckIn = 8,
    kPrepCheckOut = 16,
    kPrepCheckSend = 32,
    kPrepStaging = 64,    // staging offsets of the range from the send capacities
};

struct Shape {
    int wg;
    int items;
};

// Launchers (pm_kernels.hip).  `mixed` selects float32 field/velocities.
hipError_t launch_prep(const KArgs &a, int mode, hipStream_t st);
// Cell re-sort (pm_sort.hip): records per tile, and the launches of one sort
// (keys, `passes` radix passes of 8 bits, gather).
int sort_tile();
hipError_t launch_sort(const KArgs &a, DSort s, int passes, bool mixed, int grid,
                       hipStream_t st);
hipError_t launch_step(const KArgs &a, Shape sh, bool mixed, int grid, hipStream_t st);
hipError_t launch_advance(const KArgs &a, Shape sh, bool mixed, int grid, hipStream_t st);
hipError_t launch_classify(const KArgs &a, Shape sh, bool mixed, int grid, hipStream_t st);
hipError_t launch_compact(const KArgs &a, Shape sh, bool mixed, int grid, hipStream_t st);
hipError_t launch_append(const KArgs &a, bool mixed, int grid, hipStream_t st);
hipError_t launch_route(const KArgs &a, bool mixed, bool append, hipStream_t st,
                        bool ext = false);
hipError_t launch_interp(const KArgs &a, bool mixed, int64_t n, const double *x,
                         const double *y, const double *z, void *ux, void *uy,
                         void *uz, hipStream_t st);
hipError_t launch_touch(const KArgs &a, bool mixed, uint64_t *bitmap, hipStream_t st);
hipError_t launch_popcount(const uint64_t *bitmap, int64_t words,
                           unsigned long long *out, hipStream_t st);
hipError_t launch_fill(uint64_t *p, int64_t words, hipStream_t st);
// hdr's flag word into *dst (dst may be NULL), then cleared.
hipError_t launch_flags_move(uint32_t *hdr, uint32_t *dst, hipStream_t st);

// Workgroups per CU that fit for a launch shape of the fused kernel on a
// field of arrangement `arr` (kField*).
int step_occupancy(Shape sh, bool mixed, bool halo, bool nonlinear, int arr);
// per element type (pm_step_f64.hip, pm_step_f32.hip; the MAC variants in
// pm_mac_f64.hip, pm_mac_f32.hip, the interleaved ones in pm_ilv_f64.hip,
// pm_ilv_f32.hip)
hipError_t launch_step_f64(const KArgs &a, Shape sh, int grid, hipStream_t st);
hipError_t launch_step_f32(const KArgs &a, Shape sh, int grid, hipStream_t st);
hipError_t launch_advance_f64(const KArgs &a, Shape sh, int grid, hipStream_t st);
hipError_t launch_advance_f32(const KArgs &a, Shape sh, int grid, hipStream_t st);
int step_occupancy_f64(Shape sh, bool halo, bool nonlinear, int arr);
int step_occupancy_f32(Shape sh, bool halo, bool nonlinear, int arr);
hipError_t launch_step_mac_f64(const KArgs &a, Shape sh, int grid, hipStream_t st);
hipError_t launch_step_mac_f32(const KArgs &a, Shape sh, int grid, hipStream_t st);
hipError_t launch_advance_mac_f64(const KArgs &a, Shape sh, int grid, hipStream_t st);
hipError_t launch_advance_mac_f32(const KArgs &a, Shape sh, int grid, hipStream_t st);
int step_occupancy_mac_f64(Shape sh, bool halo, bool nonlinear);
int step_occupancy_mac_f32(Shape sh, bool halo, bool nonlinear);
hipError_t launch_step_ilv_f64(const KArgs &a, Shape sh, int grid, hipStream_t st);
hipError_t launch_step_ilv_f32(const KArgs &a, Shape sh, int grid, hipStream_t st);
hipError_t launch_advance_ilv_f64(const KArgs &a, Shape sh, int grid, hipStream_t st);
hipError_t launch_advance_ilv_f32(const KArgs &a, Shape sh, int grid, hipStream_t st);
int step_occupancy_ilv_f64(Shape sh, bool halo, bool nonlinear);
int step_occupancy_ilv_f32(Shape sh, bool halo, bool nonlinear);
// per-stage migration: the fused kernel of stage 1 or 2 (pm_staged_f64.hip,
// pm_staged_f32.hip)
bool stage_shape_supported(Shape sh);
hipError_t launch_stage(const KArgs &a, Shape sh, bool mixed, int stage, int grid,
                        hipStream_t st);
int stage_occupancy(Shape sh, bool mixed, bool halo, bool nonlinear, int stage, bool ilv);
hipError_t launch_stage_f64(const KArgs &a, Shape sh, int stage, int grid, hipStream_t st);
hipError_t launch_stage_f32(const KArgs &a, Shape sh, int stage, int grid, hipStream_t st);
int stage_occupancy_f64(Shape sh, bool halo, bool nonlinear, int stage, bool ilv);
int stage_occupancy_f32(Shape sh, bool halo, bool nonlinear, int stage, bool ilv);
// on node-interleaved fields (pm_staged_ilv_f64.hip, pm_staged_ilv_f32.hip)
hipError_t launch_stage_ilv_f64(const KArgs &a, Shape sh, int stage, int grid, hipStream_t st);
hipError_t launch_stage_ilv_f32(const KArgs &a, Shape sh, int stage, int grid, hipStream_t st);
int stage_occupancy_ilv_f64(Shape sh, bool halo, bool nonlinear, int stage);
int stage_occupancy_ilv_f32(Shape sh, bool halo, bool nonlinear, int stage);
bool shape_supported(Shape sh);

}  // namespace pm
