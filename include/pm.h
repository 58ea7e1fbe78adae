/*
 * pm.h -- C ABI of the MI355X (gfx950) Lagrangian particle step.
 *
 * Method: LCS.jl (Tominaga & Onishi, arXiv 2604.11008).  Each step moves
 * every particle of a pool partitioned into subdomains:
 *   1. U(X): trilinear interpolation of the fluid velocity from the eight
 *      surrounding cell-centre values (Sect. 2.2, Particle Phase);
 *   2. dX/dt = V, dV/dt = -(f/tau)(V - U(X)) + g, advanced with a two-stage
 *      second-order Runge-Kutta method (Heun) (Sect. 2.2), with the drag
 *      factor f = 1 (Stokes) or the paper's nonlinear correction (pm_drag);
 *   3. the boundary-crossing check against the owner subdomain, generalised
 *      from the paper's send/stay mask to 26 neighbour directions
 *      (Sect. 2.3.3, stage 1);
 *   4. a prefix scan of the send/stay mask giving every particle a unique
 *      slot (Sect. 2.3.3, stages 2-3: scan[i] = sum of mask[1..i]); the
 *      leavers' slots are then split by direction, which yields exactly the
 *      slots of per-direction counters; packing the leavers into
 *      per-direction send buffers and compacting the stayers, then appending
 *      what every subdomain receives (unpacking, Sect. 3.2.2).
 * The subdomains are virtual partitions of one device's memory, so the
 * exchange between them is an on-device copy.
 *
 * Conventions (where the paper is silent):
 *   - node (i,j,k) of the field sits at the cell centre ((i+1/2)L/n, ...);
 *   - ownership intervals are half-open: b[a] <= x < b[a+1];
 *   - direction code d = 9(oz+1) + 3(oy+1) + (ox+1), o in {-1,0,1};
 *     d == 13 (PM_STAY) means "no boundary crossed";
 *   - subdomain index s = ax + Px*(ay + Py*az);
 *   - the periodic shift is applied by the sender when it packs: x - L when
 *     leaving through L, and x + L when leaving through 0, replaced by the
 *     largest double below L if that sum rounds to L;
 *   - stayers keep their order; received particles follow them, direction
 *     code ascending, each send buffer in its own order;
 *   - a particle that would move beyond its neighbour (PM_F_SKIP) or has a
 *     non-finite coordinate (PM_F_NONFINITE) stays where it is.
 *
 * Memory: every array is device memory owned by the caller; the library
 * never allocates device memory.  Pointers must stay valid until the work
 * queued on the stream has finished.  Streams are hipStream_t values passed
 * as void* (NULL = the null stream).  Every call is asynchronous except
 * pm_get_status, pm_autotune and pm_kernel_times, which synchronise.
 * A pm_ctx is not thread-safe: use one context per stream.
 *
 * Errors: argument errors are detected on the host and returned as
 * PM_ERR_ARG before anything is queued (pm_last_error() tells why).  Errors
 * found while running set bits in the context's device flag word, read (and
 * cleared) by pm_get_status.  Capacity overflows still count exactly, so the
 * counts written are the capacities that would have sufficed; records that
 * did not fit are not written.  PM_F_LAYOUT (inconsistent segment tables)
 * turns every later call of the context into a no-op until the flags are
 * read and cleared, so that nothing is read or written out of bounds.
 */
#ifndef PM_H
#define PM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { PM_OK = 0, PM_ERR_ARG = 1, PM_ERR_HIP = 2 } pm_status;

/* Element type of the field and of the particle velocities/tau.
 * Two modes are supported:
 *   field PM_F64 with particles PM_F64 (64-byte records), and
 *   field PM_F32 with particles PM_F32 ("mixed": interpolation and drag in
 *   float32, positions, their updates and all classification in float64;
 *   48-byte records). */
typedef enum { PM_F64 = 0, PM_F32 = 1 } pm_dtype;

#define PM_STAY 13

/* Device flag bits (pm_get_status). */
#define PM_F_SEND_OVERFLOW 1u  /* a send buffer (s,d) was too small            */
#define PM_F_DEST_OVERFLOW 2u  /* an output segment was too small              */
#define PM_F_SKIP          4u  /* a particle moved beyond its neighbour        */
#define PM_F_NONFINITE     8u  /* a position coordinate was NaN or +-inf       */
#define PM_F_HALO          16u /* an interpolation stencil left the stored grid */
#define PM_F_LAYOUT        32u /* count > cap, a segment beyond the pool extent
                                  given to pm_create, or more tiles than
                                  non-overlapping segments of that extent give
                                  (overlapping segments)                        */

/* Limits. */
#define PM_MAX_P    32     /* subdomains per axis                             */
#define PM_MAX_NSUB 4096   /* subdomains in total                             */

/* Storage of the field's three components (pm_field.layout). */
typedef enum { PM_LAYOUT_SPLIT = 0, PM_LAYOUT_INTERLEAVED = 1 } pm_layout;

/* Velocity field on a uniform grid over [0,L0)x[0,L1)x[0,L2).
 * Stored nodes, x fastest:
 *   halo == 0: n0*n1*n2 nodes, node indices taken modulo n (periodic);
 *   halo == 1: (n0+2)(n1+2)(n2+2) nodes, stored index i+1 holds node i, so
 *              stored 0 and n+1 are the halo nodes -1 and n (for a periodic
 *              box: copies of nodes n-1 and 0).
 * layout == PM_LAYOUT_SPLIT: u[c] (c = x,y,z component) is a device array
 *   of one value per stored node.
 * layout == PM_LAYOUT_INTERLEAVED (collocated fields only): u[0] is one
 *   device array of three values per stored node, the node's x, y and z
 *   components next to each other (value 3m + c is component c of stored
 *   node m); u[1] and u[2] must be NULL.  A stencil row then takes one run
 *   of six values instead of three pairs from three arrays, which touches
 *   less than half as many 128-byte lines for isolated particles; the
 *   results are bitwise those of the split layout, through every entry
 *   point.  For solvers that can store the velocity this way, for many
 *   steps on one field, or for the float32 field of the mixed mode, which
 *   pm_field_interleave writes in one pass (a copy, or the rounding the
 *   mixed mode needs anyway); no step converts a field.
 * stagger == 0: collocated, node (i,j,k) of every component at the cell
 * centre ((i+1/2)L0/n0, ...), as the paper interpolates (Sect. 2.2);
 * stagger == 1: MAC arrangement, as its fluid solver stores the velocity
 * (Sect. 2.1): component c's node (i,j,k) on the face of cell (i,j,k)
 * normal to axis c, offset 0 along axis c and 1/2 along the others. */
typedef struct {
    int32_t n[3];
    int32_t halo;
    double L[3];
    int32_t dtype;      /* pm_dtype */
    int32_t stagger;    /* 0 collocated, 1 MAC */
    const void *u[3];
    int32_t layout;     /* pm_layout */
} pm_field;

/* P0 x P1 x P2 subdomains.  bounds[a] is a HOST array of p[a]+1 strictly
 * increasing doubles with bounds[a][0] == 0 and bounds[a][p[a]] == L, the
 * very double used as the box side (also pm_field.L[a] where a field is
 * given).  The values are copied into the launch; the arrays need not
 * outlive the call. */
typedef struct {
    int32_t p[3];
    int32_t pad_;
    const double *bounds[3];
} pm_decomp;

/* A pool of particle records (structure of arrays, device memory), cut
 * into nsub segments: segment s occupies records [base[s], base[s]+cap[s])
 * and holds count[s] particles at its start.  base/cap/count are device
 * int64 arrays of nsub entries.  x[c] are float64; v[c] and tau are of type
 * vdtype; id is uint64.  Segments must not overlap and must end within the
 * pool extent given to pm_create. */
typedef struct {
    int32_t nsub;
    int32_t vdtype;     /* pm_dtype */
    const int64_t *base;
    const int64_t *cap;
    int64_t *count;
    double *x[3];
    void *v[3];
    void *tau;
    uint64_t *id;
} pm_particles;

/* Send buffers: segment s*27+d holds what subdomain s sends in direction d
 * (the d == PM_STAY segments are unused and may have cap 0).  Same record
 * layout and vdtype as the particle pools; positions are stored already
 * shifted into the receiver's periodic image. */
typedef struct {
    const int64_t *base;   /* device [nsub*27] */
    const int64_t *cap;    /* device [nsub*27] */
    int64_t *count;        /* device [nsub*27], written */
    double *x[3];
    void *v[3];
    void *tau;
    uint64_t *id;
} pm_sendbufs;

/* Drag laws of the particle ODE dV/dt = -(f/tau)(V - U(X)) + g (Sect. 2.2). */
typedef enum {
    PM_DRAG_STOKES = 0,    /* f = 1                                            */
    PM_DRAG_NONLINEAR = 1  /* f = 1 + 0.15 Re_p^0.687, Re_p = 2 r |V - U| / nu,
                              r from tau = (2/9)(rho_p/rho) r^2 / nu           */
} pm_drag;

/* Mid-step records of per-stage migration (the paper exchanges the particle
 * arrays after each RK2 stage, Sect. 3.2.2): X_n (x), V_n (v), the stage-1
 * position X* (xs) and velocity V* (vs) and acceleration dV/dt (a), tau and
 * id -- 17 values, 136 bytes in FP64, the paper's 17 arrays with tau in
 * place of the diameter.  Segments as in pm_particles; x and xs float64,
 * the rest of type vdtype. */
typedef struct {
    int32_t nsub;
    int32_t vdtype;     /* pm_dtype */
    const int64_t *base;
    const int64_t *cap;
    int64_t *count;
    double *x[3];
    void *v[3];
    double *xs[3];
    void *vs[3];
    void *a[3];
    void *tau;
    uint64_t *id;
} pm_stage_particles;

/* Send buffers of the stage-1 exchange: segment s*27+d, mid-step records. */
typedef struct {
    const int64_t *base;   /* device [nsub*27] */
    const int64_t *cap;    /* device [nsub*27] */
    int64_t *count;        /* device [nsub*27], written */
    double *x[3];
    void *v[3];
    double *xs[3];
    void *vs[3];
    void *a[3];
    void *tau;
    uint64_t *id;
} pm_stage_sendbufs;

/* Time step, constant body force (gravity) added to dV/dt, and the drag law.
 * nu (kinematic viscosity) and density_ratio (rho_p/rho) are read only for
 * PM_DRAG_NONLINEAR, in the units of the field, the box and tau; both must
 * then be positive and finite. */
typedef struct {
    double dt;
    double g[3];
    int32_t drag;          /* pm_drag */
    int32_t pad_;
    double nu;
    double density_ratio;
} pm_params;

/* Launch shape of the tile kernels: workgroup size (256 or 512), records
 * per thread (1, 2, 4 or 8); tile = wg*items records.  wg = 0 in
 * pm_set_tuning selects the per-variant defaults (256 x 4; 256 x 2 for
 * mixed-precision periodic interleaved fields and for per-stage migration;
 * records per thread halved while the context's pool
 * extent gives fewer than two tiles per compute unit), which a context uses
 * until
 * pm_set_tuning or pm_autotune fixes a shape; pm_get_tuning then reports the
 * shape of the last launch.  blocks_per_cu is the persistent grid's
 * workgroups per compute unit: 0 = the runtime's occupancy estimate; an
 * explicit 1..32 may exceed it (surplus workgroups start as others retire;
 * tiles are claimed by ticket, so this cannot deadlock).  xcd_block is the
 * tile order of the persistent kernels: 0 = one ticket counter for all
 * workgroups (tiles in order, each on whichever XCD asks next); 1..65536 =
 * workgroup b takes its tiles from the counter of XCD b mod 8 and the XCDs
 * take blocks of xcd_block consecutive tiles in turn, so that each XCD's L2
 * serves neighbouring tiles (fewer field bytes fetched, not faster on the
 * measured workloads).  No tuning changes any result. */
typedef struct {
    int32_t wg;
    int32_t items;
    int32_t blocks_per_cu;
    int32_t xcd_block;
} pm_tuning;

typedef struct pm_ctx pm_ctx;

/* Bytes of device workspace a context needs for particle pools of at most
 * pool_extent records (max over segments of base+cap), send buffers of at
 * most send_extent records, and nsub subdomains.  It holds, besides small
 * tables, one look-back word per tile, one slot per pool record for the
 * plain path, and a staging area of send_extent leaver records (137 bytes
 * each: the 17 eight-byte values of a mid-step record of per-stage
 * migration, of which a per-step leaver uses 8, plus a direction byte).
 * 0 for invalid sizes (extents outside 0..2^34, nsub outside
 * 1..PM_MAX_NSUB). */
size_t pm_workspace_bytes(int64_t pool_extent, int64_t send_extent, int32_t nsub);

/* Create a context on the current device.  workspace: caller-owned device
 * memory of at least pm_workspace_bytes(pool_extent, send_extent, nsub)
 * bytes, 256-byte aligned.  Synchronous. */
pm_status pm_create(pm_ctx **ctx, void *workspace, size_t ws_bytes,
                    int64_t pool_extent, int64_t send_extent, int32_t nsub);
pm_status pm_destroy(pm_ctx *ctx);

/* U at n points (x,y,z device float64 arrays) into ux,uy,uz (device arrays
 * of the field's dtype).  Sect. 2.2 (trilinear interpolation). */
pm_status pm_interp(pm_ctx *ctx, const pm_field *field, int64_t n,
                    const double *x, const double *y, const double *z,
                    void *ux, void *uy, void *uz, void *stream);

/* The same field stored node-interleaved: writes the collocated split field
 * `field` (layout PM_LAYOUT_SPLIT, stagger 0) into `out`, a device array of
 * 3 x (stored nodes) values of type out_dtype (pm_dtype), value 3m + c =
 * component c of stored node m (PM_LAYOUT_INTERLEAVED; pass it as u[0] with
 * u[1] = u[2] = NULL and the same n, halo and L).  out_dtype is the field's
 * dtype, or PM_F32 for a PM_F64 field: each value rounded to the nearest
 * float, the field of the mixed mode written in the same pass.  For callers
 * whose solver writes the split layout but who take many steps on one field,
 * or who round it to float32 anyway: the pass reads and writes the field's
 * bytes once each, and the interleaved steps are bitwise those on the split
 * field of the same values.  `out` must not overlap the field.
 * Asynchronous on `stream`; needs no context. */
pm_status pm_field_interleave(const pm_field *field, int32_t out_dtype, void *out,
                              void *stream);

/* Steps 1-2 in place on the particles of segments [sub_first,
 * sub_first+sub_count): X and V are replaced by the Heun update.
 * Sect. 2.2 (particle ODE, two-stage second-order RK). */
pm_status pm_interp_advance(pm_ctx *ctx, const pm_field *field,
                            pm_particles *inout, const pm_params *params,
                            int32_t sub_first, int32_t sub_count, void *stream);

/* Steps 3-4 (mask, scan, pack) for segments [sub_first, sub_first+sub_count)
 * of `in` (left unchanged): writes every leaver to send segment s*27+d at
 * its scan slot, send->count for those segments, and each stayer's slot into
 * the workspace for pm_compact_append.  Sect. 2.3.3 (stages 1-3). */
pm_status pm_classify_scan_pack(pm_ctx *ctx, const pm_decomp *decomp,
                                const pm_particles *in, pm_sendbufs *send,
                                int32_t sub_first, int32_t sub_count,
                                void *stream);

/* Unpacking for destination segments [sub_first, sub_first+sub_count):
 * the stayers of `in` compacted in order into `out`, then the particles
 * sent to each destination appended; writes out->count.  Needs
 * pm_classify_scan_pack to have run on these segments and on every
 * subdomain that neighbours them, with no other classify call in between.
 * Sect. 3.2.2 (unpacking: compaction, then receive). */
pm_status pm_compact_append(pm_ctx *ctx, const pm_decomp *decomp,
                            const pm_particles *in, const pm_sendbufs *send,
                            pm_particles *out, int32_t sub_first,
                            int32_t sub_count, void *stream);

/* The whole step in -> out for all subdomains: interpolation and the Heun
 * update (Sect. 2.2), mask, scan and pack (Sect. 2.3.3), compaction and
 * receive (unpacking, Sect. 3.2.2), fused into one persistent launch plus
 * the on-device exchange; `in` is left unchanged.  Results are
 * bitwise equal to pm_interp_advance (on a copy of in), then
 * pm_classify_scan_pack, then pm_compact_append, over all subdomains.
 * With graphs enabled (pm_set_graph) the launches are captured once per
 * distinct argument set and replayed. */
pm_status pm_step(pm_ctx *ctx, const pm_field *field, const pm_decomp *decomp,
                  const pm_particles *in, pm_particles *out,
                  pm_sendbufs *send, const pm_params *params, void *stream);

/* Bytes of the fixed device array pm_step_noalloc works in (per device). */
#define PM_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* pm_step for callers that cannot allocate: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  It needs no context
 * and no workspace: its scratch (the header words, tile and staging tables,
 * look-back words and the leavers' staging area that pm_step keeps in the
 * workspace) is a fixed array of PM_NOALLOC_SCRATCH_BYTES in device memory
 * of the library, one per device, held until the process ends.  It calls no
 * allocating routine and queues only kernels, so a caller may capture it.
 *
 * Arguments as in pm_step; pool_extent is the number of records the arrays
 * of `in` and `out` hold (every segment must end within it), send_extent
 * that of `send`.  flags: caller-owned device memory of one uint32 that
 * receives this step's flag bits (PM_F_*) when its work is done.  Results
 * are bitwise those of pm_step with a context of the same extents and its
 * default launch shape.  Sizes whose scratch would exceed the array
 * (pm_workspace_bytes less the plain path's 4 bytes per pool record: about
 * 137 bytes per send-buffer record, 8 bytes per 256 pool records and 100 KB,
 * e.g. a pool of 2^24 records in 512 subdomains with up to 470,000
 * send-buffer records) are rejected with PM_ERR_ARG before anything is
 * queued.  Every call on a device uses that device's one array: calls that
 * overlap on one device (other streams, other threads) race and must not
 * be made; each call clears the flag word on entry, and the other scratch
 * contents are rebuilt by the step itself. */
pm_status pm_step_noalloc(const pm_field *field, const pm_decomp *decomp,
                          const pm_particles *in, pm_particles *out,
                          pm_sendbufs *send, const pm_params *params,
                          int64_t pool_extent, int64_t send_extent,
                          uint32_t *flags, void *stream);

/* Synchronise `stream`, return the flag word (PM_F_*) and clear it.
 * The capacities that would have sufficed after an overflow need no
 * out-parameter: the counts the step writes are exact whatever the
 * capacities (out->count[s] for every destination segment, send->count[s*27+d]
 * for every send buffer; records beyond a capacity are not written), so the
 * caller reads them from those device arrays, grows the segments and repeats
 * the step from the unchanged `in`. */
pm_status pm_get_status(pm_ctx *ctx, void *stream, uint32_t *flags);

pm_status pm_set_tuning(pm_ctx *ctx, const pm_tuning *t);
pm_status pm_get_tuning(pm_ctx *ctx, pm_tuning *t);

/* Time every supported launch shape and workgroups-per-CU setting on this
 * problem with pm_step (eager), keep the fastest in the context and, if
 * cache_path is not NULL, append it to that text file keyed by the problem
 * (grid, halo, element type, field arrangement and layout, drag law, subdomain count,
 * pool extent, tile order).  With a cache_path whose file already holds the
 * key, take that entry and time nothing.  Results do not depend on the
 * launch shape.  Synchronous; in is unchanged, out and send are
 * overwritten.  On an error the context's tuning, graph and timing settings
 * are as before the call. */
pm_status pm_autotune(pm_ctx *ctx, const pm_field *field,
                      const pm_decomp *decomp, const pm_particles *in,
                      pm_particles *out, pm_sendbufs *send,
                      const pm_params *params, void *stream,
                      const char *cache_path);

/* Capture pm_step and pm_step_staged into HIP graphs (enable != 0), one per
 * distinct argument set, launch shape and tuning (at most 16 kept), and
 * replay them; or launch eagerly (0). */
pm_status pm_set_graph(pm_ctx *ctx, int32_t enable);

/* Kernel timing: with max_records > 0, every eager pm_step records HIP
 * events around its fused kernel on the caller's stream (up to max_records
 * steps; 0 turns it off and drops the records).  pm_kernel_times
 * synchronises and returns the number of recorded launches and the total
 * and per-launch milliseconds (ms may be NULL). */
pm_status pm_set_timing(pm_ctx *ctx, int32_t max_records);
pm_status pm_kernel_times(pm_ctx *ctx, int32_t *n, double *total_ms, float *ms,
                          int32_t max_ms);

/* The step with migration after each RK2 stage, as the paper does it
 * (Sect. 3.2.2): stage 1 (X* = X_n + dt V_n, V* = V_n + dt a) for every
 * particle of `in`, which is then classified by X* and exchanged with its
 * 17 values into `mid` (leavers through `mid_send`; X_n is moved into the
 * receiver's periodic image by the same +-L as X*, in plain arithmetic);
 * stage 2 in the new owner (X' = X_n + dt/2 (V_n + V*), V' = V_n + dt/2 (a
 * + a(X*, V*))), classified by X' and exchanged into `out` (leavers through
 * `send`).  Each exchange is the same scan, pack, compact and append as
 * pm_step's.  Collocated fields (either layout); `in` is unchanged; mid must fit the
 * context's pool extent and mid_send its send extent.  Launch shapes with
 * at most 1024 records per tile (default 256 x 2, or fewer records per
 * thread for small pools as in pm_tuning).  Replayed as one HIP
 * graph of both stages under pm_set_graph, like pm_step; eager launches
 * record both stages' fused kernels under pm_set_timing. */
pm_status pm_step_staged(pm_ctx *ctx, const pm_field *field, const pm_decomp *decomp,
                         const pm_particles *in, pm_stage_particles *mid,
                         pm_stage_sendbufs *mid_send, pm_particles *out,
                         pm_sendbufs *send, const pm_params *params, void *stream);

/* Untimed diagnostic: number of distinct field nodes read by the stage-1
 * and stage-2 stencils of one pm_step from `in` (an exact count, through a
 * bitmap of nbits >= number of stored nodes bits, caller-owned device
 * memory of (nbits+63)/64 uint64, cleared here).  For a MAC field, whose
 * components have their own stencils, the bitmap needs 3 x the stored nodes
 * and the result is the number of distinct (component, node) values read,
 * divided by 3.  Synchronous. */
pm_status pm_touched_nodes(pm_ctx *ctx, const pm_field *field,
                           const pm_particles *in, const pm_params *params,
                           uint64_t *bitmap, int64_t nbits, void *stream,
                           int64_t *touched);

/* Cell re-sort of every segment of `in` into `out` (same nsub; out's
 * segments must hold in's counts): each segment's records ordered by the
 * cell they lie in -- cell (i,j,k) = floor(x_a n_a / L_a) clamped to
 * [0, n_a-1], keyed by the Z-order code of (i/2, j, k) times two plus the
 * parity of i -- and, within a cell, by their position in `in`.  Counts are
 * copied.  Not a step of the paper's method, which never reorders
 * particles: the fused step's stencil gathers share cache lines when
 * neighbouring records are neighbours in space, and particles disperse from
 * any order as they move, so a caller re-sorts every few tens of steps.
 * workspace: caller-owned device memory of at least
 * pm_sort_workspace_bytes(pool_extent, nsub) bytes for the context's pool
 * extent (below 2^32), 256-byte aligned.  Asynchronous; in is unchanged;
 * a segment of out too small for its count sets PM_F_DEST_OVERFLOW. */
size_t pm_sort_workspace_bytes(int64_t pool_extent, int32_t nsub);
pm_status pm_sort(pm_ctx *ctx, const pm_field *field, const pm_particles *in,
                  pm_particles *out, void *workspace, size_t ws_bytes, void *stream);

/* Text of the last host-side error of this thread. */
const char *pm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PM_H */
