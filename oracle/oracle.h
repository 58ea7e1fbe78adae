/*
 * oracle.h -- sequential FP64 reference of the Lagrangian particle step.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the slow, plainly written CPU
 * definition that the GPU library is checked against.  Only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product path never does.  It shares no code, header or constant with the
 * HIP library.
 *
 * What it computes (LCS.jl, arXiv 2604.11008):
 *   - trilinear interpolation of the fluid velocity from the eight
 *     surrounding cell-centre values (Sect. 2.2, Particle Phase);
 *   - the particle ODE dX/dt = V, dV/dt = -(f/tau)(V - U(X)) plus a
 *     constant body force g, advanced by a two-stage second-order
 *     Runge-Kutta method, read as Heun's method (Sect. 2.2); the drag factor
 *     is f = 1 (Stokes drag) or the paper's nonlinear correction
 *     f = 1 + 0.15 Re_p^0.687, Re_p = 2r|V - U(X)|/nu, with the radius r
 *     from tau = (2/9)(rho_p/rho)(r^2/nu) (Sect. 2.2);
 *   - the boundary-crossing check of each particle against its subdomain
 *     (Sect. 2.3.3, stage 1: the mask), generalised to the 26 neighbours;
 *   - the sequential per-direction-counter partition of the original
 *     Fortran LCS (Sect. 2.3.3, the sequential scheme), which the prefix-scan
 *     method reproduces exactly;
 *   - the unpacking step: stayers compacted in order, then the received
 *     particles appended (Sect. 3.2.2 and its particle-communication table).
 *
 * Conventions fixed where the paper is silent are listed in oracle.c.
 */
#ifndef PM_ORACLE_H
#define PM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Error bits (OR-ed over all particles of a call). */
#define ORC_SEND_OVERFLOW 1u  /* a send buffer (s,d) had too little capacity   */
#define ORC_DEST_OVERFLOW 2u  /* an output segment had too little capacity     */
#define ORC_SKIP          4u  /* moved further than one neighbouring subdomain */
#define ORC_NONFINITE     8u  /* a position component is NaN or +-inf          */
#define ORC_HALO          16u /* interpolation stencil outside the stored grid */

#define ORC_STAY 13           /* direction code of "no boundary crossed"       */

/* Velocity field on a uniform grid of a box [0,L0)x[0,L1)x[0,L2).
 * stagger == 0 (collocated): node (i,j,k) of every component sits at the
 * cell centre ((i+1/2)L0/n0, ...).  stagger == 1 (MAC): component c's node
 * (i,j,k) sits on the face of cell (i,j,k) normal to axis c, at offset 0
 * along axis c and 1/2 along the others (u_x at (i L0/n0, (j+1/2)L1/n1,
 * (k+1/2)L2/n2), ...).
 * halo == 0: arrays hold n0*n1*n2 values, indices taken modulo n (periodic).
 * halo == 1: arrays hold (n0+2)(n1+2)(n2+2) values; stored index i+1 is node
 *            i, and stored 0 and n+1 are the halo nodes -1 and n.
 * x is the fastest axis in memory. */
typedef struct {
    int n[3];
    int halo;
    int stagger;
    double L[3];
    const double *u[3];
} orc_field;

/* Px x Py x Pz subdomains; bounds b[a][0..p[a]], b[a][0] = 0, b[a][p[a]] = L.
 * Subdomain index s = ax + Px*(ay + Py*az). */
typedef struct {
    int p[3];
    const double *b[3];
} orc_decomp;

/* A pool of segments of structure-of-arrays particle records.  Segment q
 * occupies records [base[q], base[q]+cap[q]) and holds count[q] particles.
 * Particle pools have one segment per subdomain; send pools have 27 per
 * subdomain (segment s*27+d, the one with d == ORC_STAY unused). */
typedef struct {
    int nseg;
    const int64_t *base;
    const int64_t *cap;
    int64_t *count;
    double *x[3];
    double *v[3];
    double *tau;
    uint64_t *id;
} orc_pool;

/* Drag laws. */
#define ORC_DRAG_STOKES    0  /* f = 1                                        */
#define ORC_DRAG_NONLINEAR 1  /* f = 1 + 0.15 Re_p^0.687 (Sect. 2.2)          */

/* Step parameters: time step, constant body force (gravity), drag law, and
 * for the nonlinear law the kinematic viscosity nu and the particle-to-fluid
 * density ratio rho_p/rho (in the units of the field, box and tau). */
typedef struct {
    double dt;
    double g[3];
    int drag;
    double nu;
    double density_ratio;
} orc_params;

/* U(X) by trilinear interpolation.  Returns error bits (ORC_HALO). */
unsigned orc_interp(const orc_field *f, const double X[3], double U[3]);

/* orc_interp over n points given as three coordinate arrays. */
unsigned orc_interp_many(const orc_field *f, int64_t n,
                         const double *x, const double *y, const double *z,
                         double *ux, double *uy, double *uz);

/* One Heun step of n particles, in place on x[3] and v[3]. */
unsigned orc_advance(const orc_field *f, const orc_params *pr, int64_t n,
                     double *x[3], double *v[3], const double *tau);

/* Direction code d in 0..26 of a particle owned by subdomain s now at X,
 * and its position Xs as stored in the receiving subdomain (periodic shift
 * applied).  Error bits are OR-ed into *flags. */
int orc_classify(const orc_decomp *dc, int s, const double X[3], double Xs[3],
                 unsigned *flags);

/* Sequential partition of every segment of `in`: stayers to `out` (same
 * segment), migrants to `send` segment s*27+d, each in scan order.
 * stay_count[s] receives the number of stayers; send->count is written.
 * dir and slot (per pool record of `in`, may be NULL) receive each
 * particle's direction code and its 0-based slot in the destination. */
unsigned orc_partition(const orc_decomp *dc, const orc_pool *in, orc_pool *out,
                       orc_pool *send, int64_t *stay_count, int32_t *dir,
                       int64_t *slot);

/* Append to every destination t the particles sent to it, after its
 * stayers: directions ascending, each buffer in its own order.
 * Writes out->count. */
unsigned orc_append(const orc_decomp *dc, const orc_pool *send,
                    const int64_t *stay_count, orc_pool *out);

/* Whole step in -> out: advance (on a private copy; `in` is unchanged),
 * partition, append.  stay_count may be NULL. */
unsigned orc_step(const orc_field *f, const orc_decomp *dc,
                  const orc_params *pr, const orc_pool *in, orc_pool *out,
                  orc_pool *send, int64_t *stay_count);

/* Mid-step records of per-stage migration (the paper migrates after each
 * RK2 stage, Sect. 3.2.2): X_n, V_n, the stage-1 position and velocity X*,
 * V*, and the stage-1 acceleration a = dV/dt, plus tau and id: 17 values,
 * the paper's 17 arrays with tau standing for the diameter. */
typedef struct {
    int nseg;
    const int64_t *base;
    const int64_t *cap;
    int64_t *count;
    double *x[3], *v[3], *xs[3], *vs[3], *a[3];
    double *tau;
    uint64_t *id;
} orc_xpool;

/* Whole step with migration after each RK2 stage.  Stage 1: X*, V* and a
 * from X_n, V_n; every particle is classified by X* and migrated with its 17
 * values to `mid` (leavers through `mid_send`); X_n moves into the
 * receiver's periodic image by the same +-L as X* (plain arithmetic).
 * Stage 2 in the new owner: X' = X_n + dt/2 (V_n + V*), V' = V_n + dt/2 (a +
 * a(X*, V*)); classified by X' and migrated to `out` (leavers through
 * `send`).  `in` is unchanged. */
unsigned orc_step_staged(const orc_field *f, const orc_decomp *dc,
                         const orc_params *pr, const orc_pool *in, orc_xpool *mid,
                         orc_xpool *mid_send, orc_pool *out, orc_pool *send);

#ifdef __cplusplus
}
#endif
#endif
