/*
 * oracle.c -- sequential FP64 reference of the Lagrangian particle step.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  One thread, plain loops, no
 * blocking, fusion or reordering.  Build with -O2 -ffp-contract=off so that
 * every product and sum rounds on its own, exactly as written.
 *
 * Readings of points the paper leaves open:
 *  R1  RK2 tableau: Heun (explicit trapezoid).  Sect. 2.2 gives only the number
 *      of stages (two) and the order (second).
 *  R2  Drag factor f = 1 (Stokes); a constant body force g is added to dV/dt.
 *  R3  Nodes are collocated at cell centres (i+1/2)*Delta; weights use the
 *      fraction of s = X*(n/L) - 1/2 above floor(s).
 *  R4  Interpolation sums the eight weighted corners in the order
 *      (0,0,0),(1,0,0),(0,1,0),(1,1,0),(0,0,1),(1,0,1),(0,1,1),(1,1,1).
 *  R5  Ownership is half-open, b[a] <= x < b[a+1]; -0.0 counts as 0.
 *  R6  Periodic wrap happens when a particle is classified, on the sending
 *      side: x - L when leaving through L (exact), and x + L, or the largest
 *      double below L if that sum rounds up to L, when leaving through 0.
 *  R7  A particle that would land outside its one-step neighbour keeps its
 *      place and raises SKIP; one with a non-finite coordinate keeps its
 *      place and raises NONFINITE.  Counts are therefore conserved.
 *  R8  Direction code d = 9(oz+1) + 3(oy+1) + (ox+1), 13 = stay; received
 *      particles are appended after the stayers, d ascending, each send
 *      buffer in its own order.
 *  R9  A write beyond a capacity is skipped and flagged; counting goes on,
 *      so the counts returned are the capacities that would have sufficed.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Trilinear interpolation (Sect. 2.2: U(X) from the eight surrounding  */
/* cell-centre values).                                                 */
/* ------------------------------------------------------------------ */

/* Stored index of the two corners along one axis, and the fraction. */
static unsigned axis_corners(const orc_field *f, int a, double X, double half,
                             int64_t c[2], double *frac)
{
    unsigned flags = 0;
    const int n = f->n[a];
    const double r = (double)n / f->L[a];
    const double s = X * r - half;
    const double fl = floor(s);
    int64_t i;

    *frac = s - fl;
    if (isnan(s)) {
        /* The weights are NaN, so U is NaN; the classifier reports it. */
        i = 0;
    } else if (f->halo) {
        /* corners i and i+1 must lie in the stored range -1..n */
        if (!(s >= -1.0)) {
            flags |= ORC_HALO;
            i = -1;
        } else if (!(s < (double)n)) {
            flags |= ORC_HALO;
            i = n - 1;
        } else {
            i = (int64_t)fl;
        }
    } else {
        /* periodic: one wrap in either direction is addressable */
        if (!(s >= -(double)n)) {
            flags |= ORC_HALO;
            i = -n;
        } else if (!(s < 2.0 * (double)n)) {
            flags |= ORC_HALO;
            i = 2 * (int64_t)n - 1;
        } else {
            i = (int64_t)fl;
        }
    }

    if (f->halo) {
        c[0] = i + 1;
        c[1] = i + 2;
    } else {
        int64_t i0 = i % n;
        if (i0 < 0)
            i0 += n;
        c[0] = i0;
        c[1] = (i0 + 1) % n;
    }
    return flags;
}

unsigned orc_interp(const orc_field *f, const double X[3], double U[3])
{
    unsigned flags = 0;
    int64_t c[3][2];
    double fr[3];
    const int64_t sx = f->n[0] + 2 * f->halo;
    const int64_t sy = f->n[1] + 2 * f->halo;

    if (f->stagger) {
        /* MAC: component comp sits on the faces normal to axis comp, so its
         * nodes are offset by half a cell along that axis only */
        for (int comp = 0; comp < 3; ++comp) {
            for (int a = 0; a < 3; ++a)
                flags |= axis_corners(f, a, X[a], a == comp ? 0.0 : 0.5, c[a], &fr[a]);
            U[comp] = 0.0;
            for (int cz = 0; cz < 2; ++cz) {
                for (int cy = 0; cy < 2; ++cy) {
                    for (int cx = 0; cx < 2; ++cx) {
                        const double wx = cx ? fr[0] : 1.0 - fr[0];
                        const double wy = cy ? fr[1] : 1.0 - fr[1];
                        const double wz = cz ? fr[2] : 1.0 - fr[2];
                        const double w = (wx * wy) * wz;
                        const int64_t node = c[0][cx] + sx * (c[1][cy] + sy * c[2][cz]);
                        U[comp] = U[comp] + w * f->u[comp][node];
                    }
                }
            }
        }
        return flags;
    }

    for (int a = 0; a < 3; ++a)
        flags |= axis_corners(f, a, X[a], 0.5, c[a], &fr[a]);

    for (int comp = 0; comp < 3; ++comp)
        U[comp] = 0.0;

    for (int cz = 0; cz < 2; ++cz) {
        for (int cy = 0; cy < 2; ++cy) {
            for (int cx = 0; cx < 2; ++cx) {
                const double wx = cx ? fr[0] : 1.0 - fr[0];
                const double wy = cy ? fr[1] : 1.0 - fr[1];
                const double wz = cz ? fr[2] : 1.0 - fr[2];
                const double w = (wx * wy) * wz;
                const int64_t node = c[0][cx] + sx * (c[1][cy] + sy * c[2][cz]);
                for (int comp = 0; comp < 3; ++comp)
                    U[comp] = U[comp] + w * f->u[comp][node];
            }
        }
    }
    return flags;
}

unsigned orc_interp_many(const orc_field *f, int64_t n, const double *x,
                         const double *y, const double *z, double *ux,
                         double *uy, double *uz)
{
    unsigned flags = 0;
    for (int64_t p = 0; p < n; ++p) {
        const double X[3] = {x[p], y[p], z[p]};
        double U[3];
        flags |= orc_interp(f, X, U);
        ux[p] = U[0];
        uy[p] = U[1];
        uz[p] = U[2];
    }
    return flags;
}

/* ------------------------------------------------------------------ */
/* Particle ODE, two-stage second-order RK (Heun), Sect. 2.2.           */
/*   A = f (U(X) - V)/tau + g                                           */
/*   X* = X + dt V,            V* = V + dt A(X, V)                      */
/*   X' = X + dt/2 (V + V*),   V' = V + dt/2 (A(X, V) + A(X*, V*))      */
/* ------------------------------------------------------------------ */

/* Drag factor f of a particle with relaxation time t and slip U - V
 * (Sect. 2.2): 1 for Stokes drag; else r from t = (2/9)(rho_p/rho) r^2/nu,
 * Re_p = 2 r |V - U| / nu and f = 1 + 0.15 Re_p^0.687. */
static double drag_factor(const orc_params *pr, double t, const double slip[3])
{
    if (pr->drag != ORC_DRAG_NONLINEAR)
        return 1.0;
    const double r = sqrt(9.0 * pr->nu * t / (2.0 * pr->density_ratio));
    const double w = sqrt(slip[0] * slip[0] + slip[1] * slip[1] + slip[2] * slip[2]);
    const double re = 2.0 * r * w / pr->nu;
    return 1.0 + 0.15 * pow(re, 0.687);
}

unsigned orc_advance(const orc_field *f, const orc_params *pr, int64_t n,
                     double *x[3], double *v[3], const double *tau)
{
    unsigned flags = 0;
    const double dt = pr->dt;
    const double half_dt = 0.5 * dt;

    for (int64_t p = 0; p < n; ++p) {
        double X[3], V[3], U1[3], A1[3], Xs[3], Vs[3], U2[3], A2[3], s1[3], s2[3];
        const double t = tau[p];

        for (int a = 0; a < 3; ++a) {
            X[a] = x[a][p];
            V[a] = v[a][p];
        }
        flags |= orc_interp(f, X, U1);
        for (int a = 0; a < 3; ++a)
            s1[a] = U1[a] - V[a];
        const double f1 = drag_factor(pr, t, s1);
        for (int a = 0; a < 3; ++a) {
            A1[a] = f1 * s1[a] / t + pr->g[a];
            Xs[a] = X[a] + dt * V[a];
            Vs[a] = V[a] + dt * A1[a];
        }
        flags |= orc_interp(f, Xs, U2);
        for (int a = 0; a < 3; ++a)
            s2[a] = U2[a] - Vs[a];
        const double f2 = drag_factor(pr, t, s2);
        for (int a = 0; a < 3; ++a) {
            A2[a] = f2 * s2[a] / t + pr->g[a];
            x[a][p] = X[a] + half_dt * (V[a] + Vs[a]);
            v[a][p] = V[a] + half_dt * (A1[a] + A2[a]);
        }
    }
    return flags;
}

/* ------------------------------------------------------------------ */
/* Boundary-crossing check (Sect. 2.3.3, stage 1), one axis at a time.  */
/* ------------------------------------------------------------------ */

int orc_classify(const orc_decomp *dc, int s, const double X[3], double Xs[3],
                 unsigned *flags)
{
    const int own[3] = {s % dc->p[0], (s / dc->p[0]) % dc->p[1],
                        s / (dc->p[0] * dc->p[1])};
    int o[3];
    int skip = 0;

    if (!isfinite(X[0]) || !isfinite(X[1]) || !isfinite(X[2])) {
        *flags |= ORC_NONFINITE;
        for (int a = 0; a < 3; ++a)
            Xs[a] = X[a];
        return ORC_STAY;
    }

    for (int a = 0; a < 3; ++a) {
        const double *b = dc->b[a];
        const int P = dc->p[a];
        const double L = b[P];
        const int k = own[a];
        int t;
        double xs = X[a];

        if (X[a] < b[k]) {
            o[a] = -1;
            t = k - 1;
            if (k == 0) {
                const double w = X[a] + L;
                t = P - 1;
                xs = (w < L) ? w : nextafter(L, 0.0);
            }
        } else if (X[a] >= b[k + 1]) {
            o[a] = 1;
            t = k + 1;
            if (k == P - 1) {
                t = 0;
                xs = X[a] - L;
            }
        } else {
            o[a] = 0;
            t = k;
        }
        if (!(b[t] <= xs && xs < b[t + 1]))
            skip = 1;
        Xs[a] = xs;
    }

    if (skip) {
        *flags |= ORC_SKIP;
        for (int a = 0; a < 3; ++a)
            Xs[a] = X[a];
        return ORC_STAY;
    }
    return 9 * (o[2] + 1) + 3 * (o[1] + 1) + (o[0] + 1);
}

/* ------------------------------------------------------------------ */
/* Sequential per-direction-counter partition (Sect. 2.3.3: particles   */
/* are scanned in order and a counter per direction gives each one its  */
/* slot).  Stayers go to the output segment, migrants to send[s][d].    */
/* ------------------------------------------------------------------ */

static void put(orc_pool *dst, int64_t at, const double X[3], const double V[3],
                double tau, uint64_t id)
{
    for (int a = 0; a < 3; ++a) {
        dst->x[a][at] = X[a];
        dst->v[a][at] = V[a];
    }
    dst->tau[at] = tau;
    dst->id[at] = id;
}

unsigned orc_partition(const orc_decomp *dc, const orc_pool *in, orc_pool *out,
                       orc_pool *send, int64_t *stay_count, int32_t *dir,
                       int64_t *slot)
{
    unsigned flags = 0;

    for (int s = 0; s < in->nseg; ++s) {
        int64_t counter[27];
        for (int d = 0; d < 27; ++d)
            counter[d] = 0;

        for (int64_t i = 0; i < in->count[s]; ++i) {
            const int64_t p = in->base[s] + i;
            const double X[3] = {in->x[0][p], in->x[1][p], in->x[2][p]};
            const double V[3] = {in->v[0][p], in->v[1][p], in->v[2][p]};
            double Xs[3];
            const int d = orc_classify(dc, s, X, Xs, &flags);
            const int64_t k = counter[d];

            if (dir)
                dir[p] = d;
            if (slot)
                slot[p] = k;

            if (d == ORC_STAY) {
                if (k < out->cap[s])
                    put(out, out->base[s] + k, X, V, in->tau[p], in->id[p]);
                else
                    flags |= ORC_DEST_OVERFLOW;
            } else {
                const int q = s * 27 + d;
                if (k < send->cap[q])
                    put(send, send->base[q] + k, Xs, V, in->tau[p], in->id[p]);
                else
                    flags |= ORC_SEND_OVERFLOW;
            }
            counter[d] = k + 1;
        }

        stay_count[s] = counter[ORC_STAY];
        for (int d = 0; d < 27; ++d)
            send->count[s * 27 + d] = (d == ORC_STAY) ? 0 : counter[d];
    }
    return flags;
}

/* ------------------------------------------------------------------ */
/* Receive: append after the stayers (Sect. 3.2.2, unpacking).          */
/* ------------------------------------------------------------------ */

/* Subdomain reached from t by moving (ox,oy,oz) subdomains, periodic. */
static int neighbour(const orc_decomp *dc, int t, int ox, int oy, int oz)
{
    const int px = dc->p[0], py = dc->p[1], pz = dc->p[2];
    const int tx = t % px, ty = (t / px) % py, tz = t / (px * py);
    const int nx = ((tx + ox) % px + px) % px;
    const int ny = ((ty + oy) % py + py) % py;
    const int nz = ((tz + oz) % pz + pz) % pz;
    return nx + px * (ny + py * nz);
}

unsigned orc_append(const orc_decomp *dc, const orc_pool *send,
                    const int64_t *stay_count, orc_pool *out)
{
    unsigned flags = 0;

    for (int t = 0; t < out->nseg; ++t) {
        int64_t pos = stay_count[t];
        for (int d = 0; d < 27; ++d) {
            if (d == ORC_STAY)
                continue;
            /* a particle sent in direction o arrives from the subdomain at -o */
            const int ox = d % 3 - 1, oy = (d / 3) % 3 - 1, oz = d / 9 - 1;
            const int src = neighbour(dc, t, -ox, -oy, -oz);
            const int q = src * 27 + d;
            for (int64_t k = 0; k < send->count[q]; ++k) {
                if (k < send->cap[q]) {
                    const int64_t p = send->base[q] + k;
                    if (pos < out->cap[t]) {
                        const double X[3] = {send->x[0][p], send->x[1][p],
                                             send->x[2][p]};
                        const double V[3] = {send->v[0][p], send->v[1][p],
                                             send->v[2][p]};
                        put(out, out->base[t] + pos, X, V, send->tau[p],
                            send->id[p]);
                    } else {
                        flags |= ORC_DEST_OVERFLOW;
                    }
                }
                ++pos;
            }
        }
        out->count[t] = pos;
    }
    return flags;
}

/* ------------------------------------------------------------------ */
/* Whole step, out of place.                                            */
/* ------------------------------------------------------------------ */

unsigned orc_step(const orc_field *f, const orc_decomp *dc,
                  const orc_params *pr, const orc_pool *in, orc_pool *out,
                  orc_pool *send, int64_t *stay_count)
{
    unsigned flags = 0;
    int64_t extent = 0;
    int64_t *stay = stay_count;
    orc_pool tmp = *in;
    double *mem;

    for (int s = 0; s < in->nseg; ++s)
        if (in->base[s] + in->count[s] > extent)
            extent = in->base[s] + in->count[s];

    /* private copy of the advanced state, so `in` is left as it was */
    mem = (double *)malloc((size_t)(extent > 0 ? extent : 1) * 6 * sizeof(double));
    if (!mem)
        abort();
    for (int a = 0; a < 3; ++a) {
        tmp.x[a] = mem + (size_t)a * (size_t)extent;
        tmp.v[a] = mem + (size_t)(3 + a) * (size_t)extent;
        memcpy(tmp.x[a], in->x[a], (size_t)extent * sizeof(double));
        memcpy(tmp.v[a], in->v[a], (size_t)extent * sizeof(double));
    }
    if (!stay) {
        stay = (int64_t *)malloc((size_t)(in->nseg > 0 ? in->nseg : 1) * sizeof(int64_t));
        if (!stay)
            abort();
    }

    for (int s = 0; s < in->nseg; ++s) {
        double *xs[3], *vs[3];
        const int64_t b = in->base[s];
        for (int a = 0; a < 3; ++a) {
            xs[a] = tmp.x[a] + b;
            vs[a] = tmp.v[a] + b;
        }
        flags |= orc_advance(f, pr, in->count[s], xs, vs, in->tau + b);
    }
    flags |= orc_partition(dc, &tmp, out, send, stay, NULL, NULL);
    flags |= orc_append(dc, send, stay, out);

    if (stay != stay_count)
        free(stay);
    free(mem);
    return flags;
}

/* ------------------------------------------------------------------ */
/* Per-stage migration (Sect. 3.2.2: the particle arrays are exchanged  */
/* after each RK2 stage).  The partition and append above give every    */
/* record's destination; a record's index travels in the id field of a */
/* carrier pool and picks up the other arrays afterwards.               */
/* ------------------------------------------------------------------ */

static int64_t pool_extent(int nseg, const int64_t *base, const int64_t *cap)
{
    int64_t e = 0;
    for (int s = 0; s < nseg; ++s)
        if (base[s] + cap[s] > e)
            e = base[s] + cap[s];
    return e > 0 ? e : 1;
}

/* A carrier pool over the segments of (base, cap, count): x, v, tau, id
 * arrays of `extent` records in one allocation. */
static double *carrier(orc_pool *c, int nseg, const int64_t *base, const int64_t *cap,
                       int64_t *count, int64_t extent)
{
    double *mem = (double *)calloc((size_t)extent * 8, sizeof(double));
    if (!mem)
        abort();
    c->nseg = nseg;
    c->base = base;
    c->cap = cap;
    c->count = count;
    for (int a = 0; a < 3; ++a) {
        c->x[a] = mem + (size_t)a * (size_t)extent;
        c->v[a] = mem + (size_t)(3 + a) * (size_t)extent;
    }
    c->tau = mem + (size_t)6 * (size_t)extent;
    c->id = (uint64_t *)(mem + (size_t)7 * (size_t)extent);
    return mem;
}

/* X_n of record p (owned by subdomain s, sent in direction d) in the
 * receiver's periodic image: -L leaving through L, +L leaving through 0. */
static void shift_xn(const orc_decomp *dc, int s, int d, const double X[3], double Xo[3])
{
    const int own[3] = {s % dc->p[0], (s / dc->p[0]) % dc->p[1], s / (dc->p[0] * dc->p[1])};
    const int o[3] = {d % 3 - 1, (d / 3) % 3 - 1, d / 9 - 1};
    for (int a = 0; a < 3; ++a) {
        const double L = dc->b[a][dc->p[a]];
        Xo[a] = X[a];
        if (o[a] > 0 && own[a] == dc->p[a] - 1)
            Xo[a] = X[a] - L;
        else if (o[a] < 0 && own[a] == 0)
            Xo[a] = X[a] + L;
    }
}

/* Expand carrier record r (whose id is the source index p) into xp[at]. */
static void expand(orc_xpool *xp, int64_t at, const orc_pool *c, int64_t r, const orc_pool *in,
                   const double *acc, const int *seg_of, const int32_t *dir,
                   const orc_decomp *dc)
{
    const int64_t p = (int64_t)c->id[r];
    const double X[3] = {in->x[0][p], in->x[1][p], in->x[2][p]};
    double Xo[3];
    shift_xn(dc, seg_of[p], dir[p], X, Xo);
    for (int a = 0; a < 3; ++a) {
        xp->x[a][at] = Xo[a];
        xp->v[a][at] = in->v[a][p];
        xp->xs[a][at] = c->x[a][r];
        xp->vs[a][at] = c->v[a][r];
        xp->a[a][at] = acc[(size_t)p * 3 + a];
    }
    xp->tau[at] = in->tau[p];
    xp->id[at] = in->id[p];
}

unsigned orc_step_staged(const orc_field *f, const orc_decomp *dc,
                         const orc_params *pr, const orc_pool *in, orc_xpool *mid,
                         orc_xpool *mid_send, orc_pool *out, orc_pool *send)
{
    unsigned flags = 0;
    const double dt = pr->dt;
    const double half_dt = 0.5 * dt;
    const int nsub = in->nseg;
    const int64_t ext_in = pool_extent(nsub, in->base, in->cap);
    const int64_t ext_mid = pool_extent(mid->nseg, mid->base, mid->cap);
    const int64_t ext_ms = pool_extent(nsub * 27, mid_send->base, mid_send->cap);
    int64_t *stay = (int64_t *)calloc((size_t)(nsub > 0 ? nsub : 1), sizeof(int64_t));
    int32_t *dir = (int32_t *)calloc((size_t)ext_in, sizeof(int32_t));
    int *seg_of = (int *)calloc((size_t)ext_in, sizeof(int));
    double *acc = (double *)calloc((size_t)ext_in * 3, sizeof(double));
    int64_t *cnt_in = (int64_t *)calloc((size_t)(nsub > 0 ? nsub : 1), sizeof(int64_t));
    if (!stay || !dir || !seg_of || !acc || !cnt_in)
        abort();

    /* stage 1 into a carrier pool: x = X*, v = V*, id = record index */
    orc_pool c1, cm, cs;
    for (int s = 0; s < nsub; ++s)
        cnt_in[s] = in->count[s];
    double *m1 = carrier(&c1, nsub, in->base, in->cap, cnt_in, ext_in);
    for (int s = 0; s < nsub; ++s) {
        for (int64_t i = 0; i < in->count[s]; ++i) {
            const int64_t p = in->base[s] + i;
            const double t = in->tau[p];
            double X[3], V[3], U1[3], s1[3];
            for (int a = 0; a < 3; ++a) {
                X[a] = in->x[a][p];
                V[a] = in->v[a][p];
            }
            flags |= orc_interp(f, X, U1);
            for (int a = 0; a < 3; ++a)
                s1[a] = U1[a] - V[a];
            const double f1 = drag_factor(pr, t, s1);
            for (int a = 0; a < 3; ++a) {
                const double A1 = f1 * s1[a] / t + pr->g[a];
                acc[(size_t)p * 3 + a] = A1;
                c1.x[a][p] = X[a] + dt * V[a];
                c1.v[a][p] = V[a] + dt * A1;
            }
            c1.tau[p] = t;
            c1.id[p] = (uint64_t)p;
            seg_of[p] = s;
        }
    }
    int64_t *cnt_mid = mid->count;
    double *mm = carrier(&cm, mid->nseg, mid->base, mid->cap, cnt_mid, ext_mid);
    double *ms = carrier(&cs, nsub * 27, mid_send->base, mid_send->cap, mid_send->count, ext_ms);
    flags |= orc_partition(dc, &c1, &cm, &cs, stay, dir, NULL);
    flags |= orc_append(dc, &cs, stay, &cm);
    for (int t = 0; t < mid->nseg; ++t)
        for (int64_t k = 0; k < mid->count[t] && k < mid->cap[t]; ++k)
            expand(mid, mid->base[t] + k, &cm, mid->base[t] + k, in, acc, seg_of, dir, dc);
    for (int q = 0; q < nsub * 27; ++q)
        for (int64_t k = 0; k < mid_send->count[q] && k < mid_send->cap[q]; ++k)
            expand(mid_send, mid_send->base[q] + k, &cs, mid_send->base[q] + k, in, acc,
                   seg_of, dir, dc);

    /* stage 2 in the new owners, into a carrier pool of the final state */
    orc_pool c2;
    int64_t *cnt2 = (int64_t *)calloc((size_t)(mid->nseg > 0 ? mid->nseg : 1), sizeof(int64_t));
    if (!cnt2)
        abort();
    for (int t = 0; t < mid->nseg; ++t)
        cnt2[t] = mid->count[t] < mid->cap[t] ? mid->count[t] : mid->cap[t];
    double *m2 = carrier(&c2, mid->nseg, mid->base, mid->cap, cnt2, ext_mid);
    for (int t = 0; t < mid->nseg; ++t) {
        for (int64_t k = 0; k < cnt2[t]; ++k) {
            const int64_t r = mid->base[t] + k;
            const double tt = mid->tau[r];
            double Xs[3], U2[3], s2[3];
            for (int a = 0; a < 3; ++a)
                Xs[a] = mid->xs[a][r];
            flags |= orc_interp(f, Xs, U2);
            for (int a = 0; a < 3; ++a)
                s2[a] = U2[a] - mid->vs[a][r];
            const double f2 = drag_factor(pr, tt, s2);
            for (int a = 0; a < 3; ++a) {
                const double A2 = f2 * s2[a] / tt + pr->g[a];
                c2.x[a][r] = mid->x[a][r] + half_dt * (mid->v[a][r] + mid->vs[a][r]);
                c2.v[a][r] = mid->v[a][r] + half_dt * (mid->a[a][r] + A2);
            }
            c2.tau[r] = tt;
            c2.id[r] = mid->id[r];
        }
    }
    flags |= orc_partition(dc, &c2, out, send, stay, NULL, NULL);
    flags |= orc_append(dc, send, stay, out);

    free(m1);
    free(mm);
    free(ms);
    free(m2);
    free(cnt2);
    free(cnt_in);
    free(acc);
    free(seg_of);
    free(dir);
    free(stay);
    return flags;
}
