// pm_device.h -- gfx950 device code of the Lagrangian particle step: every
// kernel and device function, included by the launcher sources (the fused
// and advance kernels' FP64 and FP32 variants compile in separate units).
//
// One step of LCS.jl's particle phase (arXiv 2604.11008):
//   trilinear interpolation of U at X (Sect. 2.2), the Heun (two-stage,
//   second-order) update of dX/dt = V, dV/dt = f (U - V)/tau + g (Sect. 2.2),
//   the boundary-crossing mask generalised to 27 direction codes, the prefix
//   scan that gives each particle a unique slot, packing of the leavers,
//   compaction of the stayers (Sect. 2.3.3) and the receive/append step
//   (unpacking, Sect. 3.2.2).
//
// Design for CDNA4 (64-lane waves, per-XCD L2):
//   * particles are structure-of-arrays; a tile of wg*items records is read
//     striped (record k*wg + tid), so every load and every stayer store of a
//     wave is one contiguous run;
//   * the fused kernel is persistent: workgroups take tiles from an atomic
//     ticket, so a tile only ever waits on tiles that are already running;
//   * within a tile, ranks come from two 64-lane ballots per stripe (stay,
//     leave), a scan of the per-wave counts in LDS, and a decoupled look-back
//     over the tiles of the same segment; one status word per tile packs the
//     two 31-bit counts and a 2-bit state, read and written with agent-scope
//     atomics, so no fence is needed;
//   * the fused kernel publishes a tile's aggregate at once and resolves its
//     look-back and scatter one tile later, from an LDS stash;
//   * leavers are rare: they go to a staging area and are split by direction
//     in a second small kernel.
#ifndef PM_DEVICE_H
#define PM_DEVICE_H

#include <hip/hip_runtime.h>

#include <type_traits>

#include "pm_internal.h"

namespace pm {
namespace {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint64_t lb_load(const uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void lb_store(uint64_t *p, uint64_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void flag_or(uint32_t *hdr, uint32_t f)
{
    __hip_atomic_fetch_or(hdr + kHdrFlags, f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t flags_now(const uint32_t *hdr)
{
    return __hip_atomic_load(hdr + kHdrFlags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t shfl64(uint64_t v, int src)
{
    const int lo = __shfl((int)(uint32_t)v, src, 64);
    const int hi = __shfl((int)(uint32_t)(v >> 32), src, 64);
    return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

template <typename T>
__device__ __forceinline__ T lerp(T a, T b, T t)
{
    return fma(t, b - a, a);
}

__device__ __forceinline__ int dir_o(int d, int a)
{
    return a == 0 ? d % 3 - 1 : (a == 1 ? (d / 3) % 3 - 1 : d / 9 - 1);
}

__device__ __forceinline__ void owner_xyz(const DDecomp &dc, int s, int own[3])
{
    own[0] = s % dc.p[0];
    own[1] = (s / dc.p[0]) % dc.p[1];
    own[2] = s / (dc.p[0] * dc.p[1]);
}

// ---------------------------------------------------------------------------
// trilinear interpolation (Sect. 2.2)
// ---------------------------------------------------------------------------

// Stored corner indices of one axis and the cell fraction (float64); half is
// the nodes' offset in cells: 1/2 for cell centres, 0 for the faces of a
// MAC component along its own axis.
template <bool HALO>
__device__ __forceinline__ double axis_corner(const DField &f, int a, double X, double half,
                                              int &c0, uint32_t &fl)
{
    const int n = f.n[a];
    const double s = X * f.r[a] - half;
    const double fs = floor(s);
    int i;
    if (s != s) {
        i = 0;
    } else if (HALO) {
        if (!(s >= -1.0)) {
            fl |= PM_F_HALO;
            i = -1;
        } else if (!(s < (double)n)) {
            fl |= PM_F_HALO;
            i = n - 1;
        } else {
            i = (int)fs;
        }
    } else {
        if (!(s >= -(double)n)) {
            fl |= PM_F_HALO;
            i = -n;
        } else if (!(s < 2.0 * (double)n)) {
            fl |= PM_F_HALO;
            i = 2 * n - 1;
        } else {
            i = (int)fs;
        }
    }
    if (HALO) {
        c0 = i + 1;
    } else {
        c0 = i < 0 ? i + n : (i >= n ? i - n : i);
    }
    return s - fs;
}

template <bool HALO>
__device__ __forceinline__ int next_corner(const DField &f, int a, int c0)
{
    if (HALO)
        return c0 + 1;
    return c0 + 1 == f.n[a] ? 0 : c0 + 1;
}

// The 2x2x2 stencil of one position: stored corner indices along each axis
// and the cell fractions (computed in float64, rounded to FT).
template <typename FT, bool HALO>
__device__ __forceinline__ void stencil_index(const DField &f, const double X[3], int c0[3],
                                              FT fr[3], uint32_t &fl)
{
#pragma unroll
    for (int a = 0; a < 3; ++a)
        fr[a] = (FT)axis_corner<HALO>(f, a, X[a], 0.5, c0[a], fl);
}

// Two x-adjacent node values in one vector load (16 bytes for double, 8 for
// float).  The address is only FT-aligned, which global loads accept.
template <typename FT>
__device__ __forceinline__ void load_pair(const FT *p, FT &lo, FT &hi)
{
    struct Pair {
        FT a, b;
    } q;
    __builtin_memcpy(&q, p, sizeof q);
    lo = q.a;
    hi = q.b;
}

// Six consecutive values: the three components of two x-adjacent nodes of
// a node-interleaved field (48 bytes for double, 24 for float), in as few
// vector loads as the size allows; the address is only FT-aligned.
template <typename FT>
__device__ __forceinline__ void load_six(const FT *p, FT w[6])
{
    struct Six {
        FT w[6];
    } q;
    __builtin_memcpy(&q, p, sizeof q);
#pragma unroll
    for (int i = 0; i < 6; ++i)
        w[i] = q.w[i];
}

// The 24 node values of a stencil: v[c][2*r + x] for component c, row r
// (y and z corner: 00, 10, 01, 11) and x corner x.  Split arrays: each
// row's x pair of a component is one load.  Interleaved (ILV, the three
// components of a node next to each other): each row's two nodes are one
// run of six values.  Where a periodic field wraps (x corner n-1, then 0)
// the run starts one node earlier and the node at 0 is loaded on its own
// (n >= 2).
template <typename FT, bool HALO, bool ILV>
__device__ __forceinline__ void stencil_load(const DField &f, const int c0[3], FT v[3][8])
{
    const int cx1 = next_corner<HALO>(f, 0, c0[0]);
    const int cy1 = next_corner<HALO>(f, 1, c0[1]);
    const int cz1 = next_corner<HALO>(f, 2, c0[2]);
    const int64_t r[4] = {f.sx * (int64_t)c0[1] + f.sxy * (int64_t)c0[2],
                          f.sx * (int64_t)cy1 + f.sxy * (int64_t)c0[2],
                          f.sx * (int64_t)c0[1] + f.sxy * (int64_t)cz1,
                          f.sx * (int64_t)cy1 + f.sxy * (int64_t)cz1};
    const bool wrap = !HALO && cx1 != c0[0] + 1;
    const int xa = wrap ? c0[0] - 1 : c0[0];
    if constexpr (ILV) {
        const FT *u = (const FT *)f.u[0];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            FT w[6];
            load_six<FT>(u + 3 * (r[k] + xa), w);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                v[c][2 * k] = w[c];
                v[c][2 * k + 1] = w[3 + c];
            }
        }
        if (wrap) {
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    v[c][2 * k] = v[c][2 * k + 1];
                    v[c][2 * k + 1] = u[3 * (r[k] + cx1) + c];
                }
        }
        return;
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const FT *u = (const FT *)f.u[c];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            load_pair<FT>(u + r[k] + xa, v[c][2 * k], v[c][2 * k + 1]);
    }
    if (wrap) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const FT *u = (const FT *)f.u[c];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                v[c][2 * k] = v[c][2 * k + 1];
                v[c][2 * k + 1] = u[r[k] + cx1];
            }
        }
    }
}

// U from a loaded stencil: x-, then y-, then z-lerps.
template <typename FT>
__device__ __forceinline__ void stencil_eval(const FT v[3][8], const FT fr[3], FT U[3])
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const FT l00 = lerp(v[c][0], v[c][1], fr[0]), l10 = lerp(v[c][2], v[c][3], fr[0]);
        const FT l01 = lerp(v[c][4], v[c][5], fr[0]), l11 = lerp(v[c][6], v[c][7], fr[0]);
        U[c] = lerp(lerp(l00, l10, fr[1]), lerp(l01, l11, fr[1]), fr[2]);
    }
}

// MAC fields: each component has its own stencil.  Along axis a,
// component c uses the face-centred corner (offset 0) if a == c, else the
// cell-centred one (offset 1/2); both are found once per axis.
template <typename FT, bool HALO>
__device__ __forceinline__ void mac_index(const DField &f, const double X[3], int c0[3][3],
                                          FT fr[3][3], uint32_t &fl)
{
    int cc[3], cf[3];
    FT fc[3], ff[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        fc[a] = (FT)axis_corner<HALO>(f, a, X[a], 0.5, cc[a], fl);
        ff[a] = (FT)axis_corner<HALO>(f, a, X[a], 0.0, cf[a], fl);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            c0[c][a] = a == c ? cf[a] : cc[a];
            fr[c][a] = a == c ? ff[a] : fc[a];
        }
}

// The 8 node values of one component's stencil, v[2*r + x] as in
// stencil_load (x pairs in one load, the periodic wrap handled the same way).
template <typename FT, bool HALO>
__device__ __forceinline__ void comp_load(const DField &f, int comp, const int c0[3], FT v[8])
{
    const int cx1 = next_corner<HALO>(f, 0, c0[0]);
    const int cy1 = next_corner<HALO>(f, 1, c0[1]);
    const int cz1 = next_corner<HALO>(f, 2, c0[2]);
    const int64_t r[4] = {f.sx * (int64_t)c0[1] + f.sxy * (int64_t)c0[2],
                          f.sx * (int64_t)cy1 + f.sxy * (int64_t)c0[2],
                          f.sx * (int64_t)c0[1] + f.sxy * (int64_t)cz1,
                          f.sx * (int64_t)cy1 + f.sxy * (int64_t)cz1};
    const FT *u = (const FT *)f.u[comp];
    const bool wrap = !HALO && cx1 != c0[0] + 1;
    const int xa = wrap ? c0[0] - 1 : c0[0];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        load_pair<FT>(u + r[k] + xa, v[2 * k], v[2 * k + 1]);
    if (wrap) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[2 * k] = v[2 * k + 1];
            v[2 * k + 1] = u[r[k] + cx1];
        }
    }
}

template <typename FT>
__device__ __forceinline__ FT comp_eval(const FT v[8], const FT fr[3])
{
    const FT l00 = lerp(v[0], v[1], fr[0]), l10 = lerp(v[2], v[3], fr[0]);
    const FT l01 = lerp(v[4], v[5], fr[0]), l11 = lerp(v[6], v[7], fr[0]);
    return lerp(lerp(l00, l10, fr[1]), lerp(l01, l11, fr[1]), fr[2]);
}

// U(X) by trilinear interpolation (Sect. 2.2) from a field of arrangement FA.
template <typename FT, bool HALO, int FA = kFieldSplit>
__device__ __forceinline__ void interp(const DField &f, const double X[3], FT U[3],
                                       uint32_t &fl)
{
    if constexpr (FA == kFieldMac) {
        int c0[3][3];
        FT fr[3][3], v[3][8];
        mac_index<FT, HALO>(f, X, c0, fr, fl);
#pragma unroll
        for (int c = 0; c < 3; ++c)
            comp_load<FT, HALO>(f, c, c0[c], v[c]);
#pragma unroll
        for (int c = 0; c < 3; ++c)
            U[c] = comp_eval<FT>(v[c], fr[c]);
        return;
    }
    int c0[3];
    FT fr[3], v[3][8];
    stencil_index<FT, HALO>(f, X, c0, fr, fl);
    stencil_load<FT, HALO, FA == kFieldIlv>(f, c0, v);
    stencil_eval<FT>(v, fr, U);
}

// ---------------------------------------------------------------------------
// Heun step of the particle ODE (Sect. 2.2, f = 1, plus gravity).
// Velocity-like quantities in FT; positions always in float64.
// ---------------------------------------------------------------------------

template <typename FT> __device__ __forceinline__ FT kdt(const KArgs &a);
template <> __device__ __forceinline__ double kdt<double>(const KArgs &a) { return a.dt; }
template <> __device__ __forceinline__ float kdt<float>(const KArgs &a) { return a.dtf; }
template <typename FT> __device__ __forceinline__ FT khdt(const KArgs &a);
template <> __device__ __forceinline__ double khdt<double>(const KArgs &a) { return a.half_dt; }
template <> __device__ __forceinline__ float khdt<float>(const KArgs &a) { return a.half_dtf; }
template <typename FT> __device__ __forceinline__ FT kkappa(const KArgs &a);
template <> __device__ __forceinline__ double kkappa<double>(const KArgs &a) { return a.kappa; }
template <> __device__ __forceinline__ float kkappa<float>(const KArgs &a) { return a.kappaf; }
template <typename FT> __device__ __forceinline__ FT kg(const KArgs &a, int c);
template <> __device__ __forceinline__ double kg<double>(const KArgs &a, int c) { return a.g[c]; }
template <> __device__ __forceinline__ float kg<float>(const KArgs &a, int c) { return a.gf[c]; }

// Nonlinear drag factor (Sect. 2.2): Re_p = 2 r |V - U| / nu with r from
// tau = (2/9)(rho_p/rho) r^2 / nu is Re_p = kappa sqrt(tau) |V - U|, kappa =
// sqrt(18 / (rho_p/rho nu)) (computed on the host); f = 1 + 0.15 Re_p^0.687.
// Re_p^0.687 as exp2(0.687 log2 Re_p): Re_p >= 0, and 0 gives 0; the
// relative error, a few ulp times |0.687 ln Re_p|, stays far inside the
// tolerance, and it needs much less code and fewer registers than pow.
template <typename FT>
__device__ __forceinline__ FT drag_factor(FT kappa, FT tau, const FT s[3])
{
    const FT re = kappa * sqrt(tau * (s[0] * s[0] + s[1] * s[1] + s[2] * s[2]));
    return (FT)1 + (FT)0.15 * exp2((FT)0.687 * log2(re));
}

// Heun step of one particle.  The stage-2 position X* = X + dt V does not
// depend on the stage-1 interpolation, so both stencils are located first
// and fetched in one round trip; most stage-2 stencils fall in the stage-1
// cell and are not fetched again.  NL: the nonlinear drag factor, else f = 1.
template <typename FT, bool HALO, bool NL, int FA>
__device__ __forceinline__ void advance_one(const KArgs &a, double X[3], FT V[3], FT tau,
                                            uint32_t &fl)
{
    const FT dt = kdt<FT>(a), hdt = khdt<FT>(a);
    double Xs[3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
        Xs[c] = fma(a.dt, (double)V[c], X[c]);
    FT U1[3], U2[3];
    if constexpr (FA == kFieldMac) {
        int c1[3][3], c2[3][3];
        FT fr1[3][3], fr2[3][3], S1[3][8], S2[3][8];
        mac_index<FT, HALO>(a.f, X, c1, fr1, fl);
        mac_index<FT, HALO>(a.f, Xs, c2, fr2, fl);
        bool moved[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            moved[c] = c2[c][0] != c1[c][0] || c2[c][1] != c1[c][1] || c2[c][2] != c1[c][2];
            comp_load<FT, HALO>(a.f, c, c1[c], S1[c]);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c)
            if (moved[c])
                comp_load<FT, HALO>(a.f, c, c2[c], S2[c]);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            U1[c] = comp_eval<FT>(S1[c], fr1[c]);
            U2[c] = moved[c] ? comp_eval<FT>(S2[c], fr2[c]) : comp_eval<FT>(S1[c], fr2[c]);
        }
    } else {
        int c1[3], c2[3];
        FT fr1[3], fr2[3], S1[3][8], S2[3][8];
        stencil_index<FT, HALO>(a.f, X, c1, fr1, fl);
        stencil_index<FT, HALO>(a.f, Xs, c2, fr2, fl);
        const bool moved = c2[0] != c1[0] || c2[1] != c1[1] || c2[2] != c1[2];
        stencil_load<FT, HALO, FA == kFieldIlv>(a.f, c1, S1);
        if (moved)
            stencil_load<FT, HALO, FA == kFieldIlv>(a.f, c2, S2);
        stencil_eval<FT>(S1, fr1, U1);
        if (moved)
            stencil_eval<FT>(S2, fr2, U2);
        else
            stencil_eval<FT>(S1, fr2, U2);
    }
    FT A1[3], Vs[3], s1[3], s2[3];
    const FT it = (FT)1 / tau;
#pragma unroll
    for (int c = 0; c < 3; ++c)
        s1[c] = U1[c] - V[c];
    if (NL) {
        const FT f1 = drag_factor<FT>(kkappa<FT>(a), tau, s1);
#pragma unroll
        for (int c = 0; c < 3; ++c)
            s1[c] = f1 * s1[c];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        A1[c] = fma(s1[c], it, kg<FT>(a, c));
        Vs[c] = fma(dt, A1[c], V[c]);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c)
        s2[c] = U2[c] - Vs[c];
    if (NL) {
        const FT f2 = drag_factor<FT>(kkappa<FT>(a), tau, s2);
#pragma unroll
        for (int c = 0; c < 3; ++c)
            s2[c] = f2 * s2[c];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const FT A2 = fma(s2[c], it, kg<FT>(a, c));
        X[c] = fma(a.half_dt, (double)V[c] + (double)Vs[c], X[c]);
        V[c] = fma(hdt, A1[c] + A2, V[c]);
    }
}

// ---------------------------------------------------------------------------
// boundary-crossing check (Sect. 2.3.3, stage 1) with 27 outcomes
// ---------------------------------------------------------------------------

// Position of one coordinate as stored by the receiver.
__device__ __forceinline__ double shifted(const DDecomp &dc, int a, int k, int o, double x)
{
    if (o < 0 && k == 0) {
        const double w = x + dc.L[a];
        return w < dc.L[a] ? w : dc.predL[a];
    }
    if (o > 0 && k == dc.p[a] - 1)
        return x - dc.L[a];
    return x;
}

__device__ __forceinline__ int classify(const DDecomp &dc, const int own[3],
                                        const double X[3], uint32_t &fl)
{
    if (!isfinite(X[0]) || !isfinite(X[1]) || !isfinite(X[2])) {
        fl |= PM_F_NONFINITE;
        return PM_STAY;
    }
    int o[3];
    bool skip = false;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int k = own[a];
        const double x = X[a];
        int t;
        if (x < dc.b[a][k]) {
            o[a] = -1;
            t = k == 0 ? dc.p[a] - 1 : k - 1;
        } else if (x >= dc.b[a][k + 1]) {
            o[a] = 1;
            t = k == dc.p[a] - 1 ? 0 : k + 1;
        } else {
            o[a] = 0;
            t = k;
        }
        if (o[a] != 0) {
            const double xs = shifted(dc, a, k, o[a], x);
            if (!(dc.b[a][t] <= xs && xs < dc.b[a][t + 1]))
                skip = true;
        }
    }
    if (skip) {
        fl |= PM_F_SKIP;
        return PM_STAY;
    }
    return 9 * (o[2] + 1) + 3 * (o[1] + 1) + (o[0] + 1);
}

// ---------------------------------------------------------------------------
// tiles: ticket, segment lookup, per-tile ranks, look-back
// ---------------------------------------------------------------------------

struct TileHead {
    int64_t q, qhead, first;
    int32_t s, sl, nitems, last;
};

// The cross-tile scan carries two counts per tile, stayers and leavers
// (the paper's send/stay mask); leavers are split by direction afterwards.
template <int WG, int ITEMS>
struct TileLds {
    static constexpr int E = ITEMS * (WG / 64);
    uint32_t cnt[2][E];      // per (stripe, wave) counts, then their tile prefix
    uint32_t agg[2];         // tile totals
    uint32_t base[2];        // the tile's offset within its segment
    uint32_t dcnt[27];       // leavers per direction
    TileHead h;
};

// Segment of ticket q: the largest k with tile_start[k] <= q, searched in ts
// (the workspace's tile table, or a copy of it in LDS).
__device__ __forceinline__ void locate(const KArgs &a, int tile, int64_t q, TileHead &h,
                                       const int64_t *ts)
{
    int lo = 0, hi = a.sub_count;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (ts[mid] <= q)
            lo = mid;
        else
            hi = mid;
    }
    const int s = a.sub_first + lo;
    const int64_t qh = ts[lo];
    const int64_t j = q - qh;
    const int64_t cnt = a.in.count[s];
    const int64_t left = cnt - j * tile;
    h.q = q;
    h.qhead = qh;
    h.s = s;
    h.sl = lo;
    h.first = a.in.base[s] + j * tile;
    h.nitems = (int32_t)(left < tile ? left : tile);
    h.last = (q == ts[lo + 1] - 1);
}

__device__ __forceinline__ uint64_t wave_sum64(uint64_t v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const int lo = __shfl_xor((int)(uint32_t)v, off, 64);
        const int hi = __shfl_xor((int)(uint32_t)(v >> 32), off, 64);
        v += ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
    }
    return v;
}

// Ranks of the tile's valid records: a stayer's among the stayers, a
// leaver's among the leavers; afterwards the record's slot in its segment is
// L.base[c] + L.cnt[c][k*NW + w] + rank[k] (c = 0 stay, 1 leave).
// d == 0xff marks an absent record.
template <int WG, int ITEMS>
__device__ __forceinline__ void tile_ranks(TileLds<WG, ITEMS> &L, const int (&d)[ITEMS],
                                           uint32_t (&rank)[ITEMS])
{
    constexpr int NW = WG / 64;
    constexpr int E = TileLds<WG, ITEMS>::E;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint64_t lt = (1ull << lane) - 1ull;

    for (int e = tid; e < 2 * E; e += WG)
        (&L.cnt[0][0])[e] = 0u;
    if (tid < 27)
        L.dcnt[tid] = 0u;
    __syncthreads();

#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const bool st = d[k] == PM_STAY;
        const bool mg = d[k] < 27 && !st;
        const uint64_t stay = __ballot(st);
        const uint64_t mig = __ballot(mg);
        rank[k] = (uint32_t)__popcll((st ? stay : mig) & lt);
        if (lane == 0) {
            L.cnt[0][k * NW + w] = (uint32_t)__popcll(stay);
            L.cnt[1][k * NW + w] = (uint32_t)__popcll(mig);
        }
        if (mig && mg)
            atomicAdd(&L.dcnt[d[k]], 1u);
    }
    __syncthreads();

    if (tid < 2) {
        uint32_t run = 0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const uint32_t c = L.cnt[tid][e];
            L.cnt[tid][e] = run;
            run += c;
        }
        L.agg[tid] = run;
    }
    __syncthreads();
}

// Decoupled look-back over the tiles of one segment, by wave 0: every lane
// reads one predecessor's status word, so each round trip covers 64 tiles;
// the walk ends at the nearest predecessor with an inclusive prefix, or at
// the segment's first tile.  Writes L.base.
template <int WG, int ITEMS>
__device__ __forceinline__ void lookback(const KArgs &a, TileLds<WG, ITEMS> &L)
{
    const int lane = threadIdx.x;
    if (lane >= 64)
        return;
    const TileHead &h = L.h;
    const uint64_t agg = (uint64_t)L.agg[0] | ((uint64_t)L.agg[1] << 31);
    uint64_t *lb = a.ws.lb;
    uint64_t excl = 0;
    if (h.q == h.qhead) {
        if (lane == 0)
            lb_store(lb + h.q, kLbP | agg);
    } else {
        if (lane == 0)
            lb_store(lb + h.q, kLbA | agg);
        int64_t pb = h.q - 1;
        for (;;) {
            const int64_t t = pb - lane;
            uint64_t v = kLbP;  // before the segment's first tile: a zero prefix
            if (t >= h.qhead) {
                v = lb_load(lb + t);
                while ((v >> 62) == 0ull) {
                    __builtin_amdgcn_s_sleep(1);
                    v = lb_load(lb + t);
                }
            }
            const uint64_t pmask = __ballot((v >> 62) == 2ull);
            if (pmask) {
                const int k = __ffsll((unsigned long long)pmask) - 1;
                excl += wave_sum64(lane <= k ? (v & kLbMask) : 0ull);
                break;
            }
            excl += wave_sum64(v & kLbMask);
            pb -= 64;
        }
        if (lane == 0)
            lb_store(lb + h.q, kLbP | (excl + agg));
    }
    if (lane == 0) {
        L.base[0] = (uint32_t)(excl & kM31);
        L.base[1] = (uint32_t)((excl >> 31) & kM31);
    }
}

// The two halves of lookback() for the fused kernel, which publishes a
// tile's aggregate as soon as its counts are known and walks back later.
template <int WG, int ITEMS>
__device__ __forceinline__ void publish_aggregate(const KArgs &a, const TileLds<WG, ITEMS> &L)
{
    if (threadIdx.x == 0) {
        const uint64_t agg = (uint64_t)L.agg[0] | ((uint64_t)L.agg[1] << 31);
        lb_store(a.ws.lb + L.h.q, (L.h.q == L.h.qhead ? kLbP : kLbA) | agg);
    }
}

template <int WG, int ITEMS>
__device__ __forceinline__ void walk_back(const KArgs &a, TileLds<WG, ITEMS> &L)
{
    const int lane = threadIdx.x;
    if (lane >= 64)
        return;
    const TileHead &h = L.h;
    uint64_t excl = 0;
    if (h.q != h.qhead) {
        const uint64_t *lb = a.ws.lb;
        int64_t pb = h.q - 1;
        for (;;) {
            const int64_t t = pb - lane;
            uint64_t v = kLbP;  // before the segment's first tile: a zero prefix
            if (t >= h.qhead) {
                v = lb_load(lb + t);
                while ((v >> 62) == 0ull) {
                    __builtin_amdgcn_s_sleep(1);
                    v = lb_load(lb + t);
                }
            }
            const uint64_t pmask = __ballot((v >> 62) == 2ull);
            if (pmask) {
                const int k = __ffsll((unsigned long long)pmask) - 1;
                excl += wave_sum64(lane <= k ? (v & kLbMask) : 0ull);
                break;
            }
            excl += wave_sum64(v & kLbMask);
            pb -= 64;
        }
        if (lane == 0) {
            const uint64_t agg = (uint64_t)L.agg[0] | ((uint64_t)L.agg[1] << 31);
            lb_store(a.ws.lb + h.q, kLbP | (excl + agg));
        }
    }
    if (lane == 0) {
        L.base[0] = (uint32_t)(excl & kM31);
        L.base[1] = (uint32_t)((excl >> 31) & kM31);
    }
}

// After the scatter: per-direction leaver counts of the tile into the
// segment's send counts, and the segment totals from its last tile.
template <int WG, int ITEMS>
__device__ __forceinline__ void publish_counts(const KArgs &a, const TileLds<WG, ITEMS> &L)
{
    const int tid = threadIdx.x;
    if (tid < 27 && tid != PM_STAY && L.dcnt[tid])
        atomicAdd((unsigned long long *)&a.send.count[(int64_t)L.h.s * 27 + tid],
                  (unsigned long long)L.dcnt[tid]);
    if (L.h.last && tid == 0) {
        a.ws.stay[L.h.s] = (int64_t)L.base[0] + L.agg[0];
        a.ws.migtot[L.h.s] = (int64_t)L.base[1] + L.agg[1];
    }
}

template <typename FT>
__device__ __forceinline__ void put_record(const DPool &P, int64_t at, const double X[3],
                                           const FT V[3], FT tau, uint64_t id)
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        __builtin_nontemporal_store(X[c], &P.x[c][at]);
        __builtin_nontemporal_store(V[c], &((FT *)P.v[c])[at]);
    }
    __builtin_nontemporal_store(tau, &((FT *)P.tau)[at]);
    __builtin_nontemporal_store(id, &P.id[at]);
}

template <typename FT>
__device__ __forceinline__ void put_staged(const DWS &ws, int64_t at, const double X[3],
                                           const FT V[3], FT tau, uint64_t id, int d)
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        ws.stg_x[c][at] = X[c];
        ((FT *)ws.stg_v[c])[at] = V[c];
    }
    ((FT *)ws.stg_tau)[at] = tau;
    ws.stg_id[at] = id;
    ws.stg_d[at] = (uint8_t)d;
}

__device__ __forceinline__ int neighbour(const DDecomp &dc, int s, int d, int sign)
{
    int o[3];
    owner_xyz(dc, s, o);
    int r[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int P = dc.p[c];
        r[c] = ((o[c] + sign * dir_o(d, c)) % P + P) % P;
    }
    return r[0] + dc.p[0] * (r[1] + dc.p[1] * r[2]);
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

// Exclusive scan over the 256 threads of a workgroup (wave shuffles, then
// the four wave totals); returns the exclusive prefix, *total the sum.
__device__ __forceinline__ int64_t block_scan256(int64_t x, int64_t *wsum, int64_t *total)
{
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    int64_t incl = x;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int lo = __shfl_up((int)(uint32_t)incl, off, 64);
        const int hi = __shfl_up((int)(uint32_t)((uint64_t)incl >> 32), off, 64);
        const int64_t t = (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
        if (lane >= off)
            incl += t;
    }
    if (lane == 63)
        wsum[w] = incl;
    __syncthreads();
    int64_t before = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        before += k < w ? wsum[k] : 0;
        tot += wsum[k];
    }
    __syncthreads();
    *total = tot;
    return before + incl - x;
}

// Per-call set-up: tile table and staging offsets of the segment range
// (workgroup 0), clearing of the look-back words and counts, layout checks.
__global__ __launch_bounds__(256) void k_prep(const KArgs a, int mode)
{
    constexpr int PER = (PM_MAX_NSUB + 255) / 256;
    __shared__ int64_t wsum[4];
    uint32_t *hdr = a.ws.hdr;
    const int tid = threadIdx.x;
    const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + tid;
    const int64_t gsize = (int64_t)gridDim.x * blockDim.x;
    uint32_t bad = 0;
    // look-back words cleared below: enough for every tile of non-overlapping
    // segments within the pool extent (a layout with more tiles is rejected)
    int64_t lb_words = (int64_t)a.ws.pool_extent / a.tile + a.sub_count + 2;
    if (lb_words > a.ws.max_tiles)
        lb_words = a.ws.max_tiles;

    if ((mode & (kPrepTiles | kPrepStaging)) && blockIdx.x == 0) {
        __shared__ int64_t segv[PM_MAX_NSUB];
        for (int pass = 0; pass < 2; ++pass) {
            if (!(mode & (pass == 0 ? kPrepTiles : kPrepStaging)))
                continue;
            // per-segment values, segments strided over the threads so that a
            // segment's loads go out together, then scanned in contiguous runs
            for (int i = tid; i < a.sub_count; i += 256) {
                const int64_t s = a.sub_first + i;
                int64_t c = 0;
                if (pass == 0) {
                    c = a.in.count[s];
                    c = c > 0 ? (c + a.tile - 1) / a.tile : 0;
                } else {
                    int64_t cp[27];
#pragma unroll
                    for (int d = 0; d < 27; ++d)
                        cp[d] = a.send.cap[s * 27 + d];
#pragma unroll
                    for (int d = 0; d < 27; ++d)
                        c += (d != PM_STAY && cp[d] > 0) ? cp[d] : 0;
                    c = (c + 15) & ~(int64_t)15;  // 16-aligned staging areas
                }
                segv[i] = c;
            }
            __syncthreads();
            int64_t v[PER];
            int64_t sum = 0;
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                const int i = tid * PER + k;
                v[k] = i < a.sub_count ? segv[i] : 0;
                sum += v[k];
            }
            int64_t total;
            int64_t run = block_scan256(sum, wsum, &total);
            int64_t *dst = pass == 0 ? a.ws.tile_start : a.ws.stg_start;
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                const int i = tid * PER + k;
                if (i < a.sub_count)
                    dst[i] = run;
                run += v[k];
            }
            if (tid == 0) {
                dst[a.sub_count] = total;
                if (pass == 0) {
                    if (total > a.ws.max_tiles || ((mode & kPrepZeroLb) && total > lb_words)) {
                        bad |= PM_F_LAYOUT;
                        hdr[kHdrTiles] = 0u;
                    } else {
                        hdr[kHdrTiles] = (uint32_t)total;
                    }
                    hdr[kHdrTicket] = 0u;
#pragma unroll
                    for (int g = 0; g < kMaxGroups; ++g)
                        hdr[kHdrGroupTicket + g] = 0u;
                } else if (total > a.ws.stg_extent) {
                    bad |= PM_F_LAYOUT;
                }
            }
            __syncthreads();  // segv is rewritten by the next pass
        }
    }

    if (mode & kPrepZeroLb) {
        for (int64_t i = gtid; i < lb_words; i += gsize)
            a.ws.lb[i] = 0ull;
    }

    if (mode & kPrepZeroCounts) {
        for (int64_t i = gtid; i < (int64_t)a.sub_count * 27; i += gsize) {
            const int64_t s = a.sub_first + i / 27;
            const int d = (int)(i % 27);
            if (d == PM_STAY) {
                a.ws.stay[s] = 0;
                a.ws.migtot[s] = 0;
            }
            a.send.count[s * 27 + d] = 0;
        }
    }

    if (mode & (kPrepCheckIn | kPrepCheckOut)) {
        for (int64_t i = gtid; i < a.sub_count; i += gsize) {
            const int64_t s = a.sub_first + i;
            if (mode & kPrepCheckIn) {
                const int64_t b = a.in.base[s], c = a.in.cap[s], n = a.in.count[s];
                if (b < 0 || c < 0 || n < 0 || n > c || c > (int64_t)kM31 ||
                    b + c > a.ws.pool_extent)
                    bad |= PM_F_LAYOUT;
            }
            if (mode & kPrepCheckOut) {
                const int64_t b = a.out.base[s], c = a.out.cap[s];
                if (b < 0 || c < 0 || c > (int64_t)kM31 || b + c > a.ws.pool_extent)
                    bad |= PM_F_LAYOUT;
            }
        }
    }
    if (mode & kPrepCheckSend) {
        for (int64_t i = gtid; i < (int64_t)a.dc.nsub * 27; i += gsize) {
            const int64_t b = a.send.base[i], c = a.send.cap[i];
            if (b < 0 || c < 0 || c > (int64_t)kM31 || b + c > a.ws.send_extent)
                bad |= PM_F_LAYOUT;
        }
    }
    if (bad)
        flag_or(hdr, bad);
}

// Take the next ticket and find its tile (thread 0); false when done.
//
// With xg > 1 ticket groups, workgroup b draws from the counter of group
// b mod xg, and group g's n-th ticket is tile (n / xb) * xg * xb + g * xb +
// n mod xb: the tile order is cut into blocks of xb consecutive tiles dealt
// to the groups in turn.  A group is an XCD, so the tiles running at once
// on one XCD are neighbours in the cell-sorted order and share their stencil
// sectors in that XCD's L2, while all groups still move through the tile
// order together.  No look-back waits forever: the lowest tile without an
// aggregate is its group's next ticket, and every workgroup of that group is
// at worst walking back over lower tiles, whose aggregates all come.  This
// needs every group to have a running workgroup, which the in-order dispatch
// of workgroups 0..xg-1 gives.
template <int WG, int ITEMS>
__device__ __forceinline__ bool next_tile(const KArgs &a, TileLds<WG, ITEMS> &L,
                                          int64_t total, const int64_t *ts)
{
    if (threadIdx.x == 0) {
        int64_t q;
        if (a.xg > 1) {
            const int g = (int)(blockIdx.x % (uint32_t)a.xg);
            const int64_t n = (int64_t)__hip_atomic_fetch_add(
                a.ws.hdr + kHdrGroupTicket + g, 1u, __ATOMIC_RELAXED,
                __HIP_MEMORY_SCOPE_AGENT);
            q = (n / a.xb) * ((int64_t)a.xg * a.xb) + (int64_t)g * a.xb + n % a.xb;
        } else {
            q = (int64_t)__hip_atomic_fetch_add(a.ws.hdr + kHdrTicket, 1u, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
        }
        L.h.q = q < total ? q : total;
        if (q < total)
            locate(a, a.tile, q, L.h, ts);
    }
    __syncthreads();
    return L.h.q < total;
}

// The tile table of the fused kernel's segment range, copied into LDS when it
// fits (every ticket's segment is found by a binary search over it: in LDS
// the search costs no round trips to the L2).
constexpr int kTileTableLds = 1024;

template <int WG>
__device__ __forceinline__ const int64_t *tile_table(const KArgs &a, int64_t *lds)
{
    if (a.sub_count + 1 > kTileTableLds)
        return a.ws.tile_start;
    for (int i = threadIdx.x; i <= a.sub_count; i += WG)
        lds[i] = a.ws.tile_start[i];
    __syncthreads();
    return lds;
}

// Records of a tile between its advance and its scatter.  Each thread keeps
// its own entries (index k*WG + tid), so no barrier guards them.  Leavers
// are kept with their positions already shifted into the receiver's frame.
template <int WG, int ITEMS, typename FT>
struct TileStash {
    static constexpr int T = WG * ITEMS;
    double x[3][T];
    FT v[3][T];
    FT tau[T];
    uint64_t id[T];
    uint32_t code[T];  // (slot among the tile's stayers or leavers) << 8 | direction
};

// Scatter of a stashed tile once its offsets are known: stayers to `out`,
// leavers to the segment's staging area; then its counts.
template <int WG, int ITEMS, typename FT>
__device__ __forceinline__ void scatter_stash(const KArgs &a, const TileLds<WG, ITEMS> &L,
                                              const TileStash<WG, ITEMS, FT> &S, uint32_t &fl)
{
    const int tid = threadIdx.x;
    const int s = L.h.s;
    const int64_t obase = a.out.base[s], ocap = a.out.cap[s];
    const int64_t g0 = a.ws.stg_start[L.h.sl];
    const int64_t gcap = a.ws.stg_start[L.h.sl + 1] - g0;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const int i = k * WG + tid;
        const uint32_t code = S.code[i];
        const int b = (int)(code & 0xffu);
        if (b == 0xff)
            continue;
        double X[3];
        FT V[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            X[c] = S.x[c][i];
            V[c] = S.v[c][i];
        }
        const FT tau = S.tau[i];
        const uint64_t id = S.id[i];
        if (b == PM_STAY) {
            const int64_t slot = (int64_t)L.base[0] + (code >> 8);
            if (slot < ocap)
                put_record<FT>(a.out, obase + slot, X, V, tau, id);
            else
                fl |= PM_F_DEST_OVERFLOW;
        } else {
            const int64_t m = (int64_t)L.base[1] + (code >> 8);
            if (m < gcap)
                put_staged<FT>(a.ws, g0 + m, X, V, tau, id, b);
            else
                fl |= PM_F_SEND_OVERFLOW;
        }
    }
    publish_counts<WG, ITEMS>(a, L);
}

// The fused step: interpolate + advance + classify + scan + scatter of the
// stayers to `out` and of the leavers to the segment's staging area.
//
// Software-pipelined over the workgroup's tiles: a tile's aggregate is
// published as soon as its counts are known, its records go to the LDS
// stash, and its look-back and scatter run after the workgroup has advanced
// its next tile.  By then the tiles before it have (almost always) published
// their aggregates, so the look-back does not wait on slower neighbours.
// A tile's aggregate never waits on anything, so every walk ends.
// At least two waves per SIMD (one with 8 records per thread, which cannot
// fit two): the compiler spills a few registers rather than halve occupancy.
template <int WG, int ITEMS, typename FT, bool HALO, bool NL, int FA>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(ITEMS >= 8 ? 1 : 2))) void k_step(const KArgs a)
{
    constexpr int NW = WG / 64;
    __shared__ TileLds<WG, ITEMS> L[2];
    __shared__ TileStash<WG, ITEMS, FT> S;
    __shared__ int64_t TT[kTileTableLds];
    uint32_t *hdr = a.ws.hdr;
    if (flags_now(hdr) & PM_F_LAYOUT)
        return;
    const int64_t total = hdr[kHdrTiles];
    const int tid = threadIdx.x, w = tid >> 6;
    uint32_t fl = 0;
    int cur = 0;
    bool pend = false;
    const int64_t *ts = tile_table<WG>(a, TT);

    while (next_tile<WG, ITEMS>(a, L[cur], total, ts)) {
        TileLds<WG, ITEMS> &C = L[cur];
        const int s = C.h.s;
        const int64_t first = C.h.first;
        const int nitems = C.h.nitems;
        int own[3];
        owner_xyz(a.dc, s, own);

        double X[ITEMS][3];
        FT V[ITEMS][3], tau[ITEMS];
        uint64_t id[ITEMS];
        int d[ITEMS];
        uint32_t rank[ITEMS];
        // records past the end of a ragged tile repeat the tile's last one and
        // are dropped after classification, so no lane branches here; the
        // record streams are read once and written once, so they are loaded
        // and stored non-temporally to leave the L2 to the field
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const int i = k * WG + tid;
            const int64_t p = first + (i < nitems ? i : nitems - 1);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                X[k][c] = __builtin_nontemporal_load(&a.in.x[c][p]);
                V[k][c] = __builtin_nontemporal_load(&((const FT *)a.in.v[c])[p]);
            }
            tau[k] = __builtin_nontemporal_load(&((const FT *)a.in.tau)[p]);
            id[k] = __builtin_nontemporal_load(&a.in.id[p]);
        }
        // the stencil gathers are issued at a raised wave priority, so that a
        // SIMD serves waves that can put requests into the L1's miss queue
        // before waves in their scan or scatter (2-4% on the measured
        // workloads, same results)
        __builtin_amdgcn_s_setprio(3);
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            d[k] = 0xff;
            if (k * WG + tid < nitems) {
                advance_one<FT, HALO, NL, FA>(a, X[k], V[k], tau[k], fl);
                d[k] = classify(a.dc, own, X[k], fl);
            }
        }
        __builtin_amdgcn_s_setprio(0);

        tile_ranks<WG, ITEMS>(C, d, rank);
        publish_aggregate<WG, ITEMS>(a, C);

        if (pend) {
            TileLds<WG, ITEMS> &P = L[cur ^ 1];
            walk_back<WG, ITEMS>(a, P);
            __syncthreads();
            scatter_stash<WG, ITEMS, FT>(a, P, S, fl);
        }

#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const int i = k * WG + tid;
            uint32_t code = 0xffu;
            if (d[k] != 0xff) {
                const int b = d[k];
                const int e = k * NW + w;
                if (b == PM_STAY) {
                    code = ((C.cnt[0][e] + rank[k]) << 8) | (uint32_t)b;
                } else {
                    code = ((C.cnt[1][e] + rank[k]) << 8) | (uint32_t)b;
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        X[k][c] = shifted(a.dc, c, own[c], dir_o(b, c), X[k][c]);
                }
            }
            S.code[i] = code;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                S.x[c][i] = X[k][c];
                S.v[c][i] = V[k][c];
            }
            S.tau[i] = tau[k];
            S.id[i] = id[k];
        }
        pend = true;
        cur ^= 1;
        __syncthreads();
    }
    if (pend) {
        TileLds<WG, ITEMS> &P = L[cur ^ 1];
        walk_back<WG, ITEMS>(a, P);
        __syncthreads();
        scatter_stash<WG, ITEMS, FT>(a, P, S, fl);
    }
    if (fl)
        flag_or(hdr, fl);
}

// Plain path, steps 1-2: in-place advance of the range's records.
template <int WG, int ITEMS, typename FT, bool HALO, bool NL, int FA>
__global__ __launch_bounds__(WG) void k_advance(const KArgs a)
{
    __shared__ TileHead H;
    uint32_t *hdr = a.ws.hdr;
    if (flags_now(hdr) & PM_F_LAYOUT)
        return;
    const int64_t total = hdr[kHdrTiles];
    const int tid = threadIdx.x;
    uint32_t fl = 0;
    for (int64_t q = blockIdx.x; q < total; q += gridDim.x) {
        if (tid == 0)
            locate(a, a.tile, q, H, a.ws.tile_start);
        __syncthreads();
        const int64_t first = H.first;
        const int nitems = H.nitems;
        double X[ITEMS][3];
        FT V[ITEMS][3], tau[ITEMS];
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const int i = k * WG + tid;
            const int64_t p = first + (i < nitems ? i : nitems - 1);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                X[k][c] = a.in.x[c][p];
                V[k][c] = ((const FT *)a.in.v[c])[p];
            }
            tau[k] = ((const FT *)a.in.tau)[p];
        }
        __syncthreads();  // H is rewritten by the next tile
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const int i = k * WG + tid;
            if (i < nitems) {
                advance_one<FT, HALO, NL, FA>(a, X[k], V[k], tau[k], fl);
                const int64_t p = first + i;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    a.in.x[c][p] = X[k][c];
                    ((FT *)a.in.v[c])[p] = V[k][c];
                }
            }
        }
    }
    if (fl)
        flag_or(hdr, fl);
}

// Plain path, steps 3-4 (mask, scan): stayers' slots to the workspace,
// leavers to the staging area in scan order.
template <int WG, int ITEMS, typename FT>
__global__ __launch_bounds__(WG) void k_classify(const KArgs a)
{
    constexpr int NW = WG / 64;
    __shared__ TileLds<WG, ITEMS> L;
    uint32_t *hdr = a.ws.hdr;
    if (flags_now(hdr) & PM_F_LAYOUT)
        return;
    const int64_t total = hdr[kHdrTiles];
    const int tid = threadIdx.x, w = tid >> 6;
    uint32_t fl = 0;

    while (next_tile<WG, ITEMS>(a, L, total, a.ws.tile_start)) {
        const int s = L.h.s;
        const int64_t first = L.h.first;
        const int nitems = L.h.nitems;
        int own[3];
        owner_xyz(a.dc, s, own);

        double X[ITEMS][3];
        int d[ITEMS];
        uint32_t rank[ITEMS];
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const int i = k * WG + tid;
            d[k] = 0xff;
            if (i < nitems) {
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    X[k][c] = a.in.x[c][first + i];
                d[k] = classify(a.dc, own, X[k], fl);
            }
        }
        tile_ranks<WG, ITEMS>(L, d, rank);
        lookback<WG, ITEMS>(a, L);
        __syncthreads();

        const int64_t g0 = a.ws.stg_start[L.h.sl];
        const int64_t gcap = a.ws.stg_start[L.h.sl + 1] - g0;
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            if (d[k] == 0xff)
                continue;
            const int b = d[k];
            const int e = k * NW + w;
            const int64_t p = first + k * WG + tid;
            if (b == PM_STAY) {
                a.ws.slot[p] = L.base[0] + L.cnt[0][e] + rank[k];
            } else {
                a.ws.slot[p] = kMigrantSlot;
                const int64_t m = (int64_t)L.base[1] + L.cnt[1][e] + rank[k];
                if (m < gcap) {
                    double Xs[3];
                    FT V[3];
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        Xs[c] = shifted(a.dc, c, own[c], dir_o(b, c), X[k][c]);
                        V[c] = ((const FT *)a.in.v[c])[p];
                    }
                    put_staged<FT>(a.ws, g0 + m, Xs, V, ((const FT *)a.in.tau)[p], a.in.id[p],
                                   b);
                } else {
                    fl |= PM_F_SEND_OVERFLOW;
                }
            }
        }
        publish_counts<WG, ITEMS>(a, L);
        __syncthreads();
    }
    if (fl)
        flag_or(hdr, fl);
}

// Pack: split the staged leavers of each source segment by direction, in
// order, into the send buffers (one workgroup per (segment, direction) job).
// With APPEND the job is indexed by destination t and also appends to
// out[t] after its stayers (the fused step); the (t, stay) job writes
// out.count[t].
template <typename FT>
__device__ __forceinline__ void put_record_x(const DPool &P, int64_t at, const double X[3],
                                             const FT V[3], const double Xs[3], const FT Vs[3],
                                             const FT A[3], FT tau, uint64_t id);

// Particles that subdomain x receives in the directions below d (all 26 for
// d = 27): the send counts of its neighbours, one per lane of wave 0 (every
// lane of the wave must call).
__device__ __forceinline__ int64_t received_before(const KArgs &a, int x, int d)
{
    const int dd = threadIdx.x;
    int64_t c = 0;
    if (dd < d && dd < 27 && dd != PM_STAY) {
        c = a.send.count[(int64_t)neighbour(a.dc, x, dd, -1) * 27 + dd];
        c = c > 0 ? c : 0;
    }
    return (int64_t)wave_sum64((uint64_t)c);
}

template <typename FT, bool APPEND, bool EXT>
__global__ __launch_bounds__(256) void k_route(const KArgs a)
{
    __shared__ uint32_t wcnt[4];
    __shared__ uint32_t list[256 * 16];
    __shared__ int64_t s_off;
    uint32_t *hdr = a.ws.hdr;
    if (flags_now(hdr) & PM_F_LAYOUT)
        return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    uint32_t fl = 0;
    const int64_t jobs = (int64_t)a.sub_count * 27;
    for (int64_t job = blockIdx.x; job < jobs; job += gridDim.x) {
        const int x = a.sub_first + (int)(job / 27);
        const int d = (int)(job % 27);
        if (d == PM_STAY) {
            // out.count[x]: the stayers plus everything received, the 26
            // counts read by 26 lanes at once
            if (APPEND && tid < 64) {
                const int64_t tot = a.ws.stay[x] + received_before(a, x, 27);
                if (tid == 0) {
                    a.out.count[x] = tot;
                    if (tot > a.out.cap[x])
                        fl |= PM_F_DEST_OVERFLOW;
                }
            }
            continue;
        }
        const int src = APPEND ? neighbour(a.dc, x, d, -1) : x;
        const int64_t q = (int64_t)src * 27 + d;
        const int64_t n = a.send.count[q];
        if (n <= 0)
            continue;
        const int64_t scap = a.send.cap[q], sbase = a.send.base[q];
        if (tid == 0 && n > scap)
            fl |= PM_F_SEND_OVERFLOW;
        const int sl = src - a.sub_first;
        const int64_t g0 = a.ws.stg_start[sl];
        int64_t gn = a.ws.stg_start[sl + 1] - g0;
        if (a.ws.migtot[src] < gn)
            gn = a.ws.migtot[src];
        int64_t obase = 0, ocap = 0;
        if (APPEND) {
            if (tid < 64) {
                const int64_t off = a.ws.stay[x] + received_before(a, x, d);
                if (tid == 0)
                    s_off = off;
            }
            obase = a.out.base[x];
            ocap = a.out.cap[x];
            __syncthreads();
        }
        const int64_t off = APPEND ? s_off : 0;
        int64_t run = 0;
        // each thread takes 16 consecutive direction codes (one 16-byte load;
        // staging areas start 16-aligned), so one pass covers 4096 leavers
        for (int64_t i0 = 0; i0 < gn && run < n; i0 += 256 * 16) {
            const int64_t i = i0 + (int64_t)tid * 16;
            uint32_t m = 0;
            if (i < gn) {
                const uint4 q4 = *(const uint4 *)(a.ws.stg_d + g0 + i);
                const uint32_t wd[4] = {q4.x, q4.y, q4.z, q4.w};
#pragma unroll
                for (int b = 0; b < 16; ++b) {
                    const uint32_t code = (wd[b >> 2] >> (8 * (b & 3))) & 0xffu;
                    if (code == (uint32_t)d && i + b < gn)
                        m |= 1u << b;
                }
            }
            const uint32_t cnt = (uint32_t)__popc(m);
            uint32_t incl = cnt;
#pragma unroll
            for (int sh = 1; sh < 64; sh <<= 1) {
                const uint32_t t = (uint32_t)__shfl_up((int)incl, sh, 64);
                if (lane >= sh)
                    incl += t;
            }
            if (lane == 63)
                wcnt[w] = incl;
            __syncthreads();
            uint32_t before = 0, tot = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t c = wcnt[k];
                before += k < w ? c : 0u;
                tot += c;
            }
            // the matches' staging indices, in order, then one copy per thread
            uint32_t k = before + incl - cnt;
            while (m) {
                const int b = __ffs(m) - 1;
                m &= m - 1;
                list[k++] = (uint32_t)(i - i0 + b);
            }
            __syncthreads();
            for (uint32_t j = tid; j < tot; j += 256) {
                const int64_t slot = run + j;
                if (slot < scap) {
                    const int64_t from = g0 + i0 + list[j];
                    double X[3];
                    FT V[3];
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        X[c] = a.ws.stg_x[c][from];
                        V[c] = ((const FT *)a.ws.stg_v[c])[from];
                    }
                    const FT t = ((const FT *)a.ws.stg_tau)[from];
                    const uint64_t idv = a.ws.stg_id[from];
                    if constexpr (EXT) {
                        double Xs[3];
                        FT Vs[3], A[3];
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            Xs[c] = a.ws.stg_xs[c][from];
                            Vs[c] = ((const FT *)a.ws.stg_vs[c])[from];
                            A[c] = ((const FT *)a.ws.stg_a[c])[from];
                        }
                        put_record_x<FT>(a.send, sbase + slot, X, V, Xs, Vs, A, t, idv);
                        if (APPEND && off + slot < ocap)
                            put_record_x<FT>(a.out, obase + off + slot, X, V, Xs, Vs, A, t,
                                             idv);
                    } else {
                        put_record<FT>(a.send, sbase + slot, X, V, t, idv);
                        if (APPEND && off + slot < ocap)
                            put_record<FT>(a.out, obase + off + slot, X, V, t, idv);
                    }
                }
            }
            run += tot;
            __syncthreads();
        }
        if (APPEND)
            __syncthreads();  // s_off is rewritten by the next job
    }
    if (fl)
        flag_or(hdr, fl);
}

// Plain path, unpacking part 1: stayers of `in` to their slots in `out`.
template <int WG, int ITEMS, typename FT>
__global__ __launch_bounds__(WG) void k_compact(const KArgs a)
{
    __shared__ TileHead H;
    uint32_t *hdr = a.ws.hdr;
    if (flags_now(hdr) & PM_F_LAYOUT)
        return;
    const int64_t total = hdr[kHdrTiles];
    const int tid = threadIdx.x;
    uint32_t fl = 0;
    for (int64_t q = blockIdx.x; q < total; q += gridDim.x) {
        if (tid == 0)
            locate(a, a.tile, q, H, a.ws.tile_start);
        __syncthreads();
        const int s = H.s;
        const int64_t first = H.first;
        const int nitems = H.nitems;
        const int64_t obase = a.out.base[s], ocap = a.out.cap[s];
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const int i = k * WG + tid;
            if (i < nitems) {
                const int64_t p = first + i;
                const uint32_t sl = a.ws.slot[p];
                if (sl != kMigrantSlot) {
                    if ((int64_t)sl < ocap) {
                        double X[3];
                        FT V[3];
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            X[c] = a.in.x[c][p];
                            V[c] = ((const FT *)a.in.v[c])[p];
                        }
                        put_record<FT>(a.out, obase + sl, X, V, ((const FT *)a.in.tau)[p],
                                       a.in.id[p]);
                    } else {
                        fl |= PM_F_DEST_OVERFLOW;
                    }
                }
            }
        }
        __syncthreads();
    }
    if (fl)
        flag_or(hdr, fl);
}

// Plain path, unpacking part 2: what every destination t of the range
// receives, after its stayers, direction code ascending, each send buffer
// in order.
template <typename FT>
__global__ __launch_bounds__(256) void k_append(const KArgs a)
{
    __shared__ int64_t off[28], stored[27], sbase[27];
    uint32_t *hdr = a.ws.hdr;
    if (flags_now(hdr) & PM_F_LAYOUT)
        return;
    const int tid = threadIdx.x;
    uint32_t fl = 0;
    const int64_t jobs = (int64_t)a.sub_count * a.cpt;
    for (int64_t job = blockIdx.x; job < jobs; job += gridDim.x) {
        const int t = a.sub_first + (int)(job / a.cpt);
        const int part = (int)(job % a.cpt);
        if (tid < 27) {
            int64_t n = 0, st = 0, sb = 0;
            if (tid != PM_STAY) {
                const int64_t qq = (int64_t)neighbour(a.dc, t, tid, -1) * 27 + tid;
                n = a.send.count[qq];
                n = n < 0 ? 0 : n;
                const int64_t cp = a.send.cap[qq];
                st = n < cp ? n : cp;
                sb = a.send.base[qq];
            }
            off[tid] = n;
            stored[tid] = st;
            sbase[tid] = sb;
        }
        __syncthreads();
        if (tid == 0) {
            int64_t run = 0;
            for (int dd = 0; dd < 27; ++dd) {
                const int64_t n = off[dd];
                off[dd] = run;
                run += n;
            }
            off[27] = run;
        }
        __syncthreads();
        const int64_t stay = a.ws.stay[t] < 0 ? 0 : a.ws.stay[t];
        const int64_t recv = off[27];
        const int64_t obase = a.out.base[t], ocap = a.out.cap[t];
        if (part == 0 && tid == 0) {
            a.out.count[t] = stay + recv;
            if (stay + recv > ocap)
                fl |= PM_F_DEST_OVERFLOW;
        }
        for (int64_t i = (int64_t)part * 256 + tid; i < recv; i += (int64_t)a.cpt * 256) {
            int dd = 0;
            while (dd < 26 && off[dd + 1] <= i)
                ++dd;
            const int64_t k = i - off[dd];
            const int64_t pos = stay + i;
            if (k < stored[dd] && pos < ocap) {
                const int64_t p = sbase[dd] + k;
                double X[3];
                FT V[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    X[c] = a.send.x[c][p];
                    V[c] = ((const FT *)a.send.v[c])[p];
                }
                put_record<FT>(a.out, obase + pos, X, V, ((const FT *)a.send.tau)[p],
                               a.send.id[p]);
            }
        }
        __syncthreads();
    }
    if (fl)
        flag_or(hdr, fl);
}

template <typename FT, bool HALO, int FA>
__global__ __launch_bounds__(256) void k_interp(const KArgs a, int64_t n, const double *x,
                                                const double *y, const double *z, FT *ux,
                                                FT *uy, FT *uz)
{
    uint32_t fl = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * 256) {
        const double X[3] = {x[i], y[i], z[i]};
        FT U[3];
        interp<FT, HALO, FA>(a.f, X, U, fl);
        ux[i] = U[0];
        uy[i] = U[1];
        uz[i] = U[2];
    }
    if (fl)
        flag_or(a.ws.hdr, fl);
}

// Diagnostic: mark the nodes of the stage-1 (X) and stage-2 (X + dt V)
// stencils of every particle of the range.
template <typename FT, bool HALO>
__global__ __launch_bounds__(256) void k_touch(const KArgs a, uint64_t *bits)
{
    const int64_t total = a.ws.hdr[kHdrTiles];
    uint32_t fl = 0;
    for (int64_t q = blockIdx.x; q < total; q += gridDim.x) {
        TileHead h;
        locate(a, a.tile, q, h, a.ws.tile_start);
        for (int i = threadIdx.x; i < h.nitems; i += 256) {
            const int64_t p = h.first + i;
            double X[2][3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                X[0][c] = a.in.x[c][p];
                X[1][c] = fma(a.dt, (double)((const FT *)a.in.v[c])[p], X[0][c]);
            }
            // collocated: one stencil for all components; MAC: one per
            // component, marked in its own third of the bitmap
            const int64_t nodes = a.f.sxy * (a.f.n[2] + 2 * a.f.halo);
            const int ncomp = a.f.stagger ? 3 : 1;
            for (int st = 0; st < 2; ++st) {
                for (int comp = 0; comp < ncomp; ++comp) {
                    int c0[3];
                    for (int ax = 0; ax < 3; ++ax)
                        axis_corner<HALO>(a.f, ax, X[st][ax],
                                          a.f.stagger && ax == comp ? 0.0 : 0.5, c0[ax], fl);
                    for (int cz = 0; cz < 2; ++cz)
                        for (int cy = 0; cy < 2; ++cy)
                            for (int cx = 0; cx < 2; ++cx) {
                                const int ix = cx ? next_corner<HALO>(a.f, 0, c0[0]) : c0[0];
                                const int iy = cy ? next_corner<HALO>(a.f, 1, c0[1]) : c0[1];
                                const int iz = cz ? next_corner<HALO>(a.f, 2, c0[2]) : c0[2];
                                const int64_t node =
                                    comp * nodes + ix + a.f.sx * iy + a.f.sxy * iz;
                                atomicOr((unsigned long long *)&bits[node >> 6],
                                         1ull << (node & 63));
                            }
                }
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_popcount(const uint64_t *bits, int64_t words,
                                                  unsigned long long *out)
{
    unsigned long long c = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < words;
         i += (int64_t)gridDim.x * 256)
        c += __popcll(bits[i]);
    for (int off = 32; off > 0; off >>= 1)
        c += __shfl_down(c, off, 64);
    if ((threadIdx.x & 63) == 0)
        atomicAdd(out, c);
}

__global__ __launch_bounds__(256) void k_fill(uint64_t *p, int64_t words)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < words;
         i += (int64_t)gridDim.x * 256)
        p[i] = 0ull;
}

// The flag word of a workspace header handed to the caller (dst, when not
// NULL) and cleared, so that the next step starts without flags.  Runs
// after every other kernel of a step on the same stream.
__global__ __launch_bounds__(64) void k_flags_move(uint32_t *hdr, uint32_t *dst)
{
    if (threadIdx.x == 0) {
        const uint32_t f = flags_now(hdr);
        if (dst)
            *dst = f;
        __hip_atomic_store(hdr + kHdrFlags, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// ---------------------------------------------------------------------------
// migration after each RK2 stage (the paper's scheme, Sect. 3.2.2): the
// mid-step record carries X_n, V_n, X*, V* and the stage-1 acceleration a
// ---------------------------------------------------------------------------

// Stage 1 of the Heun step: X* = X + dt V, V* = V + dt a, a = f (U(X) - V)/tau + g
// (the same operations as advance_one's first stage).
template <typename FT, bool HALO, bool NL, int FA>
__device__ __forceinline__ void heun_stage1(const KArgs &a, const double X[3], const FT V[3],
                                            FT tau, double Xs[3], FT Vs[3], FT A1[3],
                                            uint32_t &fl)
{
    FT U1[3], s1[3];
    interp<FT, HALO, FA>(a.f, X, U1, fl);
    const FT it = (FT)1 / tau;
#pragma unroll
    for (int c = 0; c < 3; ++c)
        s1[c] = U1[c] - V[c];
    if (NL) {
        const FT f1 = drag_factor<FT>(kkappa<FT>(a), tau, s1);
#pragma unroll
        for (int c = 0; c < 3; ++c)
            s1[c] = f1 * s1[c];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        A1[c] = fma(s1[c], it, kg<FT>(a, c));
        Vs[c] = fma(kdt<FT>(a), A1[c], V[c]);
        Xs[c] = fma(a.dt, (double)V[c], X[c]);
    }
}

// Stage 2 in the new owner: X' = X + dt/2 (V + V*), V' = V + dt/2 (a + a(X*, V*)).
template <typename FT, bool HALO, bool NL, int FA>
__device__ __forceinline__ void heun_stage2(const KArgs &a, double X[3], FT V[3],
                                            const double Xs[3], const FT Vs[3],
                                            const FT A1[3], FT tau, uint32_t &fl)
{
    FT U2[3], s2[3];
    interp<FT, HALO, FA>(a.f, Xs, U2, fl);
    const FT it = (FT)1 / tau;
#pragma unroll
    for (int c = 0; c < 3; ++c)
        s2[c] = U2[c] - Vs[c];
    if (NL) {
        const FT f2 = drag_factor<FT>(kkappa<FT>(a), tau, s2);
#pragma unroll
        for (int c = 0; c < 3; ++c)
            s2[c] = f2 * s2[c];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const FT A2 = fma(s2[c], it, kg<FT>(a, c));
        X[c] = fma(a.half_dt, (double)V[c] + (double)Vs[c], X[c]);
        V[c] = fma(khdt<FT>(a), A1[c] + A2, V[c]);
    }
}

// X_n of a stage-1 leaver in the receiver's periodic image: the same +-L as
// X* (x - L leaving through L, x + L leaving through 0), plain arithmetic.
__device__ __forceinline__ double shifted_plain(const DDecomp &dc, int a, int k, int o, double x)
{
    if (o > 0 && k == dc.p[a] - 1)
        return x - dc.L[a];
    if (o < 0 && k == 0)
        return x + dc.L[a];
    return x;
}

template <typename FT>
__device__ __forceinline__ void put_record_x(const DPool &P, int64_t at, const double X[3],
                                             const FT V[3], const double Xs[3], const FT Vs[3],
                                             const FT A[3], FT tau, uint64_t id)
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        __builtin_nontemporal_store(X[c], &P.x[c][at]);
        __builtin_nontemporal_store(V[c], &((FT *)P.v[c])[at]);
        __builtin_nontemporal_store(Xs[c], &P.xs[c][at]);
        __builtin_nontemporal_store(Vs[c], &((FT *)P.vs[c])[at]);
        __builtin_nontemporal_store(A[c], &((FT *)P.a[c])[at]);
    }
    __builtin_nontemporal_store(tau, &((FT *)P.tau)[at]);
    __builtin_nontemporal_store(id, &P.id[at]);
}

template <typename FT>
__device__ __forceinline__ void put_staged_x(const DWS &ws, int64_t at, const double X[3],
                                             const FT V[3], const double Xs[3], const FT Vs[3],
                                             const FT A[3], FT tau, uint64_t id, int d)
{
    put_staged<FT>(ws, at, X, V, tau, id, d);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        ws.stg_xs[c][at] = Xs[c];
        ((FT *)ws.stg_vs[c])[at] = Vs[c];
        ((FT *)ws.stg_a[c])[at] = A[c];
    }
}

// The stash of a stage-1 tile: mid-step records.
template <int WG, int ITEMS, typename FT>
struct TileStashX {
    static constexpr int T = WG * ITEMS;
    double x[3][T], xs[3][T];
    FT v[3][T], vs[3][T], a[3][T];
    FT tau[T];
    uint64_t id[T];
    uint32_t code[T];
};

template <int WG, int ITEMS, typename FT>
__device__ __forceinline__ void scatter_stash_x(const KArgs &a, const TileLds<WG, ITEMS> &L,
                                                const TileStashX<WG, ITEMS, FT> &S,
                                                uint32_t &fl)
{
    const int tid = threadIdx.x;
    const int s = L.h.s;
    const int64_t obase = a.out.base[s], ocap = a.out.cap[s];
    const int64_t g0 = a.ws.stg_start[L.h.sl];
    const int64_t gcap = a.ws.stg_start[L.h.sl + 1] - g0;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const int i = k * WG + tid;
        const uint32_t code = S.code[i];
        const int b = (int)(code & 0xffu);
        if (b == 0xff)
            continue;
        double X[3], Xs[3];
        FT V[3], Vs[3], A[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            X[c] = S.x[c][i];
            Xs[c] = S.xs[c][i];
            V[c] = S.v[c][i];
            Vs[c] = S.vs[c][i];
            A[c] = S.a[c][i];
        }
        if (b == PM_STAY) {
            const int64_t slot = (int64_t)L.base[0] + (code >> 8);
            if (slot < ocap)
                put_record_x<FT>(a.out, obase + slot, X, V, Xs, Vs, A, S.tau[i], S.id[i]);
            else
                fl |= PM_F_DEST_OVERFLOW;
        } else {
            const int64_t m = (int64_t)L.base[1] + (code >> 8);
            if (m < gcap)
                put_staged_x<FT>(a.ws, g0 + m, X, V, Xs, Vs, A, S.tau[i], S.id[i], b);
            else
                fl |= PM_F_SEND_OVERFLOW;
        }
    }
    publish_counts<WG, ITEMS>(a, L);
}

// The fused kernel of one stage of per-stage migration, with the tile
// pipeline of k_step.  STAGE 1: plain records of `in` -> stage 1 ->
// classified by X* -> mid-step records to `out` / the staging area.
// STAGE 2: mid-step records of `in` -> stage 2 -> classified by X' -> plain
// records to `out` / the staging area.
template <int WG, int ITEMS, typename FT, bool HALO, bool NL, int STAGE, int FA>
__global__ __launch_bounds__(WG) void k_stage(const KArgs a)
{
    constexpr int NW = WG / 64;
    __shared__ TileLds<WG, ITEMS> L[2];
    using Stash = typename std::conditional<STAGE == 1, TileStashX<WG, ITEMS, FT>,
                                            TileStash<WG, ITEMS, FT>>::type;
    __shared__ Stash S;
    uint32_t *hdr = a.ws.hdr;
    if (flags_now(hdr) & PM_F_LAYOUT)
        return;
    const int64_t total = hdr[kHdrTiles];
    const int tid = threadIdx.x, w = tid >> 6;
    uint32_t fl = 0;
    int cur = 0;
    bool pend = false;

    while (next_tile<WG, ITEMS>(a, L[cur], total, a.ws.tile_start)) {
        TileLds<WG, ITEMS> &C = L[cur];
        const int s = C.h.s;
        const int64_t first = C.h.first;
        const int nitems = C.h.nitems;
        int own[3];
        owner_xyz(a.dc, s, own);

        double X[ITEMS][3], Xs[ITEMS][3];
        FT V[ITEMS][3], Vs[ITEMS][3], A[ITEMS][3], tau[ITEMS];
        uint64_t id[ITEMS];
        int d[ITEMS];
        uint32_t rank[ITEMS];
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const int i = k * WG + tid;
            const int64_t p = first + (i < nitems ? i : nitems - 1);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                X[k][c] = __builtin_nontemporal_load(&a.in.x[c][p]);
                V[k][c] = __builtin_nontemporal_load(&((const FT *)a.in.v[c])[p]);
                if (STAGE == 2) {
                    Xs[k][c] = __builtin_nontemporal_load(&a.in.xs[c][p]);
                    Vs[k][c] = __builtin_nontemporal_load(&((const FT *)a.in.vs[c])[p]);
                    A[k][c] = __builtin_nontemporal_load(&((const FT *)a.in.a[c])[p]);
                }
            }
            tau[k] = __builtin_nontemporal_load(&((const FT *)a.in.tau)[p]);
            id[k] = __builtin_nontemporal_load(&a.in.id[p]);
        }
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            d[k] = 0xff;
            if (k * WG + tid < nitems) {
                if (STAGE == 1) {
                    heun_stage1<FT, HALO, NL, FA>(a, X[k], V[k], tau[k], Xs[k], Vs[k], A[k], fl);
                    d[k] = classify(a.dc, own, Xs[k], fl);
                } else {
                    heun_stage2<FT, HALO, NL, FA>(a, X[k], V[k], Xs[k], Vs[k], A[k], tau[k], fl);
                    d[k] = classify(a.dc, own, X[k], fl);
                }
            }
        }

        tile_ranks<WG, ITEMS>(C, d, rank);
        publish_aggregate<WG, ITEMS>(a, C);

        if (pend) {
            TileLds<WG, ITEMS> &P = L[cur ^ 1];
            walk_back<WG, ITEMS>(a, P);
            __syncthreads();
            if constexpr (STAGE == 1)
                scatter_stash_x<WG, ITEMS, FT>(a, P, S, fl);
            else
                scatter_stash<WG, ITEMS, FT>(a, P, S, fl);
        }

#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const int i = k * WG + tid;
            uint32_t code = 0xffu;
            if (d[k] != 0xff) {
                const int b = d[k];
                const int e = k * NW + w;
                code = ((C.cnt[b == PM_STAY ? 0 : 1][e] + rank[k]) << 8) | (uint32_t)b;
                if (b != PM_STAY) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        if (STAGE == 1) {
                            Xs[k][c] = shifted(a.dc, c, own[c], dir_o(b, c), Xs[k][c]);
                            X[k][c] = shifted_plain(a.dc, c, own[c], dir_o(b, c), X[k][c]);
                        } else {
                            X[k][c] = shifted(a.dc, c, own[c], dir_o(b, c), X[k][c]);
                        }
                    }
                }
            }
            if constexpr (STAGE == 1) {
                S.code[i] = code;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    S.x[c][i] = X[k][c];
                    S.v[c][i] = V[k][c];
                    S.xs[c][i] = Xs[k][c];
                    S.vs[c][i] = Vs[k][c];
                    S.a[c][i] = A[k][c];
                }
                S.tau[i] = tau[k];
                S.id[i] = id[k];
            } else {
                S.code[i] = code;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    S.x[c][i] = X[k][c];
                    S.v[c][i] = V[k][c];
                }
                S.tau[i] = tau[k];
                S.id[i] = id[k];
            }
        }
        pend = true;
        cur ^= 1;
        __syncthreads();
    }
    if (pend) {
        TileLds<WG, ITEMS> &P = L[cur ^ 1];
        walk_back<WG, ITEMS>(a, P);
        __syncthreads();
        if constexpr (STAGE == 1)
            scatter_stash_x<WG, ITEMS, FT>(a, P, S, fl);
        else
            scatter_stash<WG, ITEMS, FT>(a, P, S, fl);
    }
    if (fl)
        flag_or(hdr, fl);
}

// ---------------------------------------------------------------------------
// dispatch over launch shapes and precisions
// ---------------------------------------------------------------------------

#define PM_SHAPES(X) X(256, 1) X(256, 2) X(256, 4) X(256, 8) X(512, 1) X(512, 2) X(512, 4)
// per-stage migration: tiles of at most 1024 mid-step records fit the LDS
#define PM_STAGE_SHAPES(X) X(256, 1) X(256, 2) X(256, 4) X(512, 1) X(512, 2)

// The fused and advance kernels come in element type x halo x drag law
// variants; Kern<W, I>::step/advance pick the one for the launch.
template <int W, int I>
struct Kern {
    template <typename FT, bool H, bool NL, int FA>
    static hipError_t step_t(const KArgs &a, int grid, hipStream_t st)
    {
        hipLaunchKernelGGL((k_step<W, I, FT, H, NL, FA>), dim3(grid), dim3(W), 0, st, a);
        return hipGetLastError();
    }
    template <typename FT, bool H, bool NL, int FA>
    static hipError_t advance_t(const KArgs &a, int grid, hipStream_t st)
    {
        hipLaunchKernelGGL((k_advance<W, I, FT, H, NL, FA>), dim3(grid), dim3(W), 0, st, a);
        return hipGetLastError();
    }
    template <typename FT, bool H, bool NL, int FA>
    static int occupancy_t()
    {
        int nb = 1;
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (k_step<W, I, FT, H, NL, FA>),
                                                           W, 0);
        return nb;
    }
    // the halo x drag-law variants of one element type and field arrangement FA
    template <typename FT, int FA>
    static hipError_t step_ft(const KArgs &a, int grid, hipStream_t st)
    {
        const bool h = a.f.halo != 0, nl = a.drag != 0;
        return h ? (nl ? step_t<FT, true, true, FA>(a, grid, st)
                       : step_t<FT, true, false, FA>(a, grid, st))
                 : (nl ? step_t<FT, false, true, FA>(a, grid, st)
                       : step_t<FT, false, false, FA>(a, grid, st));
    }
    template <typename FT, int FA>
    static hipError_t advance_ft(const KArgs &a, int grid, hipStream_t st)
    {
        const bool h = a.f.halo != 0, nl = a.drag != 0;
        return h ? (nl ? advance_t<FT, true, true, FA>(a, grid, st)
                       : advance_t<FT, true, false, FA>(a, grid, st))
                 : (nl ? advance_t<FT, false, true, FA>(a, grid, st)
                       : advance_t<FT, false, false, FA>(a, grid, st));
    }
    template <typename FT, bool H, bool NL, int STG, int FA>
    static hipError_t stage_t(const KArgs &a, int grid, hipStream_t st)
    {
        hipLaunchKernelGGL((k_stage<W, I, FT, H, NL, STG, FA>), dim3(grid), dim3(W), 0, st, a);
        return hipGetLastError();
    }
    template <typename FT, bool H, bool NL, int STG, int FA>
    static int stage_occ_t()
    {
        int nb = 1;
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, (k_stage<W, I, FT, H, NL, STG, FA>), W, 0);
        return nb;
    }
    // the halo x drag-law variants of one stage of per-stage migration on a
    // collocated field of layout FA (split or interleaved)
    template <typename FT, int STG, int FA>
    static hipError_t stage_ft(const KArgs &a, int grid, hipStream_t st)
    {
        const bool h = a.f.halo != 0, nl = a.drag != 0;
        return h ? (nl ? stage_t<FT, true, true, STG, FA>(a, grid, st)
                       : stage_t<FT, true, false, STG, FA>(a, grid, st))
                 : (nl ? stage_t<FT, false, true, STG, FA>(a, grid, st)
                       : stage_t<FT, false, false, STG, FA>(a, grid, st));
    }
    template <typename FT, int STG, int FA>
    static int stage_occ_ft(bool h, bool nl)
    {
        return h ? (nl ? stage_occ_t<FT, true, true, STG, FA>()
                       : stage_occ_t<FT, true, false, STG, FA>())
                 : (nl ? stage_occ_t<FT, false, true, STG, FA>()
                       : stage_occ_t<FT, false, false, STG, FA>());
    }
    template <typename FT, int FA>
    static int occupancy_ft(bool h, bool nl)
    {
        return h ? (nl ? occupancy_t<FT, true, true, FA>() : occupancy_t<FT, true, false, FA>())
                 : (nl ? occupancy_t<FT, false, true, FA>() : occupancy_t<FT, false, false, FA>());
    }
};

}  // namespace
}  // namespace pm

#endif
