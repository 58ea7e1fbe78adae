// pm_kernels.hip -- gfx950 kernels of the Lagrangian particle step.
//
// One step of LCS.jl's particle phase (arXiv 2604.11008):
//   trilinear interpolation of U at X (Sect. 2.2), the Heun (two-stage,
//   second-order) update of dX/dt = V, dV/dt = (U - V)/tau + g (Sect. 2.2),
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
//   * within a tile, ranks come from 64-lane ballots (one ballot per stripe
//     while every lane stays; one more per distinct direction otherwise),
//     a per-bucket scan of the per-wave counts in LDS, and a decoupled
//     look-back over the tiles of the same segment; each status word packs
//     two 31-bit bucket counts and a 2-bit state, so a tile's state is 14
//     words read and written with agent-scope atomics and needs no fence;
//   * migrants are rare, so they take a slow path (extra ballots, scattered
//     stores) that the common all-stay wave never enters.
#include <hip/hip_runtime.h>

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

// Stored corner indices of one axis and the cell fraction (float64).
template <bool HALO>
__device__ __forceinline__ double axis_corner(const DField &f, int a, double X, int &c0,
                                              uint32_t &fl)
{
    const int n = f.n[a];
    const double s = X * f.r[a] - 0.5;
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

// U(X) with the field in FT; the weights are the float64 fractions rounded
// to FT.  Evaluated as x-, then y-, then z-lerps.
template <typename FT, bool HALO>
__device__ __forceinline__ void interp(const DField &f, const double X[3], FT U[3],
                                       uint32_t &fl)
{
    int cx0, cy0, cz0;
    const FT fx = (FT)axis_corner<HALO>(f, 0, X[0], cx0, fl);
    const FT fy = (FT)axis_corner<HALO>(f, 1, X[1], cy0, fl);
    const FT fz = (FT)axis_corner<HALO>(f, 2, X[2], cz0, fl);
    const int cx1 = next_corner<HALO>(f, 0, cx0);
    const int cy1 = next_corner<HALO>(f, 1, cy0);
    const int cz1 = next_corner<HALO>(f, 2, cz0);
    const int64_t r00 = f.sx * (int64_t)cy0 + f.sxy * (int64_t)cz0;
    const int64_t r10 = f.sx * (int64_t)cy1 + f.sxy * (int64_t)cz0;
    const int64_t r01 = f.sx * (int64_t)cy0 + f.sxy * (int64_t)cz1;
    const int64_t r11 = f.sx * (int64_t)cy1 + f.sxy * (int64_t)cz1;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const FT *u = (const FT *)f.u[c];
        const FT a00 = u[r00 + cx0], b00 = u[r00 + cx1];
        const FT a10 = u[r10 + cx0], b10 = u[r10 + cx1];
        const FT a01 = u[r01 + cx0], b01 = u[r01 + cx1];
        const FT a11 = u[r11 + cx0], b11 = u[r11 + cx1];
        const FT l00 = lerp(a00, b00, fx), l10 = lerp(a10, b10, fx);
        const FT l01 = lerp(a01, b01, fx), l11 = lerp(a11, b11, fx);
        U[c] = lerp(lerp(l00, l10, fy), lerp(l01, l11, fy), fz);
    }
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
template <typename FT> __device__ __forceinline__ FT kg(const KArgs &a, int c);
template <> __device__ __forceinline__ double kg<double>(const KArgs &a, int c) { return a.g[c]; }
template <> __device__ __forceinline__ float kg<float>(const KArgs &a, int c) { return a.gf[c]; }

template <typename FT, bool HALO>
__device__ __forceinline__ void advance(const KArgs &a, double X[3], FT V[3], FT tau,
                                        uint32_t &fl)
{
    const FT it = (FT)1 / tau;
    const FT dt = kdt<FT>(a), hdt = khdt<FT>(a);
    FT U1[3], A1[3], Vs[3], U2[3];
    double Xs[3];
    interp<FT, HALO>(a.f, X, U1, fl);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        A1[c] = fma(U1[c] - V[c], it, kg<FT>(a, c));
        Xs[c] = fma(a.dt, (double)V[c], X[c]);
        Vs[c] = fma(dt, A1[c], V[c]);
    }
    interp<FT, HALO>(a.f, Xs, U2, fl);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const FT A2 = fma(U2[c] - Vs[c], it, kg<FT>(a, c));
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
    int32_t s, nitems, last;
};

template <int WG, int ITEMS>
struct TileLds {
    static constexpr int E = ITEMS * (WG / 64);
    uint32_t cnt[27][E];     // per (stripe, wave) counts, then their tile prefix
    uint32_t agg[27];        // tile totals
    uint32_t base[27];       // tile's offset within its segment
    uint32_t present;        // buckets that occur in the tile
    TileHead h;
};

// Segment of ticket q: the largest k with tile_start[k] <= q.
__device__ __forceinline__ void locate(const KArgs &a, int tile, int64_t q, TileHead &h)
{
    const int64_t *ts = a.ws.tile_start;
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
    h.first = a.in.base[s] + j * tile;
    h.nitems = (int32_t)(left < tile ? left : tile);
    h.last = (q == ts[lo + 1] - 1);
}

// Ranks of the tile's valid records within their bucket: afterwards
// slot = L.base[b] + L.cnt[b][k*NW + w] + rank[k] is the record's slot in
// its segment's bucket b.  d == 0xff marks an absent record.
template <int WG, int ITEMS>
__device__ __forceinline__ void tile_ranks(const KArgs &a, TileLds<WG, ITEMS> &L,
                                           const int (&d)[ITEMS], uint32_t (&rank)[ITEMS])
{
    constexpr int NW = WG / 64;
    constexpr int E = TileLds<WG, ITEMS>::E;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint64_t lt = (1ull << lane) - 1ull;

    for (int e = tid; e < 27 * E; e += WG)
        (&L.cnt[0][0])[e] = 0u;
    if (tid == 0)
        L.present = 1u << PM_STAY;
    __syncthreads();

#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const uint64_t stay = __ballot(d[k] == PM_STAY);
        uint64_t mig = __ballot(d[k] < 27 && d[k] != PM_STAY);
        rank[k] = (uint32_t)__popcll(stay & lt);
        if (lane == 0)
            L.cnt[PM_STAY][k * NW + w] = (uint32_t)__popcll(stay);
        uint32_t seen = 0;
        while (mig) {
            const int src = __ffsll((unsigned long long)mig) - 1;
            const int dd = __shfl(d[k], src, 64);
            const uint64_t same = __ballot(d[k] == dd);
            if (d[k] == dd)
                rank[k] = (uint32_t)__popcll(same & lt);
            if (lane == 0)
                L.cnt[dd][k * NW + w] = (uint32_t)__popcll(same);
            seen |= 1u << dd;
            mig &= ~same;
        }
        if (lane == 0 && seen)
            atomicOr(&L.present, seen);
    }
    __syncthreads();

    if (tid < 27) {
        uint32_t run = 0;
        if ((L.present >> tid) & 1u) {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const uint32_t c = L.cnt[tid][e];
                L.cnt[tid][e] = run;
                run += c;
            }
        }
        L.agg[tid] = run;
    }
    __syncthreads();
}

// Decoupled look-back over the tiles of one segment (wave 0 only): every
// status word carries buckets 2w and 2w+1; each word's chain is walked on
// its own until a predecessor with an inclusive prefix, or the segment's
// first tile, is reached.  Writes L.base.
template <int WG, int ITEMS>
__device__ __forceinline__ void lookback(const KArgs &a, TileLds<WG, ITEMS> &L)
{
    const int lane = threadIdx.x;
    if (lane >= 64)
        return;
    const TileHead &h = L.h;
    uint64_t agg = 0;
    if (lane < kLbWords) {
        const uint64_t lo = L.agg[2 * lane];
        const uint64_t hi = (2 * lane + 1 < 27) ? L.agg[2 * lane + 1] : 0ull;
        agg = lo | (hi << 31);
    }
    uint64_t *mine = a.ws.lb + h.q * kLbWords;
    uint64_t excl = 0;
    if (h.q == h.qhead) {
        if (lane < kLbWords)
            lb_store(mine + lane, kLbP | agg);
    } else {
        if (lane < kLbWords)
            lb_store(mine + lane, kLbA | agg);
        bool done = lane >= kLbWords;
        const int pp = lane / kLbWords, ww = lane % kLbWords;
        int64_t pb = h.q - 1;
        for (;;) {
            const int64_t t = pb - pp;
            uint64_t v = kLbP;  // before the segment's first tile: a zero prefix
            if (lane < 4 * kLbWords && t >= h.qhead) {
                const uint64_t *wp = a.ws.lb + t * kLbWords + ww;
                v = lb_load(wp);
                while ((v >> 62) == 0ull) {
                    __builtin_amdgcn_s_sleep(1);
                    v = lb_load(wp);
                }
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint64_t vk = shfl64(v, (k * kLbWords + lane) & 63);
                if (!done) {
                    excl += vk & kLbMask;
                    if ((vk >> 62) == 2ull)
                        done = true;
                }
            }
            if (__ballot(!done) == 0ull)
                break;
            pb -= 4;
        }
        if (lane < kLbWords)
            lb_store(mine + lane, kLbP | (excl + agg));
    }
    if (lane < kLbWords) {
        L.base[2 * lane] = (uint32_t)(excl & kM31);
        if (2 * lane + 1 < 27)
            L.base[2 * lane + 1] = (uint32_t)((excl >> 31) & kM31);
    }
}

// The segment's last tile publishes the segment totals.
template <int WG, int ITEMS>
__device__ __forceinline__ void publish_totals(const KArgs &a, const TileLds<WG, ITEMS> &L)
{
    const int tid = threadIdx.x;
    if (L.h.last && tid < 27) {
        const int64_t tot = (int64_t)L.base[tid] + (int64_t)L.agg[tid];
        if (tid == PM_STAY)
            a.ws.stay[L.h.s] = tot;
        else
            a.send.count[(int64_t)L.h.s * 27 + tid] = tot;
    }
}

template <typename FT>
__device__ __forceinline__ void put_record(const DPool &P, int64_t at, const double X[3],
                                           const FT V[3], FT tau, uint64_t id)
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        P.x[c][at] = X[c];
        ((FT *)P.v[c])[at] = V[c];
    }
    ((FT *)P.tau)[at] = tau;
    P.id[at] = id;
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

// Per-call set-up: the tile table of the segment range (one workgroup),
// clearing of the look-back words and counts, and layout checks.
__global__ __launch_bounds__(1024) void k_prep(const KArgs a, int mode)
{
    uint32_t *hdr = a.ws.hdr;
    const int tid = threadIdx.x;
    const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + tid;
    const int64_t gsize = (int64_t)gridDim.x * blockDim.x;
    uint32_t bad = 0;

    if ((mode & kPrepTiles) && blockIdx.x == 0) {
        // exclusive scan of ceil(count/tile) over the range, 4 per thread
        __shared__ int64_t part[1024];
        int64_t v[4];
        int64_t sum = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int i = tid * 4 + k;
            int64_t c = 0;
            if (i < a.sub_count) {
                c = a.in.count[a.sub_first + i];
                c = c > 0 ? (c + a.tile - 1) / a.tile : 0;
            }
            v[k] = c;
            sum += c;
        }
        part[tid] = sum;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const int64_t x = tid >= off ? part[tid - off] : 0;
            __syncthreads();
            part[tid] += x;
            __syncthreads();
        }
        int64_t run = part[tid] - sum;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int i = tid * 4 + k;
            if (i <= a.sub_count)
                a.ws.tile_start[i] = run;
            run += v[k];
        }
        if (tid == 1023) {
            const int64_t total = part[1023];
            a.ws.tile_start[a.sub_count] = total;
            if (total > a.ws.max_tiles) {
                bad |= PM_F_LAYOUT;
                hdr[kHdrTiles] = 0u;
            } else {
                hdr[kHdrTiles] = (uint32_t)total;
            }
            hdr[kHdrTicket] = 0u;
        }
    }

    if (mode & kPrepZeroLb) {
        int64_t words = ((int64_t)a.ws.pool_extent / a.tile + a.sub_count + 2) * kLbWords;
        const int64_t cap = a.ws.max_tiles * kLbWords;
        if (words > cap)
            words = cap;
        for (int64_t i = gtid; i < words; i += gsize)
            a.ws.lb[i] = 0ull;
    }

    if (mode & kPrepZeroCounts) {
        for (int64_t i = gtid; i < (int64_t)a.sub_count * 27; i += gsize) {
            const int64_t s = a.sub_first + i / 27;
            const int d = (int)(i % 27);
            if (d == PM_STAY)
                a.ws.stay[s] = 0;
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
        // every source segment a destination of the range may read from
        for (int64_t i = gtid; i < (int64_t)a.dc.nsub * 27; i += gsize) {
            const int64_t b = a.send.base[i], c = a.send.cap[i];
            if (b < 0 || c < 0 || c > (int64_t)kM31 || b + c > a.ws.send_extent)
                bad |= PM_F_LAYOUT;
        }
    }
    if (bad)
        flag_or(hdr, bad);
}

// The fused step: interpolate + advance + classify + scan + scatter.
template <int WG, int ITEMS, typename FT, bool HALO>
__global__ __launch_bounds__(WG) void k_step(const KArgs a)
{
    constexpr int NW = WG / 64;
    __shared__ TileLds<WG, ITEMS> L;
    uint32_t *hdr = a.ws.hdr;
    if (flags_now(hdr) & PM_F_LAYOUT)
        return;
    const int64_t total = hdr[kHdrTiles];
    const int tid = threadIdx.x, w = tid >> 6;
    uint32_t fl = 0;

    for (;;) {
        if (tid == 0) {
            const int64_t q = (int64_t)__hip_atomic_fetch_add(
                hdr + kHdrTicket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            L.h.q = q;
            if (q < total)
                locate(a, a.tile, q, L.h);
        }
        __syncthreads();
        if (L.h.q >= total)
            break;
        const int s = L.h.s;
        const int64_t first = L.h.first;
        const int nitems = L.h.nitems;
        int own[3];
        owner_xyz(a.dc, s, own);

        double X[ITEMS][3];
        FT V[ITEMS][3], tau[ITEMS];
        uint64_t id[ITEMS];
        int d[ITEMS];
        uint32_t rank[ITEMS];
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const int i = k * WG + tid;
            if (i < nitems) {
                const int64_t p = first + i;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    X[k][c] = a.in.x[c][p];
                    V[k][c] = ((const FT *)a.in.v[c])[p];
                }
                tau[k] = ((const FT *)a.in.tau)[p];
                id[k] = a.in.id[p];
            }
        }
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            d[k] = 0xff;
            if (k * WG + tid < nitems) {
                advance<FT, HALO>(a, X[k], V[k], tau[k], fl);
                d[k] = classify(a.dc, own, X[k], fl);
            }
        }

        tile_ranks<WG, ITEMS>(a, L, d, rank);
        lookback<WG, ITEMS>(a, L);
        __syncthreads();

        const int64_t obase = a.out.base[s], ocap = a.out.cap[s];
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            if (d[k] == 0xff)
                continue;
            const int b = d[k];
            const int64_t slot = (int64_t)L.base[b] + L.cnt[b][k * NW + w] + rank[k];
            if (b == PM_STAY) {
                if (slot < ocap)
                    put_record<FT>(a.out, obase + slot, X[k], V[k], tau[k], id[k]);
                else
                    fl |= PM_F_DEST_OVERFLOW;
            } else {
                const int64_t qq = (int64_t)s * 27 + b;
                if (slot < a.send.cap[qq]) {
                    double Xs[3];
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        Xs[c] = shifted(a.dc, c, own[c], dir_o(b, c), X[k][c]);
                    put_record<FT>(a.send, a.send.base[qq] + slot, Xs, V[k], tau[k], id[k]);
                } else {
                    fl |= PM_F_SEND_OVERFLOW;
                }
            }
        }
        publish_totals<WG, ITEMS>(a, L);
        __syncthreads();
    }
    if (fl)
        flag_or(hdr, fl);
}

// Plain path, step 1-2: in-place advance of the range's records.
template <int WG, int ITEMS, typename FT, bool HALO>
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
            locate(a, a.tile, q, H);
        __syncthreads();
        const int64_t first = H.first;
        const int nitems = H.nitems;
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const int i = k * WG + tid;
            if (i < nitems) {
                const int64_t p = first + i;
                double X[3];
                FT V[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    X[c] = a.in.x[c][p];
                    V[c] = ((const FT *)a.in.v[c])[p];
                }
                const FT t = ((const FT *)a.in.tau)[p];
                advance<FT, HALO>(a, X, V, t, fl);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    a.in.x[c][p] = X[c];
                    ((FT *)a.in.v[c])[p] = V[c];
                }
            }
        }
        __syncthreads();
    }
    if (fl)
        flag_or(hdr, fl);
}

// Plain path, steps 3-4: mask, scan, pack; stayers' slots to the workspace.
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

    for (;;) {
        if (tid == 0) {
            const int64_t q = (int64_t)__hip_atomic_fetch_add(
                hdr + kHdrTicket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            L.h.q = q;
            if (q < total)
                locate(a, a.tile, q, L.h);
        }
        __syncthreads();
        if (L.h.q >= total)
            break;
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
        tile_ranks<WG, ITEMS>(a, L, d, rank);
        lookback<WG, ITEMS>(a, L);
        __syncthreads();

#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            if (d[k] == 0xff)
                continue;
            const int b = d[k];
            const int64_t p = first + k * WG + tid;
            const int64_t slot = (int64_t)L.base[b] + L.cnt[b][k * NW + w] + rank[k];
            if (b == PM_STAY) {
                a.ws.slot[p] = (uint32_t)slot;
            } else {
                a.ws.slot[p] = kMigrantSlot;
                const int64_t qq = (int64_t)s * 27 + b;
                if (slot < a.send.cap[qq]) {
                    double Xs[3];
                    FT V[3];
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        Xs[c] = shifted(a.dc, c, own[c], dir_o(b, c), X[k][c]);
                        V[c] = ((const FT *)a.in.v[c])[p];
                    }
                    put_record<FT>(a.send, a.send.base[qq] + slot, Xs, V,
                                   ((const FT *)a.in.tau)[p], a.in.id[p]);
                } else {
                    fl |= PM_F_SEND_OVERFLOW;
                }
            }
        }
        publish_totals<WG, ITEMS>(a, L);
        __syncthreads();
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
            locate(a, a.tile, q, H);
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

// Receive: append what every destination t of the range receives after its
// stayers, direction code ascending, each buffer in order (unpacking).
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
                int tt[3];
                owner_xyz(a.dc, t, tt);
                int sc[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const int P = a.dc.p[c];
                    sc[c] = ((tt[c] - dir_o(tid, c)) % P + P) % P;
                }
                const int64_t src = sc[0] + (int64_t)a.dc.p[0] * (sc[1] + (int64_t)a.dc.p[1] * sc[2]);
                const int64_t qq = src * 27 + tid;
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

template <typename FT, bool HALO>
__global__ __launch_bounds__(256) void k_interp(const KArgs a, int64_t n, const double *x,
                                                const double *y, const double *z, FT *ux,
                                                FT *uy, FT *uz)
{
    uint32_t fl = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * 256) {
        const double X[3] = {x[i], y[i], z[i]};
        FT U[3];
        interp<FT, HALO>(a.f, X, U, fl);
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
        locate(a, a.tile, q, h);
        for (int i = threadIdx.x; i < h.nitems; i += 256) {
            const int64_t p = h.first + i;
            double X[2][3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                X[0][c] = a.in.x[c][p];
                X[1][c] = fma(a.dt, (double)((const FT *)a.in.v[c])[p], X[0][c]);
            }
            for (int st = 0; st < 2; ++st) {
                int c0[3];
                for (int ax = 0; ax < 3; ++ax)
                    axis_corner<HALO>(a.f, ax, X[st][ax], c0[ax], fl);
                for (int cz = 0; cz < 2; ++cz)
                    for (int cy = 0; cy < 2; ++cy)
                        for (int cx = 0; cx < 2; ++cx) {
                            const int ix = cx ? next_corner<HALO>(a.f, 0, c0[0]) : c0[0];
                            const int iy = cy ? next_corner<HALO>(a.f, 1, c0[1]) : c0[1];
                            const int iz = cz ? next_corner<HALO>(a.f, 2, c0[2]) : c0[2];
                            const int64_t node = ix + a.f.sx * iy + a.f.sxy * iz;
                            atomicOr((unsigned long long *)&bits[node >> 6],
                                     1ull << (node & 63));
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

// ---------------------------------------------------------------------------
// dispatch over launch shapes and precisions
// ---------------------------------------------------------------------------

#define PM_SHAPES(X) X(256, 1) X(256, 2) X(256, 4) X(256, 8) X(512, 1) X(512, 2) X(512, 4)

}  // namespace

bool shape_supported(Shape sh)
{
#define PM_ONE(W, I) if (sh.wg == W && sh.items == I) return true;
    PM_SHAPES(PM_ONE)
#undef PM_ONE
    return false;
}

hipError_t launch_prep(const KArgs &a, int mode, hipStream_t st)
{
    int grid = 1;
    if (mode & (kPrepZeroLb | kPrepZeroCounts | kPrepCheckSend | kPrepCheckIn | kPrepCheckOut))
        grid = 256;
    hipLaunchKernelGGL(k_prep, dim3(grid), dim3(1024), 0, st, a, mode);
    return hipGetLastError();
}

#define PM_STEP_CASE(W, I)                                                             \
    if (sh.wg == W && sh.items == I) {                                                 \
        if (mixed) {                                                                   \
            if (a.f.halo)                                                              \
                hipLaunchKernelGGL((k_step<W, I, float, true>), dim3(grid), dim3(W), 0, st, a); \
            else                                                                       \
                hipLaunchKernelGGL((k_step<W, I, float, false>), dim3(grid), dim3(W), 0, st, a); \
        } else {                                                                       \
            if (a.f.halo)                                                              \
                hipLaunchKernelGGL((k_step<W, I, double, true>), dim3(grid), dim3(W), 0, st, a); \
            else                                                                       \
                hipLaunchKernelGGL((k_step<W, I, double, false>), dim3(grid), dim3(W), 0, st, a); \
        }                                                                              \
        return hipGetLastError();                                                      \
    }

hipError_t launch_step(const KArgs &a, Shape sh, bool mixed, int grid, hipStream_t st)
{
    PM_SHAPES(PM_STEP_CASE)
    return hipErrorInvalidValue;
}

#define PM_ADV_CASE(W, I)                                                              \
    if (sh.wg == W && sh.items == I) {                                                 \
        if (mixed) {                                                                   \
            if (a.f.halo)                                                              \
                hipLaunchKernelGGL((k_advance<W, I, float, true>), dim3(grid), dim3(W), 0, st, a); \
            else                                                                       \
                hipLaunchKernelGGL((k_advance<W, I, float, false>), dim3(grid), dim3(W), 0, st, a); \
        } else {                                                                       \
            if (a.f.halo)                                                              \
                hipLaunchKernelGGL((k_advance<W, I, double, true>), dim3(grid), dim3(W), 0, st, a); \
            else                                                                       \
                hipLaunchKernelGGL((k_advance<W, I, double, false>), dim3(grid), dim3(W), 0, st, a); \
        }                                                                              \
        return hipGetLastError();                                                      \
    }

hipError_t launch_advance(const KArgs &a, Shape sh, bool mixed, int grid, hipStream_t st)
{
    PM_SHAPES(PM_ADV_CASE)
    return hipErrorInvalidValue;
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

hipError_t launch_interp(const KArgs &a, bool mixed, int64_t n, const double *x,
                         const double *y, const double *z, void *ux, void *uy, void *uz,
                         hipStream_t st)
{
    int64_t g = (n + 255) / 256;
    const int grid = (int)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
    if (mixed) {
        if (a.f.halo)
            hipLaunchKernelGGL((k_interp<float, true>), dim3(grid), dim3(256), 0, st, a, n, x,
                               y, z, (float *)ux, (float *)uy, (float *)uz);
        else
            hipLaunchKernelGGL((k_interp<float, false>), dim3(grid), dim3(256), 0, st, a, n, x,
                               y, z, (float *)ux, (float *)uy, (float *)uz);
    } else {
        if (a.f.halo)
            hipLaunchKernelGGL((k_interp<double, true>), dim3(grid), dim3(256), 0, st, a, n,
                               x, y, z, (double *)ux, (double *)uy, (double *)uz);
        else
            hipLaunchKernelGGL((k_interp<double, false>), dim3(grid), dim3(256), 0, st, a, n,
                               x, y, z, (double *)ux, (double *)uy, (double *)uz);
    }
    return hipGetLastError();
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

#define PM_OCC_CASE(W, I)                                                              \
    if (sh.wg == W && sh.items == I) {                                                 \
        if (mixed)                                                                     \
            (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (k_step<W, I, float, false>), W, 0); \
        else                                                                           \
            (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (k_step<W, I, double, false>), W, 0); \
    }

int step_occupancy(Shape sh, bool mixed)
{
    int nb = 1;
    PM_SHAPES(PM_OCC_CASE)
    return nb < 1 ? 1 : nb;
}

}  // namespace pm
