// pm_sort.hip -- cell re-sort of the particle segments (gfx950).
//
// Not a step of the particle method: particles disperse from any order as
// they move, and the fused step's stencil gathers share cache lines only when
// neighbouring records are neighbours in space.  A caller re-sorts every few
// tens of steps.  Order within each segment: by the cell key (Z-order over
// pairs of cells along x, then the parity of the cell's x index), ties by
// input position -- a stable least-significant-digit radix sort of
// (key, position) pairs, 8 bits per pass, over tiles that never straddle a
// segment, followed by one gather of the records.  Every scatter and gather
// index is checked against its segment's range; a violation sets PM_F_LAYOUT
// instead of writing.
#include "pm_device.h"

namespace pm {
namespace {

constexpr int kSortWG = 256;
constexpr int kSortItems = 32;
constexpr int kSortTile = kSortWG * kSortItems;
constexpr int kScanBatch = 32;  // tiles whose counts a scan thread loads at once

// The 21 low bits of v moved to bits 0, 3, 6, ..., 60 (the magic-mask bit
// spreading of Morton encoding: five shift-or-mask steps).
__device__ __forceinline__ uint64_t spread3(uint32_t v)
{
    uint64_t x = v & 0x1fffffu;
    x = (x | x << 32) & 0x1f00000000ffffull;
    x = (x | x << 16) & 0x1f0000ff0000ffull;
    x = (x | x << 8) & 0x100f00f00f00f00full;
    x = (x | x << 4) & 0x10c30c30c30c30c3ull;
    x = (x | x << 2) & 0x1249249249249249ull;
    return x;
}

// Z-order code of (i >> 1, j, k) (bit b of each at 3b, 3b+1, 3b+2), times
// two, plus the parity of i.
__device__ __forceinline__ uint64_t cell_key(int i, int j, int k)
{
    const uint64_t code = spread3((uint32_t)i >> 1) | spread3((uint32_t)j) << 1 |
                          spread3((uint32_t)k) << 2;
    return code * 2 + ((uint32_t)i & 1u);
}

// Cell index of x along an axis of n cells (r = n / L): floor(x r) clamped to
// [0, n-1]; a NaN lands in cell 0.
__device__ __forceinline__ int cell_of(double x, double r, int n)
{
    const double s = x * r;
    if (!(s >= 0.0))
        return 0;
    if (!(s < (double)n))
        return n - 1;
    return (int)floor(s);
}

// The range's tile count, or -1 (PM_F_LAYOUT raised) when the layout is
// inconsistent or there are more tiles than the sort's tables hold.
__device__ __forceinline__ int64_t sort_tiles(const KArgs &a, const DSort &s)
{
    uint32_t *hdr = a.ws.hdr;
    if (flags_now(hdr) & PM_F_LAYOUT)
        return -1;
    const int64_t total = hdr[kHdrTiles];
    if (total > s.tiles) {
        if (blockIdx.x == 0 && threadIdx.x == 0)
            flag_or(hdr, PM_F_LAYOUT);
        return -1;
    }
    return total;
}

// Keys and positions of every record of the range, at the record's own pool
// position.
__global__ __launch_bounds__(kSortWG) void k_sort_keys(const KArgs a, DSort s)
{
    const int64_t total = sort_tiles(a, s);
    if (total < 0)
        return;
    for (int64_t q = blockIdx.x; q < total; q += gridDim.x) {
        TileHead h;
        locate(a, kSortTile, q, h, a.ws.tile_start);
        for (int i = threadIdx.x; i < h.nitems; i += kSortWG) {
            const int64_t p = h.first + i;
            const int ci = cell_of(a.in.x[0][p], a.f.r[0], a.f.n[0]);
            const int cj = cell_of(a.in.x[1][p], a.f.r[1], a.f.n[1]);
            const int ck = cell_of(a.in.x[2][p], a.f.r[2], a.f.n[2]);
            s.keys[0][p] = cell_key(ci, cj, ck);
            s.vals[0][p] = (uint32_t)p;
        }
    }
}

// Per tile: the counts of the pass's digit.
__global__ __launch_bounds__(kSortWG) void k_sort_hist(const KArgs a, DSort s, int src,
                                                        int shift)
{
    __shared__ uint32_t cnt[256];
    const int64_t total = sort_tiles(a, s);
    if (total < 0)
        return;
    const int tid = threadIdx.x;
    for (int64_t q = blockIdx.x; q < total; q += gridDim.x) {
        TileHead h;
        locate(a, kSortTile, q, h, a.ws.tile_start);
        cnt[tid] = 0;
        __syncthreads();
        for (int i = tid; i < h.nitems; i += kSortWG) {
            const uint32_t d = (uint32_t)(s.keys[src][h.first + i] >> shift) & 255u;
            atomicAdd(&cnt[d], 1u);
        }
        __syncthreads();
        s.hist[q * 256 + tid] = cnt[tid];
        __syncthreads();
    }
}

// Per segment (one workgroup of 1024 threads: digit d = tid mod 256, part =
// tid / 256 takes a quarter of the segment's tiles): the pool position where
// each tile's records of digit d go -- the segment's base, plus the records
// of smaller digits in the segment, plus those of digit d in earlier tiles.
constexpr int kScanParts = 4;

__global__ __launch_bounds__(256 * kScanParts) void k_sort_scan(const KArgs a, DSort s)
{
    __shared__ int64_t part_sum[kScanParts][256];
    __shared__ int64_t wave_tot[4];
    if (sort_tiles(a, s) < 0)
        return;
    const int tid = threadIdx.x, d = tid & 255, part = tid >> 8;
    for (int sl = blockIdx.x; sl < a.sub_count; sl += gridDim.x) {
        const int64_t t0 = a.ws.tile_start[sl], t1 = a.ws.tile_start[sl + 1];
        const int64_t len = (t1 - t0 + kScanParts - 1) / kScanParts;
        const int64_t p0 = t0 + part * len, p1 = p0 + len < t1 ? p0 + len : t1;
        // this part's count of digit d
        int64_t tot = 0;
        int64_t t = p0;
        for (; t + kScanBatch <= p1; t += kScanBatch) {
            uint32_t c[kScanBatch];
#pragma unroll
            for (int u = 0; u < kScanBatch; ++u)
                c[u] = s.hist[(t + u) * 256 + d];
#pragma unroll
            for (int u = 0; u < kScanBatch; ++u)
                tot += c[u];
        }
        for (; t < p1; ++t)
            tot += s.hist[t * 256 + d];
        part_sum[part][d] = tot;
        __syncthreads();
        // digit totals, scanned over the digits by the first 256 threads
        int64_t digit_tot = 0;
#pragma unroll
        for (int q = 0; q < kScanParts; ++q)
            digit_tot += part_sum[q][d];
        int64_t incl = digit_tot;
        const int lane = tid & 63, w = tid >> 6;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int lo = __shfl_up((int)(uint32_t)incl, off, 64);
            const int hi = __shfl_up((int)(uint32_t)((uint64_t)incl >> 32), off, 64);
            const int64_t v = (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
            if (lane >= off)
                incl += v;
        }
        if (tid < 256 && lane == 63)
            wave_tot[w] = incl;
        __syncthreads();
        // every part of digit d starts after the smaller digits, then after
        // the earlier parts of digit d
        int64_t run = a.in.base[a.sub_first + sl] + incl - digit_tot;
        for (int v = 0; v < (d >> 6); ++v)
            run += wave_tot[v];
        for (int q = 0; q < part; ++q)
            run += part_sum[q][d];
        t = p0;
        for (; t + kScanBatch <= p1; t += kScanBatch) {
            uint32_t c[kScanBatch];
#pragma unroll
            for (int u = 0; u < kScanBatch; ++u)
                c[u] = s.hist[(t + u) * 256 + d];
#pragma unroll
            for (int u = 0; u < kScanBatch; ++u) {
                s.off[(t + u) * 256 + d] = run;
                run += c[u];
            }
        }
        for (; t < p1; ++t) {
            const uint32_t c = s.hist[t * 256 + d];
            s.off[t * 256 + d] = run;
            run += c;
        }
        __syncthreads();  // part_sum and wave_tot are reused by the next segment
    }
}

// Per tile: every record to its place for this digit, in tile order among
// the records of equal digit (so each pass is stable).  Rounds of 256
// consecutive records: a record's rank is the number of records of its digit
// before it in its wave (ballots over the 8 digit bits), in the earlier waves
// of the round, and in the earlier rounds.
__global__ __launch_bounds__(kSortWG) void k_sort_scatter(const KArgs a, DSort s, int src,
                                                           int shift)
{
    __shared__ int64_t run[256];
    __shared__ uint32_t wc[4][256];
    const int64_t total = sort_tiles(a, s);
    if (total < 0)
        return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int dst = src ^ 1;
    uint32_t fl = 0;
    for (int64_t q = blockIdx.x; q < total; q += gridDim.x) {
        TileHead h;
        locate(a, kSortTile, q, h, a.ws.tile_start);
        const int64_t lo = a.in.base[h.s], hi = lo + a.in.count[h.s];
        run[tid] = s.off[q * 256 + tid];
#pragma unroll
        for (int v = 0; v < 4; ++v)
            wc[v][tid] = 0;
        __syncthreads();
        for (int r = 0; r < kSortItems; ++r) {
            const int i = r * kSortWG + tid;
            const bool valid = i < h.nitems;
            uint64_t key = 0;
            uint32_t val = 0, d = 0;
            if (valid) {
                key = s.keys[src][h.first + i];
                val = s.vals[src][h.first + i];
                d = (uint32_t)(key >> shift) & 255u;
            }
            uint64_t m = __ballot(valid);
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const bool bit = (d >> b) & 1u;
                const uint64_t bb = __ballot(valid && bit);
                m &= bit ? bb : ~bb;
            }
            const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
            const uint32_t rank = (uint32_t)__popcll(m & below);
            if (valid && lane == 63 - __clzll(m))
                wc[w][d] = (uint32_t)__popcll(m);
            __syncthreads();
            if (valid) {
                int64_t o = run[d] + rank;
                for (int v = 0; v < w; ++v)
                    o += wc[v][d];
                if (o >= lo && o < hi) {
                    s.keys[dst][o] = key;
                    s.vals[dst][o] = val;
                } else {
                    fl |= PM_F_LAYOUT;
                }
            }
            __syncthreads();
            run[tid] += wc[0][tid] + wc[1][tid] + wc[2][tid] + wc[3][tid];
#pragma unroll
            for (int v = 0; v < 4; ++v)
                wc[v][tid] = 0;
            __syncthreads();
        }
    }
    if (fl)
        flag_or(a.ws.hdr, fl);
}

// The records in sorted order: out[out.base[s] + r] = in[vals[in.base[s] + r]].
template <typename FT>
__global__ __launch_bounds__(kSortWG) void k_sort_gather(const KArgs a, DSort s, int src)
{
    const int64_t total = sort_tiles(a, s);
    if (total < 0)
        return;
    uint32_t fl = 0;
    for (int64_t q = blockIdx.x; q < total; q += gridDim.x) {
        TileHead h;
        locate(a, kSortTile, q, h, a.ws.tile_start);
        const int64_t lo = a.in.base[h.s], hi = lo + a.in.count[h.s];
        const int64_t obase = a.out.base[h.s], ocap = a.out.cap[h.s];
        for (int i = threadIdx.x; i < h.nitems; i += kSortWG) {
            const int64_t p = h.first + i;
            const int64_t from = (int64_t)s.vals[src][p];
            const int64_t r = p - lo;
            if (from < lo || from >= hi) {
                fl |= PM_F_LAYOUT;
                continue;
            }
            if (r >= ocap) {
                fl |= PM_F_DEST_OVERFLOW;
                continue;
            }
            const int64_t to = obase + r;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                a.out.x[c][to] = a.in.x[c][from];
                ((FT *)a.out.v[c])[to] = ((const FT *)a.in.v[c])[from];
            }
            ((FT *)a.out.tau)[to] = ((const FT *)a.in.tau)[from];
            a.out.id[to] = a.in.id[from];
        }
    }
    for (int64_t sl = (int64_t)blockIdx.x * kSortWG + threadIdx.x; sl < a.sub_count;
         sl += (int64_t)gridDim.x * kSortWG) {
        const int sg = a.sub_first + (int)sl;
        a.out.count[sg] = a.in.count[sg];
        if (a.in.count[sg] > a.out.cap[sg])
            fl |= PM_F_DEST_OVERFLOW;
    }
    if (fl)
        flag_or(a.ws.hdr, fl);
}

}  // namespace

int sort_tile() { return kSortTile; }

hipError_t launch_sort(const KArgs &a, DSort s, int passes, bool mixed, int grid,
                       hipStream_t st)
{
    hipLaunchKernelGGL(k_sort_keys, dim3(grid), dim3(kSortWG), 0, st, a, s);
    int src = 0;
    for (int p = 0; p < passes; ++p) {
        hipLaunchKernelGGL(k_sort_hist, dim3(grid), dim3(kSortWG), 0, st, a, s, src, 8 * p);
        hipLaunchKernelGGL(k_sort_scan, dim3(std::max(1, std::min(a.sub_count, 4096))),
                           dim3(256 * kScanParts), 0, st, a, s);
        hipLaunchKernelGGL(k_sort_scatter, dim3(grid), dim3(kSortWG), 0, st, a, s, src,
                           8 * p);
        src ^= 1;
    }
    if (mixed)
        hipLaunchKernelGGL(k_sort_gather<float>, dim3(grid), dim3(kSortWG), 0, st, a, s, src);
    else
        hipLaunchKernelGGL(k_sort_gather<double>, dim3(grid), dim3(kSortWG), 0, st, a, s, src);
    return hipGetLastError();
}

}  // namespace pm
