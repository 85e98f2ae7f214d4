// partition.hip -- the probe over points in no spatial order, with the points
// first partitioned by the coarse region of their cell.
//
// On the Hilbert layout (and the grid with too many polygons for LDS bins) a
// point's lookup is a search in arrays of tens of millions of runs, and
// points in no order miss L2 on nearly every step.  One partition pass puts
// the points (and their values) into 256 buckets, the 16 x 16 level-4 Hilbert
// tiles of the handle's cell box; the item probe then meets the points bucket
// by bucket (each XCD a contiguous stretch of buckets), and each bucket's runs
// (1/256 of them) stay in cache.  The pass is
// one radix-partition round: per workgroup chunk a 256-bin histogram, the
// bucket offsets of every chunk, then each chunk writes its points at its
// offsets.  The order of points inside a bucket is irrelevant to the sums.
// Everything lives in a caller-provided scratch buffer.
#include "sba_internal.h"

#define PART_BLOCK 256
#define PART_CHUNK (1 << 16)  // points per workgroup

struct PartGeo {
    int64_t ox, oy;        // coordinate of the cell box's first cell
    uint32_t extx, exty;   // box extent in coordinate units (< 2^31)
    uint32_t mag;
    int32_t shift;
    int32_t sh;            // cell index >> sh = level-4 tile
};

__device__ __forceinline__ uint32_t part_digit(const PartGeo &g, int32_t x, int32_t y)
{
    const int64_t dx = (int64_t)x - g.ox, dy = (int64_t)y - g.oy;
    if ((uint64_t)dx >= g.extx || (uint64_t)dy >= g.exty) return 0;  // no cell: any bucket
    const uint32_t i = divmagic((uint32_t)dx, g.mag, g.shift) >> g.sh;
    const uint32_t j = divmagic((uint32_t)dy, g.mag, g.shift) >> g.sh;
    return (uint32_t)hilbert_index(4, i, j);
}

__global__ void k_part_zero(unsigned long long *dtot)
{
    dtot[threadIdx.x] = 0;
}

__global__ __launch_bounds__(PART_BLOCK) void k_part_hist(const int32_t *__restrict__ xy, int64_t n,
                                                          PartGeo g, int64_t *hist,
                                                          int64_t nblocks,
                                                          unsigned long long *dtot)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t a = (int64_t)blockIdx.x * PART_CHUNK, b = min(a + (int64_t)PART_CHUNK, n);
    for (int64_t t = a + threadIdx.x; t < b; t += PART_BLOCK) {
        const int2 p = ((const int2 *)xy)[t];
        atomicAdd(&h[part_digit(g, p.x, p.y)], 1u);
    }
    __syncthreads();
    const uint32_t c = h[threadIdx.x];
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = c;
    if (c) atomicAdd(&dtot[threadIdx.x], (unsigned long long)c);
}

// Each chunk goes out in tiles of PART_TILE points: the tile is ordered by
// bucket in LDS (a rank per point from an LDS counter, the tile's bucket
// offsets by a scan), then written linearly, so the points of one bucket
// leave as one contiguous run instead of scattered 8-byte stores.
#define PART_PER 16
#define PART_TILE (PART_BLOCK * PART_PER)

template <bool VALS>
__global__ __launch_bounds__(PART_BLOCK) void k_part_scatter(
    const int32_t *__restrict__ xy, const int64_t *__restrict__ vals, int64_t n, PartGeo g,
    const int64_t *__restrict__ off, int64_t nblocks, int2 *__restrict__ oxy,
    int64_t *__restrict__ ovals)
{
    __shared__ int64_t cur[256];       // next output position of each bucket
    __shared__ uint32_t cnt[256];      // the tile's points per bucket, then their offsets
    __shared__ int64_t base[256];      // output position of the tile's first point of a bucket
                                       // minus that point's position in the staged tile
    __shared__ int2 sxy[PART_TILE];
    __shared__ int64_t sv[VALS ? PART_TILE : 1];
    __shared__ uint32_t wsum[PART_BLOCK / 64];
    const int tid = threadIdx.x;
    cur[tid] = off[(int64_t)tid * nblocks + blockIdx.x];
    const int64_t a = (int64_t)blockIdx.x * PART_CHUNK, b = min(a + (int64_t)PART_CHUNK, n);
    for (int64_t t0 = a; t0 < b; t0 += PART_TILE) {
        cnt[tid] = 0;
        __syncthreads();
        int2 p[PART_PER];
        int64_t v[PART_PER];
        uint32_t d[PART_PER], r[PART_PER];
#pragma unroll
        for (int k = 0; k < PART_PER; k++) {
            const int64_t t = t0 + k * PART_BLOCK + tid;
            const bool in = t < b;
            p[k] = in ? ((const int2 *)xy)[t] : make_int2(0, 0);
            v[k] = (VALS && in) ? vals[t] : 0;
            d[k] = in ? part_digit(g, p[k].x, p[k].y) : 256u;
            r[k] = in ? atomicAdd(&cnt[d[k]], 1u) : 0u;
        }
        __syncthreads();
        // exclusive scan of the 256 bucket counts (one per thread)
        const uint32_t c = cnt[tid];
        uint32_t inc = c;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t u = __shfl_up(inc, o, 64);
            if ((tid & 63) >= o) inc += u;
        }
        if ((tid & 63) == 63) wsum[tid >> 6] = inc;
        __syncthreads();
        uint32_t excl = inc - c;
        for (int w = 0; w < (tid >> 6); w++) excl += wsum[w];
        base[tid] = cur[tid] - (int64_t)excl;
        cur[tid] += c;
        cnt[tid] = excl;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < PART_PER; k++) {
            if (d[k] >= 256u) continue;
            const uint32_t s = cnt[d[k]] + r[k];
            sxy[s] = p[k];
            if (VALS) sv[s] = v[k];
        }
        __syncthreads();
        const int m = (int)min((int64_t)PART_TILE, b - t0);
        for (int s = tid; s < m; s += PART_BLOCK) {
            const int2 q = sxy[s];
            const int64_t pos = base[part_digit(g, q.x, q.y)] + s;
            oxy[pos] = q;
            if (VALS) ovals[pos] = sv[s];
        }
        __syncthreads();
    }
}

// The runs that hold each bucket's keys when the buckets are the top 8 bits
// of a Hilbert handle's 2L-bit keys (bucket b: keys b << bshift ..): bq[b] =
// the run holding key b << bshift, bq[256] = the last run.
__global__ void k_part_bq(const uint32_t *k32, int64_t nr, int bshift, int64_t *bq)
{
    const int b = threadIdx.x;
    if (b > 256) return;
    if (b == 256) {
        bq[256] = nr - 1;
        return;
    }
    const uint32_t key = (uint32_t)((uint64_t)b << bshift);
    int64_t lo = 0, len = nr;
    while (len > 1) {
        const int64_t half = len >> 1;
        lo = k32[lo + half] <= key ? lo + half : lo;
        len -= half;
    }
    bq[b] = lo;
}

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

extern "C" size_t sba_partition_scratch_bytes(int64_t n, int with_values)
{
    if (n <= 0) return 256;
    const int64_t nblocks = (n + PART_CHUNK - 1) / PART_CHUNK;
    return align256((size_t)n * 8) + (with_values ? align256((size_t)n * 8) : 0) +
           align256((size_t)nblocks * 256 * 8) + align256(256 * 8) + align256(257 * 8);
}

extern "C" int sba_aggregate_partitioned(const int32_t *xy, const int64_t *values, int64_t n,
                                         const sba_handle *h, int32_t search, void *scratch,
                                         size_t scratch_bytes, uint64_t *counts, int64_t *sums,
                                         void *stream)
{
    if (!h || n < 0 || (n > 0 && !xy) || (h->n_polys > 0 && !counts)) return SBA_EINVAL;
    if (((uintptr_t)xy & 15) != 0 || ((uintptr_t)values & 15) != 0) return SBA_EINVAL;
    if (search != SBA_SEARCH_BINARY && search != SBA_SEARCH_LEARNED) return SBA_EINVAL;
    const bool vals = values != nullptr && sums != nullptr;
    hipStream_t st = (hipStream_t)stream;
    // nothing to gain: tiny inputs, and grids whose directory the probe keeps
    // in LDS (their lookups do not depend on the order of the points)
    if (h->n_polys == 0 || n == 0 || h->gw == 0 || n < 2 * PART_CHUNK ||
        (h->kind == SBA_KIND_GRID && h->compact))
        return probe_launch(xy, values, n, h, search, counts, sums, st);
    if (!scratch || ((uintptr_t)scratch & 255) != 0) return SBA_EINVAL;
    if (scratch_bytes < sba_partition_scratch_bytes(n, vals ? 1 : 0)) return SBA_ELIMIT;
    const int64_t nblocks = (n + PART_CHUNK - 1) / PART_CHUNK;
    char *p = (char *)scratch;
    int2 *oxy = (int2 *)p;
    p += align256((size_t)n * 8);
    int64_t *ovals = nullptr;
    if (vals) {
        ovals = (int64_t *)p;
        p += align256((size_t)n * 8);
    }
    int64_t *hist = (int64_t *)p;
    p += align256((size_t)nblocks * 256 * 8);
    unsigned long long *dtot = (unsigned long long *)p;
    p += align256(256 * 8);
    int64_t *bq = (int64_t *)p;

    PartGeo g{};
    g.ox = h->gi0 * h->s;
    g.oy = h->gj0 * h->s;
    g.extx = (uint32_t)(h->gw * h->s);
    g.exty = (uint32_t)(h->gh * h->s);
    g.mag = h->mag;
    g.shift = h->shift;
    int lb = 0;
    while (((int64_t)1 << lb) < std::max(h->gw, h->gh)) lb++;
    g.sh = lb > 4 ? lb - 4 : 0;

    hipLaunchKernelGGL(k_part_zero, dim3(1), dim3(256), 0, st, dtot);
    hipLaunchKernelGGL(k_part_hist, dim3((unsigned)nblocks), dim3(PART_BLOCK), 0, st, xy, n, g,
                       hist, nblocks, dtot);
    HIP_OK(hipGetLastError());
    RC(rs_offsets_launch(hist, nblocks, dtot, st));
    if (vals)
        hipLaunchKernelGGL(k_part_scatter<true>, dim3((unsigned)nblocks), dim3(PART_BLOCK), 0, st,
                           xy, values, n, g, hist, nblocks, oxy, ovals);
    else
        hipLaunchKernelGGL(k_part_scatter<false>, dim3((unsigned)nblocks), dim3(PART_BLOCK), 0, st,
                           xy, values, n, g, hist, nblocks, oxy, ovals);
    HIP_OK(hipGetLastError());
    // the binary search of a Hilbert handle whose buckets are the top 8 bits
    // of its keys searches each item's region (its buckets' runs) only
    PartRegions reg{}, *regp = nullptr;
    if (h->kind == SBA_KIND_HILBERT && search == SBA_SEARCH_BINARY && h->starts32 &&
        h->level >= 4 && lb == h->level && h->n_runs > 0) {
        reg = PartRegions{bq, hist, nblocks, 2 * h->level - 8};
        hipLaunchKernelGGL(k_part_bq, dim3(1), dim3(320), 0, st, h->starts32, h->n_runs,
                           reg.bshift, bq);
        HIP_OK(hipGetLastError());
        regp = &reg;
    }
    return items_launch((const int32_t *)oxy, ovals, n, h, search, regp, counts,
                        vals ? sums : nullptr, st);
}
