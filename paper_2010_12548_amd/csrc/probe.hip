// probe.hip -- the hot path: per-polygon COUNT and SUM of points, answered
// from the approximation alone (Sec. 5.1: index-nested-loop join of points
// against the cell index, aggregation fused, no point-in-polygon test).
//
// Each thread streams two points per iteration (one 128-bit load of x,y
// pairs, one 128-bit load of two int64 values), maps each point to its cell
// with a multiply-shift division by the cell side, looks up the cell's code
// and adds the point to a per-workgroup histogram in LDS.  At the end every
// workgroup writes its histogram once; a second small kernel sums the
// workgroup histograms into the caller's outputs (no global atomics on the
// hot path).  Polygon counts too large for LDS fall back to global atomics.
//
// Cell lookup per layout:
//   grid     directory entry of the cell's tile (a few hundred KB, stays in
//            L2), and for mixed tiles one more load from the tile's block;
//   hilbert  Hilbert key of the cell, then the run holding it: binary search
//            over the run starts, or the learned index's bounded search.
#include "sba_internal.h"

#define PROBE_BLOCK 256
#define LDS_MAX_POLYS 4096

struct GridView {
    int64_t ox, oy;        // coordinate of the stored box's first cell
    uint32_t extx, exty;   // box extent in coordinate units (< 2^31)
    uint32_t mag;
    int32_t shift;
    int32_t tl;
    uint32_t tw;
    uint32_t nblocks;
    const uint32_t *dir;
    const uint32_t *blocks;
};

struct HilbView {
    int64_t ox, oy;        // coordinate of the key grid's first cell (the stored box)
    uint32_t extx, exty;   // stored box extent in coordinate units (< 2^31)
    uint32_t mag;
    int32_t shift;
    int32_t L;
    int64_t n;             // runs
    const uint32_t *k32;   // run starts (L <= 16)
    const uint64_t *k64;   // run starts
    const uint32_t *code;  // run codes
    float a;               // learned root
    uint32_t nl;
    const int4 *leaves;
};

__device__ __forceinline__ uint32_t grid_code(const GridView &g, int32_t x, int32_t y)
{
    int64_t dx = (int64_t)x - g.ox, dy = (int64_t)y - g.oy;
    if ((uint64_t)dx >= g.extx || (uint64_t)dy >= g.exty) return 0;
    uint32_t i = divmagic((uint32_t)dx, g.mag, g.shift);
    uint32_t j = divmagic((uint32_t)dy, g.mag, g.shift);
    uint32_t e = g.dir[(uint64_t)(j >> g.tl) * g.tw + (i >> g.tl)];
    if (e & TILE_MIXED) {
        uint32_t b = e & ~TILE_MIXED;
        if (b >= g.nblocks) return 0;  // never taken for a well-formed handle
        uint32_t m = (1u << g.tl) - 1u;
        e = g.blocks[((uint64_t)b << (2 * g.tl)) + ((j & m) << g.tl) + (i & m)];
    }
    return e;
}

// last q with keys[q] <= key; keys[0] == 0 <= key
template <typename K>
__device__ __forceinline__ int64_t pred_search(const K *keys, int64_t lo, int64_t len, K key)
{
    while (len > 1) {
        int64_t half = len >> 1;
        lo = (keys[lo + half] <= key) ? lo + half : lo;
        len -= half;
    }
    return lo;
}

template <typename K>
__device__ __forceinline__ int64_t learned_search(const HilbView &v, const K *keys, K key)
{
    uint32_t l = root_leaf((uint64_t)key, v.a, v.nl);
    int4 lf = v.leaves[l];
    int64_t p = predict((uint64_t)(uint32_t)lf.x, __int_as_float(lf.y), __int_as_float(lf.z),
                        (uint64_t)key);
    int64_t lo = p - lf.w, hi = p + lf.w;
    lo = lo < 0 ? 0 : lo;
    hi = hi > v.n - 1 ? v.n - 1 : hi;
    if (lo <= hi && keys[lo] <= key) {
        int64_t q = pred_search<K>(keys, lo, hi - lo + 1, key);
        if (q == v.n - 1 || keys[q + 1] > key) return q;
    }
    return pred_search<K>(keys, 0, v.n, key);  // bracket missed: full search
}

template <int SEARCH>
__device__ __forceinline__ uint32_t hilbert_code(const HilbView &v, int32_t x, int32_t y)
{
    int64_t dx = (int64_t)x - v.ox, dy = (int64_t)y - v.oy;
    if ((uint64_t)dx >= v.extx || (uint64_t)dy >= v.exty) return 0;
    uint32_t i = divmagic((uint32_t)dx, v.mag, v.shift);
    uint32_t j = divmagic((uint32_t)dy, v.mag, v.shift);
    uint64_t key = hilbert_index(v.L, i, j);
    int64_t q;
    if (v.k32) {
        q = SEARCH ? learned_search<uint32_t>(v, v.k32, (uint32_t)key)
                   : pred_search<uint32_t>(v.k32, 0, v.n, (uint32_t)key);
    } else {
        q = pred_search<uint64_t>(v.k64, 0, v.n, key);
    }
    return v.code[q];
}

struct Agg {
    const int64_t *set_off;
    const int32_t *set_ids;
    uint32_t np;       // polygon ids are checked against it before any update
    uint32_t n_sets;
};

template <bool VALS>
__device__ __forceinline__ void add_lds(uint32_t code, int64_t val, const Agg &A, uint32_t *lcnt,
                                        unsigned long long *lsum)
{
    if (code == 0) return;
    if (code < CODE_SET_BASE) {
        uint32_t p = code - 1u;
        if (p >= A.np) return;
        atomicAdd(&lcnt[p], 1u);
        if (VALS) atomicAdd(&lsum[p], (unsigned long long)val);
    } else {
        uint32_t k = code - CODE_SET_BASE;
        if (k >= A.n_sets) return;
        for (int64_t t = A.set_off[k], e = A.set_off[k + 1]; t < e; t++) {
            uint32_t p = (uint32_t)A.set_ids[t];
            if (p >= A.np) continue;
            atomicAdd(&lcnt[p], 1u);
            if (VALS) atomicAdd(&lsum[p], (unsigned long long)val);
        }
    }
}

template <bool VALS>
__device__ __forceinline__ void add_global(uint32_t code, int64_t val, const Agg &A,
                                           unsigned long long *cnt, unsigned long long *sum)
{
    if (code == 0) return;
    if (code < CODE_SET_BASE) {
        uint32_t p = code - 1u;
        if (p >= A.np) return;
        atomicAdd(&cnt[p], 1ull);
        if (VALS) atomicAdd(&sum[p], (unsigned long long)val);
    } else {
        uint32_t k = code - CODE_SET_BASE;
        if (k >= A.n_sets) return;
        for (int64_t t = A.set_off[k], e = A.set_off[k + 1]; t < e; t++) {
            uint32_t p = (uint32_t)A.set_ids[t];
            if (p >= A.np) continue;
            atomicAdd(&cnt[p], 1ull);
            if (VALS) atomicAdd(&sum[p], (unsigned long long)val);
        }
    }
}

// LAYOUT: 0 grid, 1 hilbert + binary search, 2 hilbert + learned index
template <int LAYOUT>
__device__ __forceinline__ uint32_t code_of(const GridView &g, const HilbView &hv, int32_t x,
                                            int32_t y)
{
    if (LAYOUT == 0) return grid_code(g, x, y);
    return hilbert_code<LAYOUT == 2 ? 1 : 0>(hv, x, y);
}

// LDS-privatised histograms; partial[b] = {count u32 [np], sum u64 [np]}
template <int LAYOUT, bool VALS>
__global__ __launch_bounds__(PROBE_BLOCK) void k_probe_lds(const int4 *__restrict__ xy4,
                                                           const longlong2 *__restrict__ v2,
                                                           const int32_t *__restrict__ xy,
                                                           const int64_t *__restrict__ vals,
                                                           int64_t n, GridView g, HilbView hv,
                                                           Agg A, int32_t np,
                                                           uint32_t *__restrict__ pcnt,
                                                           unsigned long long *__restrict__ psum)
{
    extern __shared__ unsigned long long smem[];
    unsigned long long *lsum = smem;
    uint32_t *lcnt = (uint32_t *)(smem + np);
    for (int p = threadIdx.x; p < np; p += PROBE_BLOCK) {
        lcnt[p] = 0;
        lsum[p] = 0;
    }
    __syncthreads();
    const int64_t npairs = n >> 1;
    const int64_t stride = (int64_t)gridDim.x * PROBE_BLOCK;
    for (int64_t t = (int64_t)blockIdx.x * PROBE_BLOCK + threadIdx.x; t < npairs; t += stride) {
        int4 q = xy4[t];
        longlong2 vv = VALS ? v2[t] : make_longlong2(0, 0);
        uint32_t c0 = code_of<LAYOUT>(g, hv, q.x, q.y);
        uint32_t c1 = code_of<LAYOUT>(g, hv, q.z, q.w);
        add_lds<VALS>(c0, vv.x, A, lcnt, lsum);
        add_lds<VALS>(c1, vv.y, A, lcnt, lsum);
    }
    if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
        int64_t k = n - 1;
        uint32_t c = code_of<LAYOUT>(g, hv, xy[2 * k], xy[2 * k + 1]);
        add_lds<VALS>(c, VALS ? vals[k] : 0, A, lcnt, lsum);
    }
    __syncthreads();
    uint32_t *oc = pcnt + (int64_t)blockIdx.x * np;
    unsigned long long *os = psum + (int64_t)blockIdx.x * np;
    for (int p = threadIdx.x; p < np; p += PROBE_BLOCK) {
        oc[p] = lcnt[p];
        if (VALS) os[p] = lsum[p];
    }
}

// one block per polygon: sum the workgroup histograms, overwrite the outputs
template <bool VALS>
__global__ __launch_bounds__(256) void k_reduce(const uint32_t *pcnt, const unsigned long long *psum,
                                                int64_t nblocks, int32_t np, uint64_t *counts,
                                                int64_t *sums)
{
    const int p = blockIdx.x;
    unsigned long long c = 0, s = 0;
    for (int64_t b = threadIdx.x; b < nblocks; b += 256) {
        c += pcnt[b * np + p];
        if (VALS) s += psum[b * np + p];
    }
    for (int o = 32; o > 0; o >>= 1) {
        c += __shfl_xor(c, o, 64);
        s += __shfl_xor(s, o, 64);
    }
    __shared__ unsigned long long wc[4], ws[4];
    if ((threadIdx.x & 63) == 0) {
        wc[threadIdx.x >> 6] = c;
        ws[threadIdx.x >> 6] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        counts[p] = wc[0] + wc[1] + wc[2] + wc[3];
        if (VALS) sums[p] = (int64_t)(ws[0] + ws[1] + ws[2] + ws[3]);
    }
}

__global__ void k_zero_out(uint64_t *counts, int64_t *sums, int32_t np)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    counts[p] = 0;
    if (sums) sums[p] = 0;
}

template <int LAYOUT, bool VALS>
__global__ __launch_bounds__(PROBE_BLOCK) void k_probe_global(const int4 *__restrict__ xy4,
                                                              const longlong2 *__restrict__ v2,
                                                              const int32_t *__restrict__ xy,
                                                              const int64_t *__restrict__ vals,
                                                              int64_t n, GridView g, HilbView hv,
                                                              Agg A, uint64_t *counts, int64_t *sums)
{
    unsigned long long *cnt = (unsigned long long *)counts;
    unsigned long long *sum = (unsigned long long *)sums;
    const int64_t npairs = n >> 1;
    const int64_t stride = (int64_t)gridDim.x * PROBE_BLOCK;
    for (int64_t t = (int64_t)blockIdx.x * PROBE_BLOCK + threadIdx.x; t < npairs; t += stride) {
        int4 q = xy4[t];
        longlong2 vv = VALS ? v2[t] : make_longlong2(0, 0);
        add_global<VALS>(code_of<LAYOUT>(g, hv, q.x, q.y), vv.x, A, cnt, sum);
        add_global<VALS>(code_of<LAYOUT>(g, hv, q.z, q.w), vv.y, A, cnt, sum);
    }
    if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
        int64_t k = n - 1;
        add_global<VALS>(code_of<LAYOUT>(g, hv, xy[2 * k], xy[2 * k + 1]), VALS ? vals[k] : 0, A,
                         cnt, sum);
    }
}

// ---------------------------------------------------------------- lookups

template <int LAYOUT>
__global__ void k_lookup(const int64_t *ij, int64_t n, GridView g, HilbView hv, int64_t gi0,
                         int64_t gj0, int64_t gw, int64_t gh, int64_t s, int32_t *ref)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    int64_t i = ij[2 * t], j = ij[2 * t + 1];
    uint32_t c = 0;
    if (LAYOUT == 0) {
        int64_t x = i - gi0, y = j - gj0;
        if (x >= 0 && y >= 0 && x < gw && y < gh) {
            // the cell's lower-left corner maps back to the cell
            c = grid_code(g, (int32_t)(i * s), (int32_t)(j * s));
        }
    } else {
        int64_t x = i - gi0, y = j - gj0;
        if (x >= 0 && y >= 0 && x < gw && y < gh) {
            uint64_t key = hilbert_index(hv.L, (uint32_t)x, (uint32_t)y);
            int64_t q = hv.k32 ? pred_search<uint32_t>(hv.k32, 0, hv.n, (uint32_t)key)
                               : pred_search<uint64_t>(hv.k64, 0, hv.n, key);
            c = hv.code[q];
        }
    }
    ref[t] = code_to_ref(c);
}

// ---------------------------------------------------------------- host

static int cu_count()
{
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (dev < 0 || dev >= 64) return 256;
    if (!cached[dev]) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            v <= 0)
            v = 256;
        cached[dev] = v;
    }
    return cached[dev];
}

static void views(const sba_handle *h, GridView *g, HilbView *hv)
{
    *g = GridView{};
    *hv = HilbView{};
    if (h->kind == SBA_KIND_GRID) {
        g->ox = h->gi0 * h->s;
        g->oy = h->gj0 * h->s;
        g->extx = (uint32_t)(h->gw * h->s);
        g->exty = (uint32_t)(h->gh * h->s);
        g->mag = h->mag;
        g->shift = h->shift;
        g->tl = h->tile_log2;
        g->tw = (uint32_t)h->tw;
        g->nblocks = (uint32_t)h->n_blocks;
        g->dir = h->dir;
        g->blocks = h->blocks;
    } else {
        hv->ox = h->gi0 * h->s;
        hv->oy = h->gj0 * h->s;
        hv->extx = (uint32_t)(h->gw * h->s);
        hv->exty = (uint32_t)(h->gh * h->s);
        hv->mag = h->mag;
        hv->shift = h->shift;
        hv->L = h->level;
        hv->n = h->n_runs;
        hv->k32 = h->starts32;
        hv->k64 = h->starts;
        hv->code = h->run_code;
        hv->a = h->root_a;
        hv->nl = 1u << h->log2_leaves;
        hv->leaves = h->leaves;
    }
}

// blocks per CU for the streaming probe
static int g_blocks_per_cu = 4;

template <int LAYOUT>
static int launch_layout(const int32_t *xy, const int64_t *values, int64_t n, const sba_handle *h,
                         uint64_t *counts, int64_t *sums, hipStream_t st)
{
    GridView g;
    HilbView hv;
    views(h, &g, &hv);
    Agg A{h->set_off, h->set_ids, (uint32_t)h->n_polys, (uint32_t)h->n_sets};
    const int32_t np = h->n_polys;
    const bool vals = values != nullptr && sums != nullptr;
    const int64_t npairs = n >> 1;
    int64_t nb = (npairs + PROBE_BLOCK - 1) / PROBE_BLOCK;
    int64_t cap = (int64_t)cu_count() * g_blocks_per_cu;
    if (nb > cap) nb = cap;
    if (nb < 1) nb = 1;
    const int4 *xy4 = (const int4 *)xy;
    const longlong2 *v2 = (const longlong2 *)values;
    if (np <= LDS_MAX_POLYS) {
        uint32_t *pcnt = nullptr;
        unsigned long long *psum = nullptr;
        size_t bytes = (size_t)nb * np * (sizeof(uint32_t) + (vals ? 8 : 0));
        char *scratch = nullptr;
        RC(tmp_alloc(&scratch, (int64_t)(bytes ? bytes : 8), st));
        psum = (unsigned long long *)scratch;
        pcnt = (uint32_t *)(vals ? (char *)scratch + (size_t)nb * np * 8 : (char *)scratch);
        size_t lds = (size_t)np * 12;
        if (vals)
            hipLaunchKernelGGL((k_probe_lds<LAYOUT, true>), dim3((unsigned)nb), dim3(PROBE_BLOCK), lds,
                               st, xy4, v2, xy, values, n, g, hv, A, np, pcnt, psum);
        else
            hipLaunchKernelGGL((k_probe_lds<LAYOUT, false>), dim3((unsigned)nb), dim3(PROBE_BLOCK), lds,
                               st, xy4, v2, xy, values, n, g, hv, A, np, pcnt, psum);
        hipError_t e1 = hipGetLastError();
        if (vals)
            hipLaunchKernelGGL(k_reduce<true>, dim3((unsigned)np), dim3(256), 0, st, pcnt, psum, nb, np,
                               counts, sums);
        else
            hipLaunchKernelGGL(k_reduce<false>, dim3((unsigned)np), dim3(256), 0, st, pcnt, psum, nb,
                               np, counts, sums);
        hipError_t e2 = hipGetLastError();
        tmp_free(scratch, st);
        if (e1 != hipSuccess || e2 != hipSuccess) return SBA_EDEVICE;
        return 0;
    }
    hipLaunchKernelGGL(k_zero_out, dim3(grid_for(np)), dim3(256), 0, st, counts, vals ? sums : nullptr,
                       np);
    if (vals)
        hipLaunchKernelGGL((k_probe_global<LAYOUT, true>), dim3((unsigned)nb), dim3(PROBE_BLOCK), 0, st,
                           xy4, v2, xy, values, n, g, hv, A, counts, sums);
    else
        hipLaunchKernelGGL((k_probe_global<LAYOUT, false>), dim3((unsigned)nb), dim3(PROBE_BLOCK), 0,
                           st, xy4, v2, xy, values, n, g, hv, A, counts, sums);
    HIP_OK(hipGetLastError());
    return 0;
}

int probe_launch(const int32_t *xy, const int64_t *values, int64_t n, const sba_handle *h,
                 int32_t search, uint64_t *counts, int64_t *sums, hipStream_t st)
{
    if (h->n_polys == 0) return 0;
    if (n == 0) {
        hipLaunchKernelGGL(k_zero_out, dim3(grid_for(h->n_polys)), dim3(256), 0, st, counts, sums,
                           h->n_polys);
        HIP_OK(hipGetLastError());
        return 0;
    }
    if (h->kind == SBA_KIND_GRID) return launch_layout<0>(xy, values, n, h, counts, sums, st);
    if (search == SBA_SEARCH_LEARNED) {
        if (!h->leaves) return SBA_EINVAL;
        return launch_layout<2>(xy, values, n, h, counts, sums, st);
    }
    return launch_layout<1>(xy, values, n, h, counts, sums, st);
}

int lookup_launch(const sba_handle *h, const int64_t *ij, int64_t n, int32_t *ref, hipStream_t st)
{
    if (n <= 0) return 0;
    GridView g;
    HilbView hv;
    views(h, &g, &hv);
    if (h->n_polys == 0 || (h->kind == SBA_KIND_GRID && h->gw == 0)) {
        HIP_OK(hipMemsetAsync(ref, 0xff, (size_t)n * 4, st));
        return 0;
    }
    if (h->kind == SBA_KIND_GRID)
        hipLaunchKernelGGL(k_lookup<0>, dim3(grid_for(n)), dim3(256), 0, st, ij, n, g, hv, h->gi0,
                           h->gj0, h->gw, h->gh, h->s, ref);
    else
        hipLaunchKernelGGL(k_lookup<1>, dim3(grid_for(n)), dim3(256), 0, st, ij, n, g, hv, h->gi0,
                           h->gj0, h->gw, h->gh, h->s, ref);
    HIP_OK(hipGetLastError());
    return 0;
}

extern "C" int sba_debug_set_blocks_per_cu(int k)
{
    if (k < 1 || k > 64) return SBA_EINVAL;
    g_blocks_per_cu = k;
    return 0;
}
