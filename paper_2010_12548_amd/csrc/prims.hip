// prims.hip -- device-wide exclusive scan and LSD radix sort used by the
// approximation build.  Written for 64-lane wavefronts.
#include "sba_internal.h"

#define SCAN_BLOCK 256
#define SCAN_ITEMS 8
#define SCAN_TILE (SCAN_BLOCK * SCAN_ITEMS)

// inclusive scan across a 64-lane wavefront
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    return v;
}

// exclusive scan across the block (blockDim.x == 256); returns the block total
template <typename T>
__device__ __forceinline__ T block_excl_scan(T v, T *excl)
{
    __shared__ T wsum[SCAN_BLOCK / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    T inc = wave_incl_scan(v);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    T off = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < SCAN_BLOCK / 64; k++) {
        if (k < w) off += wsum[k];
        tot += wsum[k];
    }
    __syncthreads();
    *excl = off + inc - v;
    return tot;
}

// Small arrays (n <= SCAN_SMALL): one workgroup, one launch.
#define SCAN_SMALL_ITEMS 32
#define SCAN_SMALL (SCAN_BLOCK * SCAN_SMALL_ITEMS)

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_small(const int64_t *in, int64_t *out,
                                                           int64_t n, int64_t *total)
{
    const int64_t base = (int64_t)threadIdx.x * SCAN_SMALL_ITEMS;
    int64_t v[SCAN_SMALL_ITEMS];
    int64_t run = 0;
#pragma unroll
    for (int k = 0; k < SCAN_SMALL_ITEMS; k++) {
        int64_t idx = base + k;
        v[k] = idx < n ? in[idx] : 0;
        run += v[k];
    }
    int64_t excl;
    int64_t tot = block_excl_scan<int64_t>(run, &excl);
#pragma unroll
    for (int k = 0; k < SCAN_SMALL_ITEMS; k++) {
        int64_t idx = base + k;
        if (idx < n) out[idx] = excl;
        excl += v[k];
    }
    if (threadIdx.x == 0 && total) total[0] = tot;
}

// Large arrays: per-tile sums, scan of the sums, then each tile scanned with
// its offset (reads the input twice, writes once; in may alias out).
__device__ __forceinline__ void tile_sum(const int64_t *in, int64_t n, int64_t tile, int64_t *sum)
{
    const int64_t base = tile * SCAN_TILE;
    int64_t run = 0;
    for (int k = threadIdx.x; k < SCAN_TILE; k += SCAN_BLOCK) {
        int64_t idx = base + k;
        if (idx < n) run += in[idx];
    }
    for (int o = 32; o > 0; o >>= 1) run += __shfl_xor(run, o, 64);
    __shared__ int64_t ws[SCAN_BLOCK / 64];
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = run;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int k = 0; k < SCAN_BLOCK / 64; k++) t += ws[k];
        *sum = t;
    }
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_tile_sums(const int64_t *in, int64_t n,
                                                          int64_t *sums)
{
    tile_sum(in, n, blockIdx.x, &sums[blockIdx.x]);
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_tile_scan(const int64_t *in, int64_t *out,
                                                          int64_t n, const int64_t *offs)
{
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    int64_t v[SCAN_ITEMS];
    int64_t run = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; k++) {
        int64_t idx = base + k;
        v[k] = idx < n ? in[idx] : 0;
        run += v[k];
    }
    int64_t excl;
    block_excl_scan<int64_t>(run, &excl);
    excl += offs[blockIdx.x];
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; k++) {
        int64_t idx = base + k;
        if (idx < n) out[idx] = excl;
        excl += v[k];
    }
}

template <typename T>
static int tmp_get(Workspace *ws, T **p, int64_t n, hipStream_t st)
{
    return ws ? ws->alloc(p, n) : tmp_alloc(p, n, st);
}

static void tmp_put(Workspace *ws, void *p, hipStream_t st)
{
    if (ws) ws->put(p);
    else tmp_free(p, st);
}

// Tiles <= SCAN_TILES_DIRECT: the second pass finds each tile's offset by
// summing the sums of the tiles before it (at most SCAN_TILES_DIRECT reads
// per block), so the scan takes two launches; the last tile writes the total.
#define SCAN_TILES_DIRECT 1024
#define SCAN_MULTI 4

__device__ __forceinline__ void tile_scan_direct(const int64_t *in, int64_t *out, int64_t n,
                                                 const int64_t *sums, int64_t tiles,
                                                 int64_t *total, int64_t tile)
{
    int64_t before = 0;
    for (int64_t t = threadIdx.x; t < tile; t += SCAN_BLOCK) before += sums[t];
    for (int o = 32; o > 0; o >>= 1) before += __shfl_xor(before, o, 64);
    __shared__ int64_t wb[SCAN_BLOCK / 64];
    if ((threadIdx.x & 63) == 0) wb[threadIdx.x >> 6] = before;
    __syncthreads();
    int64_t off = 0;
#pragma unroll
    for (int k = 0; k < SCAN_BLOCK / 64; k++) off += wb[k];
    const int64_t base = tile * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    int64_t v[SCAN_ITEMS];
    int64_t run = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; k++) {
        int64_t idx = base + k;
        v[k] = idx < n ? in[idx] : 0;
        run += v[k];
    }
    int64_t excl;
    const int64_t tot = block_excl_scan<int64_t>(run, &excl);
    excl += off;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; k++) {
        int64_t idx = base + k;
        if (idx < n) out[idx] = excl;
        excl += v[k];
    }
    if (total && tile == tiles - 1 && threadIdx.x == 0) total[0] = off + tot;
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_tile_scan_direct(const int64_t *in, int64_t *out,
                                                                 int64_t n, const int64_t *sums,
                                                                 int64_t tiles, int64_t *total)
{
    tile_scan_direct(in, out, n, sums, tiles, total, blockIdx.x);
}

// Up to SCAN_MULTI independent arrays of at most SCAN_TILES_DIRECT tiles
// each, scanned by one pair of launches: blockIdx.y picks the array, and
// blocks past an array's last tile return at once.
struct ScanSet {
    const int64_t *in[SCAN_MULTI];
    int64_t *out[SCAN_MULTI];
    int64_t n[SCAN_MULTI];
    int64_t *total[SCAN_MULTI];
    int64_t *sums;  // SCAN_MULTI rows of `stride` tile sums
    int64_t stride;
};

__device__ __forceinline__ int64_t set_tiles(const ScanSet &S, int y)
{
    return S.n[y] > 0 ? (S.n[y] + SCAN_TILE - 1) / SCAN_TILE : 0;
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_tile_sums_multi(ScanSet S)
{
    const int y = blockIdx.y;
    if ((int64_t)blockIdx.x >= set_tiles(S, y)) return;
    tile_sum(S.in[y], S.n[y], blockIdx.x, &S.sums[y * S.stride + blockIdx.x]);
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_tile_scan_direct_multi(ScanSet S)
{
    const int y = blockIdx.y;
    const int64_t tiles = set_tiles(S, y);
    if (tiles == 0) {  // an empty array: its total is 0
        if (blockIdx.x == 0 && threadIdx.x == 0 && S.total[y]) S.total[y][0] = 0;
        return;
    }
    if ((int64_t)blockIdx.x >= tiles) return;
    tile_scan_direct(S.in[y], S.out[y], S.n[y], S.sums + y * S.stride, tiles, S.total[y],
                     blockIdx.x);
}

int scan_exclusive_i64(const int64_t *in, int64_t *out, int64_t n, int64_t *total, hipStream_t st,
                       Workspace *ws)
{
    if (n <= 0) {
        if (total) HIP_OK(hipMemsetAsync(total, 0, sizeof(int64_t), st));
        return 0;
    }
    if (n <= SCAN_SMALL) {
        hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(SCAN_BLOCK), 0, st, in, out, n, total);
        HIP_OK(hipGetLastError());
        return 0;
    }
    const int64_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    int64_t *sums = nullptr;
    RC(tmp_get(ws, &sums, tiles, st));
    hipLaunchKernelGGL(k_tile_sums, dim3((unsigned)tiles), dim3(SCAN_BLOCK), 0, st, in, n, sums);
    int rc = hipGetLastError() == hipSuccess ? 0 : SBA_EDEVICE;
    if (!rc && tiles <= SCAN_TILES_DIRECT) {
        hipLaunchKernelGGL(k_tile_scan_direct, dim3((unsigned)tiles), dim3(SCAN_BLOCK), 0, st, in,
                           out, n, sums, tiles, total);
        rc = hipGetLastError() == hipSuccess ? 0 : SBA_EDEVICE;
        tmp_put(ws, sums, st);
        return rc;
    }
    if (!rc) rc = scan_exclusive_i64(sums, sums, tiles, total, st, ws);
    if (!rc) {
        hipLaunchKernelGGL(k_tile_scan, dim3((unsigned)tiles), dim3(SCAN_BLOCK), 0, st, in, out, n,
                           sums);
        rc = hipGetLastError() == hipSuccess ? 0 : SBA_EDEVICE;
    }
    tmp_put(ws, sums, st);
    return rc;
}

int scan_exclusive_i64_multi(int m, const int64_t *const *in, int64_t *const *out,
                             const int64_t *n, int64_t *const *total, hipStream_t st,
                             Workspace *ws)
{
    if (m < 0) return SBA_EINVAL;
    int64_t maxt = 1;
    bool together = m <= SCAN_MULTI;
    for (int k = 0; k < m; k++) {
        const int64_t t = n[k] > 0 ? (n[k] + SCAN_TILE - 1) / SCAN_TILE : 0;
        if (t > SCAN_TILES_DIRECT) together = false;
        maxt = std::max(maxt, t);
    }
    if (!together || m <= 1) {
        for (int k = 0; k < m; k++) RC(scan_exclusive_i64(in[k], out[k], n[k], total[k], st, ws));
        return 0;
    }
    ScanSet S{};
    for (int k = 0; k < m; k++) {
        S.in[k] = in[k];
        S.out[k] = out[k];
        S.n[k] = n[k];
        S.total[k] = total[k];
    }
    S.stride = maxt;
    RC(tmp_get(ws, &S.sums, (int64_t)m * maxt, st));
    hipLaunchKernelGGL(k_tile_sums_multi, dim3((unsigned)maxt, (unsigned)m), dim3(SCAN_BLOCK), 0,
                       st, S);
    int rc = hipGetLastError() == hipSuccess ? 0 : SBA_EDEVICE;
    if (!rc) {
        hipLaunchKernelGGL(k_tile_scan_direct_multi, dim3((unsigned)maxt, (unsigned)m),
                           dim3(SCAN_BLOCK), 0, st, S);
        rc = hipGetLastError() == hipSuccess ? 0 : SBA_EDEVICE;
    }
    tmp_put(ws, S.sums, st);
    return rc;
}

// ---------------------------------------------------------------- radix sort
//
// One pass per digit of RB = 8 bits (9 bits for sorts under RS_SMALL keys
// whose key width then needs one pass fewer), least significant first.  A
// block sorts a tile of RS_TILE keys: each of its 4 waves owns a contiguous
// quarter and walks it 64 keys at a time; lanes with equal digits find each
// other with RB ballots, so the rank of a key among equal digits before it is
// a popcount and the pass is stable.  Keys are staged in LDS in digit order
// and written out in runs, which keeps the global writes coalesced.

#define RS_BLOCK 256
#define RS_WAVES (RS_BLOCK / 64)
// A block sorts ROUNDS x 256 keys: 4 rounds below RS_SMALL keys, so that a
// sort of a few hundred thousand keys still spreads over every compute unit;
// 8 below RS_MID (28 KB of LDS per block, which fits beside a persistent probe
// holding the rest of a CU); 16 for larger inputs (fewer offsets to scan).
#define RS_SMALL (4 << 20)
#define RS_MID (64 << 20)
#define RS_RADIX 256       // digits of an 8-bit pass (the partition pass uses these offsets)

// per block and digit: count, laid out digit-major (hist[d * nblocks + b]).
// A workgroup counts `span` consecutive tiles, TPW at a time with every key
// of the TPW tiles loaded before any is counted (one tile a workgroup for
// small sorts).  No digit totals are formed
// here: each row scan below leaves its digit's total, and the scatter adds
// the totals of the lower digits itself, so the pass needs no device-wide
// atomics and no zeroed counters.
template <int ROUNDS, int TPW, int RB>
__global__ __launch_bounds__(RS_BLOCK) void k_rs_hist(const uint64_t *keys, int64_t n, int shift,
                                                      int64_t *hist, int64_t nblocks, int64_t span)
{
    constexpr int RS_TILE = RS_BLOCK * ROUNDS, RADIX = 1 << RB;
    __shared__ uint32_t h[TPW][RADIX];
    const int64_t bfirst = (int64_t)blockIdx.x * span;
    const int64_t blast = min(bfirst + span, nblocks);
    for (int64_t b0 = bfirst; b0 < blast; b0 += TPW) {
#pragma unroll
        for (int t = 0; t < TPW; t++)
            for (int d = threadIdx.x; d < RADIX; d += RS_BLOCK) h[t][d] = 0;
        __syncthreads();
        uint32_t dg[TPW * ROUNDS];
#pragma unroll
        for (int k = 0; k < TPW * ROUNDS; k++) {
            const int64_t idx = b0 * RS_TILE + (int64_t)k * RS_BLOCK + threadIdx.x;
            dg[k] = (idx < n && b0 + k / ROUNDS < blast)
                        ? (uint32_t)(keys[idx] >> shift) & (uint32_t)(RADIX - 1)
                        : RADIX;
        }
#pragma unroll
        for (int k = 0; k < TPW * ROUNDS; k++)
            if (dg[k] < RADIX) atomicAdd(&h[k / ROUNDS][dg[k]], 1u);
        __syncthreads();
#pragma unroll
        for (int t = 0; t < TPW; t++) {
            if (b0 + t < blast)
                for (int d = threadIdx.x; d < RADIX; d += RS_BLOCK)
                    hist[(int64_t)d * nblocks + b0 + t] = h[t][d];
        }
    }
}

// In place, one workgroup per digit d: the exclusive scan of digit d's block
// counts; the digit's total goes to rowtot[d].
__global__ __launch_bounds__(RS_BLOCK) void k_rs_rowscan(int64_t *hist, int64_t nblocks,
                                                         int64_t *rowtot)
{
    const int d = blockIdx.x;
    int64_t *row = hist + (int64_t)d * nblocks;
    int64_t carry = 0;
    for (int64_t c0 = 0; c0 < nblocks; c0 += RS_BLOCK * SCAN_ITEMS) {
        const int64_t b0 = c0 + (int64_t)threadIdx.x * SCAN_ITEMS;
        int64_t v[SCAN_ITEMS];
        int64_t run = 0;
#pragma unroll
        for (int k = 0; k < SCAN_ITEMS; k++) {
            v[k] = b0 + k < nblocks ? row[b0 + k] : 0;
            run += v[k];
        }
        int64_t excl;
        const int64_t tot = block_excl_scan<int64_t>(run, &excl);
        excl += carry;
#pragma unroll
        for (int k = 0; k < SCAN_ITEMS; k++) {
            if (b0 + k < nblocks) row[b0 + k] = excl;
            excl += v[k];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) rowtot[d] = carry;
}

// Scatter offsets in place, one workgroup per digit d: the keys of all lower
// digits (a sum over dtot) plus the exclusive scan of digit d's block counts.
__global__ __launch_bounds__(RS_BLOCK) void k_rs_offsets(int64_t *hist, int64_t nblocks,
                                                         const unsigned long long *dtot)
{
    const int d = blockIdx.x;
    int64_t below = 0;
    for (int e = threadIdx.x; e < d; e += RS_BLOCK) below += (int64_t)dtot[e];
    for (int o = 32; o > 0; o >>= 1) below += __shfl_xor(below, o, 64);
    __shared__ int64_t wb[RS_BLOCK / 64];
    if ((threadIdx.x & 63) == 0) wb[threadIdx.x >> 6] = below;
    __syncthreads();
    int64_t carry = 0;
    for (int k = 0; k < RS_BLOCK / 64; k++) carry += wb[k];
    int64_t *row = hist + (int64_t)d * nblocks;
    for (int64_t c0 = 0; c0 < nblocks; c0 += RS_BLOCK * SCAN_ITEMS) {
        const int64_t b0 = c0 + (int64_t)threadIdx.x * SCAN_ITEMS;
        int64_t v[SCAN_ITEMS];
        int64_t run = 0;
#pragma unroll
        for (int k = 0; k < SCAN_ITEMS; k++) {
            v[k] = b0 + k < nblocks ? row[b0 + k] : 0;
            run += v[k];
        }
        int64_t excl;
        const int64_t tot = block_excl_scan<int64_t>(run, &excl);
        excl += carry;
#pragma unroll
        for (int k = 0; k < SCAN_ITEMS; k++) {
            if (b0 + k < nblocks) row[b0 + k] = excl;
            excl += v[k];
        }
        carry += tot;
    }
}

int rs_offsets_launch(int64_t *hist, int64_t nblocks, const unsigned long long *dtot,
                      hipStream_t st)
{
    hipLaunchKernelGGL(k_rs_offsets, dim3(RS_RADIX), dim3(RS_BLOCK), 0, st, hist, nblocks, dtot);
    HIP_OK(hipGetLastError());
    return 0;
}

template <bool HAS_VALS, int ROUNDS, int RB>
__global__ __launch_bounds__(RS_BLOCK) void k_rs_scatter(const uint64_t *keys, const uint32_t *vals,
                                                         uint64_t *okeys, uint32_t *ovals,
                                                         int64_t n, int shift,
                                                         const int64_t *goff, int64_t nblocks,
                                                         const int64_t *rowtot)
{
    constexpr int RS_ROUNDS = ROUNDS, RS_TILE = RS_BLOCK * ROUNDS, RADIX = 1 << RB;
    constexpr int DPT = RADIX / RS_BLOCK;  // digits per thread, consecutive
    constexpr uint32_t DMASK = RADIX - 1;
    __shared__ uint32_t wcnt[RS_WAVES][RADIX];
    __shared__ uint32_t bdoff[RADIX];
    // output position of the block's first key of each digit, less that
    // key's place in the staged tile
    __shared__ int64_t dbase[RADIX];
    __shared__ uint64_t skeys[RS_TILE];
    __shared__ uint32_t svals[HAS_VALS ? RS_TILE : 1];

    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int d0 = threadIdx.x * DPT;
    // digits d0 .. d0 + DPT - 1: the block's offset within each digit, and
    // the keys of all lower digits
    {
        int64_t rt[DPT], run = 0;
#pragma unroll
        for (int j = 0; j < DPT; j++) {
            rt[j] = rowtot[d0 + j];
            run += rt[j];
        }
        int64_t below;
        block_excl_scan<int64_t>(run, &below);
#pragma unroll
        for (int j = 0; j < DPT; j++) {
            dbase[d0 + j] = below + goff[(int64_t)(d0 + j) * nblocks + blockIdx.x];
            below += rt[j];
        }
    }
    for (int k = threadIdx.x; k < RS_WAVES * RADIX; k += RS_BLOCK) (&wcnt[0][0])[k] = 0;
    __syncthreads();

    const int64_t tbase = (int64_t)blockIdx.x * RS_TILE;
    const int64_t wbase = tbase + (int64_t)w * (64 * RS_ROUNDS);
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    uint64_t kk[RS_ROUNDS];
    uint32_t vv[RS_ROUNDS];
    uint32_t loc[RS_ROUNDS];
#pragma unroll
    for (int q = 0; q < RS_ROUNDS; q++) {
        int64_t idx = wbase + q * 64 + lane;
        bool valid = idx < n;
        uint64_t key = valid ? keys[idx] : 0;
        kk[q] = key;
        if (HAS_VALS) vv[q] = valid ? vals[idx] : 0;
        uint32_t d = (uint32_t)(key >> shift) & DMASK;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < RB; b++) {
            uint64_t bal = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? bal : ~bal;
        }
        uint32_t old = wcnt[w][d];
        uint32_t rank = (uint32_t)__popcll(peers & lt);
        loc[q] = old + rank;
        __builtin_amdgcn_wave_barrier();
        if (valid && (peers & lt) == 0) wcnt[w][d] = old + (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // digits d0 ..: totals, wave prefixes, block-wide digit offsets
    {
        uint32_t cnt[DPT], run = 0;
#pragma unroll
        for (int j = 0; j < DPT; j++) {
            uint32_t r = 0;
#pragma unroll
            for (int k = 0; k < RS_WAVES; k++) {
                uint32_t c = wcnt[k][d0 + j];
                wcnt[k][d0 + j] = r;
                r += c;
            }
            cnt[j] = r;
            run += r;
        }
        uint32_t excl;
        block_excl_scan<uint32_t>(run, &excl);
#pragma unroll
        for (int j = 0; j < DPT; j++) {
            bdoff[d0 + j] = excl;
            dbase[d0 + j] -= (int64_t)excl;
            excl += cnt[j];
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < RS_ROUNDS; q++) {
        int64_t idx = wbase + q * 64 + lane;
        if (idx < n) {
            uint32_t d = (uint32_t)(kk[q] >> shift) & DMASK;
            uint32_t p = bdoff[d] + wcnt[w][d] + loc[q];
            skeys[p] = kk[q];
            if (HAS_VALS) svals[p] = vv[q];
        }
    }
    __syncthreads();
    int64_t tn = n - tbase;
    if (tn > RS_TILE) tn = RS_TILE;
    for (int i = threadIdx.x; i < tn; i += RS_BLOCK) {
        uint64_t key = skeys[i];
        uint32_t d = (uint32_t)(key >> shift) & DMASK;
        int64_t g = dbase[d] + i;
        okeys[g] = key;
        if (HAS_VALS) ovals[g] = svals[i];
    }
}

static int rs_rounds(int64_t n) { return n < RS_SMALL ? 4 : (n < RS_MID ? 8 : 16); }

static int64_t rs_blocks(int64_t n) { return (n + RS_BLOCK * rs_rounds(n) - 1) / (RS_BLOCK * rs_rounds(n)); }

// digit width of a sort of n keys of `bits` bits: 9 where that saves a pass
// for the small sorts (the build's), else 8
static int rs_digit_bits(int64_t n, int bits)
{
    return (n < RS_SMALL && (bits + 8) / 9 < (bits + 7) / 8) ? 9 : 8;
}

// one pass over digit (keys >> shift) & (2^RB - 1)
template <int ROUNDS, int RB>
static int rs_pass_t(const uint64_t *ka, const uint32_t *va, uint64_t *kb, uint32_t *vb, int64_t n,
                     int shift, int64_t *goff, int64_t nblocks, int64_t *rowtot, hipStream_t st)
{
    // tiles per counting workgroup: one while there are at most 2048 tiles
    // (every tile its own workgroup), else 16 keys a thread and at most about
    // 2048 workgroups
    if (nblocks <= 2048) {
        hipLaunchKernelGGL((k_rs_hist<ROUNDS, 1, RB>), dim3((unsigned)nblocks), dim3(RS_BLOCK), 0,
                           st, ka, n, shift, goff, nblocks, (int64_t)1);
    } else {
        constexpr int TPW = 16 / ROUNDS;
        const int64_t span = TPW * ((nblocks + TPW * 2048 - 1) / (TPW * 2048));
        hipLaunchKernelGGL((k_rs_hist<ROUNDS, TPW, RB>),
                           dim3((unsigned)((nblocks + span - 1) / span)), dim3(RS_BLOCK), 0, st, ka,
                           n, shift, goff, nblocks, span);
    }
    hipLaunchKernelGGL(k_rs_rowscan, dim3(1u << RB), dim3(RS_BLOCK), 0, st, goff, nblocks, rowtot);
    if (va)
        hipLaunchKernelGGL((k_rs_scatter<true, ROUNDS, RB>), dim3((unsigned)nblocks),
                           dim3(RS_BLOCK), 0, st, ka, va, kb, vb, n, shift, goff, nblocks, rowtot);
    else
        hipLaunchKernelGGL((k_rs_scatter<false, ROUNDS, RB>), dim3((unsigned)nblocks),
                           dim3(RS_BLOCK), 0, st, ka, va, kb, vb, n, shift, goff, nblocks, rowtot);
    return hipGetLastError() == hipSuccess ? 0 : SBA_EDEVICE;
}

static int rs_pass(const uint64_t *ka, const uint32_t *va, uint64_t *kb, uint32_t *vb, int64_t n,
                   int shift, int rb, int64_t *goff, int64_t nblocks, int64_t *rowtot,
                   hipStream_t st)
{
    const int r = rs_rounds(n);
    if (r == 4)
        return rb == 9 ? rs_pass_t<4, 9>(ka, va, kb, vb, n, shift, goff, nblocks, rowtot, st)
                       : rs_pass_t<4, 8>(ka, va, kb, vb, n, shift, goff, nblocks, rowtot, st);
    if (r == 8) return rs_pass_t<8, 8>(ka, va, kb, vb, n, shift, goff, nblocks, rowtot, st);
    return rs_pass_t<16, 8>(ka, va, kb, vb, n, shift, goff, nblocks, rowtot, st);
}

int radix_sort_u64(uint64_t *keys, uint32_t *vals, int64_t n, int bits, hipStream_t st,
                   Workspace *ws)
{
    if (n <= 1 || bits <= 0) return 0;
    const int64_t nblocks = rs_blocks(n);
    uint64_t *k2 = nullptr;
    uint32_t *v2 = nullptr;
    int64_t *goff = nullptr, *rowtot = nullptr;
    int rc = tmp_get(ws, &k2, n, st);
    if (!rc && vals) rc = tmp_get(ws, &v2, n, st);
    const int rb = rs_digit_bits(n, bits);
    if (!rc) rc = tmp_get(ws, &goff, nblocks << rb, st);
    if (!rc) rc = tmp_get(ws, &rowtot, (int64_t)1 << rb, st);
    const int passes = (bits + rb - 1) / rb;
    uint64_t *ka = keys, *kb = k2;
    uint32_t *va = vals, *vb = v2;
    for (int p = 0; p < passes && !rc; p++) {
        rc = rs_pass(ka, va, kb, vb, n, rb * p, rb, goff, nblocks, rowtot, st);
        if (rc) break;
        uint64_t *tk = ka; ka = kb; kb = tk;
        uint32_t *tv = va; va = vb; vb = tv;
    }
    if (!rc && ka != keys) {
        if (hipMemcpyAsync(keys, ka, (size_t)n * 8, hipMemcpyDeviceToDevice, st) != hipSuccess)
            rc = SBA_EDEVICE;
        if (!rc && vals &&
            hipMemcpyAsync(vals, va, (size_t)n * 4, hipMemcpyDeviceToDevice, st) != hipSuccess)
            rc = SBA_EDEVICE;
    }
    tmp_put(ws, k2, st);
    tmp_put(ws, v2, st);
    tmp_put(ws, goff, st);
    tmp_put(ws, rowtot, st);
    return rc;
}

int radix_sort_u64_ws(uint64_t **keys, uint32_t **vals, int64_t n, int bits, Workspace &ws)
{
    if (n <= 1 || bits <= 0) return 0;
    hipStream_t st = ws.stream();
    const int64_t nblocks = rs_blocks(n);
    uint64_t *k2 = nullptr;
    uint32_t *v2 = nullptr;
    int64_t *goff = nullptr, *rowtot = nullptr;
    RC(ws.alloc(&k2, n));
    if (vals && *vals) RC(ws.alloc(&v2, n));
    const int rb = rs_digit_bits(n, bits);
    RC(ws.alloc(&goff, nblocks << rb));
    RC(ws.alloc(&rowtot, (int64_t)1 << rb));
    const int passes = (bits + rb - 1) / rb;
    uint64_t *ka = *keys, *kb = k2;
    uint32_t *va = vals ? *vals : nullptr, *vb = v2;
    for (int p = 0; p < passes; p++) {
        RC(rs_pass(ka, va, kb, vb, n, rb * p, rb, goff, nblocks, rowtot, st));
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    // the sorted data stays where the last pass wrote it; the other buffers
    // go back to the workspace
    ws.put(kb);
    if (vb) ws.put(vb);
    ws.put(goff);
    ws.put(rowtot);
    *keys = ka;
    if (vals && *vals) *vals = va;
    return 0;
}

extern "C" int sba_debug_radix_sort(uint64_t *keys, uint32_t *vals, int64_t n, int32_t bits,
                                    void *stream)
{
    if (n < 0 || bits < 1 || bits > 64 || (n > 0 && !keys)) return SBA_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    RC(radix_sort_u64(keys, vals, n, bits, st, nullptr));
    HIP_OK(hipStreamSynchronize(st));
    return 0;
}

extern "C" int sba_debug_scan_multi(int32_t m, const int64_t *const *in, int64_t *const *out,
                                    const int64_t *n, int64_t *total, void *stream)
{
    if (m < 1 || m > 8 || !in || !out || !n || !total) return SBA_EINVAL;
    for (int k = 0; k < m; k++)
        if (n[k] < 0 || (n[k] > 0 && (!in[k] || !out[k]))) return SBA_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    int64_t *tot[8];
    for (int k = 0; k < m; k++) tot[k] = total + k;
    RC(scan_exclusive_i64_multi(m, in, out, n, tot, st, nullptr));
    HIP_OK(hipStreamSynchronize(st));
    return 0;
}

// ---------------------------------------------------------------- read rate
//
// The plain streaming read that bounds what a kernel which only reads its
// input can reach on the device: each lane walks one or two equally long
// buffers (the probe's two input streams) in 16-byte non-temporal loads, four
// per buffer in flight, and folds them into an XOR (one atomic per
// wavefront), so that no load can be dropped and nothing is written but one
// word.

typedef uint32_t rd4_t __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(1024) void k_stream_read(const rd4_t *p, const rd4_t *q, int64_t n16,
                                                      unsigned int *out)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t acc = 0;
    auto fold = [](rd4_t v) { return v.x ^ v.y ^ v.z ^ v.w; };
    for (; i + 3 * stride < n16; i += 4 * stride) {
        rd4_t a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; u++) a[u] = __builtin_nontemporal_load(p + i + u * stride);
        if (q) {
#pragma unroll
            for (int u = 0; u < 4; u++) b[u] = __builtin_nontemporal_load(q + i + u * stride);
#pragma unroll
            for (int u = 0; u < 4; u++) acc ^= fold(b[u]);
        }
#pragma unroll
        for (int u = 0; u < 4; u++) acc ^= fold(a[u]);
    }
    for (; i < n16; i += stride) {
        acc ^= fold(__builtin_nontemporal_load(p + i));
        if (q) acc ^= fold(__builtin_nontemporal_load(q + i));
    }
    for (int o = 32; o > 0; o >>= 1) acc ^= (uint32_t)__shfl_xor((int)acc, o, 64);
    if ((threadIdx.x & 63) == 0) atomicXor(out, acc);
}

extern "C" int sba_debug_stream_read(const void *a, const void *b, int64_t bytes, int32_t blocks,
                                     int32_t threads, uint32_t *xor_out, void *stream)
{
    if (bytes < 0 || (bytes & 15) || ((uintptr_t)a & 15) || ((uintptr_t)b & 15) ||
        (bytes > 0 && !a) || !xor_out || blocks < 1 || blocks > 65536 || threads < 64 ||
        threads > 1024 || (threads & 63))
        return SBA_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    HIP_OK(hipMemsetAsync(xor_out, 0, sizeof(uint32_t), st));
    if (bytes)
        hipLaunchKernelGGL(k_stream_read, dim3((unsigned)blocks), dim3((unsigned)threads), 0, st,
                           (const rd4_t *)a, (const rd4_t *)b, bytes / 16, xor_out);
    HIP_OK(hipGetLastError());
    return 0;
}
