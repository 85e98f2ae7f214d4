// sba_internal.h -- types and device helpers shared by the HIP sources of
// libsba (build, probe, primitives).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string.h>

#include <algorithm>
#include <vector>

#include "../../include/sba.h"

// ---------------------------------------------------------------- device memory (alloc.hip)

// A caller's device allocator (sba_build_opts.alloc / release / alloc_ctx);
// alloc == nullptr: the library's own block cache.
struct UserAlloc {
    void *(*alloc)(size_t bytes, void *ctx) = nullptr;
    void (*release)(void *p, void *ctx) = nullptr;
    void *ctx = nullptr;
};

struct DevBlock {
    void *p;
    size_t cls;  // size of the block (its size class)
    int dev;
    UserAlloc ua;  // the caller's allocator that gave the block, if any
};

int cache_get(size_t bytes, DevBlock *out);
// a block from the caller's allocator when it has one, else from the cache
int block_get(size_t bytes, const UserAlloc &ua, DevBlock *out);
// back to the caller's allocator or to the cache
void cache_put(const DevBlock &b);

// Temporaries of one stream-ordered job; the destructor synchronises the
// stream and returns every block to the device's cache.
// reads queued for one Workspace::sync
#define WS_MAX_READS 8

class Workspace {
public:
    explicit Workspace(hipStream_t st);
    ~Workspace();
    Workspace(const Workspace &) = delete;
    Workspace &operator=(const Workspace &) = delete;
    int get(void **p, size_t bytes);
    void put(void *p);  // reusable by later requests of this job
    template <typename T>
    int alloc(T **p, int64_t n)
    {
        void *q = nullptr;
        int rc = get(&q, (size_t)(n > 0 ? n : 1) * sizeof(T));
        *p = (T *)q;
        return rc;
    }
    // queue a copy of `bytes` (<= a few KB in all) device bytes for the host;
    // the host copies are filled by sync()
    int read(void *host, const void *dev, size_t bytes);
    int sync();
    hipStream_t stream() const { return st_; }
    // later blocks come from the caller's allocator (before the first get)
    void set_allocator(const UserAlloc &ua) { ua_ = ua; }

private:
    struct Read {
        void *host;
        const void *dev;
        size_t off, bytes;
    };
    hipStream_t st_;
    int dev_ = -1;
    std::vector<DevBlock> live_, spare_;
    std::vector<Read> reads_;
    char *pinned_ = nullptr;      // staging buffer (host address)
    char *pinned_dev_ = nullptr;  // its device address
    size_t staged_ = 0;
    UserAlloc ua_;
};

// ---------------------------------------------------------------- codes
//
// A grid cell holds a 32-bit code:
//   0                     no polygon
//   1 .. 2^30-1           exactly polygon (code - 1)
//   2^30 .. 2^31-1        the polygon set with index (code - 2^30)
// A directory entry of the two-level grid holds either such a code (the
// whole tile has it) or TILE_MIXED | block index (the tile's cells are
// stored in a fine block).
// The Hilbert layout and the lookup entry point use a signed "ref":
//   -1 no polygon, p >= 0 exactly polygon p, -2-k the set with index k.
#define CODE_SET_BASE 0x40000000u
#define TILE_MIXED 0x80000000u
#define MAX_POLYS ((1 << 21) - 1)
#define MAX_DEPTH 32           // polygons per cell
#define MAX_GRID_SIDE (1 << 21)
#define COMPACT_DIR_TILES 32768       // directory <= 64 KB at 16 bits
#define COMPACT_DIR_TILES_MAX 65536   // 16-bit directory still staged in LDS up to 128 KB
#define PROBE_LDS_BYTES (160 * 1024)  // LDS of one compute unit (gfx950)

__host__ __device__ inline int32_t code_to_ref(uint32_t c)
{
    if (c == 0) return -1;
    if (c < CODE_SET_BASE) return (int32_t)(c - 1);
    return -2 - (int32_t)(c - CODE_SET_BASE);
}

// ---------------------------------------------------------------- handle

struct sba_handle {
    int32_t kind, search;
    int32_t boundary_only;  // only the boundary cells B(P) are stored
    int32_t centre_sampled; // cells whose centre is inside (non-conservative)
    int32_t n_polys;
    int64_t eps, s;
    // stored cell box
    int64_t gi0, gj0, gw, gh;
    // cell index from a coordinate: q = ((uint64)(c - origin) * mag) >> shift
    uint32_t mag;
    int32_t shift;
    // grid layout: tiles of 2^tile_log2 cells a side; a mixed tile has a
    // sub-directory of sub-tiles of 2^sub_log2 cells (sub_log2 < tile_log2)
    // or is itself a fine block (sub_log2 == tile_log2); fine blocks hold one
    // code per cell.  One of two formats:
    //   wide     dir, sub, blocks: 32-bit codes, TILE_MIXED | index
    //   compact  dir16: 16-bit short codes (0 none, p+1 polygon p,
    //            n_polys+1+k set k) or 0x8000 | index, staged in LDS by the
    //            probe; sub: 32-bit, short code or TILE_MIXED | index;
    //            blocks16: 16-bit short codes
    int32_t tile_log2, sub_log2;
    int64_t tw, th;
    bool compact;
    uint32_t *dir;       // wide: [tw*th]
    uint16_t *dir16;     // compact: [tw*th rounded up to 8]
    uint32_t *sub;       // [n_blocks << 2*(tile_log2-sub_log2)] when sub_log2 < tile_log2
    uint32_t *blocks;    // wide: [n_fine << 2*fine_log2]
    uint16_t *blocks16;  // compact: same shape
    int64_t n_blocks;    // mixed tiles
    int64_t n_sub;       // mixed sub-tiles
    // polygon sets of multi-polygon cells
    int64_t *set_off;    // [n_sets+1] (device)
    int32_t *set_ids;    // [n_set_ids] (device)
    int64_t n_sets, n_set_ids;
    // Hilbert layout
    int32_t level;
    uint64_t *starts;    // [n_runs] run start keys
    uint32_t *starts32;  // [n_runs] same keys when 2*level <= 32 (else NULL)
    uint32_t *run_code;  // [n_runs] cell code of each run
    int64_t n_runs;
    // learned index over starts
    int32_t log2_leaves;
    float root_a;        // leaf = floor((float)(key - root_k0) * root_a)
    uint64_t root_k0;
    int4 *leaves;        // [2^log2_leaves] {key base (u32 bits), slope (f32 bits), icpt (f32 bits), err}
    int32_t *leaf_lo;    // [2^log2_leaves + 1] first run position of each leaf's key range
    int64_t max_leaf_err;
    double mean_leaf_err;
    // bookkeeping
    int64_t n_segments, n_boundary;
    int64_t bytes;
    double build_ms;
    int device;
    UserAlloc ua;                        // the caller's allocator of the arrays, if any
    std::vector<DevBlock> blocks_owned;  // every device array above
};

// device array of a handle (counted in h->bytes, released by handle_put_all)
int handle_get(sba_handle *h, void **p, size_t bytes);
void handle_put_all(sba_handle *h);
template <typename T>
inline int handle_alloc(sba_handle *h, T **p, int64_t n)
{
    void *q = nullptr;
    int rc = handle_get(h, &q, (size_t)(n > 0 ? n : 1) * sizeof(T));
    *p = (T *)q;
    return rc;
}

// ---------------------------------------------------------------- helpers

__host__ __device__ inline int64_t floordiv64(int64_t a, int64_t b)  // b > 0
{
    int64_t q = a / b;
    return q - ((a % b != 0) & (a < 0));
}

__host__ __device__ inline int64_t ceildiv64(int64_t a, int64_t b)  // b > 0
{
    int64_t q = a / b;
    return q + ((a % b != 0) & (a > 0));
}

// Division by the invariant cell side s for dividends 0 <= n < 2^31
// (Granlund & Montgomery 1994, "Division by invariant integers using
// multiplication", Thm. 4.2 with N = 31): with l = ceil(log2 s) and
// m = ceil(2^(31+l) / s) < 2^32, floor(n / s) = (n * m) >> (31 + l).
// Since floor(floor(a / 2^32) / 2^k) = floor(a / 2^(32+k)), a shift of 32 or
// more is a high-half multiply and a short shift; shift 31 only occurs for
// s = 1.
__host__ __device__ inline uint32_t divmagic(uint32_t n, uint32_t mag, int32_t shift)
{
    if (shift < 32) return (uint32_t)(((uint64_t)n * mag) >> shift);
    return (uint32_t)(((uint64_t)n * mag) >> 32) >> (shift - 32);
}

void magic_for(int64_t s, uint32_t *mag, int32_t *shift);

// Cell side for distance bound eps (Sec. 2.2): the largest integer s with
// 2 s^2 <= eps^2, i.e. isqrt(floor(eps^2 / 2)), found by doubling steps.
inline int64_t cell_side(int64_t eps)
{
    const int64_t t = eps * eps / 2;
    int64_t s = 0;
    while ((s + 1) * (s + 1) <= t) {
        int64_t step = 1;
        while ((s + 2 * step) * (s + 2 * step) <= t) step *= 2;
        s += step;
    }
    return s;
}

// Hilbert index d(i,j) of cell (i,j) on the 2^L x 2^L grid: quadrant order
// (0,0),(0,1),(1,1),(1,0) at every level, sub-squares re-oriented so that
// consecutive indices are edge-adjacent (Sec. 3, linearisation of cells).
// Processed one level at a time from the top; the orientation state is kept
// as a transpose flag and a reflection flag instead of rewriting i and j.
//
// One level: the quadrant digit of cell bits (bi, bj) in the current frame,
// and the frame of the next level.
__host__ __device__ inline uint32_t hilbert_level(uint32_t bi, uint32_t bj, uint32_t *swap,
                                                  uint32_t *flip)
{
    uint32_t x = (*swap ? bj : bi) ^ *flip;
    uint32_t y = (*swap ? bi : bj) ^ *flip;
    uint32_t q = (3u * x) ^ y;  // 0:(0,0) 1:(0,1) 2:(1,1) 3:(1,0)
    if (y == 0) {               // lower quadrants are transposed,
        if (x == 1) *flip ^= 1u;  // the lower-right one also complemented
        *swap ^= 1u;
    }
    return q;
}

__host__ __device__ inline uint64_t hilbert_index(int L, uint32_t i, uint32_t j)
{
    uint64_t d = 0;
    uint32_t swap = 0, flip = 0;  // current frame: transpose, then complement
    for (int lev = L - 1; lev >= 0; --lev)
        d = (d << 2) | hilbert_level((i >> lev) & 1u, (j >> lev) & 1u, &swap, &flip);
    return d;
}

// The same index four levels at a time through a table (kept in LDS by the
// probes).  Entry (frame << 8) | (i4 << 4) | j4 holds the 8 index bits of
// four levels of cell bits i4, j4 entered in frame (bit 0 transpose, bit 1
// complement) and, in bits 8-9, the frame they leave; hilbert_tab_entry
// builds it from hilbert_level, so both give the same index.
#define HILBERT_TAB 1024

__host__ __device__ inline uint16_t hilbert_tab_entry(uint32_t e)
{
    uint32_t swap = (e >> 8) & 1u, flip = (e >> 9) & 1u, d = 0;
    for (int lev = 3; lev >= 0; --lev)
        d = (d << 2) | hilbert_level((e >> (4 + lev)) & 1u, (e >> lev) & 1u, &swap, &flip);
    return (uint16_t)(d | (swap << 8) | (flip << 9));
}

// L <= 16: the levels above the last multiple of four one at a time, then
// four at a time
__host__ __device__ inline uint32_t hilbert_index_tab(int L, uint32_t i, uint32_t j,
                                                      const uint16_t *tab)
{
    uint32_t d = 0, swap = 0, flip = 0;
    int lev = L;
    while (lev & 3) {
        --lev;
        d = (d << 2) | hilbert_level((i >> lev) & 1u, (j >> lev) & 1u, &swap, &flip);
    }
    uint32_t fr = swap | (flip << 1);
    for (; lev > 0; lev -= 4) {
        const uint32_t e = tab[(fr << 8) | (((i >> (lev - 4)) & 15u) << 4) | ((j >> (lev - 4)) & 15u)];
        d = (d << 8) | (e & 255u);
        fr = e >> 8;
    }
    return d;
}

// Inverse of hilbert_index.
__host__ __device__ inline void hilbert_cell(int L, uint64_t d, uint32_t *pi, uint32_t *pj)
{
    uint32_t i = 0, j = 0, swap = 0, flip = 0;
    for (int lev = L - 1; lev >= 0; --lev) {
        uint32_t q = (uint32_t)(d >> (2 * lev)) & 3u;
        uint32_t x = (q >> 1) & 1u;            // q: 0->(0,0) 1->(0,1) 2->(1,1) 3->(1,0)
        uint32_t y = (q == 1 || q == 2) ? 1u : 0u;
        uint32_t fx = x ^ flip, fy = y ^ flip;  // undo the frame
        uint32_t bi = swap ? fy : fx, bj = swap ? fx : fy;
        i |= bi << lev;
        j |= bj << lev;
        if (y == 0) {
            if (x == 1) flip ^= 1u;
            swap ^= 1u;
        }
    }
    *pi = i;
    *pj = j;
}

// ---------------------------------------------------------------- learned index
//
// Root: leaf = floor(key * a) in fp32, clamped to [0, nl).  Leaf: predicted
// run position floor(slope * (key - kbase) + icpt) in fp32 with separate
// rounding of the product and the sum (no fused multiply-add), so the fit and
// the probe compute bit-identical predictions.
__device__ __forceinline__ uint32_t root_leaf(uint64_t key, float a, uint32_t nl)
{
    float f = __fmul_rn((float)key, a);
    return (f >= (float)nl) ? nl - 1 : (uint32_t)f;
}

__device__ __forceinline__ int64_t predict(uint64_t kbase, float slope, float icpt, uint64_t key)
{
    float x = (float)(key - kbase);
    float f = __fadd_rn(__fmul_rn(slope, x), icpt);
    return (int64_t)floorf(f);
}

// The run holding a key of leaf l is one of lo-1 .. hi-1, where [lo, hi) are
// the positions of the run starts inside the leaf's key range: clamp the
// prediction into that range (fit and probe alike), so no leaf's error can
// exceed its own size.
__device__ __forceinline__ void leaf_range(int64_t lo, int64_t hi, int64_t *a, int64_t *b)
{
    *a = lo > 0 ? lo - 1 : 0;
    *b = hi - 1 > *a ? hi - 1 : *a;
}

__device__ __forceinline__ int64_t predict_in_leaf(int4 lf, int64_t lo, int64_t hi, uint64_t key)
{
    int64_t a, b;
    leaf_range(lo, hi, &a, &b);
    int64_t p = predict((uint64_t)(uint32_t)lf.x, __int_as_float(lf.y), __int_as_float(lf.z), key);
    return p < a ? a : (p > b ? b : p);
}

// ---------------------------------------------------------------- primitives (prims.hip)

// Exclusive scan of n int64 values (in and out may alias).  If total is
// non-null the grand total is written to total[0] (device).
// Temporaries come from ws when given, else from the stream-ordered pool.
int scan_exclusive_i64(const int64_t *in, int64_t *out, int64_t n, int64_t *total, hipStream_t st,
                       Workspace *ws = nullptr);
// m independent scans (in[k] -> out[k], total into total[k] unless null):
// one pair of launches for up to 4 arrays of moderate size, else one by one
int scan_exclusive_i64_multi(int m, const int64_t *const *in, int64_t *const *out,
                             const int64_t *n, int64_t *const *total, hipStream_t st,
                             Workspace *ws = nullptr);

// LSD radix sort by the low `bits` bits of keys (bits <= 64), stable,
// carrying the optional 32-bit values.  The passes cover ceil(bits / 8) whole
// bytes: keys must be below 2^bits (every caller's are), bytes above those
// are ignored.  On return keys/vals hold the sorted
// data (the library ping-pongs through internal temporaries).
int radix_sort_u64(uint64_t *keys, uint32_t *vals, int64_t n, int bits, hipStream_t st,
                   Workspace *ws = nullptr);

// The same with the temporaries of ws, on its stream; the sorted keys/values
// are left in whichever buffer the last pass wrote: *keys / *vals are updated
// to it and the other buffer goes back to ws (so both must come from ws).
int radix_sort_u64_ws(uint64_t **keys, uint32_t **vals, int64_t n, int bits, Workspace &ws);

// In place: hist[d * nblocks + b] (per block b the count of digit d, 256
// digits) becomes the position of block b's first key of digit d in the
// output of a stable partition; dtot[d] holds the digit totals.
int rs_offsets_launch(int64_t *hist, int64_t nblocks, const unsigned long long *dtot,
                      hipStream_t st);

// device allocation helper (persistent arrays of a handle)
template <typename T>
inline int dev_alloc(T **p, int64_t count)
{
    *p = nullptr;
    if (count <= 0) count = 1;
    if (hipMalloc((void **)p, (size_t)count * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return SBA_ENOMEM;
    }
    return 0;
}

// Stream-ordered temporaries from the device's default memory pool, which is
// told to keep freed memory (pool_setup), so repeated builds and probes do
// not go back to the driver and frees do not synchronise the device.
int pool_setup();

template <typename T>
inline int tmp_alloc(T **p, int64_t count, hipStream_t st)
{
    *p = nullptr;
    if (count <= 0) count = 1;
    int prc = pool_setup();
    if (prc) return prc;
    if (hipMallocAsync((void **)p, (size_t)count * sizeof(T), st) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return SBA_ENOMEM;
    }
    return 0;
}

inline void tmp_free(void *p, hipStream_t st)
{
    if (p) (void)hipFreeAsync(p, st);
}

inline int bits_for(uint64_t maxval)  // bits needed to hold values in [0, maxval]
{
    int b = 0;
    while (b < 64 && (maxval >> b) != 0) b++;
    return b;
}

#define HIP_OK(x)                                   \
    do {                                            \
        if ((x) != hipSuccess) {                    \
            (void)hipGetLastError();                \
            return SBA_EDEVICE;                     \
        }                                           \
    } while (0)

#define RC(x)                 \
    do {                      \
        int rc_ = (x);        \
        if (rc_) return rc_;  \
    } while (0)

// Grid-size helper for element-wise kernels.
inline unsigned grid_for(int64_t n, int block = 256)
{
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    return (unsigned)g;
}

// Probe entry points (probe.hip).
int probe_launch(const int32_t *xy, const int64_t *values, int64_t n, const sba_handle *h,
                 int32_t search, uint64_t *counts, int64_t *sums, hipStream_t st);
int lookup_launch(const sba_handle *h, const int64_t *ij, int64_t n, int32_t *ref, hipStream_t st);
// the probe over contiguous items of points with an LDS table of cell codes
// (any layout; for points in spatial order)
// Points partitioned into 256 buckets by the top 8 bits of their Hilbert
// keys (2L-bit keys, bucket = key >> bshift): bucket b starts at
// bstart[b * bstride] of the partitioned array, and runs bq[b] .. bq[b + 1]
// hold every key of bucket b (bq has 257 entries, on the device).
struct PartRegions {
    const int64_t *bq;
    const int64_t *bstart;
    int64_t bstride;
    int32_t bshift;
};

// The item probe over partitioned points (regions: NULL, or the buckets of a
// Hilbert handle's points for its binary search).
int items_launch(const int32_t *xy, const int64_t *values, int64_t n, const sba_handle *h,
                 int32_t search, const PartRegions *regions, uint64_t *counts, int64_t *sums,
                 hipStream_t st);
int range_launch(const int32_t *xy, const int64_t *values, int64_t n, const sba_handle *h,
                 const sba_handle *hb, uint64_t *counts, int64_t *sums, uint64_t *bcounts,
                 int64_t *bsums, hipStream_t st);
int batch_launch(const sba_task *tasks, int32_t n_tasks, hipStream_t st);
int batch_launch_noalloc(const sba_task *tasks, int32_t n_tasks, hipStream_t st);
int bucket_launch(const int32_t *xy, const int64_t *values, int64_t n, int32_t x0, int32_t y0,
                  int32_t cell, int32_t G, int32_t *out_xy, int64_t *out_values, int64_t *off,
                  hipStream_t st);

// Build entry point (build.hip).
extern bool g_build_wide;
int key_grid_launch(const sba_polygons *sets, int32_t n_sets, int64_t eps, hipStream_t st,
                    int32_t *level, int64_t *i0, int64_t *j0);
int build_handle(const sba_polygons *polys, int64_t eps, const sba_build_opts *opts,
                 hipStream_t st, sba_handle *h);
