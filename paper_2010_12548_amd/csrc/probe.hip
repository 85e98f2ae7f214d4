// probe.hip -- the hot path: per-polygon COUNT and SUM of points, answered
// from the approximation alone (Sec. 5.1: index-nested-loop join of points
// against the cell index, aggregation fused, no point-in-polygon test).
//
// Each thread streams two points per iteration (one 128-bit load of x,y
// pairs, one 128-bit load of two int64 values), maps each point to its cell
// with a multiply-shift division by the cell side, looks up the cell's code
// and adds the point to a per-workgroup histogram in LDS.  At the end every
// workgroup adds its non-empty bins to the caller's outputs (zeroed by a
// small kernel before the probe) with one global atomic per bin; no global
// atomics per point.  Polygon counts too large for per-polygon bins use a
// per-workgroup LDS table of the cell codes met in a contiguous item of
// points instead.  A call allocates nothing.
//
// Cell lookup per layout:
//   grid     directory entry of the cell's tile (staged in LDS in the
//            16-bit format), for mixed tiles the sub-tile's entry, for mixed
//            sub-tiles the cell's code in a fine block;
//   hilbert  Hilbert key of the cell, then the run holding it: binary search
//            over the run starts, or the learned index's bounded search.
#include <stdio.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "sba_internal.h"

#define PROBE_BLOCK 256
#define PROBE_UNROLL 4
#define LDS_MAX_POLYS 4096

struct GridView {
    int64_t ox, oy;        // coordinate of the stored box's first cell
    uint32_t extx, exty;   // box extent in coordinate units (< 2^31)
    uint32_t mag;
    int32_t shift;
    int32_t tl, sl;        // tile and sub-tile side log2 (sl == tl: no sub level)
    uint32_t tw;
    uint32_t nblocks;      // mixed tiles
    uint32_t nfine;        // fine blocks
    uint32_t np;           // compact format: short codes above np are sets
    int32_t compact;       // 1: dir16 / sub / blocks16, 0: dir / sub / blocks
    const uint32_t *dir;
    const uint16_t *dir16;
    const uint32_t *sub;
    const uint32_t *blocks;
    const uint16_t *blocks16;
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
    const int32_t *leaf_lo;
    const uint16_t *tab;   // Hilbert table in LDS (set by the kernel) or NULL
    // Region of a partitioned item (set by the kernel, NULL otherwise): runs
    // sq0 .. sq1 hold every key of the item's points, and samp (in LDS) holds
    // every sS-th of their starts, sn of them: samp[j] = k32[sq0 + j * sS].
    const uint32_t *samp;
    int32_t sq0, sq1, sS, sn;
};

// the Hilbert key of cell (i, j) of the view's grid
__device__ __forceinline__ uint64_t hkey(const HilbView &v, uint32_t i, uint32_t j)
{
    return (v.tab && v.L <= 16) ? (uint64_t)hilbert_index_tab(v.L, i, j, v.tab)
                                : hilbert_index(v.L, i, j);
}

// fills an LDS copy of the Hilbert table (all threads of the workgroup;
// the caller synchronises before use)
__device__ __forceinline__ void hilbert_tab_fill(uint16_t *tab, int nthreads)
{
    for (int e = threadIdx.x; e < HILBERT_TAB; e += nthreads) tab[e] = hilbert_tab_entry((uint32_t)e);
}

// short code (compact format) -> cell code
__device__ __forceinline__ uint32_t full_code(uint32_t sc, uint32_t np)
{
    return sc <= np ? sc : CODE_SET_BASE + (sc - np - 1);
}

// Loads and adds through pointers that address device memory.  A pointer
// the kernel reads from memory (a batch task's) is generic to the compiler,
// which would emit flat accesses: they also count against the LDS wait
// counter, so each would wait out the LDS operations in flight as well.
// (The host pass only checks these; it never runs them.)
template <typename T>
__device__ __forceinline__ T gld(const T *p)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return *(const __attribute__((address_space(1))) T *)p;
#else
    return *p;
#endif
}

__device__ __forceinline__ void gadd(unsigned long long *p, unsigned long long v)
{
#if defined(__HIP_DEVICE_COMPILE__)
    __hip_atomic_fetch_add((__attribute__((address_space(1))) unsigned long long *)p, v,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#else
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#endif
}

__device__ __forceinline__ uint32_t grid_code(const GridView &g, int32_t x, int32_t y)
{
    int64_t dx = (int64_t)x - g.ox, dy = (int64_t)y - g.oy;
    if ((uint64_t)dx >= g.extx || (uint64_t)dy >= g.exty) return 0;
    uint32_t i = divmagic((uint32_t)dx, g.mag, g.shift);
    uint32_t j = divmagic((uint32_t)dy, g.mag, g.shift);
    uint32_t ti = (j >> g.tl) * g.tw + (i >> g.tl);
    uint32_t e, b;
    bool mixed;
    if (g.compact) {
        e = gld(g.dir16 + ti);
        mixed = (e & 0x8000u) != 0;
        b = e & 0x7fffu;
    } else {
        e = gld(g.dir + ti);
        mixed = (e & TILE_MIXED) != 0;
        b = e & ~TILE_MIXED;
    }
    if (!mixed) return g.compact ? full_code(e, g.np) : e;
    if (b >= g.nblocks) return 0;  // never taken for a well-formed handle
    int fl = g.tl;
    if (g.sl < g.tl) {
        const int qs = g.tl - g.sl;
        const uint32_t mq = (1u << qs) - 1u;
        uint32_t se = gld(g.sub + ((uint64_t)b << (2 * qs)) + ((((j >> g.sl) & mq) << qs) |
                                                                ((i >> g.sl) & mq)));
        if (!(se & TILE_MIXED)) return g.compact ? full_code(se, g.np) : se;
        b = se & ~TILE_MIXED;
        fl = g.sl;
    }
    if (b >= g.nfine) return 0;
    const uint32_t m = (1u << fl) - 1u;
    uint64_t idx = ((uint64_t)b << (2 * fl)) + ((j & m) << fl) + (i & m);
    return g.compact ? full_code(gld(g.blocks16 + idx), g.np) : gld(g.blocks + idx);
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
    int64_t llo = v.leaf_lo[l], lhi = v.leaf_lo[l + 1];
    int64_t p = predict_in_leaf(lf, llo, lhi, (uint64_t)key);
    int64_t ra, rb;
    leaf_range(llo, lhi, &ra, &rb);
    int64_t lo = p - lf.w, hi = p + lf.w;
    lo = lo < ra ? ra : lo;
    hi = hi > rb ? rb : hi;
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
    uint64_t key = hkey(v, i, j);
    int64_t q;
    if (v.k32) {
        q = SEARCH ? learned_search<uint32_t>(v, v.k32, (uint32_t)key)
                   : pred_search<uint32_t>(v.k32, 0, v.n, (uint32_t)key);
    } else {
        q = pred_search<uint64_t>(v.k64, 0, v.n, key);
    }
    return v.code[q];
}


// ---------------------------------------------------------------- batched lookups
//
// NP points at a time with no data-dependent branch around a load: all NP
// directory loads are issued together, then all NP block loads (a point in
// a uniform tile re-reads the first block word, a cache hit), so one
// iteration pays two memory latencies instead of 2*NP.

// FMT: 0 the handle's format read from g.compact, 1 compact, 2 32-bit
template <int NP, int FMT = 0>
__device__ __forceinline__ void grid_codes(const GridView &g, const int32_t *xs, const int32_t *ys,
                                           uint32_t *c)
{
    const bool cpt = FMT == 0 ? g.compact != 0 : FMT == 1;
    if (g.extx == 0) {  // empty handle (a clip window that holds no cell)
#pragma unroll
        for (int k = 0; k < NP; k++) c[k] = 0;
        return;
    }
    const bool two = g.sl < g.tl;
    const int qs = g.tl - g.sl;
    const int fl = two ? g.sl : g.tl;
    const uint32_t m = (1u << fl) - 1u, mq = (1u << qs) - 1u;
    uint32_t ti[NP], lo[NP], sq[NP];
    bool ok[NP];
#pragma unroll
    for (int k = 0; k < NP; k++) {
        int64_t dx = (int64_t)xs[k] - g.ox, dy = (int64_t)ys[k] - g.oy;
        ok[k] = (uint64_t)dx < g.extx && (uint64_t)dy < g.exty;
        uint32_t i = divmagic(ok[k] ? (uint32_t)dx : 0u, g.mag, g.shift);
        uint32_t j = divmagic(ok[k] ? (uint32_t)dy : 0u, g.mag, g.shift);
        ti[k] = (j >> g.tl) * g.tw + (i >> g.tl);
        lo[k] = ((j & m) << fl) | (i & m);
        sq[k] = (((j >> g.sl) & mq) << qs) | ((i >> g.sl) & mq);
    }
    // level 1: directory entry -> (uniform code | mixed tile b)
    uint32_t v[NP], b[NP];
    bool mix[NP];
#pragma unroll
    for (int k = 0; k < NP; k++) {
        uint32_t e = cpt ? (uint32_t)gld(g.dir16 + ti[k]) : gld(g.dir + ti[k]);
        mix[k] = cpt ? (e & 0x8000u) != 0 : (e & TILE_MIXED) != 0;
        b[k] = cpt ? (e & 0x7fffu) : (e & ~TILE_MIXED);
        mix[k] = mix[k] && b[k] < g.nblocks;
        v[k] = mix[k] ? 0u : (cpt ? full_code(e, g.np) : e);
        if (!ok[k]) { mix[k] = false; v[k] = 0; }
    }
    // level 2: sub-directory entry of mixed tiles
    if (two) {
        uint32_t se[NP];
#pragma unroll
        for (int k = 0; k < NP; k++)
            se[k] = gld(g.sub + (mix[k] ? ((uint64_t)b[k] << (2 * qs)) + sq[k] : 0));
#pragma unroll
        for (int k = 0; k < NP; k++) {
            if (!mix[k]) continue;
            if (se[k] & TILE_MIXED) {
                b[k] = se[k] & ~TILE_MIXED;
                mix[k] = b[k] < g.nfine;
            } else {
                v[k] = cpt ? full_code(se[k], g.np) : se[k];
                mix[k] = false;
            }
        }
    }
    // level 3: fine block cell
    uint32_t f[NP];
#pragma unroll
    for (int k = 0; k < NP; k++) {
        uint64_t idx = mix[k] ? ((uint64_t)b[k] << (2 * fl)) + lo[k] : 0;
        f[k] = cpt ? (uint32_t)gld(g.blocks16 + idx) : gld(g.blocks + idx);
    }
#pragma unroll
    for (int k = 0; k < NP; k++) c[k] = mix[k] ? (cpt ? full_code(f[k], g.np) : f[k]) : v[k];
}

// NP predecessor searches in lockstep over keys[lo[k] .. lo[k]+len): the
// step count depends only on len, so every step issues NP loads at once.
template <typename K, int NP>
__device__ __forceinline__ void pred_search_n(const K *keys, int64_t *lo, int64_t len, const K *key)
{
    while (len > 1) {
        const int64_t half = len >> 1;
        K v[NP];
#pragma unroll
        for (int k = 0; k < NP; k++) v[k] = keys[lo[k] + half];
#pragma unroll
        for (int k = 0; k < NP; k++) lo[k] = (v[k] <= key[k]) ? lo[k] + half : lo[k];
        len -= half;
    }
}

// As pred_search_n with a window length per point: the wave steps while any
// of its lanes still has a window longer than one (lanes that are done
// re-read their current key, which changes nothing).
template <typename K, int NP>
__device__ __forceinline__ void pred_search_var(const K *keys, int64_t *lo, int64_t *len,
                                                const K *key)
{
    while (true) {
        bool more = false;
#pragma unroll
        for (int k = 0; k < NP; k++) more |= len[k] > 1;
        if (!__any(more)) break;
        K v[NP];
        int64_t half[NP];
#pragma unroll
        for (int k = 0; k < NP; k++) {
            half[k] = len[k] >> 1;
            v[k] = keys[lo[k] + half[k]];
        }
#pragma unroll
        for (int k = 0; k < NP; k++) {
            lo[k] = (v[k] <= key[k]) ? lo[k] + half[k] : lo[k];
            len[k] -= half[k];
        }
    }
}

// 4-ary predecessor search with a window per point: each step issues three
// independent loads at the window's quarter points and keeps one quarter, so
// a window of W keys costs about log4(W) dependent round trips instead of
// log2(W) (the lookups are bound by such round trips); windows shorter than
// four take binary steps.  Lanes whose windows are done re-read their
// current key, which changes nothing.
template <int NP>
__device__ __forceinline__ void pred_search_var4(const uint32_t *keys, int32_t *lo, int32_t *len,
                                                 const uint32_t *key)
{
    while (true) {
        bool more = false;
#pragma unroll
        for (int k = 0; k < NP; k++) more |= len[k] > 1;
        if (!__any(more)) break;
        int32_t c1[NP], c2[NP], c3[NP];
#pragma unroll
        for (int k = 0; k < NP; k++) {
            const int32_t L = len[k];
            if (L >= 4) {
                c1[k] = lo[k] + (L >> 2);
                c2[k] = lo[k] + (L >> 1);
                c3[k] = lo[k] + (int32_t)(((int64_t)3 * L) >> 2);
            } else {
                c1[k] = c2[k] = c3[k] = lo[k] + (L > 1 ? (L >> 1) : 0);
            }
        }
        uint32_t v1[NP], v2[NP], v3[NP];
#pragma unroll
        for (int k = 0; k < NP; k++) {
            v1[k] = keys[c1[k]];
            v2[k] = keys[c2[k]];
            v3[k] = keys[c3[k]];
        }
#pragma unroll
        for (int k = 0; k < NP; k++) {
            if (len[k] <= 1) continue;
            int32_t end = lo[k] + len[k];
            if (v3[k] <= key[k]) {
                lo[k] = c3[k];
            } else if (v2[k] <= key[k]) {
                lo[k] = c2[k];
                end = c3[k];
            } else if (v1[k] <= key[k]) {
                lo[k] = c1[k];
                end = c2[k];
            } else {
                end = c1[k];
            }
            len[k] = end - lo[k];
        }
    }
}

// NP learned-index lookups in lockstep.  The leaf's model predicts p (clamped
// into the leaf's run range); the answer lies within the leaf's stored error
// of p, and a bounded 4-ary predecessor search over that window finds it.
// The bracket is verified; a full binary search is the fallback (never taken
// for an exact error bound).
template <int NP>
__device__ __forceinline__ void learned_search_n(const HilbView &v, const uint32_t *kk,
                                                 const uint64_t *key, int64_t *q,
                                                 unsigned long long *fallbacks = nullptr)
{
    const uint32_t *keys = v.k32;
    int4 lf[NP];
    int64_t llo[NP], lhi[NP];
    int32_t lo32[NP], len[NP];  // positions fit 31 bits (runs < 2^31)
#pragma unroll
    for (int k = 0; k < NP; k++) {
        uint32_t l = root_leaf(key[k], v.a, v.nl);
        lf[k] = v.leaves[l];
        llo[k] = v.leaf_lo[l];
        lhi[k] = v.leaf_lo[l + 1];
    }
#pragma unroll
    for (int k = 0; k < NP; k++) {
        int64_t ra, rb;
        leaf_range(llo[k], lhi[k], &ra, &rb);
        int64_t p = predict_in_leaf(lf[k], llo[k], lhi[k], key[k]);
        int64_t a = p - lf[k].w < ra ? ra : p - lf[k].w;
        int64_t e = p + lf[k].w > rb ? rb : p + lf[k].w;
        lo32[k] = (int32_t)a;
        len[k] = (int32_t)(e - a + 1);
    }
    uint32_t first[NP];
#pragma unroll
    for (int k = 0; k < NP; k++) first[k] = keys[lo32[k]];
    pred_search_var4<NP>(keys, lo32, len, kk);
#pragma unroll
    for (int k = 0; k < NP; k++) q[k] = lo32[k];
    uint32_t nxt[NP];
#pragma unroll
    for (int k = 0; k < NP; k++) nxt[k] = q[k] + 1 < v.n ? keys[q[k] + 1] : 0xffffffffu;
#pragma unroll
    for (int k = 0; k < NP; k++) {
        bool good = first[k] <= kk[k] && (q[k] + 1 == v.n || nxt[k] > kk[k]);
        if (!good) {  // bracket missed (never for an exact error bound): full search
            if (fallbacks) atomicAdd(fallbacks, 1ull);
            int64_t lo1[1] = {0};
            uint32_t k1[1] = {kk[k]};
            pred_search_n<uint32_t, 1>(keys, lo1, v.n, k1);
            q[k] = lo1[0];
        }
    }
}

// The same, NP/2 points at a time when NP >= 8 (unless FULL): each lookup
// holds a leaf, its range and its bracket, and the learned probe runs with
// more waves (more points in flight on the chip) when half of them are held
// at once.  FULL keeps all NP in flight per wave: points in no order within
// their region (the partitioned probe) take this search for nearly every
// point and gain more from the loads in flight than from the waves.
template <int NP, bool FULL = false>
__device__ __forceinline__ void learned_search_halves(const HilbView &v, const uint32_t *kk,
                                                      const uint64_t *key, int64_t *q)
{
    if constexpr (NP >= 8 && !FULL) {
        learned_search_n<NP / 2>(v, kk, key, q);
        learned_search_n<NP / 2>(v, kk + NP / 2, key + NP / 2, q + NP / 2);
    } else {
        learned_search_n<NP>(v, kk, key, q);
    }
}

template <int SEARCH, int NP, bool FULL = false>
__device__ __forceinline__ void hilbert_codes(const HilbView &v, const int32_t *xs, const int32_t *ys,
                                              uint32_t *c)
{
    if (v.extx == 0) {
#pragma unroll
        for (int k = 0; k < NP; k++) c[k] = 0;
        return;
    }
    bool ok[NP];
    uint64_t key[NP];
#pragma unroll
    for (int k = 0; k < NP; k++) {
        int64_t dx = (int64_t)xs[k] - v.ox, dy = (int64_t)ys[k] - v.oy;
        ok[k] = (uint64_t)dx < v.extx && (uint64_t)dy < v.exty;
        uint32_t i = divmagic(ok[k] ? (uint32_t)dx : 0u, v.mag, v.shift);
        uint32_t j = divmagic(ok[k] ? (uint32_t)dy : 0u, v.mag, v.shift);
        key[k] = hkey(v, i, j);
    }
    int64_t q[NP];
    if (v.k32) {
        uint32_t k32[NP];
#pragma unroll
        for (int k = 0; k < NP; k++) k32[k] = (uint32_t)key[k];
        if (SEARCH) {
            learned_search_halves<NP, FULL>(v, k32, key, q);
        } else {
#pragma unroll
            for (int k = 0; k < NP; k++) q[k] = 0;
            pred_search_n<uint32_t, NP>(v.k32, q, v.n, k32);
        }
    } else {
#pragma unroll
        for (int k = 0; k < NP; k++) q[k] = 0;
        pred_search_n<uint64_t, NP>(v.k64, q, v.n, key);
    }
    uint32_t r[NP];
#pragma unroll
    for (int k = 0; k < NP; k++) r[k] = v.code[q[k]];
#pragma unroll
    for (int k = 0; k < NP; k++) c[k] = ok[k] ? r[k] : 0u;
}

// Wave-bracketed Hilbert lookups for points in spatial order.  The NP
// points of every lane of the wave (all lanes take part: the caller keeps
// the wave together) have keys in [kmin, kmax]; two searches with those
// wave-uniform keys -- binary search or the learned index, as the handle
// is searched -- give the runs qlo and qhi that hold them.  When the
// bracket spans at most 64 runs, the wave reads the bracket's starts and
// codes once (a lane each) and every point finds its run by a binary search
// over the lanes' registers: no memory access per point.  A wider bracket
// (points in no order) takes the per-point search.  Exact either way: the
// run of every key lies in [qlo, qhi].
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v)
{
    for (int o = 32; o > 0; o >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, o, 64));
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v)
{
    for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o, 64));
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

// Binary search through a partitioned item's region: the last sample
// start <= key in LDS, then the at most sS runs after it in global memory
// (one or two cache lines) instead of a search over every run.
template <int NP>
__device__ __forceinline__ void hilbert_codes_region(const HilbView &v, const uint32_t *key,
                                                     const bool *ok, uint32_t *c)
{
    int32_t j[NP];
#pragma unroll
    for (int k = 0; k < NP; k++) j[k] = 0;
    for (int32_t len = v.sn; len > 1;) {
        const int32_t half = len >> 1;
#pragma unroll
        for (int k = 0; k < NP; k++) j[k] = v.samp[j[k] + half] <= key[k] ? j[k] + half : j[k];
        len -= half;
    }
    int32_t lo[NP], len[NP];
#pragma unroll
    for (int k = 0; k < NP; k++) {
        lo[k] = v.sq0 + j[k] * v.sS;
        len[k] = min(v.sS, v.sq1 + 1 - lo[k]);
    }
    pred_search_var4<NP>(v.k32, lo, len, key);
    uint32_t r[NP];
#pragma unroll
    for (int k = 0; k < NP; k++) r[k] = v.code[lo[k]];
#pragma unroll
    for (int k = 0; k < NP; k++) c[k] = ok[k] ? r[k] : 0u;
}

template <int SEARCH, int NP, bool FULL = false>
__device__ __forceinline__ void hilbert_codes_wave(const HilbView &v, const int32_t *xs,
                                                   const int32_t *ys, uint32_t *c)
{
    if (v.extx == 0 || !v.k32) {  // empty handle; 64-bit keys take the plain path
        hilbert_codes<SEARCH, NP, FULL>(v, xs, ys, c);
        return;
    }
    bool ok[NP];
    uint32_t key[NP];
    uint32_t kmin = 0xffffffffu, kmax = 0u;
#pragma unroll
    for (int k = 0; k < NP; k++) {
        int64_t dx = (int64_t)xs[k] - v.ox, dy = (int64_t)ys[k] - v.oy;
        ok[k] = (uint64_t)dx < v.extx && (uint64_t)dy < v.exty;
        uint32_t i = divmagic(ok[k] ? (uint32_t)dx : 0u, v.mag, v.shift);
        uint32_t j = divmagic(ok[k] ? (uint32_t)dy : 0u, v.mag, v.shift);
        key[k] = (uint32_t)hkey(v, i, j);
        kmin = ok[k] ? min(kmin, key[k]) : kmin;
        kmax = ok[k] ? max(kmax, key[k]) : kmax;
    }
    if constexpr (FULL && !SEARCH) {
        if (v.samp) {  // a partitioned item's region
            hilbert_codes_region<NP>(v, key, ok, c);
            return;
        }
    }
    kmin = wave_min_u32(kmin);
    kmax = wave_max_u32(kmax);
    if (kmax < kmin) {  // no point of the wave lies in the stored box
#pragma unroll
        for (int k = 0; k < NP; k++) c[k] = 0;
        return;
    }
    // runs expected in [kmin, kmax] if they were spread evenly over the
    // 4^L keys: far more than a wave holds means points in no spatial order
    // (or spread over a partition region), where the bracket searches would
    // only add to the per-point ones
    if (((uint64_t)(kmax - kmin) * (uint64_t)v.n) >> (2 * v.L) > 1024) {
        hilbert_codes<SEARCH, NP, FULL>(v, xs, ys, c);
        return;
    }
    const int64_t qlo = SEARCH ? learned_search<uint32_t>(v, v.k32, kmin)
                               : pred_search<uint32_t>(v.k32, 0, v.n, kmin);
    const int64_t qhi = SEARCH ? learned_search<uint32_t>(v, v.k32, kmax)
                               : pred_search<uint32_t>(v.k32, 0, v.n, kmax);
    const int32_t w = (int32_t)__builtin_amdgcn_readfirstlane((int)(qhi - qlo + 1));
    if (qhi - qlo + 1 > 64) {
        // per point, a binary search restricted to the bracket; a learned
        // index searches a bracket of more than 4096 runs through its own
        // windows instead
        int64_t q[NP];
        if (SEARCH && qhi - qlo + 1 > 4096) {
            uint64_t k64[NP];
#pragma unroll
            for (int k = 0; k < NP; k++) k64[k] = key[k];
            learned_search_halves<NP, FULL>(v, key, k64, q);
        } else {
#pragma unroll
            for (int k = 0; k < NP; k++) q[k] = qlo;
            pred_search_n<uint32_t, NP>(v.k32, q, qhi - qlo + 1, key);
        }
        uint32_t r[NP];
#pragma unroll
        for (int k = 0; k < NP; k++) r[k] = v.code[q[k]];
#pragma unroll
        for (int k = 0; k < NP; k++) c[k] = ok[k] ? r[k] : 0u;
        return;
    }
    const int lane = (int)(threadIdx.x & 63);
    const int64_t mine = qlo + (lane < w ? lane : w - 1);
    const uint32_t wstart = v.k32[mine];
    const uint32_t wcode = v.code[mine];
#pragma unroll
    for (int k = 0; k < NP; k++) {
        // last lane l < w with wstart(l) <= key: keys[qlo] <= kmin <= key
        int lo = 0, len = w;
        while (len > 1) {
            const int half = len >> 1;
            const uint32_t sv = (uint32_t)__shfl((int)wstart, lo + half, 64);
            lo = sv <= key[k] ? lo + half : lo;
            len -= half;
        }
        const uint32_t cv = (uint32_t)__shfl((int)wcode, lo, 64);
        c[k] = ok[k] ? cv : 0u;
    }
}

template <int LAYOUT, int NP>
__device__ __forceinline__ void codes_of(const GridView &g, const HilbView &hv, const int32_t *xs,
                                         const int32_t *ys, uint32_t *c)
{
    if (LAYOUT == 0) grid_codes<NP>(g, xs, ys, c);
    else hilbert_codes<LAYOUT == 2 ? 1 : 0, NP>(hv, xs, ys, c);
}

// As codes_of, with the wave-bracketed lookups for the Hilbert layouts; every
// lane of the wave must call it.
template <int LAYOUT, int NP, bool FULL = false>
__device__ __forceinline__ void codes_of_wave(const GridView &g, const HilbView &hv,
                                              const int32_t *xs, const int32_t *ys, uint32_t *c)
{
    if (LAYOUT == 0) grid_codes<NP>(g, xs, ys, c);
    else hilbert_codes_wave<LAYOUT == 2 ? 1 : 0, NP, FULL>(hv, xs, ys, c);
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
                                           unsigned long long *cnt, unsigned long long *sum,
                                           unsigned long long n = 1)
{
    if (code == 0) return;
    if (code < CODE_SET_BASE) {
        uint32_t p = code - 1u;
        if (p >= A.np) return;
        gadd(&cnt[p], n);
        if (VALS) gadd(&sum[p], (unsigned long long)val);
    } else {
        uint32_t k = code - CODE_SET_BASE;
        if (k >= A.n_sets) return;
        for (int64_t t = gld(A.set_off + k), e = gld(A.set_off + k + 1); t < e; t++) {
            uint32_t p = (uint32_t)gld(A.set_ids + t);
            if (p >= A.np) continue;
            gadd(&cnt[p], n);
            if (VALS) gadd(&sum[p], (unsigned long long)val);
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

// A workgroup's LDS histogram into the outputs (zeroed before the launch):
// one global atomic per non-empty bin.  Integer addition is associative, so
// the result does not depend on the order of the workgroups.
template <bool VALS>
__device__ __forceinline__ void flush_bins(const uint32_t *lcnt, const unsigned long long *lsum,
                                           uint32_t np, uint32_t nthreads, uint64_t *counts,
                                           int64_t *sums)
{
    for (uint32_t p = threadIdx.x; p < np; p += nthreads) {
        uint32_t c = lcnt[p];
        if (c == 0) continue;
        atomicAdd((unsigned long long *)&counts[p], (unsigned long long)c);
        if (VALS && lsum[p] != 0) atomicAdd((unsigned long long *)&sums[p], lsum[p]);
    }
}

// LDS-privatised histograms, added to the outputs once per workgroup
template <int LAYOUT, bool VALS>
__global__ __launch_bounds__(PROBE_BLOCK) void k_probe_lds(const int4 *__restrict__ xy4,
                                                           const longlong2 *__restrict__ v2,
                                                           const int32_t *__restrict__ xy,
                                                           const int64_t *__restrict__ vals,
                                                           int64_t n, GridView g, HilbView hv,
                                                           Agg A, int32_t np,
                                                           uint64_t *__restrict__ counts,
                                                           int64_t *__restrict__ sums)
{
    extern __shared__ unsigned long long smem[];
    __shared__ uint16_t s_htab[LAYOUT ? HILBERT_TAB : 1];
    unsigned long long *lsum = smem;
    uint32_t *lcnt = (uint32_t *)(smem + np);
    for (int p = threadIdx.x; p < np; p += PROBE_BLOCK) {
        lcnt[p] = 0;
        lsum[p] = 0;
    }
    if (LAYOUT) {
        hilbert_tab_fill(s_htab, PROBE_BLOCK);
        hv.tab = s_htab;
    }
    __syncthreads();
    const int64_t npairs = n >> 1;
    const int64_t stride = (int64_t)gridDim.x * PROBE_BLOCK;
    // PROBE_UNROLL pairs per lane per trip: the stream loads of the trip are
    // issued together, then the cell lookups of all 2*PROBE_UNROLL points
    // (batched, see grid_codes); latency is hidden by the other waves
    for (int64_t t0 = (int64_t)blockIdx.x * PROBE_BLOCK + threadIdx.x; t0 < npairs;
         t0 += stride * PROBE_UNROLL) {
        int4 q[PROBE_UNROLL];
        longlong2 vv[PROBE_UNROLL];
#pragma unroll
        for (int u = 0; u < PROBE_UNROLL; u++) {
            int64_t t = t0 + (int64_t)u * stride;
            q[u] = t < npairs ? xy4[t] : make_int4(INT32_MIN, INT32_MIN, INT32_MIN, INT32_MIN);
            vv[u] = (VALS && t < npairs) ? v2[t] : make_longlong2(0, 0);
        }
        int32_t xs[2 * PROBE_UNROLL], ys[2 * PROBE_UNROLL];
#pragma unroll
        for (int u = 0; u < PROBE_UNROLL; u++) {
            xs[2 * u] = q[u].x;
            ys[2 * u] = q[u].y;
            xs[2 * u + 1] = q[u].z;
            ys[2 * u + 1] = q[u].w;
        }
        uint32_t c[2 * PROBE_UNROLL];
        codes_of<LAYOUT, 2 * PROBE_UNROLL>(g, hv, xs, ys, c);
#pragma unroll
        for (int u = 0; u < PROBE_UNROLL; u++) {
            add_lds<VALS>(c[2 * u], vv[u].x, A, lcnt, lsum);
            add_lds<VALS>(c[2 * u + 1], vv[u].y, A, lcnt, lsum);
        }
    }
    if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
        int64_t k = n - 1;
        uint32_t c = code_of<LAYOUT>(g, hv, xy[2 * k], xy[2 * k + 1]);
        add_lds<VALS>(c, VALS ? vals[k] : 0, A, lcnt, lsum);
    }
    __syncthreads();
    flush_bins<VALS>(lcnt, lsum, np, PROBE_BLOCK, counts, sums);
}

// one block per polygon: sum the workgroup histograms, overwrite the outputs
__global__ void k_zero_out(uint64_t *counts, int64_t *sums, int32_t np)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    counts[p] = 0;
    if (sums) sums[p] = 0;
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
        g->sl = h->sub_log2;
        g->tw = (uint32_t)h->tw;
        g->nblocks = (uint32_t)h->n_blocks;
        g->nfine = (uint32_t)(h->sub_log2 < h->tile_log2 ? h->n_sub : h->n_blocks);
        g->np = (uint32_t)h->n_polys;
        g->compact = h->compact ? 1 : 0;
        g->dir = h->dir;
        g->dir16 = h->dir16;
        g->sub = h->sub;
        g->blocks = h->blocks;
        g->blocks16 = h->blocks16;
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
        hv->leaf_lo = h->leaf_lo;
    }
}

// blocks per CU for the streaming probe
static int g_blocks_per_cu = 8;

static int launch_items(const int32_t *xy, const int64_t *values, int64_t n, const sba_handle *h,
                        int layout, bool part, uint64_t *counts, int64_t *sums, hipStream_t st,
                        const PartRegions *regions = nullptr);


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
        hipLaunchKernelGGL(k_zero_out, dim3(grid_for(np)), dim3(256), 0, st, counts,
                           vals ? sums : nullptr, np);
        size_t lds = (size_t)np * 12;
        if (vals)
            hipLaunchKernelGGL((k_probe_lds<LAYOUT, true>), dim3((unsigned)nb), dim3(PROBE_BLOCK), lds,
                               st, xy4, v2, xy, values, n, g, hv, A, np, counts, sums);
        else
            hipLaunchKernelGGL((k_probe_lds<LAYOUT, false>), dim3((unsigned)nb), dim3(PROBE_BLOCK), lds,
                               st, xy4, v2, xy, values, n, g, hv, A, np, counts, sums);
        HIP_OK(hipGetLastError());
        return 0;
    }
    return launch_items(xy, values, n, h, LAYOUT, false, counts, sums, st);
}


// ---------------------------------------------------------------- grid probe, LDS directory
//
// The 16-bit directory (<= 128 KB) is copied into LDS once per workgroup;
// a point in a uniform tile then costs one LDS read instead of a random
// global gather (1e8 scattered 4-byte gathers are bounded by the L2 request
// rate, not by bytes).  Points in mixed tiles read their cell's 16-bit code
// from the fine blocks in global memory, batched 8 points at a time.  The
// point stream uses non-temporal loads, so it does not evict the blocks.

typedef int v4i_t __attribute__((ext_vector_type(4)));
typedef long long v2l_t __attribute__((ext_vector_type(2)));

// How a workgroup of the grid probe handles multi-polygon cells:
#define SETS_GLOBAL 0  // walk the set's members in the global set table
#define SETS_LDS 1     // walk them in a 16-bit copy of the table staged in LDS
#define SETS_BINS 2    // one histogram bin per set; expanded once per workgroup

struct Grid16 {
    int64_t ox, oy;
    uint32_t extx, exty;
    uint32_t mag;
    int32_t shift;
    // floor(n / s) = mul_hi(n << pre, mag) >> post (see grid16_div)
    uint32_t pre, post;
    int32_t tl, sl;               // tile / sub-tile side log2
    uint32_t tw;
    uint32_t nt16;                // directory entries, a multiple of 8
    const uint16_t *dir16;
    const uint32_t *sub;          // short code or TILE_MIXED | fine block (SUB kernels)
    const uint16_t *blocks16;
    uint32_t np;                  // short codes: p+1 polygon p, > np set (code - np - 1)
    uint32_t sets;                // SETS_*
    uint32_t n_ids;               // set table ids
    uint32_t nsub16;              // sub-directory entries staged in LDS (level 2), multiple of 8
    uint32_t nsub;                // sub-directory entries (level 2)
};

// Loads at a 32-bit byte offset from a wave-uniform base: the compiler
// keeps the base in scalar registers and adds the offset in the load
// (global_load ... v_off, s[base]), with no 64-bit address arithmetic.
template <typename T>
__device__ __forceinline__ T load_off(const void *base, uint32_t byte_off)
{
    return *(const T *)((const char *)base + byte_off);
}
template <typename T>
__device__ __forceinline__ T load_off_nt(const void *base, uint32_t byte_off)
{
    return __builtin_nontemporal_load((const T *)((const char *)base + byte_off));
}

// Workgroup-private state of the grid probe in LDS.
struct Lds16 {
    const uint16_t *dir;
    uint32_t *cnt;                // [np] or [np + n_sets] with SETS_BINS
    unsigned long long *sum;
    const uint16_t *soff, *sids;  // SETS_LDS
};

template <bool VALS>
__device__ __forceinline__ void add_member(uint32_t p, int64_t v, uint32_t np, const Lds16 &L)
{
    if (p >= np) return;
    atomicAdd(&L.cnt[p], 1u);
    if (VALS) atomicAdd(&L.sum[p], (unsigned long long)v);
}

template <bool VALS, int SETS>
__device__ __forceinline__ void add_short(uint32_t sc, int64_t v, const Agg &A, uint32_t np,
                                          const Lds16 &L)
{
    if (SETS == SETS_BINS) {
        // polygon p has bin p and set k bin np + k: both are bin sc - 1
        if (sc - 1u >= np + A.n_sets) return;
        atomicAdd(&L.cnt[sc - 1], 1u);
        if (VALS) atomicAdd(&L.sum[sc - 1], (unsigned long long)v);
        return;
    }
    if (sc == 0) return;
    if (sc <= np) {
        atomicAdd(&L.cnt[sc - 1], 1u);
        if (VALS) atomicAdd(&L.sum[sc - 1], (unsigned long long)v);
        return;
    }
    uint32_t k = sc - np - 1;
    if (k >= A.n_sets) return;
    if (SETS == SETS_BINS) {
        atomicAdd(&L.cnt[np + k], 1u);
        if (VALS) atomicAdd(&L.sum[np + k], (unsigned long long)v);
    } else if (SETS == SETS_LDS) {
        for (uint32_t t = L.soff[k], e = L.soff[k + 1]; t < e; t++)
            add_member<VALS>(L.sids[t], v, np, L);
    } else {
        for (int64_t t = A.set_off[k], e = A.set_off[k + 1]; t < e; t++)
            add_member<VALS>((uint32_t)A.set_ids[t], v, np, L);
    }
}

// short code of one point (the odd last point)
template <bool SUB>
__device__ __forceinline__ uint32_t grid16_code(const Grid16 &g, const uint16_t *ldir, int32_t x,
                                                int32_t y)
{
    int64_t dx = (int64_t)x - g.ox, dy = (int64_t)y - g.oy;
    if ((uint64_t)dx >= g.extx || (uint64_t)dy >= g.exty) return 0;
    uint32_t i = divmagic((uint32_t)dx, g.mag, g.shift);
    uint32_t j = divmagic((uint32_t)dy, g.mag, g.shift);
    uint32_t e = ldir[(j >> g.tl) * g.tw + (i >> g.tl)];
    if (!(e & 0x8000u)) return e;
    uint32_t b = e & 0x7fffu;
    int fl = g.tl;
    if (SUB) {
        const int qs = g.tl - g.sl;
        const uint32_t mq = (1u << qs) - 1u;
        uint32_t se = g.sub[((uint64_t)b << (2 * qs)) + ((((j >> g.sl) & mq) << qs) |
                                                           ((i >> g.sl) & mq))];
        if (!(se & TILE_MIXED)) return se;
        b = se & ~TILE_MIXED;
        fl = g.sl;
    }
    const uint32_t m = (1u << fl) - 1u;
    return g.blocks16[((uint64_t)b << (2 * fl)) + (((j & m) << fl) | (i & m))];
}

// LEV: 0 no sub-tiles (mixed tiles are fine blocks), 1 sub-directory read
// from global memory, 2 sub-directory staged in LDS as 16-bit entries (short
// code or 0x8000 | fine block), so only points in mixed sub-tiles leave LDS.
template <bool VALS, int LEV, int SETS, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_probe_grid16(const int4 *__restrict__ xy4,
                                                        const longlong2 *__restrict__ v2,
                                                        const int32_t *__restrict__ xy,
                                                        const int64_t *__restrict__ vals,
                                                        int64_t n, Grid16 g, Agg A,
                                                        uint64_t *__restrict__ counts,
                                                        int64_t *__restrict__ sums)
{
    // LDS: directory (nt16 entries, a multiple of 8), with LEV 2 the
    // sub-directory (nsub16 entries, a multiple of 8), sums (u64 [nb]),
    // counts (u32 [nb]) with nb = np (+ n_sets with SETS_BINS), then with
    // SETS_LDS the set table (u16 [n_sets + 1], u16 [n_ids]).  Every pointer
    // is formed by pointer arithmetic on the shared array, so the compiler
    // keeps LDS instructions for all of them.
    constexpr bool SUB = LEV != 0;
    constexpr bool GSUB = LEV == 1;
    extern __shared__ unsigned long long smem[];
    const uint32_t np = g.np;
    const uint32_t nbins = np + (SETS == SETS_BINS ? A.n_sets : 0u);
    const uint32_t nsub16 = LEV == 2 ? g.nsub16 : 0u;
    Lds16 L;
    uint16_t *ldir = (uint16_t *)smem;
    uint16_t *lsub = ldir + g.nt16;
    L.dir = ldir;
    L.sum = smem + (g.nt16 + nsub16) / 4;
    L.cnt = (uint32_t *)(L.sum + nbins);
    L.soff = (const uint16_t *)(L.cnt + nbins);
    L.sids = L.soff + A.n_sets + 1;
    {
        const uint4 *src = (const uint4 *)g.dir16;
        uint4 *dst = (uint4 *)ldir;
        for (uint32_t q = threadIdx.x; q < g.nt16 / 8; q += BLOCK) dst[q] = src[q];
        if (LEV == 2) {
            // 32-bit entries (short code, or TILE_MIXED | fine block below
            // 2^15) to 16 bits; the padding entries read as empty
            for (uint32_t q = threadIdx.x; q < nsub16; q += BLOCK) {
                const uint32_t se = q < g.nsub ? g.sub[q] : 0u;
                lsub[q] = (uint16_t)((se & TILE_MIXED) ? (0x8000u | (se & 0x7fffu)) : se);
            }
        }
        for (uint32_t p = threadIdx.x; p < nbins; p += BLOCK) {
            L.cnt[p] = 0;
            L.sum[p] = 0;
        }
        if (SETS == SETS_LDS) {
            uint16_t *so = (uint16_t *)L.soff, *si = (uint16_t *)L.sids;
            for (uint32_t k = threadIdx.x; k <= A.n_sets; k += BLOCK)
                so[k] = (uint16_t)A.set_off[k];
            for (uint32_t t = threadIdx.x; t < g.n_ids; t += BLOCK) si[t] = (uint16_t)A.set_ids[t];
        }
    }
    __syncthreads();
    const int qs = g.tl - g.sl;
    const int fl = SUB ? g.sl : g.tl;
    const uint32_t m = (1u << fl) - 1u, mq = (1u << qs) - 1u;
    const int64_t npairs = n >> 1;
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    const int64_t trip = stride * PROBE_UNROLL;
    const int64_t tlast = npairs - 1;
    const uint32_t ox = (uint32_t)g.ox, oy = (uint32_t)g.oy;
    // Three-stage software pipeline.  Trip r covers pairs [r trip, (r + 1) trip)
    // of the whole grid, PROBE_UNROLL pairs per lane, and pass r of the loop
    //   C  adds the points of trip r - 2 (their fine-block codes have arrived),
    //   B  reads the sub-tile entries of trip r - 1 and issues its fine-block
    //      gathers and its value loads,
    //   A  looks up the LDS directory for trip r (its coordinates have
    //      arrived) and issues its sub-tile gathers,
    // and then issues the coordinate loads of trip r + 1.  Vector memory
    // loads complete in issue order, so each pass waits once for the loads of
    // the pass before (the coordinates last): the latencies of the stream and
    // of both gather levels overlap instead of adding up.  Without a global
    // sub-directory (LEV 0, or LEV 2 with it in LDS) there is no stage B: A
    // finds the fine block itself and C adds trip r - 1.
    //
    // Every load is a 32-bit byte offset from a scalar base: a lane's offset
    // inside a trip is the same in every trip (only the base moves), and
    // gathers take 32-bit offsets into arrays below 4 GB (grid16_fits).  A
    // lane with no point (past the end) or no gather to make reads offset 0,
    // in bounds.
    constexpr int K = 2 * PROBE_UNROLL;
    constexpr int LAG = GSUB ? 2 : 1;
    // A point's state between stages is one word in the sub-directory's
    // format: a short code, or TILE_MIXED | index of the block (sub-tile
    // entry or fine block) that holds its code.
    struct StA {                   // trip r: coordinates
        v4i_t q[PROBE_UNROLL];
    };
    struct StB {                   // trip r - 1: sub-tile entry (loaded), state, cell in block
        uint32_t se[K], e[K], lo[K];
    };
    struct StC {                   // trip r - LAG: fine-block code (loaded), state, values
        uint32_t f[K], e[K];
        v2l_t val[PROBE_UNROLL];
    };
    const int64_t T = (npairs + trip - 1) / trip;  // trips, the same for every lane
    const int64_t passes = T > 0 ? T + LAG : 0;    // no loads at all without pairs
    // a lane's pairs inside a trip: tb + u stride < trip <= 2^22 (at most
    // 1024 workgroups of 1024 lanes, 4 pairs each): 16-byte offsets fit 32 bits
    // (whether a pair exists is compared again where it is needed rather
    // than kept: flags kept across passes would hold scalar register pairs)
    const uint32_t tb = blockIdx.x * BLOCK + threadIdx.x;
    // all ones when a state word names a block, zero for a code: selects
    // without lane masks
    auto blk = [](uint32_t e) -> uint32_t { return (uint32_t)((int32_t)e >> 31); };
    auto trip_pairs = [&](int64_t r) -> uint32_t {
        const int64_t rem = npairs - r * trip;
        return (uint32_t)(rem < trip ? rem : trip);
    };
    auto load_xy = [&](int64_t r, StA &a) {
        const uint32_t mp = trip_pairs(r);
        const void *base = xy4 + r * trip;
#pragma unroll
        for (int u = 0; u < PROBE_UNROLL; u++) {
            const uint32_t o = tb + (uint32_t)u * (uint32_t)stride;
            a.q[u] = load_off_nt<v4i_t>(base, o < mp ? o * 16u : 0u);
        }
    };
    auto load_vals = [&](int64_t r, StC &c) {
        const uint32_t mp = trip_pairs(r);
        const void *base = v2 + r * trip;
#pragma unroll
        for (int u = 0; u < PROBE_UNROLL; u++) {
            const uint32_t o = tb + (uint32_t)u * (uint32_t)stride;
            c.val[u] = load_off_nt<v2l_t>(base, o < mp ? o * 16u : 0u);
        }
    };
    auto pass = [&](int64_t r, const StA &ai, StA &ao, const StB &bi, StB &bo, const StC &ci,
                    StC &co) {
        // C: trip r - LAG
        if (r >= LAG) {
#pragma unroll
            for (int k = 0; k < K; k++) {
                const uint32_t t = blk(ci.e[k]);
                add_short<VALS, SETS>((ci.f[k] & t) | (ci.e[k] & ~t),
                                      (k & 1) ? ci.val[k >> 1].y : ci.val[k >> 1].x, A, np, L);
            }
        }
        // B: trip r - 1: a point in a mixed tile takes its sub-tile entry
        uint32_t eB[K];
#pragma unroll
        for (int k = 0; k < K; k++) {
            const uint32_t t = GSUB ? blk(bi.e[k]) : 0u;
            eB[k] = (bi.se[k] & t) | (bi.e[k] & ~t);
        }
        // A: trip r, from the LDS directory
        uint32_t eA[K], loA[K], sqA[K];
        const uint32_t mpA = r < T ? trip_pairs(r) : 0u;
#pragma unroll
        for (int k = 0; k < K; k++) {
            int32_t x = (k & 1) ? ai.q[k >> 1].z : ai.q[k >> 1].x;
            int32_t y = (k & 1) ? ai.q[k >> 1].w : ai.q[k >> 1].y;
            // offsets from the box origin modulo 2^32: the stored box lies
            // inside (-2^30 - 2^29, 2^30 + 2^28) (polygon coordinates below
            // 2^30 in magnitude, cells below 2^28), so no int32 point is 2^32
            // away from a position in the box, and the wrapped offset is
            // below ext exactly when the point is in the box
            uint32_t dx = (uint32_t)x - ox, dy = (uint32_t)y - oy;
            bool ok = tb + (uint32_t)(k >> 1) * (uint32_t)stride < mpA && dx < g.extx &&
                      dy < g.exty;
            uint32_t i = __umulhi((ok ? dx : 0u) << g.pre, g.mag) >> g.post;
            uint32_t j = __umulhi((ok ? dy : 0u) << g.pre, g.mag) >> g.post;
            uint32_t e = ldir[(j >> g.tl) * g.tw + (i >> g.tl)];
            if (!ok) e = 0;
            loA[k] = ((j & m) << fl) | (i & m);
            sqA[k] = SUB ? (((j >> g.sl) & mq) << qs) | ((i >> g.sl) & mq) : 0u;
            if (LEV == 2) {
                // the sub-tile entry from LDS (entry 0 for a uniform tile)
                const uint32_t se =
                    lsub[((e & 0x8000u) ? ((e & 0x7fffu) << (2 * qs)) + sqA[k] : 0u)];
                e = (e & 0x8000u) ? se : e;
            }
            eA[k] = (e & 0x8000u) ? (TILE_MIXED | (e & 0x7fffu)) : e;
        }
        // every load of the pass, in the order the next pass needs them
        __builtin_amdgcn_sched_barrier(0);
        if (GSUB) {
#pragma unroll
            for (int k = 0; k < K; k++)
                bo.se[k] = load_off<uint32_t>(
                    g.sub, ((((eA[k] & ~TILE_MIXED) << (2 * qs)) + sqA[k]) << 2) & blk(eA[k]));
        }
#pragma unroll
        for (int k = 0; k < K; k++) {
            // without a global sub-directory the fine block is known in stage A
            const uint32_t e = GSUB ? eB[k] : eA[k];
            const uint32_t o = GSUB ? bi.lo[k] : loA[k];
            co.f[k] = load_off<uint16_t>(g.blocks16,
                                         ((((e & ~TILE_MIXED) << (2 * fl)) + o) << 1) & blk(e));
        }
        // values of the trip whose codes were just gathered
        const int64_t rv = r - (LAG - 1);
        if (VALS && rv >= 0 && rv < T) load_vals(rv, co);
        if (r + 1 < T) load_xy(r + 1, ao);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int k = 0; k < K; k++) {
            co.e[k] = GSUB ? eB[k] : eA[k];
            bo.e[k] = eA[k];
            bo.lo[k] = loA[k];
        }
    };
    StA a0, a1;
    StB b0, b1;
    StC c0, c1;
#pragma unroll
    for (int k = 0; k < K; k++) {
        b0.se[k] = b0.e[k] = b0.lo[k] = 0;
        c0.f[k] = c0.e[k] = 0;
    }
#pragma unroll
    for (int u = 0; u < PROBE_UNROLL; u++) {
        c0.val[u] = v2l_t{0, 0};
        a0.q[u] = v4i_t{0, 0, 0, 0};
    }
    if (T > 0) load_xy(0, a0);
    for (int64_t r = 0; r < passes; r++) {
        pass(r, a0, a1, b0, b1, c0, c1);
        a0 = a1;
        b0 = b1;
        c0 = c1;
    }
    if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
        int64_t k = n - 1;
        uint32_t sc = grid16_code<SUB>(g, ldir, xy[2 * k], xy[2 * k + 1]);
        add_short<VALS, SETS>(sc, VALS ? vals[k] : 0, A, np, L);
    }
    __syncthreads();
    if (SETS == SETS_BINS) {
        // each set's bin goes to its members' bins
        for (uint32_t k = threadIdx.x; k < A.n_sets; k += BLOCK) {
            uint32_t c = L.cnt[np + k];
            if (c == 0) continue;
            unsigned long long sv = VALS ? L.sum[np + k] : 0ull;
            for (int64_t t = A.set_off[k], e = A.set_off[k + 1]; t < e; t++) {
                uint32_t p = (uint32_t)A.set_ids[t];
                if (p >= np) continue;
                atomicAdd(&L.cnt[p], c);
                if (VALS) atomicAdd(&L.sum[p], sv);
            }
        }
        __syncthreads();
    }
    flush_bins<VALS>(L.cnt, L.sum, np, BLOCK, counts, sums);
}

#define GRID16_LDS_MAX PROBE_LDS_BYTES
// cap on workgroups per CU of the LDS-directory grid probe (0: none)
static int g_grid16_per_cu = 0;
#define GRID16_SETS_MAX (16 * 1024)  // largest set table staged in LDS (bytes)

static size_t grid16_dir_lds(const sba_handle *h)
{
    return (size_t)(((h->tw * h->th) + 7) & ~(int64_t)7) * 2;
}

// set handling and LDS bytes of the grid probe for a handle: bins when
// directory + (polygons + sets) bins fit, else the staged table when it
// fits, else the global table
static int g_grid16_sets = -1;  // forced SETS_* mode (when it fits), -1: automatic

static int g_grid16_lsub = -1;   // 0: never stage the sub-directory in LDS, -1: when it fits

// How the grid probe runs on a handle: set handling, sub-directory level and
// LDS bytes.  In order of preference: bins for polygons and sets, the set
// table in LDS, the global set table; for each, the sub-directory staged in
// LDS when its 16-bit entries fit there too (every fine block index below
// 2^15), else read from global memory.
struct Grid16Plan {
    int sets;         // SETS_*
    int lev;          // 0 no sub-tiles, 1 global sub-directory, 2 sub-directory in LDS
    uint32_t nsub, nsub16;
    size_t lds;
};

static Grid16Plan grid16_plan(const sba_handle *h)
{
    const size_t dir = grid16_dir_lds(h), np = (size_t)h->n_polys, ns = (size_t)h->n_sets;
    const bool sub = h->sub_log2 < h->tile_log2;
    Grid16Plan pl{SETS_GLOBAL, sub ? 1 : 0, 0, 0, 0};
    size_t lsub = 0;
    if (sub && g_grid16_lsub != 0 && h->n_sub < 0x8000) {
        const int64_t ne = std::max<int64_t>(h->n_blocks << (2 * (h->tile_log2 - h->sub_log2)), 1);
        if (ne < ((int64_t)1 << 24)) {
            pl.nsub = (uint32_t)ne;
            pl.nsub16 = (uint32_t)((ne + 7) & ~(int64_t)7);
            lsub = (size_t)pl.nsub16 * 2;
        }
    }
    const int want = g_grid16_sets;
    const size_t table = (ns + 1 + (size_t)h->n_set_ids) * 2;
    const bool bins_ok = (want < 0 || want == SETS_BINS) && ns > 0;
    const bool table_ok = (want < 0 || want == SETS_LDS) && ns > 0 && h->n_set_ids < 0xffff &&
                          table <= GRID16_SETS_MAX;
    const size_t need[3] = {bins_ok ? dir + (np + ns) * 12 : SIZE_MAX,
                            table_ok ? dir + np * 12 + table : SIZE_MAX, dir + np * 12};
    const int modes[3] = {SETS_BINS, SETS_LDS, SETS_GLOBAL};
    for (int t = 0; t < 3; t++) {
        if (need[t] == SIZE_MAX) continue;
        if (lsub && need[t] + lsub <= GRID16_LDS_MAX) {
            pl.sets = modes[t];
            pl.lev = 2;
            pl.lds = need[t] + lsub;
            return pl;
        }
        if (need[t] <= GRID16_LDS_MAX || t == 2) {
            pl.sets = modes[t];
            pl.nsub = pl.nsub16 = 0;
            pl.lds = need[t];
            return pl;
        }
    }
    return pl;
}

static size_t grid16_lds(const sba_handle *h) { return grid16_plan(h).lds; }

// Byte sizes of a compact grid's sub-directory and fine blocks as the build
// allocates them (one-element placeholders when nothing is mixed).
static void grid16_bytes(const sba_handle *h, uint64_t *sub_b, uint64_t *blk_b)
{
    const int qs = h->tile_log2 - h->sub_log2;
    const bool sub = qs > 0;
    *sub_b = sub ? (uint64_t)std::max<int64_t>(h->n_blocks << (2 * qs), 1) * 4 : 4;
    const int fl = sub ? h->sub_log2 : h->tile_log2;
    const int64_t nfine = sub ? h->n_sub : h->n_blocks;
    *blk_b = (uint64_t)std::max<int64_t>(nfine << (2 * fl), 1) * 2;
}

// The LDS-directory grid probe takes the handle: compact codes, directory and
// bins within the LDS, gathered arrays addressable with 32-bit offsets.
static bool grid16_fits(const sba_handle *h)
{
    if (!h->compact || grid16_lds(h) > GRID16_LDS_MAX) return false;
    uint64_t a = 0, b = 0;
    grid16_bytes(h, &a, &b);
    return a <= 0xffffffffull && b <= 0xffffffffull;
}

// 16 or more waves per CU: workgroups of 512 threads when two fit in the LDS
// (up to four, as LDS and the 32 wave slots allow), else one of 1024 threads
// per CU
static void grid16_shape(size_t lds, int *block, int *per_cu)
{
    int k = (int)std::min<size_t>((size_t)GRID16_LDS_MAX / lds, 4);
    if (g_grid16_per_cu > 0) k = std::min(k, g_grid16_per_cu);
    *block = k < 2 ? 1024 : 512;
    *per_cu = k < 2 ? 1 : k;
}

typedef void (*grid16_fn)(const int4 *, const longlong2 *, const int32_t *, const int64_t *,
                          int64_t, Grid16, Agg, uint64_t *, int64_t *);

template <bool VALS, int LEV, int BLOCK>
static grid16_fn grid16_pick_sets(int sets)
{
    if (sets == SETS_BINS) return k_probe_grid16<VALS, LEV, SETS_BINS, BLOCK>;
    if (sets == SETS_LDS) return k_probe_grid16<VALS, LEV, SETS_LDS, BLOCK>;
    return k_probe_grid16<VALS, LEV, SETS_GLOBAL, BLOCK>;
}

template <bool VALS, int BLOCK>
static grid16_fn grid16_pick_lev(int lev, int sets)
{
    if (lev == 2) return grid16_pick_sets<VALS, 2, BLOCK>(sets);
    if (lev == 1) return grid16_pick_sets<VALS, 1, BLOCK>(sets);
    return grid16_pick_sets<VALS, 0, BLOCK>(sets);
}

template <int BLOCK>
static grid16_fn grid16_pick(bool vals, int lev, int sets)
{
    return vals ? grid16_pick_lev<true, BLOCK>(lev, sets) : grid16_pick_lev<false, BLOCK>(lev, sets);
}

static int launch_grid16(const int32_t *xy, const int64_t *values, int64_t n, const sba_handle *h,
                         uint64_t *counts, int64_t *sums, hipStream_t st)
{
    Grid16 g{};
    g.ox = h->gi0 * h->s;
    g.oy = h->gj0 * h->s;
    g.extx = (uint32_t)(h->gw * h->s);
    g.exty = (uint32_t)(h->gh * h->s);
    g.mag = h->mag;
    g.shift = h->shift;
    // shift >= 32 (s >= 2): floor(floor(n m / 2^32) / 2^(shift-32)); shift 31
    // (s = 1, m = 2^31): mul_hi(2n, 2^31) = n
    g.pre = h->shift >= 32 ? 0u : 1u;
    g.post = h->shift >= 32 ? (uint32_t)(h->shift - 32) : 0u;
    g.tl = h->tile_log2;
    g.sl = h->sub_log2;
    g.tw = (uint32_t)h->tw;
    g.nt16 = (uint32_t)(((h->tw * h->th) + 7) & ~(int64_t)7);
    g.dir16 = h->dir16;
    g.sub = h->sub;
    g.blocks16 = h->blocks16;
    g.np = (uint32_t)h->n_polys;
    const Grid16Plan pl = grid16_plan(h);
    const size_t lds = pl.lds;
    g.sets = (uint32_t)pl.sets;
    g.n_ids = (uint32_t)h->n_set_ids;
    g.nsub = pl.nsub;
    g.nsub16 = pl.nsub16;
    Agg A{h->set_off, h->set_ids, (uint32_t)h->n_polys, (uint32_t)h->n_sets};
    const int32_t np = h->n_polys;
    const bool vals = values != nullptr && sums != nullptr;
    int block = 0, per_cu = 0;
    grid16_shape(lds, &block, &per_cu);
    const int64_t npairs = n >> 1;
    int64_t nb = std::min<int64_t>((npairs + block - 1) / block, (int64_t)cu_count() * per_cu);
    // the kernel's byte offsets inside a trip (16 B x PROBE_UNROLL pairs per
    // lane of the grid) are 32-bit
    nb = std::min<int64_t>(nb, ((int64_t)1 << 26) / ((int64_t)block * PROBE_UNROLL));
    if (nb < 1) nb = 1;
    grid16_fn kern = block == 512 ? grid16_pick<512>(vals, pl.lev, pl.sets)
                                  : grid16_pick<1024>(vals, pl.lev, pl.sets);
    // dynamic LDS above 64 KB has to be allowed explicitly
    (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_zero_out, dim3(grid_for(np)), dim3(256), 0, st, counts,
                       vals ? sums : nullptr, np);
    hipLaunchKernelGGL(kern, dim3((unsigned)nb), dim3(block), lds, st, (const int4 *)xy,
                       (const longlong2 *)values, xy, values, n, g, A, counts, sums);
    return hipGetLastError() != hipSuccess ? SBA_EDEVICE : 0;
}

// ---------------------------------------------------------------- result range in one pass
//
// The full approximation A(P) and the boundary-only B(P) of the same
// polygons, stored on the same tiles, probed together (Sec. 6: alpha and the
// boundary partial beta in one pass over the points): each point's cell is
// computed once and looked up in both directories (both staged in LDS), and
// each handle has its own LDS bins (polygons, then sets, expanded once per
// workgroup).

template <bool VALS>
__device__ __forceinline__ void expand_set_bins(uint32_t *cnt, unsigned long long *sum,
                                                uint32_t np, const Agg &A, int block)
{
    for (uint32_t k = threadIdx.x; k < A.n_sets; k += block) {
        uint32_t c = cnt[np + k];
        if (c == 0) continue;
        unsigned long long sv = VALS ? sum[np + k] : 0ull;
        for (int64_t t = A.set_off[k], e = A.set_off[k + 1]; t < e; t++) {
            uint32_t p = (uint32_t)A.set_ids[t];
            if (p >= np) continue;
            atomicAdd(&cnt[p], c);
            if (VALS) atomicAdd(&sum[p], sv);
        }
    }
}

template <bool VALS, bool SUB, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_probe_range16(
    const int4 *__restrict__ xy4, const longlong2 *__restrict__ v2, const int32_t *__restrict__ xy,
    const int64_t *__restrict__ vals, int64_t n, Grid16 ga, Grid16 gb, Agg A, Agg B,
    uint64_t *__restrict__ counts, int64_t *__restrict__ sums, uint64_t *__restrict__ bcounts,
    int64_t *__restrict__ bsums)
{
    // LDS: directory A, directory B (each nt16 u16, a multiple of 8), sums A,
    // sums B (u64), counts A, counts B (u32)
    extern __shared__ unsigned long long smem[];
    const uint32_t np = ga.np;
    const uint32_t nba = np + A.n_sets, nbb = np + B.n_sets;
    uint16_t *dira = (uint16_t *)smem, *dirb = dira + ga.nt16;
    Lds16 La, Lb;
    La.dir = dira;
    Lb.dir = dirb;
    La.sum = smem + (ga.nt16 + gb.nt16) / 4;
    Lb.sum = La.sum + nba;
    La.cnt = (uint32_t *)(Lb.sum + nbb);
    Lb.cnt = La.cnt + nba;
    La.soff = La.sids = Lb.soff = Lb.sids = nullptr;
    {
        const uint4 *src = (const uint4 *)ga.dir16;
        uint4 *dst = (uint4 *)dira;
        for (uint32_t q = threadIdx.x; q < ga.nt16 / 8; q += BLOCK) dst[q] = src[q];
        src = (const uint4 *)gb.dir16;
        dst = (uint4 *)dirb;
        for (uint32_t q = threadIdx.x; q < gb.nt16 / 8; q += BLOCK) dst[q] = src[q];
        for (uint32_t p = threadIdx.x; p < nba; p += BLOCK) {
            La.cnt[p] = 0;
            La.sum[p] = 0;
        }
        for (uint32_t p = threadIdx.x; p < nbb; p += BLOCK) {
            Lb.cnt[p] = 0;
            Lb.sum[p] = 0;
        }
    }
    __syncthreads();
    const int qs = ga.tl - ga.sl;
    const int fl = SUB ? ga.sl : ga.tl;
    const uint32_t m = (1u << fl) - 1u, mq = (1u << qs) - 1u;
    const int64_t npairs = n >> 1;
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    const int64_t tlast = npairs - 1;
    const uint32_t ox = (uint32_t)ga.ox, oy = (uint32_t)ga.oy;
    for (int64_t t0 = (int64_t)blockIdx.x * BLOCK + threadIdx.x; t0 < npairs;
         t0 += stride * PROBE_UNROLL) {
        v4i_t q[PROBE_UNROLL];
        v2l_t vv[PROBE_UNROLL];
        bool in[PROBE_UNROLL];
#pragma unroll
        for (int u = 0; u < PROBE_UNROLL; u++) {
            int64_t t = t0 + (int64_t)u * stride;
            in[u] = t < npairs;
            int64_t tc = in[u] ? t : tlast;
            q[u] = __builtin_nontemporal_load((const v4i_t *)(xy4 + tc));
            vv[u] = VALS ? __builtin_nontemporal_load((const v2l_t *)(v2 + tc)) : v2l_t{0, 0};
        }
        uint32_t ea[2 * PROBE_UNROLL], eb[2 * PROBE_UNROLL], lo[2 * PROBE_UNROLL],
            sq[2 * PROBE_UNROLL];
#pragma unroll
        for (int k = 0; k < 2 * PROBE_UNROLL; k++) {
            int32_t x = (k & 1) ? q[k >> 1].z : q[k >> 1].x;
            int32_t y = (k & 1) ? q[k >> 1].w : q[k >> 1].y;
            uint32_t dx = (uint32_t)x - ox, dy = (uint32_t)y - oy;
            bool ok = in[k >> 1] && dx < ga.extx && dy < ga.exty;
            uint32_t i = __umulhi((ok ? dx : 0u) << ga.pre, ga.mag) >> ga.post;
            uint32_t j = __umulhi((ok ? dy : 0u) << ga.pre, ga.mag) >> ga.post;
            const uint32_t te = (j >> ga.tl) * ga.tw + (i >> ga.tl);
            ea[k] = ok ? dira[te] : 0u;
            eb[k] = ok ? dirb[te] : 0u;
            lo[k] = ((j & m) << fl) | (i & m);
            if (SUB) sq[k] = (((j >> ga.sl) & mq) << qs) | ((i >> ga.sl) & mq);
        }
        // both handles, the same three levels as the single probe
        uint32_t fa[2 * PROBE_UNROLL], fbk[2 * PROBE_UNROLL], va[2 * PROBE_UNROLL],
            vb[2 * PROBE_UNROLL];
#pragma unroll
        for (int k = 0; k < 2 * PROBE_UNROLL; k++) {
            bool ma = (ea[k] & 0x8000u) != 0, mb = (eb[k] & 0x8000u) != 0;
            fa[k] = ma ? (ea[k] & 0x7fffu) : ~0u;
            va[k] = ma ? 0u : ea[k];
            fbk[k] = mb ? (eb[k] & 0x7fffu) : ~0u;
            vb[k] = mb ? 0u : eb[k];
        }
        if (SUB) {
            uint32_t sa[2 * PROBE_UNROLL], sb[2 * PROBE_UNROLL];
#pragma unroll
            for (int k = 0; k < 2 * PROBE_UNROLL; k++) {
                sa[k] = ga.sub[fa[k] != ~0u ? ((uint64_t)fa[k] << (2 * qs)) + sq[k] : 0];
                sb[k] = gb.sub[fbk[k] != ~0u ? ((uint64_t)fbk[k] << (2 * qs)) + sq[k] : 0];
            }
#pragma unroll
            for (int k = 0; k < 2 * PROBE_UNROLL; k++) {
                if (fa[k] != ~0u) {
                    bool mx = (sa[k] & TILE_MIXED) != 0;
                    va[k] = mx ? 0u : sa[k];
                    fa[k] = mx ? (sa[k] & ~TILE_MIXED) : ~0u;
                }
                if (fbk[k] != ~0u) {
                    bool mx = (sb[k] & TILE_MIXED) != 0;
                    vb[k] = mx ? 0u : sb[k];
                    fbk[k] = mx ? (sb[k] & ~TILE_MIXED) : ~0u;
                }
            }
        }
        uint32_t ca[2 * PROBE_UNROLL], cb[2 * PROBE_UNROLL];
#pragma unroll
        for (int k = 0; k < 2 * PROBE_UNROLL; k++) {
            ca[k] = ga.blocks16[fa[k] != ~0u ? ((uint64_t)fa[k] << (2 * fl)) + lo[k] : 0];
            cb[k] = gb.blocks16[fbk[k] != ~0u ? ((uint64_t)fbk[k] << (2 * fl)) + lo[k] : 0];
        }
#pragma unroll
        for (int k = 0; k < 2 * PROBE_UNROLL; k++) {
            const int64_t v = (k & 1) ? vv[k >> 1].y : vv[k >> 1].x;
            add_short<VALS, SETS_BINS>(fa[k] != ~0u ? ca[k] : va[k], v, A, np, La);
            add_short<VALS, SETS_BINS>(fbk[k] != ~0u ? cb[k] : vb[k], v, B, np, Lb);
        }
    }
    if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
        int64_t k = n - 1;
        const int64_t v = VALS ? vals[k] : 0;
        add_short<VALS, SETS_BINS>(grid16_code<SUB>(ga, dira, xy[2 * k], xy[2 * k + 1]), v, A, np,
                                   La);
        add_short<VALS, SETS_BINS>(grid16_code<SUB>(gb, dirb, xy[2 * k], xy[2 * k + 1]), v, B, np,
                                   Lb);
    }
    __syncthreads();
    expand_set_bins<VALS>(La.cnt, La.sum, np, A, BLOCK);
    expand_set_bins<VALS>(Lb.cnt, Lb.sum, np, B, BLOCK);
    __syncthreads();
    flush_bins<VALS>(La.cnt, La.sum, np, BLOCK, counts, sums);
    flush_bins<VALS>(Lb.cnt, Lb.sum, np, BLOCK, bcounts, bsums);
}

static Grid16 grid16_of(const sba_handle *h)
{
    Grid16 g{};
    g.ox = h->gi0 * h->s;
    g.oy = h->gj0 * h->s;
    g.extx = (uint32_t)(h->gw * h->s);
    g.exty = (uint32_t)(h->gh * h->s);
    g.mag = h->mag;
    g.shift = h->shift;
    g.pre = h->shift >= 32 ? 0u : 1u;
    g.post = h->shift >= 32 ? (uint32_t)(h->shift - 32) : 0u;
    g.tl = h->tile_log2;
    g.sl = h->sub_log2;
    g.tw = (uint32_t)h->tw;
    g.nt16 = (uint32_t)(((h->tw * h->th) + 7) & ~(int64_t)7);
    g.dir16 = h->dir16;
    g.sub = h->sub;
    g.blocks16 = h->blocks16;
    g.np = (uint32_t)h->n_polys;
    g.sets = SETS_BINS;
    g.n_ids = (uint32_t)h->n_set_ids;
    return g;
}

// LDS bytes of the one-pass range probe, or 0 when the two handles cannot
// share it (different grids, 32-bit format, too large for LDS)
static size_t range_lds(const sba_handle *h, const sba_handle *hb)
{
    if (h->kind != SBA_KIND_GRID || hb->kind != SBA_KIND_GRID || !h->compact || !hb->compact)
        return 0;
    if (h->s != hb->s || h->gi0 != hb->gi0 || h->gj0 != hb->gj0 || h->gw != hb->gw ||
        h->gh != hb->gh || h->tile_log2 != hb->tile_log2 || h->sub_log2 != hb->sub_log2 ||
        h->n_polys != hb->n_polys || h->gw == 0)
        return 0;
    const size_t lds = grid16_dir_lds(h) + grid16_dir_lds(hb) +
                       ((size_t)2 * h->n_polys + h->n_sets + hb->n_sets) * 12;
    return lds <= GRID16_LDS_MAX ? lds : 0;
}

typedef void (*range16_fn)(const int4 *, const longlong2 *, const int32_t *, const int64_t *,
                           int64_t, Grid16, Grid16, Agg, Agg, uint64_t *, int64_t *, uint64_t *,
                           int64_t *);

template <int BLOCK>
static range16_fn range16_pick(bool vals, bool sub)
{
    if (vals) return sub ? k_probe_range16<true, true, BLOCK> : k_probe_range16<true, false, BLOCK>;
    return sub ? k_probe_range16<false, true, BLOCK> : k_probe_range16<false, false, BLOCK>;
}

int range_launch(const int32_t *xy, const int64_t *values, int64_t n, const sba_handle *h,
                 const sba_handle *hb, uint64_t *counts, int64_t *sums, uint64_t *bcounts,
                 int64_t *bsums, hipStream_t st)
{
    const size_t lds = n > 0 && h->n_polys > 0 ? range_lds(h, hb) : 0;
    if (lds == 0) {  // two passes
        RC(probe_launch(xy, values, n, h, h->search, counts, sums, st));
        return probe_launch(xy, values, n, hb, hb->search, bcounts, bsums, st);
    }
    const Grid16 ga = grid16_of(h), gb = grid16_of(hb);
    Agg A{h->set_off, h->set_ids, (uint32_t)h->n_polys, (uint32_t)h->n_sets};
    Agg B{hb->set_off, hb->set_ids, (uint32_t)hb->n_polys, (uint32_t)hb->n_sets};
    const int32_t np = h->n_polys;
    const bool vals = values != nullptr && sums != nullptr && bsums != nullptr;
    const bool sub = h->sub_log2 < h->tile_log2;
    int block = 0, per_cu = 0;
    grid16_shape(lds, &block, &per_cu);
    const int64_t npairs = n >> 1;
    int64_t nb = std::min<int64_t>((npairs + block - 1) / block, (int64_t)cu_count() * per_cu);
    if (nb < 1) nb = 1;
    range16_fn kern = block == 512 ? range16_pick<512>(vals, sub) : range16_pick<1024>(vals, sub);
    (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_zero_out, dim3(grid_for(np)), dim3(256), 0, st, counts,
                       vals ? sums : nullptr, np);
    hipLaunchKernelGGL(k_zero_out, dim3(grid_for(np)), dim3(256), 0, st, bcounts,
                       vals ? bsums : nullptr, np);
    hipLaunchKernelGGL(kern, dim3((unsigned)nb), dim3(block), lds, st, (const int4 *)xy,
                       (const longlong2 *)values, xy, values, n, ga, gb, A, B, counts, sums,
                       bcounts, bsums);
    return hipGetLastError() != hipSuccess ? SBA_EDEVICE : 0;
}

int items_launch(const int32_t *xy, const int64_t *values, int64_t n, const sba_handle *h,
                 int32_t search, const PartRegions *regions, uint64_t *counts, int64_t *sums,
                 hipStream_t st)
{
    if (h->n_polys == 0) return 0;
    int layout = 0;
    if (h->kind == SBA_KIND_HILBERT) {
        if (search == SBA_SEARCH_LEARNED && !h->leaves) return SBA_EINVAL;
        layout = search == SBA_SEARCH_LEARNED ? 2 : 1;
    }
    return launch_items(xy, values, n, h, layout, true, counts, sums, st,
                        layout == 1 ? regions : nullptr);
}

// Name of the kernel a range call launches ("" when it takes two passes).
extern "C" const char *sba_range_kernel(const sba_handle *h, const sba_handle *hb, int with_values)
{
    static thread_local char buf[96];
    if (!h || !hb || h->n_polys == 0) return "";
    const size_t lds = range_lds(h, hb);
    if (lds == 0) return "";
    int block = 0, per_cu = 0;
    grid16_shape(lds, &block, &per_cu);
    snprintf(buf, sizeof(buf), "k_probe_range16<%s, %s, %d>", with_values ? "true" : "false",
             h->sub_log2 < h->tile_log2 ? "true" : "false", block);
    return buf;
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
    if (h->kind == SBA_KIND_GRID) {
        if (grid16_fits(h)) return launch_grid16(xy, values, n, h, counts, sums, st);
        return launch_layout<0>(xy, values, n, h, counts, sums, st);
    }
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

// Name of the kernel an aggregate call on h launches (as profilers print it,
// without arguments).
extern "C" const char *sba_probe_kernel(const sba_handle *h, int with_values)
{
    static thread_local char buf[96];
    if (!h || h->n_polys == 0) return "";
    const char *v = with_values ? "true" : "false";
    if (h->kind == SBA_KIND_GRID && grid16_fits(h)) {
        const Grid16Plan pl = grid16_plan(h);
        int block = 0, per_cu = 0;
        grid16_shape(pl.lds, &block, &per_cu);
        snprintf(buf, sizeof(buf), "k_probe_grid16<%s, %d, %d, %d>", v, pl.lev, pl.sets, block);
        return buf;
    }
    int layout = h->kind == SBA_KIND_GRID ? 0 : (h->search == SBA_SEARCH_LEARNED ? 2 : 1);
    if (h->n_polys <= LDS_MAX_POLYS)
        snprintf(buf, sizeof(buf), "k_probe_lds<%d, %s>", layout, v);
    else
        snprintf(buf, sizeof(buf), "k_probe_items<%d, %s, false>", layout, v);
    return buf;
}

// Learned run search over the cells of n points, counted: fb[0] = searches
// whose bracket check failed (full binary search taken), fb[1] = points whose
// learned answer differs from the binary search's.
__global__ void k_debug_learned(HilbView v, const int32_t *xy, int64_t n, unsigned long long *fb)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int64_t dx = (int64_t)xy[2 * t] - v.ox, dy = (int64_t)xy[2 * t + 1] - v.oy;
    if ((uint64_t)dx >= v.extx || (uint64_t)dy >= v.exty) return;
    const uint32_t i = divmagic((uint32_t)dx, v.mag, v.shift);
    const uint32_t j = divmagic((uint32_t)dy, v.mag, v.shift);
    const uint64_t key[1] = {hilbert_index(v.L, i, j)};
    const uint32_t k32[1] = {(uint32_t)key[0]};
    int64_t q[1], qb[1] = {0};
    learned_search_n<1>(v, k32, key, q, fb);
    pred_search_n<uint32_t, 1>(v.k32, qb, v.n, k32);
    if (q[0] != qb[0]) atomicAdd(&fb[1], 1ull);
}

extern "C" int sba_debug_learned_fallbacks(const sba_handle *h, const int32_t *xy, int64_t n,
                                           int64_t *fallbacks, int64_t *mismatches, void *stream)
{
    if (!h || n < 0 || (n > 0 && !xy) || !fallbacks || !mismatches) return SBA_EINVAL;
    *fallbacks = *mismatches = 0;
    if (h->kind != SBA_KIND_HILBERT || !h->leaves || !h->starts32) return SBA_EINVAL;
    if (n == 0 || h->n_runs == 0) return 0;
    hipStream_t st = (hipStream_t)stream;
    GridView g;
    HilbView hv;
    views(h, &g, &hv);
    Workspace ws(st);
    unsigned long long *fb = nullptr;
    RC(ws.alloc(&fb, 2));
    HIP_OK(hipMemsetAsync(fb, 0, 2 * sizeof(unsigned long long), st));
    hipLaunchKernelGGL(k_debug_learned, dim3(grid_for(n)), dim3(256), 0, st, hv, xy, n, fb);
    HIP_OK(hipGetLastError());
    unsigned long long hfb[2];
    RC(ws.read(hfb, fb, sizeof(hfb)));
    RC(ws.sync());
    *fallbacks = (int64_t)hfb[0];
    *mismatches = (int64_t)hfb[1];
    return 0;
}

extern "C" int sba_debug_grid16_lsub(int mode)
{
    if (mode != -1 && mode != 0) return SBA_EINVAL;
    g_grid16_lsub = mode;
    return 0;
}

extern "C" int sba_debug_grid16_sets(int mode)
{
    if (mode < -1 || mode > SETS_BINS) return SBA_EINVAL;
    g_grid16_sets = mode;
    return 0;
}

extern "C" int sba_debug_set_grid16_per_cu(int k)
{
    if (k < 0 || k > 4) return SBA_EINVAL;
    g_grid16_per_cu = k;
    return 0;
}

extern "C" int sba_debug_set_blocks_per_cu(int k)
{
    if (k < 1 || k > 64) return SBA_EINVAL;
    g_blocks_per_cu = k;
    return 0;
}

// ---------------------------------------------------------------- batches
//
// Serving: many aggregation tasks (each: a point range, a handle, an optional
// viewport, outputs) answered by one persistent launch.  The tasks' point
// ranges are cut into items of at most BATCH_ITEM points; workgroups pull
// items from a device counter until none is left, so uneven tasks balance
// across the chip.  An item aggregates into a table of the cell codes it
// meets in LDS and adds the table to the task's outputs with global atomics
// (a polygon set to each member); tasks that share outputs therefore
// accumulate into them.

#define BATCH_ITEM (1 << 18)
#define BATCH_PER_CU 4
#define ITEM_MIN 4096
#define ITEMS_PER_WG 8

struct TaskDev {
    GridView g;
    HilbView hv;
    Agg A;
    int32_t layout;        // 0 grid, 1 hilbert + binary, 2 hilbert + learned
    int32_t np;
    int64_t n;             // points (the items kernel's range is [0, n))
    const int32_t *xy;
    const int64_t *vals;
    int32_t filt;
    int32_t vx0, vy0, vx1, vy1;  // viewport [vx0, vx1] x [vy0, vy1] (inclusive)
    unsigned long long *counts;
    unsigned long long *sums;
    PartRegions reg;             // the items kernel over partitioned points (bq NULL: none)
};

struct ItemDev {
    int64_t lo, hi;
    int32_t task;
    int32_t pad;
};

__device__ __forceinline__ bool in_view(const TaskDev &T, int32_t x, int32_t y)
{
    return !T.filt || (x >= T.vx0 && x <= T.vx1 && y >= T.vy0 && y <= T.vy1);
}

// Per-workgroup table of the codes an item meets (polygon or polygon set,
// open addressing in LDS): the serving loop keeps its points bucketed, so the
// points of one item come from a small area and meet few codes; a code that
// finds no free slot within BATCH_PROBES steps goes to the outputs directly.
// The item probe's table has ITEM_SLOTS slots (its items may hold points
// in no order); the batch's has BATCH_SLOTS (bucketed points), which keeps
// a batch workgroup's LDS small enough for several per compute unit.
#define ITEM_SLOTS_LOG2 11
#define BATCH_SLOTS_LOG2 10
#define ITEM_SLOTS (1 << ITEM_SLOTS_LOG2)
#define BATCH_SLOTS (1 << BATCH_SLOTS_LOG2)
#define BATCH_PROBES 16
#define BATCH_EMPTY 0xffffffffu

struct CodeTable {
    uint32_t *key;                 // [2^bits] code or BATCH_EMPTY
    uint32_t *cnt;                 // [2^bits]
    unsigned long long *sum;       // [2^bits]
    int *full;                     // set once a code found no slot: later codes
                                   // look at one slot only (points in no
                                   // spatial order meet more codes than fit)
    int bits;
};

// n points of one code, v the sum of their values
template <bool VALS>
__device__ __forceinline__ void table_add(const CodeTable &H, uint32_t code, int64_t v,
                                          const TaskDev &T, uint32_t n = 1)
{
    if (code == 0) return;
    uint32_t h = (code * 2654435761u) >> (32 - H.bits);
    const uint32_t mask = (1u << H.bits) - 1u;
    const int probes = *H.full ? 1 : BATCH_PROBES;
    for (int k = 0; k < probes; k++) {
        uint32_t old = H.key[h];
        if (old == BATCH_EMPTY) old = atomicCAS(&H.key[h], BATCH_EMPTY, code);
        if (old == BATCH_EMPTY || old == code) {
            atomicAdd(&H.cnt[h], n);
            if (VALS) atomicAdd(&H.sum[h], (unsigned long long)v);
            return;
        }
        h = (h + 1) & mask;
    }
    if (probes > 1) *H.full = 1;
    add_global<VALS>(code, v, T.A, T.counts, T.sums, n);
}

// FMT (grid layout): the handle's format, as for grid_codes; FULL: as for
// the learned search
template <int LAYOUT, bool VALS, int FMT = 0, bool FULL = false>
__device__ __forceinline__ void batch_item(const TaskDev &T, int64_t lo, int64_t hi,
                                           const CodeTable &H)
{
    auto one = [&](int32_t x, int32_t y, int64_t v) {
        if (!in_view(T, x, y)) return;
        table_add<VALS>(H, code_of<LAYOUT>(T.g, T.hv, x, y), v, T);
    };
    // ragged ends one point at a time, the aligned middle two points per load
    int64_t a = lo, b = hi;
    if ((a & 1) && a < b) {
        if (threadIdx.x == 0) one(T.xy[2 * a], T.xy[2 * a + 1], VALS ? T.vals[a] : 0);
        a++;
    }
    if ((b & 1) && b > a) {
        if (threadIdx.x == 0) one(T.xy[2 * (b - 1)], T.xy[2 * (b - 1) + 1], VALS ? T.vals[b - 1] : 0);
        b--;
    }
    const int4 *xy4 = (const int4 *)T.xy;
    const longlong2 *v2 = (const longlong2 *)T.vals;
    const int64_t pb = b >> 1;
    // Each wave takes blocks of 64 PROBE_UNROLL consecutive pairs (the
    // waves of the workgroup in turn), so the points of one wave's trip are
    // neighbours in the input, and in space when the input is in spatial
    // order.  The lanes of a wave leave the loop together (the lookups work
    // across the wave): a wave runs while its block starts before the end,
    // and lanes past the end take a point no cell holds.
    constexpr int64_t WB = 64 * PROBE_UNROLL;
    const int64_t nw = PROBE_BLOCK / 64;
    const int64_t lane = (int64_t)(threadIdx.x & 63u);
    for (int64_t w0 = (a >> 1) + (int64_t)(threadIdx.x >> 6) * WB; w0 < pb; w0 += nw * WB) {
        int4 q[PROBE_UNROLL];
        longlong2 vv[PROBE_UNROLL];
#pragma unroll
        for (int u = 0; u < PROBE_UNROLL; u++) {
            int64_t t = w0 + (int64_t)u * 64 + lane;
            q[u] = t < pb ? gld(xy4 + t) : make_int4(INT32_MIN, INT32_MIN, INT32_MIN, INT32_MIN);
            vv[u] = (VALS && t < pb) ? gld(v2 + t) : make_longlong2(0, 0);
        }
        // points outside the viewport become a coordinate no cell holds
        int32_t xs[2 * PROBE_UNROLL], ys[2 * PROBE_UNROLL];
#pragma unroll
        for (int u = 0; u < PROBE_UNROLL; u++) {
            bool k0 = in_view(T, q[u].x, q[u].y), k1 = in_view(T, q[u].z, q[u].w);
            xs[2 * u] = k0 ? q[u].x : INT32_MIN;
            ys[2 * u] = k0 ? q[u].y : INT32_MIN;
            xs[2 * u + 1] = k1 ? q[u].z : INT32_MIN;
            ys[2 * u + 1] = k1 ? q[u].w : INT32_MIN;
        }
        uint32_t c[2 * PROBE_UNROLL];
        if (LAYOUT == 0)
            grid_codes<2 * PROBE_UNROLL, FMT>(T.g, xs, ys, c);
        else
            codes_of_wave<LAYOUT, 2 * PROBE_UNROLL, FULL>(T.g, T.hv, xs, ys, c);
        // a lane's points of the trip (pairs 64 apart) often share their code
        // when the input is in spatial order: runs of one code take one add
        uint32_t cur = c[0], run = 1;
        int64_t rs = vv[0].x;
#pragma unroll
        for (int k = 1; k < 2 * PROBE_UNROLL; k++) {
            const int64_t v = (k & 1) ? vv[k >> 1].y : vv[k >> 1].x;
            if (c[k] == cur) {
                run++;
                rs += v;
            } else {
                table_add<VALS>(H, cur, rs, T, run);
                cur = c[k];
                run = 1;
                rs = v;
            }
        }
        table_add<VALS>(H, cur, rs, T, run);
    }
}

// the item's codes to the task's outputs (sets to each member), and the
// table back to empty
__device__ __forceinline__ void table_flush(const CodeTable &H, const TaskDev &T, bool vals)
{
    for (int k = threadIdx.x; k < (1 << H.bits); k += PROBE_BLOCK) {
        const uint32_t code = H.key[k];
        if (code == BATCH_EMPTY) continue;
        const unsigned long long c = H.cnt[k], sv = H.sum[k];
        H.key[k] = BATCH_EMPTY;
        H.cnt[k] = 0;
        H.sum[k] = 0;
        if (c == 0) continue;
        if (code < CODE_SET_BASE) {
            const uint32_t p = code - 1u;
            if (p >= T.A.np) continue;
            gadd(&T.counts[p], c);
            if (vals) gadd(&T.sums[p], sv);
        } else {
            const uint32_t ks = code - CODE_SET_BASE;
            if (ks >= T.A.n_sets) continue;
            for (int64_t t = gld(T.A.set_off + ks), e = gld(T.A.set_off + ks + 1); t < e; t++) {
                const uint32_t p = (uint32_t)gld(T.A.set_ids + t);
                if (p >= T.A.np) continue;
                gadd(&T.counts[p], c);
                if (vals) gadd(&T.sums[p], sv);
            }
        }
    }
    if (threadIdx.x == 0) *H.full = 0;
}

// One aggregate over all points when the polygon count is too large for
// per-polygon LDS bins: workgroups take contiguous items (round robin, so
// no counter is needed) and count each in the LDS table of cell codes; points
// in spatial order (bucketed, Hilbert-sorted) meet few codes per item and
// almost never reach global memory, points in no order fall back to a global
// atomic per point once the table is full.
// Items are dealt to the chip's 8 XCDs in contiguous eighths (workgroup b
// runs on XCD b mod 8, the dispatcher's round robin), so the points the
// workgroups of one XCD hold at a time come from one stretch of the input:
// for spatially ordered or partitioned points, one region whose part of the
// structure fits that XCD's L2.  The grid size is a multiple of 8.
// The region of a partitioned item [lo, hi): the buckets of its first and
// last points, the runs that hold their keys, and every S-th start of those
// runs in LDS (S the smallest step that fits ITEM_SAMPLES of them).  Every
// thread of the workgroup calls it; it returns after a barrier.
#define ITEM_SAMPLES 4096
__device__ __forceinline__ void stage_region(const TaskDev &T, int64_t lo, int64_t hi,
                                             uint32_t *samp, int32_t *reg)
{
    if (threadIdx.x == 0) {
        // last bucket b with start <= p: buckets may be empty, so this is
        // the bucket that holds point p
        auto bucket_of = [&](int64_t p) {
            int32_t b = 0, len = 256;
            while (len > 1) {
                const int32_t half = len >> 1;
                b = gld(T.reg.bstart + (int64_t)(b + half) * T.reg.bstride) <= p ? b + half : b;
                len -= half;
            }
            return b;
        };
        const int32_t b0 = bucket_of(lo), b1 = bucket_of(hi - 1);
        const int64_t q0 = gld(T.reg.bq + b0), q1 = gld(T.reg.bq + b1 + 1);
        const int64_t m = q1 - q0 + 1;
        const int64_t step = (m + ITEM_SAMPLES - 1) / ITEM_SAMPLES;
        reg[0] = (int32_t)q0;
        reg[1] = (int32_t)q1;
        reg[2] = (int32_t)step;
        reg[3] = (int32_t)((m + step - 1) / step);
    }
    __syncthreads();
    const int32_t q0 = reg[0], step = reg[2], ns = reg[3];
    for (int32_t j = threadIdx.x; j < ns; j += PROBE_BLOCK)
        samp[j] = gld(T.hv.k32 + q0 + (int64_t)j * step);
    __syncthreads();
}

// PART: the points come partitioned by region but in no order inside one
// (the partitioned probe): nearly every lookup takes the plain search,
// which keeps all its loads in flight per wave; otherwise the workgroup is
// held to 4 waves per SIMD worth of registers, which points in spatial
// order (bracketed lookups) turn into throughput.
template <int LAYOUT, bool VALS, bool PART>
__global__ __launch_bounds__(PROBE_BLOCK, PART ? 1 : 4) void k_probe_items(const TaskDev T0, int64_t item,
                                                             int64_t n_items)
{
    __shared__ uint32_t s_key[ITEM_SLOTS];
    __shared__ uint32_t s_cnt[ITEM_SLOTS];
    __shared__ unsigned long long s_sum[ITEM_SLOTS];
    __shared__ int s_full;
    __shared__ uint16_t s_htab[LAYOUT ? HILBERT_TAB : 1];
    constexpr bool REGIONS = PART && LAYOUT == 1;
    __shared__ uint32_t s_samp[REGIONS ? ITEM_SAMPLES : 1];
    __shared__ int32_t s_reg[4];
    const CodeTable H{s_key, s_cnt, s_sum, &s_full, ITEM_SLOTS_LOG2};
    for (int k = threadIdx.x; k < ITEM_SLOTS; k += PROBE_BLOCK) {
        s_key[k] = BATCH_EMPTY;
        s_cnt[k] = 0;
        s_sum[k] = 0;
    }
    if (threadIdx.x == 0) s_full = 0;
    TaskDev T = T0;
    if (LAYOUT) {
        hilbert_tab_fill(s_htab, PROBE_BLOCK);
        T.hv.tab = s_htab;
    }
    __syncthreads();
    const int64_t nx = gridDim.x >> 3, per = (n_items + 7) >> 3;
    const int64_t first = (int64_t)(blockIdx.x & 7) * per;
    const int64_t last = min(first + per, n_items);
    for (int64_t it = first + (blockIdx.x >> 3); it < last; it += nx) {
        const int64_t lo = it * item, hi = min(lo + item, T.n);
        if constexpr (REGIONS) {
            if (T.reg.bq) {
                stage_region(T, lo, hi, s_samp, s_reg);
                T.hv.samp = s_samp;
                T.hv.sq0 = s_reg[0];
                T.hv.sq1 = s_reg[1];
                T.hv.sS = s_reg[2];
                T.hv.sn = s_reg[3];
            }
        }
        batch_item<LAYOUT, VALS, 0, PART>(T, lo, hi, H);
        __syncthreads();
        table_flush(H, T, VALS);
        __syncthreads();
    }
}

static int launch_items(const int32_t *xy, const int64_t *values, int64_t n, const sba_handle *h,
                        int layout, bool part, uint64_t *counts, int64_t *sums, hipStream_t st,
                        const PartRegions *regions)
{
    const bool vals = values != nullptr && sums != nullptr;
    TaskDev T{};
    views(h, &T.g, &T.hv);
    T.A = Agg{h->set_off, h->set_ids, (uint32_t)h->n_polys, (uint32_t)h->n_sets};
    T.layout = layout;
    T.np = h->n_polys;
    T.n = n;
    T.xy = xy;
    T.vals = vals ? values : nullptr;
    T.counts = (unsigned long long *)counts;
    T.sums = vals ? (unsigned long long *)sums : nullptr;
    if (regions && layout == 1 && h->starts32) T.reg = *regions;
    // about ITEMS_PER_WG items per workgroup (even sizes keep the pairs
    // aligned), so the round robin ends evenly
    int64_t nb = std::max<int64_t>(
        1, std::min<int64_t>((n + ITEM_MIN - 1) / ITEM_MIN, (int64_t)cu_count() * g_blocks_per_cu));
    nb = (nb + 7) & ~(int64_t)7;  // whole rounds of the 8 XCDs
    int64_t item = (n + nb * ITEMS_PER_WG - 1) / (nb * ITEMS_PER_WG);
    item = std::max<int64_t>(ITEM_MIN, (item + 1) & ~(int64_t)1);
    const int64_t n_items = (n + item - 1) / item;
    hipLaunchKernelGGL(k_zero_out, dim3(grid_for(h->n_polys)), dim3(256), 0, st, counts,
                       vals ? sums : nullptr, h->n_polys);
    const dim3 grid((unsigned)nb);
#define ITEMS_CASE(L, V, P)                                                                        \
    hipLaunchKernelGGL((k_probe_items<L, V, P>), grid, dim3(PROBE_BLOCK), 0, st, T, item, n_items)
    switch (layout * 4 + (vals ? 2 : 0) + (part ? 1 : 0)) {
    case 0: ITEMS_CASE(0, false, false); break;
    case 1: ITEMS_CASE(0, false, true); break;
    case 2: ITEMS_CASE(0, true, false); break;
    case 3: ITEMS_CASE(0, true, true); break;
    case 4: ITEMS_CASE(1, false, false); break;
    case 5: ITEMS_CASE(1, false, true); break;
    case 6: ITEMS_CASE(1, true, false); break;
    case 7: ITEMS_CASE(1, true, true); break;
    case 8: ITEMS_CASE(2, false, false); break;
    case 9: ITEMS_CASE(2, false, true); break;
    case 10: ITEMS_CASE(2, true, false); break;
    default: ITEMS_CASE(2, true, true); break;
    }
#undef ITEMS_CASE
    HIP_OK(hipGetLastError());
    return 0;
}

// Items of one layout (each layout its own launch, so that the grid
// probe's workgroups are not sized by the Hilbert searches' registers).
template <int LAYOUT>
__global__ __launch_bounds__(PROBE_BLOCK, 4) void k_batch(const TaskDev *__restrict__ tasks,
                                                       const ItemDev *__restrict__ items,
                                                       int32_t n_items, int *__restrict__ next)
{
    __shared__ uint32_t s_key[BATCH_SLOTS];
    __shared__ uint32_t s_cnt[BATCH_SLOTS];
    __shared__ unsigned long long s_sum[BATCH_SLOTS];
    __shared__ int s_item, s_full;
    __shared__ uint16_t s_htab[LAYOUT ? HILBERT_TAB : 1];
    const CodeTable H{s_key, s_cnt, s_sum, &s_full, BATCH_SLOTS_LOG2};
    for (int k = threadIdx.x; k < BATCH_SLOTS; k += PROBE_BLOCK) {
        s_key[k] = BATCH_EMPTY;
        s_cnt[k] = 0;
        s_sum[k] = 0;
    }
    if (threadIdx.x == 0) s_full = 0;
    if (LAYOUT) hilbert_tab_fill(s_htab, PROBE_BLOCK);
    while (true) {
        if (threadIdx.x == 0) s_item = atomicAdd(next, 1);
        __syncthreads();
        const int it = s_item;
        __syncthreads();
        if (it >= n_items) break;  // every wave of the workgroup leaves here together
        const ItemDev I = items[it];
        TaskDev T = tasks[I.task];
        if (LAYOUT) T.hv.tab = s_htab;
        const bool vals = T.vals != nullptr && T.sums != nullptr;
        if constexpr (LAYOUT == 0) {
            // one code path per format keeps the other format's pointers out
            // of the registers
            const int f = T.g.compact ? 1 : 2;
            if (vals && f == 1) batch_item<0, true, 1>(T, I.lo, I.hi, H);
            else if (vals) batch_item<0, true, 2>(T, I.lo, I.hi, H);
            else if (f == 1) batch_item<0, false, 1>(T, I.lo, I.hi, H);
            else batch_item<0, false, 2>(T, I.lo, I.hi, H);
        } else {
            if (vals) batch_item<LAYOUT, true>(T, I.lo, I.hi, H);
            else batch_item<LAYOUT, false>(T, I.lo, I.hi, H);
        }
        __syncthreads();
        table_flush(H, T, vals);
        __syncthreads();
    }
}

// next: one item counter per layout
__global__ void k_batch_zero(const TaskDev *__restrict__ tasks, int32_t n_tasks, int *next)
{
    const int t = blockIdx.x;
    if (t == 0 && threadIdx.x < 3) next[threadIdx.x] = 0;
    if (t >= n_tasks) return;
    const TaskDev &T = tasks[t];
    for (int p = threadIdx.x; p < T.np; p += blockDim.x) {
        T.counts[p] = 0;
        if (T.sums) T.sums[p] = 0;
    }
}

// The tasks and items of a batch on the host (ItemDev ranges of at most
// BATCH_ITEM points), the items grouped by layout: n_layout[l] items of
// layout l, layout 0 first.
static void batch_prepare(const sba_task *tasks, int32_t n_tasks, std::vector<TaskDev> &td,
                          std::vector<ItemDev> &items, int64_t n_layout[3])
{
    td.assign(n_tasks, TaskDev{});
    items.clear();
    std::vector<ItemDev> by[3];
    for (int32_t k = 0; k < n_tasks; k++) {
        const sba_task &q = tasks[k];
        const sba_handle *h = q.h;
        TaskDev &T = td[k];
        views(h, &T.g, &T.hv);
        T.A = Agg{h->set_off, h->set_ids, (uint32_t)h->n_polys, (uint32_t)h->n_sets};
        T.layout = h->kind == SBA_KIND_GRID ? 0 : (q.search == SBA_SEARCH_LEARNED ? 2 : 1);
        T.np = h->n_polys;
        T.xy = q.xy;
        T.vals = q.values;
        T.filt = (q.vw > 0 && q.vh > 0) ? 1 : 0;
        // the last coordinate inside, clamped to the int32 coordinates
        T.vx0 = q.vx;
        T.vy0 = q.vy;
        T.vx1 = (int32_t)std::min<int64_t>((int64_t)q.vx + q.vw - 1, INT32_MAX);
        T.vy1 = (int32_t)std::min<int64_t>((int64_t)q.vy + q.vh - 1, INT32_MAX);
        T.counts = (unsigned long long *)q.counts;
        T.sums = (unsigned long long *)q.sums;
        for (int64_t a = q.lo; a < q.hi; a += BATCH_ITEM)
            by[T.layout].push_back(ItemDev{a, std::min<int64_t>(q.hi, a + BATCH_ITEM), k, 0});
    }
    for (int l = 0; l < 3; l++) {
        n_layout[l] = (int64_t)by[l].size();
        items.insert(items.end(), by[l].begin(), by[l].end());
    }
}

// bytes of device scratch a batch needs: tasks, items (+1), the item
// counters
static size_t batch_bytes(int32_t n_tasks, size_t n_items)
{
    return sizeof(TaskDev) * n_tasks + sizeof(ItemDev) * (n_items + 1) + 64;
}

// Copies the tasks and items into buf (batch_bytes long, device memory) and
// launches the batch on st.
static int batch_run(const std::vector<TaskDev> &td, const std::vector<ItemDev> &items,
                     const int64_t n_layout[3], char *buf, hipStream_t st)
{
    const int32_t n_tasks = (int32_t)td.size();
    const int32_t n_items = (int32_t)items.size();
    const size_t tbytes = sizeof(TaskDev) * n_tasks, ibytes = sizeof(ItemDev) * (n_items + 1);
    TaskDev *dtasks = (TaskDev *)buf;
    ItemDev *ditems = (ItemDev *)(buf + tbytes);
    int *next = (int *)(buf + tbytes + ibytes);
    if (hipMemcpyAsync(dtasks, td.data(), tbytes, hipMemcpyHostToDevice, st) != hipSuccess ||
        (n_items && hipMemcpyAsync(ditems, items.data(), sizeof(ItemDev) * n_items,
                                   hipMemcpyHostToDevice, st) != hipSuccess))
        return SBA_EDEVICE;
    // zeroes the outputs and the item counters
    hipLaunchKernelGGL(k_batch_zero, dim3((unsigned)n_tasks), dim3(256), 0, st, dtasks, n_tasks,
                       next);
    if (hipGetLastError() != hipSuccess) return SBA_EDEVICE;
    int64_t first = 0;
    for (int l = 0; l < 3; l++) {
        const int64_t ni = n_layout[l];
        if (ni == 0) continue;
        // at most BATCH_PER_CU persistent workgroups per CU (part of its LDS
        // and wave slots), so the builds of later queries, queued on other
        // streams, find room to run beside the batch
        const dim3 grid((unsigned)std::min<int64_t>(ni, (int64_t)cu_count() * BATCH_PER_CU));
        const ItemDev *it = ditems + first;
        if (l == 0)
            hipLaunchKernelGGL(k_batch<0>, grid, dim3(PROBE_BLOCK), 0, st, dtasks, it, (int32_t)ni,
                               next);
        else if (l == 1)
            hipLaunchKernelGGL(k_batch<1>, grid, dim3(PROBE_BLOCK), 0, st, dtasks, it, (int32_t)ni,
                               next + 1);
        else
            hipLaunchKernelGGL(k_batch<2>, grid, dim3(PROBE_BLOCK), 0, st, dtasks, it, (int32_t)ni,
                               next + 2);
        if (hipGetLastError() != hipSuccess) return SBA_EDEVICE;
        first += ni;
    }
    return first == n_items ? 0 : SBA_EDEVICE;
}

int batch_launch(const sba_task *tasks, int32_t n_tasks, hipStream_t st)
{
    if (n_tasks <= 0) return 0;
    std::vector<TaskDev> td;
    std::vector<ItemDev> items;
    int64_t n_layout[3];
    batch_prepare(tasks, n_tasks, td, items, n_layout);
    char *buf = nullptr;
    RC(tmp_alloc(&buf, (int64_t)batch_bytes(n_tasks, items.size()), st));
    const int rc = batch_run(td, items, n_layout, buf, st);
    tmp_free(buf, st);
    return rc;
}

// ---------------------------------------------------------------- batches without allocation
//
// The same batch with its tasks, items and counter in a fixed device array of
// the library (BATCH_SCRATCH_BYTES on every device it runs on, held until the
// process ends) instead of memory taken per call.  In host code the array's
// name does not stand for its device address: that address is looked up once
// per device (hipGetSymbolAddress, with the device current) and only the
// looked-up pointer is used.  Calls on one device share the array: calls
// that overlap on a device (different streams, or host threads) race.

#define BATCH_SCRATCH_BYTES (4u << 20)
static __device__ __align__(256) unsigned char batch_scratch[BATCH_SCRATCH_BYTES];

static int batch_scratch_ptr(char **out)
{
    constexpr int MAX_DEV = 64;
    static std::mutex mu;
    static char *ptr[MAX_DEV] = {};
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEV) {
        (void)hipGetLastError();
        return SBA_EDEVICE;
    }
    std::lock_guard<std::mutex> lk(mu);
    if (!ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(batch_scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return SBA_EDEVICE;
        }
        ptr[dev] = (char *)p;
    }
    *out = ptr[dev];
    return 0;
}

int batch_launch_noalloc(const sba_task *tasks, int32_t n_tasks, hipStream_t st)
{
    if (n_tasks <= 0) return 0;
    std::vector<TaskDev> td;
    std::vector<ItemDev> items;
    int64_t n_layout[3];
    batch_prepare(tasks, n_tasks, td, items, n_layout);
    if (batch_bytes(n_tasks, items.size()) > BATCH_SCRATCH_BYTES) return SBA_ELIMIT;
    char *buf = nullptr;
    RC(batch_scratch_ptr(&buf));
    return batch_run(td, items, n_layout, buf, st);
}

extern "C" size_t sba_batch_noalloc_bytes(void) { return BATCH_SCRATCH_BYTES; }

extern "C" int64_t sba_batch_scratch_bytes(const sba_task *tasks, int32_t n_tasks)
{
    if (n_tasks < 0 || (n_tasks > 0 && !tasks)) return -1;
    int64_t n_items = 0;
    for (int32_t k = 0; k < n_tasks; k++) {
        if (tasks[k].hi < tasks[k].lo) return -1;
        n_items += (tasks[k].hi - tasks[k].lo + BATCH_ITEM - 1) / BATCH_ITEM;
    }
    return (int64_t)batch_bytes(n_tasks, (size_t)n_items);
}

extern "C" int sba_debug_force_wide_grid(int on)
{
    g_build_wide = on != 0;
    return 0;
}
