// build.hip -- construction of the conservative eps-approximation on the GPU.
//
// Sec. 2.2 of the paper defines the approximation: cells of side
// eps/sqrt(2) along the boundary, every cell that touches the boundary kept
// (conservative raster), interior cells kept whole.  In integers, cell (i,j)
// is in A(P) when its closed square [is,(i+1)s]x[js,(j+1)s] meets an edge of
// P, or when it meets none and its corner (is,js) is inside P by the
// crossing-number rule.
//
// The build never visits a cell that is not on a boundary.  It works on
// rows of cells:
//   1. per edge and per row strip the edge touches: the closed x-range of the
//      edge inside the strip gives one interval of boundary cells;
//   2. per edge and per row line y = js it crosses (half-open rule): the
//      crossing's cell index k = ceil(xc/s); in order per (polygon, row), the
//      crossings pair up into the intervals [k1,k2), [k3,k4) ... of cells
//      whose corner is inside;
//   3. boundary intervals and crossings become events keyed (polygon, row,
//      x); one scan over them in key order yields each polygon's coverage
//      count, whose changes give its maximal covered intervals per row;
//   4. the distinct interval ends of a row cut it into pieces; each covered
//      interval adds its polygon to the pieces it spans, and the non-empty
//      pieces are the maximal row segments of constant polygon set;
//   5. sets of two or more polygons are deduplicated into a set table;
//   6. the segments are written into the chosen layout: a two-level tiled
//      grid (uniform tiles stored once in a directory, mixed tiles as fine
//      blocks) or, in hilbert.hip, the runs of the Hilbert order.
#include <atomic>
#include <chrono>
#include <vector>

#include "sba_internal.h"
#include "build_state.h"

// ---------------------------------------------------------------- kernels

// event kinds (payload of the (polygon, row, x) event keys)
#define EV_OPEN 0u   // first cell of a boundary interval
#define EV_CLOSE 1u  // one past the last cell of a boundary interval
#define EV_CROSS 2u  // crossing of the row line y = j s

__global__ void k_edges(const int32_t *ring_off, int32_t n_polys, const int64_t *vert_off,
                        int32_t n_rings, const int32_t *xy, int64_t n_verts, int4 *edges,
                        int32_t *epoly)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n_verts) return;
    int lo = 0, hi = n_rings;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (vert_off[mid] <= v) lo = mid + 1; else hi = mid;
    }
    int r = lo - 1;
    lo = 0;
    hi = n_polys;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (ring_off[mid] <= r) lo = mid + 1; else hi = mid;
    }
    int p = lo - 1;
    int64_t w = (v + 1 < vert_off[r + 1]) ? v + 1 : vert_off[r];
    edges[v] = make_int4(xy[2 * v], xy[2 * v + 1], xy[2 * w], xy[2 * w + 1]);
    epoly[v] = p;
}

// offsets: ring_off[0] = 0 and non-decreasing; sizes[0] = n_rings (err bit 2)
__global__ void k_check_rings(const int32_t *ring_off, int32_t n_polys, int64_t *sizes, int *err)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p > n_polys) return;
    if (p == 0 && ring_off[0] != 0) atomicOr(err, 2);
    if (p < n_polys && ring_off[p + 1] < ring_off[p]) atomicOr(err, 2);
    if (p == n_polys) sizes[0] = ring_off[n_polys];
}

// vert_off[0] = 0 and non-decreasing over the n_rings+1 entries; sizes[1] =
// n_verts.  Reads nothing if the ring offsets were already refused.
__global__ void k_check_verts(const int64_t *vert_off, int64_t *sizes, int *err)
{
    if (*err) return;
    const int64_t nr = sizes[0];
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r <= nr;
         r += (int64_t)gridDim.x * blockDim.x) {
        if (r == 0 && vert_off[0] != 0) atomicOr(err, 2);
        if (r < nr && vert_off[r + 1] < vert_off[r]) atomicOr(err, 2);
        if (r == nr) sizes[1] = vert_off[nr];
    }
}

// one wavefront per polygon: coordinate bounding box, range check (err bit
// 1), empty polygon (err bit 2); skipped when the offsets were refused
__global__ void k_poly_bbox(const int32_t *ring_off, const int64_t *vert_off, const int32_t *xy,
                            int32_t n_polys, int4 *bbox, int *err)
{
    int64_t gw = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    int lane = threadIdx.x & 63;
    if (gw >= n_polys || (*err & 2)) return;
    int p = (int)gw;
    int64_t v0 = vert_off[ring_off[p]], v1 = vert_off[ring_off[p + 1]];
    if (v1 == v0 && lane == 0) atomicOr(err, 2);
    int xmin = INT32_MAX, ymin = INT32_MAX, xmax = INT32_MIN, ymax = INT32_MIN;
    bool bad = false;
    for (int64_t v = v0 + lane; v < v1; v += 64) {
        int x = xy[2 * v], y = xy[2 * v + 1];
        bad |= (x <= -(1 << 30)) | (x >= (1 << 30)) | (y <= -(1 << 30)) | (y >= (1 << 30));
        xmin = min(xmin, x); ymin = min(ymin, y);
        xmax = max(xmax, x); ymax = max(ymax, y);
    }
    for (int o = 32; o > 0; o >>= 1) {
        xmin = min(xmin, __shfl_xor(xmin, o, 64));
        ymin = min(ymin, __shfl_xor(ymin, o, 64));
        xmax = max(xmax, __shfl_xor(xmax, o, 64));
        ymax = max(ymax, __shfl_xor(ymax, o, 64));
    }
    if (bad) atomicOr(err, 1);
    if (lane == 0) bbox[p] = make_int4(xmin, ymin, xmax, ymax);
}

// union of the polygons' cell boxes (one workgroup): box = {min over p of
// ceil(xmin/s) - 1, same for y, max over p of floor(xmax/s), same for y}.
// ceil and floor are monotone, so the extremes of the coordinates are found
// first and divided once.
#define BOX_BLOCK 256
__global__ __launch_bounds__(BOX_BLOCK) void k_union_box(const int4 *bbox, int32_t n_polys,
                                                         int64_t s, int64_t *box)
{
    __shared__ int32_t red[4][BOX_BLOCK / 64];
    int32_t v[4] = {INT32_MAX, INT32_MAX, INT32_MIN, INT32_MIN};
    for (int p = threadIdx.x; p < n_polys; p += BOX_BLOCK) {
        int4 b = bbox[p];
        v[0] = min(v[0], b.x);
        v[1] = min(v[1], b.y);
        v[2] = max(v[2], b.z);
        v[3] = max(v[3], b.w);
    }
    for (int o = 32; o > 0; o >>= 1) {
        v[0] = min(v[0], __shfl_xor(v[0], o, 64));
        v[1] = min(v[1], __shfl_xor(v[1], o, 64));
        v[2] = max(v[2], __shfl_xor(v[2], o, 64));
        v[3] = max(v[3], __shfl_xor(v[3], o, 64));
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int k = 0; k < 4; k++) red[k][w] = v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < BOX_BLOCK / 64; q++) {
            v[0] = min(v[0], red[0][q]);
            v[1] = min(v[1], red[1][q]);
            v[2] = max(v[2], red[2][q]);
            v[3] = max(v[3], red[3][q]);
        }
        box[0] = ceildiv64(v[0], s) - 1;
        box[1] = ceildiv64(v[1], s) - 1;
        box[2] = floordiv64(v[2], s);
        box[3] = floordiv64(v[3], s);
    }
}

// per edge: number of boundary row strips and of row-line crossings inside
// the stored box [gi0,gi1] x [gj0,gj1] (the box is the union of the cell
// boxes, cut by the clip window if there is one); polygons whose cell box
// misses the box in x contribute nothing inside it
__global__ void k_edge_counts(const int4 *edges, const int32_t *epoly, const int4 *bbox,
                              int64_t n_edges, int64_t s, int64_t gi0, int64_t gj0, int64_t gi1,
                              int64_t gj1, int centre, int64_t *nb, int64_t *nc)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_edges) return;
    int4 E = edges[e];
    int4 bb = bbox[epoly[e]];
    if (floordiv64(bb.z, s) < gi0 || ceildiv64(bb.x, s) - 1 > gi1) {
        nb[e] = 0;
        nc[e] = 0;
        return;
    }
    int64_t ey0 = min(E.y, E.w), ey1 = max(E.y, E.w);
    int64_t ja = max(ceildiv64(ey0, s) - 1, gj0), jb = min(floordiv64(ey1, s), gj1);
    nb[e] = jb >= ja ? jb - ja + 1 : 0;
    // row lines y = js (corners) or y = (j+1/2)s (centres) crossed under the
    // half-open rule: ey0 <= y < ey1
    int64_t ka, kb;
    if (centre) {
        ka = max(ceildiv64(2 * ey0 - s, 2 * s), gj0);
        kb = min(ceildiv64(2 * ey1 - s, 2 * s) - 1, gj1);
    } else {
        ka = max(ceildiv64(ey0, s), gj0);
        kb = min(ceildiv64(ey1, s) - 1, gj1);
    }
    nc[e] = (E.y != E.w && kb >= ka) ? kb - ka + 1 : 0;
}

__device__ __forceinline__ int64_t upper_bound_i64(const int64_t *a, int64_t n, int64_t v)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (a[mid] <= v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// boundary item t -> interval of cells [c0, c1] of row j touched by its edge,
// cut to the stored box, written as a start and an end event keyed
// (polygon, row, x) (an interval cut away entirely becomes an empty
// start/end pair at x = 0)
__global__ void k_emit_boundary(const int4 *edges, const int32_t *epoly, int64_t n_edges,
                                const int64_t *boff, int64_t nb_total, int64_t s, int64_t gi0,
                                int64_t gj0, int64_t gi1, int xbits, int rbits, uint64_t *evkey,
                                uint32_t *evpay)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nb_total) return;
    int64_t e = upper_bound_i64(boff, n_edges, t) - 1;
    int4 E = edges[e];
    int64_t x1 = E.x, y1 = E.y, x2 = E.z, y2 = E.w;
    int64_t ey0 = min(y1, y2), ey1 = max(y1, y2);
    int64_t j = max(ceildiv64(ey0, s) - 1, gj0) + (t - boff[e]);
    int64_t c0, c1;
    if (y1 == y2) {
        c0 = ceildiv64(min(x1, x2), s) - 1;
        c1 = floordiv64(max(x1, x2), s);
    } else {
        int64_t ya = max(ey0, j * s), yb = min(ey1, (j + 1) * s);
        int64_t den = y2 - y1;
        // x(y) = (x1*den + (y - y1)*(x2 - x1)) / den ; |numerator| < 2^63
        int64_t na = x1 * den + (ya - y1) * (x2 - x1);
        int64_t nbv = x1 * den + (yb - y1) * (x2 - x1);
        if (den < 0) { den = -den; na = -na; nbv = -nbv; }
        int64_t lo = min(na, nbv), hi = max(na, nbv);
        c0 = ceildiv64(lo, den * s) - 1;
        c1 = floordiv64(hi, den * s);
    }
    c0 = max(c0, gi0);
    c1 = min(c1, gi1);
    if (c0 > c1) { c0 = gi0; c1 = gi0 - 1; }
    uint64_t pr = ((uint64_t)epoly[e] << (rbits + xbits)) | ((uint64_t)(j - gj0) << xbits);
    evkey[2 * t] = pr | (uint64_t)(c0 - gi0);
    evpay[2 * t] = EV_OPEN;
    evkey[2 * t + 1] = pr | (uint64_t)(c1 + 1 - gi0);
    evpay[2 * t + 1] = EV_CLOSE;
}

// crossing item t -> event (polygon, row, k) with k = ceil(xc / s), k cut to
// [gi0, gi1 + 1] (inside spans are then cut to the stored box)
__global__ void k_emit_cross(const int4 *edges, const int32_t *epoly, int64_t n_edges,
                             const int64_t *coff, int64_t nc_total, int64_t s, int64_t gi0,
                             int64_t gj0, int64_t gi1, int centre, int xbits, int rbits,
                             uint64_t *evkey, uint32_t *evpay)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nc_total) return;
    int64_t e = upper_bound_i64(coff, n_edges, t) - 1;
    int4 E = edges[e];
    int64_t x1 = E.x, y1 = E.y, x2 = E.z, y2 = E.w;
    int64_t ey0 = min(y1, y2);
    int64_t den = y2 - y1, k;
    if (centre) {
        // centre line y = (j+1/2)s; with 2 xc = num / den the centre of cell i
        // lies left of the crossing iff (2i+1) s den < num (den > 0).  The
        // terms stay below 2^63 for coordinates under 2^30 in magnitude.
        int64_t j = max(ceildiv64(2 * ey0 - s, 2 * s), gj0) + (t - coff[e]);
        int64_t num = 2 * x1 * den + ((2 * j + 1) * s - 2 * y1) * (x2 - x1);
        if (den < 0) { den = -den; num = -num; }
        k = ceildiv64(num - s * den, 2 * s * den);
        k = min(max(k, gi0), gi1 + 1);
        evkey[t] = ((uint64_t)epoly[e] << (rbits + xbits)) | ((uint64_t)(j - gj0) << xbits) |
                   (uint64_t)(k - gi0);
        evpay[t] = EV_CROSS;
        return;
    }
    int64_t j = max(ceildiv64(ey0, s), gj0) + (t - coff[e]);
    int64_t num = x1 * den + (j * s - y1) * (x2 - x1);
    if (den < 0) { den = -den; num = -num; }
    k = ceildiv64(num, den * s);
    k = min(max(k, gi0), gi1 + 1);
    evkey[t] = ((uint64_t)epoly[e] << (rbits + xbits)) | ((uint64_t)(j - gj0) << xbits) |
               (uint64_t)(k - gi0);
    evpay[t] = EV_CROSS;
}

// ------------------------------------------------ events sorted per polygon
//
// The events come out of the emit kernels grouped by polygon (edges are
// numbered polygon by polygon): the boundary events of polygon p, in edge
// order, and further on its crossings.  Ordering them by (polygon, row, x)
// therefore only needs each polygon's events ordered by (row, x), which one
// workgroup does in LDS when the polygon has at most SEG_CAP events: the
// (row, x) key, re-based to the polygon's own row and column range, and the
// 2-bit kind packed in 32 bits, sorted by an LSD radix sort of 7-bit digits
// over the packed word (the order among events of equal (row, x) is not
// used: the coverage test reads only whole groups).  The
// polygon's sorted events land where a sort of all events by (polygon, row,
// x) puts them: after the events of the polygons before it.  The same
// workgroup then takes the coverage step for its polygon: the prefix sums of
// the event values over the polygon (the rows before any event are balanced:
// matched starts and ends, an even number of crossings, so this gives the
// same coverage as the prefix over all events), each (row, x) group's toggle
// flag, and the
// toggle's index among the polygon's toggles; a scan of the per-polygon
// toggle counts places every toggle.

#define SEG_BLOCK 1024
#define SEG_ROUNDS 16
#define SEG_CAP (SEG_BLOCK * SEG_ROUNDS)
#define SEG_DBITS 7
#define SEG_RADIX (1 << SEG_DBITS)
#define SEG_WAVES (SEG_BLOCK / 64)

struct EventSegs {
    const int32_t *ring_off;
    const int64_t *vert_off;
    const int64_t *boff, *coff;  // exclusive scans of the per-edge boundary items and crossings
    const int64_t *tot;          // tot[0], tot[1]: their totals
    int64_t nv;                  // edges
    int use_b, use_c;            // boundary events / crossings among the sorted events
    int64_t cbase;               // where the crossings start in the event arrays
};

// polygon p: its sorted events' first input slot of each kind, their counts,
// and its first output slot
__device__ __forceinline__ void event_seg(const EventSegs &S, int p, int64_t *ib, int64_t *nbv,
                                          int64_t *ic, int64_t *ncv, int64_t *o0)
{
    const int64_t e0 = S.vert_off[S.ring_off[p]], e1 = S.vert_off[S.ring_off[p + 1]];
    const int64_t b0 = e0 < S.nv ? S.boff[e0] : S.tot[0], b1 = e1 < S.nv ? S.boff[e1] : S.tot[0];
    const int64_t c0 = e0 < S.nv ? S.coff[e0] : S.tot[1], c1 = e1 < S.nv ? S.coff[e1] : S.tot[1];
    *ib = 2 * b0;
    *nbv = S.use_b ? 2 * (b1 - b0) : 0;
    *ic = S.cbase + c0;
    *ncv = S.use_c ? c1 - c0 : 0;
    *o0 = (S.use_b ? 2 * b0 : 0) + (S.use_c ? c0 : 0);
}

// the largest polygon's event count, into *mx (zeroed before); also zeroes
// the per-row toggle counters rowcnt[0..gh]
__global__ void k_event_seg_max(EventSegs S, int32_t np, unsigned long long *mx,
                                unsigned long long *rowcnt, int64_t gh)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t <= gh) rowcnt[t] = 0;
    const int p = (int)t;
    if (t >= np) return;
    int64_t ib, nbv, ic, ncv, o0;
    event_seg(S, p, &ib, &nbv, &ic, &ncv, &o0);
    atomicMax(mx, (unsigned long long)(nbv + ncv));
}

// exclusive scan across a workgroup of SEG_BLOCK lanes (wsum: SEG_WAVES words)
__device__ __forceinline__ uint32_t seg_excl_scan(uint32_t v, uint32_t *wsum)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t u = (uint32_t)__shfl_up((int)incl, o, 64);
        if (lane >= o) incl += u;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    uint32_t before = 0;
    for (int k = 0; k < w; k++) before += wsum[k];
    __syncthreads();
    return before + incl - v;
}

// event value in 32 bits: starts and ends add +1 / -1 to the count of open
// boundary intervals (bits 0-30, at most the polygon's event count), a
// crossing flips bit 31 (the parity of the crossings so far)
__device__ __forceinline__ uint32_t ev_word(uint32_t kind)
{
    return kind == EV_CROSS ? 0x80000000u : (kind == EV_OPEN ? 1u : 0xffffffffu);
}

__device__ __forceinline__ uint32_t cov_of(uint32_t P) { return (P & 0x7fffffffu) + (P >> 31); }

// Stable LSD radix sort, by one workgroup of SEG_BLOCK lanes, of n <= SEG_CAP
// 32-bit words in LDS by their bits [0, kbits): 7-bit digits; wave w ranks
// its own rpw x 64 consecutive words (rpw = the fewest rounds that spread
// the words over every wave), 64 at a time, equal digits finding each other
// with SEG_DBITS ballots.  The words end in *src (the two buffers swap once
// per pass); wcnt holds SEG_WAVES x SEG_RADIX counters.
__device__ __forceinline__ void lds_radix_u32(uint32_t *&src, uint32_t *&dst, int n, int kbits,
                                              uint32_t *wcnt, uint32_t *doff, uint32_t *wtot)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    const int rpw = (n + SEG_BLOCK - 1) / SEG_BLOCK;  // <= SEG_ROUNDS
    const int wbase = w * 64 * rpw;
    for (int shift = 0; shift < kbits; shift += SEG_DBITS) {
        for (int k = threadIdx.x; k < SEG_WAVES * SEG_RADIX; k += SEG_BLOCK) wcnt[k] = 0;
        __syncthreads();
        // wave w ranks its own rpw x 64 consecutive words, 64 at a time:
        // equal digits find each other with SEG_DBITS ballots, so the order
        // is stable
        uint32_t kk[SEG_ROUNDS], loc[SEG_ROUNDS];
#pragma unroll
        for (int q = 0; q < SEG_ROUNDS; q++) {
            // rounds past the wave's share or past the words are skipped
            // (uniform per wave)
            if (q >= rpw || wbase + q * 64 >= n) break;
            const int idx = wbase + q * 64 + lane;
            const bool valid = idx < n;
            const uint32_t key = valid ? src[idx] : 0u;
            kk[q] = key;
            const uint32_t d = (key >> shift) & (SEG_RADIX - 1);
            uint64_t peers = __ballot(valid);
#pragma unroll
            for (int b = 0; b < SEG_DBITS; b++) {
                const uint64_t bal = __ballot((d >> b) & 1u);
                peers &= ((d >> b) & 1u) ? bal : ~bal;
            }
            const uint32_t old = wcnt[w * SEG_RADIX + d];
            loc[q] = old + (uint32_t)__popcll(peers & lt);
            __builtin_amdgcn_wave_barrier();
            if (valid && (peers & lt) == 0) wcnt[w * SEG_RADIX + d] = old + (uint32_t)__popcll(peers);
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();
        // digit d = threadIdx.x: offsets of the waves within the digit, then
        // the digit's first slot
        uint32_t run = 0, incl = 0;
        if (threadIdx.x < SEG_RADIX) {
            const int d = threadIdx.x;
#pragma unroll
            for (int k = 0; k < SEG_WAVES; k++) {
                const uint32_t c = wcnt[k * SEG_RADIX + d];
                wcnt[k * SEG_RADIX + d] = run;
                run += c;
            }
            incl = run;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t u = (uint32_t)__shfl_up((int)incl, o, 64);
                if (lane >= o) incl += u;
            }
            if (lane == 63) wtot[w] = incl;
        }
        __syncthreads();
        if (threadIdx.x < SEG_RADIX) {
            uint32_t before = 0;
            for (int k = 0; k < w; k++) before += wtot[k];
            doff[threadIdx.x] = before + incl - run;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < SEG_ROUNDS; q++) {
            const int idx = wbase + q * 64 + lane;
            if (q < rpw && idx < n) {
                const uint32_t d = (kk[q] >> shift) & (SEG_RADIX - 1);
                dst[doff[d] + wcnt[w * SEG_RADIX + d] + loc[q]] = kk[q];
            }
        }
        __syncthreads();
        uint32_t *t = src;
        src = dst;
        dst = t;
    }
}

// one workgroup per polygon; dynamic LDS: two buffers of `cap` words (the
// largest polygon's event count rounded up to whole waves' rounds, at most
// SEG_CAP) and the per-wave digit counts.  Out: the sorted events (kind in
// bits 0-1 of opay, bit 2 set on a toggle), each event's index among the
// polygon's toggles before it (otl), the polygon's toggle count (ptot[p]),
// and error bit 2 when a row ends inside the polygon
__global__ __launch_bounds__(SEG_BLOCK) void k_event_seg_sort(EventSegs S, const uint64_t *evkey,
                                                              const uint32_t *evpay, int rxbits,
                                                              int xbits, int cap, uint64_t *okey,
                                                              uint32_t *opay, int32_t *otl,
                                                              int64_t *ptot, int *err,
                                                              unsigned long long *rowcnt)
{
    extern __shared__ uint32_t seg_lds[];
    uint32_t *src = seg_lds, *dst = seg_lds + cap;
    uint32_t *wcnt = seg_lds + 2 * cap;  // [SEG_WAVES][SEG_RADIX]
    __shared__ uint32_t doff[SEG_RADIX];
    __shared__ uint32_t wtot[SEG_RADIX / 64];
    __shared__ uint32_t wsum[SEG_WAVES];
    const int p = blockIdx.x;
    int64_t ib, nbv, ic, ncv, o0;
    event_seg(S, p, &ib, &nbv, &ic, &ncv, &o0);
    const int n = (int)(nbv + ncv);  // <= cap (checked by the host)
    const uint64_t rxm = (1ull << rxbits) - 1;
    {
        // every load of the lane issued before the first LDS store (a
        // load-store loop would wait for each load in turn)
        uint64_t kq[SEG_ROUNDS];
        uint32_t pq[SEG_ROUNDS];
#pragma unroll
        for (int q = 0; q < SEG_ROUNDS; q++) {
            const int i = q * SEG_BLOCK + threadIdx.x;
            if (i < n) {
                const int64_t at = i < nbv ? ib + i : ic + (i - nbv);
                kq[q] = evkey[at];
                pq[q] = evpay[at];
            }
        }
#pragma unroll
        for (int q = 0; q < SEG_ROUNDS; q++) {
            const int i = q * SEG_BLOCK + threadIdx.x;
            if (i < n) src[i] = (uint32_t)(((kq[q] & rxm) << 2) | pq[q]);
        }
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    // the polygon's own row and column range: keys re-based to it need fewer
    // bits, so fewer passes (a polygon spans a few hundred rows and columns)
    __shared__ uint32_t rng[4];
    if (threadIdx.x < 4) rng[threadIdx.x] = (threadIdx.x & 1) ? 0u : 0xffffffffu;
    __syncthreads();
    const uint32_t xmask = (1u << xbits) - 1;
    {
        uint32_t r0 = 0xffffffffu, r1 = 0, x0 = 0xffffffffu, x1 = 0;
        for (int i = threadIdx.x; i < n; i += SEG_BLOCK) {
            const uint32_t rx = src[i] >> 2, r = rx >> xbits, x = rx & xmask;
            r0 = min(r0, r);
            r1 = max(r1, r);
            x0 = min(x0, x);
            x1 = max(x1, x);
        }
        for (int o = 32; o > 0; o >>= 1) {
            r0 = min(r0, (uint32_t)__shfl_xor((int)r0, o, 64));
            r1 = max(r1, (uint32_t)__shfl_xor((int)r1, o, 64));
            x0 = min(x0, (uint32_t)__shfl_xor((int)x0, o, 64));
            x1 = max(x1, (uint32_t)__shfl_xor((int)x1, o, 64));
        }
        if (lane == 0) {
            atomicMin(&rng[0], r0);
            atomicMax(&rng[1], r1);
            atomicMin(&rng[2], x0);
            atomicMax(&rng[3], x1);
        }
    }
    __syncthreads();
    const uint32_t rmin = rng[0], xmin = rng[2];
    const int xw = n ? 32 - __clz((int)(rng[3] - xmin)) : 0;
    const int rw = n ? 32 - __clz((int)(rng[1] - rmin)) : 0;
    for (int i = threadIdx.x; i < n; i += SEG_BLOCK) {
        const uint32_t v = src[i], rx = v >> 2;
        src[i] = ((((rx >> xbits) - rmin) << xw | ((rx & xmask) - xmin)) << 2) | (v & 3u);
    }
    __syncthreads();
    const int kbits = n ? rw + xw + 2 : 0;
    lds_radix_u32(src, dst, n, kbits, wcnt, doff, wtot);
    // coverage: each lane takes `per` consecutive sorted events; dst gets
    // the inclusive prefix words
    const int per = (n + SEG_BLOCK - 1) / SEG_BLOCK;
    const int i0 = threadIdx.x * per, i1 = min(i0 + per, n);
    uint32_t sum = 0;
    for (int i = i0; i < i1; i++) sum += ev_word(src[i] & 3u);
    uint32_t run = seg_excl_scan(sum, wsum);
    for (int i = i0; i < i1; i++) {
        run += ev_word(src[i] & 3u);
        dst[i] = run;
    }
    __syncthreads();
    // toggles: the last event of a (row, x) group where membership changes
    // from just before the group to just after it
    uint32_t fbits = 0, cnt = 0;
    for (int k = 0; k < per; k++) {
        const int i = i0 + k;
        if (i >= n) break;
        const uint32_t key = src[i] >> 2;  // re-based (row, x): row above bit xw
        if (i + 1 < n && (src[i + 1] >> 2) == key) continue;
        int a = i;
        while (a > 0 && (src[a - 1] >> 2) == key) a--;
        const uint32_t row = key >> xw;
        const uint32_t before =
            (a > 0 && ((src[a - 1] >> 2) >> xw) == row) ? cov_of(dst[a - 1]) : 0u;
        const uint32_t after = cov_of(dst[i]);
        if ((before > 0) != (after > 0)) {
            fbits |= 1u << k;
            cnt++;
            if (rowcnt) atomicAdd(rowcnt + rmin + row, 1ull);
        }
        if ((i + 1 == n || ((src[i + 1] >> 2) >> xw) != row) && after != 0) atomicOr(err, 2);
    }
    const uint32_t tex = seg_excl_scan(cnt, wsum);
    if (threadIdx.x == SEG_BLOCK - 1) ptot[p] = tex + cnt;
    // dst (the prefix words, no longer needed) takes each event's toggle
    // index and flag, so the outputs below leave in coalesced stores
    uint32_t t = tex;
    for (int k = 0; k < per; k++) {
        const int i = i0 + k;
        if (i >= n) break;
        const uint32_t f = (fbits >> k) & 1u;
        dst[i] = t | (f << 31);
        t += f;
    }
    __syncthreads();
    const uint64_t pk = (uint64_t)p << rxbits;
    const uint32_t lxm = (1u << xw) - 1;
    for (int i = threadIdx.x; i < n; i += SEG_BLOCK) {
        const uint32_t v = src[i], tl = dst[i], key = v >> 2;
        const uint32_t rx = (((key >> xw) + rmin) << xbits) | ((key & lxm) + xmin);
        okey[o0 + i] = pk | (uint64_t)rx;
        opay[o0 + i] = (v & 3u) | ((tl >> 31) << 2);
        otl[o0 + i] = (int32_t)(tl & 0x7fffffffu);
    }
}

// toggles of the per-polygon path: event t with its toggle bit set goes to
// slot o = ptoff[polygon] + otl[t] (polygon, then row and x order); with row
// buckets, (x << 32 | o) also goes to the bucket of its row, in no order
// (rowcnt: fill counters, zero on entry)
__global__ void k_toggle_emit_seg(const uint64_t *key, const uint32_t *pay, const int32_t *otl,
                                  const int64_t *ptoff, int64_t n, int rxbits, int xbits,
                                  uint64_t *tkey, int32_t *tpoly, const int64_t *rowoff,
                                  unsigned long long *rowcnt, uint64_t *rb)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n || !(pay[t] & 4u)) return;
    const uint64_t k = key[t];
    const int32_t p = (int32_t)(k >> rxbits);
    const int64_t o = ptoff[p] + otl[t];
    const uint64_t rx = k & ((1ull << rxbits) - 1);
    if (tkey) tkey[o] = rx;
    tpoly[o] = p;
    if (rb) {
        const uint64_t row = rx >> xbits, x = rx & ((1ull << xbits) - 1);
        const int64_t at = rowoff[row] + (int64_t)atomicAdd(rowcnt + row, 1ull);
        rb[at] = (x << 32) | (uint64_t)o;
    }
}

// One workgroup: row offsets of the toggle buckets (exclusive scan of
// rowcnt[0..gh) into rowoff[0..gh], total at rowoff[gh]), the largest row's
// count into *mx, and rowcnt zeroed again for use as fill counters.  The
// rows go by in chunks of one count per lane, the next chunk's counts loaded
// while the current one is scanned.
__global__ __launch_bounds__(SEG_BLOCK) void k_row_scan_max(unsigned long long *rowcnt, int64_t gh,
                                                            int64_t *rowoff,
                                                            unsigned long long *mx)
{
    __shared__ uint32_t wsum[SEG_WAVES];
    __shared__ uint32_t chunk_tot, smax;
    if (threadIdx.x == 0) smax = 0;
    __syncthreads();
    uint32_t carry = 0, m = 0;
    uint32_t next = threadIdx.x < gh ? (uint32_t)rowcnt[threadIdx.x] : 0u;
    for (int64_t c0 = 0; c0 < gh; c0 += SEG_BLOCK) {
        const int64_t r = c0 + threadIdx.x;
        const uint32_t cur = next;  // 0 past the last row
        next = r + SEG_BLOCK < gh ? (uint32_t)rowcnt[r + SEG_BLOCK] : 0u;
        m = max(m, cur);
        const uint32_t ex = seg_excl_scan(cur, wsum);
        if (r < gh) {
            rowoff[r] = carry + ex;
            rowcnt[r] = 0;
        }
        if (threadIdx.x == SEG_BLOCK - 1) chunk_tot = ex + cur;
        __syncthreads();
        carry += chunk_tot;
        __syncthreads();
    }
    for (int o = 32; o > 0; o >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, o, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(&smax, m);
    __syncthreads();
    if (threadIdx.x == 0) {
        rowoff[gh] = carry;
        *mx = smax;
    }
}

// Rows of at most ROW_CAP toggles: one wavefront per row ranks the row's
// (x, slot) words in LDS (a word's rank is the number of smaller words:
// slots are distinct), then walks them in order.  The distinct positions of
// row r take indices rowoff[r] + 0, 1, ... (a row's toggle count bounds its
// distinct positions; the indices left over up to rowoff[r + 1] stay holes
// of depth 0, which no piece reads), and each toggle learns its index.
#define ROW_CAP 512
#define ROW_WAVES 4
__global__ __launch_bounds__(64 * ROW_WAVES) void k_row_pieces(const uint64_t *rb,
                                                                const int64_t *rowoff, int64_t gh,
                                                                int xbits, int64_t nt, uint64_t *E,
                                                                int64_t *rank, int64_t *diff)
{
    __shared__ uint64_t raw[ROW_WAVES][ROW_CAP];
    __shared__ uint64_t sorted[ROW_WAVES][ROW_CAP];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t r = (int64_t)blockIdx.x * ROW_WAVES + wv;
    if (r >= gh) return;  // whole wavefronts leave; no workgroup barrier below
    const int64_t base = rowoff[r];
    const int c = (int)(rowoff[r + 1] - base);  // <= ROW_CAP (checked by the host)
    uint64_t *w = raw[wv], *s = sorted[wv];
    {
        uint64_t v[ROW_CAP / 64];
#pragma unroll
        for (int q = 0; q < ROW_CAP / 64; q++)
            if (q * 64 + lane < c) v[q] = rb[base + q * 64 + lane];
#pragma unroll
        for (int q = 0; q < ROW_CAP / 64; q++)
            if (q * 64 + lane < c) w[q * 64 + lane] = v[q];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int i = lane; i < c; i += 64) {
        const uint64_t v = w[i];
        int rk = 0;
        for (int j = 0; j < c; j++) rk += w[j] < v ? 1 : 0;
        s[rk] = v;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    int64_t nd = 0;  // distinct positions so far
    for (int q0 = 0; q0 < c; q0 += 64) {
        const int q = q0 + lane;
        const bool valid = q < c;
        const uint64_t v = valid ? s[q] : 0ull;
        const uint32_t x = (uint32_t)(v >> 32);
        const bool first = valid && (q == 0 || (uint32_t)(s[q - 1] >> 32) != x);
        const uint64_t fb = __ballot(first);
        const uint64_t le = fb & ((2ull << lane) - 1);
        const int64_t idx = base + nd + __popcll(le) - 1;
        if (valid) {
            const uint32_t slot = (uint32_t)v;
            rank[slot] = idx;
            if (first) {
                E[idx] = ((uint64_t)r << xbits) | x;
                int64_t d = 0;
                for (int u = q; u < c && (uint32_t)(s[u] >> 32) == x; u++)
                    d += ((uint32_t)s[u] & 1u) ? -1 : 1;
                diff[idx] = d;
            }
        }
        nd += __popcll(fb);
    }
    for (int64_t q = nd + lane; q < c; q += 64) diff[base + q] = 0;
    if (r == gh - 1 && lane == 0) diff[nt] = 0;
}

// ------------------------------------------------ coverage of each row
//
// Events carry the key (polygon, row, x) and one of three kinds: the start
// of a boundary interval, one past its end, or a crossing of the row line.
// Sorted by key, each (polygon, row) group holds matched starts and ends and
// an even number of crossings; cells from the 2m-th to the (2m+1)-th
// crossing have their corner inside (Sec. 2.2, crossing-number rule).  The
// polygon covers x when a boundary interval is open there or the crossings
// seen so far are odd in number.  One global scan gives both counts at every
// event: starts and ends add +1/-1 to the low 32 bits, crossings add 1 to
// the high bits.  Groups before the current one are balanced, so the prefix
// equals the prefix within the group.
__device__ __forceinline__ int64_t ev_value(uint32_t kind)
{
    return kind == EV_CROSS ? ((int64_t)1 << 32) : (kind == EV_OPEN ? 1 : -1);
}

// coverage count of the event's polygon just after event t (cex = exclusive
// scan of ev_value); the low part never goes negative because the sort is
// stable and every interval's start precedes its end
__device__ __forceinline__ int64_t cov_after(const int64_t *cex, const uint32_t *kind, int64_t t)
{
    int64_t S = cex[t] + ev_value(kind[t]);
    return (S & 0xffffffffll) + ((S >> 32) & 1);
}

__global__ void k_ev_values(const uint32_t *kind, int64_t n, int64_t *v)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) v[t] = ev_value(kind[t]);
}

// flag[t] = 1 when t is the last event of its (polygon, row, x) group and
// the polygon's membership at x differs from its membership just before x
// (a toggle).  Toggles of one (polygon, row) alternate on/off, starting with
// on, so consecutive pairs are the maximal covered intervals [a, b).  The
// group's first event comes from a ballot of the wavefront's group heads; only
// a group that began in an earlier wavefront is walked back in memory.
__global__ __launch_bounds__(256) void k_toggle_flags(const uint64_t *key, const uint32_t *kind,
                                                      const int64_t *cex, int64_t n, int xbits,
                                                      int64_t *flag, int *err)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const bool in = t < n;
    const uint64_t k = in ? key[t] : 0;
    const bool head = in && (t == 0 || key[t - 1] != k);
    const uint64_t heads = __ballot(head);
    if (!in) return;
    int64_t f = 0;
    if (t + 1 == n || key[t + 1] != k) {
        // heads at or before this lane (2 << 63 wraps to 0: all lanes)
        const uint64_t le = heads & ((2ull << lane) - 1);
        int64_t a = t - lane;
        if (le) {
            a += 63 - __clzll(le);
        } else {
            while (a > 0 && key[a - 1] == k) a--;
        }
        uint64_t g = k >> xbits;
        int64_t before = (a > 0 && (key[a - 1] >> xbits) == g) ? cov_after(cex, kind, a - 1) : 0;
        int64_t after = cov_after(cex, kind, t);
        f = (before > 0) != (after > 0);
        if ((t + 1 == n || (key[t + 1] >> xbits) != g) && after != 0) atomicOr(err, 2);
    }
    flag[t] = f;
}

__global__ void k_toggle_emit(const uint64_t *key, const int64_t *toff, int64_t n, int64_t nt,
                              int rxbits, uint64_t *tkey, int32_t *tpoly)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    int64_t o = toff[t];
    int64_t o1 = t + 1 < n ? toff[t + 1] : nt;
    if (o1 == o) return;
    uint64_t k = key[t];
    tkey[o] = k & ((1ull << rxbits) - 1);
    tpoly[o] = (int32_t)(k >> rxbits);
}

__global__ void k_iota_u32(uint32_t *v, int64_t n)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) v[t] = (uint32_t)t;
}

// One pass over the toggles sorted by position (row << xbits | x), each
// carrying its original slot src[t] (slot 2m opens covered interval m, slot
// 2m + 1 closes it).  pos is the exclusive count of first occurrences, nu
// its total (the number of distinct positions).  Writes
//  * E: the sorted distinct positions, which cut every row into elementary
//    pieces [E[k], E[k+1]) of constant polygon set;
//  * rank[slot]: the index in E of every toggle;
//  * diff[k]: intervals opening at E[k] less intervals closing there (the
//    depth of piece k is the prefix sum), formed by the first toggle of each
//    distinct position over its run of equal positions; entries nu..n are
//    zeroed here.
__global__ void k_unique_rank(const uint64_t *keys, int64_t n, const int64_t *pos,
                              const int64_t *nu_p, const uint32_t *src, uint64_t *E,
                              int64_t *rank, int64_t *diff)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const uint64_t k = keys[t];
    const bool first = t == 0 || k != keys[t - 1];
    const int64_t r = pos[t] - (first ? 0 : 1);
    rank[src[t]] = r;
    if (first) {
        E[r] = k;
        int64_t d = 0;
        for (int64_t u = t; u < n && keys[u] == k; u++) d += (src[u] & 1u) ? -1 : 1;
        diff[r] = d;
    }
    const int64_t nu = *nu_p;
    if (t >= nu) diff[t] = 0;
    if (t == n - 1) diff[n] = 0;
}

// Covered interval m spans pieces [ka, kb), the indices in E of its two
// toggles.
__global__ void k_interval_span(const int64_t *rank, int64_t nint, int64_t *ika, int64_t *cnt)
{
    int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= nint) return;
    const int64_t ka = rank[2 * m], kb = rank[2 * m + 1];
    ika[m] = ka;
    cnt[m] = kb - ka;
}

// per piece: packed counters (non-empty << 32 | multi) and multi member count
__global__ void k_piece_classify(const int64_t *dex, const int64_t *diff, int64_t n, int64_t *segc,
                                 int64_t *mm, int *err)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int64_t d = dex[k] + diff[k];
    if (d > MAX_DEPTH) atomicOr(err, 8);
    segc[k] = (d >= 1 ? ((int64_t)1 << 32) : 0) | (d >= 2 ? 1 : 0);
    mm[k] = d >= 2 ? d : 0;
}

// one thread per (interval, piece) pair: record the interval's polygon in
// the piece (a piece of depth 1 keeps its polygon directly)
__global__ void k_piece_members(const int64_t *xoff, int64_t nint, int64_t nx, const int64_t *ika,
                                const int32_t *tpoly, const int64_t *dex, const int64_t *diff,
                                const int64_t *mmoff, int32_t *sid, int32_t *fill, int32_t *mem_ids)
{
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= nx) return;
    int64_t lo = 0, hi = nint;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (xoff[mid] <= u) lo = mid + 1; else hi = mid;
    }
    int64_t m = lo - 1;
    int64_t k = ika[m] + (u - xoff[m]);
    int32_t p = tpoly[2 * m];
    if (dex[k] + diff[k] == 1) {
        sid[k] = p;
    } else {
        int32_t r = atomicAdd(&fill[k], 1);
        mem_ids[mmoff[k] + r] = p;
    }
}

// non-empty pieces become the row segments; members of multi-polygon
// segments are put in ascending order (the set's canonical form)
__global__ void k_piece_emit(const uint64_t *E, int64_t n, const int64_t *dex, const int64_t *diff,
                             const int64_t *segc, const int64_t *mmoff, const int32_t *sid,
                             int xbits, int32_t *seg_x0, int32_t *seg_x1, uint32_t *seg_code,
                             uint32_t *seg_row, int64_t *multi_seg, int64_t *multi_mem,
                             int32_t *mem_ids)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int64_t d = dex[k] + diff[k];
    if (d < 1) return;
    const uint64_t xm = (1ull << xbits) - 1;
    int64_t sc = segc[k];
    int64_t o = sc >> 32;
    uint64_t e0 = E[k], e1 = E[k + 1];
    seg_x0[o] = (int32_t)(e0 & xm);
    seg_x1[o] = (int32_t)(e1 & xm);
    seg_row[o] = (uint32_t)(e0 >> xbits);
    if (d == 1) {
        seg_code[o] = (uint32_t)sid[k] + 1u;
        return;
    }
    int64_t a = mmoff[k];
    for (int64_t i = a + 1; i < a + d; i++) {
        int32_t v = mem_ids[i];
        int64_t j = i;
        while (j > a && mem_ids[j - 1] > v) { mem_ids[j] = mem_ids[j - 1]; j--; }
        mem_ids[j] = v;
    }
    int64_t mi = sc & 0xffffffffll;
    multi_seg[mi] = o;
    multi_mem[mi] = a;
    seg_code[o] = 0xffffffffu;
}

__global__ void k_seg_row_off(const uint32_t *seg_row, int64_t ns, int64_t gh, int64_t *row_off)
{
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r > gh) return;
    int64_t lo = 0, hi = ns;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if ((int64_t)seg_row[mid] < r) lo = mid + 1; else hi = mid;
    }
    row_off[r] = lo;
}

// ------------------------------------------------ multi-polygon set dedup

// Sets of 2 or 3 polygons are packed exactly into fb-bit fields (fb bits hold
// id+1); larger sets get a key of their own above that range (not shared).
__global__ void k_multi_keys(const int64_t *multi_mem, int64_t n_multi, int64_t n_mem,
                             const int32_t *mem_ids, int fb, uint64_t *key, uint32_t *val)
{
    int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n_multi) return;
    int64_t a = multi_mem[m], b = (m + 1 < n_multi) ? multi_mem[m + 1] : n_mem;
    uint64_t k = 0;
    if (b - a <= 3) {
        for (int64_t t = a; t < b; t++) k |= (uint64_t)(mem_ids[t] + 1) << (fb * (t - a));
    } else {
        k = (1ull << (3 * fb)) | (uint64_t)m;
    }
    key[m] = k;
    val[m] = (uint32_t)m;
}

__global__ void k_flag_new(const uint64_t *key, int64_t n, int64_t *flag)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    flag[t] = (t == 0 || key[t] != key[t - 1]) ? 1 : 0;
}

__global__ void k_set_sizes(const uint64_t *key, const uint32_t *val, const int64_t *gexcl,
                            int64_t n, const int64_t *multi_mem, int64_t n_multi, int64_t n_mem,
                            int64_t *set_sz)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    if (t == 0 || key[t] != key[t - 1]) {
        int64_t m = val[t];
        int64_t a = multi_mem[m], b = (m + 1 < n_multi) ? multi_mem[m + 1] : n_mem;
        set_sz[gexcl[t]] = b - a;
    }
}

__global__ void k_set_fill(const uint64_t *key, const uint32_t *val, const int64_t *gexcl,
                           int64_t n, const int64_t *multi_mem, int64_t n_multi, int64_t n_mem,
                           const int32_t *mem_ids, const int64_t *set_off, int32_t *set_ids,
                           const int64_t *multi_seg, uint32_t *seg_code)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    bool first = (t == 0 || key[t] != key[t - 1]);
    int64_t g = gexcl[t] + (first ? 1 : 0) - 1;
    int64_t m = val[t];
    if (first) {
        int64_t a = multi_mem[m], b = (m + 1 < n_multi) ? multi_mem[m + 1] : n_mem;
        int64_t o = set_off[g];
        for (int64_t q = a; q < b; q++) set_ids[o + (q - a)] = mem_ids[q];
    }
    seg_code[multi_seg[m]] = CODE_SET_BASE + (uint32_t)g;
}

// Sets of at most SET_CAP distinct keys (keys below 2^31) take a shorter
// path than the global sort of all NM keys: a hash table collects the
// distinct keys (each first insert appends its key to a list), one workgroup
// sorts the list in LDS, numbers the sets in key order (the numbering the
// global sort gives), lays out and fills the set table and records each
// key's number in a table beside the hash, and one lookup per multi segment
// writes its code.
#define SET_CAP 8192
#define SET_EMPTY 0xffffffffu

__device__ __forceinline__ uint32_t set_slot(uint32_t k, int hb)
{
    return (k * 2654435761u) >> (32 - hb);
}

__global__ void k_set_insert(const uint64_t *key, int64_t n, uint32_t *tab, int hb,
                             uint32_t *list, unsigned long long *cnt)
{
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    const uint32_t k = (uint32_t)key[m], mask = (1u << hb) - 1u;
    // neighbouring multi segments mostly share their set: only the first of
    // a run of equal keys inserts it
    if (m > 0 && (uint32_t)key[m - 1] == k) return;
    uint32_t s = set_slot(k, hb);
    // the table has at least twice as many slots as keys: a free slot is
    // always ahead; a slot already holding the key is seen without an atomic
    while (true) {
        const uint32_t seen = tab[s];
        if (seen == k) return;
        if (seen != SET_EMPTY) {
            s = (s + 1) & mask;
            continue;
        }
        const uint32_t prev = atomicCAS(tab + s, SET_EMPTY, k);
        if (prev == SET_EMPTY) {
            const unsigned long long at = atomicAdd(cnt, 1ull);
            if (at < SET_CAP) list[at] = k;
            return;
        }
        if (prev == k) return;
        s = (s + 1) & mask;
    }
}

__device__ __forceinline__ uint32_t set_find(const uint32_t *tab, uint32_t k, int hb)
{
    const uint32_t mask = (1u << hb) - 1u;
    uint32_t s = set_slot(k, hb);
    while (tab[s] != k) s = (s + 1) & mask;
    return s;
}

// members of the set with key k: fb-bit fields of id + 1 (ascending ids) for
// sets of 2 or 3, else the members of multi segment k - 2^(3 fb)
__device__ __forceinline__ int64_t set_members(uint32_t k, int fb, const int64_t *multi_mem,
                                               int64_t n_multi, int64_t n_mem, int64_t *a)
{
    if (k < (1u << (3 * fb))) {
        const uint32_t fm = (1u << fb) - 1u;
        *a = -1;
        return ((k & fm) != 0) + (((k >> fb) & fm) != 0) + (((k >> (2 * fb)) & fm) != 0);
    }
    const int64_t m = (int64_t)(k - (1u << (3 * fb)));
    *a = multi_mem[m];
    return ((m + 1 < n_multi) ? multi_mem[m + 1] : n_mem) - *a;
}

// one workgroup; dynamic LDS: two buffers of SET_CAP words and the digit
// counters.  Leaves at once when the list overflowed (the host then takes
// the global sort).  Out: set_off[0..nd], set_ids, rank[slot] for every
// key's slot, *nids = the total member count.
__global__ __launch_bounds__(SEG_BLOCK) void k_set_table(const uint32_t *list,
                                                         const unsigned long long *cnt,
                                                         const uint32_t *tab, int hb, int kbits,
                                                         int fb, const int64_t *multi_mem,
                                                         int64_t n_multi, int64_t n_mem,
                                                         const int32_t *mem_ids, uint32_t *rank,
                                                         int64_t *set_off, int32_t *set_ids,
                                                         unsigned long long *nids)
{
    extern __shared__ uint32_t set_lds[];
    uint32_t *src = set_lds, *dst = set_lds + SET_CAP;
    uint32_t *wcnt = set_lds + 2 * SET_CAP;
    __shared__ uint32_t doff[SEG_RADIX];
    __shared__ uint32_t wtot[SEG_RADIX / 64];
    __shared__ uint32_t wsum[SEG_WAVES];
    const unsigned long long nd = *cnt;
    if (nd > SET_CAP) return;
    const int n = (int)nd;
    for (int i = threadIdx.x; i < n; i += SEG_BLOCK) src[i] = list[i];
    __syncthreads();
    lds_radix_u32(src, dst, n, kbits, wcnt, doff, wtot);
    // set r = src[r]: sizes, offsets (each lane `per` consecutive sets)
    const int per = (n + SEG_BLOCK - 1) / SEG_BLOCK;
    const int i0 = threadIdx.x * per, i1 = min(i0 + per, n);
    uint32_t sum = 0;
    int64_t a;
    for (int i = i0; i < i1; i++) sum += (uint32_t)set_members(src[i], fb, multi_mem, n_multi, n_mem, &a);
    uint32_t off = seg_excl_scan(sum, wsum);
    for (int i = i0; i < i1; i++) {
        const uint32_t k = src[i];
        const int64_t c = set_members(k, fb, multi_mem, n_multi, n_mem, &a);
        set_off[i] = off;
        if (a < 0) {
            const uint32_t fm = (1u << fb) - 1u;
            for (int64_t t = 0; t < c; t++) set_ids[off + t] = (int32_t)(((k >> (fb * t)) & fm) - 1);
        } else {
            for (int64_t t = 0; t < c; t++) set_ids[off + t] = mem_ids[a + t];
        }
        rank[set_find(tab, k, hb)] = (uint32_t)i;
        off += (uint32_t)c;
    }
    if (threadIdx.x == SEG_BLOCK - 1) {
        set_off[n] = off;
        *nids = off;
    }
}

// code of every multi segment: its key's set number
__global__ void k_set_codes(const uint64_t *key, int64_t n, const unsigned long long *cnt,
                            const uint32_t *tab, int hb, const uint32_t *rank,
                            const int64_t *multi_seg, uint32_t *seg_code)
{
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n || *cnt > SET_CAP) return;
    const uint32_t g = rank[set_find(tab, (uint32_t)key[m], hb)];
    seg_code[multi_seg[m]] = CODE_SET_BASE + g;
}

// ------------------------------------------------ segment lookups

__device__ __forceinline__ uint32_t seg_code_at(const int64_t *seg_row_off, const int32_t *seg_x0,
                                                const int32_t *seg_x1, const uint32_t *seg_code,
                                                int64_t r, int32_t x)
{
    int64_t lo = seg_row_off[r], hi = seg_row_off[r + 1];
    int64_t a = lo;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (seg_x0[mid] <= x) lo = mid + 1; else hi = mid;
    }
    if (lo > a && x < seg_x1[lo - 1]) return seg_code[lo - 1];
    return 0;
}

__global__ void k_lookup_ij(const int64_t *seg_row_off, const int32_t *seg_x0, const int32_t *seg_x1,
                            const uint32_t *seg_code, int64_t gi0, int64_t gj0, int64_t gw, int64_t gh,
                            const int64_t *ij, int64_t n, uint32_t *out)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    int64_t i = ij[2 * t] - gi0, j = ij[2 * t + 1] - gj0;
    out[t] = (i < 0 || j < 0 || i >= gw || j >= gh)
                 ? 0u
                 : seg_code_at(seg_row_off, seg_x0, seg_x1, seg_code, j, (int32_t)i);
}

// ------------------------------------------------ tiled grid
//
// The grid is stored in up to three levels: a directory of tiles of 2^tl
// cells a side, for mixed tiles a sub-directory of sub-tiles of 2^sl cells a
// side (sl < tl), and for mixed sub-tiles (or mixed tiles when sl == tl) a
// fine block of one code per cell.  A uniform square stores its code once.

// 16-bit short code of a cell code: 0 none, p+1 polygon p, np+1+k set k
__device__ __forceinline__ uint32_t short_code(uint32_t c, uint32_t np)
{
    return c < CODE_SET_BASE ? c : np + 1 + (c - CODE_SET_BASE);
}

// origin (first column, first row) of square u: a tile (mt == NULL), or
// sub-tile u % Q of mixed tile mt[u / Q]
__device__ __forceinline__ void square_origin(int64_t u, const int64_t *mt, int tl, int sl,
                                              int64_t tw, int32_t *x0, int64_t *r0)
{
    if (!mt) {
        *x0 = (int32_t)((u % tw) << tl);
        *r0 = (u / tw) << tl;
        return;
    }
    const int qs = tl - sl;  // sub-tiles per tile side: 2^qs
    int64_t q = u & (((int64_t)1 << (2 * qs)) - 1);
    int64_t tile = mt[u >> (2 * qs)];
    *x0 = (int32_t)(((tile % tw) << tl) + ((q & (((int64_t)1 << qs) - 1)) << sl));
    *r0 = ((tile / tw) << tl) + ((q >> qs) << sl);
}

// G lanes per square (G = min(side, 64)): uniform code of the square, or
// 0xffffffff and mixed[u] = 1
template <int G>
__global__ void k_square_classify(const int64_t *seg_row_off, const int32_t *seg_x0,
                                  const int32_t *seg_x1, const uint32_t *seg_code, int64_t gw,
                                  int64_t gh, const int64_t *mt, int tl, int sl, int64_t tw,
                                  int64_t n_sq, uint32_t *code, int64_t *mixed)
{
    int64_t u = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    int lane = threadIdx.x & (G - 1);
    if (u >= n_sq) return;  // whole groups leave together (G divides the block)
    const int side_log2 = mt ? sl : tl;
    int32_t x0;
    int64_t r0;
    square_origin(u, mt, tl, sl, tw, &x0, &r0);
    int32_t x1 = (int32_t)min((int64_t)x0 + (1 << side_log2), gw);
    int64_t r1 = min(r0 + (1 << side_log2), gh);
    uint32_t lo_c = 0xffffffffu, hi_c = 0;
    if (x0 >= gw || r0 >= gh) {  // square wholly outside the stored box
        lo_c = hi_c = 0;
    }
    for (int64_t r = r0 + lane; r < r1 && x0 < gw; r += G) {
        int64_t a = seg_row_off[r], lo = a, hi = seg_row_off[r + 1], e = hi;
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            if (seg_x0[mid] <= x0) lo = mid + 1; else hi = mid;
        }
        uint32_t c;
        if (lo > a && x0 < seg_x1[lo - 1]) {
            c = (seg_x1[lo - 1] >= x1) ? seg_code[lo - 1] : 0xffffffffu;
        } else {
            c = (lo >= e || seg_x0[lo] >= x1) ? 0u : 0xffffffffu;
        }
        lo_c = min(lo_c, c);
        hi_c = max(hi_c, c);
    }
    // a square cut by the edge of the box is uniform only if its stored part
    // is; cells beyond the box read as 0 through the probe's range test
    for (int o = G / 2; o > 0; o >>= 1) {
        lo_c = min(lo_c, (uint32_t)__shfl_xor((int)lo_c, o, 64));
        hi_c = max(hi_c, (uint32_t)__shfl_xor((int)hi_c, o, 64));
    }
    if (lane == 0) {
        bool uni = (lo_c == hi_c) && (hi_c != 0xffffffffu);
        code[u] = uni ? hi_c : 0xffffffffu;
        mixed[u] = uni ? 0 : 1;
    }
}

// list[pos[u]] = u for every flagged u (pos = exclusive scan of the flags)
__global__ void k_flag_list(const int64_t *pos, int64_t n, int64_t total, int64_t *list)
{
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    int64_t o = pos[u], o1 = u + 1 < n ? pos[u + 1] : total;
    if (o1 != o) list[o] = u;
}

// Fine blocks: one thread per (block, row, run of up to 16 cells): one
// binary search for the run's first cell, then a walk along the row's
// segments.  Block k holds square sq[k] of side 2^side_log2 (sq indexes the
// squares of k_square_classify).  OUT = uint32_t full codes or uint16_t
// short codes.
template <typename OUT>
__global__ __launch_bounds__(256) void k_block_fill(const int64_t *seg_row_off, const int32_t *seg_x0,
                             const int32_t *seg_x1, const uint32_t *seg_code, int64_t gw,
                             int64_t gh, const int64_t *sq, int64_t nblk, const int64_t *mt,
                             int tl, int sl, int64_t tw, int side_log2, uint32_t np, OUT *blocks)
{
    const int side = 1 << side_log2;
    const int runs = side > 16 ? side >> 4 : 1;
    const int rlen = side > 16 ? 16 : side;
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nblk * side * runs) return;
    int64_t k = t / ((int64_t)side * runs);
    int rem = (int)(t - k * side * runs);
    int row = rem / runs, run = rem - row * runs;
    int32_t x0;
    int64_t r0;
    square_origin(sq[k], mt, tl, sl, tw, &x0, &r0);
    OUT *out = blocks + (k << (2 * side_log2)) + ((int64_t)row << side_log2) + run * rlen;
    int64_t r = r0 + row;
    int32_t xa = x0 + run * rlen;
    if (r >= gh) {
        for (int c = 0; c < rlen; c++) out[c] = 0;
        return;
    }
    const int64_t lo = seg_row_off[r], hi = seg_row_off[r + 1];
    int64_t a = lo, e = hi;
    while (a < e) {
        int64_t mid = (a + e) >> 1;
        if (seg_x0[mid] <= xa) a = mid + 1; else e = mid;
    }
    const int64_t q0 = a - 1;  // last segment starting at or before xa (lo-1 if none)
    // the run's codes go to registers first and leave in 16-byte stores (a
    // run starts at a multiple of 16 bytes: blocks and rows are multiples of
    // 8 bytes long and runs of 16 codes are 32 or 64 bytes)
    OUT buf[16] __attribute__((aligned(16)));
    // Segments q0 .. q0 + 3 are loaded at once (no chain of dependent loads
    // along the row); they cover the run unless segment q0 + 4 starts inside
    // it, and then the run walks the row's segments one by one.  Segments of
    // a row are disjoint, so at most one holds a cell.
    constexpr int W = 4;
    int32_t wx0[W], wx1[W];
    uint32_t wc[W];
#pragma unroll
    for (int j = 0; j < W; j++) {
        const int64_t q = q0 + j;
        const bool in = q >= lo && q < hi;
        wx0[j] = in ? seg_x0[q] : INT32_MAX;
        wx1[j] = in ? seg_x1[q] : INT32_MIN;
        wc[j] = in ? seg_code[q] : 0u;
    }
    if (!(q0 + W < hi && seg_x0[q0 + W] < xa + rlen)) {
#pragma unroll
        for (int c = 0; c < 16; c++) {
            if (c >= rlen) break;
            const int32_t x = xa + c;
            uint32_t v = 0;
#pragma unroll
            for (int j = 0; j < W; j++) v = (wx0[j] <= x && x < wx1[j]) ? wc[j] : v;
            if (x >= gw) v = 0;
            buf[c] = sizeof(OUT) == 2 ? (OUT)short_code(v, np) : (OUT)v;
        }
    } else {
        int64_t q = q0;
#pragma unroll
        for (int c = 0; c < 16; c++) {
            if (c >= rlen) break;
            int32_t x = xa + c;
            while (q + 1 < hi && seg_x0[q + 1] <= x) q++;
            uint32_t v = 0;
            if (x < gw && q >= lo && x < seg_x1[q]) v = seg_code[q];
            buf[c] = sizeof(OUT) == 2 ? (OUT)short_code(v, np) : (OUT)v;
        }
    }
    // constant indices only, so buf stays in registers (a dynamically
    // indexed array would be moved to LDS, which the kernel then reserves)
    const int bytes = rlen * (int)sizeof(OUT);
    if (bytes % 16 == 0) {
        uint4 *o4 = (uint4 *)out;
        const uint4 *b4 = (const uint4 *)buf;
#pragma unroll
        for (int k = 0; k < (int)sizeof(OUT); k++)  // 16 codes = sizeof(OUT) x 16 bytes
            if (k < bytes / 16) o4[k] = b4[k];
    } else {
#pragma unroll
        for (int c = 0; c < 16; c++)
            if (c < rlen) out[c] = buf[c];
    }
}

// final directory / sub-directory entries: the square's code (short codes
// in the compact format), or TILE_MIXED | index of its fine block or
// sub-directory.  Compact directory entries are 16-bit: 0x8000 | index.
__global__ void k_entries(const uint32_t *code, const int64_t *pos, int64_t n, int64_t n_pad,
                          uint32_t np, int mode, uint32_t *out32, uint16_t *out16)
{
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n_pad) return;
    if (u >= n) { out16[u] = 0; return; }  // padding exists only in mode 2
    uint32_t c = code[u];
    bool mixed = c == 0xffffffffu;
    uint32_t idx = (uint32_t)pos[u];
    if (mode == 0) out32[u] = mixed ? (TILE_MIXED | idx) : c;                   // wide
    else if (mode == 1) out32[u] = mixed ? (TILE_MIXED | idx) : short_code(c, np);  // compact sub
    else out16[u] = (uint16_t)(mixed ? (0x8000u | idx) : short_code(c, np));   // compact dir
}

// ---------------------------------------------------------------- host side

void magic_for(int64_t s, uint32_t *mag, int32_t *shift)
{
    int l = 0;
    while (((int64_t)1 << l) < s) l++;  // l = ceil(log2 s)
    // m = ceil(2^(31+l) / s)
    unsigned __int128 num = (unsigned __int128)1 << (31 + l);
    uint64_t m = (uint64_t)((num + (unsigned __int128)(s - 1)) / (unsigned __int128)s);
    *mag = (uint32_t)m;  // < 2^32 (== 2^31 for s == 1)
    *shift = 31 + l;
}

int pool_setup()
{
    static bool done[64] = {false};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return SBA_EDEVICE;
    if (done[dev]) return 0;
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) != hipSuccess) {
        (void)hipGetLastError();
        return SBA_EDEVICE;
    }
    uint64_t keep = ~0ull;
    if (hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep) != hipSuccess) {
        (void)hipGetLastError();
        return SBA_EDEVICE;
    }
    done[dev] = true;
    return 0;
}

// Hilbert key grid covering the cell boxes of several polygon sets: each
// set's offsets are checked and its union cell box found by the kernels of
// the build (k_check_rings, k_check_verts, k_poly_bbox, k_union_box); the
// grid is anchored at the first cell of the union of the boxes and has the
// smallest level L >= 1 with 2^L cells covering the union's longer side,
// the level the Hilbert layout takes for a stored box of that size.
int key_grid_launch(const sba_polygons *sets, int32_t n_sets, int64_t eps, hipStream_t st,
                    int32_t *level, int64_t *i0, int64_t *j0)
{
    const int64_t s = cell_side(eps);
    constexpr int SLOTS = 8;  // per set: [0] error bits, [1..2] sizes, [3..6] cell box
    Workspace ws(st);
    int64_t *sc = nullptr;
    RC(ws.alloc(&sc, (int64_t)n_sets * SLOTS));
    HIP_OK(hipMemsetAsync(sc, 0, sizeof(int64_t) * SLOTS * n_sets, st));
    std::vector<int4 *> bbox(n_sets, nullptr);
    for (int32_t k = 0; k < n_sets; k++) {
        const sba_polygons &P = sets[k];
        const int32_t np = P.n_polys;
        if (np == 0) continue;
        int *err = (int *)(sc + SLOTS * k);
        int64_t *sizes = sc + SLOTS * k + 1, *dbox = sc + SLOTS * k + 3;
        hipLaunchKernelGGL(k_check_rings, dim3(grid_for(np + 1)), dim3(256), 0, st, P.ring_off, np,
                           sizes, err);
        hipLaunchKernelGGL(k_check_verts, dim3(1024), dim3(256), 0, st, P.vert_off, sizes, err);
        RC(ws.alloc(&bbox[k], np));
        hipLaunchKernelGGL(k_poly_bbox, dim3(grid_for((int64_t)np * 64)), dim3(256), 0, st,
                           P.ring_off, P.vert_off, P.xy, np, bbox[k], err);
        hipLaunchKernelGGL(k_union_box, dim3(1), dim3(BOX_BLOCK), 0, st, bbox[k], np, s, dbox);
        HIP_OK(hipGetLastError());
    }
    std::vector<int64_t> hsc((size_t)SLOTS * n_sets);
    RC(ws.read(hsc.data(), sc, sizeof(int64_t) * SLOTS * n_sets));
    RC(ws.sync());
    bool any = false;
    int64_t bi0 = 0, bj0 = 0, bi1 = 0, bj1 = 0;
    for (int32_t k = 0; k < n_sets; k++) {
        if (sets[k].n_polys == 0) continue;
        const int64_t *v = hsc.data() + SLOTS * k;
        const int herr = (int)(uint32_t)v[0];
        if (herr & 2) return SBA_EINVAL;
        if (herr & 1) return SBA_ERANGE;
        bi0 = any ? std::min(bi0, v[3]) : v[3];
        bj0 = any ? std::min(bj0, v[4]) : v[4];
        bi1 = any ? std::max(bi1, v[5]) : v[5];
        bj1 = any ? std::max(bj1, v[6]) : v[6];
        any = true;
    }
    if (!any) return SBA_EINVAL;
    const int64_t side = std::max(bi1 - bi0 + 1, bj1 - bj0 + 1);
    int L = 1;
    while (L <= 21 && ((int64_t)1 << L) < side) L++;
    if (L > 21) return SBA_ELIMIT;
    *level = L;
    *i0 = bi0;
    *j0 = bj0;
    return 0;
}

// paths of the coverage stages: bits set in g_build_paths_off turn a path
// off (1: the per-polygon event sort, 2: the toggle row buckets, 4: the set
// table through a hash); the last build's paths taken, same bits (tests of
// both sides of each choice)
static std::atomic<int> g_build_paths_off{0}, g_build_paths_last{0};

extern "C" int sba_debug_build_paths(int off)
{
    if (off < 0 || off > 7) return SBA_EINVAL;
    g_build_paths_off = off;
    return 0;
}

extern "C" int sba_debug_last_build_paths(void) { return g_build_paths_last.load(); }

int build_segments(const sba_polygons *polys, int64_t eps, hipStream_t st, sba_handle *h,
                   BuildState &B, bool need_boundary_cells)
{
    (void)need_boundary_cells;
    const int32_t np = polys->n_polys;
    // device scalars read back together (one copy per synchronisation):
    // [0] error bits (int), [1..2] ring and vertex counts, [3..6] union cell
    // box, [8..13] totals of the scans
    RC(B.alloc(&B.sc, SC_SLOTS));
    HIP_OK(hipMemsetAsync(B.sc, 0, sizeof(int64_t) * SC_SLOTS, st));
    int *err = (int *)B.sc;
    int64_t *sizes = B.sc + 1, *dbox = B.sc + 3, *tot = B.sc + 8;
    int64_t hsc[SC_READ];
    auto fetch = [&]() -> int {
        RC(B.ws.read(hsc, B.sc, sizeof(hsc)));
        return B.ws.sync();
    };

    // validate the offsets on the device (each stage reads only what the
    // previous one validated) and read sizes and bounding boxes in one sync
    hipLaunchKernelGGL(k_check_rings, dim3(grid_for(np + 1)), dim3(256), 0, st, polys->ring_off, np,
                       sizes, err);
    hipLaunchKernelGGL(k_check_verts, dim3(1024), dim3(256), 0, st, polys->vert_off, sizes, err);
    HIP_OK(hipGetLastError());
    int4 *bbox = nullptr;
    RC(B.alloc(&bbox, np));
    hipLaunchKernelGGL(k_poly_bbox, dim3(grid_for((int64_t)np * 64)), dim3(256), 0, st,
                       polys->ring_off, polys->vert_off, polys->xy, np, bbox, err);
    HIP_OK(hipGetLastError());
    hipLaunchKernelGGL(k_union_box, dim3(1), dim3(BOX_BLOCK), 0, st, bbox, np, h->s, dbox);
    HIP_OK(hipGetLastError());
    RC(fetch());
    int herr = (int)(uint32_t)hsc[0];
    if (herr & 2) return SBA_EINVAL;
    if (herr & 1) return SBA_ERANGE;
    const int32_t nr = (int32_t)hsc[1];
    const int64_t nv = hsc[2];
    if (nv > ((int64_t)1 << 31) - 1) return SBA_ELIMIT;
    B.n_edges = nv;
    RC(B.alloc(&B.edges, nv));
    RC(B.alloc(&B.epoly, nv));
    hipLaunchKernelGGL(k_edges, dim3(grid_for(nv)), dim3(256), 0, st, polys->ring_off, np,
                       polys->vert_off, nr, polys->xy, nv, B.edges, B.epoly);
    HIP_OK(hipGetLastError());

    const int64_t s = h->s;
    int64_t gi0 = hsc[3], gj0 = hsc[4], gi1 = hsc[5], gj1 = hsc[6];
    if (B.window) {
        gi0 = std::max(gi0, floordiv64(B.wx0, s));
        gj0 = std::max(gj0, floordiv64(B.wy0, s));
        gi1 = std::min(gi1, floordiv64(B.wx1 - 1, s));
        gj1 = std::min(gj1, floordiv64(B.wy1 - 1, s));
        if (gi0 > gi1 || gj0 > gj1) {  // nothing of any polygon inside the window
            h->gi0 = h->gj0 = 0;
            h->gw = h->gh = 0;
            B.empty = true;
            return 0;
        }
    }
    if (B.key_level > 0) {
        // a given key grid: cells outside it are cut off (at the grid's own
        // edges, which the curve never crosses, so no border keys are
        // needed), and the stored box starts at the grid's first cell
        const int64_t side = (int64_t)1 << B.key_level;
        gi0 = std::max(gi0, B.key_i0);
        gj0 = std::max(gj0, B.key_j0);
        gi1 = std::min(gi1, B.key_i0 + side - 1);
        gj1 = std::min(gj1, B.key_j0 + side - 1);
        if (gi0 > gi1 || gj0 > gj1) {
            h->gi0 = h->gj0 = 0;
            h->gw = h->gh = 0;
            B.empty = true;
            return 0;
        }
        gi0 = B.key_i0;
        gj0 = B.key_j0;
    }
    h->gi0 = gi0;
    h->gj0 = gj0;
    h->gw = gi1 - gi0 + 1;
    h->gh = gj1 - gj0 + 1;
    if (h->gw > MAX_GRID_SIDE || h->gh > MAX_GRID_SIDE) return SBA_ELIMIT;
    if (h->gw * s >= ((int64_t)1 << 31) || h->gh * s >= ((int64_t)1 << 31)) return SBA_ELIMIT;
    const int64_t gw = h->gw, gh = h->gh;
    B.xbits = bits_for((uint64_t)gw);
    B.rbits = bits_for((uint64_t)(gh - 1));
    if (B.rbits < 1) B.rbits = 1;
    const int pbits = bits_for((uint64_t)(np - 1)) < 1 ? 1 : bits_for((uint64_t)(np - 1));

    // 1-2: boundary intervals and crossings per edge
    int64_t *nb = nullptr, *nc = nullptr;
    RC(B.alloc(&nb, nv + 1));
    RC(B.alloc(&nc, nv + 1));
    hipLaunchKernelGGL(k_edge_counts, dim3(grid_for(nv)), dim3(256), 0, st, B.edges, B.epoly, bbox,
                       nv, s, gi0, gj0, gi1, gj1, B.centre ? 1 : 0, nb, nc);
    HIP_OK(hipGetLastError());
    {
        const int64_t *in[2] = {nb, nc}, n[2] = {nv, nv};
        int64_t *out[2] = {nb, nc}, *sum[2] = {tot, tot + 1};
        RC(scan_exclusive_i64_multi(2, in, out, n, sum, st, &B.ws));
    }
    // the events of the coverage, polygon by polygon: the largest polygon's
    // count decides whether they are sorted per polygon in LDS
    EventSegs S{polys->ring_off, polys->vert_off, nb, nc, tot, nv, B.centre ? 0 : 1,
                B.boundary_only ? 0 : 1, 0};
    // per-row toggle counters of the row-bucket path, zeroed by the same launch
    unsigned long long *rowcnt = nullptr;
    RC(B.alloc(&rowcnt, gh + 1));
    hipLaunchKernelGGL(k_event_seg_max, dim3(grid_for(std::max<int64_t>(np, gh + 1))), dim3(256), 0,
                       st, S, np, (unsigned long long *)(B.sc + SC_SEG_MAX), rowcnt, gh);
    HIP_OK(hipGetLastError());
    RC(fetch());
    const int64_t seg_max = hsc[SC_SEG_MAX];
    // boundary-only approximations take no row-line crossings (no interior
    // spans); centre-sampled ones no boundary cells, except as the Hilbert
    // layout's candidate keys (where the cell sets can change along the curve)
    const bool need_b = !B.centre || B.on_boundary_events;
    const int64_t NB = need_b ? hsc[8] : 0, NC = B.boundary_only ? 0 : hsc[9];
    if (NC % 2) return SBA_EDEVICE;
    h->n_boundary = NB;
    B.NB = NB;
    const int64_t NB_cov = B.centre ? 0 : NB;  // boundary intervals in the coverage
    int64_t NE = 2 * NB + NC;
    if (NE >= ((int64_t)1 << 32)) return SBA_ELIMIT;
    RC(B.alloc(&B.evkey, NE));
    RC(B.alloc(&B.evpay, NE));
    uint64_t *ckey = B.evkey + 2 * NB;
    uint32_t *cpay = B.evpay + 2 * NB;
    if (B.centre && NB) {  // crossings in arrays of their own, coverage input alone
        RC(B.alloc(&ckey, std::max<int64_t>(NC, 1)));
        RC(B.alloc(&cpay, std::max<int64_t>(NC, 1)));
    }
    if (NB)
        hipLaunchKernelGGL(k_emit_boundary, dim3(grid_for(NB)), dim3(256), 0, st, B.edges, B.epoly,
                           nv, nb, NB, s, gi0, gj0, gi1, B.xbits, B.rbits, B.evkey, B.evpay);
    if (NC)
        hipLaunchKernelGGL(k_emit_cross, dim3(grid_for(NC)), dim3(256), 0, st, B.edges, B.epoly, nv,
                           nc, NC, s, gi0, gj0, gi1, B.centre ? 1 : 0, B.xbits, B.rbits, ckey,
                           cpay);
    HIP_OK(hipGetLastError());

    // the Hilbert layout needs the boundary cells before the events are sorted
    if (B.on_boundary_events) RC(B.on_boundary_events(B, h, st));
    if (B.centre && NB) {
        B.release(B.evkey);
        B.release(B.evpay);
        B.evkey = ckey;
        B.evpay = cpay;
    }
    NE = 2 * NB_cov + NC;
    // 3: coverage.  Events by (polygon, row, x); one scan gives every
    // polygon's coverage count at every event, whose changes (toggles) are
    // the maximal covered intervals of each polygon in each row.
    const int rxbits = B.rbits + B.xbits;
    int64_t NT = 0;
    uint64_t *tkey = nullptr, *E = nullptr;
    int32_t *tpoly = nullptr;
    int64_t *tf = nullptr;
    // row buckets of the toggles (per-polygon path, rows of at most ROW_CAP
    // toggles): each row's distinct positions are found in one wavefront
    bool rows = false, seg_path = false;
    uint64_t *rb = nullptr;
    int64_t *rowoff = nullptr;
    const int paths_off = g_build_paths_off.load();
    // Clip-window builds (viewport queries) keep the global sorts: they run
    // beside persistent probe kernels that hold most of every compute unit's
    // wave slots and registers, where the per-polygon workgroups of 1024
    // lanes would wait for those kernels to end; their event counts are
    // small, so the global passes cost little there.
    if (NE > 0 && seg_max <= SEG_CAP && rxbits + 2 <= 32 && !(paths_off & 1) && !B.window) {
        // per polygon in LDS: sort, coverage and toggle flags in one launch
        seg_path = true;
        uint64_t *k2 = nullptr;
        uint32_t *v2 = nullptr;
        int32_t *tl = nullptr;
        int64_t *ptot = nullptr, *ptoff = nullptr;
        RC(B.alloc(&k2, NE));
        RC(B.alloc(&v2, NE));
        RC(B.alloc(&tl, NE));
        RC(B.alloc(&ptot, np));
        RC(B.alloc(&ptoff, np));
        S.cbase = B.centre ? 0 : 2 * NB;
        const int cap = (int)std::max<int64_t>(64, (seg_max + 63) & ~(int64_t)63);
        const int lds = (2 * cap + SEG_WAVES * SEG_RADIX) * (int)sizeof(uint32_t);
        (void)hipFuncSetAttribute((const void *)k_event_seg_sort,
                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (2 * SEG_CAP + SEG_WAVES * SEG_RADIX) * (int)sizeof(uint32_t));
        (void)hipGetLastError();
        hipLaunchKernelGGL(k_event_seg_sort, dim3((unsigned)np), dim3(SEG_BLOCK), lds, st, S,
                           B.evkey, B.evpay, rxbits, B.xbits, cap, k2, v2, tl, ptot, err, rowcnt);
        HIP_OK(hipGetLastError());
        RC(B.alloc(&rowoff, gh + 1));
        hipLaunchKernelGGL(k_row_scan_max, dim3(1), dim3(SEG_BLOCK), 0, st, rowcnt, gh, rowoff,
                           (unsigned long long *)(B.sc + SC_ROW_MAX));
        HIP_OK(hipGetLastError());
        B.release(nb);  // the edge offsets: read by the launch above, free after it in stream order
        B.release(nc);
        B.release(B.evkey);
        B.release(B.evpay);
        B.evkey = k2;
        B.evpay = v2;
        RC(scan_exclusive_i64(ptot, ptoff, np, tot, st, &B.ws));
        RC(fetch());
        NT = hsc[8];
        herr = (int)(uint32_t)hsc[0];
        if (herr || (NT & 1)) return SBA_EDEVICE;
        rows = hsc[SC_ROW_MAX] <= ROW_CAP && !(paths_off & 2);
        if (!rows) RC(B.alloc(&tkey, std::max<int64_t>(NT, 1)));
        if (rows) RC(B.alloc(&rb, std::max<int64_t>(NT, 1)));
        RC(B.alloc(&tpoly, std::max<int64_t>(NT, 1)));
        hipLaunchKernelGGL(k_toggle_emit_seg, dim3(grid_for(NE)), dim3(256), 0, st, B.evkey,
                           B.evpay, tl, ptoff, NE, rxbits, B.xbits, tkey, tpoly,
                           rows ? rowoff : nullptr, rowcnt, rb);
        HIP_OK(hipGetLastError());
        B.release(tl);
        B.release(ptot);
        B.release(ptoff);
    } else {
        B.release(nb);
        B.release(nc);
        RC(radix_sort_u64_ws(&B.evkey, &B.evpay, NE, pbits + rxbits, B.ws));
        int64_t *cex = nullptr;
        RC(B.alloc(&cex, NE));
        RC(B.alloc(&tf, NE));
        hipLaunchKernelGGL(k_ev_values, dim3(grid_for(NE)), dim3(256), 0, st, B.evpay, NE, cex);
        HIP_OK(hipGetLastError());
        RC(scan_exclusive_i64(cex, cex, NE, tot, st, &B.ws));
        hipLaunchKernelGGL(k_toggle_flags, dim3(grid_for(NE)), dim3(256), 0, st, B.evkey,
                           B.evpay, cex, NE, B.xbits, tf, err);
        HIP_OK(hipGetLastError());
        RC(scan_exclusive_i64(tf, tf, NE, tot, st, &B.ws));
        RC(fetch());
        NT = hsc[8];
        herr = (int)(uint32_t)hsc[0];
        if (herr || (NT & 1)) return SBA_EDEVICE;
        B.release(cex);
        RC(B.alloc(&tkey, std::max<int64_t>(NT, 1)));
        RC(B.alloc(&tpoly, std::max<int64_t>(NT, 1)));
        hipLaunchKernelGGL(k_toggle_emit, dim3(grid_for(NE)), dim3(256), 0, st, B.evkey, tf, NE,
                           NT, rxbits, tkey, tpoly);
        HIP_OK(hipGetLastError());
    }
    if (tf) B.release(tf);
    B.release(B.evkey);
    B.evkey = nullptr;
    B.release(B.evpay);
    B.evpay = nullptr;

    // 4: elementary pieces between distinct toggle positions of a row, their
    // depth, and the polygons of each piece
    const int64_t NI = NT / 2;                     // covered intervals
    const int64_t NP = std::max<int64_t>(NT, 1);   // pieces (upper bound)
    int64_t *pos = nullptr, *ika = nullptr, *xoff = nullptr, *diff = nullptr, *dex = nullptr;
    int64_t *segc = nullptr, *mm = nullptr;
    RC(B.alloc(&E, NP));
    RC(B.alloc(&pos, NP));
    RC(B.alloc(&ika, std::max<int64_t>(NI, 1)));
    RC(B.alloc(&xoff, std::max<int64_t>(NI, 1)));
    RC(B.alloc(&diff, NP + 1));
    RC(B.alloc(&dex, NP));
    RC(B.alloc(&segc, NP));
    RC(B.alloc(&mm, NP));
    if (NT == 0) HIP_OK(hipMemsetAsync(diff, 0, sizeof(int64_t) * (NP + 1), st));
    if (NT && rows) {
        int64_t *rank = nullptr;
        RC(B.alloc(&rank, NT));
        hipLaunchKernelGGL(k_row_pieces, dim3((unsigned)((gh + ROW_WAVES - 1) / ROW_WAVES)),
                           dim3(64 * ROW_WAVES), 0, st, rb, rowoff, gh, B.xbits, NT, E, rank,
                           diff);
        HIP_OK(hipGetLastError());
        hipLaunchKernelGGL(k_interval_span, dim3(grid_for(NI)), dim3(256), 0, st, rank, NI, ika,
                           xoff);
        HIP_OK(hipGetLastError());
        B.release(rank);
    } else if (NT) {
        if (NT >= ((int64_t)1 << 32)) return SBA_ELIMIT;
        // sorted with each toggle's slot as payload, so that every toggle
        // learns its index in E without a search (the toggle keys are not
        // needed in slot order afterwards)
        uint32_t *src = nullptr;
        int64_t *rank = nullptr;
        RC(B.alloc(&src, NT));
        RC(B.alloc(&rank, NT));
        hipLaunchKernelGGL(k_iota_u32, dim3(grid_for(NT)), dim3(256), 0, st, src, NT);
        HIP_OK(hipGetLastError());
        RC(radix_sort_u64_ws(&tkey, &src, NT, rxbits, B.ws));
        hipLaunchKernelGGL(k_flag_new, dim3(grid_for(NT)), dim3(256), 0, st, tkey, NT, pos);
        HIP_OK(hipGetLastError());
        RC(scan_exclusive_i64(pos, pos, NT, tot + 1, st, &B.ws));
        hipLaunchKernelGGL(k_unique_rank, dim3(grid_for(NT)), dim3(256), 0, st, tkey, NT, pos,
                           tot + 1, src, E, rank, diff);
        HIP_OK(hipGetLastError());
        B.release(src);
        hipLaunchKernelGGL(k_interval_span, dim3(grid_for(NI)), dim3(256), 0, st, rank, NI, ika,
                           xoff);
        HIP_OK(hipGetLastError());
        B.release(rank);
    }
    B.release(pos);
    B.release(rb);
    B.release(rowoff);
    B.release(rowcnt);
    g_build_paths_last = (seg_path ? 1 : 0) | (rows ? 2 : 0);
    RC(scan_exclusive_i64(diff, dex, NP, tot + 2, st, &B.ws));
    hipLaunchKernelGGL(k_piece_classify, dim3(grid_for(NP)), dim3(256), 0, st, dex, diff, NP, segc,
                       mm, err);
    HIP_OK(hipGetLastError());
    {
        const int64_t *in[3] = {segc, mm, xoff}, n[3] = {NP, NP, std::max<int64_t>(NI, 1)};
        int64_t *out[3] = {segc, mm, xoff}, *sum[3] = {tot + 3, tot + 4, tot + 5};
        RC(scan_exclusive_i64_multi(3, in, out, n, sum, st, &B.ws));
    }
    RC(fetch());
    const int64_t *h6 = hsc + 8;
    herr = (int)(uint32_t)hsc[0];
    if (herr & 8) return SBA_ELIMIT;
    if (herr) return SBA_EDEVICE;
    const int64_t NS = h6[3] >> 32, NM = h6[3] & 0xffffffffll, NMEM = h6[4];
    const int64_t NX = NI ? h6[5] : 0;
    if (NS >= ((int64_t)1 << 31)) return SBA_ELIMIT;
    h->n_segments = NS;
    B.NS = NS;
    int64_t *cs = nullptr;
    uint32_t *seg_row = nullptr;
    int32_t *sid = nullptr, *fill = nullptr;
    RC(B.alloc(&cs, gh + 1));
    RC(B.alloc(&B.seg_x0, std::max<int64_t>(NS, 1)));
    RC(B.alloc(&B.seg_x1, std::max<int64_t>(NS, 1)));
    RC(B.alloc(&B.seg_code, std::max<int64_t>(NS, 1)));
    RC(B.alloc(&seg_row, std::max<int64_t>(NS, 1)));
    RC(B.alloc(&sid, NP));
    RC(B.alloc(&fill, NP));
    int64_t *multi_seg = nullptr, *multi_mem = nullptr;
    int32_t *mem_ids = nullptr;
    RC(B.alloc(&multi_seg, std::max<int64_t>(NM, 1)));
    RC(B.alloc(&multi_mem, std::max<int64_t>(NM, 1)));
    RC(B.alloc(&mem_ids, std::max<int64_t>(NMEM, 1)));
    HIP_OK(hipMemsetAsync(fill, 0, sizeof(int32_t) * NP, st));
    if (NX)
        hipLaunchKernelGGL(k_piece_members, dim3(grid_for(NX)), dim3(256), 0, st, xoff, NI, NX,
                           ika, tpoly, dex, diff, mm, sid, fill, mem_ids);
    if (NT)
        hipLaunchKernelGGL(k_piece_emit, dim3(grid_for(NT)), dim3(256), 0, st, E, NT, dex, diff,
                           segc, mm, sid, B.xbits, B.seg_x0, B.seg_x1, B.seg_code, seg_row,
                           multi_seg, multi_mem, mem_ids);
    hipLaunchKernelGGL(k_seg_row_off, dim3(grid_for(gh + 1)), dim3(256), 0, st, seg_row, NS, gh,
                       cs);
    HIP_OK(hipGetLastError());
    B.seg_row_off = cs;
    for (void *p : {(void *)tkey, (void *)tpoly, (void *)E, (void *)ika, (void *)xoff,
                    (void *)diff, (void *)dex, (void *)segc, (void *)mm, (void *)seg_row,
                    (void *)sid, (void *)fill})
        B.release(p);

    // 5: deduplicate the sets of multi-polygon segments
    h->n_sets = 0;
    h->n_set_ids = 0;
    bool set_path = false;
    if (NM > 0) {
        uint64_t *mkey = nullptr;
        uint32_t *mval = nullptr;
        RC(B.alloc(&mkey, NM));
        RC(B.alloc(&mval, NM));
        const int fb = std::min(pbits + 1, 21);  // ids + 1 < 2^21
        const int kbits = std::max(3 * fb + 1, bits_for(((uint64_t)1 << (3 * fb)) | (uint64_t)NM));
        if (kbits > 64) return SBA_ELIMIT;
        hipLaunchKernelGGL(k_multi_keys, dim3(grid_for(NM)), dim3(256), 0, st, multi_mem, NM, NMEM,
                           mem_ids, fb, mkey, mval);
        HIP_OK(hipGetLastError());
        // sizes are bounded by the multi segments (NM sets, NMEM ids), so the
        // set table is laid out before its counts reach the host
        RC(handle_alloc(h, &h->set_off, NM + 1));
        RC(handle_alloc(h, &h->set_ids, NMEM));
        if (kbits <= 31 && !(g_build_paths_off.load() & 4)) {
            // distinct keys through a hash table, sorted by one workgroup
            int hb = 1;
            while (((int64_t)1 << hb) < 2 * NM) hb++;
            if (hb > 31) return SBA_ELIMIT;
            uint32_t *tab = nullptr, *rank = nullptr, *list = nullptr;
            RC(B.alloc(&tab, (int64_t)1 << hb));
            RC(B.alloc(&rank, (int64_t)1 << hb));
            RC(B.alloc(&list, SET_CAP));
            HIP_OK(hipMemsetAsync(tab, 0xff, sizeof(uint32_t) << hb, st));
            unsigned long long *nd = (unsigned long long *)(B.sc + SC_SET_N);
            unsigned long long *nids = (unsigned long long *)(B.sc + SC_SET_IDS);
            hipLaunchKernelGGL(k_set_insert, dim3(grid_for(NM)), dim3(256), 0, st, mkey, NM, tab, hb,
                               list, nd);
            HIP_OK(hipGetLastError());
            constexpr int lds = (2 * SET_CAP + SEG_WAVES * SEG_RADIX) * (int)sizeof(uint32_t);
            (void)hipFuncSetAttribute((const void *)k_set_table,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, lds);
            (void)hipGetLastError();
            hipLaunchKernelGGL(k_set_table, dim3(1), dim3(SEG_BLOCK), lds, st, list, nd, tab, hb,
                               kbits, fb, multi_mem, NM, NMEM, mem_ids, rank, h->set_off,
                               h->set_ids, nids);
            HIP_OK(hipGetLastError());
            hipLaunchKernelGGL(k_set_codes, dim3(grid_for(NM)), dim3(256), 0, st, mkey, NM, nd, tab,
                               hb, rank, multi_seg, B.seg_code);
            HIP_OK(hipGetLastError());
            RC(B.ws.read(hsc, B.sc, sizeof(hsc)));
            RC(B.ws.sync());
            B.release(tab);
            B.release(rank);
            B.release(list);
            if (hsc[SC_SET_N] <= SET_CAP) {
                set_path = true;
                h->n_sets = hsc[SC_SET_N];
                h->n_set_ids = hsc[SC_SET_IDS];
            }
        }
        if (!set_path) {
            // all keys through the global radix sort
            int64_t *g = nullptr, *set_sz = nullptr;
            RC(B.alloc(&g, NM + 1));
            RC(radix_sort_u64_ws(&mkey, &mval, NM, kbits, B.ws));
            hipLaunchKernelGGL(k_flag_new, dim3(grid_for(NM)), dim3(256), 0, st, mkey, NM, g);
            HIP_OK(hipGetLastError());
            RC(scan_exclusive_i64(g, g, NM, tot, st, &B.ws));
            RC(B.alloc(&set_sz, NM + 1));
            HIP_OK(hipMemsetAsync(set_sz, 0, sizeof(int64_t) * (NM + 1), st));
            hipLaunchKernelGGL(k_set_sizes, dim3(grid_for(NM)), dim3(256), 0, st, mkey, mval, g, NM,
                               multi_mem, NM, NMEM, set_sz);
            HIP_OK(hipGetLastError());
            RC(scan_exclusive_i64(set_sz, h->set_off, NM, h->set_off + NM, st, &B.ws));
            hipLaunchKernelGGL(k_set_fill, dim3(grid_for(NM)), dim3(256), 0, st, mkey, mval, g, NM,
                               multi_mem, NM, NMEM, mem_ids, h->set_off, h->set_ids, multi_seg,
                               B.seg_code);
            HIP_OK(hipGetLastError());
            int64_t nids = 0;
            RC(B.ws.read(hsc, B.sc, sizeof(hsc)));
            RC(B.ws.read(&nids, h->set_off + NM, sizeof(int64_t)));
            RC(B.ws.sync());
            h->n_sets = hsc[8];
            h->n_set_ids = nids;
            B.release(g);
            B.release(set_sz);
        }
        B.release(mkey);
        B.release(mval);
    }
    g_build_paths_last = g_build_paths_last.load() | (set_path ? 4 : 0);
    B.release(multi_seg);
    B.release(multi_mem);
    B.release(mem_ids);
    if (h->n_sets >= (int64_t)(TILE_MIXED - CODE_SET_BASE)) return SBA_ELIMIT;
    return 0;
}

// debug switch: store the grid in the 32-bit format even where the compact
// one would fit
bool g_build_wide = false;

template <int G>
static void launch_classify(const BuildState &B, const sba_handle *h, const int64_t *mt, int tl,
                            int sl, int64_t n_sq, uint32_t *code, int64_t *mixed, hipStream_t st)
{
    hipLaunchKernelGGL(k_square_classify<G>, dim3(grid_for(n_sq * G)), dim3(256), 0, st,
                       B.seg_row_off, B.seg_x0, B.seg_x1, B.seg_code, h->gw, h->gh, mt, tl, sl,
                       h->tw, n_sq, code, mixed);
}

static void classify(const BuildState &B, const sba_handle *h, const int64_t *mt, int tl, int sl,
                     int64_t n_sq, uint32_t *code, int64_t *mixed, hipStream_t st)
{
    int side_log2 = mt ? sl : tl;
    if (side_log2 >= 6) launch_classify<64>(B, h, mt, tl, sl, n_sq, code, mixed, st);
    else if (side_log2 == 5) launch_classify<32>(B, h, mt, tl, sl, n_sq, code, mixed, st);
    else if (side_log2 == 4) launch_classify<16>(B, h, mt, tl, sl, n_sq, code, mixed, st);
    else if (side_log2 == 3) launch_classify<8>(B, h, mt, tl, sl, n_sq, code, mixed, st);
    else launch_classify<4>(B, h, mt, tl, sl, n_sq, code, mixed, st);
}

int build_grid(sba_handle *h, BuildState &B, int tile_log2, int sub_log2, hipStream_t st)
{
    int tl = tile_log2;
    if (tl == 0) {
        // the smallest tile whose 16-bit directory, with the probe's LDS bins
        // (12 B per polygon and per set), fits the LDS of a compute unit: the
        // finer the directory, the fewer points need a lookup in global memory
        auto tiles = [&](int t) {
            return ((h->gw + (1 << t) - 1) >> t) * ((h->gh + (1 << t) - 1) >> t);
        };
        auto fits = [&](int t, int64_t bins) {
            int64_t nt16 = (tiles(t) + 7) & ~(int64_t)7;
            return tiles(t) <= COMPACT_DIR_TILES_MAX && nt16 * 2 + bins * 12 <= PROBE_LDS_BYTES;
        };
        const int64_t all = (int64_t)h->n_polys + h->n_sets;
        tl = 2;
        while (tl < 10 && !fits(tl, all)) tl++;
        if (!fits(tl, all)) {  // set bins never fit: directory and polygon bins
            tl = 2;
            while (tl < 10 && !fits(tl, h->n_polys)) tl++;
            if (!fits(tl, h->n_polys)) {  // polygon bins do not fit either
                tl = 2;
                while (tl < 10 && tiles(tl) > COMPACT_DIR_TILES) tl++;
            }
        }
    }
    if (tl < 2 || tl > 10) return SBA_EINVAL;
    // sub-tiles of 16 x 16 cells under big tiles, of 8 x 8 under tiles of 32
    // (until the mixed tiles are known, see below)
    int sl = sub_log2 ? sub_log2 : (tl >= 6 ? 4 : (tl == 5 ? 3 : tl));
    if (sl < 1 || sl > tl) return SBA_EINVAL;
    h->tile_log2 = tl;
    h->sub_log2 = sl;
    h->tw = (h->gw + (1 << tl) - 1) >> tl;
    h->th = (h->gh + (1 << tl) - 1) >> tl;
    const int64_t nt = h->tw * h->th;
    if (nt >= ((int64_t)1 << 31)) return SBA_ELIMIT;
    const uint32_t np = (uint32_t)h->n_polys;
    uint32_t *tcode = nullptr;
    int64_t *tpos = nullptr, *tot = B.sc + 16;
    int64_t hsc[SC_READ];
    RC(B.alloc(&tcode, nt));
    RC(B.alloc(&tpos, nt + 1));
    classify(B, h, nullptr, tl, sl, nt, tcode, tpos, st);
    HIP_OK(hipGetLastError());
    RC(scan_exclusive_i64(tpos, tpos, nt, tot, st, &B.ws));
    RC(B.ws.read(hsc, B.sc, sizeof(hsc)));
    RC(B.ws.sync());
    const int64_t nblk = hsc[16];
    if (nblk >= (int64_t)TILE_MIXED) return SBA_ELIMIT;
    h->n_blocks = nblk;
    const bool compact = !g_build_wide && (int64_t)np + h->n_sets < 0x8000 && nblk < 0x8000 &&
                         nt <= COMPACT_DIR_TILES_MAX;
    h->compact = compact;
    if (sub_log2 == 0 && compact && nblk > 0) {
        // the smallest sub-tile whose 16-bit sub-directory fits the LDS of a
        // compute unit beside the directory and the bins: the probe then
        // stages it there, and only points in mixed sub-tiles read a fine
        // block from global memory
        const int64_t dir = ((nt + 7) & ~(int64_t)7) * 2, bins = ((int64_t)np + h->n_sets) * 12;
        for (int t = 1; t < tl; t++) {
            const int64_t ne = ((nblk << (2 * (tl - t))) + 7) & ~(int64_t)7;
            if (dir + ne * 2 + bins <= PROBE_LDS_BYTES) {
                sl = t;
                break;
            }
        }
        h->sub_log2 = sl;
    }

    // directory
    if (compact) {
        const int64_t nt16 = (nt + 7) & ~(int64_t)7;  // LDS copies move 16 bytes at a time
        RC(handle_alloc(h, &h->dir16, nt16));
        hipLaunchKernelGGL(k_entries, dim3(grid_for(nt16)), dim3(256), 0, st, tcode, tpos, nt, nt16,
                           np, 2, (uint32_t *)nullptr, h->dir16);
    } else {
        RC(handle_alloc(h, &h->dir, nt));
        hipLaunchKernelGGL(k_entries, dim3(grid_for(nt)), dim3(256), 0, st, tcode, tpos, nt, nt, np,
                           0, h->dir, (uint16_t *)nullptr);
    }
    HIP_OK(hipGetLastError());
    if (nblk == 0) {
        // one-element placeholders: the batched lookups read element 0 of
        // the lower levels for points that need nothing from them
        if (sl < tl) {
            RC(handle_alloc(h, &h->sub, 1));
            HIP_OK(hipMemsetAsync(h->sub, 0, 4, st));
        }
        if (compact) {
            RC(handle_alloc(h, &h->blocks16, 1));
            HIP_OK(hipMemsetAsync(h->blocks16, 0, 2, st));
        } else {
            RC(handle_alloc(h, &h->blocks, 1));
            HIP_OK(hipMemsetAsync(h->blocks, 0, 4, st));
        }
        return 0;
    }
    int64_t *mt = nullptr;  // mixed tiles in order
    RC(B.alloc(&mt, nblk));
    hipLaunchKernelGGL(k_flag_list, dim3(grid_for(nt)), dim3(256), 0, st, tpos, nt, nblk, mt);
    HIP_OK(hipGetLastError());

    // sub-directories of the mixed tiles
    const int64_t *fine_sq = mt;        // squares stored as fine blocks
    const int64_t *fine_mt = nullptr;   // their tile list (sub-tiles) or NULL (tiles)
    int64_t nfine = nblk;
    int fine_log2 = tl;
    if (sl < tl) {
        const int64_t nq = nblk << (2 * (tl - sl));
        uint32_t *scode = nullptr;
        int64_t *spos = nullptr, *ms = nullptr;
        RC(B.alloc(&scode, nq));
        RC(B.alloc(&spos, nq + 1));
        classify(B, h, mt, tl, sl, nq, scode, spos, st);
        HIP_OK(hipGetLastError());
        RC(scan_exclusive_i64(spos, spos, nq, tot + 1, st, &B.ws));
        RC(B.ws.read(hsc, B.sc, sizeof(hsc)));
        RC(B.ws.sync());
        const int64_t nsub = hsc[17];
        if (nsub >= (int64_t)TILE_MIXED) return SBA_ELIMIT;
        h->n_sub = nsub;
        RC(handle_alloc(h, &h->sub, nq));
        hipLaunchKernelGGL(k_entries, dim3(grid_for(nq)), dim3(256), 0, st, scode, spos, nq, nq, np,
                           compact ? 1 : 0, h->sub, (uint16_t *)nullptr);
        HIP_OK(hipGetLastError());
        RC(B.alloc(&ms, std::max<int64_t>(nsub, 1)));
        hipLaunchKernelGGL(k_flag_list, dim3(grid_for(nq)), dim3(256), 0, st, spos, nq, nsub, ms);
        HIP_OK(hipGetLastError());
        fine_sq = ms;
        fine_mt = mt;
        nfine = nsub;
        fine_log2 = sl;
    }

    // fine blocks
    const int64_t cells = nfine << (2 * fine_log2);
    const int side = 1 << fine_log2;
    const int64_t threads = nfine * side * (side > 16 ? side >> 4 : 1);
    if (compact) {
        RC(handle_alloc(h, &h->blocks16, std::max<int64_t>(cells, 1)));
        if (nfine)
            hipLaunchKernelGGL(k_block_fill<uint16_t>, dim3(grid_for(threads)), dim3(256), 0, st,
                               B.seg_row_off, B.seg_x0, B.seg_x1, B.seg_code, h->gw, h->gh, fine_sq,
                               nfine, fine_mt, tl, sl, h->tw, fine_log2, np, h->blocks16);
    } else {
        RC(handle_alloc(h, &h->blocks, std::max<int64_t>(cells, 1)));
        if (nfine)
            hipLaunchKernelGGL(k_block_fill<uint32_t>, dim3(grid_for(threads)), dim3(256), 0, st,
                               B.seg_row_off, B.seg_x0, B.seg_x1, B.seg_code, h->gw, h->gh, fine_sq,
                               nfine, fine_mt, tl, sl, h->tw, fine_log2, np, h->blocks);
    }
    HIP_OK(hipGetLastError());
    return 0;
}

int segments_lookup(const BuildState &B, const sba_handle *h, const int64_t *ij, int64_t n,
                    uint32_t *out, hipStream_t st)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_lookup_ij, dim3(grid_for(n)), dim3(256), 0, st, B.seg_row_off, B.seg_x0,
                       B.seg_x1, B.seg_code, h->gi0, h->gj0, h->gw, h->gh, ij, n, out);
    HIP_OK(hipGetLastError());
    return 0;
}

int build_handle(const sba_polygons *polys, int64_t eps, const sba_build_opts *opts,
                 hipStream_t st, sba_handle *h)
{
    auto t0 = std::chrono::steady_clock::now();
    sba_build_opts o{};
    o.kind = SBA_KIND_GRID;
    o.search = SBA_SEARCH_BINARY;
    o.log2_leaves = 16;
    if (opts) o = *opts;
    if ((o.alloc == nullptr) != (o.release == nullptr)) return SBA_EINVAL;
    h->ua = UserAlloc{o.alloc, o.release, o.alloc_ctx};
    if (o.use_window && (o.win_x1 <= o.win_x0 || o.win_y1 <= o.win_y0)) return SBA_EINVAL;
    if (o.log2_leaves == 0) o.log2_leaves = 16;
    if (o.kind != SBA_KIND_GRID && o.kind != SBA_KIND_HILBERT) return SBA_EINVAL;
    if (o.search != SBA_SEARCH_BINARY && o.search != SBA_SEARCH_LEARNED) return SBA_EINVAL;
    if (o.log2_leaves < 1 || o.log2_leaves > 24) return SBA_EINVAL;
    if (o.key_level < 0 || o.key_level > 21 || (o.key_level > 0 && o.kind != SBA_KIND_HILBERT))
        return SBA_EINVAL;
    if (o.centre_sampled != 0 && o.centre_sampled != 1) return SBA_EINVAL;
    if (o.centre_sampled && o.boundary_only) return SBA_EINVAL;
    if (o.key_level > 0 && (o.key_i0 < -((int64_t)1 << 31) || o.key_i0 >= ((int64_t)1 << 31) ||
                            o.key_j0 < -((int64_t)1 << 31) || o.key_j0 >= ((int64_t)1 << 31)))
        return SBA_EINVAL;
    h->kind = o.kind;
    h->search = o.search;
    h->eps = eps;
    const int64_t s = cell_side(eps);
    h->s = s;
    magic_for(s, &h->mag, &h->shift);
    h->n_polys = polys->n_polys;
    if (polys->n_polys == 0) {
        h->gw = h->gh = 0;
        h->build_ms = 0;
        return 0;
    }
    BuildState B(st);
    B.ws.set_allocator(h->ua);
    B.boundary_only = o.boundary_only != 0;
    h->boundary_only = o.boundary_only != 0;
    B.centre = o.centre_sampled != 0;
    h->centre_sampled = o.centre_sampled != 0;
    B.window = o.use_window != 0;
    B.wx0 = o.win_x0;
    B.wy0 = o.win_y0;
    B.wx1 = o.win_x1;
    B.wy1 = o.win_y1;
    B.key_level = o.key_level;
    B.key_i0 = o.key_i0;
    B.key_j0 = o.key_j0;
    if (h->kind == SBA_KIND_HILBERT) RC(hilbert_prepare(B, h));
    RC(build_segments(polys, eps, st, h, B, h->kind == SBA_KIND_HILBERT));
    if (B.empty) {
        HIP_OK(hipStreamSynchronize(st));
        h->build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
                          .count();
        return 0;
    }
    if (h->kind == SBA_KIND_GRID) {
        RC(build_grid(h, B, o.tile_log2, o.sub_log2, st));
    } else {
        RC(hilbert_finish(B, h, o, st));
    }
    HIP_OK(hipStreamSynchronize(st));
    auto t1 = std::chrono::steady_clock::now();
    h->build_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    return 0;
}
