// pindex.hip -- point-side pre-aggregation (Sec. 3, point indexing).
//
// The points are mapped to the cells of the same grid as the polygon
// approximations (side s(eps)), the cells linearised with the Hilbert curve,
// and the keys sorted; the values are permuted the same way and turned into
// an exclusive prefix-sum array.  Then for any key range [a, b)
//     COUNT = lb(b) - lb(a),   SUM = prefix[lb(b)] - prefix[lb(a)],
// with lb the lower bound in the sorted keys.  A Hilbert handle built on the
// index's key grid stores its approximation as runs of consecutive keys with
// one polygon set each, so a polygon query costs two lower bounds per run (a
// run is a union of aligned quadtree cells, the query cells of the method)
// and no pass over the points.
//
// Lower bounds come from a binary search or from a RadixSpline (Sec. 3):
// spline knots on the step function F(v) = lb(v) with every key's error at
// most E positions, and a radix table over the top bits of the key that
// narrows the knot search.  The estimate is followed by a binary search in a
// window of 2E + 3 positions, checked at both ends, and a full binary search
// if the check ever fails.
//
// Spline (greedy corridor, Neumann & Michel 2008, the construction RadixSpline
// uses): F is a step function, so it is enough to bound the error at the two
// ends of every step: for distinct keys D_0 < ... < D_{M-1} with first
// positions P_m, the corners (D_{m-1} + 1, P_m) and (D_m, P_m) (D_{-1} + 1 =
// 0), then (D_{M-1} + 1, n) and (4^L, n).  The distinct keys are cut into
// chunks; one thread runs the greedy corridor over the corners of each chunk
// from its first to its last corner (both become knots).  Two consecutive
// corners are exact on every integer key between them, so the chunk seams add
// no error.
#include <chrono>
#include <new>
#include <vector>

#include "sba_internal.h"

struct sba_pindex {
    int device = 0;
    int64_t n = 0, eps = 0, s = 0;
    int64_t gi0 = 0, gj0 = 0;  // key grid origin (cells)
    int32_t L = 1;             // key grid side 2^L cells
    uint32_t mag = 0;
    int32_t shift = 0;
    uint64_t *keys = nullptr;  // [n] ascending Hilbert keys of the points' cells
    int64_t *psum = nullptr;   // [n + 1] exclusive prefix sums of the values (NULL: none)
    int64_t n_distinct = 0;
    // RadixSpline
    int32_t radix_bits = 0, spline_err = 0, rshift = 0;
    int64_t n_knots = 0;
    uint64_t *kx = nullptr;    // [n_knots] knot keys, kx[0] = 0, last = 4^L, non-decreasing
    int64_t *ky = nullptr;     // [n_knots] knot positions
    uint32_t *rtab = nullptr;  // [2^radix_bits + 2] knots whose key prefix is below p
    int64_t bytes = 0;
    double build_ms = 0;
    std::vector<DevBlock> owned;
};

template <typename T>
static int ix_alloc(sba_pindex *ix, T **p, int64_t n)
{
    DevBlock b{};
    const size_t bytes = (size_t)(n > 0 ? n : 1) * sizeof(T);
    RC(cache_get(bytes, &b));
    ix->owned.push_back(b);
    ix->bytes += (int64_t)bytes;
    *p = (T *)b.p;
    return 0;
}

static void ix_release(sba_pindex *ix)
{
    for (const DevBlock &b : ix->owned) cache_put(b);
    ix->owned.clear();
}

// ---------------------------------------------------------------- build kernels

__global__ void k_box_init(int32_t *b)
{
    if (threadIdx.x == 0) {
        b[0] = INT32_MAX;
        b[1] = INT32_MAX;
        b[2] = INT32_MIN;
        b[3] = INT32_MIN;
    }
}

// min x, min y, max x, max y of the points
__global__ void k_box(const int32_t *__restrict__ xy, int64_t n, int32_t *b)
{
    int32_t x0 = INT32_MAX, y0 = INT32_MAX, x1 = INT32_MIN, y1 = INT32_MIN;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int2 p = ((const int2 *)xy)[t];
        x0 = min(x0, p.x);
        y0 = min(y0, p.y);
        x1 = max(x1, p.x);
        y1 = max(y1, p.y);
    }
    for (int o = 32; o > 0; o >>= 1) {
        x0 = min(x0, __shfl_xor(x0, o, 64));
        y0 = min(y0, __shfl_xor(y0, o, 64));
        x1 = max(x1, __shfl_xor(x1, o, 64));
        y1 = max(y1, __shfl_xor(y1, o, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMin(&b[0], x0);
        atomicMin(&b[1], y0);
        atomicMax(&b[2], x1);
        atomicMax(&b[3], y1);
    }
}

// Hilbert key of each point's cell (the box holds every point, so the
// offsets from the grid origin lie in [0, 2^31))
__global__ void k_point_keys(const int32_t *__restrict__ xy, int64_t n, int64_t ox, int64_t oy,
                             uint32_t mag, int32_t shift, int L, uint64_t *keys, uint32_t *idx)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int2 p = ((const int2 *)xy)[t];
    const uint32_t i = divmagic((uint32_t)((int64_t)p.x - ox), mag, shift);
    const uint32_t j = divmagic((uint32_t)((int64_t)p.y - oy), mag, shift);
    keys[t] = hilbert_index(L, i, j);
    idx[t] = (uint32_t)t;
}

__global__ void k_gather_values(const int64_t *__restrict__ values, const uint32_t *__restrict__ idx,
                                int64_t n, int64_t *out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) out[t] = values[idx[t]];
}

__global__ void k_distinct_flags(const uint64_t *keys, int64_t n, int64_t *flag)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) flag[t] = (t == 0 || keys[t] != keys[t - 1]) ? 1 : 0;
}

__global__ void k_distinct_write(const uint64_t *keys, int64_t n, const int64_t *pos, uint64_t *D,
                                 int64_t *P)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    if (t == 0 || keys[t] != keys[t - 1]) {
        D[pos[t]] = keys[t];
        P[pos[t]] = t;
    }
}

struct Corners {
    const uint64_t *D;
    const int64_t *P;
    int64_t M, n;
    uint64_t total;
};

// Greedy corridor over the corners of the distinct keys [c*CHM, min((c+1)*CHM,
// M)) (the last chunk also takes the two corners after the last key): the
// knot moves to the previous corner as soon as a corner's slope from the knot
// leaves the band of slopes that keeps every corner since the knot within E.
// Slopes are compared as cross products (no divisions; positive run lengths).
// Pass 1 counts the knots, pass 2 writes them at off[c] (off[nch] = total).
#define SPLINE_PF 8

template <bool WRITE>
__global__ void k_spline(Corners C, int64_t CHM, double E, int64_t *cnt, const int64_t *off,
                         uint64_t *kx, int64_t *ky)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t a = c * CHM;
    if (a >= C.M) return;
    const int64_t b = min(a + CHM, C.M);
    int64_t k = 0;
    const int64_t base = WRITE ? off[c] : 0, lim = WRITE ? off[c + 1] - base : 0;
    auto emit = [&](uint64_t x, int64_t y) {
        if (WRITE && k < lim) {  // the second pass repeats the first one's count
            kx[base + k] = x;
            ky[base + k] = y;
        }
        k++;
    };
    uint64_t x0 = a == 0 ? 0 : C.D[a - 1] + 1, lx;
    int64_t y0 = C.P[a], ly;
    emit(x0, y0);
    lx = x0;
    ly = y0;
    double un = 0, ud = 1, ln = 0, ld = 1;  // band: slopes in [ln/ld, un/ud]
    bool band = false;
    auto feed = [&](uint64_t x, int64_t y) {
        if (x == lx) return;  // the same corner again (equal keys, equal positions)
        double dx = (double)(x - x0), dy = (double)(y - y0);
        if (band && (dy * ud > un * dx || dy * ld < ln * dx)) {
            emit(lx, ly);
            x0 = lx;
            y0 = ly;
            dx = (double)(x - x0);
            dy = (double)(y - y0);
            band = false;
        }
        if (!band || (dy + E) * ud < un * dx) {
            un = dy + E;
            ud = dx;
        }
        if (!band || (dy - E) * ld > ln * dx) {
            ln = dy - E;
            ld = dx;
        }
        band = true;
        lx = x;
        ly = y;
    };
    uint64_t prev = C.D[a];
    feed(prev, y0);
    // the chunk's keys and positions are read SPLINE_PF at a time, all loads
    // issued before the corridor consumes them: one memory round trip per
    // SPLINE_PF keys instead of one per key
    for (int64_t m0 = a + 1; m0 < b; m0 += SPLINE_PF) {
        uint64_t dd[SPLINE_PF];
        int64_t pp[SPLINE_PF];
#pragma unroll
        for (int t = 0; t < SPLINE_PF; t++) {
            const int64_t m = m0 + t < b ? m0 + t : b - 1;
            dd[t] = C.D[m];
            pp[t] = C.P[m];
        }
#pragma unroll
        for (int t = 0; t < SPLINE_PF; t++) {
            if (m0 + t < b) {
                feed(prev + 1, pp[t]);
                feed(dd[t], pp[t]);
                prev = dd[t];
            }
        }
    }
    if (b == C.M) {
        feed(prev + 1, C.n);
        feed(C.total, C.n);
    }
    if (lx != x0) emit(lx, ly);
    if (!WRITE) cnt[c] = k;
}

// rtab[p] = number of knots whose key is below p << rshift
__global__ void k_radix_table(const uint64_t *kx, int64_t nk, int32_t rshift, int64_t entries,
                              uint32_t *rtab)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= entries) return;
    const uint64_t v = (uint64_t)p << rshift;
    int64_t lo = 0, hi = nk;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (kx[mid] < v) lo = mid + 1; else hi = mid;
    }
    rtab[p] = (uint32_t)lo;
}

// ---------------------------------------------------------------- query

struct IxView {
    const uint64_t *keys;
    const int64_t *psum;
    int64_t n;
    uint64_t total;  // 4^L
    const uint64_t *kx;
    const int64_t *ky;
    const uint32_t *rtab;
    int64_t nk;
    int32_t rshift, err;
};

struct RunsView {
    const uint64_t *starts;
    const uint32_t *code;
    int64_t n;
    const int64_t *set_off;
    const int32_t *set_ids;
    uint32_t np, n_sets;
};

// first position in [lo, hi) whose key is >= v (hi if none)
__device__ __forceinline__ int64_t lower_bound_in(const uint64_t *keys, int64_t lo, int64_t hi,
                                                  uint64_t v)
{
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (keys[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ int64_t rs_lower_bound(const IxView &V, uint64_t v,
                                                  unsigned long long *fallbacks = nullptr)
{
    // last knot with key <= v lies in [rtab[p] - 1, rtab[p+1] - 1]
    const uint64_t p = v >> V.rshift;
    int64_t lo = V.rtab[p], hi = (int64_t)V.rtab[p + 1] - 1;
    lo = lo > 0 ? lo - 1 : 0;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (V.kx[mid] <= v) lo = mid; else hi = mid - 1;
    }
    double y = (double)V.ky[lo];
    if (lo + 1 < V.nk)
        y += (double)(v - V.kx[lo]) * (double)(V.ky[lo + 1] - V.ky[lo]) /
             (double)(V.kx[lo + 1] - V.kx[lo]);
    const int64_t est = (int64_t)y;
    int64_t a = est - V.err - 1, b = est + V.err + 2;
    a = a < 0 ? 0 : (a > V.n ? V.n : a);
    b = b < a ? a : (b > V.n ? V.n : b);
    // the answer lies in [a, b] when the keys just outside the window agree
    if ((a == 0 || V.keys[a - 1] < v) && (b == V.n || V.keys[b] >= v))
        return lower_bound_in(V.keys, a, b, v);
    if (fallbacks) atomicAdd(fallbacks, 1ull);
    return lower_bound_in(V.keys, 0, V.n, v);
}

// (count, sum) of a run to its polygon or to every member of its set
template <bool VALS>
__device__ __forceinline__ void add_run(const RunsView &R, uint32_t code, unsigned long long c,
                                        unsigned long long sv, unsigned long long *counts,
                                        unsigned long long *sums)
{
    if (code < CODE_SET_BASE) {
        const uint32_t p = code - 1u;
        if (p >= R.np) return;
        atomicAdd(&counts[p], c);
        if (VALS) atomicAdd(&sums[p], sv);
    } else {
        const uint32_t k = code - CODE_SET_BASE;
        if (k >= R.n_sets) return;
        for (int64_t q = R.set_off[k], e = R.set_off[k + 1]; q < e; q++) {
            const uint32_t p = (uint32_t)R.set_ids[q];
            if (p >= R.np) continue;
            atomicAdd(&counts[p], c);
            if (VALS) atomicAdd(&sums[p], sv);
        }
    }
}

// A wavefront takes 63 consecutive runs: lane k finds the lower bound of
// start k (start R.n is 4^L), so run k's points are [lb_k, lb_{k+1}) with
// one search per lane.  Lanes with the same code then combine their counts
// and sums (runs along the curve meet few polygons), and one lane per code
// adds them to the outputs.
template <bool VALS, bool RS>
__global__ __launch_bounds__(256) void k_pindex_agg(IxView V, RunsView R,
                                                    unsigned long long *counts,
                                                    unsigned long long *sums)
{
    const int lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; w * 63 < R.n;
         w += nw) {
        const int64_t t = w * 63 + lane;
        int64_t lb = 0;
        if (t <= R.n) {
            const uint64_t v = t < R.n ? R.starts[t] : V.total;
            lb = RS ? rs_lower_bound(V, v) : lower_bound_in(V.keys, 0, V.n, v);
        }
        const int64_t ub = __shfl_down(lb, 1, 64);
        uint32_t code = 0;
        unsigned long long c = 0, sv = 0;
        if (lane < 63 && t < R.n) {
            code = R.code[t];
            c = (unsigned long long)(ub - lb);
            if (VALS && c) sv = (unsigned long long)(V.psum[ub] - V.psum[lb]);
            if (c == 0) code = 0;
        }
        unsigned long long todo = __ballot(code != 0);
        while (todo) {
            const int leader = __ffsll((long long)todo) - 1;
            const uint32_t lc = __shfl(code, leader, 64);
            const bool mine = code == lc;
            unsigned long long cc = mine ? c : 0ull, ss = mine ? sv : 0ull;
            for (int o = 32; o > 0; o >>= 1) {
                cc += __shfl_xor(cc, o, 64);
                if (VALS) ss += __shfl_xor(ss, o, 64);
            }
            if (lane == leader) add_run<VALS>(R, lc, cc, ss, counts, sums);
            todo &= ~__ballot(mine);
        }
    }
}

__global__ void k_pindex_zero(uint64_t *counts, int64_t *sums, int32_t np)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    counts[p] = 0;
    if (sums) sums[p] = 0;
}

// ---------------------------------------------------------------- build

static int pindex_build(const int32_t *xy, const int64_t *values, int64_t n, sba_pindex *ix,
                        hipStream_t st)
{
    Workspace ws(st);
    if (n == 0) return 0;
    int32_t *box = nullptr;
    RC(ws.alloc(&box, 4));
    hipLaunchKernelGGL(k_box_init, dim3(1), dim3(64), 0, st, box);
    hipLaunchKernelGGL(k_box, dim3(std::min<unsigned>(grid_for(n), 2048)), dim3(256), 0, st, xy,
                       n, box);
    HIP_OK(hipGetLastError());
    int32_t hb[4];
    RC(ws.read(hb, box, sizeof(hb)));
    RC(ws.sync());
    const int64_t s = ix->s;
    const int64_t gi0 = floordiv64(hb[0], s), gj0 = floordiv64(hb[1], s);
    const int64_t gw = floordiv64(hb[2], s) - gi0 + 1, gh = floordiv64(hb[3], s) - gj0 + 1;
    if (gw > MAX_GRID_SIDE || gh > MAX_GRID_SIDE) return SBA_ELIMIT;
    if (gw * s >= ((int64_t)1 << 31) || gh * s >= ((int64_t)1 << 31)) return SBA_ELIMIT;
    int L = 1;
    while (((int64_t)1 << L) < std::max(gw, gh)) L++;
    ix->gi0 = gi0;
    ix->gj0 = gj0;
    ix->L = L;
    const uint64_t total = (uint64_t)1 << (2 * L);

    // keys, sorted with the point index as payload
    uint64_t *keys = nullptr;
    uint32_t *idx = nullptr;
    RC(ws.alloc(&keys, n));
    RC(ws.alloc(&idx, n));
    hipLaunchKernelGGL(k_point_keys, dim3(grid_for(n)), dim3(256), 0, st, xy, n, gi0 * s, gj0 * s,
                       ix->mag, ix->shift, L, keys, idx);
    HIP_OK(hipGetLastError());
    RC(radix_sort_u64_ws(&keys, &idx, n, 2 * L, ws));
    RC(ix_alloc(ix, &ix->keys, n));
    HIP_OK(hipMemcpyAsync(ix->keys, keys, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, st));
    ws.put(keys);

    // values in key order, exclusive prefix sums, total at psum[n]
    if (values) {
        int64_t *v = nullptr;
        RC(ws.alloc(&v, n));
        hipLaunchKernelGGL(k_gather_values, dim3(grid_for(n)), dim3(256), 0, st, values, idx, n, v);
        HIP_OK(hipGetLastError());
        RC(ix_alloc(ix, &ix->psum, n + 1));
        RC(scan_exclusive_i64(v, ix->psum, n, ix->psum + n, st, &ws));
        ws.put(v);
    }
    ws.put(idx);

    // distinct keys and their first positions
    int64_t *flag = nullptr, *tot = nullptr;
    RC(ws.alloc(&flag, n + 1));
    RC(ws.alloc(&tot, 1));
    hipLaunchKernelGGL(k_distinct_flags, dim3(grid_for(n)), dim3(256), 0, st, ix->keys, n, flag);
    HIP_OK(hipGetLastError());
    RC(scan_exclusive_i64(flag, flag, n, tot, st, &ws));
    int64_t M = 0;
    RC(ws.read(&M, tot, sizeof(int64_t)));
    RC(ws.sync());
    ix->n_distinct = M;
    uint64_t *D = nullptr;
    int64_t *P = nullptr;
    RC(ws.alloc(&D, M));
    RC(ws.alloc(&P, M));
    hipLaunchKernelGGL(k_distinct_write, dim3(grid_for(n)), dim3(256), 0, st, ix->keys, n, flag, D,
                       P);
    HIP_OK(hipGetLastError());
    ws.put(flag);

    // RadixSpline knots over the corners of F, then the radix table
    const Corners C{D, P, M, n, total};
    const int64_t CHM = 1024, nch = (M + CHM - 1) / CHM;
    int64_t *cnt = nullptr;
    RC(ws.alloc(&cnt, nch + 1));
    hipLaunchKernelGGL(k_spline<false>, dim3(grid_for(nch)), dim3(256), 0, st, C, CHM,
                       (double)ix->spline_err, cnt, (const int64_t *)nullptr, (uint64_t *)nullptr,
                       (int64_t *)nullptr);
    HIP_OK(hipGetLastError());
    RC(scan_exclusive_i64(cnt, cnt, nch, cnt + nch, st, &ws));
    int64_t nk = 0;
    RC(ws.read(&nk, cnt + nch, sizeof(int64_t)));
    RC(ws.sync());
    ix->n_knots = nk;
    RC(ix_alloc(ix, &ix->kx, nk));
    RC(ix_alloc(ix, &ix->ky, nk));
    hipLaunchKernelGGL(k_spline<true>, dim3(grid_for(nch)), dim3(256), 0, st, C, CHM,
                       (double)ix->spline_err, (int64_t *)nullptr, (const int64_t *)cnt, ix->kx,
                       ix->ky);
    HIP_OK(hipGetLastError());
    ix->radix_bits = std::min(ix->radix_bits, 2 * L);
    ix->rshift = 2 * L - ix->radix_bits;
    const int64_t entries = ((int64_t)1 << ix->radix_bits) + 2;
    RC(ix_alloc(ix, &ix->rtab, entries));
    hipLaunchKernelGGL(k_radix_table, dim3(grid_for(entries)), dim3(256), 0, st, ix->kx, nk,
                       ix->rshift, entries, ix->rtab);
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(st));
    return 0;
}

extern "C" int sba_pindex_build(const int32_t *xy, const int64_t *values, int64_t n, int64_t eps,
                                const sba_pindex_opts *opts, void *stream, sba_pindex **out)
{
    if (!out) return SBA_EINVAL;
    *out = nullptr;
    if (n < 0 || (n > 0 && !xy)) return SBA_EINVAL;
    if (((uintptr_t)xy & 7) != 0 || ((uintptr_t)values & 7) != 0) return SBA_EINVAL;
    if (eps < 2 || eps > ((int64_t)1 << 28)) return SBA_EINVAL;
    if (n >= ((int64_t)1 << 31)) return SBA_ELIMIT;
    sba_pindex_opts o{0, 0};
    if (opts) o = *opts;
    if (o.radix_bits == 0) o.radix_bits = 20;
    if (o.spline_err == 0) o.spline_err = 32;
    if (o.radix_bits < 1 || o.radix_bits > 28 || o.spline_err < 1 || o.spline_err > (1 << 20))
        return SBA_EINVAL;
    auto t0 = std::chrono::steady_clock::now();
    sba_pindex *ix = new (std::nothrow) sba_pindex();
    if (!ix) return SBA_ENOMEM;
    (void)hipGetDevice(&ix->device);
    ix->n = n;
    ix->eps = eps;
    ix->s = cell_side(eps);
    magic_for(ix->s, &ix->mag, &ix->shift);
    ix->radix_bits = o.radix_bits;
    ix->spline_err = o.spline_err;
    const int rc = pindex_build(xy, values, n, ix, (hipStream_t)stream);
    if (rc) {
        (void)hipStreamSynchronize((hipStream_t)stream);
        ix_release(ix);
        delete ix;
        return rc;
    }
    ix->build_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = ix;
    return SBA_OK;
}

extern "C" int sba_pindex_info(const sba_pindex *ix, sba_pindex_info_t *info)
{
    if (!ix || !info) return SBA_EINVAL;
    sba_pindex_info_t o{};
    o.n = ix->n;
    o.eps = ix->eps;
    o.s = ix->s;
    o.key_i0 = ix->gi0;
    o.key_j0 = ix->gj0;
    o.key_level = ix->L;
    o.has_values = ix->psum != nullptr || ix->n == 0 ? 1 : 0;
    o.n_distinct = ix->n_distinct;
    o.n_knots = ix->n_knots;
    o.radix_bits = ix->radix_bits;
    o.spline_err = ix->spline_err;
    o.bytes = ix->bytes;
    o.build_ms = ix->build_ms;
    *info = o;
    return SBA_OK;
}

extern "C" int sba_pindex_aggregate(const sba_pindex *ix, const sba_handle *h, int32_t search,
                                    uint64_t *counts, int64_t *sums, void *stream)
{
    if (!ix || !h) return SBA_EINVAL;
    if (search != SBA_SEARCH_BINARY && search != SBA_SEARCH_LEARNED) return SBA_EINVAL;
    if (h->n_polys > 0 && !counts) return SBA_EINVAL;
    if (sums && ix->n > 0 && !ix->psum) return SBA_EINVAL;
    if (h->n_polys == 0) return 0;
    hipStream_t st = (hipStream_t)stream;
    if (h->kind != SBA_KIND_HILBERT || h->s != ix->s) return SBA_EINVAL;
    const bool has_cells = h->gw > 0 && h->n_runs > 0;
    if (has_cells && (h->level != ix->L || h->gi0 != ix->gi0 || h->gj0 != ix->gj0))
        return SBA_EINVAL;
    hipLaunchKernelGGL(k_pindex_zero, dim3(grid_for(h->n_polys)), dim3(256), 0, st, counts, sums,
                       h->n_polys);
    HIP_OK(hipGetLastError());
    if (!has_cells || ix->n == 0) return 0;
    const IxView V{ix->keys, ix->psum, ix->n, (uint64_t)1 << (2 * ix->L), ix->kx, ix->ky,
                   ix->rtab, ix->n_knots, ix->rshift, ix->spline_err};
    const RunsView R{h->starts, h->run_code, h->n_runs, h->set_off, h->set_ids,
                     (uint32_t)h->n_polys, (uint32_t)h->n_sets};
    const dim3 grid(std::min<unsigned>(grid_for((h->n_runs + 62) / 63 * 64), 8192));
    unsigned long long *c = (unsigned long long *)counts, *sv = (unsigned long long *)sums;
    const bool vals = sums != nullptr;
    if (search == SBA_SEARCH_LEARNED) {
        if (vals) hipLaunchKernelGGL((k_pindex_agg<true, true>), grid, dim3(256), 0, st, V, R, c, sv);
        else hipLaunchKernelGGL((k_pindex_agg<false, true>), grid, dim3(256), 0, st, V, R, c, sv);
    } else {
        if (vals) hipLaunchKernelGGL((k_pindex_agg<true, false>), grid, dim3(256), 0, st, V, R, c, sv);
        else hipLaunchKernelGGL((k_pindex_agg<false, false>), grid, dim3(256), 0, st, V, R, c, sv);
    }
    HIP_OK(hipGetLastError());
    return 0;
}

__global__ void k_debug_lb(IxView V, const uint64_t *v, int64_t n, int32_t rs, int64_t *out,
                           unsigned long long *fallbacks)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const uint64_t q = v[t] < V.total ? v[t] : V.total;
    out[t] = rs ? rs_lower_bound(V, q, fallbacks) : lower_bound_in(V.keys, 0, V.n, q);
}

extern "C" int sba_debug_pindex_lb(const sba_pindex *ix, const uint64_t *v, int64_t n,
                                   int32_t search, int64_t *out, int64_t *fallbacks, void *stream)
{
    if (!ix || n < 0 || (n > 0 && (!v || !out))) return SBA_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    if (fallbacks) *fallbacks = 0;
    if (n == 0) return 0;
    if (ix->n == 0) {
        HIP_OK(hipMemsetAsync(out, 0, sizeof(int64_t) * n, st));
        HIP_OK(hipStreamSynchronize(st));
        return 0;
    }
    Workspace ws(st);
    unsigned long long *fb = nullptr;
    RC(ws.alloc(&fb, 1));
    HIP_OK(hipMemsetAsync(fb, 0, sizeof(unsigned long long), st));
    const IxView V{ix->keys, ix->psum, ix->n, (uint64_t)1 << (2 * ix->L), ix->kx, ix->ky,
                   ix->rtab, ix->n_knots, ix->rshift, ix->spline_err};
    hipLaunchKernelGGL(k_debug_lb, dim3(grid_for(n)), dim3(256), 0, st, V, v, n,
                       search == SBA_SEARCH_LEARNED ? 1 : 0, out, fb);
    HIP_OK(hipGetLastError());
    unsigned long long h = 0;
    RC(ws.read(&h, fb, sizeof(h)));
    RC(ws.sync());
    if (fallbacks) *fallbacks = (int64_t)h;
    return 0;
}

extern "C" void sba_pindex_free(sba_pindex *ix)
{
    if (!ix) return;
    ix_release(ix);
    delete ix;
}
