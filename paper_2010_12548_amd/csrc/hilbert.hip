// hilbert.hip -- the adaptive-quadtree layout: the approximation stored as
// the maximal runs of consecutive Hilbert keys whose cells carry the same
// polygon set (Sec. 3: cells linearised on a space-filling curve and kept in
// a sorted array; a run of the curve is a union of aligned quadtree blocks,
// so interior cells come out as large cells, Sec. 2.2), and the learned
// index that predicts a key's run (Sec. 3, learned index over the sorted
// cell array).
//
// The key grid is anchored at the first cell of the stored box (the union of
// the polygons' cell boxes), so every cell of every approximation has a key;
// or at a grid the caller gives (a point index's), the box cut to it.
//
// Runs are found without visiting interior cells.  Consecutive Hilbert cells
// share an edge; two edge-adjacent cells that are boundary cells of no
// polygon have the same polygon set (a polygon boundary separating them
// would touch both closed squares).  So the polygon set is constant on every
// gap between consecutive boundary keys, and one lookup at the gap's first
// cell gives it.
#include "sba_internal.h"
#include "build_state.h"

__device__ __forceinline__ int64_t ub_i64(const int64_t *a, int64_t n, int64_t v)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (a[mid] <= v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// cells of boundary interval t (relative to the stored box, which is also
// the origin of the Hilbert key grid); event keys are (polygon, row, x)
__global__ void k_bcell_counts(const uint64_t *evkey, int64_t nb, int xbits, int64_t *cnt)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nb) return;
    uint64_t xm = (1ull << xbits) - 1;
    cnt[t] = (int64_t)(evkey[2 * t + 1] & xm) - (int64_t)(evkey[2 * t] & xm);
}

__global__ void k_bcell_keys(const uint64_t *evkey, int64_t nb, int xbits, int rbits,
                             const int64_t *off, int64_t ncells, int L, uint64_t *keys)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncells) return;
    int64_t t = ub_i64(off, nb, c) - 1;
    uint64_t xm = (1ull << xbits) - 1;
    uint32_t j = (uint32_t)((evkey[2 * t] >> xbits) & ((1ull << rbits) - 1));
    uint32_t i = (uint32_t)((evkey[2 * t] & xm) + (uint64_t)(c - off[t]));
    keys[c] = hilbert_index(L, i, j);
}

// cells on the border of the stored box (used when a clip window cut the
// box through polygon interiors: a gap of the curve must not run from a cell
// inside the box to an empty cell outside it without a key in between)
__global__ void k_border_keys(int64_t gw, int64_t gh, int L, uint64_t *keys)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * (gw + gh)) return;
    uint32_t i, j;
    if (t < gw) { i = (uint32_t)t; j = 0; }
    else if (t < 2 * gw) { i = (uint32_t)(t - gw); j = (uint32_t)(gh - 1); }
    else if (t < 2 * gw + gh) { i = 0; j = (uint32_t)(t - 2 * gw); }
    else { i = (uint32_t)(gw - 1); j = (uint32_t)(t - 2 * gw - gh); }
    keys[t] = hilbert_index(L, i, j);
}

__global__ void k_flag_first(const uint64_t *keys, int64_t n, int64_t *flag)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    flag[t] = (t == 0 || keys[t] != keys[t - 1]) ? 1 : 0;
}

__global__ void k_compact_first(const uint64_t *keys, int64_t n, const int64_t *pos, uint64_t *out)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    if (t == 0 || keys[t] != keys[t - 1]) out[pos[t]] = keys[t];
}

static int hilbert_boundary_cells(BuildState &B, sba_handle *h, hipStream_t st)
{
    const int64_t NB = B.NB;
    if (NB == 0 && !B.window) return 0;
    int64_t *cnt = nullptr, *tot = nullptr;
    RC(B.alloc(&cnt, NB + 1));
    RC(B.alloc(&tot, 1));
    hipLaunchKernelGGL(k_bcell_counts, dim3(grid_for(NB)), dim3(256), 0, st, B.evkey, NB, B.xbits,
                       cnt);
    HIP_OK(hipGetLastError());
    RC(scan_exclusive_i64(cnt, cnt, NB, tot, st, &B.ws));
    int64_t ncb = 0;
    RC(B.ws.read(&ncb, tot, sizeof(int64_t)));
    RC(B.ws.sync());
    const int64_t nborder = B.window ? 2 * (h->gw + h->gh) : 0;
    const int64_t nc = ncb + nborder;
    if (nc == 0) return 0;
    uint64_t *keys = nullptr;
    RC(B.alloc(&keys, nc));
    if (ncb)
        hipLaunchKernelGGL(k_bcell_keys, dim3(grid_for(ncb)), dim3(256), 0, st, B.evkey, NB, B.xbits,
                           B.rbits, cnt, ncb, h->level, keys);
    if (nborder)
        hipLaunchKernelGGL(k_border_keys, dim3(grid_for(nborder)), dim3(256), 0, st, h->gw, h->gh,
                           h->level, keys + ncb);
    HIP_OK(hipGetLastError());
    B.release(cnt);
    RC(radix_sort_u64_ws(&keys, nullptr, nc, 2 * h->level, B.ws));
    int64_t *flag = nullptr;
    RC(B.alloc(&flag, nc + 1));
    hipLaunchKernelGGL(k_flag_first, dim3(grid_for(nc)), dim3(256), 0, st, keys, nc, flag);
    HIP_OK(hipGetLastError());
    RC(scan_exclusive_i64(flag, flag, nc, tot, st, &B.ws));
    int64_t nu = 0;
    RC(B.ws.read(&nu, tot, sizeof(int64_t)));
    RC(B.ws.sync());
    RC(B.alloc(&B.bkeys, nu));
    hipLaunchKernelGGL(k_compact_first, dim3(grid_for(nc)), dim3(256), 0, st, keys, nc, flag,
                       B.bkeys);
    HIP_OK(hipGetLastError());
    B.nbkeys = nu;
    B.release(keys);
    B.release(flag);
    return 0;
}

int hilbert_prepare(BuildState &B, sba_handle *h)
{
    (void)h;
    B.on_boundary_events = [](BuildState &b, sba_handle *hh, hipStream_t st) -> int {
        // key grid: the stored cell box, padded to 2^L x 2^L
        int L = 1;
        while (((int64_t)1 << L) < std::max(hh->gw, hh->gh)) L++;
        if (b.key_level > 0) L = b.key_level;  // the box was cut to fit it
        if (L > 21) return SBA_ELIMIT;
        hh->level = L;
        return hilbert_boundary_cells(b, hh, st);
    };
    return 0;
}

// ---------------------------------------------------------------- runs

__device__ __forceinline__ uint32_t code_of_cell(const int64_t *seg_row_off, const int32_t *seg_x0,
                                                 const int32_t *seg_x1, const uint32_t *seg_code,
                                                 int64_t gi0, int64_t gj0, int64_t gw, int64_t gh,
                                                 int64_t i, int64_t j)
{
    int64_t x = i - gi0, r = j - gj0;
    if (x < 0 || r < 0 || x >= gw || r >= gh) return 0;
    int64_t lo = seg_row_off[r], hi = seg_row_off[r + 1], a = lo;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (seg_x0[mid] <= (int32_t)x) lo = mid + 1; else hi = mid;
    }
    if (lo > a && (int32_t)x < seg_x1[lo - 1]) return seg_code[lo - 1];
    return 0;
}

struct SegView {
    const int64_t *row_off;
    const int32_t *x0, *x1;
    const uint32_t *code;
    int64_t gi0, gj0, gw, gh;
};

__device__ __forceinline__ uint32_t code_of_key(const SegView &S, int L, uint64_t key)
{
    uint32_t i, j;
    hilbert_cell(L, key, &i, &j);
    return code_of_cell(S.row_off, S.x0, S.x1, S.code, S.gi0, S.gj0, S.gw, S.gh, S.gi0 + i,
                        S.gj0 + j);
}

// candidate run starts: every boundary key, the key after it when a gap
// follows, and key 0 when the first boundary key is not 0
__global__ void k_cand_counts(const uint64_t *bk, int64_t nb, uint64_t total, int64_t *cnt)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nb) return;
    uint64_t next = (t + 1 < nb) ? bk[t + 1] : total;
    cnt[t] = 1 + ((next > bk[t] + 1) ? 1 : 0);
}

__global__ void k_cand_write(const uint64_t *bk, int64_t nb, uint64_t total, const int64_t *off,
                             int64_t lead, SegView S, int L, uint64_t *ckey, uint32_t *ccode)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t == 0 && lead) {
        ckey[0] = 0;
        ccode[0] = code_of_key(S, L, 0);
    }
    if (t >= nb) return;
    int64_t o = lead + off[t];
    uint64_t k = bk[t];
    ckey[o] = k;
    ccode[o] = code_of_key(S, L, k);
    uint64_t next = (t + 1 < nb) ? bk[t + 1] : total;
    if (next > k + 1) {
        ckey[o + 1] = k + 1;
        ccode[o + 1] = code_of_key(S, L, k + 1);
    }
}

__global__ void k_run_flags(const uint32_t *ccode, int64_t n, int64_t *flag)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    flag[t] = (t == 0 || ccode[t] != ccode[t - 1]) ? 1 : 0;
}

__global__ void k_run_write(const uint64_t *ckey, const uint32_t *ccode, int64_t n,
                            const int64_t *pos, uint64_t *starts, uint32_t *starts32,
                            uint32_t *rcode)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    if (t == 0 || ccode[t] != ccode[t - 1]) {
        int64_t g = pos[t];
        starts[g] = ckey[t];
        if (starts32) starts32[g] = (uint32_t)ckey[t];
        rcode[g] = ccode[t];
    }
}

// ---------------------------------------------------------------- learned index
//
// Two-level piecewise-linear model over the sorted run starts (the idea of a
// learned index over a sorted cell array with a bounded last-mile search,
// Sec. 3).  Root: leaf = floor(key * a) in fp32, clamped, monotone in key.
// Leaf l covers the keys [K_l, K_{l+1}); it predicts the position of the run
// holding a key as floor(slope * (key - K_l) + icpt) in fp32 (no fused
// multiply-add, identical in the fit and in the probe), fitted by least
// squares on the leaf's run starts.  Its stored error bounds |prediction -
// answer| over EVERY key of [K_l, K_{l+1}), not only the stored ones: the
// answer is a step function of the key and the prediction is monotone, so the
// largest gap sits at an end of a step, and the fit evaluates exactly those
// keys.  The probe still verifies the bracket and falls back to a full binary
// search if it ever fails.

// smallest key whose leaf is >= l (keys in [0, total])
__device__ uint64_t leaf_first_key(uint32_t l, float a, uint32_t nl, uint64_t total)
{
    if (l == 0) return 0;
    uint64_t lo = 0, hi = total;
    while (lo < hi) {
        uint64_t mid = lo + ((hi - lo) >> 1);
        if (root_leaf(mid, a, nl) >= l) hi = mid; else lo = mid + 1;
    }
    return lo;
}

__device__ __forceinline__ int64_t lower_bound_u64(const uint64_t *a, int64_t n, uint64_t v)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (a[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// first q >= from with a[q] >= v (a[from - 1] < v when from > 0): doubling
// steps from `from`, then a binary search in the last step (a leaf holds a
// few dozen runs, so this takes a few loads where a search over all runs
// would take about 25)
__device__ __forceinline__ int64_t lower_bound_from(const uint64_t *a, int64_t n, int64_t from,
                                                    uint64_t v)
{
    if (from >= n || a[from] >= v) return from;
    int64_t base = from, step = 1;  // a[base] < v
    while (base + step < n && a[base + step] < v) {
        base += step;
        step <<= 1;
    }
    int64_t lo = base + 1, hi = min(base + step, n);  // the answer is in [lo, hi]
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (a[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// The fit of leaf l over the run starts [lo, hi) of its keys [K0, K1) by one
// wavefront; returns its error bound (every lane).
__device__ int64_t leaf_fit_one(const uint64_t *starts, int64_t n, uint32_t nl, uint32_t l,
                                uint64_t K0, uint64_t K1, int64_t lo, int64_t hi, int lane,
                                int4 *leaves, int32_t *leaf_lo)
{
    // least squares of y = q - lo against x = starts[q] - K0 over q in [lo, hi)
    double sx = 0, sy = 0, sxx = 0, sxy = 0;
    for (int64_t q = lo + lane; q < hi; q += 64) {
        double x = (double)(starts[q] - K0), y = (double)(q - lo);
        sx += x; sy += y; sxx += x * x; sxy += x * y;
    }
    for (int o = 32; o > 0; o >>= 1) {
        sx += __shfl_xor(sx, o, 64);
        sy += __shfl_xor(sy, o, 64);
        sxx += __shfl_xor(sxx, o, 64);
        sxy += __shfl_xor(sxy, o, 64);
    }
    double cnt = (double)(hi - lo);
    float slope = 0.f, icpt;
    if (hi - lo >= 2) {
        double mx = sx / cnt, my = sy / cnt;
        double var = sxx / cnt - mx * mx, cov = sxy / cnt - mx * my;
        double sl = var > 0 ? cov / var : 0.0;
        if (sl < 0) sl = 0;
        slope = (float)sl;
        icpt = (float)(my - sl * mx + (double)lo);
    } else if (hi - lo == 1) {
        icpt = (float)lo;
    } else {
        icpt = (float)(lo - 1);
    }
    const int4 lf = make_int4((int)(uint32_t)K0, __float_as_int(slope), __float_as_int(icpt), 0);
    // error over every key of [K0, K1): the answer is q on [max(starts[q],K0),
    // min(starts[q+1],K1) - 1] for q in [lo-1, hi-1]; the clamped prediction is
    // monotone, so both ends of each step bound it
    int64_t err = 0;
    if (K1 > K0) {
        for (int64_t q = lo - 1 + lane; q <= hi - 1; q += 64) {
            if (q < 0) continue;  // keys before the first start do not occur (starts[0] = 0)
            uint64_t ka = starts[q] > K0 ? starts[q] : K0;
            uint64_t kb = (q + 1 < n && starts[q + 1] < K1) ? starts[q + 1] - 1 : K1 - 1;
            if (ka > kb) continue;
            int64_t pa = predict_in_leaf(lf, lo, hi, ka), pb = predict_in_leaf(lf, lo, hi, kb);
            int64_t e1 = pa > q ? pa - q : q - pa, e2 = pb > q ? pb - q : q - pb;
            err = max(err, max(e1, e2));
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        int64_t v = __shfl_xor(err, o, 64);
        err = max(err, v);
    }
    if (lane == 0) {
        leaves[l] = make_int4(lf.x, lf.y, lf.z, (int)err);
        leaf_lo[l] = (int32_t)lo;
        if (l == nl - 1) leaf_lo[nl] = (int32_t)n;
    }
    return err;
}

// Each wavefront fits a contiguous chunk of leaves: key range, least-squares
// fit, exact error bound.  A leaf's end (key and run position) is the next
// leaf's start, found from it by doubling steps, and the wave adds the
// largest and the summed error of its leaves to err_stats once.
__global__ void k_leaf_fit(const uint64_t *starts, int64_t n, float a, uint32_t nl, uint64_t total,
                           int4 *leaves, int32_t *leaf_lo, unsigned long long *err_stats)
{
    const int lane = threadIdx.x & 63;
    const int64_t waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t chunk = ((int64_t)nl + waves - 1) / waves;
    const int64_t l0 = (((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * chunk;
    const int64_t l1 = min(l0 + chunk, (int64_t)nl);
    unsigned long long emax = 0, esum = 0;
    if (l0 < l1) {
        uint64_t K0 = leaf_first_key((uint32_t)l0, a, nl, total);
        int64_t lo = lower_bound_u64(starts, n, K0);
        for (int64_t l = l0; l < l1; l++) {
            const uint64_t K1 = (l + 1 < nl) ? leaf_first_key((uint32_t)l + 1, a, nl, total) : total;
            const int64_t hi = lower_bound_from(starts, n, lo, K1);
            const int64_t err =
                leaf_fit_one(starts, n, nl, (uint32_t)l, K0, K1, lo, hi, lane, leaves, leaf_lo);
            emax = max(emax, (unsigned long long)err);
            esum += (unsigned long long)err;
            K0 = K1;
            lo = hi;
        }
    }
    if (lane == 0 && esum + emax > 0) {
        atomicMax(&err_stats[0], emax);
        atomicAdd(&err_stats[1], esum);
    }
}


int hilbert_finish(BuildState &B, sba_handle *h, const sba_build_opts &o, hipStream_t st)
{
    const int L = h->level;
    const uint64_t total = (uint64_t)1 << (2 * L);
    const int64_t nb = B.nbkeys;
    const int64_t lead = 1;  // key 0 always opens a run (a boundary key 0 repeats it)
    SegView S{B.seg_row_off, B.seg_x0, B.seg_x1, B.seg_code, h->gi0, h->gj0, h->gw, h->gh};
    int64_t *cnt = nullptr, *tot = nullptr;
    RC(B.alloc(&cnt, nb + 1));
    RC(B.alloc(&tot, 1));
    if (nb)
        hipLaunchKernelGGL(k_cand_counts, dim3(grid_for(nb)), dim3(256), 0, st, B.bkeys, nb, total,
                           cnt);
    HIP_OK(hipGetLastError());
    RC(scan_exclusive_i64(cnt, cnt, nb, tot, st, &B.ws));
    int64_t nc = 0;
    if (nb) {
        RC(B.ws.read(&nc, tot, sizeof(int64_t)));
        RC(B.ws.sync());
    }
    nc += lead;
    uint64_t *ckey = nullptr;
    uint32_t *ccode = nullptr;
    RC(B.alloc(&ckey, nc));
    RC(B.alloc(&ccode, nc));
    // a boundary key equal to 0 writes over the leading candidate with the same values
    hipLaunchKernelGGL(k_cand_write, dim3(grid_for(nb > 0 ? nb : 1)), dim3(256), 0, st, B.bkeys, nb,
                       total, cnt, lead, S, L, ckey, ccode);
    HIP_OK(hipGetLastError());
    int64_t *flag = nullptr;
    RC(B.alloc(&flag, nc + 1));
    hipLaunchKernelGGL(k_run_flags, dim3(grid_for(nc)), dim3(256), 0, st, ccode, nc, flag);
    HIP_OK(hipGetLastError());
    RC(scan_exclusive_i64(flag, flag, nc, tot, st, &B.ws));
    int64_t nr = 0;
    RC(B.ws.read(&nr, tot, sizeof(int64_t)));
    RC(B.ws.sync());
    if (nr >= ((int64_t)1 << 31)) return SBA_ELIMIT;
    h->n_runs = nr;
    RC(handle_alloc(h, &h->starts, nr));
    RC(handle_alloc(h, &h->run_code, nr));
    if (2 * L <= 32) {
        RC(handle_alloc(h, &h->starts32, nr));
    }
    hipLaunchKernelGGL(k_run_write, dim3(grid_for(nc)), dim3(256), 0, st, ckey, ccode, nc, flag,
                       h->starts, h->starts32, h->run_code);
    HIP_OK(hipGetLastError());

    if (o.search == SBA_SEARCH_LEARNED) {
        if (2 * L > 32) return SBA_ELIMIT;  // leaves store 32-bit key bases
        const uint32_t nl = 1u << o.log2_leaves;
        h->log2_leaves = o.log2_leaves;
        uint64_t last = 0;
        RC(B.ws.read(&last, h->starts + (nr - 1), sizeof(uint64_t)));
        RC(B.ws.sync());
        h->root_k0 = 0;
        h->root_a = (float)nl / (float)(last + 1);
        unsigned long long *stats = nullptr;
        RC(B.alloc(&stats, 2));
        HIP_OK(hipMemsetAsync(stats, 0, 2 * sizeof(unsigned long long), st));
        RC(handle_alloc(h, &h->leaves, nl));
        RC(handle_alloc(h, &h->leaf_lo, (int64_t)nl + 1));
        const int64_t fit_blocks = std::min<int64_t>(grid_for((int64_t)nl * 64), 4096);
        hipLaunchKernelGGL(k_leaf_fit, dim3((unsigned)fit_blocks), dim3(256), 0, st, h->starts,
                           nr, h->root_a, nl, total, h->leaves, h->leaf_lo, stats);
        HIP_OK(hipGetLastError());
        unsigned long long hs[2];
        RC(B.ws.read(hs, stats, sizeof(hs)));
        RC(B.ws.sync());
        h->max_leaf_err = (int64_t)hs[0];
        h->mean_leaf_err = (double)hs[1] / (double)nl;
    }
    return 0;
}
