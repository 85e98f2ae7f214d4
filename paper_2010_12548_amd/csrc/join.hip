// join.hip -- polygon-polygon join over cells (Sec. 4: two rasterized
// canvases blended cell by cell, masked to the cells that hold a polygon of
// each, aggregated per polygon pair).
//
// Both canvases are Hilbert handles on one key grid, so each is a sorted
// list of runs (first key, code) that partitions [0, 4^L).  Blending them is
// a merge of the two run lists: the union of their first keys cuts the key
// range into elementary intervals on which both codes are constant.  Masking
// keeps the intervals whose two codes are both non-empty; every member pair
// of the two codes (polygon sets expand to their members) then shares the
// interval's cells.  Sorting the (p, q) keys and summing the interval
// lengths of equal keys gives each pair's shared cell count.
#include "sba_internal.h"

namespace {

// run holding key v: last start <= v (starts[0] = 0)
__device__ __forceinline__ int64_t run_of(const uint64_t *starts, int64_t n, uint64_t v)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (starts[mid] <= v) lo = mid + 1; else hi = mid;
    }
    return lo - 1;
}

struct CanvasView {
    const uint64_t *starts;
    const uint32_t *code;
    int64_t n;
    const int64_t *set_off;
    const int32_t *set_ids;
    uint32_t np, n_sets;
};

__device__ __forceinline__ int64_t members(const CanvasView &C, uint32_t code)
{
    if (code == 0) return 0;
    if (code < CODE_SET_BASE) return code - 1u < C.np ? 1 : 0;
    const uint32_t k = code - CODE_SET_BASE;
    return k < C.n_sets ? C.set_off[k + 1] - C.set_off[k] : 0;
}

__device__ __forceinline__ uint32_t member(const CanvasView &C, uint32_t code, int64_t t)
{
    if (code < CODE_SET_BASE) return code - 1u;
    return (uint32_t)C.set_ids[C.set_off[code - CODE_SET_BASE] + t];
}

__global__ void k_first_flags(const uint64_t *keys, int64_t n, int64_t *flag)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) flag[t] = (t == 0 || keys[t] != keys[t - 1]) ? 1 : 0;
}

__global__ void k_first_write(const uint64_t *keys, int64_t n, const int64_t *pos, uint64_t *out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n && (t == 0 || keys[t] != keys[t - 1])) out[pos[t]] = keys[t];
}

// per elementary interval: both codes, its length, its number of pairs
__global__ void k_blend(const uint64_t *U, int64_t K, uint64_t total, CanvasView A, CanvasView B,
                        uint32_t *ca, uint32_t *cb, uint64_t *len, int64_t *cnt)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    const uint64_t u = U[k];
    const uint32_t a = A.code[run_of(A.starts, A.n, u)], b = B.code[run_of(B.starts, B.n, u)];
    ca[k] = a;
    cb[k] = b;
    len[k] = (k + 1 < K ? U[k + 1] : total) - u;
    cnt[k] = members(A, a) * members(B, b);  // mask: zero unless both hold a polygon
}

// every member pair of interval k: key p << 21 | q, payload k
__global__ void k_pairs(const uint32_t *ca, const uint32_t *cb, const int64_t *off, int64_t K,
                        CanvasView A, CanvasView B, uint64_t *key, uint32_t *pay)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    const int64_t mb = members(B, cb[k]);
    const int64_t n = off[k + 1] - off[k];
    for (int64_t t = 0; t < n; t++) {
        const uint32_t p = member(A, ca[k], t / mb), q = member(B, cb[k], t % mb);
        key[off[k] + t] = ((uint64_t)p << 21) | q;
        pay[off[k] + t] = (uint32_t)k;
    }
}

__global__ void k_pair_flags(const uint64_t *key, const uint32_t *pay, const uint64_t *len,
                             int64_t n, int64_t *flag, int64_t *plen)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    flag[t] = (t == 0 || key[t] != key[t - 1]) ? 1 : 0;
    plen[t] = (int64_t)len[pay[t]];
}

__global__ void k_pair_starts(const int64_t *flag, const int64_t *pos, int64_t n, int64_t *sidx)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n && flag[t]) sidx[pos[t]] = t;
}

// pair u = the keys [sidx[u], sidx[u+1]); its cells are the difference of the
// length prefix sums at the two ends
__global__ void k_pair_out(const uint64_t *key, const int64_t *sidx, const int64_t *psum,
                           int64_t nw, int64_t nu, int64_t n, int32_t *pa, int32_t *pb,
                           int64_t *cells)
{
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= nw) return;  // the first nw of the nu pairs
    const int64_t t = sidx[u], e = u + 1 < nu ? sidx[u + 1] : n;
    pa[u] = (int32_t)(key[t] >> 21);
    pb[u] = (int32_t)(key[t] & ((1u << 21) - 1));
    cells[u] = psum[e] - psum[t];
}

CanvasView view_of(const sba_handle *h)
{
    return CanvasView{h->starts, h->run_code, h->n_runs, h->set_off, h->set_ids,
                      (uint32_t)h->n_polys, (uint32_t)h->n_sets};
}

}  // namespace

extern "C" int sba_join_pairs(const sba_handle *a, const sba_handle *b, int64_t cap, int32_t *pa,
                              int32_t *pb, int64_t *cells, int64_t *n_pairs, void *stream)
{
    if (!a || !b || !n_pairs || cap < 0 || (cap > 0 && (!pa || !pb || !cells))) return SBA_EINVAL;
    *n_pairs = 0;
    if (a->kind != SBA_KIND_HILBERT || b->kind != SBA_KIND_HILBERT || a->s != b->s)
        return SBA_EINVAL;
    if (a->n_polys == 0 || b->n_polys == 0 || a->n_runs == 0 || b->n_runs == 0) return 0;
    if (a->level != b->level || a->gi0 != b->gi0 || a->gj0 != b->gj0) return SBA_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    Workspace ws(st);
    const uint64_t total = (uint64_t)1 << (2 * a->level);
    const CanvasView A = view_of(a), B = view_of(b);

    // blend: the union of the two run partitions
    const int64_t R = a->n_runs + b->n_runs;
    uint64_t *keys = nullptr;
    RC(ws.alloc(&keys, R));
    HIP_OK(hipMemcpyAsync(keys, a->starts, sizeof(uint64_t) * a->n_runs, hipMemcpyDeviceToDevice, st));
    HIP_OK(hipMemcpyAsync(keys + a->n_runs, b->starts, sizeof(uint64_t) * b->n_runs,
                          hipMemcpyDeviceToDevice, st));
    RC(radix_sort_u64_ws(&keys, nullptr, R, 2 * a->level, ws));
    int64_t *flag = nullptr, *tot = nullptr;
    RC(ws.alloc(&flag, R + 1));
    RC(ws.alloc(&tot, 2));
    hipLaunchKernelGGL(k_first_flags, dim3(grid_for(R)), dim3(256), 0, st, keys, R, flag);
    HIP_OK(hipGetLastError());
    RC(scan_exclusive_i64(flag, flag, R, tot, st, &ws));
    int64_t K = 0;
    RC(ws.read(&K, tot, sizeof(int64_t)));
    RC(ws.sync());
    uint64_t *U = nullptr;
    RC(ws.alloc(&U, K));
    hipLaunchKernelGGL(k_first_write, dim3(grid_for(R)), dim3(256), 0, st, keys, R, flag, U);
    HIP_OK(hipGetLastError());
    ws.put(keys);
    ws.put(flag);

    // mask: intervals holding a polygon of each canvas, and their pair counts
    uint32_t *ca = nullptr, *cb = nullptr;
    uint64_t *len = nullptr;
    int64_t *off = nullptr;
    RC(ws.alloc(&ca, K));
    RC(ws.alloc(&cb, K));
    RC(ws.alloc(&len, K));
    RC(ws.alloc(&off, K + 1));
    hipLaunchKernelGGL(k_blend, dim3(grid_for(K)), dim3(256), 0, st, U, K, total, A, B, ca, cb,
                       len, off);
    HIP_OK(hipGetLastError());
    RC(scan_exclusive_i64(off, off, K, off + K, st, &ws));
    int64_t NP = 0;
    RC(ws.read(&NP, off + K, sizeof(int64_t)));
    RC(ws.sync());
    if (NP == 0) return 0;
    if (NP >= ((int64_t)1 << 32)) return SBA_ELIMIT;

    // aggregate per pair: sort the pair keys, sum the lengths of equal keys
    uint64_t *pkey = nullptr;
    uint32_t *pay = nullptr;
    RC(ws.alloc(&pkey, NP));
    RC(ws.alloc(&pay, NP));
    hipLaunchKernelGGL(k_pairs, dim3(grid_for(K)), dim3(256), 0, st, ca, cb, off, K, A, B, pkey,
                       pay);
    HIP_OK(hipGetLastError());
    RC(radix_sort_u64_ws(&pkey, &pay, NP, 42, ws));
    int64_t *pf = nullptr, *plen = nullptr, *pos = nullptr;
    RC(ws.alloc(&pf, NP + 1));
    RC(ws.alloc(&plen, NP + 1));
    RC(ws.alloc(&pos, NP + 1));
    hipLaunchKernelGGL(k_pair_flags, dim3(grid_for(NP)), dim3(256), 0, st, pkey, pay, len, NP, pf,
                       plen);
    HIP_OK(hipGetLastError());
    {
        const int64_t *in[2] = {pf, plen}, n[2] = {NP, NP};
        int64_t *out[2] = {pos, plen}, *sum[2] = {tot, plen + NP};
        RC(scan_exclusive_i64_multi(2, in, out, n, sum, st, &ws));
    }
    int64_t NU = 0;
    RC(ws.read(&NU, tot, sizeof(int64_t)));
    RC(ws.sync());
    const int64_t nw = std::min(NU, cap);
    if (nw > 0) {
        int64_t *sidx = nullptr;
        RC(ws.alloc(&sidx, NU));
        hipLaunchKernelGGL(k_pair_starts, dim3(grid_for(NP)), dim3(256), 0, st, pf, pos, NP, sidx);
        hipLaunchKernelGGL(k_pair_out, dim3(grid_for(nw)), dim3(256), 0, st, pkey, sidx, plen, nw,
                           NU, NP, pa, pb, cells);
        HIP_OK(hipGetLastError());
        HIP_OK(hipStreamSynchronize(st));
    }
    *n_pairs = NU;
    return 0;
}
