// api.hip -- the C ABI declared in include/sba.h.
#include <new>
#include <vector>

#include "sba_internal.h"

// The handle's arrays go back to the device's block cache; nothing is
// synchronised (the caller guarantees that no queued work still reads them).
static void handle_release(sba_handle *h) { handle_put_all(h); }

extern "C" int sba_build_approx(const sba_polygons *polys, int64_t eps, const sba_build_opts *opts,
                                void *stream, sba_handle **out)
{
    if (!out) return SBA_EINVAL;
    *out = nullptr;
    if (!polys || polys->n_polys < 0) return SBA_EINVAL;
    if (polys->n_polys > MAX_POLYS) return SBA_ELIMIT;
    if (polys->n_polys > 0 && (!polys->ring_off || !polys->vert_off || !polys->xy))
        return SBA_EINVAL;
    if (eps < 2 || eps > ((int64_t)1 << 28)) return SBA_EINVAL;
    sba_handle *h = new (std::nothrow) sba_handle();
    if (!h) return SBA_ENOMEM;
    (void)hipGetDevice(&h->device);
    int rc = build_handle(polys, eps, opts, (hipStream_t)stream, h);
    if (rc) {
        (void)hipStreamSynchronize((hipStream_t)stream);
        handle_release(h);
        delete h;
        return rc;
    }
    *out = h;
    return SBA_OK;
}

extern "C" int sba_key_grid(const sba_polygons *sets, int32_t n_sets, int64_t eps, void *stream,
                            int32_t *level, int64_t *i0, int64_t *j0)
{
    if (!sets || n_sets < 1 || !level || !i0 || !j0) return SBA_EINVAL;
    if (n_sets > 64) return SBA_ELIMIT;
    if (eps < 2 || eps > ((int64_t)1 << 28)) return SBA_EINVAL;
    for (int32_t k = 0; k < n_sets; k++) {
        const sba_polygons &P = sets[k];
        if (P.n_polys < 0) return SBA_EINVAL;
        if (P.n_polys > MAX_POLYS) return SBA_ELIMIT;
        if (P.n_polys > 0 && (!P.ring_off || !P.vert_off || !P.xy)) return SBA_EINVAL;
    }
    return key_grid_launch(sets, n_sets, eps, (hipStream_t)stream, level, i0, j0);
}

static int check_probe_args(const int32_t *xy, const int64_t *values, int64_t n,
                            const sba_handle *h, uint64_t *counts)
{
    if (!h || n < 0) return SBA_EINVAL;
    if (h->n_polys > 0 && !counts) return SBA_EINVAL;
    if (n > 0 && !xy) return SBA_EINVAL;
    if (((uintptr_t)xy & 15) != 0 || ((uintptr_t)values & 15) != 0) return SBA_EINVAL;
    return 0;
}

extern "C" int sba_aggregate_search(const int32_t *xy, const int64_t *values, int64_t n,
                                    const sba_handle *h, int32_t search, uint64_t *counts,
                                    int64_t *sums, void *stream)
{
    RC(check_probe_args(xy, values, n, h, counts));
    if (search != SBA_SEARCH_BINARY && search != SBA_SEARCH_LEARNED) return SBA_EINVAL;
    return probe_launch(xy, values, n, h, search, counts, sums, (hipStream_t)stream);
}

extern "C" int sba_aggregate(const int32_t *xy, const int64_t *values, int64_t n,
                             const sba_handle *h, uint64_t *counts, int64_t *sums, void *stream)
{
    RC(check_probe_args(xy, values, n, h, counts));
    return probe_launch(xy, values, n, h, h->search, counts, sums, (hipStream_t)stream);
}

extern "C" int sba_aggregate_range(const int32_t *xy, const int64_t *values, int64_t n,
                                   const sba_handle *h, const sba_handle *hb, uint64_t *counts,
                                   int64_t *sums, uint64_t *bcounts, int64_t *bsums, void *stream)
{
    RC(check_probe_args(xy, values, n, h, counts));
    RC(check_probe_args(xy, values, n, hb, bcounts));
    if (h->n_polys != hb->n_polys || h->boundary_only || !hb->boundary_only || h->s != hb->s)
        return SBA_EINVAL;
    if ((sums == nullptr) != (bsums == nullptr)) return SBA_EINVAL;
    return range_launch(xy, values, n, h, hb, counts, sums, bcounts, bsums, (hipStream_t)stream);
}

static int check_tasks(const sba_task *tasks, int32_t n_tasks)
{
    if (n_tasks < 0 || (n_tasks > 0 && !tasks)) return SBA_EINVAL;
    for (int32_t k = 0; k < n_tasks; k++) {
        const sba_task &t = tasks[k];
        if (!t.h || t.lo < 0 || t.hi < t.lo) return SBA_EINVAL;
        if (t.h->n_polys > 0 && !t.counts) return SBA_EINVAL;
        if (t.hi > t.lo && !t.xy) return SBA_EINVAL;
        if (((uintptr_t)t.xy & 15) != 0 || ((uintptr_t)t.values & 15) != 0) return SBA_EINVAL;
        if (t.search == SBA_SEARCH_LEARNED && t.h->kind == SBA_KIND_HILBERT && !t.h->leaves)
            return SBA_EINVAL;
    }
    return 0;
}

extern "C" int sba_aggregate_batch(const sba_task *tasks, int32_t n_tasks, void *stream)
{
    RC(check_tasks(tasks, n_tasks));
    return batch_launch(tasks, n_tasks, (hipStream_t)stream);
}

extern "C" int sba_aggregate_batch_noalloc(const sba_task *tasks, int32_t n_tasks, void *stream)
{
    RC(check_tasks(tasks, n_tasks));
    return batch_launch_noalloc(tasks, n_tasks, (hipStream_t)stream);
}

extern "C" int sba_bucket_points(const int32_t *xy, const int64_t *values, int64_t n, int32_t x0,
                                 int32_t y0, int32_t cell, int32_t G, int32_t *out_xy,
                                 int64_t *out_values, int64_t *bucket_off, void *stream)
{
    if (n < 0 || G < 1 || G > 4096 || cell < 1 || !bucket_off) return SBA_EINVAL;
    if (n > 0 && (!xy || !out_xy || (values && !out_values))) return SBA_EINVAL;
    return bucket_launch(xy, values, n, x0, y0, cell, G, out_xy, out_values, bucket_off,
                         (hipStream_t)stream);
}

extern "C" int sba_lookup_cells(const sba_handle *h, const int64_t *ij, int64_t n, int32_t *ref,
                                void *stream)
{
    if (!h || n < 0 || (n > 0 && (!ij || !ref))) return SBA_EINVAL;
    return lookup_launch(h, ij, n, ref, (hipStream_t)stream);
}

extern "C" int sba_get_sets(const sba_handle *h, int64_t *n_sets, int64_t *n_ids, int64_t *off,
                            int32_t *ids)
{
    if (!h) return SBA_EINVAL;
    if (n_sets) *n_sets = h->n_sets;
    if (n_ids) *n_ids = h->n_set_ids;
    if (off && h->n_sets > 0)
        HIP_OK(hipMemcpy(off, h->set_off, sizeof(int64_t) * (h->n_sets + 1), hipMemcpyDeviceToHost));
    else if (off)
        off[0] = 0;
    if (ids && h->n_set_ids > 0)
        HIP_OK(hipMemcpy(ids, h->set_ids, sizeof(int32_t) * h->n_set_ids, hipMemcpyDeviceToHost));
    return SBA_OK;
}

__global__ void k_codes_to_refs(const uint32_t *code, int64_t n, int32_t *ref)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) ref[t] = code_to_ref(code[t]);
}

extern "C" int sba_get_runs(const sba_handle *h, uint64_t *starts, int32_t *ids, void *stream)
{
    if (!h || h->kind != SBA_KIND_HILBERT) return SBA_EINVAL;
    if (h->n_runs == 0) return SBA_OK;
    hipStream_t st = (hipStream_t)stream;
    if (starts)
        HIP_OK(hipMemcpyAsync(starts, h->starts, sizeof(uint64_t) * h->n_runs,
                              hipMemcpyDeviceToDevice, st));
    if (ids) {
        hipLaunchKernelGGL(k_codes_to_refs, dim3(grid_for(h->n_runs)), dim3(256), 0, st,
                           h->run_code, h->n_runs, ids);
        HIP_OK(hipGetLastError());
    }
    return SBA_OK;
}

extern "C" int sba_info(const sba_handle *h, sba_info_t *info)
{
    if (!h || !info) return SBA_EINVAL;
    sba_info_t o{};
    o.kind = h->kind;
    o.search = h->search;
    o.n_polys = h->n_polys;
    o.tile_log2 = h->tile_log2;
    o.level = h->level;
    o.log2_leaves = h->leaves ? h->log2_leaves : 0;
    o.eps = h->eps;
    o.s = h->s;
    o.gi0 = h->gi0;
    o.gj0 = h->gj0;
    o.gw = h->gw;
    o.gh = h->gh;
    o.n_tiles = h->tw * h->th;
    o.n_blocks = h->n_blocks;
    o.n_sub = h->n_sub;
    o.sub_log2 = h->sub_log2;
    o.compact = h->compact ? 1 : 0;
    o.boundary_only = h->boundary_only;
    o.centre_sampled = h->centre_sampled;
    o.n_sets = h->n_sets;
    o.n_set_ids = h->n_set_ids;
    o.n_segments = h->n_segments;
    o.n_boundary = h->n_boundary;
    o.n_runs = h->n_runs;
    o.max_leaf_err = h->max_leaf_err;
    o.mean_leaf_err = h->mean_leaf_err;
    o.bytes = h->bytes;
    o.build_ms = h->build_ms;
    *info = o;
    return SBA_OK;
}

extern "C" void sba_free(sba_handle *h)
{
    if (!h) return;
    handle_release(h);
    delete h;
}

extern "C" const char *sba_strerror(int code)
{
    switch (code) {
    case SBA_OK: return "success";
    case SBA_EINVAL: return "invalid argument";
    case SBA_ERANGE: return "coordinate out of range";
    case SBA_ENOMEM: return "device allocation failed";
    case SBA_EDEVICE: return "HIP runtime error";
    case SBA_ELIMIT: return "size limit exceeded";
    default: return "unknown error";
    }
}

extern "C" const char *sba_version(void) { return "sba 0.1 (gfx950)"; }

// Host-side check of the cell-side division used by the probes: q[k] =
// floor(n[k] / s) computed the way the kernels do.  Test support.
extern "C" int sba_debug_celldiv(int64_t s, const uint32_t *n, int64_t count, uint32_t *q)
{
    if (s < 1 || s > ((int64_t)1 << 28) || count < 0) return SBA_EINVAL;
    uint32_t mag;
    int32_t shift;
    magic_for(s, &mag, &shift);
    for (int64_t k = 0; k < count; k++) q[k] = divmagic(n[k], mag, shift);
    return SBA_OK;
}

// Host-side Hilbert index and its inverse as used by the kernels.  Test support.
extern "C" uint64_t sba_debug_hilbert(int L, uint32_t i, uint32_t j) { return hilbert_index(L, i, j); }

// the probes' four-levels-at-a-time encoder (host copy of its table), L <= 16
extern "C" uint64_t sba_debug_hilbert_tab(int L, uint32_t i, uint32_t j)
{
    static uint16_t tab[HILBERT_TAB];
    static bool ready = false;
    if (!ready) {
        for (uint32_t e = 0; e < HILBERT_TAB; e++) tab[e] = hilbert_tab_entry(e);
        ready = true;
    }
    if (L < 0 || L > 16) return ~(uint64_t)0;
    return hilbert_index_tab(L, i, j, tab);
}

extern "C" void sba_debug_hilbert_cell(int L, uint64_t d, uint32_t *i, uint32_t *j)
{
    hilbert_cell(L, d, i, j);
}
