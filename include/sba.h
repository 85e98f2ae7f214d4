/*
 * sba.h -- C ABI of the distance-bounded spatial aggregation library for
 * AMD MI355X (gfx950).
 *
 * The library answers the spatial aggregation query of Sec. 5 of
 * Tzirita Zacharatou et al., "The Case for Distance-Bounded Spatial
 * Approximations" (CIDR 2021):
 *
 *     SELECT COUNT(*), SUM(value) FROM points, polygons
 *     WHERE point INSIDE polygon GROUP BY polygon.id
 *
 * without any point-in-polygon test: every polygon P is replaced by its
 * conservative raster approximation A(P) (Sec. 2.2), a set of grid cells of
 * side s = the largest integer with 2 s^2 <= eps^2 (cell diagonal <= eps).
 * A cell belongs to A(P) when its closed square touches an edge of P
 * (boundary cell) or when it touches no edge and its lower-left corner is
 * inside P by the crossing-number rule (interior cell).  A point counts for
 * every polygon whose approximation holds the point's cell, so every point
 * that is counted wrongly lies within eps of that polygon's boundary, and no
 * point inside a polygon is ever missed (false positives only).
 *
 * Conventions shared by every entry point:
 *   - Coordinates are int32 fixed-point; the grid is anchored at (0,0) and
 *     cell(p) = (floor(x/s), floor(y/s)).  Polygon vertex coordinates must
 *     satisfy |c| < 2^30.  eps must lie in [2, 2^28].
 *   - Every array argument is a DEVICE pointer (memory of the GPU that is
 *     current when the call is made) unless the comment says "host".
 *     The caller owns all of them; the library never frees them.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls are asynchronous on that stream except where noted.
 *   - Return 0 on success or a negative SBA_E* code; nothing is thrown.
 */
#ifndef SBA_H
#define SBA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SBA_OK        0
#define SBA_EINVAL   (-1)  /* null pointer, negative size, bad offsets, eps out of range */
#define SBA_ERANGE   (-2)  /* vertex coordinate out of range (|c| >= 2^30) */
#define SBA_ENOMEM   (-3)  /* device allocation failed */
#define SBA_EDEVICE  (-4)  /* a HIP call failed */
#define SBA_ELIMIT   (-5)  /* a documented size limit is exceeded (see sba_build_approx) */

/* Layouts of the approximation. */
#define SBA_KIND_GRID     0  /* two-level tiled uniform grid of cell codes          */
#define SBA_KIND_HILBERT  1  /* sorted Hilbert-key runs (adaptive quadtree cells)    */

/* Search used by the Hilbert layout's probe. */
#define SBA_SEARCH_BINARY   0  /* predecessor by binary search over all run starts   */
#define SBA_SEARCH_LEARNED  1  /* two-level linear model + bounded search (+ fallback) */

typedef struct sba_handle sba_handle;

/* Polygons in CSR form, all DEVICE pointers.
 *   ring_off[n_polys+1]  ring index range of polygon p: [ring_off[p], ring_off[p+1])
 *   vert_off[n_rings+1]  vertex index range of ring r (rings are closed implicitly)
 *   xy[2*n_verts]        x, y interleaved, int32
 * A polygon with several rings is read even-odd (holes, multi-polygons).
 * Polygons may overlap; a cell then belongs to every polygon that claims it. */
typedef struct {
    int32_t        n_polys;
    const int32_t *ring_off;
    const int64_t *vert_off;
    const int32_t *xy;
} sba_polygons;

typedef struct {
    int32_t kind;         /* SBA_KIND_GRID (default) or SBA_KIND_HILBERT                 */
    int32_t search;       /* Hilbert only: SBA_SEARCH_BINARY (default) or _LEARNED       */
    int32_t log2_leaves;  /* learned index: number of leaves = 2^log2_leaves (0 -> 16)   */
    int32_t tile_log2;    /* grid: tile side 2^tile_log2 cells, 2..10 (0 -> the smallest
                             tile whose 16-bit directory, with 12 B per polygon and per
                             polygon set, fits the 160 KB LDS of a compute unit)          */
    int32_t use_window;   /* 1: store only the cells that overlap the clip window        */
    int32_t win_x0, win_y0, win_x1, win_y1;  /* clip window [x0,x1) x [y0,y1), coordinates;
                             cells outside it are empty in the handle (for viewport
                             queries: the answer inside the window is unchanged)         */
    int32_t sub_log2;     /* grid: sub-tile side 2^sub_log2 cells inside mixed tiles,
                             1..tile_log2; == tile_log2: mixed tiles are stored cell by
                             cell (0 -> the smallest side whose 16-bit sub-directory fits
                             the LDS of a compute unit beside the directory and the
                             probe's bins, so the probe reads it there; if none fits, 4
                             for tiles of 64 cells or more, 3 for tiles of 32 cells,
                             else tile_log2)                                             */
    int32_t boundary_only; /* 1: store only the boundary cells B(P) of every polygon
                             (no interior cells).  sba_aggregate over such a handle gives
                             the partial count beta (and sum) over the boundary cells, so
                             the exact answer lies in [alpha - beta, alpha] for the full
                             approximation's alpha (Sec. 6, result range estimation;
                             sums: for non-negative values)                             */
    int32_t key_level;    /* Hilbert only: > 0 anchors the 2^key_level x 2^key_level key
                             grid at cell (key_i0, key_j0) instead of the stored box's
                             first cell (the key grid of a point index, sba_pindex_info,
                             so that sba_pindex_aggregate can answer from the handle's
                             runs); cells outside that grid are not stored.  1..21     */
    int64_t key_i0, key_j0;
    int32_t centre_sampled; /* 1: the non-conservative approximation C(P) (Sec. 2.2: cells
                             with little overlap may be left out): a cell belongs to P
                             when its centre ((i+1/2)s, (j+1/2)s) is inside P by the
                             crossing-number rule.  False negatives as well as false
                             positives, every misclassified point within eps/2 of P's
                             boundary; on a partition every point counts once.  Not with
                             boundary_only.                                             */
    /* Device memory of the build.  alloc == NULL: the library's own block cache
       (hipMalloc, kept for later builds).  Otherwise every device block of the build --
       its temporaries and the handle's arrays -- comes from alloc(bytes, alloc_ctx),
       which returns device memory of the current device, at least `bytes` long and
       256-byte aligned, or NULL to refuse (the build then gives back every block it
       took and fails with SBA_ENOMEM; a misaligned block fails it with SBA_EINVAL).
       Each block goes back through release(p, alloc_ctx): the temporaries before
       sba_build_approx returns (their work has completed), the handle's arrays in
       sba_free (which does not synchronise).  Both are called on the thread that
       calls sba_build_approx / sba_free; release must be set when alloc is.       */
    void *(*alloc)(size_t bytes, void *ctx);
    void (*release)(void *p, void *ctx);
    void *alloc_ctx;
} sba_build_opts;

typedef struct {
    int32_t kind, search;
    int32_t n_polys;
    int32_t tile_log2;      /* grid */
    int32_t level;          /* Hilbert: L, keys in [0, 4^L) */
    int32_t log2_leaves;
    int64_t eps, s;         /* distance bound and cell side */
    int64_t gi0, gj0;       /* first cell of the stored box (grid) */
    int64_t gw, gh;         /* stored box size in cells */
    int64_t n_tiles, n_blocks;  /* grid: directory entries, mixed tiles */
    int64_t n_sets, n_set_ids;  /* multi-polygon cell sets */
    int64_t n_segments;     /* row segments of constant polygon set (build intermediate) */
    int64_t n_boundary;     /* (edge, row strip) boundary intervals */
    int64_t n_runs;         /* Hilbert runs */
    int64_t max_leaf_err;   /* learned index: largest stored error */
    double  mean_leaf_err;  /* learned index: mean stored error over the leaves */
    int64_t bytes;          /* device bytes held by the handle */
    double  build_ms;       /* wall time of the build, host clock (includes its syncs) */
    int64_t n_sub;          /* grid: mixed sub-tiles (stored cell by cell) */
    int32_t sub_log2;       /* grid: sub-tile side log2 (== tile_log2: no sub level) */
    int32_t compact;        /* grid: 1 = 16-bit codes (directory staged in LDS), 0 = 32-bit */
    int32_t boundary_only;  /* built with sba_build_opts.boundary_only */
    int32_t centre_sampled; /* built with sba_build_opts.centre_sampled */
} sba_info_t;

/*
 * Build the approximation A(P) of every polygon for distance bound eps
 * (Sec. 2.2: cell side eps/sqrt(2) at the boundary; conservative raster;
 * Sec. 3: cells linearised on the Hilbert curve for the Hilbert layout).
 *
 *   polys   host struct of DEVICE arrays (see sba_polygons); read during the
 *           call only.
 *   eps     distance bound in coordinate units, 2 <= eps <= 2^28.
 *   opts    host pointer or NULL for defaults.
 *   stream  work is queued on it; the call synchronises it several times
 *           (it reads sizes back) and returns once the handle is complete.
 *   out     host pointer; receives the new handle (NULL on failure).
 *
 * The stored cell box is the union of the polygons' cell boxes; the grid
 * layout tiles it, the Hilbert layout anchors its 2^L x 2^L key grid at its
 * first cell (L = smallest level covering the box).
 * Limits (SBA_ELIMIT): at most 2^21-1 polygons; the stored cell box at most
 * 2^21 cells per side and less than 2^31 coordinate units per side; a cell
 * may belong to at most 32 polygons; learned index: L <= 16.
 * Errors: SBA_EINVAL (null/negative/non-monotone offsets, eps out of range),
 * SBA_ERANGE, SBA_ENOMEM, SBA_EDEVICE, SBA_ELIMIT.
 */
int sba_build_approx(const sba_polygons *polys, int64_t eps, const sba_build_opts *opts,
                     void *stream, sba_handle **out);

/*
 * The Hilbert key grid that covers the cells of several polygon sets at
 * distance bound eps (Sec. 2.2: cell side s = floor(eps / sqrt(2)); Sec. 3:
 * cells linearised along one space-filling curve), so that handles built on
 * it (sba_build_opts.key_level / key_i0 / key_j0) share one curve, as
 * sba_join_pairs requires.  The cell box of a set is
 * [ceil(xmin/s) - 1, floor(xmax/s)] x [ceil(ymin/s) - 1, floor(ymax/s)] over
 * its vertices (the cells its approximations can touch); the grid is
 * anchored at the first cell (i0, j0) of the union of the boxes and has
 * 2^level cells a side, level the smallest in 1..21 that covers the union.
 *   sets    HOST array of n_sets (1..64) polygon sets, each as for
 *           sba_build_approx (DEVICE arrays); sets without polygons are skipped.
 *   level, i0, j0  HOST pointers that receive the grid.
 * Synchronises `stream`.  Errors: SBA_EINVAL (null pointers, bad offsets,
 * an empty polygon, no polygon at all, eps out of range), SBA_ERANGE
 * (|coordinate| >= 2^30), SBA_ELIMIT (more than 64 sets or polygons than
 * sba_build_approx takes; the union wider than 2^21 cells), SBA_ENOMEM,
 * SBA_EDEVICE.
 */
int sba_key_grid(const sba_polygons *sets, int32_t n_sets, int64_t eps, void *stream,
                 int32_t *level, int64_t *i0, int64_t *j0);

/*
 * Per-polygon COUNT and SUM over the points (Sec. 5: the aggregation query
 * answered from the approximation alone, join and aggregation fused).
 *
 *   xy      [2n] int32 x,y interleaved.  16-byte alignment lets the probe use
 *           128-bit loads (torch allocations are aligned).
 *   values  [n] int64 or NULL (COUNT only; sums is then ignored).
 *   n       number of points, >= 0.
 *   counts  [n_polys] uint64, overwritten.
 *   sums    [n_polys] int64, overwritten (may be NULL).
 * A point whose cell lies in no approximation contributes nothing; one whose
 * cell lies in k approximations contributes to all k.  With n == 0 both
 * outputs are zeroed (sums if non-NULL).  Asynchronous on `stream`.  Sums
 * wrap modulo 2^64 if they overflow (not checked).
 */
int sba_aggregate(const int32_t *xy, const int64_t *values, int64_t n, const sba_handle *h,
                  uint64_t *counts, int64_t *sums, void *stream);

/* As sba_aggregate, with the Hilbert layout's search chosen per call
 * (SBA_SEARCH_BINARY or SBA_SEARCH_LEARNED; learned needs a handle built with
 * search = SBA_SEARCH_LEARNED).  Ignored for the grid layout. */
int sba_aggregate_search(const int32_t *xy, const int64_t *values, int64_t n,
                         const sba_handle *h, int32_t search, uint64_t *counts,
                         int64_t *sums, void *stream);

/*
 * sba_aggregate over points in no spatial order, for the layouts whose
 * lookups search large arrays (Hilbert runs; grids with more polygons than
 * LDS bins hold): the points and values are first partitioned into 256
 * buckets, the level-4 Hilbert tiles of the handle's cell box, then probed
 * bucket by bucket so each bucket's part of the structure stays in cache.
 * The answer is sba_aggregate's (search as in sba_aggregate_search).
 *   scratch        DEVICE buffer, 256-byte aligned, of at least
 *                  sba_partition_scratch_bytes(n, values != NULL && sums !=
 *                  NULL) bytes (about 16 B per point), else SBA_ELIMIT; its
 *                  contents are overwritten.  The call allocates nothing.
 * Inputs of fewer than 2^17 points take the direct probe.  Asynchronous.
 */
size_t sba_partition_scratch_bytes(int64_t n, int with_values);
int sba_aggregate_partitioned(const int32_t *xy, const int64_t *values, int64_t n,
                              const sba_handle *h, int32_t search, void *scratch,
                              size_t scratch_bytes, uint64_t *counts, int64_t *sums,
                              void *stream);

/*
 * Result range in one pass (Sec. 6): alpha (COUNT/SUM over A(P)) and the
 * boundary partial beta (over B(P)) of every polygon, so that the exact
 * answer lies in [alpha - beta, alpha] (sums: for non-negative values).
 *   h        the full approximation; hb the boundary-only one
 *            (opts.boundary_only) of the same polygons and eps, else
 *            SBA_EINVAL.
 *   counts, sums    alpha, as sba_aggregate.
 *   bcounts, bsums  beta, as sba_aggregate (sums and bsums both or neither).
 * When both are grid handles in the 16-bit format on the same tiles (build
 * hb with h's tile_log2 and sub_log2, see sba_info) and both directories fit
 * in LDS together, one kernel reads the points once and looks each cell up
 * in both; otherwise two probes run one after the other.  Asynchronous.
 */
int sba_aggregate_range(const int32_t *xy, const int64_t *values, int64_t n,
                        const sba_handle *h, const sba_handle *hb, uint64_t *counts,
                        int64_t *sums, uint64_t *bcounts, int64_t *bsums, void *stream);

/* Name of the one-pass kernel sba_aggregate_range launches for (h, hb), as
 * profilers list it; "" when the call takes two passes.  Per-thread static
 * storage. */
const char *sba_range_kernel(const sba_handle *h, const sba_handle *hb, int with_values);

/*
 * One aggregation task of a batch (serving: viewport queries).
 *   xy, values   the point table (as for sba_aggregate); the task reads the
 *                points with index in [lo, hi).  values may be NULL (COUNT).
 *   h            approximation handle; search: SBA_SEARCH_* for the Hilbert
 *                layout (ignored for the grid).
 *   vx, vy, vw, vh  viewport: only points with vx <= x < vx+vw and
 *                vy <= y < vy+vh count; vw <= 0 or vh <= 0 means no filter.
 *   counts, sums [h->n_polys] outputs (sums may be NULL).
 */
typedef struct {
    const int32_t    *xy;
    const int64_t    *values;
    int64_t           lo, hi;
    const sba_handle *h;
    int32_t           search;
    int32_t           vx, vy, vw, vh;
    uint64_t         *counts;
    int64_t          *sums;
} sba_task;

/*
 * Answer n_tasks aggregation tasks with one persistent launch on `stream`
 * (continuous batching of uneven queries; Sec. 1: interactive level-of-detail
 * exploration).  The outputs of all tasks are zeroed first, then every task
 * adds its points; tasks that name the same output buffers therefore
 * accumulate into them (a query split into several point ranges).  Results
 * are identical to running the tasks one by one.
 *   tasks  HOST array of n_tasks descriptors (copied during the call).
 * Asynchronous on `stream`.  Errors: SBA_EINVAL (null task fields, lo > hi,
 * misaligned xy/values), SBA_ENOMEM, SBA_EDEVICE.
 */
int sba_aggregate_batch(const sba_task *tasks, int32_t n_tasks, void *stream);

/*
 * sba_aggregate_batch without any device allocation, for callers that cannot
 * allocate (code under graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  The same tasks, semantics and results; the tasks'
 * descriptors, their items of at most 2^18 points and the work counter go to
 * a fixed scratch array in the library's device memory of
 * sba_batch_noalloc_bytes() bytes (4 MB) on each device the library runs on,
 * held until the process ends.  A batch that needs more
 * (sba_batch_scratch_bytes) fails with SBA_ELIMIT and leaves the outputs
 * untouched.  Every call on one device uses that device's array, so calls
 * that overlap on a device (other streams, other host threads) race: the
 * caller orders them.  The array's address is looked up on the first call
 * on each device.  Errors: as sba_aggregate_batch, and SBA_ELIMIT.
 */
int sba_aggregate_batch_noalloc(const sba_task *tasks, int32_t n_tasks, void *stream);

/* Scratch bytes a batch needs (-1 for invalid arguments), and the size of the
 * no-allocation entry point's array. */
int64_t sba_batch_scratch_bytes(const sba_task *tasks, int32_t n_tasks);
size_t sba_batch_noalloc_bytes(void);

/*
 * Reorder a point table into G x G buckets of `cell` x `cell` units,
 * row-major, anchored at (x0, y0) (points outside the bucket grid go to the
 * nearest border bucket), so that the points of a viewport are a few
 * contiguous ranges (one per bucket row).  Serving preprocessing.
 *   xy [2n], values [n] (may be NULL) in; out_xy [2n], out_values [n] out.
 *   bucket_off [G*G+1] out: bucket b holds points [bucket_off[b], bucket_off[b+1]).
 *   1 <= G <= 4096, cell >= 1.  Order inside a bucket is unspecified.
 * Asynchronous on `stream`.
 */
int sba_bucket_points(const int32_t *xy, const int64_t *values, int64_t n, int32_t x0,
                      int32_t y0, int32_t cell, int32_t G, int32_t *out_xy,
                      int64_t *out_values, int64_t *bucket_off, void *stream);

/*
 * Cell lookup, for checking the approximation itself.
 *   ij    [2n] int64 cell indices (i, j) interleaved.
 *   ref   [n] int32 out: -1 = no polygon, p >= 0 = exactly polygon p,
 *         <= -2 = the polygon set with index -2-ref (see sba_get_sets).
 * Asynchronous on `stream`.
 */
int sba_lookup_cells(const sba_handle *h, const int64_t *ij, int64_t n, int32_t *ref,
                     void *stream);

/* Multi-polygon sets (host copies).  Pass NULL arrays to query sizes only.
 *   n_sets, n_ids  host out: number of sets and of ids over all sets
 *   off  host [n_sets+1], ids host [n_ids]: ids of set k (ascending) are
 *        ids[off[k] .. off[k+1]).
 * Synchronous. */
int sba_get_sets(const sba_handle *h, int64_t *n_sets, int64_t *n_ids, int64_t *off,
                 int32_t *ids);

/* Hilbert layout: copy the runs into caller DEVICE buffers.
 *   starts [n_runs] uint64: first key of each run (starts[0] = 0, ascending;
 *          the runs partition [0, 4^L) and neighbours differ in their set)
 *   ids    [n_runs] int32: ref of the run, encoded as in sba_lookup_cells.
 * Asynchronous on `stream`. */
int sba_get_runs(const sba_handle *h, uint64_t *starts, int32_t *ids, void *stream);

/* Handle metadata (host struct). */
int sba_info(const sba_handle *h, sba_info_t *info);

/* Name of the probe kernel that sba_aggregate launches for h, with values
 * (with_values != 0) or counts only, as profilers list it (template
 * arguments, no parameters).  Static per-thread storage, valid until the
 * next call on the same thread; "" for a null handle or one without
 * polygons. */
const char *sba_probe_kernel(const sba_handle *h, int with_values);

/* Release the handle's device memory.  The caller must make sure no work
 * using the handle is still queued (synchronise its streams first). */
void sba_free(sba_handle *h);

/*
 * Polygon-polygon join over cells (Sec. 4: blend two rasterized canvases,
 * mask the cells that hold a polygon of each): every pair (p, q), p a
 * polygon of a and q one of b, whose approximations share at least one cell,
 * with the number of shared cells (x s^2: an estimate of the intersection
 * area; conservative approximations pair every two polygons that meet).
 *   a, b     Hilbert handles with the same cell side and key grid (build
 *            both with the same eps and opts.key_level / key_i0 / key_j0),
 *            else SBA_EINVAL.  Either may be boundary-only or centre-sampled.
 *   cap      capacity of the outputs, >= 0.
 *   pa, pb   [cap] int32 DEVICE arrays: polygon of a, polygon of b.
 *   cells    [cap] int64 DEVICE array: shared cells.
 *   n_pairs  host; receives the number of pairs.  Pairs are written in
 *            (p, q) order; if there are more than cap, only the first cap.
 * Synchronous: returns after the outputs are written (it reads sizes back).
 * Errors: SBA_EINVAL, SBA_ENOMEM, SBA_EDEVICE, SBA_ELIMIT (2^32 or more
 * (cell interval, pair) incidences).
 */
int sba_join_pairs(const sba_handle *a, const sba_handle *b, int64_t cap, int32_t *pa,
                   int32_t *pb, int64_t *cells, int64_t *n_pairs, void *stream);

/* ------------------------------------------------------------ point index
 *
 * Point-side pre-aggregation (Sec. 3, point indexing): the points are
 * linearised to the Hilbert keys of their cells and kept as a sorted key
 * array with a prefix-sum array of their values.  A polygon query then costs
 * a lower-bound search at both ends of each query cell instead of a pass over
 * the points: the query cells are the runs of a Hilbert handle built on the
 * index's key grid (each run is a contiguous key range and a union of aligned
 * quadtree cells), COUNT of a run = ub - lb, SUM = prefix[ub] - prefix[lb].
 * The searches are binary searches or a RadixSpline (Sec. 3: spline knots
 * with a bounded error plus a radix table over the key prefixes).  The
 * answer is the one sba_aggregate gives over the same points and handle.
 */
typedef struct sba_pindex sba_pindex;

typedef struct {
    int32_t radix_bits;   /* RadixSpline radix table: 2^radix_bits + 2 entries over the top
                             bits of the key (0 -> 20; 1..28, capped at 2L)             */
    int32_t spline_err;   /* RadixSpline error bound in positions (0 -> 32; 1..2^20)     */
} sba_pindex_opts;

typedef struct {
    int64_t n;            /* points indexed */
    int64_t eps, s;       /* distance bound and cell side (as for a handle)           */
    int64_t key_i0, key_j0;  /* key grid origin, in cells                              */
    int32_t key_level;    /* key grid side 2^key_level cells                          */
    int32_t has_values;   /* prefix sums stored                                        */
    int64_t n_distinct;   /* distinct cell keys                                        */
    int64_t n_knots;      /* RadixSpline knots                                         */
    int32_t radix_bits, spline_err;
    int64_t bytes;        /* device bytes held by the index                           */
    double  build_ms;     /* wall time of the build, host clock                       */
} sba_pindex_info_t;

/*
 * Build the point index of n points for cell side s(eps) (the same cells as
 * a handle built with eps).
 *   xy      [2n] int32 x,y interleaved (DEVICE), read during the call only.
 *   values  [n] int64 (DEVICE) or NULL (COUNT only).
 *   eps     2 <= eps <= 2^28.   opts: host pointer or NULL for defaults.
 *   stream  work is queued on it; the call synchronises it (it reads the
 *           point box and sizes back) and returns once the index is complete.
 * The key grid is anchored at the first cell of the points' cell box, L =
 * smallest level covering it.  Limits (SBA_ELIMIT): n < 2^31; the points'
 * cell box at most 2^21 cells and less than 2^31 coordinate units per side.
 * Errors: SBA_EINVAL, SBA_ENOMEM, SBA_EDEVICE, SBA_ELIMIT.
 */
int sba_pindex_build(const int32_t *xy, const int64_t *values, int64_t n, int64_t eps,
                     const sba_pindex_opts *opts, void *stream, sba_pindex **out);

/* Index metadata (host struct). */
int sba_pindex_info(const sba_pindex *ix, sba_pindex_info_t *info);

/*
 * Per-polygon COUNT and SUM of the indexed points over the approximation h.
 *   h       a Hilbert handle whose cell side and key grid are the index's
 *           (built with opts.key_level / key_i0 / key_j0 from sba_pindex_info
 *           and the same eps), else SBA_EINVAL.  A handle without polygons
 *           or with no cell in the key grid gives zero outputs.
 *   search  SBA_SEARCH_BINARY (binary searches over the keys) or
 *           SBA_SEARCH_LEARNED (RadixSpline estimate, bounded search, full
 *           binary search if the bound ever fails).
 *   counts  [n_polys] uint64, overwritten.  sums [n_polys] int64, overwritten
 *           (may be NULL; SBA_EINVAL if non-NULL and the index has no values).
 * Asynchronous on `stream`; allocates nothing.  Sums wrap modulo 2^64.
 */
int sba_pindex_aggregate(const sba_pindex *ix, const sba_handle *h, int32_t search,
                         uint64_t *counts, int64_t *sums, void *stream);

/* Release the index's device memory (no work using it may still be queued). */
void sba_pindex_free(sba_pindex *ix);

/* Static string describing an error code. */
const char *sba_strerror(int code);

/* Library version string. */
const char *sba_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SBA_H */
