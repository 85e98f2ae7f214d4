/*
 * sba_debug.h -- helpers of libsba for its own tests and tuning: the integer
 * arithmetic the kernels use, evaluated on the host so that it can be checked
 * without a GPU; process-wide launch-shape switches; and entry points that run
 * internal device primitives and searches on their own so that tests can check
 * them against plain definitions.  Not needed by applications.
 */
#ifndef SBA_DEBUG_H
#define SBA_DEBUG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* q[k] = floor(n[k] / s) by the probes' multiply-shift division (Granlund and
 * Montgomery, 1994, Thm. 4.2 with 31-bit dividends).  Host arrays of `count`
 * entries; every n[k] must be < 2^31.  SBA_EINVAL if s is outside [1, 2^28]. */
int sba_debug_celldiv(int64_t s, const uint32_t *n, int64_t count, uint32_t *q);

/* Hilbert index of cell (i, j) at level L (Sec. 3 linearisation), and its
 * inverse, exactly as the kernels compute them. */
uint64_t sba_debug_hilbert(int L, uint32_t i, uint32_t j);
/* The probes' Hilbert encoder that takes four levels at a time through a
 * table (built from the one-level step), host copy; L <= 16. */
uint64_t sba_debug_hilbert_tab(int L, uint32_t i, uint32_t j);

void sba_debug_hilbert_cell(int L, uint64_t d, uint32_t *i, uint32_t *j);

/* Workgroups per compute unit of the streaming probes (default 8, 1..64).
 * Process-wide; for launch-shape sweeps. */
int sba_debug_set_blocks_per_cu(int k);

/* Cap on workgroups per compute unit of the grid probe with the LDS-staged
 * directory (0: as many as LDS and wave slots allow, the default; 1..4).
 * Process-wide; for launch-shape sweeps. */
int sba_debug_set_grid16_per_cu(int k);

/* How the LDS-directory grid probe adds points of multi-polygon cells:
 * -1 automatic (default), 0 walk the global set table, 1 walk a copy staged
 * in LDS, 2 one LDS bin per set, expanded once per workgroup.  A mode that
 * does not fit the LDS falls back to the next one down.  Process-wide. */
int sba_debug_grid16_sets(int mode);

/* Whether the LDS-directory grid probe may stage the sub-directory in LDS as
 * well (16-bit entries, when they fit beside the directory and the bins):
 * -1 when it fits (default), 0 never (read from global memory).
 * Process-wide; for comparison runs and tests of both paths. */
int sba_debug_grid16_lsub(int mode);

/* Build paths, process-wide, read at build time.  Bits set in `off` turn a
 * path off: 1 = sorting each polygon's events in LDS (fused with the
 * coverage step), so that all events take the global radix sort and scans;
 * 2 = bucketing the toggles by row, so that they take the global radix sort;
 * 4 = collecting the distinct polygon sets through a hash table and numbering
 * them in one workgroup, so that all multi-polygon segments take the global
 * radix sort.  0 (default) takes each path wherever it applies (builds
 * without a clip window, polygons of at most 16,384 events, rows of at most
 * 512 toggles; set keys below 2^31 and at most 8,192 distinct sets).
 * SBA_EINVAL outside 0..7.  For tests of both sides of each choice. */
int sba_debug_build_paths(int off);

/* The paths the last build in the process took, same bits (1: per-polygon
 * event sort, 2: toggle row buckets, 4: hashed set table).  Test support. */
int sba_debug_last_build_paths(void);

/* 1: grid builds store the 32-bit format (directory read from global memory
 * by the probes) even where the 16-bit LDS-staged format would fit
 * (comparison runs); 0: default.  Process-wide, read at build time. */
int sba_debug_force_wide_grid(int on);

/* The learned run search of a Hilbert handle (built with the learned
 * index) over the cells of n points (DEVICE xy, x,y interleaved): the host
 * *fallbacks receives how many searches failed their bracket check and took
 * the full binary search (an exact leaf error bound makes that 0), and
 * *mismatches how many answers differ from the binary search's (must be 0).
 * Points outside the key grid are skipped.  Synchronous.  Test support. */
struct sba_handle;
int sba_debug_learned_fallbacks(const struct sba_handle *h, const int32_t *xy, int64_t n,
                                int64_t *fallbacks, int64_t *mismatches, void *stream);

/* Lower bounds in a point index: out[k] = number of indexed points whose cell
 * key is below v[k] (0 <= v[k] <= 4^L), by binary search (search 0) or the
 * RadixSpline (search 1).  v and out are DEVICE arrays of n entries; the host
 * *fallbacks receives how many RadixSpline windows failed their check and
 * needed the full search (the spline's error bound makes that 0).
 * Synchronous (synchronises `stream`).  Test support. */
struct sba_pindex;
int sba_debug_pindex_lb(const struct sba_pindex *ix, const uint64_t *v, int64_t n, int32_t search,
                        int64_t *out, int64_t *fallbacks, void *stream);

/* The build's stable LSD radix sort: n DEVICE keys ordered by their low
 * `bits` bits (1..64), the optional DEVICE uint32 payload `vals` (may be
 * null) moved with them; the result is left in keys/vals.  The passes take
 * 8-bit digits, or 9-bit ones for fewer than 4,194,304 keys where
 * ceil(bits / 9) < ceil(bits / 8), and cover whole digits, so keys must be
 * below 2^bits (as the build's are); bits above the last digit are ignored
 * (for a multiple of 8 bits: the bytes above them).  SBA_EINVAL for a bad
 * size or bit count.  Synchronous.  Test support. */
int sba_debug_radix_sort(uint64_t *keys, uint32_t *vals, int64_t n, int32_t bits, void *stream);

/* A plain streaming read of `bytes` DEVICE bytes at `a` and, unless `b` is
 * null, as many at `b` (the probe's two input streams; sizes and addresses
 * multiples of 16, SBA_EINVAL otherwise, or for blocks outside 1..65536 or
 * threads not a multiple of 64 in 64..1024): `blocks` workgroups of
 * `threads` lanes read the buffers in 16-byte non-temporal loads and leave
 * the XOR of all their 32-bit words in the DEVICE word *xor_out (zeroed
 * first).  It measures the read rate a kernel that only reads its input can
 * reach, the yardstick of the probes' fraction of peak.  Asynchronous on
 * `stream`.  Test and benchmark support. */
int sba_debug_stream_read(const void *a, const void *b, int64_t bytes, int32_t blocks,
                          int32_t threads, uint32_t *xor_out, void *stream);

/* The build's batched exclusive prefix sums: for k < m (1..8), out[k][i] =
 * in[k][0] + ... + in[k][i-1] over n[k] entries (out[k] may be in[k]) and
 * total[k] = the sum of all n[k].  in, out and n are HOST arrays of m
 * entries; in[k], out[k] and total (m entries) are DEVICE memory.  Up to 4
 * arrays of at most 2^21 entries share one pair of launches; others are
 * scanned one by one.  Synchronous.  Test support. */
int sba_debug_scan_multi(int32_t m, const int64_t *const *in, int64_t *const *out,
                         const int64_t *n, int64_t *total, void *stream);

#ifdef __cplusplus
}
#endif
#endif
