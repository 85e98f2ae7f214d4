/*
 * sba_oracle.c -- plain CPU oracle for the distance-bounded approximate
 * point-in-polygon aggregation join of Tzirita Zacharatou, Kipf, Sabek,
 * Pandey, Doraiswamy and Markl, "The Case for Distance-Bounded Spatial
 * Approximations" (CIDR 2021).
 *
 * TEST INFRASTRUCTURE.  This library is the checker of the GPU library, not a
 * part of it: only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark load it.  It shares no source, header, table or helper with the
 * GPU path, and it is written to be read against the paper, not to be fast.
 *
 * Everything is exact integer arithmetic (int64, and int128 wherever a
 * product of two coordinate differences is formed).  Coordinates are int32
 * fixed-point; the grid of cells is anchored at (0,0).
 *
 * Definitions followed (section numbers are the paper's):
 *
 *   s      Cell side (Sec. 2.2): boundary cells have side eps/sqrt(2), i.e. a
 *          diagonal of at most eps.  In integers: the largest s >= 1 with
 *          2 s^2 <= eps^2.
 *   cell   cell(p) = (floor(px / s), floor(py / s)); cell (i,j) covers the
 *          half-open square [is,(i+1)s) x [js,(j+1)s) and has the closed
 *          square Q(i,j) = [is,(i+1)s] x [js,(j+1)s].
 *   B(P)   Boundary cells (Sec. 2.2, conservative raster: every cell that
 *          overlaps the boundary, however slightly, is part of the
 *          approximation): cells whose closed square meets a closed edge of
 *          any ring of P.
 *   I(P)   Interior cells (Sec. 2.2: interior cells add no error): cells not
 *          in B(P) whose lower-left corner (is, js) is inside P by the
 *          crossing-number rule.  Such a square touches no edge, so every one
 *          of its points is on the same side; the corner stands for all.
 *   A(P)   = B(P) u I(P), the conservative eps-approximation of P.
 *   inside Crossing-number rule, even-odd over all rings: the edge
 *          (x1,y1)->(x2,y2) counts for point (px,py) iff exactly one of
 *          y1 > py, y2 > py holds and px < x1 + (py-y1)(x2-x1)/(y2-y1).
 *   aggregate (Sec. 5, the spatial aggregation query; Sec. 5.1, the join is
 *          answered from the approximation alone and fused with the
 *          aggregation): for every point p and every P with cell(p) in A(P),
 *          count[P] += 1 and sum[P] += value[p].  A point whose cell lies in
 *          several approximations counts for each of them.
 *   exact  The same aggregate with "p inside P" in place of cell membership.
 *   invariant (Sec. 2.2, Hausdorff eps-approximation): every (p, P) on which
 *          the approximate and the exact predicate differ has p within
 *          distance eps of the boundary of P, and no point inside P is
 *          missed (conservative raster: false positives only).
 *   C(P)   Centre-sampled approximation (Sec. 2.2, non-conservative raster:
 *          cells with little overlap may be left out, so false negatives are
 *          allowed): the cells whose centre ((i+1/2)s, (j+1/2)s) is inside P
 *          by the crossing-number rule.  A point whose membership differs
 *          from its cell centre's is separated from the centre by the
 *          boundary, so it lies within half a diagonal, eps/2, of it.
 *   hilbert (Sec. 3, linearisation of cells by a space-filling curve): the
 *          Hilbert index d(i,j) at level L with (0,0)->0, (0,1)->1,
 *          (1,1)->2, (1,0)->3 at level 1, and the maximal runs of
 *          consecutive indices whose cells carry the same polygon set.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef __int128 i128;

/* ------------------------------------------------------------------ */
/* integer helpers                                                     */
/* ------------------------------------------------------------------ */

/* floor(a / b) for b > 0 */
static i128 fdiv(i128 a, i128 b)
{
    i128 q = a / b;
    if (a % b != 0 && a < 0) q -= 1;
    return q;
}

/* ceil(a / b) for b > 0 */
static i128 cdiv(i128 a, i128 b)
{
    i128 q = a / b;
    if (a % b != 0 && a > 0) q += 1;
    return q;
}

static int64_t min64(int64_t a, int64_t b) { return a < b ? a : b; }
static int64_t max64(int64_t a, int64_t b) { return a > b ? a : b; }

/* Cell side: the largest s with 2 s^2 <= eps^2 (diagonal s*sqrt(2) <= eps).
 * Returns 0 when no cell side >= 1 exists or eps is beyond the supported
 * range (eps must lie in [2, 2^28]). */
int64_t orc_cell_side(int64_t eps)
{
    if (eps < 2 || eps > ((int64_t)1 << 28)) return 0;
    int64_t t = eps * eps / 2;                 /* floor(eps^2 / 2) */
    int64_t s = (int64_t)sqrt((double)t);
    while (s > 0 && s * s > t) s--;
    while ((s + 1) * (s + 1) <= t) s++;
    return s;
}

/* ------------------------------------------------------------------ */
/* geometry predicates, straight from the definitions                  */
/* ------------------------------------------------------------------ */

/* Does the closed segment a-b meet the closed axis-aligned square
 * [qx0,qx1] x [qy0,qy1]?  The two convex sets are disjoint iff one of the
 * three candidate axes separates them: the x axis, the y axis (bounding
 * boxes disjoint), or the segment's normal (all four corners strictly on
 * one side of the segment's line). */
static int seg_meets_square(int64_t ax, int64_t ay, int64_t bx, int64_t by,
                            int64_t qx0, int64_t qy0, int64_t qx1, int64_t qy1)
{
    if (max64(ax, bx) < qx0 || min64(ax, bx) > qx1) return 0;
    if (max64(ay, by) < qy0 || min64(ay, by) > qy1) return 0;
    int64_t cx[4] = {qx0, qx1, qx1, qx0};
    int64_t cy[4] = {qy0, qy0, qy1, qy1};
    int pos = 0, neg = 0;
    for (int k = 0; k < 4; k++) {
        i128 c = (i128)(bx - ax) * (cy[k] - ay) - (i128)(by - ay) * (cx[k] - ax);
        if (c > 0) pos++;
        else if (c < 0) neg++;
    }
    return !(pos == 4 || neg == 4);
}

/* Crossing-number contribution of edge (x1,y1)->(x2,y2) for point (px,py):
 * the rightward ray from p crosses the edge under the half-open rule. */
static int edge_crosses_ray(int64_t px, int64_t py,
                            int64_t x1, int64_t y1, int64_t x2, int64_t y2)
{
    if ((y1 > py) == (y2 > py)) return 0;
    /* px < x1 + (py - y1)(x2 - x1)/(y2 - y1), multiplied out by (y2 - y1) */
    i128 lhs = (i128)(px - x1) * (y2 - y1);
    i128 rhs = (i128)(py - y1) * (x2 - x1);
    return (y2 > y1) ? (lhs < rhs) : (lhs > rhs);
}

/* ------------------------------------------------------------------ */
/* polygons                                                            */
/* ------------------------------------------------------------------ */

typedef struct {
    int32_t n_polys;
    const int32_t *ring_off;   /* [n_polys+1] ring ranges per polygon */
    const int64_t *vert_off;   /* [n_rings+1] vertex ranges per ring   */
    const int32_t *xy;         /* [2*n_verts] x,y interleaved           */
} polyset;

/* Visit every edge of polygon p: calls body with (x1,y1,x2,y2); rings are
 * implicitly closed (last vertex joins the first). */
#define FOR_EACH_EDGE(ps, p, X1, Y1, X2, Y2, ...)                             \
    for (int32_t r_ = (ps)->ring_off[p]; r_ < (ps)->ring_off[(p) + 1]; r_++) { \
        int64_t v0_ = (ps)->vert_off[r_], v1_ = (ps)->vert_off[r_ + 1];        \
        for (int64_t v_ = v0_; v_ < v1_; v_++) {                               \
            int64_t w_ = (v_ + 1 < v1_) ? v_ + 1 : v0_;                        \
            int64_t X1 = (ps)->xy[2 * v_], Y1 = (ps)->xy[2 * v_ + 1];          \
            int64_t X2 = (ps)->xy[2 * w_], Y2 = (ps)->xy[2 * w_ + 1];          \
            __VA_ARGS__                                                        \
        }                                                                      \
    }

static int point_in_poly(const polyset *ps, int32_t p, int64_t px, int64_t py)
{
    int odd = 0;
    FOR_EACH_EDGE(ps, p, x1, y1, x2, y2, { odd ^= edge_crosses_ray(px, py, x1, y1, x2, y2); })
    return odd;
}

/* point_in_poly at a point given in doubled coordinates (2px, 2py): the
 * polygon is doubled with it, which changes no incidence */
static int point_in_poly2(const polyset *ps, int32_t p, int64_t px2, int64_t py2)
{
    int odd = 0;
    FOR_EACH_EDGE(ps, p, x1, y1, x2, y2,
                  { odd ^= edge_crosses_ray(px2, py2, 2 * x1, 2 * y1, 2 * x2, 2 * y2); })
    return odd;
}

static int cell_in_boundary(const polyset *ps, int32_t p, int64_t s, int64_t i, int64_t j)
{
    int64_t qx0 = i * s, qy0 = j * s, qx1 = qx0 + s, qy1 = qy0 + s;
    FOR_EACH_EDGE(ps, p, x1, y1, x2, y2, {
        if (seg_meets_square(x1, y1, x2, y2, qx0, qy0, qx1, qy1)) return 1;
    })
    return 0;
}

/* Exact test k * dist(p, [a,b])^2 <= eps^2 for the closed segment a-b, with
 * k = 1 (distance at most eps) or k = 4 (distance at most eps/2).
 *
 * With v = b - a and w = p - a, the closest point of the segment is a when
 * w.v <= 0, b when w.v >= |v|^2, and otherwise the foot of the perpendicular,
 * at distance |v x w| / |v|.  The interior case is compared squared and
 * multiplied out: k (v x w)^2 <= eps^2 |v|^2.  Coordinates are below 2^30 in
 * magnitude, so every difference is below 2^31, |v x w| < 2^63,
 * k (v x w)^2 < 2^128 and eps^2 |v|^2 < 2^56 * 2^63: both sides fit an
 * unsigned 128-bit integer, and the endpoint cases fit int128. */
static int seg_within_k(int64_t px, int64_t py, int64_t ax, int64_t ay,
                        int64_t bx, int64_t by, int64_t eps, int k)
{
    typedef unsigned __int128 u128;
    i128 vx = bx - ax, vy = by - ay, wx = px - ax, wy = py - ay;
    i128 e2 = (i128)eps * eps;
    i128 t = wx * vx + wy * vy;
    i128 l2 = vx * vx + vy * vy;
    if (t <= 0) return k * (wx * wx + wy * wy) <= e2;
    if (t >= l2) {
        i128 ux = px - bx, uy = py - by;
        return k * (ux * ux + uy * uy) <= e2;
    }
    i128 cr = vx * wy - vy * wx;
    u128 c = (u128)(cr < 0 ? -cr : cr);
    return (u128)k * (c * c) <= (u128)e2 * (u128)l2;
}

/* p within eps (half = 0) or eps/2 (half = 1) of some edge of polygon p */
static int near_boundary(const polyset *ps, int32_t p, int64_t px, int64_t py, int64_t eps,
                         int half)
{
    FOR_EACH_EDGE(ps, p, x1, y1, x2, y2, {
        if (seg_within_k(px, py, x1, y1, x2, y2, eps, half ? 4 : 1)) return 1;
    })
    return 0;
}

static void poly_bbox(const polyset *ps, int32_t p, int64_t *xmin, int64_t *ymin,
                      int64_t *xmax, int64_t *ymax)
{
    int64_t a = INT64_MAX, b = INT64_MAX, c = INT64_MIN, d = INT64_MIN;
    for (int32_t r = ps->ring_off[p]; r < ps->ring_off[p + 1]; r++)
        for (int64_t v = ps->vert_off[r]; v < ps->vert_off[r + 1]; v++) {
            a = min64(a, ps->xy[2 * v]);
            b = min64(b, ps->xy[2 * v + 1]);
            c = max64(c, ps->xy[2 * v]);
            d = max64(d, ps->xy[2 * v + 1]);
        }
    *xmin = a; *ymin = b; *xmax = c; *ymax = d;
}

/* Validate the CSR arrays; 0 if usable, -1 otherwise. */
static int polys_ok(const polyset *ps)
{
    if (ps->n_polys < 0) return -1;
    if (ps->ring_off[0] != 0) return -1;
    for (int32_t p = 0; p < ps->n_polys; p++)
        if (ps->ring_off[p + 1] < ps->ring_off[p]) return -1;
    int32_t nr = ps->ring_off[ps->n_polys];
    if (ps->vert_off[0] != 0) return -1;
    for (int32_t r = 0; r < nr; r++)
        if (ps->vert_off[r + 1] < ps->vert_off[r]) return -1;
    int64_t nv = ps->vert_off[nr];
    for (int64_t v = 0; v < 2 * nv; v++)
        if (ps->xy[v] <= -(1 << 30) || ps->xy[v] >= (1 << 30)) return -1;
    for (int32_t p = 0; p < ps->n_polys; p++)
        if (ps->vert_off[ps->ring_off[p + 1]] == ps->vert_off[ps->ring_off[p]]) return -1;
    return 0;
}

/* ------------------------------------------------------------------ */
/* brute-force raster: the definition, cell by cell, edge by edge      */
/* ------------------------------------------------------------------ */

/* For every polygon p and every cell (i,j) of the window
 * [i0,i0+nw) x [j0,j0+nh):  out[(p*nh + (j-j0))*nw + (i-i0)] =
 *   2 if the cell is in B(P), 1 if in I(P), 0 otherwise.
 * Cost: cells x edges.  For tiny inputs only. */
int orc_raster_brute(int32_t n_polys, const int32_t *ring_off, const int64_t *vert_off,
                     const int32_t *xy, int64_t s, int64_t i0, int64_t j0,
                     int64_t nw, int64_t nh, uint8_t *out)
{
    polyset ps = {n_polys, ring_off, vert_off, xy};
    if (s < 1 || nw < 0 || nh < 0 || polys_ok(&ps)) return -1;
    for (int32_t p = 0; p < n_polys; p++)
        for (int64_t j = j0; j < j0 + nh; j++)
            for (int64_t i = i0; i < i0 + nw; i++) {
                uint8_t m = 0;
                if (cell_in_boundary(&ps, p, s, i, j)) m = 2;
                else if (point_in_poly(&ps, p, i * s, j * s)) m = 1;
                out[((int64_t)p * nh + (j - j0)) * nw + (i - i0)] = m;
            }
    return 0;
}

/* The centre-sampled approximation by its definition, cell by cell:
 * out[(p*nh + (j-j0))*nw + (i-i0)] = 1 if the centre of cell (i,j) is inside
 * P, else 0.  For tiny inputs only. */
int orc_centre_brute(int32_t n_polys, const int32_t *ring_off, const int64_t *vert_off,
                     const int32_t *xy, int64_t s, int64_t i0, int64_t j0,
                     int64_t nw, int64_t nh, uint8_t *out)
{
    polyset ps = {n_polys, ring_off, vert_off, xy};
    if (s < 1 || nw < 0 || nh < 0 || polys_ok(&ps)) return -1;
    for (int32_t p = 0; p < n_polys; p++)
        for (int64_t j = j0; j < j0 + nh; j++)
            for (int64_t i = i0; i < i0 + nw; i++)
                out[((int64_t)p * nh + (j - j0)) * nw + (i - i0)] =
                    (uint8_t)point_in_poly2(&ps, p, (2 * i + 1) * s, (2 * j + 1) * s);
    return 0;
}

/* ------------------------------------------------------------------ */
/* scanline raster: A(P) as sorted, disjoint row intervals             */
/* ------------------------------------------------------------------ */

typedef struct { int64_t row, x0, x1; } ivl;   /* cells [x0, x1) of a row */

typedef struct { ivl *a; int64_t n, cap; } ivec;

static int ivec_push(ivec *v, int64_t row, int64_t x0, int64_t x1)
{
    if (v->n == v->cap) {
        int64_t nc = v->cap ? 2 * v->cap : 64;
        ivl *na = (ivl *)realloc(v->a, (size_t)nc * sizeof(ivl));
        if (!na) return -1;
        v->a = na; v->cap = nc;
    }
    v->a[v->n].row = row; v->a[v->n].x0 = x0; v->a[v->n].x1 = x1;
    v->n++;
    return 0;
}

static int ivl_cmp(const void *pa, const void *pb)
{
    const ivl *a = (const ivl *)pa, *b = (const ivl *)pb;
    if (a->row != b->row) return a->row < b->row ? -1 : 1;
    if (a->x0 != b->x0) return a->x0 < b->x0 ? -1 : 1;
    if (a->x1 != b->x1) return a->x1 < b->x1 ? -1 : 1;
    return 0;
}

typedef struct {
    int64_t ci0, ci1, cj0, cj1;   /* cell bounding box of A(P), inclusive */
    int64_t *row_off;             /* [cj1-cj0+2] offsets into x0/x1        */
    int64_t *x0, *x1;             /* disjoint sorted intervals per row     */
    int64_t n_iv;
} prows;

/* Scan form of A(P), equal to the brute form cell for cell:
 *
 *  boundary part -- every edge meets the closed strip [js,(j+1)s] of rows
 *  j in [ceil(ymin/s)-1, floor(ymax/s)] (ymin,ymax of the edge).  The part
 *  of the edge inside the strip is a segment with x-range [xlo, xhi]; the
 *  closed squares of that strip it meets are exactly those whose x-range
 *  [is,(i+1)s] overlaps [xlo,xhi], i.e. i in [ceil(xlo/s)-1, floor(xhi/s)].
 *
 *  interior part -- the row line y = js is crossed (half-open rule) by the
 *  edges with js in [ymin, ymax).  The crossing at x = xc lies to the right
 *  of the corner is exactly for i < ceil(xc/s).  With the crossings of the
 *  row sorted as k1 <= k2 <= ..., corner (is,js) is inside P iff an odd
 *  number of k exceed i, i.e. i in [k1,k2) u [k3,k4) u ...
 *
 *  A(P) = B(P) u I(P) = B(P) u {cells whose corner is inside}, since the
 *  second set differs from I(P) only by cells of B(P).
 *
 *  centre-sampled (mode ORC_CENTRE) -- no boundary part; the row line is the
 *  line of the centres, y = (j+1/2)s, crossed by the edges with
 *  2 ymin <= (2j+1)s < 2 ymax.  With 2xc = N/D (D = y2-y1 > 0 after a sign
 *  change) the centre of cell i lies left of the crossing iff
 *  (2i+1) s D < N, i.e. i < ceil((N - sD) / (2sD)); spans as above.
 *
 *  mode: ORC_FULL A(P), ORC_BOUNDARY B(P) only, ORC_CENTRE C(P). */
enum { ORC_FULL = 0, ORC_BOUNDARY = 1, ORC_CENTRE = 2 };

static int build_rows(const polyset *ps, int32_t p, int64_t s, int mode, prows *out)
{
    const int with_interior = mode != ORC_BOUNDARY, with_boundary = mode != ORC_CENTRE;
    int64_t xmin, ymin, xmax, ymax;
    poly_bbox(ps, p, &xmin, &ymin, &xmax, &ymax);
    out->ci0 = (int64_t)cdiv(xmin, s) - 1;
    out->ci1 = (int64_t)fdiv(xmax, s);
    out->cj0 = (int64_t)cdiv(ymin, s) - 1;
    out->cj1 = (int64_t)fdiv(ymax, s);

    ivec iv = {0, 0, 0};
    ivec cr = {0, 0, 0};          /* crossings: row, k (x1 unused) */
    int err = 0;

    FOR_EACH_EDGE(ps, p, x1, y1, x2, y2, {
        int64_t ey0 = min64(y1, y2), ey1 = max64(y1, y2);
        /* boundary strips */
        int64_t ja = (int64_t)cdiv(ey0, s) - 1, jb = (int64_t)fdiv(ey1, s);
        if (!with_boundary) jb = ja - 1;
        for (int64_t j = ja; j <= jb && !err; j++) {
            int64_t c0, c1;
            if (y1 == y2) {
                c0 = (int64_t)cdiv(min64(x1, x2), s) - 1;
                c1 = (int64_t)fdiv(max64(x1, x2), s);
            } else {
                int64_t ya = max64(ey0, j * s), yb = min64(ey1, (j + 1) * s);
                if (ya > yb) continue;
                /* x(y) = (x1*(y2-y1) + (y-y1)*(x2-x1)) / (y2-y1) */
                i128 den = (i128)(y2 - y1);
                i128 na = (i128)x1 * den + (i128)(ya - y1) * (x2 - x1);
                i128 nb = (i128)x1 * den + (i128)(yb - y1) * (x2 - x1);
                if (den < 0) { den = -den; na = -na; nb = -nb; }
                i128 lo = na < nb ? na : nb, hi = na < nb ? nb : na;
                c0 = (int64_t)cdiv(lo, den * s) - 1;
                c1 = (int64_t)fdiv(hi, den * s);
            }
            if (ivec_push(&iv, j, c0, c1 + 1)) err = 1;
        }
        /* crossings of centre lines y = (j+1/2)s with (2j+1)s in [2 ey0, 2 ey1) */
        if (y1 != y2 && mode == ORC_CENTRE) {
            int64_t ka = (int64_t)cdiv(2 * ey0 - s, 2 * s), kb = (int64_t)cdiv(2 * ey1 - s, 2 * s) - 1;
            for (int64_t j = ka; j <= kb && !err; j++) {
                i128 den = (i128)(y2 - y1);
                i128 num = (i128)2 * x1 * den + ((i128)(2 * j + 1) * s - 2 * y1) * (x2 - x1);
                if (den < 0) { den = -den; num = -num; }
                int64_t k = (int64_t)cdiv(num - s * den, 2 * s * den);
                if (ivec_push(&cr, j, k, 0)) err = 1;
            }
        }
        /* crossings of row lines y = js with js in [ey0, ey1) */
        if (y1 != y2 && mode != ORC_CENTRE) {
            int64_t ka = (int64_t)cdiv(ey0, s), kb = (int64_t)cdiv(ey1, s) - 1;
            for (int64_t j = ka; j <= kb && !err; j++) {
                i128 den = (i128)(y2 - y1);
                i128 num = (i128)x1 * den + (i128)(j * s - y1) * (x2 - x1);
                if (den < 0) { den = -den; num = -num; }
                int64_t k = (int64_t)cdiv(num, den * s);
                if (ivec_push(&cr, j, k, 0)) err = 1;
            }
        }
    })
    if (!err && cr.n) {
        qsort(cr.a, (size_t)cr.n, sizeof(ivl), ivl_cmp);
        /* each row line meets a closed ring an even number of times */
        for (int64_t t = 0; t + 1 < cr.n && !err; t += 2) {
            if (cr.a[t].row != cr.a[t + 1].row) { err = 2; break; }
            if (with_interior && cr.a[t].x0 < cr.a[t + 1].x0)
                if (ivec_push(&iv, cr.a[t].row, cr.a[t].x0, cr.a[t + 1].x0)) err = 1;
        }
        if (cr.n % 2) err = 2;
    }
    free(cr.a);
    if (err) { free(iv.a); return -1; }

    if (iv.n > 1) qsort(iv.a, (size_t)iv.n, sizeof(ivl), ivl_cmp);
    int64_t nrows = out->cj1 - out->cj0 + 1;
    out->row_off = (int64_t *)calloc((size_t)nrows + 1, sizeof(int64_t));
    out->x0 = (int64_t *)malloc((size_t)(iv.n ? iv.n : 1) * sizeof(int64_t));
    out->x1 = (int64_t *)malloc((size_t)(iv.n ? iv.n : 1) * sizeof(int64_t));
    if (!out->row_off || !out->x0 || !out->x1) { free(iv.a); return -1; }
    int64_t m = 0;
    for (int64_t t = 0; t < iv.n; t++) {
        int64_t r = iv.a[t].row;
        if (m > 0 && iv.a[t - 1].row == r && iv.a[t].x0 <= out->x1[m - 1]) {
            if (iv.a[t].x1 > out->x1[m - 1]) out->x1[m - 1] = iv.a[t].x1;
            continue;
        }
        out->x0[m] = iv.a[t].x0;
        out->x1[m] = iv.a[t].x1;
        out->row_off[r - out->cj0 + 1]++;
        m++;
    }
    for (int64_t r = 0; r < nrows; r++) out->row_off[r + 1] += out->row_off[r];
    out->n_iv = m;
    free(iv.a);
    return 0;
}

static int prows_contains(const prows *pr, int64_t i, int64_t j)
{
    if (j < pr->cj0 || j > pr->cj1 || i < pr->ci0 || i > pr->ci1) return 0;
    int64_t lo = pr->row_off[j - pr->cj0], hi = pr->row_off[j - pr->cj0 + 1];
    /* last interval with x0 <= i */
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (pr->x0[mid] <= i) lo = mid + 1; else hi = mid;
    }
    return lo > pr->row_off[j - pr->cj0] && i < pr->x1[lo - 1];
}

/* ------------------------------------------------------------------ */
/* the approximation object                                            */
/* ------------------------------------------------------------------ */

typedef struct {
    int64_t eps, s;
    int mode;                     /* ORC_FULL, ORC_BOUNDARY or ORC_CENTRE */
    int32_t n_polys;
    int32_t *ring_off; int64_t *vert_off; int32_t *xy;   /* own copy */
    polyset ps;
    prows *rows;
    /* candidate filter: uniform buckets over the union of the cell boxes */
    int64_t ui0, uj0, uw, uh;     /* union cell box                     */
    int64_t bsz, bw, bh;          /* bucket side (cells), bucket counts */
    int64_t *boff;                /* [bw*bh+1]                          */
    int32_t *bids;
} orc_approx;

void orc_free(orc_approx *a)
{
    if (!a) return;
    if (a->rows) {
        for (int32_t p = 0; p < a->n_polys; p++) {
            free(a->rows[p].row_off); free(a->rows[p].x0); free(a->rows[p].x1);
        }
        free(a->rows);
    }
    free(a->ring_off); free(a->vert_off); free(a->xy);
    free(a->boff); free(a->bids);
    free(a);
}

/* mode 1: only the boundary cells B(P) of every polygon (the cells over
 * which the partial count of Sec. 6's result range is taken); 2: the
 * centre-sampled C(P); 0: A(P) = B(P) u I(P). */
orc_approx *orc_build_mode(int32_t n_polys, const int32_t *ring_off, const int64_t *vert_off,
                           const int32_t *xy, int64_t eps, int mode)
{
    int64_t s = orc_cell_side(eps);
    polyset in = {n_polys, ring_off, vert_off, xy};
    if (s < 1 || n_polys < 0 || polys_ok(&in) || mode < 0 || mode > 2) return NULL;
    orc_approx *a = (orc_approx *)calloc(1, sizeof(orc_approx));
    if (!a) return NULL;
    a->eps = eps; a->s = s; a->n_polys = n_polys; a->mode = mode;
    int32_t nr = ring_off[n_polys];
    int64_t nv = vert_off[nr];
    a->ring_off = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n_polys + 1));
    a->vert_off = (int64_t *)malloc(sizeof(int64_t) * ((size_t)nr + 1));
    a->xy = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * nv + 1));
    a->rows = (prows *)calloc((size_t)(n_polys ? n_polys : 1), sizeof(prows));
    if (!a->ring_off || !a->vert_off || !a->xy || !a->rows) { orc_free(a); return NULL; }
    memcpy(a->ring_off, ring_off, sizeof(int32_t) * ((size_t)n_polys + 1));
    memcpy(a->vert_off, vert_off, sizeof(int64_t) * ((size_t)nr + 1));
    memcpy(a->xy, xy, sizeof(int32_t) * (size_t)(2 * nv));
    a->ps.n_polys = n_polys; a->ps.ring_off = a->ring_off;
    a->ps.vert_off = a->vert_off; a->ps.xy = a->xy;

    int fail = 0;
    #pragma omp parallel for schedule(dynamic, 1) reduction(|:fail)
    for (int32_t p = 0; p < n_polys; p++)
        if (build_rows(&a->ps, p, s, mode, &a->rows[p])) fail = 1;
    if (fail) { orc_free(a); return NULL; }

    /* bucket filter */
    if (n_polys == 0) {
        a->ui0 = a->uj0 = 0; a->uw = a->uh = 0; a->bsz = 1; a->bw = a->bh = 0;
        a->boff = (int64_t *)calloc(1, sizeof(int64_t));
        a->bids = (int32_t *)malloc(sizeof(int32_t));
        return a;
    }
    int64_t i0 = INT64_MAX, j0 = INT64_MAX, i1 = INT64_MIN, j1 = INT64_MIN;
    for (int32_t p = 0; p < n_polys; p++) {
        i0 = min64(i0, a->rows[p].ci0); j0 = min64(j0, a->rows[p].cj0);
        i1 = max64(i1, a->rows[p].ci1); j1 = max64(j1, a->rows[p].cj1);
    }
    a->ui0 = i0; a->uj0 = j0; a->uw = i1 - i0 + 1; a->uh = j1 - j0 + 1;
    int64_t side = max64(a->uw, a->uh);
    a->bsz = (side + 1023) / 1024;
    if (a->bsz < 1) a->bsz = 1;
    a->bw = (a->uw + a->bsz - 1) / a->bsz;
    a->bh = (a->uh + a->bsz - 1) / a->bsz;
    a->boff = (int64_t *)calloc((size_t)(a->bw * a->bh + 1), sizeof(int64_t));
    if (!a->boff) { orc_free(a); return NULL; }
    for (int pass = 0; pass < 2; pass++) {
        int64_t *fill = NULL;
        if (pass == 1) {
            for (int64_t b = 0; b < a->bw * a->bh; b++) a->boff[b + 1] += a->boff[b];
            a->bids = (int32_t *)malloc(sizeof(int32_t) * (size_t)(a->boff[a->bw * a->bh] + 1));
            fill = (int64_t *)calloc((size_t)(a->bw * a->bh), sizeof(int64_t));
            if (!a->bids || !fill) { free(fill); orc_free(a); return NULL; }
        }
        for (int32_t p = 0; p < n_polys; p++) {
            int64_t bx0 = (a->rows[p].ci0 - i0) / a->bsz, bx1 = (a->rows[p].ci1 - i0) / a->bsz;
            int64_t by0 = (a->rows[p].cj0 - j0) / a->bsz, by1 = (a->rows[p].cj1 - j0) / a->bsz;
            for (int64_t by = by0; by <= by1; by++)
                for (int64_t bx = bx0; bx <= bx1; bx++) {
                    int64_t b = by * a->bw + bx;
                    if (pass == 0) a->boff[b + 1]++;
                    else a->bids[a->boff[b] + fill[b]++] = p;
                }
        }
        free(fill);
    }
    return a;
}

orc_approx *orc_build(int32_t n_polys, const int32_t *ring_off, const int64_t *vert_off,
                      const int32_t *xy, int64_t eps)
{
    return orc_build_mode(n_polys, ring_off, vert_off, xy, eps, 0);
}

int64_t orc_cell_side_of(const orc_approx *a) { return a->s; }

/* candidate polygons of cell (i,j); returns count and sets *ids */
static int64_t candidates(const orc_approx *a, int64_t i, int64_t j, const int32_t **ids)
{
    if (i < a->ui0 || j < a->uj0 || i >= a->ui0 + a->uw || j >= a->uj0 + a->uh) return 0;
    int64_t b = ((j - a->uj0) / a->bsz) * a->bw + (i - a->ui0) / a->bsz;
    *ids = a->bids + a->boff[b];
    return a->boff[b + 1] - a->boff[b];
}

static int64_t fdiv64(int64_t a, int64_t b) { return (int64_t)fdiv(a, b); }

/* Number of intervals over all polygons, and their export (poly,row,x0,x1). */
int64_t orc_n_intervals(const orc_approx *a)
{
    int64_t n = 0;
    for (int32_t p = 0; p < a->n_polys; p++) n += a->rows[p].n_iv;
    return n;
}

void orc_export_intervals(const orc_approx *a, int32_t *poly, int64_t *row,
                          int64_t *x0, int64_t *x1)
{
    int64_t m = 0;
    for (int32_t p = 0; p < a->n_polys; p++) {
        const prows *pr = &a->rows[p];
        for (int64_t r = 0; r <= pr->cj1 - pr->cj0; r++)
            for (int64_t t = pr->row_off[r]; t < pr->row_off[r + 1]; t++) {
                poly[m] = p; row[m] = pr->cj0 + r; x0[m] = pr->x0[t]; x1[m] = pr->x1[t];
                m++;
            }
    }
}

/* S(c): ascending ids of the polygons whose approximation holds cell (i,j).
 * Writes at most cap ids; returns the full count. */
int orc_cell_set(const orc_approx *a, int64_t i, int64_t j, int32_t *ids, int cap)
{
    const int32_t *cand = NULL;
    int64_t nc = candidates(a, i, j, &cand);
    int n = 0;
    for (int64_t t = 0; t < nc; t++)          /* bucket lists are ascending */
        if (prows_contains(&a->rows[cand[t]], i, j)) {
            if (n < cap) ids[n] = cand[t];
            n++;
        }
    return n;
}

static int nthreads_of(int nthreads)
{
#ifdef _OPENMP
    return nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

/* Approximate aggregate (the quantity the GPU path must reproduce). */
int orc_aggregate(const orc_approx *a, const int32_t *xy, const int64_t *vals, int64_t n,
                  uint64_t *counts, int64_t *sums, int nthreads)
{
    int nt = nthreads_of(nthreads);
    int32_t np = a->n_polys;
    uint64_t *pc = (uint64_t *)calloc((size_t)nt * (np ? np : 1), sizeof(uint64_t));
    int64_t *psum = (int64_t *)calloc((size_t)nt * (np ? np : 1), sizeof(int64_t));
    if (!pc || !psum) { free(pc); free(psum); return -1; }
    #pragma omp parallel num_threads(nt)
    {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        uint64_t *c = pc + (size_t)t * np;
        int64_t *sm = psum + (size_t)t * np;
        #pragma omp for schedule(static)
        for (int64_t k = 0; k < n; k++) {
            int64_t i = fdiv64(xy[2 * k], a->s), j = fdiv64(xy[2 * k + 1], a->s);
            const int32_t *cand = NULL;
            int64_t nc = candidates(a, i, j, &cand);
            for (int64_t q = 0; q < nc; q++)
                if (prows_contains(&a->rows[cand[q]], i, j)) {
                    c[cand[q]] += 1;
                    if (vals) sm[cand[q]] += vals[k];
                }
        }
    }
    for (int32_t p = 0; p < np; p++) {
        uint64_t cc = 0; int64_t ss = 0;
        for (int t = 0; t < nt; t++) { cc += pc[(size_t)t * np + p]; ss += psum[(size_t)t * np + p]; }
        counts[p] = cc;
        if (sums) sums[p] = ss;
    }
    free(pc); free(psum);
    return nt;
}

/* Exact join by the crossing-number rule (Sec. 5: filter, then PIP). */
int orc_exact_join(const orc_approx *a, const int32_t *xy, const int64_t *vals, int64_t n,
                   uint64_t *counts, int64_t *sums, int nthreads)
{
    int nt = nthreads_of(nthreads);
    int32_t np = a->n_polys;
    uint64_t *pc = (uint64_t *)calloc((size_t)nt * (np ? np : 1), sizeof(uint64_t));
    int64_t *psum = (int64_t *)calloc((size_t)nt * (np ? np : 1), sizeof(int64_t));
    if (!pc || !psum) { free(pc); free(psum); return -1; }
    #pragma omp parallel num_threads(nt)
    {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        uint64_t *c = pc + (size_t)t * np;
        int64_t *sm = psum + (size_t)t * np;
        #pragma omp for schedule(dynamic, 4096)
        for (int64_t k = 0; k < n; k++) {
            int64_t px = xy[2 * k], py = xy[2 * k + 1];
            int64_t i = fdiv64(px, a->s), j = fdiv64(py, a->s);
            const int32_t *cand = NULL;
            int64_t nc = candidates(a, i, j, &cand);
            for (int64_t q = 0; q < nc; q++) {
                int32_t p = cand[q];
                const prows *pr = &a->rows[p];
                if (i < pr->ci0 || i > pr->ci1 || j < pr->cj0 || j > pr->cj1) continue;
                if (point_in_poly(&a->ps, p, px, py)) {
                    c[p] += 1;
                    if (vals) sm[p] += vals[k];
                }
            }
        }
    }
    for (int32_t p = 0; p < np; p++) {
        uint64_t cc = 0; int64_t ss = 0;
        for (int t = 0; t < nt; t++) { cc += pc[(size_t)t * np + p]; ss += psum[(size_t)t * np + p]; }
        counts[p] = cc;
        if (sums) sums[p] = ss;
    }
    free(pc); free(psum);
    return nt;
}

/* Invariant check over the given points (Sec. 2.2, Hausdorff
 * eps-approximation), with the distance bound given apart from the build:
 * out[0] = (point, polygon) pairs where approximate and exact membership
 * differ; out[1] = such pairs farther than check_eps (half = 1: farther than
 * check_eps / 2) from the boundary of P; out[2] = false negatives, i.e. p
 * inside P with cell(p) not in the approximation; out[3] = pairs inside P
 * (exact).  Candidate polygons come from the bucket filter, which holds every
 * polygon whose cell box contains cell(p); a point outside a polygon's cell
 * box is outside both the polygon and its approximation. */
int orc_invariant_at(const orc_approx *a, const int32_t *xy, int64_t n, int64_t check_eps,
                     int half, int64_t *out, int nthreads)
{
    int nt = nthreads_of(nthreads);
    int64_t diff = 0, far = 0, fneg = 0, ins = 0;
    #pragma omp parallel for num_threads(nt) schedule(dynamic, 4096) reduction(+:diff,far,fneg,ins)
    for (int64_t k = 0; k < n; k++) {
        int64_t px = xy[2 * k], py = xy[2 * k + 1];
        int64_t i = fdiv64(px, a->s), j = fdiv64(py, a->s);
        const int32_t *cand = NULL;
        int64_t nc = candidates(a, i, j, &cand);
        for (int64_t q = 0; q < nc; q++) {
            int32_t p = cand[q];
            int ap = prows_contains(&a->rows[p], i, j);
            int ex = point_in_poly(&a->ps, p, px, py);
            ins += ex;
            if (ap != ex) {
                diff++;
                if (!near_boundary(&a->ps, p, px, py, check_eps, half)) far++;
                if (ex && !ap) fneg++;
            }
        }
    }
    out[0] = diff; out[1] = far; out[2] = fneg; out[3] = ins;
    return 0;
}

/* The invariant the approximation must satisfy: misclassified points within
 * eps of the boundary (centre-sampled: within eps/2), no false negatives
 * (centre-sampled: allowed).  out[1] must be 0; see orc_invariant_at. */
int orc_invariant(const orc_approx *a, const int32_t *xy, int64_t n, int64_t *out, int nthreads)
{
    return orc_invariant_at(a, xy, n, a->eps, a->mode == ORC_CENTRE, out, nthreads);
}

/* Exhaustive version for tiny inputs: every polygon, no candidate filter. */
int orc_invariant_all_at(const orc_approx *a, const int32_t *xy, int64_t n, int64_t check_eps,
                         int half, int64_t *out)
{
    int64_t diff = 0, far = 0, fneg = 0, ins = 0;
    for (int64_t k = 0; k < n; k++) {
        int64_t px = xy[2 * k], py = xy[2 * k + 1];
        int64_t i = fdiv64(px, a->s), j = fdiv64(py, a->s);
        for (int32_t p = 0; p < a->n_polys; p++) {
            int ap = prows_contains(&a->rows[p], i, j);
            int ex = point_in_poly(&a->ps, p, px, py);
            ins += ex;
            if (ap != ex) {
                diff++;
                if (!near_boundary(&a->ps, p, px, py, check_eps, half)) far++;
                if (ex && !ap) fneg++;
            }
        }
    }
    out[0] = diff; out[1] = far; out[2] = fneg; out[3] = ins;
    return 0;
}

int orc_invariant_all(const orc_approx *a, const int32_t *xy, int64_t n, int64_t *out)
{
    return orc_invariant_all_at(a, xy, n, a->eps, a->mode == ORC_CENTRE, out);
}

/* The distance predicate itself, for its pins: 1 if (px,py) lies within eps
 * (half = 1: eps/2) of the closed segment (ax,ay)-(bx,by), by the exact test
 * above.  Coordinates must satisfy |c| < 2^30 and 0 <= eps <= 2^28, else -1. */
int orc_seg_within(int64_t px, int64_t py, int64_t ax, int64_t ay, int64_t bx, int64_t by,
                   int64_t eps, int half)
{
    const int64_t lim = (int64_t)1 << 30;
    int64_t c[6] = {px, py, ax, ay, bx, by};
    for (int t = 0; t < 6; t++)
        if (c[t] <= -lim || c[t] >= lim) return -1;
    if (eps < 0 || eps > ((int64_t)1 << 28)) return -1;
    return seg_within_k(px, py, ax, ay, bx, by, eps, half ? 4 : 1);
}

/* 1 if (px,py) lies within eps (half: eps/2) of the boundary of polygon p of
 * the approximation's polygon set (any edge of any ring), else 0. */
int orc_near_boundary(const orc_approx *a, int32_t p, int64_t px, int64_t py, int64_t eps,
                      int half)
{
    if (p < 0 || p >= a->n_polys) return -1;
    return near_boundary(&a->ps, p, px, py, eps, half);
}

/* ------------------------------------------------------------------ */
/* polygon-polygon join over cells (Sec. 4: blend two rasterized       */
/* canvases, mask the cells that hold both, aggregate per pair)        */
/* ------------------------------------------------------------------ */

/* cells shared by polygon p of a and polygon q of b: per common row, the
 * overlap of the two sorted disjoint interval lists */
static int64_t shared_cells(const prows *x, const prows *y)
{
    int64_t r0 = max64(x->cj0, y->cj0), r1 = min64(x->cj1, y->cj1), n = 0;
    if (max64(x->ci0, y->ci0) > min64(x->ci1, y->ci1)) return 0;
    for (int64_t r = r0; r <= r1; r++) {
        int64_t s = x->row_off[r - x->cj0], se = x->row_off[r - x->cj0 + 1];
        int64_t t = y->row_off[r - y->cj0], te = y->row_off[r - y->cj0 + 1];
        while (s < se && t < te) {
            int64_t lo = max64(x->x0[s], y->x0[t]), hi = min64(x->x1[s], y->x1[t]);
            if (hi > lo) n += hi - lo;
            if (x->x1[s] < y->x1[t]) s++; else t++;
        }
    }
    return n;
}

/* Every pair (p, q), p a polygon of a and q one of b (same cell side), whose
 * approximations share at least one cell, with the number of shared cells,
 * in (p, q) order.  Writes at most cap pairs; returns the number of pairs,
 * or -1 if the cell sides differ. */
int64_t orc_join_pairs(const orc_approx *a, const orc_approx *b, int64_t cap, int32_t *pa,
                       int32_t *pb, int64_t *cells)
{
    if (a->s != b->s) return -1;
    int64_t m = 0;
    for (int32_t p = 0; p < a->n_polys; p++)
        for (int32_t q = 0; q < b->n_polys; q++) {
            int64_t n = shared_cells(&a->rows[p], &b->rows[q]);
            if (n == 0) continue;
            if (m < cap) { pa[m] = p; pb[m] = q; cells[m] = n; }
            m++;
        }
    return m;
}

/* ------------------------------------------------------------------ */
/* Hilbert curve (Sec. 3, dimensionality reduction)                    */
/* ------------------------------------------------------------------ */

/* Hilbert index of cell (x,y) on the 2^L x 2^L grid.  Walk the levels from
 * the top: the quadrant bits (rx, ry) pick the quarter of the curve
 * (0,0)->0, (0,1)->1, (1,1)->2, (1,0)->3, and the coordinates are then
 * mapped into that quarter's own frame (a transpose for the two lower
 * quarters, preceded by a reflection for the right one) before descending. */
uint64_t orc_hilbert_d(int L, int64_t x, int64_t y)
{
    uint64_t d = 0;
    int64_t full = ((int64_t)1 << L) - 1;
    for (int lev = L - 1; lev >= 0; lev--) {
        int64_t h = (int64_t)1 << lev;
        int rx = (x & h) ? 1 : 0;
        int ry = (y & h) ? 1 : 0;
        d += (uint64_t)h * (uint64_t)h * (uint64_t)((3 * rx) ^ ry);
        if (ry == 0) {
            if (rx == 1) { x = full - x; y = full - y; }
            int64_t t = x; x = y; y = t;
        }
    }
    return d;
}

/* Key grid of the Hilbert layout: the cell box of the union of the
 * approximations, anchored at its first cell (ui0, uj0) and padded to
 * 2^L x 2^L cells with L the smallest level >= 1 that covers it.  Every cell
 * of every approximation then has a key. */
int orc_hilbert_level(const orc_approx *a)
{
    int L = 1;
    while (((int64_t)1 << L) < max64(a->uw, a->uh)) L++;
    return L;
}

void orc_union_box(const orc_approx *a, int64_t *out)
{
    out[0] = a->ui0; out[1] = a->uj0; out[2] = a->uw; out[3] = a->uh;
}

/* Maximal runs of consecutive Hilbert indices in [0, 4^L) whose cells have
 * equal S(c) (the empty set included, so the runs partition the index
 * range); index d stands for cell (ui0 + x, uj0 + y) where (x, y) is the
 * cell of d on the 2^L grid.  By enumeration of every index: tiny L only.
 * Writes run starts, and per run the ascending polygon ids as CSR
 * (run_off[n_runs+1], run_ids).  Returns 0 if everything fit, -1 otherwise;
 * *n_runs / *n_ids get the sizes needed. */
static int cmp_ids(const int32_t *a, int na, const int32_t *b, int nb)
{
    if (na != nb) return 0;
    for (int t = 0; t < na; t++) if (a[t] != b[t]) return 0;
    return 1;
}

int orc_hilbert_runs(const orc_approx *a, int L, uint64_t *starts, int64_t *run_off,
                     int32_t *run_ids, int64_t cap_runs, int64_t cap_ids,
                     int64_t *n_runs, int64_t *n_ids)
{
    if (L < 0 || L > 15) return -2;
    uint64_t total = (uint64_t)1 << (2 * L);
    int64_t side = (int64_t)1 << L;
    /* inverse map by enumeration of the cells */
    uint32_t *cx = (uint32_t *)malloc(sizeof(uint32_t) * total);
    uint32_t *cy = (uint32_t *)malloc(sizeof(uint32_t) * total);
    if (!cx || !cy) { free(cx); free(cy); return -3; }
    for (int64_t j = 0; j < side; j++)
        for (int64_t i = 0; i < side; i++) {
            uint64_t d = orc_hilbert_d(L, i, j);
            cx[d] = (uint32_t)i; cy[d] = (uint32_t)j;
        }
    int cap = a->n_polys > 0 ? a->n_polys : 1;
    int32_t *cur = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
    int32_t *prev = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
    int np = -1;
    int64_t nr = 0, ni = 0;
    for (uint64_t d = 0; d < total; d++) {
        int n = orc_cell_set(a, a->ui0 + cx[d], a->uj0 + cy[d], cur, cap);
        if (np >= 0 && cmp_ids(cur, n, prev, np)) continue;
        if (nr < cap_runs) {
            starts[nr] = d;
            run_off[nr] = ni;
        }
        for (int t = 0; t < n; t++) {
            if (ni < cap_ids) run_ids[ni] = cur[t];
            ni++;
        }
        nr++;
        memcpy(prev, cur, sizeof(int32_t) * (size_t)n);
        np = n;
    }
    if (nr <= cap_runs) run_off[nr] = ni;
    free(cx); free(cy); free(cur); free(prev);
    *n_runs = nr; *n_ids = ni;
    return (nr <= cap_runs && ni <= cap_ids) ? 0 : -1;
}
