"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: hand-derived
rasterisations (tests/golden), closed forms for rectangles and right
triangles, the definition evaluated cell by cell (brute form), the
eps-invariant of Sec. 2.2 checked with exact distances, the partition
property, nested grids, and the Hilbert curve's defining properties.
"""
import itertools
import os

import numpy as np
import pytest
import yaml

from gen import polygons_from_rings, star_polygons, voronoi_partition, uniform_points

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_examples.yaml")


def lattice(lo, hi):
    xs, ys = np.meshgrid(np.arange(lo, hi), np.arange(lo, hi))
    return np.c_[xs.ravel(), ys.ravel()].astype(np.int32).ravel()


def member_from_intervals(A, p, i0, j0, nw, nh):
    m = np.zeros((nh, nw), bool)
    P, R, X0, X1 = A.intervals()
    sel = P == p
    for r, a, b in zip(R[sel], X0[sel], X1[sel]):
        if j0 <= r < j0 + nh:
            a2, b2 = max(a, i0), min(b, i0 + nw)
            if a2 < b2:
                m[r - j0, a2 - i0:b2 - i0] = True
    return m


def cell_window(polys, s, pad=2):
    xy = polys.xy.reshape(-1, 2).astype(np.int64)
    i0 = int(np.floor(xy[:, 0].min() / s)) - pad
    j0 = int(np.floor(xy[:, 1].min() / s)) - pad
    i1 = int(np.floor(xy[:, 0].max() / s)) + pad
    j1 = int(np.floor(xy[:, 1].max() / s)) + pad
    return i0, j0, i1 - i0 + 1, j1 - j0 + 1


# ---------------------------------------------------------------- cell side

@pytest.mark.parametrize("eps,s", [(2, 1), (3, 2), (5, 3), (64, 45), (100, 70), (1000, 707),
                                   (10000, 7071), (15000, 10606), (1 << 28, 189812531)])
def test_cell_side_values(orc, eps, s):
    assert orc.cell_side(eps) == s
    # defining inequality: 2 s^2 <= eps^2 < 2 (s+1)^2
    assert 2 * s * s <= eps * eps < 2 * (s + 1) * (s + 1)


def test_cell_side_tiny_grid_matches_workload_text(orc):
    # eps = 64 units over [0, 65536): a grid of about 1450^2 cells
    s = orc.cell_side(64)
    assert -(-65536 // s) == 1457


def test_cell_side_rejects(orc):
    assert orc.cell_side(1) == 0
    assert orc.cell_side(0) == 0
    assert orc.cell_side((1 << 28) + 1) == 0


# ---------------------------------------------------------------- golden

def _golden():
    with open(GOLDEN) as f:
        return yaml.safe_load(f)["examples"]


@pytest.mark.parametrize("ex", _golden(), ids=lambda e: e["name"])
def test_hand_examples(orc, ex):
    polys = polygons_from_rings([[np.array(r) for r in ex["rings"]]])
    s = orc.cell_side(ex["eps"])
    assert s == ex["s"]
    i0, j0, nw, nh = -3, -3, 12, 12
    br = orc.raster_brute(polys, s, i0, j0, nw, nh)[0]
    bset = {(i0 + i, j0 + j) for j, i in zip(*np.nonzero(br == 2))}
    iset = {(i0 + i, j0 + j) for j, i in zip(*np.nonzero(br == 1))}
    assert bset == {tuple(c) for c in ex["boundary"]}
    assert iset == {tuple(c) for c in ex["interior"]}
    A = orc.Approx(polys, ex["eps"])
    m = member_from_intervals(A, 0, i0, j0, nw, nh)
    assert {(i0 + i, j0 + j) for j, i in zip(*np.nonzero(m))} == bset | iset
    xy = lattice(*ex["window"])
    c, _ = A.aggregate(xy)
    e, _ = A.exact(xy)
    assert int(c[0]) == ex["approx_count"]
    assert int(e[0]) == ex["exact_count"]


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("s,a,b,c,d", [(5, 0, 35, 0, 40), (5, -15, 20, 10, 25), (3, 3, 6, -9, 30),
                                       (7, 14, 70, 7, 21)])
def test_rectangle_closed_form(orc, s, a, b, c, d):
    # cell-aligned rectangle [a,b]x[c,d]: exact lattice count (b-a)(d-c) (half-open
    # crossing rule keeps [a,b)x[c,d)); conservative raster adds one cell ring:
    # (b-a+2s)(d-c+2s)
    eps = {3: 5, 5: 8, 7: 10}[s]
    assert orc.cell_side(eps) == s
    polys = polygons_from_rings([[np.array([[a, c], [b, c], [b, d], [a, d]])]])
    xy = lattice(min(a, c) - 3 * s, max(b, d) + 3 * s)
    A = orc.Approx(polys, eps)
    cnt, _ = A.aggregate(xy)
    ex, _ = A.exact(xy)
    assert int(ex[0]) == (b - a) * (d - c)
    assert int(cnt[0]) == (b - a + 2 * s) * (d - c + 2 * s)


@pytest.mark.parametrize("s,m,rot", [(5, 10, 0), (3, 7, 1), (4, 5, 2), (2, 9, 3)])
def test_right_triangle_closed_form(orc, s, m, rot):
    # legs L = m s at a cell-aligned corner: exact L(L+1)/2 for the corner at the
    # origin with legs along +x,+y; approx s^2 [(m+1)(m+2)/2 + 2m + 3] (cells whose
    # closed square meets the triangle).  Other orientations: the approximate count
    # is invariant under the grid's symmetries that map cells to cells.
    eps = {2: 3, 3: 5, 4: 6, 5: 8}[s]
    assert orc.cell_side(eps) == s
    L = m * s
    tri = np.array([[0, 0], [L, 0], [0, L]])
    R = [np.array([[1, 0], [0, 1]]), np.array([[0, -1], [1, 0]]),
         np.array([[-1, 0], [0, -1]]), np.array([[0, 1], [-1, 0]])][rot]
    v = tri @ R.T
    polys = polygons_from_rings([[v]])
    xy = lattice(-L - 3 * s, L + 3 * s)
    A = orc.Approx(polys, eps)
    cnt, _ = A.aggregate(xy)
    assert int(cnt[0]) == s * s * ((m + 1) * (m + 2) // 2 + 2 * m + 3)
    if rot == 0:
        ex, _ = A.exact(xy)
        assert int(ex[0]) == L * (L + 1) // 2


# ---------------------------------------------------------------- brute vs scan

def _hand_shapes():
    S = []
    S.append([[[0, 0], [30, 0], [30, 10], [10, 10], [10, 20], [30, 20], [30, 30], [0, 30]]])  # C
    S.append([[[0, 0], [40, 0], [20, 1], [20, 30]]])                                      # spike
    S.append([[[0, 0], [10, 0], [20, 0], [20, 10], [20, 20], [0, 20]]])                   # collinear
    S.append([[[5, 5], [25, 5], [25, 5], [15, 25]]])                                      # repeated vertex
    S.append([[[-17, -9], [12, -9], [12, 6], [-17, 6]]])                                  # negative coords
    S.append([[[0, 0], [30, 0], [30, 30], [0, 30]], [[10, 10], [20, 10], [20, 20], [10, 20]]])  # hole
    S.append([[[0, 0], [10, 0], [10, 10], [0, 10]], [[20, 0], [30, 0], [30, 10], [20, 10]]])    # two parts
    S.append([[[3, 3], [3, 3], [9, 3]]])                                                  # degenerate (zero area)
    S.append([[[0, 0], [24, 12], [0, 24], [12, 12]]])                                     # arrow, concave
    S.append([[[1, 2], [2, 1], [3, 2], [2, 3]]])                                          # tiny diamond
    return [[np.array(r) for r in p] for p in S]


@pytest.mark.parametrize("eps", [2, 3, 5, 8, 9, 15])
def test_scan_form_equals_definition_hand(orc, eps):
    s = orc.cell_side(eps)
    polys = polygons_from_rings(_hand_shapes())
    i0, j0, nw, nh = cell_window(polys, s)
    br = orc.raster_brute(polys, s, i0, j0, nw, nh)
    A = orc.Approx(polys, eps)
    for p in range(polys.n_polys):
        np.testing.assert_array_equal(member_from_intervals(A, p, i0, j0, nw, nh), br[p] > 0,
                                      err_msg=f"polygon {p}")


@pytest.mark.parametrize("seed", range(6))
def test_scan_form_equals_definition_random_stars(orc, seed):
    rng = np.random.default_rng(seed)
    polys = star_polygons(4, int(rng.integers(3, 12)), 5.0, 60.0, 200, 1000 + seed)
    for eps in (2, 4, 7, 13):
        s = orc.cell_side(eps)
        i0, j0, nw, nh = cell_window(polys, s)
        br = orc.raster_brute(polys, s, i0, j0, nw, nh)
        A = orc.Approx(polys, eps)
        for p in range(polys.n_polys):
            np.testing.assert_array_equal(member_from_intervals(A, p, i0, j0, nw, nh), br[p] > 0)


def test_scan_form_grid_aligned_edges(orc):
    # vertices on cell corners and edges along grid lines, s = 4
    eps = 6
    s = orc.cell_side(eps)
    assert s == 4
    rings = [[np.array([[0, 0], [16, 0], [16, 8], [8, 8], [8, 16], [0, 16]])],
             [np.array([[4, 4], [12, 12], [4, 12]])],
             [np.array([[-8, 20], [8, 20], [0, 28]])]]
    polys = polygons_from_rings(rings)
    i0, j0, nw, nh = cell_window(polys, s)
    br = orc.raster_brute(polys, s, i0, j0, nw, nh)
    A = orc.Approx(polys, eps)
    for p in range(polys.n_polys):
        np.testing.assert_array_equal(member_from_intervals(A, p, i0, j0, nw, nh), br[p] > 0)


# ---------------------------------------------------------------- aggregate

def test_aggregate_equals_brute_membership(orc):
    rng = np.random.default_rng(5)
    polys = star_polygons(6, 9, 10.0, 70.0, 150, 77)
    eps = 9
    s = orc.cell_side(eps)
    i0, j0, nw, nh = cell_window(polys, s)
    br = orc.raster_brute(polys, s, i0, j0, nw, nh) > 0
    xy = rng.integers(-30, 200, size=2 * 20000).astype(np.int32)
    vals = rng.integers(-1000, 1000, size=20000).astype(np.int64)
    A = orc.Approx(polys, eps)
    cnt, sm = A.aggregate(xy, vals, nthreads=3)
    ci = np.floor_divide(xy[0::2].astype(np.int64), s) - i0
    cj = np.floor_divide(xy[1::2].astype(np.int64), s) - j0
    ok = (ci >= 0) & (ci < nw) & (cj >= 0) & (cj < nh)
    for p in range(polys.n_polys):
        m = np.zeros(ci.shape, bool)
        m[ok] = br[p][cj[ok], ci[ok]]
        assert int(cnt[p]) == int(m.sum())
        assert int(sm[p]) == int(vals[m].sum())


def test_aggregate_thread_count_independent(orc):
    rng = np.random.default_rng(1)
    polys = star_polygons(10, 20, 50.0, 400.0, 2000, 9)
    xy = rng.integers(0, 2000, size=2 * 100000).astype(np.int32)
    vals = rng.integers(1, 10000, size=100000).astype(np.int64)
    A = orc.Approx(polys, 20)
    c1, s1 = A.aggregate(xy, vals, nthreads=1)
    c4, s4 = A.aggregate(xy, vals, nthreads=4)
    np.testing.assert_array_equal(c1, c4)
    np.testing.assert_array_equal(s1, s4)


def test_empty_inputs(orc):
    polys = star_polygons(3, 8, 10.0, 50.0, 300, 2)
    A = orc.Approx(polys, 10)
    c, s = A.aggregate(np.zeros(0, np.int32), np.zeros(0, np.int64))
    assert c.sum() == 0 and s.sum() == 0
    empty = polygons_from_rings([])
    A0 = orc.Approx(empty, 10)
    c, _ = A0.aggregate(np.array([1, 2], np.int32))
    assert c.shape == (0,)


# ---------------------------------------------------------------- invariant

@pytest.mark.parametrize("eps", [2, 6, 23, 64])
def test_eps_invariant_stars(orc, eps):
    rng = np.random.default_rng(eps)
    polys = star_polygons(8, 16, 30.0, 300.0, 1000, 31 + eps)
    xy = rng.integers(-300, 1300, size=2 * 60000).astype(np.int32)
    A = orc.Approx(polys, eps)
    inv = A.invariant(xy, exhaustive=True)
    assert inv["far"] == 0
    assert inv["false_neg"] == 0
    assert inv["differ"] > 0
    inv2 = A.invariant(xy)
    assert inv2 == inv


def test_invariant_counts_near_mismatch_as_near(orc):
    # a point deep inside is not a mismatch; a point just outside the square,
    # in a boundary cell, is a mismatch within eps (distance 3 <= 10)
    big = polygons_from_rings([[np.array([[0, 0], [100, 0], [100, 100], [0, 100]])]])
    A = orc.Approx(big, 10)
    far_in = np.array([50, 50], np.int32)
    assert A.invariant(far_in, exhaustive=True) == {"differ": 0, "far": 0, "false_neg": 0, "inside": 1}
    near_out = np.array([103, 50], np.int32)
    inv = A.invariant(near_out, exhaustive=True)
    assert inv["differ"] == 1 and inv["far"] == 0
    # the same mismatch checked against a bound below its distance is far
    assert A.invariant(near_out, exhaustive=True, check_eps=2)["far"] == 1
    assert A.invariant(near_out, exhaustive=True, check_eps=3)["far"] == 0


# ---------------------------------------------------------------- distance predicate
#
# The invariant's distance test (Sec. 2.2) pinned on its own: hand-derived
# distances with ties at the bound (tests/golden/distances.yaml), and a
# brute force by the clamped projection onto the segment in exact rationals
# (a different formulation from the oracle's cross-product comparison).

DISTANCES = os.path.join(os.path.dirname(__file__), "golden", "distances.yaml")


def _distance_cases():
    with open(DISTANCES) as f:
        return yaml.safe_load(f)["cases"]


def _d2_projection(p, a, b):
    from fractions import Fraction
    vx, vy = b[0] - a[0], b[1] - a[1]
    wx, wy = p[0] - a[0], p[1] - a[1]
    l2 = vx * vx + vy * vy
    t = Fraction(0) if l2 == 0 else min(max(Fraction(wx * vx + wy * vy, l2), Fraction(0)), Fraction(1))
    cx, cy = a[0] + t * vx, a[1] + t * vy
    return (p[0] - cx) ** 2 + (p[1] - cy) ** 2


@pytest.mark.parametrize("case", _distance_cases(), ids=lambda c: c["name"])
def test_seg_within_hand_cases(orc, case):
    p, a, b = case["p"], case["a"], case["b"]
    assert _d2_projection(p, a, b) == case["d2"]          # the fixture's own derivation
    for eps, want in case["full"]:
        assert orc.seg_within(p, a, b, eps) is want, ("full", eps)
        assert orc.seg_within(p, b, a, eps) is want        # orientation-free
    for eps, want in case["half"]:
        assert orc.seg_within(p, a, b, eps, half=True) is want, ("half", eps)
        assert orc.seg_within(p, b, a, eps, half=True) is want


def test_seg_within_matches_projection_brute_force(orc):
    # random segments and points, including coordinates near +-2^30, each
    # bound placed at the exact distance (tie) and one unit below it
    import math
    rng = np.random.default_rng(77)
    lim = (1 << 30) - 1
    n_checked = 0
    for scale in (50, 5000, 1 << 20, lim):
        for _ in range(300):
            a = [int(v) for v in rng.integers(-scale, scale + 1, 2)]
            b = [int(v) for v in rng.integers(-scale, scale + 1, 2)]
            p = [int(v) for v in rng.integers(-scale, scale + 1, 2)]
            d2 = _d2_projection(p, a, b)
            for half in (False, True):
                k = 4 if half else 1
                # smallest integer eps with eps^2 >= k d2, and the one below
                e = math.isqrt(int(k * d2))
                while e * e < k * d2:
                    e += 1
                if e <= (1 << 28):
                    assert orc.seg_within(p, a, b, e, half) is True
                    n_checked += 1
                if 1 <= e - 1 <= (1 << 28):
                    assert orc.seg_within(p, a, b, e - 1, half) is False
    assert n_checked > 1000


def test_seg_within_rejects_out_of_range(orc):
    with pytest.raises(ValueError):
        orc.seg_within((1 << 30, 0), (0, 0), (1, 1), 5)
    with pytest.raises(ValueError):
        orc.seg_within((0, 0), (0, 0), (1, 1), (1 << 28) + 1)


def _rect_dist2(x, y, x0, y0, x1, y1):
    """Squared distance from lattice points to the boundary of the rectangle
    [x0,x1] x [y0,y1]: clamped distance outside, nearest side inside."""
    x = x.astype(np.int64)
    y = y.astype(np.int64)
    dx = np.maximum(np.maximum(x0 - x, x - x1), 0)
    dy = np.maximum(np.maximum(y0 - y, y - y1), 0)
    out = dx * dx + dy * dy
    inside = (x > x0) & (x < x1) & (y > y0) & (y < y1)
    m = np.minimum(np.minimum(x - x0, x1 - x), np.minimum(y - y0, y1 - y))
    return np.where(inside, m * m, out)


@pytest.mark.parametrize("check", [10, 9, 8, 7, 5, 3, 1])
def test_invariant_far_count_rectangle_closed_form(orc, check):
    # square [0,70]^2 at eps = 10 (s = 7): A(P) is the cells -1..10 in both
    # axes, i.e. the points of [-7,77)^2; the exact set is [0,70)^2 (half-open
    # crossing rule).  The mismatches are the points of the ring between, and
    # those farther than `check` from the square's boundary are counted by
    # the clamped distance -- none for check >= 10 (the largest is
    # sqrt(7^2+7^2) < 10), some below
    x0, y0, x1, y1 = 0, 0, 70, 70
    A = orc.Approx(polygons_from_rings([[np.array([[x0, y0], [x1, y0], [x1, y1], [x0, y1]])]]), 10)
    assert A.s == 7
    xy = lattice(-14, 84)
    px, py = xy[0::2], xy[1::2]
    approx = (px >= -7) & (px < 77) & (py >= -7) & (py < 77)
    exact = (px >= x0) & (px < x1) & (py >= y0) & (py < y1)
    mism = approx != exact
    d2 = _rect_dist2(px, py, x0, y0, x1, y1)
    want_far = int(np.count_nonzero(mism & (d2 > check * check)))
    inv = A.invariant(xy, exhaustive=True, check_eps=check)
    assert inv["differ"] == int(np.count_nonzero(mism))
    assert inv["far"] == want_far
    assert inv["false_neg"] == 0
    assert A.invariant(xy, check_eps=check) == inv           # candidate filter agrees
    if check >= 10:
        assert want_far == 0
    if check <= 9:
        assert want_far > 0                                   # the bound bites


@pytest.mark.parametrize("check", [10, 9, 8, 6, 4, 2])
def test_invariant_far_count_centre_rectangle_closed_form(orc, check):
    # square [3,66]^2 at eps = 10 (s = 7), centre-sampled: the cells whose
    # centre 7i + 3.5 lies in [3,66) are i = 0..8, i.e. the points of
    # [0,63)^2; exact [3,66)^2.  Mismatches lie within eps/2 = 5 (the corner
    # point (0,0) is sqrt(18) from the corner (3,3)); at bound check/2 they
    # are counted by the clamped distance
    x0, y0, x1, y1 = 3, 3, 66, 66
    polys = polygons_from_rings([[np.array([[x0, y0], [x1, y0], [x1, y1], [x0, y1]])]])
    C = orc.Approx(polys, 10, centre=True)
    xy = lattice(-14, 84)
    px, py = xy[0::2], xy[1::2]
    approx = (px >= 0) & (px < 63) & (py >= 0) & (py < 63)
    exact = (px >= x0) & (px < x1) & (py >= y0) & (py < y1)
    mism = approx != exact
    d2 = _rect_dist2(px, py, x0, y0, x1, y1)
    want_far = int(np.count_nonzero(mism & (4 * d2 > check * check)))
    inv = C.invariant(xy, exhaustive=True, check_eps=check)   # half by default here
    assert inv["differ"] == int(np.count_nonzero(mism))
    assert inv["far"] == want_far
    assert inv["false_neg"] == int(np.count_nonzero(exact & ~approx))
    if check == 10:
        assert want_far == 0
    if check == 8:
        assert want_far == 1                                  # only the point (0,0)


@pytest.mark.parametrize("eps,check", [(64, 32), (64, 16), (23, 8)])
def test_invariant_far_count_stars_brute_force(orc, eps, check):
    # random stars: the far mismatches at a bound below eps, counted by a
    # floating-point distance to every edge (cases within 1e-6 of the bound
    # are left out of the comparison and must be rare)
    rng = np.random.default_rng(eps * 10 + check)
    polys = star_polygons(4, 12, 30.0, 300.0, 700, 500 + eps)
    xy = rng.integers(-300, 1000, size=2 * 8000).astype(np.int32)
    A = orc.Approx(polys, eps)
    inv = A.invariant(xy, exhaustive=True, check_eps=check)
    assert A.invariant(xy, exhaustive=True)["far"] == 0
    P, R, X0, X1 = A.intervals()
    pts = xy.reshape(-1, 2).astype(np.float64)
    i = np.floor_divide(xy[0::2].astype(np.int64), A.s)
    j = np.floor_divide(xy[1::2].astype(np.int64), A.s)
    far = amb = diff = 0
    for p in range(polys.n_polys):
        ring = polys.rings_of(p)[0].astype(np.float64)
        sel = P == p
        ap = np.zeros(len(pts), bool)
        for r, a0, a1 in zip(R[sel], X0[sel], X1[sel]):
            ap |= (j == r) & (i >= a0) & (i < a1)
        # exact membership of a mismatch candidate: the oracle's exact join
        # of that one point (the crossing rule is pinned by the closed forms
        # above; the distance is what this test checks)
        a_ = ring
        b_ = np.roll(ring, -1, axis=0)
        v = b_ - a_
        l2 = (v * v).sum(1)
        for k in range(len(pts)):
            ex = A.exact(xy[2 * k:2 * k + 2])[0][p] == 1
            if ex == ap[k]:
                continue
            diff += 1
            w = pts[k] - a_
            t = np.clip((w * v).sum(1) / np.where(l2 > 0, l2, 1), 0.0, 1.0)
            d = np.sqrt((((a_ + t[:, None] * v) - pts[k]) ** 2).sum(1)).min()
            if abs(d - check) < 1e-6:
                amb += 1
            elif d > check:
                far += 1
    assert amb <= 2
    assert diff == inv["differ"]
    assert abs(inv["far"] - far) <= amb
    assert far > 0


def test_centre_large_extent_within_half_eps(orc):
    # a triangle spanning the whole accepted coordinate range, centre-sampled
    # at a large eps: every mismatch within eps/2 (coordinates near 2^30
    # make the squared cross products exceed 2^120)
    lim = (1 << 30) - 1
    tri = polygons_from_rings([[np.array([[-lim, -lim], [lim, -lim], [0, lim]])]])
    eps = 1 << 26
    C = orc.Approx(tri, eps, centre=True)
    rng = np.random.default_rng(5)
    xy = rng.integers(-lim, lim + 1, size=2 * 40000).astype(np.int32)
    inv = C.invariant(xy, exhaustive=True)
    assert inv["far"] == 0 and inv["differ"] > 0
    A = orc.Approx(tri, eps)
    inv = A.invariant(xy, exhaustive=True)
    assert inv["far"] == 0 and inv["false_neg"] == 0 and inv["differ"] > 0
    # at a bound of eps/8 some mismatches of the centre cells are far
    assert C.invariant(xy, exhaustive=True, check_eps=eps // 8)["far"] > 0


# ---------------------------------------------------------------- nested grids

def test_nested_grids_monotone(orc):
    rng = np.random.default_rng(3)
    polys = star_polygons(6, 24, 200.0, 2000.0, 8000, 13)
    xy = rng.integers(-2000, 10000, size=2 * 200000).astype(np.int32)
    sides = [(8, 5), (15, 10), (29, 20), (57, 40)]   # eps -> s, each s twice the previous
    prev = None
    ex = None
    for eps, s in sides:
        assert orc.cell_side(eps) == s
        A = orc.Approx(polys, eps)
        c, _ = A.aggregate(xy)
        if ex is None:
            ex, _ = A.exact(xy)
            assert np.all(ex <= c)
        if prev is not None:
            assert np.all(prev <= c)
        prev = c


# ---------------------------------------------------------------- partition

def test_partition_property(orc):
    polys = voronoi_partition(30, 200000, (3, 20), seed=3, jitter_seed=4)
    pts = uniform_points(300000, 0, 200000, 11)
    for eps in (100, 1500):
        A = orc.Approx(polys, eps)
        ex, _ = A.exact(pts)
        ap, _ = A.aggregate(pts)
        assert int(ex.sum()) == 300000          # each point in exactly one cell
        assert int(ap.sum()) >= 300000
        inv = A.invariant(pts)
        assert inv["far"] == 0 and inv["false_neg"] == 0


# ---------------------------------------------------------------- hilbert

def test_hilbert_level1(orc):
    assert [orc.hilbert_d(1, *c) for c in [(0, 0), (0, 1), (1, 1), (1, 0)]] == [0, 1, 2, 3]


@pytest.mark.parametrize("L", [1, 2, 3, 4, 5, 6])
def test_hilbert_bijection_and_adjacency(orc, L):
    n = 1 << L
    inv = {}
    for i in range(n):
        for j in range(n):
            inv[orc.hilbert_d(L, i, j)] = (i, j)
    assert sorted(inv) == list(range(n * n))
    for d in range(n * n - 1):
        (a, b), (c, e) = inv[d], inv[d + 1]
        assert abs(a - c) + abs(b - e) == 1
    assert inv[0] == (0, 0)
    assert inv[n * n - 1] == (n - 1, 0)


@pytest.mark.parametrize("L", [2, 3, 4, 5])
def test_hilbert_quadrant_blocks(orc, L):
    # every aligned block of 4^k consecutive indices is an aligned 2^k square
    n = 1 << L
    inv = {orc.hilbert_d(L, i, j): (i, j) for i in range(n) for j in range(n)}
    for k in range(1, L):
        bs = 4 ** k
        for start in range(0, n * n, bs):
            cells = [inv[d] for d in range(start, start + bs)]
            xs = {c[0] // (1 << k) for c in cells}
            ys = {c[1] // (1 << k) for c in cells}
            assert len(xs) == 1 and len(ys) == 1


def test_hilbert_runs_against_brute(orc):
    polys = star_polygons(5, 10, 10.0, 60.0, 120, 21)
    eps = 5
    s = orc.cell_side(eps)
    A = orc.Approx(polys, eps)
    i0, j0, w, h = A.union_box()
    L = A.hilbert_level()
    assert (1 << L) >= max(w, h) and (L == 1 or (1 << (L - 1)) < max(w, h))
    starts, off, ids = A.hilbert_runs(L)
    assert starts[0] == 0 and np.all(np.diff(starts.astype(np.int64)) > 0)
    sets = [tuple(ids[off[r]:off[r + 1]]) for r in range(len(starts))]
    assert all(sets[r] != sets[r + 1] for r in range(len(sets) - 1))    # maximal
    n = 1 << L
    br = orc.raster_brute(polys, s, i0, j0, n, n) > 0
    for x in range(n):
        for y in range(n):
            d = orc.hilbert_d(L, x, y)
            r = int(np.searchsorted(starts, d, side="right")) - 1
            want = tuple(int(p) for p in np.nonzero(br[:, y, x])[0])
            assert sets[r] == want
    # every cell of every approximation lies inside the key grid
    P, R, X0, X1 = A.intervals()
    assert X0.min() >= i0 and X1.max() <= i0 + n and R.min() >= j0 and R.max() < j0 + n


# ---------------------------------------------------------------- workloads

def test_invariant_every_point_tiny_workload(orc):
    """Tiny workload (1M points, 16 overlapping stars, eps = 64): every point
    on which the approximation and the exact join differ lies within eps of
    the polygon's boundary, and no point inside a polygon is missed."""
    from gen import tiny_workload
    xy, vals, polys = tiny_workload()
    A = orc.Approx(polys, 64)
    inv = A.invariant(xy)
    assert inv["far"] == 0 and inv["false_neg"] == 0 and inv["differ"] > 0
    ap, _ = A.aggregate(xy)
    ex, _ = A.exact(xy)
    assert np.all(ex <= ap)


@pytest.mark.parametrize("eps", [100, 1000, 10000])
def test_invariant_city_sample(orc, eps):
    """City partition (260 jittered Voronoi cells), 2M mixture points."""
    from gen import city_points, city_polygons
    polys = city_polygons()
    xy, _ = city_points(2_000_000)
    A = orc.Approx(polys, eps)
    inv = A.invariant(xy)
    assert inv["far"] == 0 and inv["false_neg"] == 0
    ex, _ = A.exact(xy)
    assert int(ex.sum()) == 2_000_000           # a partition of the box


def test_invariant_quadtree_polygons(orc):
    """The quadtree workload's polygon set (40,000 jittered Voronoi cells, 32
    to 675 vertices each; the analogue of Sec. 5.1's census blocks) at
    eps = 1 m, 2M mixture points: no point farther than eps from the boundary
    of a polygon it is wrongly counted in, no point missed, the cells a
    partition of the box, and the check reports far points once the distance
    bound is cut below the cell diagonal."""
    from gen import city_points, quadtree_polygons
    polys = quadtree_polygons()
    xy, vals = city_points(2_000_000, config=3)
    A = orc.Approx(polys, 100)
    inv = A.invariant(xy)
    assert inv["far"] == 0 and inv["false_neg"] == 0 and inv["differ"] > 0
    ex, exs = A.exact(xy, vals)
    ap, aps = A.aggregate(xy, vals)
    assert int(ex.sum()) == 2_000_000           # a partition of the box
    assert np.all(ex <= ap) and np.all(exs <= aps)
    # the boundary cells' points lie up to a diagonal (70 sqrt 2 ~ 99 units)
    # from the boundary; with a bound of 40 units some must be reported
    assert A.invariant(xy, check_eps=40)["far"] > 0


# ---------------------------------------------------------------- result range (Sec. 6)
#
# beta = the partial count over the boundary cells B(P); with the conservative
# approximation every wrong point lies in a boundary cell, so the exact count
# lies in [alpha - beta, alpha].

@pytest.mark.parametrize("eps", [2, 3, 5, 8, 9, 15])
def test_boundary_only_equals_definition_hand(orc, eps):
    s = orc.cell_side(eps)
    polys = polygons_from_rings(_hand_shapes())
    i0, j0, nw, nh = cell_window(polys, s)
    br = orc.raster_brute(polys, s, i0, j0, nw, nh)
    B = orc.Approx(polys, eps, boundary_only=True)
    for p in range(polys.n_polys):
        np.testing.assert_array_equal(member_from_intervals(B, p, i0, j0, nw, nh), br[p] == 2,
                                      err_msg=f"polygon {p}")


@pytest.mark.parametrize("seed", range(4))
def test_boundary_only_equals_definition_random_stars(orc, seed):
    rng = np.random.default_rng(seed)
    polys = star_polygons(4, int(rng.integers(3, 12)), 5.0, 60.0, 200, 2000 + seed)
    for eps in (2, 4, 7, 13):
        s = orc.cell_side(eps)
        i0, j0, nw, nh = cell_window(polys, s)
        br = orc.raster_brute(polys, s, i0, j0, nw, nh)
        B = orc.Approx(polys, eps, boundary_only=True)
        for p in range(polys.n_polys):
            np.testing.assert_array_equal(member_from_intervals(B, p, i0, j0, nw, nh), br[p] == 2)


@pytest.mark.parametrize("s,a,b,c,d", [(5, 0, 35, 0, 40), (5, -15, 20, 10, 25), (3, 3, 12, -9, 30),
                                       (7, 14, 70, 7, 35)])
def test_rectangle_result_range_closed_form(orc, s, a, b, c, d):
    # cell-aligned rectangle: the boundary cells are two cells thick along every
    # side (cells i with is <= a <= (i+1)s touch x = a), the interior cells
    # cover (b-a-2s)(d-c-2s) lattice points, so beta = (b-a+2s)(d-c+2s) -
    # (b-a-2s)(d-c-2s); the exact (b-a)(d-c) lies in [alpha - beta, alpha]
    eps = {3: 5, 5: 8, 7: 10}[s]
    polys = polygons_from_rings([[np.array([[a, c], [b, c], [b, d], [a, d]])]])
    xy = lattice(min(a, c) - 3 * s, max(b, d) + 3 * s)
    alpha, _ = orc.Approx(polys, eps).aggregate(xy)
    beta, _ = orc.Approx(polys, eps, boundary_only=True).aggregate(xy)
    inner = max(b - a - 2 * s, 0) * max(d - c - 2 * s, 0)
    assert int(alpha[0]) == (b - a + 2 * s) * (d - c + 2 * s)
    assert int(beta[0]) == int(alpha[0]) - inner
    assert int(alpha[0]) - int(beta[0]) <= (b - a) * (d - c) <= int(alpha[0])


@pytest.mark.parametrize("eps", [2, 6, 23, 64])
def test_result_range_contains_exact(orc, eps):
    # counts and (non-negative) sums: alpha - beta <= exact <= alpha, for every
    # polygon; overlapping stars, points on and off the polygons
    rng = np.random.default_rng(100 + eps)
    polys = star_polygons(8, 16, 30.0, 300.0, 1000, 131 + eps)
    xy = rng.integers(-300, 1300, size=2 * 60000).astype(np.int32)
    vals = rng.integers(0, 10000, size=60000).astype(np.int64)
    A = orc.Approx(polys, eps)
    ac, asum = A.aggregate(xy, vals)
    bc, bsum = orc.Approx(polys, eps, boundary_only=True).aggregate(xy, vals)
    ec, esum = A.exact(xy, vals)
    ac, bc, ec = ac.astype(np.int64), bc.astype(np.int64), ec.astype(np.int64)
    assert np.all(bc <= ac)
    assert np.all(ac - bc <= ec) and np.all(ec <= ac)
    assert np.all(asum - bsum <= esum) and np.all(esum <= asum)
    assert np.any(ac - bc < ec) and np.any(ec < ac)   # the bounds are not trivially tight


# ---------------------------------------------------------------- centre-sampled cells
#
# The non-conservative raster (Sec. 2.2): a cell belongs to P when its centre
# is inside P.  Pinned by the per-cell definition, closed forms on rectangles
# and right triangles (ties on edges decided by the half-open crossing rule),
# the eps/2 bound on every misclassified point, and the partition property.

def _centre_cells_1d(a, b, s):
    # number of integers i with a <= (i + 1/2) s < b
    return max(0, -(-(2 * b - s) // (2 * s)) - (-(-(2 * a - s) // (2 * s))))


@pytest.mark.parametrize("eps", [2, 3, 5, 8, 9, 15])
def test_centre_equals_definition_hand(orc, eps):
    s = orc.cell_side(eps)
    polys = polygons_from_rings(_hand_shapes())
    i0, j0, nw, nh = cell_window(polys, s)
    br = orc.centre_brute(polys, s, i0, j0, nw, nh)
    C = orc.Approx(polys, eps, centre=True)
    for p in range(polys.n_polys):
        np.testing.assert_array_equal(member_from_intervals(C, p, i0, j0, nw, nh), br[p] == 1,
                                      err_msg=f"polygon {p}")


@pytest.mark.parametrize("seed", range(4))
def test_centre_equals_definition_random_stars(orc, seed):
    rng = np.random.default_rng(seed)
    polys = star_polygons(4, int(rng.integers(3, 12)), 5.0, 60.0, 200, 3000 + seed)
    for eps in (2, 3, 4, 7, 13):
        s = orc.cell_side(eps)
        i0, j0, nw, nh = cell_window(polys, s)
        br = orc.centre_brute(polys, s, i0, j0, nw, nh)
        C = orc.Approx(polys, eps, centre=True)
        for p in range(polys.n_polys):
            np.testing.assert_array_equal(member_from_intervals(C, p, i0, j0, nw, nh), br[p] == 1)


@pytest.mark.parametrize("s,a,b,c,d", [(5, 0, 35, 0, 40), (5, -15, 20, 10, 25), (4, 2, 18, 6, 22),
                                       (4, -3, 13, 1, 30), (7, 3, 40, -11, 17), (1, -4, 9, 2, 5)])
def test_centre_rectangle_closed_form(orc, s, a, b, c, d):
    # the cells whose centre lies in [a,b) x [c,d) (left and bottom edges
    # inclusive by the half-open crossing rule); on the full lattice each cell
    # holds s^2 points.  Cell-aligned rectangles give exactly the exact count.
    eps = {1: 2, 4: 6, 5: 8, 7: 10}[s]
    assert orc.cell_side(eps) == s
    polys = polygons_from_rings([[np.array([[a, c], [b, c], [b, d], [a, d]])]])
    lo = (min(a, c) // s - 3) * s
    hi = (max(b, d) // s + 4) * s
    xy = lattice(lo, hi)
    C = orc.Approx(polys, eps, centre=True)
    cnt, _ = C.aggregate(xy)
    assert int(cnt[0]) == s * s * _centre_cells_1d(a, b, s) * _centre_cells_1d(c, d, s)
    if a % s == 0 and b % s == 0 and c % s == 0 and d % s == 0:
        ex, _ = C.exact(xy)
        assert int(cnt[0]) == int(ex[0]) == (b - a) * (d - c)


@pytest.mark.parametrize("s,m", [(5, 10), (3, 7), (4, 5), (1, 9)])
def test_centre_right_triangle_closed_form(orc, s, m):
    # legs L = m s.  Triangle (0,0),(L,0),(0,L): centres with i + j = m - 1 lie
    # on the hypotenuse, where the crossing rule puts them outside: m(m-1)/2
    # cells, fewer lattice points than the exact L(L+1)/2 (false negatives).
    # Triangle (0,0),(L,0),(L,L): the diagonal centres (i = j) lie on the
    # hypotenuse with the right edge to their right, inside: m(m+1)/2 cells.
    eps = {1: 2, 3: 5, 4: 6, 5: 8}[s]
    assert orc.cell_side(eps) == s
    L = m * s
    xy = lattice(-2 * s, L + 2 * s)
    lo = orc.Approx(polygons_from_rings([[np.array([[0, 0], [L, 0], [0, L]])]]), eps, centre=True)
    cnt, _ = lo.aggregate(xy)
    ex, _ = lo.exact(xy)
    assert int(cnt[0]) == s * s * m * (m - 1) // 2
    assert int(ex[0]) == L * (L + 1) // 2
    up = orc.Approx(polygons_from_rings([[np.array([[0, 0], [L, 0], [L, L]])]]), eps, centre=True)
    cnt, _ = up.aggregate(xy)
    assert int(cnt[0]) == s * s * m * (m + 1) // 2


@pytest.mark.parametrize("eps", [2, 6, 23, 64])
def test_centre_within_half_eps(orc, eps):
    # every point whose membership differs from its cell centre's lies within
    # eps/2 of the boundary (checked exactly); false negatives do occur
    rng = np.random.default_rng(200 + eps)
    polys = star_polygons(8, 16, 30.0, 300.0, 1000, 231 + eps)
    xy = rng.integers(-300, 1300, size=2 * 60000).astype(np.int32)
    C = orc.Approx(polys, eps, centre=True)
    inv = C.invariant(xy, exhaustive=True)
    assert inv["far"] == 0
    assert inv["differ"] > 0 and inv["false_neg"] > 0
    assert C.invariant(xy) == inv
    # the conservative approximation of the same polygons is further off: its
    # misclassified points are not all within eps/2, so the check at eps/2
    # does report far points when they exist
    A = orc.Approx(polys, eps)
    assert A.invariant(xy, exhaustive=True)["differ"] > inv["differ"]
    assert A.invariant(xy, exhaustive=True, half=True)["far"] > 0


def test_centre_partition_counts_each_point_once(orc):
    # on a partition of the box every cell centre inside the box lies in
    # exactly one polygon, so the counts add up to the number of points whose
    # cell centre is inside the box (no double counting on shared boundaries)
    B = 200000
    polys = voronoi_partition(30, B, (3, 20), seed=3, jitter_seed=4)
    pts = uniform_points(300000, 0, B, 11)
    for eps in (100, 1500, 7777):
        s = orc.cell_side(eps)
        C = orc.Approx(polys, eps, centre=True)
        cnt, _ = C.aggregate(pts)
        p = pts.reshape(-1, 2).astype(np.int64)
        cx, cy = (2 * (p[:, 0] // s) + 1) * s, (2 * (p[:, 1] // s) + 1) * s
        inside = int(np.count_nonzero((cx < 2 * B) & (cy < 2 * B)))
        assert int(cnt.sum()) == inside
        inv = C.invariant(pts)
        assert inv["far"] == 0


# ---------------------------------------------------------------- polygon-polygon join
#
# Sec. 4: blending two rasterized canvases and masking the cells that hold
# both gives the pairs of polygons whose approximations intersect, with the
# shared cell count.  Pinned by the per-cell definition (brute membership),
# the rectangle closed form, symmetry, the diagonal of a self-join and the
# conservative guarantee (polygons sharing a point are always paired).

def _pairs_dict(pa, pb, cells):
    return {(int(p), int(q)): int(c) for p, q, c in zip(pa, pb, cells)}


@pytest.mark.parametrize("s,r1,r2", [
    (5, (0, 35, 0, 40), (20, 60, 10, 25)),      # overlapping
    (5, (0, 35, 0, 40), (40, 60, 0, 40)),       # 5 apart: the cell rings still meet
    (5, (0, 35, 0, 40), (45, 60, 0, 40)),       # 10 apart: one cell ring each, adjacent
    (3, (3, 12, -9, 30), (-30, 0, 0, 3)),
    (7, (14, 70, 7, 35), (84, 98, 35, 49))])    # corner to corner at distance 14
def test_join_rectangles_closed_form(orc, s, r1, r2):
    # a cell-aligned rectangle [a,b] x [c,d] covers the cells a/s-1 .. b/s and
    # c/s-1 .. d/s; two such ranges share the product of their 1-D overlaps
    eps = {3: 5, 5: 8, 7: 10}[s]
    A = orc.Approx(polygons_from_rings([[np.array([[r1[0], r1[2]], [r1[1], r1[2]],
                                                   [r1[1], r1[3]], [r1[0], r1[3]]])]]), eps)
    B = orc.Approx(polygons_from_rings([[np.array([[r2[0], r2[2]], [r2[1], r2[2]],
                                                   [r2[1], r2[3]], [r2[0], r2[3]]])]]), eps)

    def ov(a0, a1, b0, b1):
        return max(0, min(a1 // s, b1 // s) - max(a0 // s - 1, b0 // s - 1) + 1)

    want = ov(r1[0], r1[1], r2[0], r2[1]) * ov(r1[2], r1[3], r2[2], r2[3])
    got = _pairs_dict(*orc.join_pairs(A, B))
    assert got == ({(0, 0): want} if want else {})


@pytest.mark.parametrize("eps", [2, 4, 7, 13])
def test_join_equals_definition_random_stars(orc, eps):
    a = star_polygons(4, 9, 5.0, 60.0, 200, 4000 + eps)
    b = star_polygons(5, 7, 5.0, 50.0, 200, 5000 + eps)
    s = orc.cell_side(eps)
    ia, ja, wa, ha = cell_window(a, s)
    ib, jb, wb, hb = cell_window(b, s)
    i0, j0 = min(ia, ib), min(ja, jb)
    nw, nh = max(ia + wa, ib + wb) - i0, max(ja + ha, jb + hb) - j0
    ma = orc.raster_brute(a, s, i0, j0, nw, nh) > 0
    mb = orc.raster_brute(b, s, i0, j0, nw, nh) > 0
    want = {}
    for p in range(a.n_polys):
        for q in range(b.n_polys):
            n = int(np.count_nonzero(ma[p] & mb[q]))
            if n:
                want[(p, q)] = n
    A, B = orc.Approx(a, eps), orc.Approx(b, eps)
    assert _pairs_dict(*orc.join_pairs(A, B)) == want
    # symmetry
    assert _pairs_dict(*orc.join_pairs(B, A)) == {(q, p): n for (p, q), n in want.items()}
    # centre-sampled canvases join the same way
    mca = orc.centre_brute(a, s, i0, j0, nw, nh) > 0
    mcb = orc.centre_brute(b, s, i0, j0, nw, nh) > 0
    wc = {}
    for p in range(a.n_polys):
        for q in range(b.n_polys):
            n = int(np.count_nonzero(mca[p] & mcb[q]))
            if n:
                wc[(p, q)] = n
    got = _pairs_dict(*orc.join_pairs(orc.Approx(a, eps, centre=True),
                                      orc.Approx(b, eps, centre=True)))
    assert got == wc


def test_join_self_partition_and_no_false_negatives(orc):
    polys = voronoi_partition(20, 50000, (3, 12), seed=6, jitter_seed=7)
    eps = 300
    A = orc.Approx(polys, eps)
    got = _pairs_dict(*orc.join_pairs(A, A))
    # the diagonal is each approximation's own size
    P, R, X0, X1 = A.intervals()
    for p in range(polys.n_polys):
        assert got[(p, p)] == int((X1[P == p] - X0[P == p]).sum())
    # neighbours (a shared boundary point) are always paired; here: two
    # polygons that hold the two ends of a short segment across their border
    stars = star_polygons(6, 9, 100.0, 1500.0, 6000, 99)
    S = orc.Approx(stars, 40)
    pairs = _pairs_dict(*orc.join_pairs(S, S))
    rng = np.random.default_rng(8)
    pts = rng.integers(0, 6000, size=(3000, 2)).astype(np.int32)
    for x, y in pts.tolist():
        c, _ = S.exact(np.array([x, y], np.int32))
        ins = np.nonzero(c)[0]
        for p in ins:
            for q in ins:
                assert (int(p), int(q)) in pairs
