"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Per-cell polygon sets and per-polygon COUNT / SUM must be identical (integer
work, bit-exact).  Sizes are chosen so that the oracle finishes in seconds
while the GPU structures still span many tiles, blocks and ragged borders.
"""
import numpy as np
import pytest

from gen import (CITY_BOX, city_points, polygons_from_rings, star_polygons, tiny_workload,
                 uniform_points, voronoi_partition)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sba():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2010_12548_amd as m
    m.lib()
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run_agg(A, xy, vals=None, search=None):
    c, s = A.aggregate(dev(xy), dev(vals) if vals is not None else None, search=search)
    torch.cuda.synchronize()
    return c.cpu().numpy().astype(np.uint64), (s.cpu().numpy() if s is not None else None)


def expected_sets(orc_A, n_polys, i0, j0, nw, nh):
    """Per-cell polygon tuples over a window, from the oracle's row intervals."""
    m = np.zeros((n_polys, nh, nw), bool)
    P, R, X0, X1 = orc_A.intervals()
    for p, r, a, b in zip(P, R, X0, X1):
        if j0 <= r < j0 + nh:
            a2, b2 = max(a, i0), min(b, i0 + nw)
            if a2 < b2:
                m[p, r - j0, a2 - i0:b2 - i0] = True
    out = {}
    for j in range(nh):
        for i in range(nw):
            out[(i0 + i, j0 + j)] = tuple(int(p) for p in np.nonzero(m[:, j, i])[0])
    return out


def gpu_sets(A, cells):
    ij = np.array(cells, dtype=np.int64).reshape(-1)
    refs = A.lookup(dev(ij)).cpu().numpy()
    return dict(zip(cells, A.decode(refs)))


def window_of(polys, s, pad=3):
    xy = polys.xy.reshape(-1, 2).astype(np.int64)
    i0 = int(np.floor(xy[:, 0].min() / s)) - pad
    j0 = int(np.floor(xy[:, 1].min() / s)) - pad
    i1 = int(np.floor(xy[:, 0].max() / s)) + pad
    j1 = int(np.floor(xy[:, 1].max() / s)) + pad
    return i0, j0, i1 - i0 + 1, j1 - j0 + 1


def shifted(polys, d):
    return polygons_from_rings([[r + d for r in polys.rings_of(p)] for p in range(polys.n_polys)])


# --------------------------------------------------------------- cell sets

HAND = [
    [[[1, 1], [7, 1], [1, 5]]],
    [[[0, 0], [10, 0], [10, 10], [0, 10]], [[4, 4], [6, 4], [6, 6], [4, 6]]],
    [[[0, 0], [30, 0], [30, 10], [10, 10], [10, 20], [30, 20], [30, 30], [0, 30]]],
    [[[0, 0], [40, 0], [20, 1], [20, 30]]],
    [[[5, 5], [25, 5], [25, 5], [15, 25]]],
    [[[3, 3], [3, 3], [9, 3]]],
    [[[-17, -9], [12, -9], [12, 6], [-17, 6]]],
    [[[0, 0], [24, 12], [0, 24], [12, 12]]],
]


@pytest.mark.parametrize("eps", [2, 3, 5, 9, 15])
def test_cell_sets_hand_shapes_grid(sba, orc, eps):
    polys = polygons_from_rings([[np.array(r) for r in p] for p in HAND])
    A = sba.Approx.from_polygons(polys, eps)
    O = orc.Approx(polys, eps)
    i0, j0, nw, nh = window_of(polys, O.s)
    want = expected_sets(O, polys.n_polys, i0, j0, nw, nh)
    got = gpu_sets(A, list(want.keys()))
    assert got == want


@pytest.mark.parametrize("seed,eps,tl", [(0, 4, 3), (1, 7, 4), (2, 13, 3), (3, 25, 5), (4, 3, 8)])
def test_cell_sets_random_stars_grid(sba, orc, seed, eps, tl):
    polys = star_polygons(12, 9 + seed, 20.0, 400.0, 1500, 500 + seed)
    A = sba.Approx.from_polygons(polys, eps, tile_log2=tl)
    O = orc.Approx(polys, eps)
    i0, j0, nw, nh = window_of(polys, O.s)
    want = expected_sets(O, polys.n_polys, i0, j0, nw, nh)
    got = gpu_sets(A, list(want.keys()))
    bad = [k for k in want if got[k] != want[k]]
    assert not bad, (len(bad), bad[:5], [want[k] for k in bad[:5]], [got[k] for k in bad[:5]])
    info = A.info()
    assert info["n_blocks"] > 0 and info["n_tiles"] > info["n_blocks"]


@pytest.mark.parametrize("seed,eps", [(0, 4), (1, 9), (2, 30)])
def test_cell_sets_random_stars_hilbert(sba, orc, seed, eps):
    polys = star_polygons(10, 11, 20.0, 300.0, 1200, 700 + seed)
    A = sba.Approx.from_polygons(polys, eps, kind="hilbert")
    O = orc.Approx(polys, eps)
    i0, j0, nw, nh = window_of(polys, O.s)
    want = expected_sets(O, polys.n_polys, i0, j0, nw, nh)
    got = gpu_sets(A, list(want.keys()))
    bad = [k for k in want if got[k] != want[k]]
    assert not bad, (len(bad), bad[:5])


@pytest.mark.parametrize("seed,eps,d", [(0, 6, 150), (1, 11, -300), (2, 40, 0), (3, 3, -1000)])
def test_hilbert_runs_equal_oracle(sba, orc, seed, eps, d):
    polys = shifted(star_polygons(6, 10, 10.0, 120.0, 500, 900 + seed), d)
    A = sba.Approx.from_polygons(polys, eps, kind="hilbert")
    info = A.info()
    O = orc.Approx(polys, eps)
    L = O.hilbert_level()
    assert info["level"] == L
    assert (info["gi0"], info["gj0"], info["gw"], info["gh"]) == O.union_box()
    st_o, off_o, ids_o = O.hilbert_runs(L)
    st_g, ref_g = A.runs()
    st_g = st_g.cpu().numpy().astype(np.uint64)
    np.testing.assert_array_equal(st_g, st_o)
    sets_o = [tuple(int(v) for v in ids_o[off_o[r]:off_o[r + 1]]) for r in range(len(st_o))]
    assert A.decode(ref_g.cpu().numpy()) == sets_o


# --------------------------------------------------------------- aggregates

def test_tiny_workload_bit_exact(sba, orc):
    xy, vals, polys = tiny_workload()
    O = orc.Approx(polys, 64)
    want_c, want_s = O.aggregate(xy, vals)
    A = sba.Approx.from_polygons(polys, 64)
    c, s = run_agg(A, xy, vals)
    np.testing.assert_array_equal(c, want_c)
    np.testing.assert_array_equal(s, want_s)
    c2, s2 = run_agg(A, xy, None)
    np.testing.assert_array_equal(c2, want_c)
    assert s2 is None


@pytest.mark.parametrize("tl", [3, 5, 8])
def test_tiny_workload_tile_sizes(sba, orc, tl):
    xy, vals, polys = tiny_workload(300_001)
    want_c, want_s = orc.Approx(polys, 64).aggregate(xy, vals)
    A = sba.Approx.from_polygons(polys, 64, tile_log2=tl)
    c, s = run_agg(A, xy, vals)
    np.testing.assert_array_equal(c, want_c)
    np.testing.assert_array_equal(s, want_s)


@pytest.mark.parametrize("n", [0, 1, 2, 3, 5, 255, 513])
def test_small_and_ragged_n(sba, orc, n):
    rng = np.random.default_rng(n)
    polys = star_polygons(5, 12, 50.0, 400.0, 1000, 31)
    xy = rng.integers(-100, 1100, size=2 * n).astype(np.int32)
    vals = rng.integers(-10**6, 10**6, size=n).astype(np.int64)
    O = orc.Approx(polys, 10)
    want_c, want_s = O.aggregate(xy, vals)
    A = sba.Approx.from_polygons(polys, 10)
    c, s = run_agg(A, xy, vals)
    np.testing.assert_array_equal(c, want_c)
    np.testing.assert_array_equal(s, want_s)


def test_extreme_point_coordinates(sba, orc):
    polys = star_polygons(4, 10, 50.0, 400.0, 1000, 5)
    ext = np.array([-2**31, -2**31, 2**31 - 1, 2**31 - 1, -2**31, 2**31 - 1, 0, 0, 500, 500,
                    2**30, -2**30], dtype=np.int64).astype(np.int32)
    vals = np.arange(6, dtype=np.int64) * 1000 + 7
    want_c, want_s = orc.Approx(polys, 20).aggregate(ext, vals)
    for kind in ("grid", "hilbert"):
        A = sba.Approx.from_polygons(polys, 20, kind=kind)
        c, s = run_agg(A, ext, vals)
        np.testing.assert_array_equal(c, want_c)
        np.testing.assert_array_equal(s, want_s)


def test_shuffle_invariance(sba):
    xy, vals, polys = tiny_workload(400_000)
    A = sba.Approx.from_polygons(polys, 64)
    c1, s1 = run_agg(A, xy, vals)
    perm = np.random.default_rng(9).permutation(400_000)
    xy2 = xy.reshape(-1, 2)[perm].reshape(-1)
    c2, s2 = run_agg(A, xy2, vals[perm])
    np.testing.assert_array_equal(c1, c2)
    np.testing.assert_array_equal(s1, s2)
    c3, s3 = run_agg(A, xy, vals)
    np.testing.assert_array_equal(c1, c3)
    np.testing.assert_array_equal(s1, s3)


@pytest.mark.parametrize("eps", [6, 40, 700, 6000])
def test_partition_all_layouts(sba, orc, eps):
    polys = voronoi_partition(40, 200_000, (3, 25), seed=3, jitter_seed=4)
    xy = uniform_points(500_000, -1000, 201_000, 77)
    vals = np.random.default_rng(1).integers(1, 10**7, size=500_000).astype(np.int64)
    O = orc.Approx(polys, eps)
    want_c, want_s = O.aggregate(xy, vals)
    G = sba.Approx.from_polygons(polys, eps)
    c, s = run_agg(G, xy, vals)
    np.testing.assert_array_equal(c, want_c)
    np.testing.assert_array_equal(s, want_s)
    H = sba.Approx.from_polygons(polys, eps, kind="hilbert", search="learned", log2_leaves=8)
    for search in ("binary", "learned"):
        c, s = run_agg(H, xy, vals, search=search)
        np.testing.assert_array_equal(c, want_c)
        np.testing.assert_array_equal(s, want_s)


def test_overlap_depth_and_limit(sba, orc):
    rings = [[np.array([[-k, -k], [100 + k, -k], [100 + k, 100 + k], [-k, 100 + k]])] for k in range(20)]
    polys = polygons_from_rings(rings)
    xy = uniform_points(100_000, -40, 140, 3)
    want_c, _ = orc.Approx(polys, 3).aggregate(xy)
    A = sba.Approx.from_polygons(polys, 3)
    c, _ = run_agg(A, xy)
    np.testing.assert_array_equal(c, want_c)
    deep = polygons_from_rings(rings + [[np.array([[-k, -k], [100 + k, -k], [100 + k, 100 + k],
                                                    [-k, 100 + k]])] for k in range(20, 40)])
    with pytest.raises(sba.SbaError) as e:
        sba.Approx.from_polygons(deep, 3)
    assert e.value.code == -5


def test_error_codes(sba):
    polys = star_polygons(3, 8, 50.0, 200.0, 1000, 2)
    big = polygons_from_rings([[np.array([[0, 0], [1 << 30, 0], [0, 5]])]])
    with pytest.raises(sba.SbaError) as e:
        sba.Approx.from_polygons(big, 10)
    assert e.value.code == -2
    A = sba.Approx.from_polygons(polys, 10)
    buf = torch.zeros(9, dtype=torch.int32, device="cuda")
    with pytest.raises(sba.SbaError):
        A.aggregate(buf[1:5])        # not 16-byte aligned
    empty = polygons_from_rings([])
    E = sba.Approx.from_polygons(empty, 10)
    c, _ = E.aggregate(dev(np.array([1, 2, 3, 4], np.int32)))
    assert c.numel() == 0


def test_city_partition_sampled(sba, orc):
    """City-like partition (260 jittered Voronoi cells), 4M mixture points,
    the three distance bounds; full oracle comparison."""
    from gen import city_polygons
    polys = city_polygons()
    xy, vals = city_points(4_000_000)
    for eps in (100, 1000, 10000):
        O = orc.Approx(polys, eps)
        want_c, want_s = O.aggregate(xy, vals)
        A = sba.Approx.from_polygons(polys, eps)
        c, s = run_agg(A, xy, vals)
        np.testing.assert_array_equal(c, want_c)
        np.testing.assert_array_equal(s, want_s)
        assert int(c.sum()) >= 4_000_000


@pytest.mark.parametrize("eps", [100, 1000, 10000])
def test_compact_and_wide_formats_agree(sba, orc, eps):
    """The grid stored with 16-bit codes (directory staged in LDS by the
    probe) and with 32-bit codes (directory read from global memory) give
    the oracle's answer and the oracle's cell sets."""
    from gen import city_polygons
    polys = city_polygons()
    xy, vals = city_points(1_000_000)
    O = orc.Approx(polys, eps)
    want_c, want_s = O.aggregate(xy, vals)
    for wide in (0, 1):
        sba.lib().sba_debug_force_wide_grid(wide)
        try:
            A = sba.Approx.from_polygons(polys, eps)
        finally:
            sba.lib().sba_debug_force_wide_grid(0)
        assert A.info()["compact"] == 1 - wide
        c, s = run_agg(A, xy, vals)
        np.testing.assert_array_equal(c, want_c)
        np.testing.assert_array_equal(s, want_s)
        c, _ = run_agg(A, xy, None)
        np.testing.assert_array_equal(c, want_c)
        A.close()


@pytest.mark.parametrize("tl,sl", [(4, 1), (6, 1), (6, 2), (6, 3), (6, 4), (6, 6), (8, 4), (8, 5),
                                   (10, 4)])
@pytest.mark.parametrize("wide", [0, 1])
def test_sub_tile_levels(sba, orc, tl, sl, wide):
    """Every tile / sub-tile split, in both formats, stores the oracle's cell
    sets and gives its aggregates (overlapping stars: multi-polygon sets in
    fine blocks, sub-tiles cut by the edge of the stored box)."""
    polys = star_polygons(12, 9, 20.0, 400.0, 1500, 77)
    eps = 5
    O = orc.Approx(polys, eps)
    sba.lib().sba_debug_force_wide_grid(wide)
    try:
        A = sba.Approx.from_polygons(polys, eps, tile_log2=tl, sub_log2=sl)
    finally:
        sba.lib().sba_debug_force_wide_grid(0)
    info = A.info()
    assert (info["tile_log2"], info["sub_log2"], info["compact"]) == (tl, sl, 1 - wide)
    assert info["n_blocks"] > 0
    if sl < tl:
        assert info["n_sub"] > 0
    i0, j0, nw, nh = window_of(polys, O.s)
    want = expected_sets(O, polys.n_polys, i0, j0, nw, nh)
    got = gpu_sets(A, list(want.keys()))
    bad = [k for k in want if got[k] != want[k]]
    assert not bad, (len(bad), bad[:5])
    rng = np.random.default_rng(tl * 16 + sl)
    n = 200_001
    xy = rng.integers(-50, 1600, size=2 * n).astype(np.int32)
    vals = rng.integers(100, 10000, size=n).astype(np.int64)
    want_c, want_s = O.aggregate(xy, vals)
    # the sub-directory staged in LDS where it fits, and read from global memory
    for lsub in (-1, 0):
        sba.lib().sba_debug_grid16_lsub(lsub)
        try:
            c, s = run_agg(A, xy, vals)
        finally:
            sba.lib().sba_debug_grid16_lsub(-1)
        np.testing.assert_array_equal(c, want_c)
        np.testing.assert_array_equal(s, want_s)


def test_sub_level_rejects_bad_split(sba):
    polys = star_polygons(3, 9, 20.0, 400.0, 1500, 78)
    for tl, sl in ((5, 6), (6, -1)):
        with pytest.raises(RuntimeError):
            sba.Approx.from_polygons(polys, 5, tile_log2=tl, sub_log2=sl)


@pytest.mark.parametrize("eps", [100, 1000, 10000])
def test_lds_sub_directory_city(sba, orc, eps):
    """City partition with the automatic layout: where the 16-bit
    sub-directory fits the LDS beside the directory and the bins (10 m, 100 m)
    the probe stages it there (level 2 in the kernel name) and must give the
    oracle's answer; the same handle read through the global sub-directory
    (level 1) too."""
    from gen import city_polygons
    polys = city_polygons()
    xy, vals = city_points(1_000_001)
    want_c, want_s = orc.Approx(polys, eps).aggregate(xy, vals)
    A = sba.Approx.from_polygons(polys, eps)
    info = A.info()
    kern = A.probe_kernel(True)
    if eps >= 1000:
        assert info["sub_log2"] < info["tile_log2"]
        assert kern.startswith("k_probe_grid16<true, 2,"), kern
    for lsub in (-1, 0):
        sba.lib().sba_debug_grid16_lsub(lsub)
        try:
            c, s = run_agg(A, xy, vals)
            c2, _ = run_agg(A, xy, None)
            if lsub == 0 and info["sub_log2"] < info["tile_log2"]:
                assert A.probe_kernel(True).startswith("k_probe_grid16<true, 1,")
        finally:
            sba.lib().sba_debug_grid16_lsub(-1)
        np.testing.assert_array_equal(c, want_c)
        np.testing.assert_array_equal(s, want_s)
        np.testing.assert_array_equal(c2, want_c)


@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("eps,tl,sl", [(1000, 5, 5), (1000, 5, 3), (100, 0, 0)])
def test_set_modes_of_grid_probe(sba, orc, mode, eps, tl, sl):
    """Points in multi-polygon cells are added the same way whether the probe
    walks the global set table, a copy in LDS, or keeps one bin per set (at
    1 m the bins do not fit and every mode falls back)."""
    from gen import city_polygons
    polys = city_polygons()
    xy, vals = city_points(1_000_001)
    want_c, want_s = orc.Approx(polys, eps).aggregate(xy, vals)
    A = sba.Approx.from_polygons(polys, eps, tile_log2=tl, sub_log2=sl)
    assert A.info()["n_sets"] > 0
    sba.lib().sba_debug_grid16_sets(mode)
    try:
        c, s = run_agg(A, xy, vals)
        c2, _ = run_agg(A, xy, None)
    finally:
        sba.lib().sba_debug_grid16_sets(-1)
    np.testing.assert_array_equal(c, want_c)
    np.testing.assert_array_equal(s, want_s)
    np.testing.assert_array_equal(c2, want_c)


@pytest.mark.parametrize("eps", [2, 3, 4])
def test_unit_and_small_cells_aggregate(sba, orc, eps):
    """Cell side 1 (eps = 2: the probe's division by one) and side 2 (eps 3
    and 4): the aggregates equal the oracle's."""
    polys = star_polygons(8, 10, 5.0, 60.0, 300, 41)
    rng = np.random.default_rng(eps)
    n = 100_003
    xy = rng.integers(-20, 330, size=2 * n).astype(np.int32)
    vals = rng.integers(-1000, 1000, size=n).astype(np.int64)
    O = orc.Approx(polys, eps)
    A = sba.Approx.from_polygons(polys, eps)
    assert A.info()["s"] == O.s
    want_c, want_s = O.aggregate(xy, vals)
    c, s = run_agg(A, xy, vals)
    np.testing.assert_array_equal(c, want_c)
    np.testing.assert_array_equal(s, want_s)


@pytest.mark.parametrize("eps", [300, 3000])
def test_many_polygons_item_probe(sba, orc, eps):
    """More polygons than per-polygon LDS bins hold: the probe counts each
    item of points in an LDS table of cell codes.  Points in no order (the
    table fills and later codes go to global atomics) and in row-band order
    (few codes per item) give the oracle's aggregates on every layout."""
    polys = voronoi_partition(6000, 1_000_000, (2, 6), seed=31, jitter_seed=32)
    n = 600_001
    xy = uniform_points(n, -2000, 1_002_000, 5)
    vals = np.random.default_rng(2).integers(0, 10**6, size=n).astype(np.int64)
    pts = xy.reshape(-1, 2)
    order = np.lexsort((pts[:, 0], pts[:, 1] // 5000))
    xy_sorted = np.ascontiguousarray(pts[order]).reshape(-1)
    vals_sorted = vals[order]
    O = orc.Approx(polys, eps)
    want_c, want_s = O.aggregate(xy, vals)
    handles = []
    sba.lib().sba_debug_force_wide_grid(1)
    try:
        handles.append(sba.Approx.from_polygons(polys, eps))
    finally:
        sba.lib().sba_debug_force_wide_grid(0)
    handles.append(sba.Approx.from_polygons(polys, eps, kind="hilbert", search="binary"))
    handles.append(sba.Approx.from_polygons(polys, eps, kind="hilbert", search="learned",
                                            log2_leaves=10))
    for A in handles:
        assert A.probe_kernel(True).startswith("k_probe_items")
        for p, v in ((xy, vals), (xy_sorted, vals_sorted)):
            c, s = run_agg(A, p, v)
            np.testing.assert_array_equal(c, want_c)
            np.testing.assert_array_equal(s, want_s)
            c, _ = run_agg(A, p, None)
            np.testing.assert_array_equal(c, want_c)
        A.close()


# --------------------------------------------------------------- result range (Sec. 6)

@pytest.mark.parametrize("kind,search", [("grid", None), ("hilbert", "binary"),
                                         ("hilbert", "learned")])
@pytest.mark.parametrize("seed,eps", [(0, 4), (1, 9), (2, 30)])
def test_boundary_only_cells_and_aggregates(sba, orc, kind, search, seed, eps):
    """A boundary-only handle stores the oracle's boundary cells B(P) and its
    aggregate is the oracle's partial count and sum over them."""
    polys = star_polygons(10, 11, 20.0, 300.0, 1200, 900 + seed)
    OB = orc.Approx(polys, eps, boundary_only=True)
    kw = {"kind": kind, "boundary_only": True}
    if search:
        kw["search"] = search
    A = sba.Approx.from_polygons(polys, eps, **kw)
    assert A.info()["boundary_only"] == 1
    i0, j0, nw, nh = window_of(polys, OB.s)
    want = expected_sets(OB, polys.n_polys, i0, j0, nw, nh)
    got = gpu_sets(A, list(want.keys()))
    bad = [k for k in want if got[k] != want[k]]
    assert not bad, (len(bad), bad[:5])
    rng = np.random.default_rng(seed)
    n = 150_001
    xy = rng.integers(-100, 1300, size=2 * n).astype(np.int32)
    vals = rng.integers(0, 10000, size=n).astype(np.int64)
    want_c, want_s = OB.aggregate(xy, vals)
    c, s = run_agg(A, xy, vals)
    np.testing.assert_array_equal(c, want_c)
    np.testing.assert_array_equal(s, want_s)


@pytest.mark.parametrize("eps", [100, 1000, 10000])
def test_city_result_range_contains_exact(sba, orc, eps):
    """GPU alpha and beta on the city partition: beta equals the oracle's, and
    alpha - beta <= exact <= alpha for every polygon (counts and sums)."""
    from gen import city_polygons
    polys = city_polygons()
    xy, vals = city_points(1_000_000)
    A = sba.Approx.from_polygons(polys, eps)
    Bh = sba.Approx.from_polygons(polys, eps, boundary_only=True)
    ac, asum = run_agg(A, xy, vals)
    bc, bsum = run_agg(Bh, xy, vals)
    wb_c, wb_s = orc.Approx(polys, eps, boundary_only=True).aggregate(xy, vals)
    np.testing.assert_array_equal(bc, wb_c)
    np.testing.assert_array_equal(bsum, wb_s)
    ec, esum = orc.Approx(polys, eps).exact(xy, vals)
    ac, bc, ec = ac.astype(np.int64), bc.astype(np.int64), ec.astype(np.int64)
    assert np.all(ac - bc <= ec) and np.all(ec <= ac)
    assert np.all(asum - bsum <= esum) and np.all(esum <= asum)


# --------------------------------------------------------------- centre-sampled cells (Sec. 2.2)

@pytest.mark.parametrize("kind,search", [("grid", None), ("hilbert", "binary"),
                                         ("hilbert", "learned")])
@pytest.mark.parametrize("seed,eps", [(0, 2), (1, 4), (2, 9), (3, 30)])
def test_centre_sampled_cells_and_aggregates(sba, orc, kind, search, seed, eps):
    """A centre-sampled handle stores the oracle's C(P) (cells whose centre is
    inside) in every layout, and aggregates like the oracle."""
    polys = star_polygons(10, 11, 20.0, 300.0, 1200, 700 + seed)
    OC = orc.Approx(polys, eps, centre=True)
    kw = {"kind": kind, "centre_sampled": True}
    if search:
        kw["search"] = search
    A = sba.Approx.from_polygons(polys, eps, **kw)
    assert A.info()["centre_sampled"] == 1
    i0, j0, nw, nh = window_of(polys, OC.s)
    want = expected_sets(OC, polys.n_polys, i0, j0, nw, nh)
    got = gpu_sets(A, list(want.keys()))
    bad = [k for k in want if got[k] != want[k]]
    assert not bad, (len(bad), bad[:5])
    rng = np.random.default_rng(seed)
    n = 150_001
    xy = rng.integers(-100, 1300, size=2 * n).astype(np.int32)
    vals = rng.integers(-5000, 10000, size=n).astype(np.int64)
    want_c, want_s = OC.aggregate(xy, vals)
    c, s = run_agg(A, xy, vals)
    np.testing.assert_array_equal(c, want_c)
    np.testing.assert_array_equal(s, want_s)


@pytest.mark.parametrize("tl,sl", [(6, 3), (8, 4), (5, 5)])
@pytest.mark.parametrize("wide", [0, 1])
def test_centre_sampled_grid_levels(sba, orc, tl, sl, wide):
    polys = star_polygons(12, 9, 20.0, 400.0, 1500, 77)
    eps = 5
    OC = orc.Approx(polys, eps, centre=True)
    sba.lib().sba_debug_force_wide_grid(wide)
    try:
        A = sba.Approx.from_polygons(polys, eps, tile_log2=tl, sub_log2=sl, centre_sampled=True)
    finally:
        sba.lib().sba_debug_force_wide_grid(0)
    rng = np.random.default_rng(tl * 16 + sl)
    n = 200_001
    xy = rng.integers(-50, 1600, size=2 * n).astype(np.int32)
    vals = rng.integers(100, 10000, size=n).astype(np.int64)
    want_c, want_s = OC.aggregate(xy, vals)
    c, s = run_agg(A, xy, vals)
    np.testing.assert_array_equal(c, want_c)
    np.testing.assert_array_equal(s, want_s)


def test_centre_sampled_city_partition(sba, orc):
    """City partition: the oracle's centre-sampled aggregates, and every point
    whose cell centre lies in the box is counted exactly once."""
    from gen import city_polygons
    polys = city_polygons()
    xy, vals = city_points(2_000_000)
    B = CITY_BOX
    p = xy.reshape(-1, 2).astype(np.int64)
    for eps in (100, 1000, 10000):
        OC = orc.Approx(polys, eps, centre=True)
        want_c, want_s = OC.aggregate(xy, vals)
        A = sba.Approx.from_polygons(polys, eps, centre_sampled=True)
        c, s = run_agg(A, xy, vals)
        np.testing.assert_array_equal(c, want_c)
        np.testing.assert_array_equal(s, want_s)
        sc = OC.s
        cx, cy = (2 * (p[:, 0] // sc) + 1) * sc, (2 * (p[:, 1] // sc) + 1) * sc
        assert int(c.sum()) == int(np.count_nonzero((cx < 2 * B) & (cy < 2 * B)))


def test_centre_sampled_rejects_boundary_only(sba):
    polys = star_polygons(3, 8, 50.0, 200.0, 1000, 2)
    with pytest.raises(sba.SbaError):
        sba.Approx.from_polygons(polys, 10, centre_sampled=True, boundary_only=True)


def _range(sba, A, Bh, xy, vals):
    c, s, bc, bs = sba.aggregate_range(A, Bh, dev(xy), dev(vals) if vals is not None else None)
    torch.cuda.synchronize()
    f = lambda t: t.cpu().numpy() if t is not None else None  # noqa: E731
    return f(c).astype(np.uint64), f(s), f(bc).astype(np.uint64), f(bs)


@pytest.mark.parametrize("eps", [100, 1000, 10000])
def test_result_range_one_pass_city(sba, orc, eps):
    """alpha and beta from one kernel over the points equal the oracle's full
    and boundary-only aggregates."""
    from gen import city_polygons
    polys = city_polygons()
    xy, vals = city_points(1_000_001)
    A = sba.Approx.from_polygons(polys, eps)
    inf = A.info()
    Bh = sba.Approx.from_polygons(polys, eps, boundary_only=True, tile_log2=inf["tile_log2"],
                                  sub_log2=inf["sub_log2"])
    if eps >= 1000:
        assert sba.range_kernel(A, Bh).startswith("k_probe_range16")
    wa_c, wa_s = orc.Approx(polys, eps).aggregate(xy, vals)
    wb_c, wb_s = orc.Approx(polys, eps, boundary_only=True).aggregate(xy, vals)
    c, s, bc, bs = _range(sba, A, Bh, xy, vals)
    np.testing.assert_array_equal(c, wa_c)
    np.testing.assert_array_equal(s, wa_s)
    np.testing.assert_array_equal(bc, wb_c)
    np.testing.assert_array_equal(bs, wb_s)
    c, s, bc, bs = _range(sba, A, Bh, xy, None)
    assert s is None and bs is None
    np.testing.assert_array_equal(c, wa_c)
    np.testing.assert_array_equal(bc, wb_c)


@pytest.mark.parametrize("tl,sl", [(6, 3), (5, 5), (8, 4)])
def test_result_range_one_pass_stars(sba, orc, tl, sl):
    polys = star_polygons(12, 9, 20.0, 400.0, 1500, 88)
    eps = 5
    A = sba.Approx.from_polygons(polys, eps, tile_log2=tl, sub_log2=sl)
    Bh = sba.Approx.from_polygons(polys, eps, boundary_only=True, tile_log2=tl, sub_log2=sl)
    assert sba.range_kernel(A, Bh) != ""
    rng = np.random.default_rng(tl)
    n = 200_001
    xy = rng.integers(-50, 1600, size=2 * n).astype(np.int32)
    vals = rng.integers(0, 10000, size=n).astype(np.int64)
    wa = orc.Approx(polys, eps).aggregate(xy, vals)
    wb = orc.Approx(polys, eps, boundary_only=True).aggregate(xy, vals)
    c, s, bc, bs = _range(sba, A, Bh, xy, vals)
    np.testing.assert_array_equal(c, wa[0])
    np.testing.assert_array_equal(s, wa[1])
    np.testing.assert_array_equal(bc, wb[0])
    np.testing.assert_array_equal(bs, wb[1])
    # different tiles: two passes, same answer
    B2 = sba.Approx.from_polygons(polys, eps, boundary_only=True, tile_log2=4, sub_log2=4)
    if (tl, sl) != (4, 4):
        assert sba.range_kernel(A, B2) == ""
    c, s, bc, bs = _range(sba, A, B2, xy, vals)
    np.testing.assert_array_equal(c, wa[0])
    np.testing.assert_array_equal(bc, wb[0])
    np.testing.assert_array_equal(bs, wb[1])
    with pytest.raises(sba.SbaError):       # beta must be the boundary-only handle
        _range(sba, A, A, xy, vals)


@pytest.mark.parametrize("log2_leaves", [4, 8, 12, 16])
def test_learned_search_never_falls_back(sba, log2_leaves):
    """The leaves' stored error bounds every key of their key range, so the
    learned search's bracket check never fails and its answers equal binary
    search for every point (in and out of the polygons)."""
    from gen import city_polygons
    polys = city_polygons()
    xy, _ = city_points(1_000_000)
    for eps in (100, 1000):
        H = sba.Approx.from_polygons(polys, eps, kind="hilbert", search="learned",
                                     log2_leaves=log2_leaves)
        fb, mm = H.learned_fallbacks(dev(xy))
        assert (fb, mm) == (0, 0)
    rng = np.random.default_rng(log2_leaves)
    stars = star_polygons(12, 9, 20.0, 400.0, 1500, 55)
    pts = rng.integers(-100, 1700, size=2 * 300_000).astype(np.int32)
    for eps in (3, 9):
        H = sba.Approx.from_polygons(stars, eps, kind="hilbert", search="learned",
                                     log2_leaves=log2_leaves)
        assert H.learned_fallbacks(dev(pts)) == (0, 0)


def test_partitioned_probe_equals_oracle(sba, orc):
    """Points partitioned by coarse region, then probed: the oracle's answer
    on every layout, with and without values, odd sizes, too-small scratch."""
    polys = voronoi_partition(6000, 1_000_000, (2, 6), seed=31, jitter_seed=32)
    n = 600_001
    xy = uniform_points(n, -2000, 1_002_000, 6)
    vals = np.random.default_rng(9).integers(-10**6, 10**6, size=n).astype(np.int64)
    eps = 300
    want_c, want_s = orc.Approx(polys, eps).aggregate(xy, vals)
    handles = [sba.Approx.from_polygons(polys, eps, kind="hilbert", search="learned"),
               sba.Approx.from_polygons(polys, eps)]
    sba.lib().sba_debug_force_wide_grid(1)
    try:
        handles.append(sba.Approx.from_polygons(polys, eps))
    finally:
        sba.lib().sba_debug_force_wide_grid(0)
    txy, tv = dev(xy), dev(vals)
    for A in handles:
        searches = ("binary", "learned") if A.kind == "hilbert" else ("binary",)
        for search in searches:
            c, s = A.aggregate_partitioned(txy, tv, search=search)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(c.cpu().numpy().astype(np.uint64), want_c)
            np.testing.assert_array_equal(s.cpu().numpy(), want_s)
            c, _ = A.aggregate_partitioned(txy, None, search=search)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(c.cpu().numpy().astype(np.uint64), want_c)
    A = handles[0]
    small = torch.empty(A.scratch_bytes(n) - 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(sba.SbaError):
        A.aggregate_partitioned(txy, tv, scratch=small)
    # below the partition threshold the direct probe answers
    c, s = A.aggregate_partitioned(txy[:2 * 1001], tv[:1001])
    wc, ws = orc.Approx(polys, eps).aggregate(xy[:2 * 1001], vals[:1001])
    np.testing.assert_array_equal(c.cpu().numpy().astype(np.uint64), wc)
    np.testing.assert_array_equal(s.cpu().numpy(), ws)


def test_partitioned_probe_city_hilbert(sba, orc):
    from gen import city_polygons
    polys = city_polygons()
    xy, vals = city_points(1_000_001)
    for eps in (100, 1000):
        want_c, want_s = orc.Approx(polys, eps).aggregate(xy, vals)
        A = sba.Approx.from_polygons(polys, eps, kind="hilbert", search="learned")
        c, s = A.aggregate_partitioned(dev(xy), dev(vals))
        torch.cuda.synchronize()
        np.testing.assert_array_equal(c.cpu().numpy().astype(np.uint64), want_c)
        np.testing.assert_array_equal(s.cpu().numpy(), want_s)


def test_edge_sizes_of_range_and_partitioned(sba, orc):
    """Empty and odd point counts through the one-pass range probe, and the
    partitioned probe just above its threshold with a ragged last chunk."""
    polys = star_polygons(12, 9, 20.0, 400.0, 1500, 88)
    eps = 5
    A = sba.Approx.from_polygons(polys, eps, tile_log2=6, sub_log2=3)
    Bh = sba.Approx.from_polygons(polys, eps, boundary_only=True, tile_log2=6, sub_log2=3)
    OA, OB = orc.Approx(polys, eps), orc.Approx(polys, eps, boundary_only=True)
    rng = np.random.default_rng(77)
    for n in (0, 1, 2, 1001, (1 << 17) + 3):
        xy = rng.integers(-50, 1600, size=2 * n).astype(np.int32)
        vals = rng.integers(-100, 10000, size=n).astype(np.int64)
        txy = torch.from_numpy(xy).cuda() if n else torch.zeros(0, dtype=torch.int32, device="cuda")
        tv = torch.from_numpy(vals).cuda() if n else torch.zeros(0, dtype=torch.int64, device="cuda")
        c, s, bc, bs = sba.aggregate_range(A, Bh, txy, tv)
        torch.cuda.synchronize()
        wa, wb = OA.aggregate(xy, vals), OB.aggregate(xy, vals)
        np.testing.assert_array_equal(c.cpu().numpy().astype(np.uint64), wa[0])
        np.testing.assert_array_equal(s.cpu().numpy(), wa[1])
        np.testing.assert_array_equal(bc.cpu().numpy().astype(np.uint64), wb[0])
        np.testing.assert_array_equal(bs.cpu().numpy(), wb[1])
    H = sba.Approx.from_polygons(polys, eps, kind="hilbert", search="learned")
    for n in ((1 << 17), (1 << 17) + 1, 3 * (1 << 16) + 5):
        xy = rng.integers(-50, 1600, size=2 * n).astype(np.int32)
        vals = rng.integers(-100, 10000, size=n).astype(np.int64)
        c, s = H.aggregate_partitioned(dev(xy), dev(vals))
        torch.cuda.synchronize()
        wa = OA.aggregate(xy, vals)
        np.testing.assert_array_equal(c.cpu().numpy().astype(np.uint64), wa[0])
        np.testing.assert_array_equal(s.cpu().numpy(), wa[1])


# --------------------------------------------------------------- build paths

@pytest.mark.parametrize("case", ["city_grid", "city_hilbert", "city_centre", "city_boundary",
                                  "stars_grid"])
def test_every_build_path_gives_the_oracles_answer(sba, orc, case):
    """The build stages choose between work in LDS (each polygon's events
    sorted and scanned by one workgroup; each row's toggles ranked by one
    wavefront; the distinct polygon sets collected by a hash and numbered by
    one workgroup) and global radix sorts and scans.  Every combination,
    forced through the debug switch, stores the oracle's cell sets and gives
    its aggregates with the same structures; the default takes every LDS path
    here."""
    from gen import city_polygons
    if case.startswith("city"):
        polys, eps = city_polygons(), 1000
        xy, vals = city_points(400_000)
    else:
        polys, eps = star_polygons(12, 9, 20.0, 400.0, 1500, 77), 5
        rng = np.random.default_rng(91)
        xy = rng.integers(-50, 1600, size=2 * 400_001).astype(np.int32)
        vals = rng.integers(100, 10000, size=400_001).astype(np.int64)
    kw = {"kind": "hilbert"} if case == "city_hilbert" else {}
    okw = {}
    if case == "city_centre":
        kw["centre_sampled"] = okw["centre"] = True
    if case == "city_boundary":
        kw["boundary_only"] = okw["boundary_only"] = True
    O = orc.Approx(polys, eps, **okw)
    want_c, want_s = O.aggregate(xy, vals)
    got = {}
    try:
        for off in range(8):
            assert sba.lib().sba_debug_build_paths(off) == 0
            A = sba.Approx.from_polygons(polys, eps, **kw)
            taken = sba.lib().sba_debug_last_build_paths()
            # bit 2 (row buckets) exists only on the per-polygon path; bit 4
            # (hashed set table) wherever there are polygon sets
            assert taken & 3 == {0: 3, 1: 0, 2: 1, 3: 0}[off & 3], (off, taken)
            assert bool(taken & 4) == (not off & 4 and A.info()["n_sets"] > 0), (off, taken)
            c, s = run_agg(A, xy, vals)
            np.testing.assert_array_equal(c, want_c)
            np.testing.assert_array_equal(s, want_s)
            info = A.info()
            got[off] = {k: info[k] for k in ("n_runs", "n_segments", "n_sets", "n_blocks",
                                             "n_sub", "bytes")}
            A.close()
    finally:
        sba.lib().sba_debug_build_paths(0)
    assert all(g == got[0] for g in got.values()), got


@pytest.mark.parametrize("eps", [2000, 2800, 4000, 5500, 8000])
def test_row_buckets_across_grid_heights(sba, orc, eps):
    """The toggle row buckets' offsets are scanned in chunks of 1024 rows;
    grid heights from about 700 to 2,800 rows end those chunks at different
    places.  Both LDS paths are taken and the answer is the oracle's."""
    from gen import city_polygons
    polys = city_polygons()
    xy, vals = city_points(300_000)
    want_c, want_s = orc.Approx(polys, eps).aggregate(xy, vals)
    A = sba.Approx.from_polygons(polys, eps)
    assert sba.lib().sba_debug_last_build_paths() & 3 == 3
    assert A.info()["gh"] % 1024 != 0
    c, s = run_agg(A, xy, vals)
    np.testing.assert_array_equal(c, want_c)
    np.testing.assert_array_equal(s, want_s)
    A.close()


def test_more_polygon_sets_than_the_hashed_table_takes(sba, orc):
    """500 overlapping stars at eps 5 make about 14,700 distinct polygon sets
    (at most 13 polygons on a cell), more than the one-workgroup set table
    sorts (8,192): the build finds that at its readback and takes the global
    sort instead, with the oracle's answer."""
    polys = star_polygons(500, 12, 40.0, 200.0, 2000, 5)
    eps = 5
    O = orc.Approx(polys, eps)
    rng = np.random.default_rng(55)
    n = 300_001
    xy = rng.integers(-50, 2050, size=2 * n).astype(np.int32)
    vals = rng.integers(100, 10000, size=n).astype(np.int64)
    want_c, want_s = O.aggregate(xy, vals)
    A = sba.Approx.from_polygons(polys, eps)
    assert A.info()["n_sets"] > 8192
    assert not sba.lib().sba_debug_last_build_paths() & 4
    c, s = run_agg(A, xy, vals)
    np.testing.assert_array_equal(c, want_c)
    np.testing.assert_array_equal(s, want_s)
    i0, j0, nw, nh = window_of(polys, O.s, pad=1)
    cells = [(i0 + i, j0 + j) for j in range(0, nh, 7) for i in range(0, nw, 7)]
    want = expected_sets(O, polys.n_polys, i0, j0, nw, nh)
    got = gpu_sets(A, cells)
    bad = [k for k in cells if got[k] != want[k]]
    assert not bad, (len(bad), bad[:5])
    A.close()
