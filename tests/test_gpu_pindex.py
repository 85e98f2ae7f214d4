"""GPU parity of the point index (point-side pre-aggregation, Sec. 3 point
indexing): per-polygon COUNT and SUM answered from the sorted cell keys of
the points, their prefix sums and the runs of a Hilbert handle built on the
index's key grid, with binary searches and with the RadixSpline.  The answer
must equal the oracle's aggregate over the same points bit for bit (it is the
same quantity: the points whose cell lies in each approximation)."""
import numpy as np
import pytest

from gen import city_points, polygons_from_rings, star_polygons, uniform_points, voronoi_partition

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


def pindex_agg(ix, A, search, with_values=True):
    c, s = ix.aggregate(A, search=search, with_values=with_values)
    torch.cuda.synchronize()
    return c.cpu().numpy().astype(np.uint64), (s.cpu().numpy() if s is not None else None)


def check_index(sba, orc, polys, xy, vals, eps, searches=("binary", "learned"), **ix_kw):
    O = orc.Approx(polys, eps)
    want_c, want_s = O.aggregate(xy, vals)
    ix = sba.PointIndex(dev(xy), dev(vals) if vals is not None else None, eps, **ix_kw)
    A = sba.Approx.from_polygons(polys, eps, kind="hilbert", key_grid=ix)
    info = A.info()
    lvl, i0, j0 = ix.key_grid()
    if info["n_runs"]:
        assert (info["level"], info["gi0"], info["gj0"]) == (lvl, i0, j0)
    for search in searches:
        c, s = pindex_agg(ix, A, search, with_values=vals is not None)
        np.testing.assert_array_equal(c, want_c)
        if vals is not None:
            np.testing.assert_array_equal(s, want_s)
        c, _ = pindex_agg(ix, A, search, with_values=False)
        np.testing.assert_array_equal(c, want_c)
    return ix, A


@pytest.mark.parametrize("eps", [3, 10, 60, 700, 6000])
def test_partition_binary_and_spline(sba, orc, eps):
    polys = voronoi_partition(40, 200_000, (3, 25), seed=3, jitter_seed=4)
    xy = uniform_points(400_001, -1000, 201_000, 77)
    vals = np.random.default_rng(1).integers(-10**6, 10**7, size=400_001).astype(np.int64)
    check_index(sba, orc, polys, xy, vals, eps)


@pytest.mark.parametrize("seed,eps", [(0, 4), (1, 9), (2, 30)])
def test_overlapping_stars_sets(sba, orc, seed, eps):
    """Overlapping polygons: runs whose code is a polygon set add their
    count and sum to every member."""
    polys = star_polygons(12, 9, 20.0, 400.0, 1500, 300 + seed)
    rng = np.random.default_rng(seed)
    n = 150_001
    xy = rng.integers(-100, 1600, size=2 * n).astype(np.int32)
    vals = rng.integers(0, 10000, size=n).astype(np.int64)
    _, A = check_index(sba, orc, polys, xy, vals, eps)
    assert A.info()["n_sets"] > 0


@pytest.mark.parametrize("radix_bits,spline_err", [(1, 1), (4, 2), (12, 8), (24, 32), (20, 1000)])
def test_spline_parameters(sba, orc, radix_bits, spline_err):
    """Any radix table size and error bound gives the same answer; heavy
    duplicates (points clustered in few cells) exercise the flat steps."""
    polys = voronoi_partition(30, 100_000, (3, 20), seed=5, jitter_seed=6)
    rng = np.random.default_rng(radix_bits)
    n = 200_000
    centres = rng.integers(0, 100_000, size=(20, 2))
    pick = rng.integers(0, 20, size=n)
    pts = centres[pick] + rng.integers(-300, 300, size=(n, 2))
    xy = pts.astype(np.int32).reshape(-1)
    vals = rng.integers(1, 1000, size=n).astype(np.int64)
    ix, _ = check_index(sba, orc, polys, xy, vals, 50, radix_bits=radix_bits,
                        spline_err=spline_err)
    inf = ix.info()
    assert inf["spline_err"] == spline_err
    assert inf["radix_bits"] == min(radix_bits, 2 * inf["key_level"])
    assert 2 <= inf["n_knots"] <= 2 * inf["n_distinct"] + 2


def test_key_grid_cuts_polygons(sba, orc):
    """Points cover only part of the polygons: the handle on the index's key
    grid drops the cells outside the grid, keeps the oracle's cell sets inside
    it, and the scan over its cells and the index both give the oracle's
    answer."""
    polys = voronoi_partition(25, 100_000, (3, 20), seed=8, jitter_seed=9)
    eps = 40
    xy = uniform_points(100_000, 30_000, 70_000, 12)
    vals = np.random.default_rng(3).integers(0, 100, size=100_000).astype(np.int64)
    ix, A = check_index(sba, orc, polys, xy, vals, eps)
    c, s = A.aggregate(dev(xy), dev(vals))
    want_c, want_s = orc.Approx(polys, eps).aggregate(xy, vals)
    np.testing.assert_array_equal(c.cpu().numpy().astype(np.uint64), want_c)
    np.testing.assert_array_equal(s.cpu().numpy(), want_s)
    # cell sets on a sample of cells inside and around the key grid
    O = orc.Approx(polys, eps)
    lvl, i0, j0 = ix.key_grid()
    side = 1 << lvl
    rng = np.random.default_rng(4)
    ij = np.stack([rng.integers(i0 - 50, i0 + side + 50, size=20000),
                   rng.integers(j0 - 50, j0 + side + 50, size=20000)], axis=1)
    P, R, X0, X1 = (np.asarray(a) for a in O.intervals())
    order = np.argsort(R, kind="stable")
    P, R, X0, X1 = P[order], R[order], X0[order], X1[order]
    got = A.decode(A.lookup(dev(ij.reshape(-1))).cpu().numpy())
    for (i, j), g in zip(ij.tolist(), got):
        inside = i0 <= i < i0 + side and j0 <= j < j0 + side
        a, b = np.searchsorted(R, j, "left"), np.searchsorted(R, j, "right")
        hit = (X0[a:b] <= i) & (i < X1[a:b])
        want = tuple(sorted(int(p) for p in P[a:b][hit])) if inside else ()
        assert tuple(sorted(g)) == want, (i, j, g, want)


def test_many_polygons(sba, orc):
    polys = voronoi_partition(6000, 1_000_000, (2, 6), seed=31, jitter_seed=32)
    xy = uniform_points(600_001, -2000, 1_002_000, 5)
    vals = np.random.default_rng(2).integers(0, 10**6, size=600_001).astype(np.int64)
    check_index(sba, orc, polys, xy, vals, 300)


def test_city_partition(sba, orc):
    from gen import city_polygons
    polys = city_polygons()
    xy, vals = city_points(2_000_000)
    for eps in (1000, 10000):
        check_index(sba, orc, polys, xy, vals, eps)


def test_edge_cases(sba, orc):
    polys = star_polygons(5, 9, 20.0, 200.0, 800, 7)
    eps = 6
    # one point; points all in one cell; no values
    for xy in (np.array([400, 400], np.int32), np.tile(np.array([401, 399], np.int32), 1001)):
        vals = np.arange(xy.size // 2, dtype=np.int64) - 7
        check_index(sba, orc, polys, xy, vals, eps)
        check_index(sba, orc, polys, xy, None, eps)
    # empty index: zero outputs from any handle on its grid
    ix = sba.PointIndex(torch.zeros(0, dtype=torch.int32, device="cuda"), None, eps)
    A = sba.Approx.from_polygons(polys, eps, kind="hilbert", key_grid=ix)
    c, _ = pindex_agg(ix, A, "binary", with_values=False)
    assert c.shape[0] == polys.n_polys and not c.any()
    # a handle with no cell in the key grid: zeros
    far = polygons_from_rings([[np.array([[10**6, 10**6], [10**6 + 50, 10**6], [10**6, 10**6 + 50]])]])
    xy = uniform_points(1000, 0, 800, 3)
    ix = sba.PointIndex(dev(xy), dev(np.ones(1000, np.int64)), eps)
    B = sba.Approx.from_polygons(far, eps, kind="hilbert", key_grid=ix)
    c, s = pindex_agg(ix, B, "learned")
    assert not c.any() and not s.any()


def test_rejects_mismatched_handles(sba):
    polys = star_polygons(5, 9, 20.0, 200.0, 800, 7)
    xy = uniform_points(5000, 0, 800, 3)
    ix = sba.PointIndex(dev(xy), None, 6)
    own_grid = sba.Approx.from_polygons(polys, 6, kind="hilbert")
    other_eps = sba.Approx.from_polygons(polys, 9, kind="hilbert", key_grid=ix)
    grid = sba.Approx.from_polygons(polys, 6)
    for A in (other_eps, grid):
        with pytest.raises(sba.SbaError):
            ix.aggregate(A, with_values=False)
    if own_grid.info()["gi0"] != ix.key_grid()[1] or own_grid.info()["level"] != ix.key_grid()[0]:
        with pytest.raises(sba.SbaError):
            ix.aggregate(own_grid, with_values=False)
    with pytest.raises(sba.SbaError):           # sums from an index without values
        ix.aggregate(sba.Approx.from_polygons(polys, 6, kind="hilbert", key_grid=ix),
                     with_values=True)
    with pytest.raises(sba.SbaError):           # key grid on the grid layout
        sba.Approx.from_polygons(polys, 6, key_grid=ix)
    for bad in ({"radix_bits": 29}, {"spline_err": -1}):
        with pytest.raises(sba.SbaError):
            sba.PointIndex(dev(xy), None, 6, **bad)


@pytest.mark.parametrize("eps,radix_bits,spline_err", [(6, 20, 32), (6, 6, 4), (50, 2, 1),
                                                       (50, 24, 64)])
def test_spline_error_bound(sba, orc, eps, radix_bits, spline_err):
    """Lower bounds of keys present, absent, at both ends and in between
    equal numpy's over the points' keys (from the oracle's Hilbert index),
    and no RadixSpline window ever fails its check (the error bound holds at
    every key, not only the stored ones)."""
    rng = np.random.default_rng(eps + radix_bits)
    n = 20_000
    centres = rng.integers(0, 3000, size=(8, 2))
    pts = np.concatenate([centres[rng.integers(0, 8, size=n // 2)]
                          + rng.integers(-40, 40, size=(n // 2, 2)),
                          rng.integers(0, 3000, size=(n - n // 2, 2))]).astype(np.int32)
    ix = sba.PointIndex(dev(pts.reshape(-1)), None, eps, radix_bits=radix_bits,
                        spline_err=spline_err)
    L, i0, j0 = ix.key_grid()
    s = ix.info()["s"]
    keys = np.sort(np.array([orc.hilbert_d(L, x // s - i0, y // s - j0) for x, y in pts.tolist()],
                            dtype=np.uint64))
    total = 1 << (2 * L)
    q = np.concatenate([keys, keys + 1, np.maximum(keys, 1) - 1,
                        rng.integers(0, total + 1, size=20_000, dtype=np.uint64),
                        np.array([0, 1, total - 1, total], np.uint64)]).astype(np.int64)
    want = np.searchsorted(keys, q.astype(np.uint64), side="left")
    for search in ("binary", "learned"):
        got, fb = ix.lower_bounds(dev(q), search)
        np.testing.assert_array_equal(got.cpu().numpy(), want)
        assert fb == 0


@pytest.mark.parametrize("eps", [4, 40])
def test_centre_sampled_handle(sba, orc, eps):
    """The point index answers a centre-sampled Hilbert handle on its key grid
    like the oracle's centre-sampled aggregate."""
    polys = star_polygons(12, 9, 20.0, 400.0, 1500, 303)
    rng = np.random.default_rng(eps)
    n = 150_001
    xy = rng.integers(-100, 1600, size=2 * n).astype(np.int32)
    vals = rng.integers(0, 10000, size=n).astype(np.int64)
    want_c, want_s = orc.Approx(polys, eps, centre=True).aggregate(xy, vals)
    ix = sba.PointIndex(dev(xy), dev(vals), eps)
    A = sba.Approx.from_polygons(polys, eps, kind="hilbert", key_grid=ix, centre_sampled=True)
    for search in ("binary", "learned"):
        c, s = pindex_agg(ix, A, search)
        np.testing.assert_array_equal(c, want_c)
        np.testing.assert_array_equal(s, want_s)
