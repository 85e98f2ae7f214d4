"""GPU parity of the polygon-polygon join over cells (Sec. 4: blend of two
rasterized canvases, mask of the cells that hold a polygon of each,
aggregate per pair): the pairs and their shared cell counts must equal the
oracle's, exactly and in (p, q) order."""
import numpy as np
import pytest

from gen import star_polygons, voronoi_partition

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sba():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2010_12548_amd as m
    m.lib()
    return m


def gpu_join(sba, a, b, eps, **kw):
    g = sba.key_grid_for(eps, a, b)
    A = sba.Approx.from_polygons(a, eps, kind="hilbert", key_grid=g, **kw)
    B = sba.Approx.from_polygons(b, eps, kind="hilbert", key_grid=g, **kw)
    pa, pb, cells = sba.join_pairs(A, B)
    torch.cuda.synchronize()
    return pa.cpu().numpy(), pb.cpu().numpy(), cells.cpu().numpy()


def check(sba, orc, a, b, eps, mode=None):
    okw = {mode: True} if mode else {}
    gkw = {"centre": {"centre_sampled": True}, "boundary_only": {"boundary_only": True}}.get(mode, {})
    want = orc.join_pairs(orc.Approx(a, eps, **okw), orc.Approx(b, eps, **okw))
    got = gpu_join(sba, a, b, eps, **gkw)
    for w, g in zip(want, got):
        np.testing.assert_array_equal(g, w)
    return want


@pytest.mark.parametrize("mode", [None, "centre", "boundary_only"])
@pytest.mark.parametrize("eps", [2, 4, 7, 13, 40])
def test_random_stars(sba, orc, eps, mode):
    a = star_polygons(6, 9, 5.0, 120.0, 400, 4100 + eps)
    b = star_polygons(7, 7, 5.0, 100.0, 400, 5100 + eps)
    want = check(sba, orc, a, b, eps, mode)
    assert want[0].size > 0


def test_self_join_partition(sba, orc):
    polys = voronoi_partition(40, 200_000, (3, 25), seed=3, jitter_seed=4)
    for eps in (60, 700):
        pa, pb, cells = check(sba, orc, polys, polys, eps)
        assert np.all(np.isin(np.arange(polys.n_polys), pa[pa == pb]))   # the diagonal


def test_many_polygons_against_stars(sba, orc):
    a = voronoi_partition(6000, 1_000_000, (2, 6), seed=31, jitter_seed=32)
    b = star_polygons(12, 11, 2000.0, 90000.0, 1_000_000, 77)
    check(sba, orc, a, b, 300)
    check(sba, orc, b, a, 3000)


def test_city_self_join(sba, orc):
    from gen import city_polygons
    polys = city_polygons()
    check(sba, orc, polys, polys, 10000)


def test_capacity_and_rejects(sba, orc):
    a = star_polygons(6, 9, 5.0, 120.0, 400, 4107)
    b = star_polygons(7, 7, 5.0, 100.0, 400, 5107)
    eps = 7
    want = orc.join_pairs(orc.Approx(a, eps), orc.Approx(b, eps))
    g = sba.key_grid_for(eps, a, b)
    A = sba.Approx.from_polygons(a, eps, kind="hilbert", key_grid=g)
    B = sba.Approx.from_polygons(b, eps, kind="hilbert", key_grid=g)
    import ctypes as C
    n = C.c_int64(0)
    k = 3
    pa = torch.full((k,), -1, dtype=torch.int32, device="cuda")
    pb = torch.full((k,), -1, dtype=torch.int32, device="cuda")
    cells = torch.full((k,), -1, dtype=torch.int64, device="cuda")
    rc = sba.lib().sba_join_pairs(A._h, B._h, k, pa.data_ptr(), pb.data_ptr(), cells.data_ptr(),
                                  C.byref(n), None)
    assert rc == 0 and n.value == want[0].size > k
    np.testing.assert_array_equal(pa.cpu().numpy(), want[0][:k])
    np.testing.assert_array_equal(cells.cpu().numpy(), want[2][:k])
    # different eps, different key grid, grid layout
    other_eps = sba.Approx.from_polygons(b, 9, kind="hilbert", key_grid=g)
    own_grid = sba.Approx.from_polygons(b, eps, kind="hilbert")
    grid = sba.Approx.from_polygons(b, eps)
    for X in (other_eps, grid):
        with pytest.raises(sba.SbaError):
            sba.join_pairs(A, X)
    info = own_grid.info()
    if (info["level"], info["gi0"], info["gj0"]) != g:
        with pytest.raises(sba.SbaError):
            sba.join_pairs(A, own_grid)


def test_join_with_empty_sets(sba, orc):
    from gen import polygons_from_rings
    a = star_polygons(6, 9, 5.0, 120.0, 400, 4107)
    empty = polygons_from_rings([])
    far = polygons_from_rings([[np.array([[10**6, 10**6], [10**6 + 50, 10**6], [10**6, 10**6 + 50]])]])
    eps = 7
    g = sba.key_grid_for(eps, a)
    A = sba.Approx.from_polygons(a, eps, kind="hilbert", key_grid=g)
    E = sba.Approx.from_polygons(empty, eps, kind="hilbert", key_grid=g)
    F = sba.Approx.from_polygons(far, eps, kind="hilbert", key_grid=g)   # no cell in the grid
    for X in (E, F):
        pa, pb, cells = sba.join_pairs(A, X)
        assert pa.numel() == 0 and pb.numel() == 0 and cells.numel() == 0
