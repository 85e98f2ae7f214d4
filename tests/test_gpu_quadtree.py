"""GPU parity at the quadtree workload's real shape (the analogue of
Sec. 5.1's census-block join): 40,000 jittered Voronoi cells of 32 to 675
vertices, eps = 1 m, so the Hilbert layout holds tens of millions of runs on
a 2^16 key grid (32-bit run starts) and the grid layout more than 4,096
polygons (the item probe).  Every probe path -- binary search, the learned
index, the partitioned probe, points in Hilbert order through the batch
entry point, the grid layout -- must give the oracle's per-polygon counts and
sums bit for bit on 4M mixture points, and the cell sets of a window must be
the oracle's."""
import collections

import numpy as np
import pytest

from gen import city_points, quadtree_polygons

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

EPS = 100
N = 4_000_001          # odd: the last point takes the single-point path


@pytest.fixture(scope="module")
def sba():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2010_12548_amd as m
    m.lib()
    return m


@pytest.fixture(scope="module")
def qt(orc):
    polys = quadtree_polygons()
    xy, vals = city_points(N, config=3)
    O = orc.Approx(polys, EPS)
    want = O.aggregate(xy, vals)
    return polys, xy, vals, O, want


@pytest.fixture(scope="module")
def hil(sba, qt):
    polys = qt[0]
    H = sba.Approx.from_polygons(polys, EPS, kind="hilbert", search="learned")
    yield H
    H.close()


def same(c, s, want):
    torch.cuda.synchronize()
    np.testing.assert_array_equal(c.cpu().numpy().astype(np.uint64), want[0])
    if s is not None:
        np.testing.assert_array_equal(s.cpu().numpy(), want[1])


def test_shape_of_the_workload(hil, qt):
    info = hil.info()
    assert info["n_polys"] == 40_000
    assert info["level"] == 16                    # keys below 2^32: 32-bit starts
    assert info["n_runs"] > 20_000_000
    assert info["log2_leaves"] == 16 and info["max_leaf_err"] > 0


@pytest.mark.parametrize("search", ["binary", "learned"])
def test_direct_probe(hil, qt, search):
    _, xy, vals, _, want = qt
    txy = torch.from_numpy(xy).cuda()
    c, s = hil.aggregate(txy, torch.from_numpy(vals).cuda(), search=search)
    same(c, s, want)
    c, _ = hil.aggregate(txy, None, search=search)
    same(c, None, want)


@pytest.mark.parametrize("search", ["binary", "learned"])
def test_partitioned_probe(hil, qt, search):
    _, xy, vals, _, want = qt
    c, s = hil.aggregate_partitioned(torch.from_numpy(xy).cuda(), torch.from_numpy(vals).cuda(),
                                     search=search)
    same(c, s, want)


def test_learned_index_never_falls_back(hil, qt):
    assert hil.learned_fallbacks(torch.from_numpy(qt[1]).cuda()) == (0, 0)


def test_hilbert_sorted_points_through_the_batch_entry(sba, hil, qt):
    """Points in the Hilbert order of their cells (a server's resident
    layout) answered by one persistent launch over three uneven ranges that
    share the outputs: the same sums as the points in any order."""
    _, xy, vals, _, want = qt
    info = hil.info()
    s, L = info["s"], info["level"]
    i = np.clip(xy[0::2].astype(np.int64) // s - info["gi0"], 0, (1 << L) - 1)
    j = np.clip(xy[1::2].astype(np.int64) // s - info["gj0"], 0, (1 << L) - 1)
    # the host ordering below follows the kernels' curve (checked on 2,000 cells)
    d = np.array([sba.hilbert(L, int(a), int(b)) for a, b in zip(i[:2000], j[:2000])], np.int64)
    np.testing.assert_array_equal(_hilbert_keys(L, i[:2000], j[:2000]), d)
    order = np.argsort(_hilbert_keys(L, i, j), kind="stable")
    sxy = np.ascontiguousarray(xy.reshape(-1, 2)[order].reshape(-1))
    sv = np.ascontiguousarray(vals[order])
    txy, tv = torch.from_numpy(sxy).cuda(), torch.from_numpy(sv).cuda()
    n = sv.shape[0]
    counts = torch.empty(hil.n_polys, dtype=torch.int64, device="cuda")
    sums = torch.empty_like(counts)
    cuts = [0, 1, n // 3, n]
    for search in ("binary", "learned"):
        tasks = [sba.Task(hil, txy, tv, a, b, None, counts, sums, search=search)
                 for a, b in zip(cuts[:-1], cuts[1:])]
        sba.aggregate_batch(tasks)
        same(counts, sums, want)


def _hilbert_keys(L, i, j):
    """Hilbert index of cells (i, j) on the 2^L grid, vectorised (the
    classic bit walk, level 1: (0,0) 0, (0,1) 1, (1,1) 2, (1,0) 3)."""
    i = i.astype(np.int64).copy()
    j = j.astype(np.int64).copy()
    d = np.zeros_like(i)
    n = 1 << L
    sq = n // 2
    while sq > 0:
        ri = ((i & sq) > 0).astype(np.int64)
        rj = ((j & sq) > 0).astype(np.int64)
        d += sq * sq * ((3 * ri) ^ rj)
        # rotate the quadrant
        flip = (rj == 0) & (ri == 1)
        i = np.where(flip, sq - 1 - i, i)
        j = np.where(flip, sq - 1 - j, j)
        swap = rj == 0
        i, j = np.where(swap, j, i), np.where(swap, i, j)
        sq //= 2
    return d


def test_grid_layout_item_probe(sba, qt):
    polys, xy, vals, _, want = qt
    G = sba.Approx.from_polygons(polys, EPS)
    c, s = G.aggregate(torch.from_numpy(xy).cuda(), torch.from_numpy(vals).cuda())
    same(c, s, want)
    G.close()


def test_cell_sets_of_a_window(sba, hil, qt):
    """Per-cell polygon sets of a 300 x 300-cell window in the densest part
    of the box, Hilbert and grid layouts, against the oracle's rows."""
    polys, xy, _, O, _ = qt
    s = hil.info()["s"]
    ci = np.median(xy[0::2].astype(np.int64) // s).astype(np.int64)
    cj = np.median(xy[1::2].astype(np.int64) // s).astype(np.int64)
    i0, j0, w = int(ci) - 150, int(cj) - 150, 300
    want = collections.defaultdict(list)
    P, R, X0, X1 = O.intervals()
    sel = (R >= j0) & (R < j0 + w) & (X1 > i0) & (X0 < i0 + w)
    for p, r, a, b in zip(P[sel], R[sel], X0[sel], X1[sel]):
        for i in range(max(a, i0), min(b, i0 + w)):
            want[(i, int(r))].append(int(p))
    cells = [(i0 + i, j0 + j) for j in range(w) for i in range(w)]
    ij = torch.from_numpy(np.array(cells, dtype=np.int64).reshape(-1)).cuda()
    G = sba.Approx.from_polygons(polys, EPS)
    for A in (hil, G):
        got = A.decode(A.lookup(ij).cpu().numpy())
        n_multi = 0
        for c, g in zip(cells, got):
            assert tuple(g) == tuple(sorted(want.get(c, []))), (A.kind, c)
            n_multi += len(g) > 1
        assert n_multi > 100                  # the window crosses many boundaries
    G.close()
