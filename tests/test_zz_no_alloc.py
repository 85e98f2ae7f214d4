"""The batch entry point that allocates nothing (sba_aggregate_batch_noalloc):
its scratch lives in the library's fixed device array, and its results must
equal sba_aggregate_batch's, call after call, whatever the previous call left
in the array (a large batch, then a smaller one); a batch too large for the
array is refused with SBA_ELIMIT before anything runs."""
import numpy as np
import pytest

from gen import uniform_points, voronoi_partition

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SBA_ELIMIT = -5


@pytest.fixture(scope="module")
def sba():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2010_12548_amd as m
    m.lib()
    return m


@pytest.fixture(scope="module")
def data(sba):
    polys = voronoi_partition(50, 400_000, (3, 20), seed=41, jitter_seed=42)
    n = 1_500_001
    xy = uniform_points(n, -3000, 403_000, 43)
    vals = np.random.default_rng(44).integers(-10**6, 10**6, size=n).astype(np.int64)
    txy = torch.from_numpy(xy).cuda()
    tv = torch.from_numpy(vals).cuda()
    handles = [sba.Approx.from_polygons(polys, 400),
               sba.Approx.from_polygons(polys, 250, kind="hilbert", search="learned",
                                        log2_leaves=10),
               sba.Approx.from_polygons(polys, 900, kind="hilbert")]
    return polys, txy, tv, handles


def make_tasks(sba, txy, tv, handles, ranges, views, searches):
    tasks = []
    for k, ((lo, hi), view, search) in enumerate(zip(ranges, views, searches)):
        A = handles[k % len(handles)]
        counts = torch.full((A.n_polys,), -7, dtype=torch.int64, device="cuda")
        sums = torch.full((A.n_polys,), -7, dtype=torch.int64, device="cuda") if k % 3 else None
        tasks.append(sba.Task(A, txy, tv if sums is not None else None, lo, hi, view, counts, sums,
                              search=search if A.search == "learned" else "binary"))
    return tasks


def results(tasks):
    torch.cuda.synchronize()
    return [(t.counts.cpu().numpy().copy(), None if t.sums is None else t.sums.cpu().numpy().copy())
            for t in tasks]


def run_both(sba, txy, tv, handles, ranges, views, searches):
    a = make_tasks(sba, txy, tv, handles, ranges, views, searches)
    b = make_tasks(sba, txy, tv, handles, ranges, views, searches)
    sba.aggregate_batch(a)
    sba.aggregate_batch(b, no_alloc=True)
    ra, rb = results(a), results(b)
    for (ca, sa), (cb, sb) in zip(ra, rb):
        np.testing.assert_array_equal(cb, ca)
        if sa is not None:
            np.testing.assert_array_equal(sb, sa)
    return ra


def test_noalloc_batch_equals_allocating_batch_twice(sba, data):
    _, txy, tv, handles = data
    n = tv.numel()
    rng = np.random.default_rng(5)
    # a large batch: uneven ranges (several items each), viewports, both searches
    cuts = np.sort(rng.integers(0, n, size=23))
    ranges = [(0, n)] + [(int(a), int(b)) for a, b in zip(cuts[:-1], cuts[1:])] + [(n - 1, n)]
    views = [None if k % 2 else (int(rng.integers(0, 300_000)), int(rng.integers(0, 300_000)),
                                 int(rng.integers(1000, 150_000)), int(rng.integers(1000, 150_000)))
             for k in range(len(ranges))]
    searches = ["learned" if k % 2 else "binary" for k in range(len(ranges))]
    first = run_both(sba, txy, tv, handles, ranges, views, searches)
    assert any(c.sum() > 0 for c, _ in first)
    # then a smaller one: fewer tasks, shorter ranges; nothing of the first
    # batch's scratch may leak into it
    ranges2 = [(5, 300_005), (1_000_000, 1_000_000), (7, 8)]
    views2 = [None, None, (0, 0, 10**6, 10**6)]
    run_both(sba, txy, tv, handles, ranges2, views2, ["binary", "learned", "binary"])


def test_noalloc_batch_refuses_more_than_its_array(sba, data):
    _, txy, tv, handles = data
    A = handles[0]
    one = [sba.Task(A, txy, None, 0, 0, None)]
    b1 = sba.batch_scratch_bytes(one)
    per = sba.batch_scratch_bytes(one * 2) - b1
    cap = sba.batch_noalloc_bytes()
    k = (cap - b1) // per + 2
    counts = torch.full((A.n_polys,), -7, dtype=torch.int64, device="cuda")
    tasks = [sba.Task(A, txy, None, 0, 0, None, counts)] * k
    assert sba.batch_scratch_bytes(tasks) > cap
    with pytest.raises(sba.SbaError) as e:
        sba.aggregate_batch(tasks, no_alloc=True)
    assert e.value.code == SBA_ELIMIT
    torch.cuda.synchronize()
    assert int((counts != -7).sum().item()) == 0          # nothing ran
    # and the entry point still answers afterwards
    run_both(sba, txy, tv, handles, [(0, 1000), (2000, 900_000)], [None, None],
             ["binary", "learned"])
