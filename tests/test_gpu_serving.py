"""GPU tests of the serving pieces: clip-window builds, the batched probe
(one persistent launch over many uneven tasks) and the bucketed point table.

Every task's answer must be identical alone and in a mixed batch (tolerance
0, integer results), and equal to the oracle on the viewport's points.
"""
import numpy as np
import pytest

from gen import city_points, polygons_from_rings, star_polygons, voronoi_partition, uniform_points

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


def in_view(xy, v):
    x, y = xy[0::2].astype(np.int64), xy[1::2].astype(np.int64)
    vx, vy, vw, vh = v
    return (x >= vx) & (x < vx + vw) & (y >= vy) & (y < vy + vh)


def oracle_view(orc_A, xy, vals, v):
    m = in_view(xy, v)
    sel = np.repeat(m, 2)
    return orc_A.aggregate(xy[sel], vals[m] if vals is not None else None)


@pytest.fixture(scope="module")
def part():
    polys = voronoi_partition(60, 300_000, (3, 30), seed=13, jitter_seed=14)
    xy = uniform_points(600_000, -5000, 305_000, 15)
    vals = np.random.default_rng(16).integers(1, 10**6, size=600_000).astype(np.int64)
    return polys, xy, vals


@pytest.mark.parametrize("kind", ["grid", "hilbert"])
@pytest.mark.parametrize("win", [(50_000, 60_000, 90_000, 140_000), (-10_000, -10_000, 5_000, 5_000),
                                 (299_000, 0, 400_000, 300_000), (0, 0, 300_000, 300_000),
                                 (500_000, 500_000, 600_000, 600_000)])
def test_window_build_matches_oracle_inside(sba, orc, part, kind, win):
    polys, xy, vals = part
    eps = 300
    O = orc.Approx(polys, eps)
    x0, y0, x1, y1 = win
    v = (x0, y0, x1 - x0, y1 - y0)
    m = in_view(xy, v)
    sel = np.repeat(m, 2)
    want_c, want_s = O.aggregate(xy[sel], vals[m])
    A = sba.Approx.from_polygons(polys, eps, kind=kind, window=win)
    c, s = A.aggregate(dev(xy[sel]), dev(vals[m]))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(c.cpu().numpy().astype(np.uint64), want_c)
    np.testing.assert_array_equal(s.cpu().numpy(), want_s)


def test_batch_alone_equals_mixed_and_oracle(sba, orc, part):
    polys, xy, vals = part
    txy, tv = dev(xy), dev(vals)
    n = xy.shape[0] // 2
    rng = np.random.default_rng(7)
    handles = {
        "grid300": (sba.Approx.from_polygons(polys, 300), "binary", orc.Approx(polys, 300)),
        "hil700": (sba.Approx.from_polygons(polys, 700, kind="hilbert", search="learned",
                                            log2_leaves=10), "learned", orc.Approx(polys, 700)),
        "hil90": (sba.Approx.from_polygons(polys, 90, kind="hilbert"), "binary",
                  orc.Approx(polys, 90)),
    }
    stars = star_polygons(9, 14, 3000.0, 40000.0, 300_000, 5)
    handles["stars"] = (sba.Approx.from_polygons(stars, 2000), "binary", orc.Approx(stars, 2000))
    specs = []
    for k in range(24):
        name = list(handles)[k % len(handles)]
        lo = int(rng.integers(0, n))
        hi = int(min(n, lo + rng.integers(0, n // 3)))
        if k % 5 == 0:
            lo, hi = 0, n                     # a large task next to small ones
        if k % 7 == 3:
            hi = lo                           # an empty range
        w = int(rng.integers(1_000, 200_000))
        vx, vy = int(rng.integers(-20_000, 300_000)), int(rng.integers(-20_000, 300_000))
        view = (vx, vy, w, w) if k % 4 else (0, 0, 0, 0)
        specs.append((name, lo, hi, view, k % 3 != 0))
    # alone
    alone = []
    for name, lo, hi, view, with_vals in specs:
        A, search, _ = handles[name]
        t = sba.Task(A, txy, tv if with_vals else None, lo, hi, view, search=search)
        sba.aggregate_batch([t])
        torch.cuda.synchronize()
        alone.append((t.counts.cpu().numpy().copy(),
                      t.sums.cpu().numpy().copy() if t.sums is not None else None))
    # mixed, one launch
    tasks = []
    for name, lo, hi, view, with_vals in specs:
        A, search, _ = handles[name]
        tasks.append(sba.Task(A, txy, tv if with_vals else None, lo, hi, view, search=search))
    sba.aggregate_batch(tasks)
    torch.cuda.synchronize()
    for (name, lo, hi, view, with_vals), t, (ac, as_) in zip(specs, tasks, alone):
        np.testing.assert_array_equal(t.counts.cpu().numpy(), ac)
        if with_vals:
            np.testing.assert_array_equal(t.sums.cpu().numpy(), as_)
        # and the oracle on the same points
        O = handles[name][2]
        sub = xy[2 * lo:2 * hi]
        subv = vals[lo:hi]
        if view[2] > 0:
            m = in_view(sub, view)
            sub, subv = sub[np.repeat(m, 2)], subv[m]
        wc, ws = O.aggregate(sub, subv if with_vals else None)
        np.testing.assert_array_equal(t.counts.cpu().numpy().astype(np.uint64), wc)
        if with_vals:
            np.testing.assert_array_equal(t.sums.cpu().numpy(), ws)


def test_batch_shared_outputs_accumulate(sba, orc, part):
    polys, xy, vals = part
    txy, tv = dev(xy), dev(vals)
    n = xy.shape[0] // 2
    A = sba.Approx.from_polygons(polys, 500)
    c = torch.empty(polys.n_polys, dtype=torch.int64, device="cuda")
    s = torch.empty_like(c)
    cuts = [0, 1, 77_777, 300_001, n - 3, n]
    tasks = [sba.Task(A, txy, tv, cuts[k], cuts[k + 1], None, c, s) for k in range(len(cuts) - 1)]
    sba.aggregate_batch(tasks)
    torch.cuda.synchronize()
    wc, ws = orc.Approx(polys, 500).aggregate(xy, vals)
    np.testing.assert_array_equal(c.cpu().numpy().astype(np.uint64), wc)
    np.testing.assert_array_equal(s.cpu().numpy(), ws)


def test_batch_many_polygons_global_path(sba, orc):
    polys = voronoi_partition(5000, 2_000_000, (2, 6), seed=23, jitter_seed=24)
    xy, vals = city_points(400_000, config=5)
    xy = np.minimum(xy, 1_999_999).astype(np.int32)
    A = sba.Approx.from_polygons(polys, 2000)
    t = sba.Task(A, dev(xy), dev(vals), 0, None, (100_000, 200_000, 1_500_000, 1_700_000))
    sba.aggregate_batch([t])
    torch.cuda.synchronize()
    wc, ws = oracle_view(orc.Approx(polys, 2000), xy, vals, t.viewport)
    np.testing.assert_array_equal(t.counts.cpu().numpy().astype(np.uint64), wc)
    np.testing.assert_array_equal(t.sums.cpu().numpy(), ws)


@pytest.mark.parametrize("G,cell", [(1, 1000), (16, 20_000), (256, 1500)])
def test_bucket_points(sba, part, G, cell):
    _, xy, vals = part
    oxy, ov, off = sba.bucket_points(dev(xy), dev(vals), 0, 0, cell, G)
    torch.cuda.synchronize()
    oxy, ov, off = oxy.cpu().numpy(), ov.cpu().numpy(), off.cpu().numpy()
    n = xy.shape[0] // 2
    assert off[0] == 0 and off[-1] == n and np.all(np.diff(off) >= 0)
    bx = np.clip(np.maximum(oxy[0::2].astype(np.int64), 0) // cell, 0, G - 1)
    by = np.clip(np.maximum(oxy[1::2].astype(np.int64), 0) // cell, 0, G - 1)
    b = by * G + bx
    want = np.repeat(np.arange(G * G), np.diff(off))
    np.testing.assert_array_equal(b, want)
    # same multiset of (x, y, value) records
    a1 = np.lexsort((vals, xy[1::2], xy[0::2]))
    a2 = np.lexsort((ov, oxy[1::2], oxy[0::2]))
    np.testing.assert_array_equal(xy[0::2][a1], oxy[0::2][a2])
    np.testing.assert_array_equal(xy[1::2][a1], oxy[1::2][a2])
    np.testing.assert_array_equal(vals[a1], ov[a2])


# --------------------------------------------------------------- server

@pytest.fixture(scope="module")
def city_small():
    from gen import CITY_BOX, city_points, viewport_queries, voronoi_partition
    sets = [voronoi_partition(40, CITY_BOX, (3, 12), seed=503, jitter_seed=504),
            voronoi_partition(300, CITY_BOX, (2, 8), seed=513, jitter_seed=514)]
    xy, vals = city_points(2_000_000, config=5)
    qs = viewport_queries(48, seed=505, n_sets=len(sets))
    return sets, xy, vals, qs


def _queries(serve, qs):
    return [serve.Query(q["vx"], q["vy"], q["vw"], q["eps"], q["set"], q["agg"]) for q in qs]


def test_server_results_alone_mixed_and_oracle(sba, orc, city_small):
    from gen import CITY_BOX
    import paper_2010_12548_amd.serve as serve
    sets, xy, vals, qs = city_small
    S = serve.Server(dev(xy), dev(vals), sets, (0, 0, CITY_BOX), G=64)
    Q = _queries(serve, qs)
    try:
        alone = [S.submit(q).result(timeout=60) for q in Q]        # one at a time
        n_alone = len(S.batches)
        S.pause()                                                  # let every query get built,
        futs = [S.submit(q) for q in Q]                            # then one mixed launch
        import time
        t0 = time.time()
        while S.n_ready() < len(Q) and time.time() - t0 < 60:
            time.sleep(0.01)
        S.resume()
        mixed = [f.result(timeout=60) for f in futs]
    finally:
        S.close()
    assert all(n == 1 for n, _ in S.batches[:n_alone])
    assert S.batches[n_alone][0] == len(Q)                        # all in one batch
    for q, a, m in zip(Q, alone, mixed):
        np.testing.assert_array_equal(a.counts, m.counts)
        if q.agg == "sum":
            np.testing.assert_array_equal(a.sums, m.sums)
        else:
            assert a.sums is None and m.sums is None
    for q, r in list(zip(Q, mixed))[::4]:
        O = orc.Approx(sets[q.set_id], q.eps)
        wc, ws = oracle_view(O, xy, vals if q.agg == "sum" else None, (q.vx, q.vy, q.vw, q.vw))
        np.testing.assert_array_equal(r.counts.astype(np.uint64), wc)
        if q.agg == "sum":
            np.testing.assert_array_equal(r.sums, ws)


def test_server_admission_waits_under_small_budget(sba, city_small):
    from gen import CITY_BOX
    import paper_2010_12548_amd.serve as serve
    sets, xy, vals, qs = city_small
    Q = _queries(serve, qs[:16])
    S0 = serve.Server(dev(xy), dev(vals), sets, (0, 0, CITY_BOX), G=64)
    need = max(S0.estimate_bytes(q) for q in Q)
    S0.close()
    S = serve.Server(dev(xy), dev(vals), sets, (0, 0, CITY_BOX), G=64, mem_budget=need + 1)
    try:
        res = [f.result(timeout=120) for f in [S.submit(q) for q in Q]]
        assert S.peak_reserved <= need + 1
        assert len(res) == len(Q)
        big = serve.Query(0, 0, CITY_BOX, 2, 0, "count")            # can never fit
        with pytest.raises(serve.Rejected):
            S.submit(big).result(timeout=10)
    finally:
        S.close()
    assert S.reserved == 0


def test_memory_estimate_bounds_the_builds_of_the_query_mix(sba):
    """Admission reserves estimate_bytes(q) for a query's build: over the
    serving workload's query mix (viewports at zoom 10-18, eps one pixel,
    the 260 / 4,000 / 40,000-polygon sets) it must be at least what the
    build really holds at its peak (its temporaries and the handle, counted
    by a caller allocator)."""
    import paper_2010_12548_amd.serve as serve
    from gen import city_polygons, quadtree_polygons, seeds, viewport_queries
    sets = [city_polygons(), city_polygons(4000, (4, 40), config=5), quadtree_polygons()]
    S = serve.Server.__new__(serve.Server)
    S.sets = [(dev(p.ring_off), dev(p.vert_off), dev(p.xy), int(p.n_polys),
               int(p.xy.shape[0] // 2)) for p in sets]
    qs = viewport_queries(240, seeds(5)["queries"], n_sets=3)
    al = sba.TorchAllocator()
    worst = 0.0
    for q in qs:
        Q = serve.Query(q["vx"], q["vy"], q["vw"], q["eps"], q["set"], q["agg"])
        ro, vo, pxy, _, _ = S.sets[Q.set_id]
        al.reset_peak()
        A = sba.Approx(ro, vo, pxy, Q.eps, window=(Q.vx, Q.vy, Q.vx + Q.vw, Q.vy + Q.vw),
                       allocator=al)
        peak = al.peak_bytes
        assert A.info()["bytes"] <= al.live_bytes
        A.close()
        est = S.estimate_bytes(Q)
        assert est >= peak, (q, est, peak)
        worst = max(worst, peak / est)
    assert al.live_bytes == 0
    assert worst > 0.05            # the estimate is not vacuous
