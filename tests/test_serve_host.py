"""Host-side logic of the serving loop (no GPU): viewport -> point ranges of
the bucketed table, memory estimates, latency summary."""
import numpy as np

import paper_2010_12548_amd.serve as serve


def _fake_server(G, cell, off, x0=0, y0=0):
    S = serve.Server.__new__(serve.Server)
    S.box = (x0, y0, G * cell)
    S.G, S.cell = G, cell
    S.bucket_off = off
    S.sets = [(None, None, None, 260, 150_000)]
    return S


def test_ranges_cover_exactly_the_touched_buckets():
    G, cell = 8, 100
    rng = np.random.default_rng(0)
    sizes = rng.integers(0, 5, size=G * G)
    off = np.r_[0, np.cumsum(sizes)]
    S = _fake_server(G, cell, off)
    for _ in range(200):
        vx, vy = rng.integers(-150, 900, size=2)
        vw = int(rng.integers(1, 500))
        q = serve.Query(int(vx), int(vy), vw, 50, 0)
        got = set()
        for a, b in S.ranges_of(q):
            got.update(range(a, b))
        want = set()
        for by in range(G):
            for bx in range(G):
                # bucket of a point is clamped into the grid, so border buckets
                # also hold everything beyond them
                lo_x = -10**9 if bx == 0 else bx * cell
                hi_x = 10**9 if bx == G - 1 else (bx + 1) * cell
                lo_y = -10**9 if by == 0 else by * cell
                hi_y = 10**9 if by == G - 1 else (by + 1) * cell
                if vx < hi_x and vx + vw > lo_x and vy < hi_y and vy + vw > lo_y:
                    b = by * G + bx
                    want.update(range(off[b], off[b + 1]))
        assert got == want
        rs = S.ranges_of(q)
        assert all(a < b for a, b in rs) and all(rs[k][1] < rs[k + 1][0] for k in range(len(rs) - 1))


def test_estimate_grows_with_resolution():
    S = _fake_server(4, 1000, np.zeros(17, np.int64))
    a = S.estimate_bytes(serve.Query(0, 0, 100_000, 1000, 0))
    b = S.estimate_bytes(serve.Query(0, 0, 100_000, 100, 0))
    assert b > a > 0


def test_latency_summary():
    rs = [serve.Result(np.zeros(1), None, float(v), 0.0, 0) for v in range(1, 101)]
    s = serve.latency_summary(rs)
    assert s["n"] == 100 and abs(s["p50_ms"] - 50.5) < 1e-9 and s["max_ms"] == 100.0
    assert 99.0 <= s["p99_ms"] <= 100.0
