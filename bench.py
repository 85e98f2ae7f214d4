"""Benchmark of the distance-bounded approximate aggregation join on one MI355X.

A step is one pass of the whole hot path over one batch of points already
resident in HBM: build the eps-approximation of every polygon
(sba_build_approx: boundary strips, scanline crossings, row sweep, set table,
cell layout) and answer the per-polygon COUNT and SUM of all points from it
(sba_aggregate).  Prints one JSON line.

Default run, in one process:

* city scale (the line's value): 100M points from a 50-component Gaussian
  mixture in a 40 km x 40 km box at 1 cm units, lognormal cents, 260 jittered
  Voronoi polygons, eps = 10 m; build + probe steps, the probe's roofline,
  the oracle on the host as the CPU baseline (all cores and one thread, and
  the exact crossing-number join as context);
* quadtree (the ``quadtree`` object): 1e9 points of the same mixture, 40,000
  jittered Voronoi polygons, eps = 1 m, Hilbert runs; binary search against
  the learned index for points as generated, partitioned by the call, and in
  Hilbert order; a 1e8-point sample compared with the oracle;
* serving (the ``serving`` object): 1e9 resident points, three polygon sets
  (260 / 4,000 / 40,000), viewport queries at zoom 10-18 with eps = one
  pixel; capacity, then Poisson arrivals at 0.5 / 0.8 / 0.95 of it.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "points/s + HBM GB/s, eps-bounded agg join; learned vs binary probe; p99 query ms"
HBM_PEAK_GBS = 8000.0
PROBE_SRC = os.path.join(ROOT, "paper_2010_12548_amd", "csrc", "probe.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def probe_source_sha() -> str:
    with open(PROBE_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


# HBM bytes per launch of the probe, from rocprofv3 counter runs (FETCH_SIZE
# and WRITE_SIZE per dispatch, KiB, each scaled by what the counter reads for
# a device copy of known size), keyed by the workload and by the hash of the
# probe kernels' source the counters were taken on: any change to that source
# makes the entry stale, and the line then reports null.
TRAFFIC = {
    # profiles/city_eps10m_probe_counters.md: FETCH_SIZE 898,833 KiB and
    # WRITE_SIZE 1,040 KiB per dispatch (mean of 6); the 1 GiB copy read
    # 524,320 / wrote 1,048,576 KiB (factors 1.99988 and 1.0)
    ("city", 1000, 100_000_000, "k_probe_grid16<true, 2, 2, 1024>", "60bed7791b6fc4ec"):
        {"fetch_bytes": 1840697637, "write_bytes": 1064960},
}


def traffic_of(workload, eps, n, kernel):
    t = TRAFFIC.get((workload, int(eps), int(n), kernel, probe_source_sha()))
    return None if t is None else t["fetch_bytes"] + t["write_bytes"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="city", choices=["city", "tiny", "quadtree", "serve"])
    ap.add_argument("--queries", type=int, default=2000, help="serving: queries per load phase")
    ap.add_argument("--batch-rounds", type=int, default=0,
                    help="serving: instead of the load phases, time the batch probe alone: per "
                         "round, build --queries queries with the server paused, then run "
                         "their batches")
    ap.add_argument("--points", type=int, default=0, help="0 = the workload's size")
    ap.add_argument("--qt-points", type=int, default=1_000_000_000,
                    help="points of the quadtree and serving parts of the default run")
    ap.add_argument("--eps", type=int, default=0, help="0 = the workload's default")
    ap.add_argument("--layout", default="", choices=["", "grid", "hilbert"])
    ap.add_argument("--search", default="", choices=["", "binary", "learned"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baselines")
    ap.add_argument("--no-sweep", action="store_true", help="skip the eps sweep")
    ap.add_argument("--no-quadtree", action="store_true", help="city: skip the quadtree part")
    ap.add_argument("--no-serve", action="store_true", help="city: skip the serving part")
    ap.add_argument("--no-extras", action="store_true",
                    help="city: skip result range, centre-sampled cells, polygon join, point index")
    ap.add_argument("--overlap", action="store_true",
                    help="also time the steps with builds and probes on two streams (step "
                         "k+1's build beside step k's probe), reported separately")
    ap.add_argument("--no-pindex", action="store_true",
                    help="skip the point-index (pre-aggregated points) measurement")
    ap.add_argument("--blocks-per-cu", type=int, default=0)
    ap.add_argument("--grid16-per-cu", type=int, default=0,
                    help="cap on workgroups per CU of the LDS-directory grid probe (0 = none)")
    ap.add_argument("--log2-leaves", type=int, default=20,
                    help="learned index leaves (log2); 2^20 keeps the quadtree leaves' error "
                         "below 56 runs (2^16: 238)")
    ap.add_argument("--tile-log2", type=int, default=0, help="grid tile side log2 (0 = auto)")
    ap.add_argument("--sub-log2", type=int, default=0, help="grid sub-tile side log2 (0 = auto)")
    ap.add_argument("--force-wide", action="store_true",
                    help="grid probe: 32-bit directory in global memory instead of the LDS copy")
    ap.add_argument("--probe-only", action="store_true",
                    help="build once, then run only --steps aggregate calls (for counter runs)")
    ap.add_argument("--copy-gib", type=float, default=0.0,
                    help="with --probe-only: first run a device-to-device copy of this many GiB "
                         "(calibrates the memory counters against a kernel of known traffic)")
    return ap.parse_args()


def timed(torch, fn, reps):
    """Mean ms of fn() over reps calls between two events on the current stream."""
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def stream_read_rate(sba, torch, txy, tv, reps):
    """The yardstick beside the peak: the read rate of the library's plain
    streaming-read kernel (16-byte non-temporal loads, XOR-folded, nothing
    written) over the probe's own inputs (x, y and values: the same bytes in
    the same place, both streams in one launch), best over a few launch
    shapes."""
    out = torch.empty(1, dtype=torch.int32, device=txy.device)
    nbytes = txy.numel() * txy.element_size() + tv.numel() * tv.element_size()
    best = None
    for blocks, threads in ((256, 512), (256, 1024), (512, 512), (1024, 256), (2048, 256)):
        def run():
            sba.stream_read(txy, tv, blocks=blocks, threads=threads, out=out)
        run()
        ms = timed(torch, run, reps)
        gbps = nbytes / (ms * 1e-3) / 1e9
        if best is None or gbps > best["gbps"]:
            best = {"gbps": gbps, "ms": ms, "blocks": blocks, "threads": threads,
                    "bytes": nbytes, "kernel": "k_stream_read"}
    log(f"[bench] streaming read of the probe's inputs: {json.dumps(best)}")
    return best


def same_result(cc, ss, res_c, res_s):
    return bool(np.array_equal(cc.cpu().numpy().astype(np.uint64), res_c)
                and np.array_equal(ss.cpu().numpy(), res_s))


def probe_only(args, sba, torch, txy, tv, ro, vo, pxy, eps, layout, search, n):
    if args.copy_gib > 0:
        nb = int(args.copy_gib * 2**30)
        src = torch.empty(nb, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        src.fill_(1)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy: {nb} bytes read, {nb} bytes written")
        del src, dst
    a = sba.Approx(ro, vo, pxy, eps, kind=layout, search=search, log2_leaves=args.log2_leaves,
                   tile_log2=args.tile_log2, sub_log2=args.sub_log2)
    counts = torch.empty(a.n_polys, dtype=torch.int64, device="cuda")
    sums = torch.empty(a.n_polys, dtype=torch.int64, device="cuda")
    for _ in range(args.warmup):
        a.aggregate(txy, tv, counts, sums)
    torch.cuda.synchronize()
    t = timed(torch, lambda: a.aggregate(txy, tv, counts, sums), args.steps)
    info = a.info()
    log(f"[bench] probe-only: {args.steps} calls, {t:.4f} ms per call, "
        f"{16.0 * n / (t * 1e-3) / 1e9:.1f} GB/s algorithmic; kernel {a.probe_kernel(True)}; "
        f"probe source {probe_source_sha()}; approx {json.dumps(info)}")
    a.close()


# ------------------------------------------------------------------ serving

def serve_batches_only(torch, txy, tv, n_queries, rounds, sets):
    """The batch probe without the builds beside it: per round the server
    builds the approximations of n_queries queries while paused, then runs
    their batches; points scanned per second over the batch phases."""
    import paper_2010_12548_amd.serve as serve
    from gen import CITY_BOX, seeds, viewport_queries
    qs = viewport_queries(n_queries * rounds + 64, seeds(5)["queries"], n_sets=len(sets))
    Q = [serve.Query(q["vx"], q["vy"], q["vw"], q["eps"], q["set"], q["agg"]) for q in qs]
    S = serve.Server(txy, tv, sets, (0, 0, CITY_BOX), G=256)
    out = {"rounds": []}
    try:
        [f.result() for f in [S.submit(q) for q in Q[-64:]]]
        t_all, p_all = 0.0, 0
        for r in range(rounds):
            S.pause()
            futs = [S.submit(q) for q in Q[r * n_queries:(r + 1) * n_queries]]
            t_wait = time.perf_counter()
            while S.n_ready() < n_queries and time.perf_counter() - t_wait < 60:
                time.sleep(0.005)
            ready = S.n_ready()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            S.resume()
            res = [f.result() for f in futs]
            dt = time.perf_counter() - t0
            pts = sum(x.points_scanned for x in res)
            t_all += dt
            p_all += pts
            row = {"queries": n_queries, "built_before_batches": ready,
                   "queries_per_s": n_queries / dt, "points_per_s": pts / dt}
            out["rounds"].append(row)
            log(f"[bench] serve batches only: {json.dumps(row)}")
        out["points_per_s"] = p_all / t_all
    finally:
        S.close()
    return out


def serve_bench(torch, txy, tv, n_queries, sets):
    """Viewport-query serving on the resident points: capacity (closed loop),
    then Poisson arrivals at 0.5 / 0.8 / 0.95 of it; p50 / p99 latency from
    arrival to result on the host.  Every load phase replays the same queries
    with the same arrival pattern, scaled to its rate, so that the phases
    differ in load only (not in their mix of cheap and costly viewports)."""
    import paper_2010_12548_amd.serve as serve
    from gen import CITY_BOX, seeds, viewport_queries
    qs = viewport_queries(4 * n_queries + 64, seeds(5)["queries"], n_sets=len(sets))
    Q = [serve.Query(q["vx"], q["vy"], q["vw"], q["eps"], q["set"], q["agg"]) for q in qs]
    S = serve.Server(txy, tv, sets, (0, 0, CITY_BOX), G=256)
    out = {"points": int(txy.numel() // 2), "polygon_sets": [p.n_polys for p in sets],
           "bucket_prep_ms": round(S.prep_ms, 2), "mem_budget_bytes": S.budget,
           "queries_per_phase": n_queries}
    try:
        # warm-up, then capacity with everything submitted at once
        [f.result() for f in [S.submit(q) for q in Q[-64:]]]
        phase = Q[:n_queries]
        t1 = time.perf_counter()
        res = [f.result() for f in [S.submit(q) for q in phase]]
        wall = time.perf_counter() - t1
        cap = len(phase) / wall
        out["closed_loop"] = {"queries_per_s": cap, **serve.latency_summary(res),
                              "mean_build_ms": float(np.mean([r.build_ms for r in res])),
                              "mean_points": float(np.mean([r.points_scanned for r in res]))}
        log(f"[bench] serve closed loop: {json.dumps(out['closed_loop'])}")
        rng = np.random.default_rng(seeds(5)["queries"] + 1)
        out["open_loop"] = []
        qs_k = Q[n_queries:2 * n_queries]
        unit_gaps = rng.exponential(1.0, size=len(qs_k))
        for frac in (0.5, 0.8, 0.95):
            lam = frac * cap
            gaps = unit_gaps / lam
            futs = []
            t_start = time.perf_counter()
            due = t_start
            for q, g in zip(qs_k, gaps):
                due += g
                while True:
                    now = time.perf_counter()
                    if now >= due:
                        break
                    time.sleep(min(0.0005, due - now))
                futs.append(S.submit(q))
            res = [f.result() for f in futs]
            wall = time.perf_counter() - t_start
            row = {"load": frac, "arrival_rate": lam, "queries_per_s": len(res) / wall,
                   **serve.latency_summary(res)}
            out["open_loop"].append(row)
            log(f"[bench] serve open loop: {json.dumps(row)}")
        # each result identical alone and in the mix
        probe = Q[:48]
        mixed = [f.result() for f in [S.submit(q) for q in probe]]
        alone = [S.submit(q).result() for q in probe]
        same = all(np.array_equal(a.counts, m.counts) and
                   (a.sums is None or np.array_equal(a.sums, m.sums)) for a, m in zip(alone, mixed))
        out["alone_equals_mixed"] = bool(same)
        out["max_batch_queries"] = max(b for b, _ in S.batches)
        out["peak_reserved_bytes"] = S.peak_reserved
    finally:
        S.close()
    out["p50_ms_closed_loop"] = out["closed_loop"]["p50_ms"]
    out["p99_ms_by_load"] = {str(r["load"]): r["p99_ms"] for r in out["open_loop"]}
    return out


# ------------------------------------------------------------------ quadtree

def hilbert_sorted(torch, txy, tv, info):
    """The points reordered by the Hilbert index of their cell on the handle's
    key grid (input preparation for a comparison run, in torch)."""
    L, s = info["level"], info["s"]
    x = txy[0::2].to(torch.int64) - info["gi0"] * s
    y = txy[1::2].to(torch.int64) - info["gj0"] * s
    top = (1 << L) - 1
    i = torch.clamp(torch.div(x, s, rounding_mode="floor"), 0, top)
    j = torch.clamp(torch.div(y, s, rounding_mode="floor"), 0, top)
    del x, y
    d = torch.zeros_like(i)
    swap = torch.zeros_like(i)
    flip = torch.zeros_like(i)
    for lev in range(L - 1, -1, -1):
        bi = (i >> lev) & 1
        bj = (j >> lev) & 1
        xx = torch.where(swap == 1, bj, bi) ^ flip
        yy = torch.where(swap == 1, bi, bj) ^ flip
        d = (d << 2) | ((3 * xx) ^ yy)
        low = yy == 0
        flip = torch.where(low & (xx == 1), flip ^ 1, flip)
        swap = torch.where(low, swap ^ 1, swap)
    del i, j, swap, flip
    order = torch.argsort(d)
    del d
    sx = txy.view(-1, 2)[order].reshape(-1).contiguous()
    sv = tv[order].contiguous()
    return sx, sv


def quadtree_bench(args, sba, torch, n, polys, xy, vals, eps=100, cpu=True):
    """Config 3/4: the Hilbert-run layout of 40,000 polygons at 1 m probed by
    binary search and by the learned index over the same handle, for points
    as generated, partitioned by the call, and in Hilbert order."""
    dev = torch.device("cuda:0")
    txy = torch.from_numpy(xy).to(dev)
    tv = torch.from_numpy(vals).to(dev)
    ro = torch.from_numpy(polys.ring_off).to(dev)
    vo = torch.from_numpy(polys.vert_off).to(dev)
    pxy = torch.from_numpy(polys.xy).to(dev)
    alg_bytes = 16.0 * n
    builds = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        a = sba.Approx(ro, vo, pxy, eps, kind="hilbert", search="learned",
                       log2_leaves=args.log2_leaves)
        builds.append(1000.0 * (time.perf_counter() - t0))
        if len(builds) < 3:
            a.close()
    ai = a.info()
    out = {"workload": (f"quadtree: {n} Gaussian-mixture points, {polys.n_polys} jittered Voronoi "
                        f"polygons, eps={eps / 100:g} m, Hilbert runs"),
           "points": n, "polygons": polys.n_polys, "eps_units": eps, "n_runs": ai["n_runs"],
           "level": ai["level"], "leaves": 1 << ai["log2_leaves"],
           "max_leaf_err": ai["max_leaf_err"], "mean_leaf_err": ai["mean_leaf_err"],
           "build_ms_median": round(float(np.median(builds)), 3),
           "approx_MB": round(ai["bytes"] / 2**20, 1), "kernel_learned": a.probe_kernel(True)}
    np_ = max(a.n_polys, 1)
    cc = torch.empty(np_, dtype=torch.int64, device=dev)
    ss = torch.empty_like(cc)

    def row(t):
        return {"probe_ms": round(t, 4), "points_per_s": n / (t * 1e-3),
                "gbps": round(alg_bytes / (t * 1e-3) / 1e9, 1)}

    direct, res = {}, {}
    for srch in ("binary", "learned"):
        for _ in range(2):
            a.aggregate(txy, tv, cc, ss, search=srch)
        torch.cuda.synchronize()
        direct[srch] = row(timed(torch, lambda: a.aggregate(txy, tv, cc, ss, search=srch), 5))
        res[srch] = (cc.cpu().numpy().astype(np.uint64), ss.cpu().numpy())
    res_c, res_s = res["binary"]
    identical = bool(np.array_equal(res["learned"][0], res_c)
                     and np.array_equal(res["learned"][1], res_s))
    fb, mm = a.learned_fallbacks(txy)
    out["direct"] = direct
    log(f"[bench] quadtree direct: {json.dumps(direct)}")
    # points partitioned into coarse Hilbert regions by the call itself
    scratch = torch.empty(a.scratch_bytes(n), dtype=torch.uint8, device=dev)
    part = {}
    for srch in ("binary", "learned"):
        a.aggregate_partitioned(txy, tv, cc, ss, search=srch, scratch=scratch)
        torch.cuda.synchronize()
        part[srch] = row(timed(torch, lambda: a.aggregate_partitioned(
            txy, tv, cc, ss, search=srch, scratch=scratch), 3))
        part[srch]["same_as_direct"] = same_result(cc, ss, res_c, res_s)
    del scratch
    out["partitioned"] = part
    log(f"[bench] quadtree partitioned: {json.dumps(part)}")
    # the same points in the Hilbert order of their cells (a resident layout
    # a serving system keeps): neighbouring lookups share cache lines
    sx, sv = hilbert_sorted(torch, txy, tv, ai)
    srt = {}
    for srch in ("binary", "learned"):
        a.aggregate(sx, sv, cc, ss, search=srch)
        torch.cuda.synchronize()
        srt[srch] = row(timed(torch, lambda: a.aggregate(sx, sv, cc, ss, search=srch), 3))
        srt[srch]["same_as_direct"] = same_result(cc, ss, res_c, res_s)
        task = sba.Task(a, sx, sv, 0, n, None, cc, ss, search=srch)
        sba.aggregate_batch([task])
        torch.cuda.synchronize()
        tb = timed(torch, lambda: sba.aggregate_batch([task]), 3)
        srt[srch]["batch_probe_ms"] = round(tb, 4)
        srt[srch]["batch_same"] = same_result(cc, ss, res_c, res_s)
    del sx, sv
    out["hilbert_sorted"] = srt
    log(f"[bench] quadtree sorted: {json.dumps(srt)}")
    out["identical"] = bool(identical and all(v["same_as_direct"] for v in part.values())
                            and all(v["same_as_direct"] and v["batch_same"] for v in srt.values()))
    out["fallbacks"] = fb
    out["learned_ne_binary"] = mm
    out["learned_speedup"] = {
        "direct": round(direct["binary"]["probe_ms"] / direct["learned"]["probe_ms"], 3),
        "partitioned": round(part["binary"]["probe_ms"] / part["learned"]["probe_ms"], 3),
        "hilbert_sorted": round(srt["binary"]["probe_ms"] / srt["learned"]["probe_ms"], 3)}
    # a sample of the points against the oracle (the same approximation,
    # built and probed on the host)
    if cpu:
        import oracle
        m = min(n, 100_000_000)
        t0 = time.perf_counter()
        O = oracle.Approx(polys, eps)
        tb = time.perf_counter() - t0
        t0 = time.perf_counter()
        oc, os_ = O.aggregate(xy[:2 * m], vals[:m])
        ta = time.perf_counter() - t0
        c2, s2 = a.aggregate(txy[:2 * m], tv[:m], search="learned")
        out["oracle_sample"] = {"points": m, "matches_gpu": same_result(c2, s2, oc, os_),
                                "oracle_build_s": round(tb, 3), "oracle_aggregate_s": round(ta, 3),
                                "oracle_points_per_s": m / ta, "cores": int(O.threads_used)}
        log(f"[bench] quadtree oracle sample: {json.dumps(out['oracle_sample'])}")
    # the polygon-polygon join of this set with the city set (Sec. 4)
    from gen import city_polygons
    out["polygon_join"] = join_bench(sba, torch, polys, city_polygons(), eps,
                                     "40,000-cell partition with the 260-cell partition")
    if not args.no_pindex:
        scan = direct["learned"]["probe_ms"]
        out["point_index"] = pindex_bench(sba, torch, txy, tv, ro, vo, pxy, eps, res_c, res_s, scan)
    a.close()
    return out


# ------------------------------------------------------------------ city extras

def pindex_bench(sba, torch, txy, tv, ro, vo, pxy, eps, res_c, res_s, scan_ms):
    """Point-side pre-aggregation (Sec. 3, point indexing): build the point
    index once, then answer the same query from the runs of a Hilbert handle
    on the index's key grid with binary searches and with the RadixSpline.
    The answer must equal the scan's."""
    n = txy.numel() // 2
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ix = sba.PointIndex(txy, tv, eps)
    t_ix = 1000.0 * (time.perf_counter() - t0)
    t0 = time.perf_counter()
    a = sba.Approx(ro, vo, pxy, eps, kind="hilbert", key_grid=ix)
    t_h = 1000.0 * (time.perf_counter() - t0)
    ii, ai = ix.info(), a.info()
    out = {"index_build_ms": round(t_ix, 3), "handle_build_ms": round(t_h, 3),
           "n_runs": ai["n_runs"], "key_level": ii["key_level"], "n_distinct": ii["n_distinct"],
           "n_knots": ii["n_knots"], "radix_bits": ii["radix_bits"],
           "spline_err": ii["spline_err"], "index_MB": round(ii["bytes"] / 2**20, 1),
           "scan_probe_ms": round(scan_ms, 4)}
    counts = torch.empty(max(a.n_polys, 1), dtype=torch.int64, device=txy.device)
    sums = torch.empty_like(counts)
    for srch in ("binary", "learned"):
        for _ in range(2):
            ix.aggregate(a, srch, counts, sums)
        torch.cuda.synchronize()
        t = timed(torch, lambda: ix.aggregate(a, srch, counts, sums), 10)
        same = same_result(counts[:a.n_polys], sums[:a.n_polys], res_c, res_s)
        out[srch] = {"query_ms": round(t, 4), "points_per_s_equiv": n / (t * 1e-3),
                     "speedup_vs_scan": round(scan_ms / t, 2), "same_as_scan": same}
    a.close()
    ix.close()
    log(f"[bench] point index: {json.dumps(out)}")
    return out


def join_bench(sba, torch, a, b, eps, desc):
    """Polygon-polygon join over cells (Sec. 4): both sets as Hilbert runs on
    one key grid, then sba_join_pairs (synchronous) timed end to end."""
    g = sba.key_grid_for(eps, a, b)
    t0 = time.perf_counter()
    A = sba.Approx.from_polygons(a, eps, kind="hilbert", key_grid=g)
    B = sba.Approx.from_polygons(b, eps, kind="hilbert", key_grid=g)
    t_build = 1000.0 * (time.perf_counter() - t0)
    sba.join_pairs(A, B)
    ts = []
    for _ in range(5):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pa, pb, cells = sba.join_pairs(A, B)
        ts.append(1000.0 * (time.perf_counter() - t0))
    out = {"what": desc, "eps_units": eps, "runs": [A.info()["n_runs"], B.info()["n_runs"]],
           "builds_ms": round(t_build, 3), "join_ms_median": round(float(np.median(ts)), 3),
           "pairs": int(pa.numel()), "shared_cells": int(cells.sum().item())}
    A.close()
    B.close()
    log(f"[bench] polygon join: {json.dumps(out)}")
    return out


def city_extras(args, sba, torch, txy, tv, ro, vo, pxy, eps, info, kw, counts, sums, res_c,
                res_s, polys, probe_avg, n):
    extra = {}
    # result range [alpha - beta, alpha] (Sec. 6): beta from a boundary-only
    # approximation over the same points
    t0 = time.perf_counter()
    bh = sba.Approx(ro, vo, pxy, eps, boundary_only=True, tile_log2=info["tile_log2"],
                    sub_log2=info["sub_log2"])
    t_bb = 1000.0 * (time.perf_counter() - t0)
    bc = torch.empty_like(counts)
    bs = torch.empty_like(sums)
    bh.aggregate(txy, tv, bc, bs)
    torch.cuda.synchronize()
    beta_probe = timed(torch, lambda: bh.aggregate(txy, tv, bc, bs), 10)
    beta = bc.cpu().numpy().astype(np.float64)
    alpha = res_c.astype(np.float64)
    a_full = sba.Approx(ro, vo, pxy, eps, **kw)
    rr = sba.aggregate_range(a_full, bh, txy, tv)
    torch.cuda.synchronize()
    one_pass = timed(torch, lambda: sba.aggregate_range(a_full, bh, txy, tv), 10)
    rr = sba.aggregate_range(a_full, bh, txy, tv)
    same = bool(np.array_equal(rr[0].cpu().numpy().astype(np.uint64), res_c)
                and np.array_equal(rr[2].cpu().numpy(), bc.cpu().numpy()))
    extra["result_range"] = {
        "beta_build_ms": round(t_bb, 3), "beta_probe_ms": round(beta_probe, 4),
        "alpha_plus_beta_one_pass_ms": round(one_pass, 4),
        "one_pass_kernel": sba.range_kernel(a_full, bh), "one_pass_same_as_two": same,
        "beta_over_alpha_total": float(beta.sum() / max(alpha.sum(), 1.0)),
        "beta_over_alpha_median_polygon": float(np.median(beta / np.maximum(alpha, 1.0))),
        "kernel": bh.probe_kernel(True)}
    a_full.close()
    bh.close()
    log(f"[bench] result range: {json.dumps(extra['result_range'])}")
    # the non-conservative approximation (cells whose centre is inside)
    t0 = time.perf_counter()
    ch = sba.Approx(ro, vo, pxy, eps, centre_sampled=True, tile_log2=args.tile_log2,
                    sub_log2=args.sub_log2)
    t_cb = 1000.0 * (time.perf_counter() - t0)
    cc = torch.empty_like(counts)
    cs = torch.empty_like(sums)
    ch.aggregate(txy, tv, cc, cs)
    torch.cuda.synchronize()
    t_cp = timed(torch, lambda: ch.aggregate(txy, tv, cc, cs), 10)
    extra["centre_sampled"] = {
        "build_ms": round(t_cb, 3), "probe_ms": round(t_cp, 4),
        "counted_over_points": int(cc.sum().item()) / n,
        "conservative_counted_over_points": float(res_c.sum()) / n,
        "kernel": ch.probe_kernel(True)}
    ch.close()
    log(f"[bench] centre-sampled: {json.dumps(extra['centre_sampled'])}")
    extra["polygon_join"] = join_bench(sba, torch, polys, polys, eps, "city partition with itself")
    if not args.no_pindex:
        extra["point_index"] = pindex_bench(sba, torch, txy, tv, ro, vo, pxy, eps, res_c, res_s,
                                            probe_avg)
    return extra


def eps_sweep(sba, torch, txy, tv, ro, vo, pxy, counts, sums, n):
    sweep = {}
    for e in (100, 1000, 10000):
        a = sba.Approx(ro, vo, pxy, e, kind="grid")
        for _ in range(2):
            a.aggregate(txy, tv, counts, sums)
        torch.cuda.synchronize()
        t = timed(torch, lambda: a.aggregate(txy, tv, counts, sums), 10)
        ai = a.info()
        sweep[f"{e / 100:g}m"] = {"probe_ms": round(t, 4), "probe_points_per_s": n / (t * 1e-3),
                                  "probe_gbps": round(16.0 * n / (t * 1e-3) / 1e9, 1),
                                  "build_ms": round(ai["build_ms"], 3),
                                  "tile": 1 << ai["tile_log2"], "sub": 1 << ai["sub_log2"],
                                  "blocks": ai["n_blocks"], "approx_MB": round(ai["bytes"] / 2**20, 2),
                                  "kernel": a.probe_kernel(True)}
        a.close()
    log(f"[bench] eps sweep: {json.dumps(sweep)}")
    return sweep


def cpu_baselines(polys, xy, vals, eps, n, res_c, res_s, compare):
    """The oracle on the host: the same approximate join on all cores (the
    baseline), on one thread, and the exact crossing-number join as context."""
    import oracle
    t0 = time.perf_counter()
    O = oracle.Approx(polys, eps)
    tb = time.perf_counter() - t0
    t0 = time.perf_counter()
    oc, os_ = O.aggregate(xy, vals)
    ta = time.perf_counter() - t0
    cores = int(O.threads_used)
    cpu = {"value": n / (tb + ta), "unit": "points/s", "cores": cores, "kind": "oracle",
           "sample": (f"oracle build of all {polys.n_polys} polygons ({tb:.2f}s) + oracle "
                      f"aggregate of all {n} points ({ta:.2f}s) on {cores} threads")}
    if compare:
        cpu["matches_gpu"] = bool(np.array_equal(oc, res_c) and np.array_equal(os_, res_s))
    m1 = min(n, 30_000_000)
    t0 = time.perf_counter()
    O.aggregate(xy[:2 * m1], vals[:m1], nthreads=1)
    t1 = time.perf_counter() - t0
    cpu["single_thread"] = {"value": m1 / (t1 + tb), "unit": "points/s", "cores": 1,
                            "sample": f"oracle aggregate of the first {m1} points ({t1:.2f}s) "
                                      f"on one thread, plus the build"}
    me = min(n, 20_000_000)
    t0 = time.perf_counter()
    O.exact(xy[:2 * me], vals[:me])
    te = time.perf_counter() - t0
    cpu["exact_join"] = {"value": me / te, "unit": "points/s", "cores": int(O.threads_used),
                         "sample": f"exact crossing-number join (bounding-box filter, then "
                                   f"point-in-polygon) of the first {me} points ({te:.2f}s)"}
    log(f"[bench] cpu oracle: {json.dumps(cpu)}")
    return cpu


# ------------------------------------------------------------------ main

def workload(args):
    from gen import city_points, city_polygons, quadtree_polygons, tiny_workload
    if args.workload == "tiny":
        n = args.points or 1_000_000
        xy, vals, polys = tiny_workload(n)
        eps = args.eps or 64
        desc = (f"tiny: {n} uniform points in [0,65536)^2, uniform cents, 16 star polygons of "
                f"32 vertices, eps={eps} units")
        return xy, vals, polys, eps, desc, "grid"
    if args.workload == "city":
        n = args.points or 100_000_000
        polys = city_polygons()
        xy, vals = city_points(n)
        eps = args.eps or 1000
        desc = (f"city: {n} Gaussian-mixture points (50 comps, sigma 200-3000 m) in 40x40 km at "
                f"1 cm, lognormal(7,0.8) cents, 260 jittered Voronoi polygons, eps={eps / 100:g} m")
        return xy, vals, polys, eps, desc, "grid"
    n = args.points or 1_000_000_000
    polys = quadtree_polygons()
    xy, vals = city_points(n, config=3)
    eps = args.eps or 100
    desc = (f"quadtree: {n} Gaussian-mixture points, 40,000 jittered Voronoi polygons, "
            f"eps={eps / 100:g} m, Hilbert runs")
    return xy, vals, polys, eps, desc, "hilbert"


def serving_part(args, torch, qt_polys=None):
    """Config 5 on its own 1e9 resident points (freed afterwards)."""
    from gen import city_points, city_polygons, quadtree_polygons
    t0 = time.time()
    n = args.points if args.workload == "serve" and args.points else args.qt_points
    xy, vals = city_points(n, config=5)
    sets = [city_polygons(), city_polygons(4000, (4, 40), config=5),
            qt_polys if qt_polys is not None else quadtree_polygons()]
    log(f"[bench] serve: {n} points, polygon sets {[p.n_polys for p in sets]} in "
        f"{time.time() - t0:.1f}s")
    txy = torch.from_numpy(xy).cuda()
    tv = torch.from_numpy(vals).cuda()
    del xy, vals
    if args.batch_rounds:
        res = serve_batches_only(torch, txy, tv, args.queries, args.batch_rounds, sets)
    else:
        res = serve_bench(torch, txy, tv, args.queries, sets)
    del txy, tv
    torch.cuda.empty_cache()
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the per-polygon partial results would be combined by one all-reduce; "
              "not built)", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2010_12548_amd as sba

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.blocks_per_cu:
        sba.lib().sba_debug_set_blocks_per_cu(args.blocks_per_cu)
    if args.grid16_per_cu:
        sba.lib().sba_debug_set_grid16_per_cu(args.grid16_per_cu)
    if args.force_wide:
        sba.lib().sba_debug_force_wide_grid(1)
    dev = torch.device("cuda:0")
    t_start = time.time()

    if args.workload == "serve":
        res = serving_part(args, torch)
        if args.batch_rounds:
            print(json.dumps({"metric": "serving batch probe points/s", "value": res["points_per_s"],
                              "unit": "points/s", "n_gpus": 1, "higher_is_better": True,
                              "scaling": "weak", "vs_baseline": None, "dtype": "int64",
                              "data": "synthetic",
                              "config": {"workload": "serve: batches of paused queries"},
                              "serving": res}), flush=True)
            return
        cl = res["closed_loop"]
        print(json.dumps({"metric": METRIC, "value": cl["queries_per_s"], "unit": "queries/s",
                          "n_gpus": 1, "higher_is_better": True, "scaling": "weak",
                          "vs_baseline": None, "dtype": "int64", "data": "synthetic",
                          "config": {"workload": "serve: 1e9 resident points, 3 polygon sets, "
                                                 "viewport queries at zoom 10-18"},
                          "serving": res}), flush=True)
        return

    xy, vals, polys, eps, desc, layout = workload(args)
    layout = args.layout or layout
    search = args.search or ("learned" if layout == "hilbert" else "binary")
    n = xy.shape[0] // 2
    log(f"[bench] workload ready in {time.time() - t_start:.1f}s: {desc}")
    txy = torch.from_numpy(xy).to(dev)
    tv = torch.from_numpy(vals).to(dev)
    ro = torch.from_numpy(polys.ring_off).to(dev)
    vo = torch.from_numpy(polys.vert_off).to(dev)
    pxy = torch.from_numpy(polys.xy).to(dev)
    counts = torch.empty(polys.n_polys, dtype=torch.int64, device=dev)
    sums = torch.empty(polys.n_polys, dtype=torch.int64, device=dev)
    torch.cuda.synchronize()
    kw = dict(kind=layout, search=search, log2_leaves=args.log2_leaves, tile_log2=args.tile_log2,
              sub_log2=args.sub_log2)
    if args.probe_only:
        probe_only(args, sba, torch, txy, tv, ro, vo, pxy, eps, layout, search, n)
        return

    # A step builds the approximation and probes every point with it, both
    # on the current stream.  --overlap also times the same steps with the
    # builds on one stream and the probes on another and reports that
    # figure separately.
    import contextlib
    bstream = pstream = None

    def step(ev=None):
        a = sba.Approx(ro, vo, pxy, eps, stream=bstream, **kw)   # returns complete
        with (torch.cuda.stream(pstream) if pstream is not None else contextlib.nullcontext()):
            if ev is not None:
                ev[0].record()
            a.aggregate(txy, tv, counts, sums, stream=pstream)
            if ev is not None:
                ev[1].record()
        return a

    def timed_steps(k_steps):
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(k_steps)]
        hs = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(k_steps):
            a = step(evs[k])
            if pstream is None and hs:
                # on one stream the build just made has synchronised it, so
                # the previous step's probe is done: its approximation goes
                # back to the library's memory cache for the next build
                hs[-1].close(sync=False)
            hs.append(a)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, evs, hs

    for _ in range(args.warmup):
        step().close()
    torch.cuda.synchronize()
    t_total, evs, handles = timed_steps(args.steps)
    probe_ms = [e0.elapsed_time(e1) for e0, e1 in evs]
    info = handles[-1].info()
    kernel = handles[-1].probe_kernel(True)
    ms_step = 1000.0 * t_total / args.steps
    ms_step_overlap = None
    if args.overlap:
        bstream, pstream = torch.cuda.Stream(), torch.cuda.Stream()
        t_ov, _, hs = timed_steps(args.steps)
        ms_step_overlap = 1000.0 * t_ov / args.steps
        for h in hs:
            h.close()
        bstream = pstream = None
    probe_in_step = float(np.mean(probe_ms))
    alg_bytes = 16.0 * n          # 8 B x,y + 8 B value per point
    # the probe kernel's own time: back-to-back calls on the current stream
    # between one pair of events (each call: a zeroing kernel of the outputs,
    # a few microseconds, and the probe kernel)
    last = handles[-1]
    probe_avg = timed(torch, lambda: last.aggregate(txy, tv, counts, sums), max(args.steps, 10))
    achieved = alg_bytes / (probe_avg * 1e-3) / 1e9
    read_rate = stream_read_rate(sba, torch, txy, tv, max(args.steps, 10))
    # build time on its own
    iso = []
    for _ in range(5):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        a = sba.Approx(ro, vo, pxy, eps, **kw)
        iso.append(1000.0 * (time.perf_counter() - t0))
        a.close()
    build_iso = float(np.median(iso))
    ser = f" (two streams: {ms_step_overlap:.3f} ms/step)" if ms_step_overlap else ""
    log(f"[bench] {args.steps} steps: {ms_step:.3f} ms/step{ser}, probe in step "
        f"{probe_in_step:.4f} ms, probe back-to-back {probe_avg:.4f} ms, build alone median "
        f"{build_iso:.3f} ms, kernel {kernel}")
    for h in handles:
        h.close()
    res_c = counts.cpu().numpy().astype(np.uint64)
    res_s = sums.cpu().numpy()

    extra = {}
    if args.workload == "city" and not args.no_extras:
        extra.update(city_extras(args, sba, torch, txy, tv, ro, vo, pxy, eps, info, kw, counts,
                                 sums, res_c, res_s, polys, probe_avg, n))
    sweep = None
    if args.workload == "city" and not args.no_sweep:
        sweep = eps_sweep(sba, torch, txy, tv, ro, vo, pxy, counts, sums, n)
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baselines(polys, xy, vals, eps, n, res_c, res_s, compare=layout == "grid")
    del txy, tv
    torch.cuda.empty_cache()

    quad = None
    qt_polys = None
    if args.workload == "quadtree":
        quad = quadtree_bench(args, sba, torch, n, polys, xy, vals, eps=eps, cpu=not args.no_cpu)
    elif args.workload == "city" and not args.no_quadtree:
        from gen import city_points, quadtree_polygons
        t0 = time.time()
        qt_polys = quadtree_polygons()
        qxy, qvals = city_points(args.qt_points, config=3)
        log(f"[bench] quadtree workload ready in {time.time() - t0:.1f}s")
        quad = quadtree_bench(args, sba, torch, args.qt_points, qt_polys, qxy, qvals,
                              cpu=not args.no_cpu)
        del qxy, qvals
    torch.cuda.empty_cache()
    serving = None
    if args.workload == "city" and not args.no_serve:
        serving = serving_part(args, torch, qt_polys)

    line = {
        "metric": METRIC,
        "value": n / (ms_step * 1e-3),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "ms_per_step_overlapped": ms_step_overlap,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic (seeded generators stand in for the NYC taxi / census data)",
        "config": {"workload": desc, "points": n, "polygons": polys.n_polys, "eps_units": eps,
                   "layout": layout, "search": search if layout == "hilbert" else None,
                   "step": "sba_build_approx + sba_aggregate (COUNT+SUM)",
                   "streams": "one"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic_of(args.workload, eps, n, kernel),
                     "kernel": kernel, "probe_source": probe_source_sha(),
                     "algorithmic_bytes_per_launch": alg_bytes,
                     "read_stream": read_rate,
                     "frac_of_read_stream": achieved / read_rate["gbps"]},
        "cpu_baseline": cpu,
        "probe_ms": probe_avg,
        "probe_ms_in_step": probe_in_step,
        "probe_points_per_s": n / (probe_avg * 1e-3),
        "build_ms_median": build_iso,
        "approx": {k: info[k] for k in ("s", "gw", "gh", "tile_log2", "sub_log2", "n_tiles",
                                        "n_blocks", "n_sub", "n_sets", "n_segments",
                                        "n_boundary", "n_runs", "bytes")},
        "eps_sweep": sweep,
        "quadtree": quad,
        "serving": serving,
        "bench_wall_s": round(time.time() - t_start, 1),
        **extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
