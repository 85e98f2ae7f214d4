"""Benchmark of the distance-bounded approximate aggregation join on one MI355X.

A step is one pass of the whole hot path over one batch of points already
resident in HBM: build the eps-approximation of every polygon
(sba_build_approx: boundary strips, scanline crossings, row sweep, set table,
cell layout) and answer the per-polygon COUNT and SUM of all points from it
(sba_aggregate).  Prints one JSON line.

Default workload (city scale): 100M points from a 50-component Gaussian
mixture in a 40 km x 40 km box at 1 cm units, lognormal cents, 260 jittered
Voronoi polygons, eps = 10 m.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "points/s + HBM GB/s, eps-bounded agg join; learned vs binary probe; p99 query ms"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# HBM bytes per launch of the probe, from rocprofv3 counter runs of this
# kernel version (FETCH_SIZE and WRITE_SIZE per dispatch, KiB, each scaled by
# what the counter reads for a device copy of known size); keyed by the
# workload it was taken on.  Re-measure after any change to the kernel.
TRAFFIC = {
    # profiles/city_eps10m_probe_counters.md: FETCH_SIZE 800568.97 KiB (x 1.99993: a 1 GiB
    # device copy reads 524306.5 KiB), WRITE_SIZE 2080 KiB (x 1.00000)
    ("city", 1000, 100_000_000, "k_probe_grid16<true, true, 2, 512>"):
        {"fetch_bytes": 1639507396, "write_bytes": 2129920},
}


def traffic_of(workload, eps, n, kernel):
    t = TRAFFIC.get((workload, int(eps), int(n), kernel))
    return None if t is None else t["fetch_bytes"] + t["write_bytes"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="city", choices=["city", "tiny", "quadtree", "serve"])
    ap.add_argument("--queries", type=int, default=300, help="serve: queries per phase")
    ap.add_argument("--serve", action="store_true",
                    help="city: also run the viewport-query server on the resident points")
    ap.add_argument("--points", type=int, default=0, help="0 = the workload's size")
    ap.add_argument("--eps", type=int, default=0, help="0 = the workload's default")
    ap.add_argument("--layout", default="", choices=["", "grid", "hilbert"])
    ap.add_argument("--search", default="", choices=["", "binary", "learned"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-sweep", action="store_true", help="skip the eps sweep")
    ap.add_argument("--overlap", action="store_true",
                    help="also time the steps with builds and probes on two streams (step "
                         "k+1's build beside step k's probe), reported separately")
    ap.add_argument("--no-pindex", action="store_true",
                    help="skip the point-index (pre-aggregated points) measurement")
    ap.add_argument("--blocks-per-cu", type=int, default=0)
    ap.add_argument("--grid16-per-cu", type=int, default=0,
                    help="cap on workgroups per CU of the LDS-directory grid probe (0 = none)")
    ap.add_argument("--log2-leaves", type=int, default=16, help="learned index leaves (log2)")
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
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        a.aggregate(txy, tv, counts, sums)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / args.steps
    info = a.info()
    log(f"[bench] probe-only: {args.steps} calls, {t:.4f} ms per call, "
        f"{16.0 * n / (t * 1e-3) / 1e9:.1f} GB/s algorithmic; approx {json.dumps(info)}")
    a.close()


def serve_bench(args, torch, txy, tv, n_queries, with_big_set=True):
    """Viewport-query serving on the resident points: capacity (closed loop),
    then Poisson arrivals at 0.5 / 0.8 / 0.95 of it; p50 / p99 latency from
    arrival to result on the host."""
    import paper_2010_12548_amd.serve as serve
    from gen import CITY_BOX, city_polygons, quadtree_polygons, seeds, viewport_queries
    t0 = time.time()
    sets = [city_polygons(), city_polygons(4000, (4, 40), config=5)]
    if with_big_set:
        sets.append(quadtree_polygons())
    log(f"[bench] serve: polygon sets {[p.n_polys for p in sets]} in {time.time() - t0:.1f}s")
    qs = viewport_queries(4 * n_queries, seeds(5)["queries"], n_sets=len(sets))
    Q = [serve.Query(q["vx"], q["vy"], q["vw"], q["eps"], q["set"], q["agg"]) for q in qs]
    S = serve.Server(txy, tv, sets, (0, 0, CITY_BOX), G=256, mem_budget=16 << 30)
    out = {"points": int(txy.numel() // 2), "polygon_sets": [p.n_polys for p in sets],
           "bucket_prep_ms": round(S.prep_ms, 2)}
    try:
        # warm-up, then capacity with everything submitted at once
        [f.result() for f in [S.submit(q) for q in Q[:32]]]
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
        for k, frac in enumerate((0.5, 0.8, 0.95)):
            lam = frac * cap
            qs_k = Q[n_queries * (k + 1):n_queries * (k + 2)]
            gaps = rng.exponential(1.0 / lam, size=len(qs_k))
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
        probe = Q[:24]
        mixed = [f.result() for f in [S.submit(q) for q in probe]]
        alone = [S.submit(q).result() for q in probe]
        same = all(np.array_equal(a.counts, m.counts) and
                   (a.sums is None or np.array_equal(a.sums, m.sums)) for a, m in zip(alone, mixed))
        out["alone_equals_mixed"] = bool(same)
        out["max_batch_queries"] = max(b for b, _ in S.batches)
        out["peak_reserved_bytes"] = S.peak_reserved
    finally:
        S.close()
    return out


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
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 10
        e0.record()
        for _ in range(reps):
            ix.aggregate(a, srch, counts, sums)
        e1.record()
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) / reps
        same = bool(np.array_equal(counts[:a.n_polys].cpu().numpy().astype(np.uint64), res_c)
                    and np.array_equal(sums[:a.n_polys].cpu().numpy(), res_s))
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
    if args.workload == "serve":
        n = args.points or 1_000_000_000
        xy, vals = city_points(n, config=5)
        desc = (f"serve: {n} resident Gaussian-mixture points, polygon sets of 260 / 4,000 / "
                f"40,000 jittered Voronoi cells, viewport queries at zoom 10-18 with eps = one "
                f"pixel, Poisson arrivals")
        return xy, vals, None, 0, desc, "grid"
    n = args.points or 1_000_000_000
    polys = quadtree_polygons()
    xy, vals = city_points(n, config=3)
    eps = args.eps or 100
    desc = (f"quadtree: {n} Gaussian-mixture points, 40,000 jittered Voronoi polygons, "
            f"eps={eps / 100:g} m, Hilbert runs")
    return xy, vals, polys, eps, desc, "hilbert"


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
    t0 = time.time()
    xy, vals, polys, eps, desc, layout = workload(args)
    layout = args.layout or layout
    search = args.search or ("learned" if layout == "hilbert" else "binary")
    n = xy.shape[0] // 2
    log(f"[bench] workload ready in {time.time() - t0:.1f}s: {desc}")
    txy = torch.from_numpy(xy).to(dev)
    tv = torch.from_numpy(vals).to(dev)
    if args.workload == "serve":
        del xy, vals
        res = serve_bench(args, torch, txy, tv, args.queries)
        cl = res["closed_loop"]
        p99 = max(r["p99_ms"] for r in res["open_loop"])
        print(json.dumps({"metric": METRIC, "value": cl["queries_per_s"], "unit": "queries/s",
                          "n_gpus": 1, "higher_is_better": True, "scaling": "weak",
                          "vs_baseline": None, "dtype": "int64", "data": "synthetic",
                          "config": {"workload": desc}, "p99_ms_worst_open_loop": p99,
                          "serving": res}), flush=True)
        return
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
    # builds on one stream and the probes on another (the build of step k+1,
    # host-bound, beside the probe of step k, bound by HBM bandwidth; every
    # step still does its whole build and its whole probe) and reports that
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
            hs.append(step(evs[k]))
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
    # between one pair of events (the per-step events above also hold the
    # launch gaps of a step); each call is a zeroing kernel of the outputs
    # (a few microseconds) and the probe kernel
    last = handles[-1]
    reps = max(args.steps, 10)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        last.aggregate(txy, tv, counts, sums)
    e1.record()
    torch.cuda.synchronize()
    probe_avg = e0.elapsed_time(e1) / reps
    achieved = alg_bytes / (probe_avg * 1e-3) / 1e9
    # build time on its own (in a one-stream step loop a build's first wait
    # also covers the previous step's probe)
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
        f"{build_iso:.3f} ms")

    for h in handles:
        h.close()
    res_c = counts.cpu().numpy().astype(np.uint64)
    res_s = sums.cpu().numpy()

    extra = {}
    if layout == "hilbert":
        # binary and learned probe on the same handle, identical results required
        a = sba.Approx(ro, vo, pxy, eps, kind="hilbert", search="learned",
                       log2_leaves=args.log2_leaves)
        out = {}
        for srch in ("binary", "learned"):
            cc = torch.empty_like(counts)
            ss = torch.empty_like(sums)
            for _ in range(2):
                a.aggregate(txy, tv, cc, ss, search=srch)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            reps = 5
            e0.record()
            for _ in range(reps):
                a.aggregate(txy, tv, cc, ss, search=srch)
            e1.record()
            torch.cuda.synchronize()
            t = e0.elapsed_time(e1) / reps
            out[srch] = {"probe_ms": round(t, 4), "points_per_s": n / (t * 1e-3),
                         "gbps": alg_bytes / (t * 1e-3) / 1e9,
                         "_res": (cc.cpu().numpy(), ss.cpu().numpy())}
        same = (np.array_equal(out["binary"]["_res"][0], out["learned"]["_res"][0])
                and np.array_equal(out["binary"]["_res"][1], out["learned"]["_res"][1]))
        for v in out.values():
            v.pop("_res")
        ai = a.info()
        fb, mm = a.learned_fallbacks(txy)
        # the same probes over the points in Hilbert order of their cells (a
        # resident layout a serving system would keep): lookups of neighbouring
        # points share cache lines; results must not change
        sx, sv = hilbert_sorted(torch, txy, tv, ai)
        srt = {}
        for srch in ("binary", "learned"):
            cc = torch.empty_like(counts)
            ss = torch.empty_like(sums)
            a.aggregate(sx, sv, cc, ss, search=srch)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(3):
                a.aggregate(sx, sv, cc, ss, search=srch)
            e1.record()
            torch.cuda.synchronize()
            t = e0.elapsed_time(e1) / 3
            srt[srch] = {"probe_ms": round(t, 4), "points_per_s": n / (t * 1e-3),
                         "gbps": alg_bytes / (t * 1e-3) / 1e9,
                         "same_as_unsorted": bool(np.array_equal(cc.cpu().numpy(), res_c.astype(np.int64))
                                                  and np.array_equal(ss.cpu().numpy(), res_s))}
            # the batch entry point over the same range: workgroups take
            # contiguous items and count them in an LDS table of cell codes,
            # which sorted points keep small
            task = sba.Task(a, sx, sv, 0, n, None, cc, ss, search=srch)
            sba.aggregate_batch([task])
            torch.cuda.synchronize()
            e0.record()
            for _ in range(3):
                sba.aggregate_batch([task])
            e1.record()
            torch.cuda.synchronize()
            tb = e0.elapsed_time(e1) / 3
            srt[srch]["batch_probe_ms"] = round(tb, 4)
            srt[srch]["batch_points_per_s"] = n / (tb * 1e-3)
            srt[srch]["batch_same"] = bool(np.array_equal(cc.cpu().numpy(), res_c.astype(np.int64))
                                           and np.array_equal(ss.cpu().numpy(), res_s))
        del sx, sv
        extra["hilbert_sorted_points"] = srt
        # the points as generated, partitioned into 256 coarse regions by the
        # call itself and then probed region by region (scratch 16 B/point)
        scratch = torch.empty(a.scratch_bytes(n), dtype=torch.uint8, device=dev)
        part = {}
        for srch in ("binary", "learned"):
            cc = torch.empty_like(counts)
            ss = torch.empty_like(sums)
            a.aggregate_partitioned(txy, tv, cc, ss, search=srch, scratch=scratch)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(3):
                a.aggregate_partitioned(txy, tv, cc, ss, search=srch, scratch=scratch)
            e1.record()
            torch.cuda.synchronize()
            t = e0.elapsed_time(e1) / 3
            part[srch] = {"ms": round(t, 4), "points_per_s": n / (t * 1e-3),
                          "same_as_direct": bool(
                              np.array_equal(cc.cpu().numpy(), res_c.astype(np.int64))
                              and np.array_equal(ss.cpu().numpy(), res_s))}
        del scratch
        extra["partitioned_probe"] = part
        log(f"[bench] partitioned probe: {json.dumps(part)}")
        extra["learned_vs_binary"] = {**out, "identical": bool(same),
                                      "speedup": out["binary"]["probe_ms"] / out["learned"]["probe_ms"],
                                      "fallbacks": fb, "learned_ne_binary": mm,
                                      "n_runs": ai["n_runs"], "max_leaf_err": ai["max_leaf_err"],
                                      "mean_leaf_err": ai["mean_leaf_err"],
                                      "leaves": 1 << ai["log2_leaves"]}
        a.close()

    if args.workload == "city":
        # result range [alpha - beta, alpha] (Sec. 6): beta from a
        # boundary-only approximation over the same points
        t0 = time.perf_counter()
        bh = sba.Approx(ro, vo, pxy, eps, boundary_only=True, tile_log2=info["tile_log2"],
                        sub_log2=info["sub_log2"])
        t_bb = 1000.0 * (time.perf_counter() - t0)
        bc = torch.empty_like(counts)
        bs = torch.empty_like(sums)
        bh.aggregate(txy, tv, bc, bs)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            bh.aggregate(txy, tv, bc, bs)
        e1.record()
        torch.cuda.synchronize()
        beta_probe = e0.elapsed_time(e1) / 10
        beta = bc.cpu().numpy().astype(np.float64)
        alpha = res_c.astype(np.float64)
        # alpha and beta in one pass over the points
        a_full = sba.Approx(ro, vo, pxy, eps, **kw)
        rr = sba.aggregate_range(a_full, bh, txy, tv)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(10):
            rr = sba.aggregate_range(a_full, bh, txy, tv)
        e1.record()
        torch.cuda.synchronize()
        one_pass = e0.elapsed_time(e1) / 10
        same = bool(np.array_equal(rr[0].cpu().numpy().astype(np.uint64), res_c)
                    and np.array_equal(rr[2].cpu().numpy(), bc.cpu().numpy()))
        extra["result_range"] = {
            "beta_build_ms": round(t_bb, 3), "beta_probe_ms": round(beta_probe, 4),
            "alpha_plus_beta_one_pass_ms": round(one_pass, 4),
            "one_pass_kernel": sba.range_kernel(a_full, bh),
            "one_pass_same_as_two": same,
            "beta_over_alpha_total": float(beta.sum() / max(alpha.sum(), 1.0)),
            "beta_over_alpha_median_polygon": float(np.median(beta / np.maximum(alpha, 1.0))),
            "kernel": bh.probe_kernel(True)}
        a_full.close()
        bh.close()
        log(f"[bench] result range: {json.dumps(extra['result_range'])}")

    if args.workload == "city":
        # the non-conservative approximation (cells whose centre is inside):
        # same probe kernel, no double counting on the partition's shared
        # boundaries, misclassified points within eps/2
        t0 = time.perf_counter()
        ch = sba.Approx(ro, vo, pxy, eps, centre_sampled=True, tile_log2=args.tile_log2,
                        sub_log2=args.sub_log2)
        t_cb = 1000.0 * (time.perf_counter() - t0)
        cc = torch.empty_like(counts)
        cs = torch.empty_like(sums)
        ch.aggregate(txy, tv, cc, cs)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            ch.aggregate(txy, tv, cc, cs)
        e1.record()
        torch.cuda.synchronize()
        csum = int(cc.sum().item())
        extra["centre_sampled"] = {
            "build_ms": round(t_cb, 3), "probe_ms": round(e0.elapsed_time(e1) / 10, 4),
            "counted_over_points": csum / n,
            "conservative_counted_over_points": float(res_c.sum()) / n,
            "kernel": ch.probe_kernel(True)}
        ch.close()
        log(f"[bench] centre-sampled: {json.dumps(extra['centre_sampled'])}")

    if args.workload == "city":
        extra["polygon_join"] = join_bench(sba, torch, polys, polys, eps,
                                           "city partition with itself")
    if args.workload == "quadtree":
        from gen import city_polygons
        extra["polygon_join"] = join_bench(sba, torch, polys, city_polygons(), eps,
                                           "40,000-cell partition with the 260-cell partition")

    if args.workload in ("city", "quadtree") and not args.no_pindex:
        extra["point_index"] = pindex_bench(sba, torch, txy, tv, ro, vo, pxy, eps, res_c, res_s,
                                            probe_avg)

    sweep = {}
    if args.workload == "city" and not args.no_sweep:
        for e in (100, 1000, 10000):
            a = sba.Approx(ro, vo, pxy, e, kind="grid")
            for _ in range(2):
                a.aggregate(txy, tv, counts, sums)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            reps = 10
            e0.record()
            for _ in range(reps):
                a.aggregate(txy, tv, counts, sums)
            e1.record()
            torch.cuda.synchronize()
            t = e0.elapsed_time(e1) / reps
            ai = a.info()
            sweep[f"{e / 100:g}m"] = {"probe_ms": round(t, 4), "probe_points_per_s": n / (t * 1e-3),
                                      "probe_gbps": round(alg_bytes / (t * 1e-3) / 1e9, 1),
                                      "build_ms": round(ai["build_ms"], 3),
                                      "tile": 1 << ai["tile_log2"], "blocks": ai["n_blocks"],
                                      "approx_MB": round(ai["bytes"] / 2**20, 2)}
            a.close()
        log(f"[bench] eps sweep: {json.dumps(sweep)}")

    serving = None
    if args.serve and args.workload == "city":
        serving = serve_bench(args, torch, txy, tv, args.queries)

    cpu = None
    if not args.no_cpu:
        import oracle
        t0 = time.perf_counter()
        O = oracle.Approx(polys, eps)
        tb = time.perf_counter() - t0
        sample = min(n, 200_000_000)
        t0 = time.perf_counter()
        oc, os_ = O.aggregate(xy[:2 * sample], vals[:sample])
        ta = time.perf_counter() - t0
        t_step = tb + ta * (n / sample)
        cpu = {"value": n / t_step, "unit": "points/s", "cores": int(O.threads_used),
               "kind": "oracle",
               "sample": (f"oracle build of all {polys.n_polys} polygons ({tb:.2f}s) + oracle "
                          f"aggregate of the first {sample} points ({ta:.2f}s), aggregate time "
                          f"scaled to all {n} points")}
        if sample == n and layout == "grid":
            cpu["matches_gpu"] = bool(np.array_equal(oc, res_c) and np.array_equal(os_, res_s))
        log(f"[bench] cpu oracle: {json.dumps(cpu)}")

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
                     "kernel": kernel,
                     "algorithmic_bytes_per_launch": alg_bytes},
        "cpu_baseline": cpu,
        "probe_ms": probe_avg,
        "probe_ms_in_step": probe_in_step,
        "probe_points_per_s": n / (probe_avg * 1e-3),
        "build_ms_median": build_iso,
        "approx": {k: info[k] for k in ("s", "gw", "gh", "tile_log2", "n_tiles", "n_blocks",
                                        "n_sets", "n_segments", "n_boundary", "n_runs", "bytes")},
        "eps_sweep": sweep or None,
        "serving": serving,
        **extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
