"""Seeded synthetic inputs with the shapes of the paper's workloads.

The paper measures on NYC taxi pickups joined with NYC census blocks,
neighbourhoods and boroughs (Sec. 3 "Performance", Sec. 5.1, Sec. 5.2).  None
of that data is available here, so every input is drawn from a seeded
generator instead:

* points  -- int32 fixed-point coordinates, interleaved ``[x0, y0, x1, y1, ...]``
  (uniform in a square, or a Gaussian mixture standing in for a city's
  pickup density);
* values  -- int64 cents (uniform, or lognormal standing in for fares);
* polygons -- CSR rings (random star-shaped polygons that may overlap, or a
  Voronoi partition of a box whose shared edges are jittered into polylines,
  standing in for census blocks / neighbourhoods).

Nothing here approximates, rasterises or aggregates anything.
"""
from __future__ import annotations

import concurrent.futures as _cf
import dataclasses
import math
import os

import numpy as np

__all__ = [
    "Polygons", "polygons_from_rings", "uniform_points", "uniform_cents",
    "star_polygons", "mixture_points", "lognormal_cents", "voronoi_partition",
    "seeds", "tiny_workload", "city_polygons", "city_points", "quadtree_polygons",
    "viewport_queries", "CITY_BOX", "TINY_BOX",
]

TINY_BOX = 65536            # tiny workload: coordinates in [0, 65536)
CITY_BOX = 4_000_000        # 40 km at 1 cm per unit


@dataclasses.dataclass
class Polygons:
    """Polygons in CSR form.

    ring_off[n_polys+1]  ring index range of each polygon
    vert_off[n_rings+1]  vertex index range of each ring (rings are closed
                         implicitly: the last vertex joins the first)
    xy[2*n_verts]        int32 x, y interleaved
    """
    ring_off: np.ndarray
    vert_off: np.ndarray
    xy: np.ndarray

    @property
    def n_polys(self) -> int:
        return int(self.ring_off.shape[0] - 1)

    @property
    def n_rings(self) -> int:
        return int(self.vert_off.shape[0] - 1)

    @property
    def n_verts(self) -> int:
        return int(self.xy.shape[0] // 2)

    def rings_of(self, p: int):
        out = []
        for r in range(int(self.ring_off[p]), int(self.ring_off[p + 1])):
            v0, v1 = int(self.vert_off[r]), int(self.vert_off[r + 1])
            out.append(self.xy[2 * v0:2 * v1].reshape(-1, 2).copy())
        return out

    def subset(self, ids) -> "Polygons":
        return polygons_from_rings([self.rings_of(int(p)) for p in ids])


def polygons_from_rings(polys) -> Polygons:
    """polys: list (per polygon) of lists (per ring) of (n,2) integer arrays."""
    ring_off = [0]
    vert_off = [0]
    chunks = []
    for rings in polys:
        for ring in rings:
            ring = np.asarray(ring, dtype=np.int64).reshape(-1, 2)
            chunks.append(ring)
            vert_off.append(vert_off[-1] + ring.shape[0])
        ring_off.append(len(vert_off) - 1)
    xy = (np.concatenate(chunks).reshape(-1) if chunks else np.zeros(0, np.int64))
    return Polygons(np.asarray(ring_off, np.int32), np.asarray(vert_off, np.int64),
                    np.ascontiguousarray(xy.astype(np.int32)))


def seeds(config: int) -> dict:
    """Seed of each input stream of workload number ``config`` (1-based)."""
    base = 100 * config
    return {"points": base + 1, "values": base + 2, "polygons": base + 3,
            "jitter": base + 4, "queries": base + 5}


# --------------------------------------------------------------------------
# points and values
# --------------------------------------------------------------------------

def uniform_points(n: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """n points with x, y uniform integers in [lo, hi); int32 [2n]."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.integers(lo, hi, size=2 * n, dtype=np.int64).astype(np.int32))


def uniform_cents(n: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """n int64 values uniform in [lo, hi] (inclusive)."""
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, size=n, dtype=np.int64)


def _chunks(n: int, chunk: int):
    return [(a, min(n, a + chunk)) for a in range(0, n, chunk)]


def _pool_size(threads):
    if threads:
        return threads
    return max(1, min(16, os.cpu_count() or 1))


def mixture_points(n: int, box: int, seed: int, k: int = 50,
                   sigma=(20_000.0, 300_000.0), chunk: int = 1 << 23,
                   threads: int | None = None) -> np.ndarray:
    """Gaussian mixture in [0, box)^2, quantised by floor to int32 units.

    k isotropic components: centres uniform in the box, sigma uniform in
    ``sigma`` (units), weights proportional to U(0.5, 1.5).  Samples outside
    the box are drawn again.  Chunks use independent child seeds, so the
    result does not depend on the number of threads.
    """
    ss = np.random.SeedSequence(seed)
    prng = np.random.default_rng(ss.spawn(1)[0])
    centres = prng.uniform(0.0, box, size=(k, 2))
    sig = prng.uniform(sigma[0], sigma[1], size=k)
    w = prng.uniform(0.5, 1.5, size=k)
    w = w / w.sum()
    cw = np.cumsum(w)
    cw[-1] = 1.0
    out = np.empty(2 * n, dtype=np.int32)
    parts = _chunks(n, chunk)
    kids = np.random.SeedSequence([seed, 7]).spawn(len(parts))

    def work(idx):
        a, b = parts[idx]
        rng = np.random.default_rng(kids[idx])
        m = b - a
        res = np.empty((m, 2), dtype=np.float64)
        todo = np.arange(m)
        while todo.size:
            comp = np.searchsorted(cw, rng.random(todo.size), side="right")
            comp = np.minimum(comp, k - 1)
            pts = centres[comp] + sig[comp, None] * rng.standard_normal((todo.size, 2))
            ok = (pts[:, 0] >= 0) & (pts[:, 0] < box) & (pts[:, 1] >= 0) & (pts[:, 1] < box)
            res[todo[ok]] = pts[ok]
            todo = todo[~ok]
        q = np.floor(res).astype(np.int64)
        np.clip(q, 0, box - 1, out=q)
        out[2 * a:2 * b] = q.reshape(-1).astype(np.int32)

    with _cf.ThreadPoolExecutor(_pool_size(threads)) as ex:
        list(ex.map(work, range(len(parts))))
    return out


def lognormal_cents(n: int, seed: int, mu: float = 7.0, sigma: float = 0.8,
                    chunk: int = 1 << 23, threads: int | None = None) -> np.ndarray:
    """int64 cents: round-half-up of exp(mu + sigma z), clamped to [1, 10^7]."""
    out = np.empty(n, dtype=np.int64)
    parts = _chunks(n, chunk)
    kids = np.random.SeedSequence([seed, 11]).spawn(len(parts))

    def work(idx):
        a, b = parts[idx]
        rng = np.random.default_rng(kids[idx])
        v = np.floor(np.exp(mu + sigma * rng.standard_normal(b - a)) + 0.5)
        out[a:b] = np.clip(v, 1, 10_000_000).astype(np.int64)

    with _cf.ThreadPoolExecutor(_pool_size(threads)) as ex:
        list(ex.map(work, range(len(parts))))
    return out


# --------------------------------------------------------------------------
# polygons
# --------------------------------------------------------------------------

def star_polygons(n: int, n_vert: int, rmin: float, rmax: float, box: int,
                  seed: int) -> Polygons:
    """Random star-shaped simple polygons, overlaps allowed.

    Centre uniform in [0, box)^2, n_vert angles sorted uniform in [0, 2 pi),
    a radius uniform in [rmin, rmax] drawn per vertex; vertices rounded
    half-up to integers.
    """
    rng = np.random.default_rng(seed)
    polys = []
    for _ in range(n):
        c = rng.uniform(0, box, size=2)
        ang = np.sort(rng.uniform(0, 2 * math.pi, size=n_vert))
        rad = rng.uniform(rmin, rmax, size=n_vert)
        v = np.floor(c[None, :] + rad[:, None] * np.c_[np.cos(ang), np.sin(ang)] + 0.5)
        polys.append([v.astype(np.int64)])
    return polygons_from_rings(polys)


def _seg_point_dist(px, py, ax, ay, bx, by):
    vx, vy = bx - ax, by - ay
    l2 = vx * vx + vy * vy
    t = np.where(l2 > 0, ((px - ax) * vx + (py - ay) * vy) / np.where(l2 > 0, l2, 1), 0.0)
    t = np.clip(t, 0.0, 1.0)
    dx, dy = ax + t * vx - px, ay + t * vy - py
    return np.sqrt(dx * dx + dy * dy)


def voronoi_partition(n_sites: int, box: int, edge_verts=(10, 200), seed: int = 3,
                      jitter_seed: int = 4) -> Polygons:
    """Voronoi cells of seeded sites, clipped to [0, box]^2, edges jittered.

    Clipping is exact through mirroring the sites across the four sides of
    the box.  Every edge shared by two cells is replaced by one polyline with
    a number of interior vertices drawn from ``edge_verts``; both cells use
    the same polyline (one of them reversed), so the cells still tile the
    box.  Edges on the box sides stay straight.  The perpendicular offset of
    each interior vertex is kept inside two narrow cones at the edge's
    endpoints (a fraction of half the smallest angle between edges meeting
    there), below 0.3 times the distance to any other non-adjacent edge of
    the two cells and below a quarter of the spacing of its neighbours, so
    the polylines cannot cross.
    """
    from scipy.spatial import Voronoi

    rng = np.random.default_rng(seed)
    sites = rng.uniform(0.0, float(box), size=(n_sites, 2))
    s = sites
    allp = np.vstack([s, np.c_[-s[:, 0], s[:, 1]], np.c_[2.0 * box - s[:, 0], s[:, 1]],
                      np.c_[s[:, 0], -s[:, 1]], np.c_[s[:, 0], 2.0 * box - s[:, 1]]])
    vor = Voronoi(allp)
    vq = np.floor(vor.vertices + 0.5).astype(np.int64)
    # vertices that coincide after rounding become one vertex
    _, vcanon = np.unique(vq, axis=0, return_inverse=True)
    vcanon = vcanon.reshape(-1)
    first_of = np.full(vcanon.max() + 1, -1, np.int64)
    for v in range(len(vcanon) - 1, -1, -1):
        first_of[vcanon[v]] = v
    vrep = first_of[vcanon]            # representative vertex index of each vertex

    # cyclic vertex order of each original cell, by angle about its site
    cells = []
    for i in range(n_sites):
        reg = np.array([v for v in vor.regions[vor.point_region[i]] if v >= 0], np.int64)
        vv = vor.vertices[reg]
        order = np.argsort(np.arctan2(vv[:, 1] - s[i, 1], vv[:, 0] - s[i, 0]))
        ring = vrep[reg[order]]
        keep = np.r_[True, ring[1:] != ring[:-1]]
        ring = ring[keep]
        if len(ring) > 1 and ring[0] == ring[-1]:
            ring = ring[:-1]
        cells.append(ring)

    # edges of every cell, keyed by the (min, max) vertex pair
    ca = np.concatenate([c for c in cells])
    cb = np.concatenate([np.roll(c, -1) for c in cells])
    cid = np.concatenate([np.full(len(c), k) for k, c in enumerate(cells)])
    lo_v, hi_v = np.minimum(ca, cb), np.maximum(ca, cb)
    ekey = lo_v * (len(vq) + 1) + hi_v
    ukey, eidx, ecount = np.unique(ekey, return_inverse=True, return_counts=True)
    eidx = eidx.reshape(-1)
    E = len(ukey)
    ea = (ukey // (len(vq) + 1)).astype(np.int64)
    eb = (ukey % (len(vq) + 1)).astype(np.int64)
    A = vq[ea].astype(np.float64)
    B = vq[eb].astype(np.float64)
    shared = ecount == 2

    # smallest angle between edges meeting at each vertex
    ends = np.r_[ea, eb]
    dirs = np.r_[np.arctan2(B[:, 1] - A[:, 1], B[:, 0] - A[:, 0]),
                 np.arctan2(A[:, 1] - B[:, 1], A[:, 0] - B[:, 0])]
    order = np.lexsort((dirs, ends))
    ends_s, dirs_s = ends[order], dirs[order]
    same = np.r_[ends_s[1:] == ends_s[:-1], False]
    gap = np.where(same, np.r_[dirs_s[1:] - dirs_s[:-1], 0.0], np.inf)
    starts = np.r_[True, ends_s[1:] != ends_s[:-1]]
    grp_first = np.maximum.accumulate(np.where(starts, np.arange(len(ends_s)), 0))
    wrap = np.where(~same, 2 * np.pi - (dirs_s - dirs_s[grp_first]), np.inf)
    cand = np.minimum(gap, wrap)
    nv_all = len(vq)
    min_ang = np.full(nv_all, np.inf)
    np.minimum.at(min_ang, ends_s, cand)
    single = np.bincount(ends_s, minlength=nv_all) <= 1
    min_ang[single] = np.pi
    min_ang = np.clip(min_ang, 1e-6, np.pi)

    # distance from each edge to the non-adjacent edges of its cells
    pa, pb = [], []
    off = 0
    for c in cells:
        m = len(c)
        if m >= 4:
            x, y = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
            d = (y - x) % m
            sel = (d != 0) & (d != 1) & (d != m - 1)
            pa.append(eidx[off + x[sel]])
            pb.append(eidx[off + y[sel]])
        off += m
    dsep = np.full(E, np.inf)
    if pa:
        pa = np.concatenate(pa)
        pb = np.concatenate(pb)
        d = np.minimum.reduce([
            _seg_point_dist(A[pb, 0], A[pb, 1], A[pa, 0], A[pa, 1], B[pa, 0], B[pa, 1]),
            _seg_point_dist(B[pb, 0], B[pb, 1], A[pa, 0], A[pa, 1], B[pa, 0], B[pa, 1]),
            _seg_point_dist(A[pa, 0], A[pa, 1], A[pb, 0], A[pb, 1], B[pb, 0], B[pb, 1]),
            _seg_point_dist(B[pa, 0], B[pa, 1], A[pb, 0], A[pb, 1], B[pb, 0], B[pb, 1]),
        ])
        np.minimum.at(dsep, pa, d)

    # jitter, all shared edges at once
    jr = np.random.default_rng(jitter_seed)
    lo, hi = edge_verts
    L = np.hypot(B[:, 0] - A[:, 0], B[:, 1] - A[:, 1])
    m_want = jr.integers(lo, hi + 1, size=E)
    phA, phB = min_ang[ea], min_ang[eb]
    hA = np.minimum(0.5, 0.4 * np.tan(phA / 2))
    hB = np.minimum(0.5, 0.4 * np.tan(phB / 2))
    # keep interior vertices away from the ends, where rounding could
    # otherwise cross a neighbouring polyline meeting at a small angle
    rA = 8.0 / np.maximum(np.sin(phA / 2), 1e-9)
    rB = 8.0 / np.maximum(np.sin(phB / 2), 1e-9)
    Ls = np.where(L > 0, L, 1.0)
    t_lo = np.where(L > 0, rA / Ls, 1.0)
    t_hi = np.where(L > 0, 1.0 - rB / Ls, 0.0)
    room = np.maximum(0.0, t_hi - t_lo) * L / 4.0
    m = np.where(shared & (t_hi > t_lo), np.minimum(m_want, room.astype(np.int64)), 0)
    tot = int(m.sum())
    eid = np.repeat(np.arange(E), m)
    t = t_lo[eid] + (t_hi[eid] - t_lo[eid]) * jr.random(tot)
    order = np.lexsort((t, eid))
    t = t[order]
    seg_start = np.r_[0, np.cumsum(m)[:-1]]
    first = np.zeros(tot, bool)
    first[seg_start[m > 0]] = True
    last = np.zeros(tot, bool)
    last[(seg_start + m - 1)[m > 0]] = True
    prev_t = np.where(first, 0.0, np.r_[0.0, t[:-1]])
    next_t = np.where(last, 1.0, np.r_[t[1:], 1.0])
    spacing = np.minimum(t - prev_t, next_t - t) * L[eid]
    cap = np.minimum(np.minimum(hA[eid] * t, hB[eid] * (1.0 - t)) * L[eid], 0.25 * spacing)
    cap = np.minimum(cap, 0.3 * dsep[eid])
    u = jr.uniform(-1.0, 1.0, size=tot) * cap
    dx, dy = (B[:, 0] - A[:, 0])[eid], (B[:, 1] - A[:, 1])[eid]
    nx, ny = -dy / Ls[eid], dx / Ls[eid]
    px = A[eid, 0] + t * dx + u * nx
    py = A[eid, 1] + t * dy + u * ny
    q = np.floor(np.c_[px, py] + 0.5).astype(np.int64)
    # drop points equal to their predecessor on the same edge or to an endpoint
    dup = np.r_[False, np.all(q[1:] == q[:-1], axis=1) & (eid[1:] == eid[:-1])]
    endp = np.all(q == vq[ea[eid]], axis=1) | np.all(q == vq[eb[eid]], axis=1)
    keep = ~(dup | endp)
    q, eid_k = q[keep], eid[keep]
    cnt = np.bincount(eid_k, minlength=E)
    eoff = np.r_[0, np.cumsum(cnt)]

    polys = []
    off = 0
    for c in cells:
        mm = len(c)
        out = []
        for k in range(mm):
            a, b = int(c[k]), int(c[(k + 1) % mm])
            out.append(vq[a][None, :])
            e = int(eidx[off + k])
            seg = q[eoff[e]:eoff[e + 1]]
            if len(seg):
                out.append(seg if a < b else seg[::-1])
        off += mm
        polys.append([np.concatenate(out, axis=0)])
    return polygons_from_rings(polys)


# --------------------------------------------------------------------------
# workload presets
# --------------------------------------------------------------------------

def tiny_workload(n_points: int = 1_000_000):
    """Workload 1: uniform points in [0, 65536)^2, uniform cents in
    [100, 10000], 16 star polygons of 32 vertices, radius in [2000, 12000]."""
    sd = seeds(1)
    xy = uniform_points(n_points, 0, TINY_BOX, sd["points"])
    vals = uniform_cents(n_points, 100, 10_000, sd["values"])
    polys = star_polygons(16, 32, 2000.0, 12000.0, TINY_BOX, sd["polygons"])
    return xy, vals, polys


def city_polygons(n_sites: int = 260, edge_verts=(10, 200), config: int = 2) -> Polygons:
    """Workload 2 polygons: Voronoi partition of the 40 km box (1 cm units)."""
    sd = seeds(config)
    return voronoi_partition(n_sites, CITY_BOX, edge_verts, sd["polygons"], sd["jitter"])


def city_points(n_points: int, config: int = 2, threads=None):
    """Workload 2 points (50-component Gaussian mixture, sigma 200-3000 m) and
    lognormal(7, 0.8) cents."""
    sd = seeds(config)
    xy = mixture_points(n_points, CITY_BOX, sd["points"], threads=threads)
    vals = lognormal_cents(n_points, sd["values"], threads=threads)
    return xy, vals


def quadtree_polygons(n_sites: int = 40_000) -> Polygons:
    """Workload 3 polygons: 40,000-cell partition, 50-500 vertices each."""
    return city_polygons(n_sites, (8, 83), config=3)


def viewport_queries(n: int, seed: int, box: int = CITY_BOX, n_sets: int = 3):
    """Viewport aggregation queries at zoom levels 10..18.

    Side = 40 km * 40^(-(z-10)/8) * U(0.8, 1.25), centre uniform in the box
    (clamped so the viewport stays inside), eps = 15000 >> (z - 10) units
    (one pixel), COUNT or SUM with equal odds, polygon set uniform.
    Returns a structured list of dicts.
    """
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        z = int(rng.integers(10, 19))
        side = int(box * 40.0 ** (-(z - 10) / 8.0) * rng.uniform(0.8, 1.25))
        side = max(1, min(side, box))
        cx = int(rng.integers(0, box - side + 1))
        cy = int(rng.integers(0, box - side + 1))
        out.append({"zoom": z, "vx": cx, "vy": cy, "vw": side,
                    "eps": int(15000 >> (z - 10)), "agg": "sum" if rng.random() < 0.5 else "count",
                    "set": int(rng.integers(0, n_sets))})
    return out
