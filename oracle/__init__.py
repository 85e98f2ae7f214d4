"""ctypes wrapper of the plain CPU oracle (``sba_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the CPU-baseline leg of the benchmark -- never by the GPU library or its
binding.  See the header of ``sba_oracle.c`` for the definitions it follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sba_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# ORACLE_LIBRARY names another build of this source to load instead (the
# mutation tests load deliberately broken copies built in a temporary folder)
_LIB_OVERRIDE = os.environ.get("ORACLE_LIBRARY")
_lib = None

_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")


def build(extra_flags=()) -> str:
    """Compile the oracle with gcc (plain C, OpenMP)."""
    cmd = ["gcc", "-O2", "-std=gnu11", "-Wall", "-Wextra", "-fopenmp", "-fPIC", "-shared",
           *extra_flags, "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if _LIB_OVERRIDE:
        L = C.CDLL(_LIB_OVERRIDE)
    else:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
    L.orc_cell_side.restype = C.c_int64
    L.orc_cell_side.argtypes = [C.c_int64]
    L.orc_raster_brute.restype = C.c_int
    L.orc_raster_brute.argtypes = [C.c_int32, _i32p, _i64p, _i32p, C.c_int64, C.c_int64,
                                   C.c_int64, C.c_int64, C.c_int64, _u8p]
    L.orc_centre_brute.restype = C.c_int
    L.orc_centre_brute.argtypes = [C.c_int32, _i32p, _i64p, _i32p, C.c_int64, C.c_int64,
                                   C.c_int64, C.c_int64, C.c_int64, _u8p]
    L.orc_join_pairs.restype = C.c_int64
    L.orc_join_pairs.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, _i32p, _i32p, _i64p]
    L.orc_build.restype = C.c_void_p
    L.orc_build.argtypes = [C.c_int32, _i32p, _i64p, _i32p, C.c_int64]
    L.orc_build_mode.restype = C.c_void_p
    L.orc_build_mode.argtypes = [C.c_int32, _i32p, _i64p, _i32p, C.c_int64, C.c_int]
    L.orc_free.restype = None
    L.orc_free.argtypes = [C.c_void_p]
    L.orc_cell_side_of.restype = C.c_int64
    L.orc_cell_side_of.argtypes = [C.c_void_p]
    L.orc_n_intervals.restype = C.c_int64
    L.orc_n_intervals.argtypes = [C.c_void_p]
    L.orc_export_intervals.restype = None
    L.orc_export_intervals.argtypes = [C.c_void_p, _i32p, _i64p, _i64p, _i64p]
    L.orc_cell_set.restype = C.c_int
    L.orc_cell_set.argtypes = [C.c_void_p, C.c_int64, C.c_int64, _i32p, C.c_int]
    for name in ("orc_aggregate", "orc_exact_join"):
        f = getattr(L, name)
        f.restype = C.c_int
        f.argtypes = [C.c_void_p, _i32p, C.c_void_p, C.c_int64, _u64p, C.c_void_p, C.c_int]
    L.orc_invariant.restype = C.c_int
    L.orc_invariant.argtypes = [C.c_void_p, _i32p, C.c_int64, _i64p, C.c_int]
    L.orc_invariant_all.restype = C.c_int
    L.orc_invariant_all.argtypes = [C.c_void_p, _i32p, C.c_int64, _i64p]
    L.orc_invariant_at.restype = C.c_int
    L.orc_invariant_at.argtypes = [C.c_void_p, _i32p, C.c_int64, C.c_int64, C.c_int, _i64p,
                                   C.c_int]
    L.orc_invariant_all_at.restype = C.c_int
    L.orc_invariant_all_at.argtypes = [C.c_void_p, _i32p, C.c_int64, C.c_int64, C.c_int, _i64p]
    L.orc_seg_within.restype = C.c_int
    L.orc_seg_within.argtypes = [C.c_int64] * 7 + [C.c_int]
    L.orc_near_boundary.restype = C.c_int
    L.orc_near_boundary.argtypes = [C.c_void_p, C.c_int32, C.c_int64, C.c_int64, C.c_int64,
                                    C.c_int]
    L.orc_hilbert_d.restype = C.c_uint64
    L.orc_hilbert_d.argtypes = [C.c_int, C.c_int64, C.c_int64]
    L.orc_hilbert_level.restype = C.c_int
    L.orc_hilbert_level.argtypes = [C.c_void_p]
    L.orc_union_box.restype = None
    L.orc_union_box.argtypes = [C.c_void_p, _i64p]
    L.orc_hilbert_runs.restype = C.c_int
    L.orc_hilbert_runs.argtypes = [C.c_void_p, C.c_int, _u64p, _i64p, _i32p, C.c_int64,
                                   C.c_int64, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    _lib = L
    return L


def _poly_arrays(polys):
    return (np.ascontiguousarray(polys.ring_off, np.int32),
            np.ascontiguousarray(polys.vert_off, np.int64),
            np.ascontiguousarray(polys.xy, np.int32))


def cell_side(eps: int) -> int:
    """Largest s with 2 s^2 <= eps^2 (0 if eps is outside [2, 2^28])."""
    return int(lib().orc_cell_side(int(eps)))


def raster_brute(polys, s: int, i0: int, j0: int, nw: int, nh: int) -> np.ndarray:
    """Per-polygon cell classes over a window: uint8 [P, nh, nw],
    2 = boundary cell, 1 = interior cell, 0 = neither.  Definition form."""
    ro, vo, xy = _poly_arrays(polys)
    out = np.zeros(polys.n_polys * nh * nw, np.uint8)
    rc = lib().orc_raster_brute(polys.n_polys, ro, vo, xy, s, i0, j0, nw, nh, out)
    if rc:
        raise ValueError("orc_raster_brute rejected its input")
    return out.reshape(polys.n_polys, nh, nw)


def centre_brute(polys, s: int, i0: int, j0: int, nw: int, nh: int) -> np.ndarray:
    """Per-polygon membership of the centre-sampled approximation over a
    window: uint8 [P, nh, nw], 1 if the cell's centre is inside P.
    Definition form (Sec. 2.2, non-conservative raster)."""
    ro, vo, xy = _poly_arrays(polys)
    out = np.zeros(polys.n_polys * nh * nw, np.uint8)
    rc = lib().orc_centre_brute(polys.n_polys, ro, vo, xy, s, i0, j0, nw, nh, out)
    if rc:
        raise ValueError("orc_centre_brute rejected its input")
    return out.reshape(polys.n_polys, nh, nw)


def join_pairs(a: "Approx", b: "Approx"):
    """Polygon pairs (p of a, q of b) whose approximations share cells, with
    the number of shared cells: (pa int32, pb int32, cells int64) in (p, q)
    order (Sec. 4: blend of two rasterized canvases, mask of the cells that
    hold both)."""
    z32, z64 = np.zeros(1, np.int32), np.zeros(1, np.int64)
    n = int(lib().orc_join_pairs(a._h, b._h, 0, z32, z32, z64))
    if n < 0:
        raise ValueError("the approximations have different cell sides")
    pa, pb, cells = np.zeros(max(n, 1), np.int32), np.zeros(max(n, 1), np.int32), np.zeros(max(n, 1), np.int64)
    lib().orc_join_pairs(a._h, b._h, n, pa, pb, cells)
    return pa[:n], pb[:n], cells[:n]


def seg_within(p, a, b, eps: int, half: bool = False) -> bool:
    """Is point p within eps (half: eps/2) of the closed segment a-b?  Exact
    (Sec. 2.2: the distance bound every misclassified point must meet)."""
    r = lib().orc_seg_within(int(p[0]), int(p[1]), int(a[0]), int(a[1]), int(b[0]), int(b[1]),
                             int(eps), 1 if half else 0)
    if r < 0:
        raise ValueError("coordinates or eps out of range")
    return bool(r)


def hilbert_d(L: int, i: int, j: int) -> int:
    return int(lib().orc_hilbert_d(L, int(i), int(j)))


class Approx:
    """The oracle's A(P) for every polygon, held as sorted row intervals.

    boundary_only=True holds B(P) instead: the boundary cells alone, over
    which the partial count of the result range [alpha - beta, alpha]
    (Sec. 6, result range estimation) is taken.  centre=True holds the
    centre-sampled approximation C(P) (Sec. 2.2, non-conservative): the cells
    whose centre is inside P.
    """

    def __init__(self, polys, eps: int, boundary_only: bool = False, centre: bool = False):
        ro, vo, xy = _poly_arrays(polys)
        self._keep = (ro, vo, xy)
        self.n_polys = polys.n_polys
        self.eps = int(eps)
        self.boundary_only = bool(boundary_only)
        if boundary_only and centre:
            raise ValueError("boundary_only and centre exclude each other")
        self.centre = bool(centre)
        self._h = lib().orc_build_mode(polys.n_polys, ro, vo, xy, int(eps),
                                       1 if boundary_only else (2 if centre else 0))
        if not self._h:
            raise ValueError("oracle rejected the polygons or eps")
        self.s = int(lib().orc_cell_side_of(self._h))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_free(h)
            self._h = None

    def intervals(self):
        """(poly, row, x0, x1): cells [x0, x1) of row `row` are in A(poly)."""
        n = int(lib().orc_n_intervals(self._h))
        p = np.zeros(n, np.int32)
        r = np.zeros(n, np.int64)
        a = np.zeros(n, np.int64)
        b = np.zeros(n, np.int64)
        lib().orc_export_intervals(self._h, p, r, a, b)
        return p, r, a, b

    def cell_set(self, i: int, j: int) -> list:
        buf = np.zeros(max(1, self.n_polys), np.int32)
        n = lib().orc_cell_set(self._h, int(i), int(j), buf, buf.shape[0])
        return buf[:n].tolist()

    def _agg(self, fn, xy, vals, nthreads):
        xy = np.ascontiguousarray(xy, np.int32)
        n = xy.shape[0] // 2
        counts = np.zeros(max(1, self.n_polys), np.uint64)
        sums = np.zeros(max(1, self.n_polys), np.int64)
        vptr = None
        if vals is not None:
            vals = np.ascontiguousarray(vals, np.int64)
            assert vals.shape[0] == n
            vptr = vals.ctypes.data
        rc = fn(self._h, xy, vptr, n, counts, sums.ctypes.data if vals is not None else None,
                int(nthreads))
        if rc < 0:
            raise MemoryError("oracle aggregate failed")
        self.threads_used = rc
        return counts[:self.n_polys], (sums[:self.n_polys] if vals is not None else None)

    def aggregate(self, xy, vals=None, nthreads: int = 0):
        """Approximate per-polygon COUNT and SUM (the GPU parity target)."""
        return self._agg(lib().orc_aggregate, xy, vals, nthreads)

    def exact(self, xy, vals=None, nthreads: int = 0):
        """Exact per-polygon COUNT and SUM by the crossing-number rule."""
        return self._agg(lib().orc_exact_join, xy, vals, nthreads)

    def invariant(self, xy, nthreads: int = 0, exhaustive: bool = False,
                  check_eps: int | None = None, half: bool | None = None) -> dict:
        """Points misclassified by the approximation ("differ"), those farther
        than the distance bound from the polygon's boundary ("far", must be 0),
        false negatives and exact inside pairs.  The bound is the build's eps
        (eps/2 for a centre-sampled approximation) unless check_eps / half
        name another one."""
        xy = np.ascontiguousarray(xy, np.int32)
        out = np.zeros(4, np.int64)
        n = xy.shape[0] // 2
        if check_eps is None and half is None:
            if exhaustive:
                lib().orc_invariant_all(self._h, xy, n, out)
            else:
                lib().orc_invariant(self._h, xy, n, out, int(nthreads))
        else:
            ce = self.eps if check_eps is None else int(check_eps)
            hf = (1 if self.centre else 0) if half is None else (1 if half else 0)
            if exhaustive:
                lib().orc_invariant_all_at(self._h, xy, n, ce, hf, out)
            else:
                lib().orc_invariant_at(self._h, xy, n, ce, hf, out, int(nthreads))
        return {"differ": int(out[0]), "far": int(out[1]), "false_neg": int(out[2]),
                "inside": int(out[3])}

    def near_boundary(self, p: int, x: int, y: int, eps: int | None = None,
                      half: bool = False) -> bool:
        """Is (x, y) within eps (default: the build's; half: eps/2) of the
        boundary of polygon p?"""
        r = lib().orc_near_boundary(self._h, int(p), int(x), int(y),
                                    self.eps if eps is None else int(eps), 1 if half else 0)
        if r < 0:
            raise ValueError("no such polygon")
        return bool(r)

    def union_box(self):
        """(i0, j0, w, h): the cell box of the union of all approximations."""
        out = np.zeros(4, np.int64)
        lib().orc_union_box(self._h, out)
        return tuple(int(v) for v in out)

    def hilbert_level(self) -> int:
        return int(lib().orc_hilbert_level(self._h))

    def hilbert_runs(self, L: int):
        """Maximal runs over [0, 4^L), key grid anchored at the union box:
        (starts uint64, run_off int64, run_ids int32)."""
        cap_r, cap_i = 1024, 1024
        while True:
            st = np.zeros(cap_r, np.uint64)
            ro = np.zeros(cap_r + 1, np.int64)
            ri = np.zeros(cap_i, np.int32)
            nr, ni = C.c_int64(0), C.c_int64(0)
            rc = lib().orc_hilbert_runs(self._h, L, st, ro, ri, cap_r, cap_i,
                                        C.byref(nr), C.byref(ni))
            if rc == 0:
                return st[:nr.value], ro[:nr.value + 1], ri[:ni.value]
            if rc < -1:
                raise ValueError("orc_hilbert_runs: level out of range")
            cap_r, cap_i = nr.value + 1, max(1, ni.value)
