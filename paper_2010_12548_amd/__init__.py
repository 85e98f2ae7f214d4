"""Python binding of libsba, the MI355X library for distance-bounded
approximate point-in-polygon aggregation (Tzirita Zacharatou et al., "The
Case for Distance-Bounded Spatial Approximations", CIDR 2021).

Argument marshalling only: every step of the build and of the probe runs in
the HIP kernels of ``libsba.so`` (sources in ``csrc/``).  PyTorch provides
device memory and streams.  There is no CPU fallback: if the library is not
built, or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

__all__ = ["Approx", "PointIndex", "SbaError", "join_pairs", "key_grid_for", "aggregate_range", "lib", "library_path", "celldiv", "hilbert", "hilbert_cell",
           "aggregate_batch", "bucket_points", "Task",
           "KIND_GRID", "KIND_HILBERT", "SEARCH_BINARY", "SEARCH_LEARNED"]

_HERE = os.path.dirname(os.path.abspath(__file__))
# SBA_LIBRARY may point at another build of the same library (e.g. a variant
# compiled with different launch parameters)
_LIB_PATH = os.environ.get("SBA_LIBRARY") or os.path.join(_HERE, "libsba.so")
_lib = None

KIND_GRID, KIND_HILBERT = 0, 1
SEARCH_BINARY, SEARCH_LEARNED = 0, 1


class SbaError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        msg = lib().sba_strerror(code).decode() if _lib is not None else str(code)
        super().__init__(f"{what}: {msg} ({code})")


class _Polys(C.Structure):
    _fields_ = [("n_polys", C.c_int32), ("ring_off", C.c_void_p), ("vert_off", C.c_void_p),
                ("xy", C.c_void_p)]


class _Opts(C.Structure):
    _fields_ = [("kind", C.c_int32), ("search", C.c_int32), ("log2_leaves", C.c_int32),
                ("tile_log2", C.c_int32), ("use_window", C.c_int32), ("win_x0", C.c_int32),
                ("win_y0", C.c_int32), ("win_x1", C.c_int32), ("win_y1", C.c_int32),
                ("sub_log2", C.c_int32), ("boundary_only", C.c_int32),
                ("key_level", C.c_int32), ("key_i0", C.c_int64), ("key_j0", C.c_int64),
                ("centre_sampled", C.c_int32), ("alloc", C.c_void_p), ("release", C.c_void_p),
                ("alloc_ctx", C.c_void_p)]


# the build's device allocator callbacks (sba_build_opts.alloc / release)
_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_RELEASE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class DeviceAllocator:
    """Device memory for builds from the caller (``sba_build_opts.alloc`` /
    ``release``).  Subclasses implement alloc(nbytes) -> device address (int,
    256-byte aligned) or 0 to refuse, and release(address).  An Approx built
    with it keeps it until the handle is freed (the handle's arrays go back
    through release in sba_free)."""

    def alloc(self, nbytes: int) -> int:
        raise NotImplementedError

    def release(self, addr: int) -> None:
        raise NotImplementedError

    def _callbacks(self):
        def a(nbytes, _ctx):
            try:
                return self.alloc(int(nbytes)) or None
            except Exception:
                return None

        def r(ptr, _ctx):
            self.release(int(ptr or 0))
        return _ALLOC_FN(a), _RELEASE_FN(r)


class TorchAllocator(DeviceAllocator):
    """Builds take their device memory from torch's caching allocator on the
    current device (so the library and torch share one pool).  Counts the
    bytes held (live_bytes) and their peak (peak_bytes, reset_peak()).
    ``fail_at`` (test support): refuse the k-th request (1-based)."""

    def __init__(self, fail_at: int = 0):
        self.fail_at = int(fail_at)
        self.requests = 0
        self.live = {}
        self.live_bytes = 0
        self.peak_bytes = 0

    def reset_peak(self):
        self.peak_bytes = self.live_bytes

    def alloc(self, nbytes: int) -> int:
        torch = _torch()
        self.requests += 1
        if self.fail_at and self.requests == self.fail_at:
            return 0
        p = torch.cuda.caching_allocator_alloc(nbytes, torch.cuda.current_device())
        self.live[p] = nbytes
        self.live_bytes += nbytes
        self.peak_bytes = max(self.peak_bytes, self.live_bytes)
        return p

    def release(self, addr: int) -> None:
        if addr in self.live:
            self.live_bytes -= self.live.pop(addr)
            _torch().cuda.caching_allocator_delete(addr)


class _PiOpts(C.Structure):
    _fields_ = [("radix_bits", C.c_int32), ("spline_err", C.c_int32)]


class _PiInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("eps", C.c_int64), ("s", C.c_int64), ("key_i0", C.c_int64),
                ("key_j0", C.c_int64), ("key_level", C.c_int32), ("has_values", C.c_int32),
                ("n_distinct", C.c_int64), ("n_knots", C.c_int64), ("radix_bits", C.c_int32),
                ("spline_err", C.c_int32), ("bytes", C.c_int64), ("build_ms", C.c_double)]


class _Task(C.Structure):
    _fields_ = [("xy", C.c_void_p), ("values", C.c_void_p), ("lo", C.c_int64), ("hi", C.c_int64),
                ("h", C.c_void_p), ("search", C.c_int32), ("vx", C.c_int32), ("vy", C.c_int32),
                ("vw", C.c_int32), ("vh", C.c_int32), ("counts", C.c_void_p),
                ("sums", C.c_void_p)]


class _Info(C.Structure):
    _fields_ = [("kind", C.c_int32), ("search", C.c_int32), ("n_polys", C.c_int32),
                ("tile_log2", C.c_int32), ("level", C.c_int32), ("log2_leaves", C.c_int32),
                ("eps", C.c_int64), ("s", C.c_int64), ("gi0", C.c_int64), ("gj0", C.c_int64),
                ("gw", C.c_int64), ("gh", C.c_int64), ("n_tiles", C.c_int64),
                ("n_blocks", C.c_int64), ("n_sets", C.c_int64), ("n_set_ids", C.c_int64),
                ("n_segments", C.c_int64), ("n_boundary", C.c_int64), ("n_runs", C.c_int64),
                ("max_leaf_err", C.c_int64), ("mean_leaf_err", C.c_double), ("bytes", C.c_int64),
                ("build_ms", C.c_double), ("n_sub", C.c_int64), ("sub_log2", C.c_int32),
                ("compact", C.c_int32), ("boundary_only", C.c_int32),
                ("centre_sampled", C.c_int32)]


def library_path() -> str:
    return _LIB_PATH


def lib():
    """Load libsba.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = C.CDLL(_LIB_PATH)
    vp, i64, i32 = C.c_void_p, C.c_int64, C.c_int32
    L.sba_build_approx.restype = C.c_int
    L.sba_build_approx.argtypes = [C.POINTER(_Polys), i64, C.POINTER(_Opts), vp, C.POINTER(vp)]
    L.sba_key_grid.restype = C.c_int
    L.sba_key_grid.argtypes = [C.POINTER(_Polys), i32, i64, vp, C.POINTER(i32), C.POINTER(i64),
                               C.POINTER(i64)]
    L.sba_aggregate.restype = C.c_int
    L.sba_aggregate.argtypes = [vp, vp, i64, vp, vp, vp, vp]
    L.sba_aggregate_search.restype = C.c_int
    L.sba_aggregate_search.argtypes = [vp, vp, i64, vp, i32, vp, vp, vp]
    L.sba_aggregate_batch.restype = C.c_int
    L.sba_aggregate_batch.argtypes = [C.POINTER(_Task), i32, vp]
    L.sba_aggregate_batch_noalloc.restype = C.c_int
    L.sba_aggregate_batch_noalloc.argtypes = [C.POINTER(_Task), i32, vp]
    L.sba_batch_scratch_bytes.restype = C.c_int64
    L.sba_batch_scratch_bytes.argtypes = [C.POINTER(_Task), i32]
    L.sba_batch_noalloc_bytes.restype = C.c_size_t
    L.sba_batch_noalloc_bytes.argtypes = []
    L.sba_bucket_points.restype = C.c_int
    L.sba_bucket_points.argtypes = [vp, vp, i64, i32, i32, i32, i32, vp, vp, vp, vp]
    L.sba_lookup_cells.restype = C.c_int
    L.sba_lookup_cells.argtypes = [vp, vp, i64, vp, vp]
    L.sba_get_sets.restype = C.c_int
    L.sba_get_sets.argtypes = [vp, C.POINTER(i64), C.POINTER(i64), vp, vp]
    L.sba_get_runs.restype = C.c_int
    L.sba_get_runs.argtypes = [vp, vp, vp, vp]
    L.sba_info.restype = C.c_int
    L.sba_info.argtypes = [vp, C.POINTER(_Info)]
    L.sba_free.restype = None
    L.sba_free.argtypes = [vp]
    L.sba_strerror.restype = C.c_char_p
    L.sba_strerror.argtypes = [C.c_int]
    L.sba_version.restype = C.c_char_p
    L.sba_version.argtypes = []
    L.sba_debug_celldiv.restype = C.c_int
    L.sba_debug_celldiv.argtypes = [i64, vp, i64, vp]
    L.sba_debug_hilbert.restype = C.c_uint64
    L.sba_debug_hilbert.argtypes = [C.c_int, C.c_uint32, C.c_uint32]
    L.sba_debug_hilbert_tab.restype = C.c_uint64
    L.sba_debug_hilbert_tab.argtypes = [C.c_int, C.c_uint32, C.c_uint32]
    L.sba_debug_hilbert_cell.restype = None
    L.sba_debug_hilbert_cell.argtypes = [C.c_int, C.c_uint64, C.POINTER(C.c_uint32),
                                         C.POINTER(C.c_uint32)]
    L.sba_probe_kernel.restype = C.c_char_p
    L.sba_probe_kernel.argtypes = [C.c_void_p, C.c_int]
    L.sba_debug_grid16_sets.restype = C.c_int
    L.sba_debug_grid16_sets.argtypes = [C.c_int]
    L.sba_debug_grid16_lsub.restype = C.c_int
    L.sba_debug_grid16_lsub.argtypes = [C.c_int]
    L.sba_debug_set_grid16_per_cu.restype = C.c_int
    L.sba_debug_set_grid16_per_cu.argtypes = [C.c_int]
    L.sba_debug_force_wide_grid.restype = C.c_int
    L.sba_debug_force_wide_grid.argtypes = [C.c_int]
    L.sba_debug_set_blocks_per_cu.restype = C.c_int
    L.sba_debug_set_blocks_per_cu.argtypes = [C.c_int]
    L.sba_pindex_build.restype = C.c_int
    L.sba_pindex_build.argtypes = [vp, vp, i64, i64, C.POINTER(_PiOpts), vp, C.POINTER(vp)]
    L.sba_pindex_info.restype = C.c_int
    L.sba_pindex_info.argtypes = [vp, C.POINTER(_PiInfo)]
    L.sba_pindex_aggregate.restype = C.c_int
    L.sba_pindex_aggregate.argtypes = [vp, vp, i32, vp, vp, vp]
    L.sba_pindex_free.restype = None
    L.sba_pindex_free.argtypes = [vp]
    L.sba_partition_scratch_bytes.restype = C.c_size_t
    L.sba_partition_scratch_bytes.argtypes = [i64, C.c_int]
    L.sba_aggregate_partitioned.restype = C.c_int
    L.sba_aggregate_partitioned.argtypes = [vp, vp, i64, vp, i32, vp, C.c_size_t, vp, vp, vp]
    L.sba_aggregate_range.restype = C.c_int
    L.sba_aggregate_range.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp, vp, vp]
    L.sba_range_kernel.restype = C.c_char_p
    L.sba_range_kernel.argtypes = [vp, vp, C.c_int]
    L.sba_join_pairs.restype = C.c_int
    L.sba_join_pairs.argtypes = [vp, vp, i64, vp, vp, vp, C.POINTER(i64), vp]
    L.sba_debug_learned_fallbacks.restype = C.c_int
    L.sba_debug_learned_fallbacks.argtypes = [vp, vp, i64, C.POINTER(i64), C.POINTER(i64), vp]
    L.sba_debug_pindex_lb.restype = C.c_int
    L.sba_debug_pindex_lb.argtypes = [vp, vp, i64, i32, vp, C.POINTER(i64), vp]
    L.sba_debug_radix_sort.restype = C.c_int
    L.sba_debug_radix_sort.argtypes = [vp, vp, i64, i32, vp]
    L.sba_debug_build_paths.restype = C.c_int
    L.sba_debug_build_paths.argtypes = [C.c_int]
    L.sba_debug_last_build_paths.restype = C.c_int
    L.sba_debug_last_build_paths.argtypes = []
    L.sba_debug_stream_read.restype = C.c_int
    L.sba_debug_stream_read.argtypes = [vp, vp, i64, i32, i32, vp, vp]
    L.sba_debug_scan_multi.restype = C.c_int
    L.sba_debug_scan_multi.argtypes = [i32, C.POINTER(vp), C.POINTER(vp), C.POINTER(i64), vp, vp]
    _lib = L
    return L


def _check(rc: int, what: str):
    if rc != 0:
        raise SbaError(rc, what)


def _torch():
    import torch
    return torch


def _stream_ptr(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _dev(t, dtype, device):
    torch = _torch()
    if isinstance(t, np.ndarray):
        t = torch.from_numpy(np.ascontiguousarray(t))
    t = t.to(device=device, dtype=dtype).contiguous()
    if t.device.type != "cuda":
        raise ValueError("libsba works on GPU tensors only")
    return t


def celldiv(s: int, n) -> np.ndarray:
    """floor(n / s) computed with the probes' multiply-shift (host copy)."""
    n = np.ascontiguousarray(n, dtype=np.uint32)
    q = np.zeros_like(n)
    _check(lib().sba_debug_celldiv(int(s), n.ctypes.data, n.shape[0], q.ctypes.data), "celldiv")
    return q


def radix_sort(keys, vals=None, bits: int = 64, stream=None):
    """Sort the int64 GPU tensor `keys` in place by its low `bits` bits, read
    as unsigned, with the build's stable radix sort; the int32 GPU tensor
    `vals` (same length) moves along.  Keys must be below 2^bits: the passes
    cover whole digits (8 bits, or 9 for small sorts where that saves a
    pass).  Test support."""
    torch = _torch()
    if keys.dtype != torch.int64 or not keys.is_cuda or not keys.is_contiguous():
        raise ValueError("keys: contiguous int64 GPU tensor")
    vp = None
    if vals is not None:
        if (vals.dtype != torch.int32 or not vals.is_cuda or not vals.is_contiguous()
                or vals.numel() != keys.numel()):
            raise ValueError("vals: contiguous int32 GPU tensor of the keys' length")
        vp = vals.data_ptr() or None
    _check(lib().sba_debug_radix_sort(keys.data_ptr() or None, vp, keys.numel(), int(bits),
                                      _stream_ptr(stream)), "radix_sort")
    return keys, vals


def stream_read(a, b=None, blocks: int = 256, threads: int = 512, out=None, stream=None):
    """Read the contiguous GPU tensor `a` and, if given, `b` (the same size in
    bytes, a multiple of 16) with the library's plain streaming-read kernel
    (`blocks` workgroups of `threads` lanes); returns the one-element int32
    GPU tensor that receives the XOR of all their 32-bit words.  Benchmark and
    test support (the read rate a kernel that only reads can reach)."""
    torch = _torch()
    nbytes = a.numel() * a.element_size()
    for t in (a, b):
        if t is not None and (not t.is_cuda or not t.is_contiguous()):
            raise ValueError("a, b: contiguous GPU tensors")
    if b is not None and b.numel() * b.element_size() != nbytes:
        raise ValueError("b: as many bytes as a")
    if out is None:
        out = torch.empty(1, dtype=torch.int32, device=a.device)
    _check(lib().sba_debug_stream_read(a.data_ptr() or None,
                                       None if b is None else (b.data_ptr() or None), nbytes,
                                       int(blocks), int(threads), out.data_ptr(),
                                       _stream_ptr(stream)), "stream_read")
    return out


def scan_multi(arrays, in_place: bool = False, stream=None):
    """Exclusive prefix sums of several int64 GPU tensors by the build's
    batched scan; returns (outputs, totals).  Test support."""
    torch = _torch()
    m = len(arrays)
    for a in arrays:
        if a.dtype != torch.int64 or not a.is_cuda or not a.is_contiguous():
            raise ValueError("arrays: contiguous int64 GPU tensors")
    outs = list(arrays) if in_place else [torch.empty_like(a) for a in arrays]
    dev = arrays[0].device if m else torch.device("cuda")
    total = torch.full((max(m, 1),), -1, dtype=torch.int64, device=dev)
    ins = (C.c_void_p * max(m, 1))(*[a.data_ptr() or None for a in arrays])
    ous = (C.c_void_p * max(m, 1))(*[o.data_ptr() or None for o in outs])
    ns = (C.c_int64 * max(m, 1))(*[a.numel() for a in arrays])
    _check(lib().sba_debug_scan_multi(m, ins, ous, ns, total.data_ptr(), _stream_ptr(stream)),
           "scan_multi")
    return outs, total[:m]


def hilbert(L: int, i: int, j: int) -> int:
    """Hilbert index of cell (i, j) as computed by the kernels (host copy)."""
    return int(lib().sba_debug_hilbert(int(L), int(i), int(j)))


def hilbert_cell(L: int, d: int):
    i, j = C.c_uint32(0), C.c_uint32(0)
    lib().sba_debug_hilbert_cell(int(L), int(d), C.byref(i), C.byref(j))
    return int(i.value), int(j.value)


class Approx:
    """Handle of the approximation of a polygon set (``sba_build_approx``).

    ring_off (int32 [P+1]), vert_off (int64 [R+1]) and xy (int32 [2V]) are the
    polygons in CSR form (torch tensors or numpy arrays; copied to the GPU).
    window: optional clip window (x0, y0, x1, y1), half-open, in coordinates.
    boundary_only: store only the boundary cells; aggregate() then returns the
    partial counts and sums beta of the result range [alpha - beta, alpha].
    key_grid: Hilbert only; a PointIndex (or its (level, i0, j0)) whose key
    grid the runs are built on, so that PointIndex.aggregate can answer them.
    centre_sampled: the non-conservative approximation (cells whose centre is
    inside the polygon; misclassified points within eps/2 of the boundary).
    """

    def __init__(self, ring_off, vert_off, xy, eps: int, kind: str = "grid",
                 search: str = "binary", log2_leaves: int = 16, tile_log2: int = 0,
                 window=None, device: str = "cuda", stream=None, sub_log2: int = 0,
                 boundary_only: bool = False, key_grid=None, centre_sampled: bool = False,
                 allocator: "DeviceAllocator | None" = None):
        torch = _torch()
        self._h = C.c_void_p(None)
        self.device = torch.device(device)
        ro = _dev(ring_off, torch.int32, self.device)
        vo = _dev(vert_off, torch.int64, self.device)
        pxy = _dev(xy, torch.int32, self.device)
        self.n_polys = int(ro.shape[0] - 1)
        polys = _Polys(self.n_polys, ro.data_ptr(), vo.data_ptr(), pxy.data_ptr())
        win = (0, 0, 0, 0, 0) if window is None else (1, *[int(v) for v in window])
        opts = _Opts({"grid": KIND_GRID, "hilbert": KIND_HILBERT}[kind],
                     {"binary": SEARCH_BINARY, "learned": SEARCH_LEARNED}[search],
                     int(log2_leaves), int(tile_log2), *win, int(sub_log2),
                     1 if boundary_only else 0, *_key_grid(key_grid),
                     1 if centre_sampled else 0)
        self._allocator = None
        if allocator is not None:
            cbs = allocator._callbacks()
            opts.alloc = C.cast(cbs[0], C.c_void_p)
            opts.release = C.cast(cbs[1], C.c_void_p)
            # kept until sba_free has given the handle's arrays back
            self._allocator = (allocator, cbs)
        h = C.c_void_p(None)
        with torch.cuda.device(self.device):
            rc = lib().sba_build_approx(C.byref(polys), int(eps), C.byref(opts),
                                        _stream_ptr(stream), C.byref(h))
        _check(rc, "sba_build_approx")
        self._h = h
        self.eps = int(eps)
        self.kind = kind
        self.search = search

    @classmethod
    def from_polygons(cls, polys, eps: int, **kw) -> "Approx":
        """polys: any object with numpy ring_off / vert_off / xy arrays."""
        return cls(polys.ring_off, polys.vert_off, polys.xy, eps, **kw)

    def close(self, sync: bool = True):
        """Free the handle.  With sync=False the caller guarantees that no
        queued GPU work still uses it (nothing is synchronised)."""
        if self._h:
            if sync:
                _torch().cuda.synchronize(self.device)
            lib().sba_free(self._h)
            self._h = C.c_void_p(None)
            self._allocator = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def probe_kernel(self, with_values: bool = True) -> str:
        """Name of the kernel aggregate() launches (as profilers list it)."""
        return lib().sba_probe_kernel(self._h, 1 if with_values else 0).decode()

    def info(self) -> dict:
        inf = _Info()
        _check(lib().sba_info(self._h, C.byref(inf)), "sba_info")
        return {k: getattr(inf, k) for k, _ in _Info._fields_}

    def aggregate(self, xy, values=None, counts=None, sums=None, search: str | None = None,
                  stream=None):
        """Per-polygon (counts, sums) as int64 GPU tensors (sums None for COUNT).

        xy: int32 GPU tensor [2n] (x, y interleaved); values: int64 [n] or None.
        Asynchronous on the current (or given) stream.
        """
        torch = _torch()
        if xy.dtype != torch.int32 or xy.device.type != "cuda" or not xy.is_contiguous():
            raise ValueError("xy must be a contiguous int32 GPU tensor")
        n = xy.numel() // 2
        if values is not None:
            if values.dtype != torch.int64 or values.numel() != n or not values.is_contiguous():
                raise ValueError("values must be a contiguous int64 GPU tensor of n entries")
        if counts is None:
            counts = torch.empty(max(self.n_polys, 1), dtype=torch.int64, device=xy.device)
        if values is not None and sums is None:
            sums = torch.empty(max(self.n_polys, 1), dtype=torch.int64, device=xy.device)
        vptr = values.data_ptr() if values is not None else None
        sptr = sums.data_ptr() if (values is not None and sums is not None) else None
        sp = _stream_ptr(stream)
        if search is None:
            rc = lib().sba_aggregate(xy.data_ptr(), vptr, n, self._h, counts.data_ptr(), sptr, sp)
        else:
            code = {"binary": SEARCH_BINARY, "learned": SEARCH_LEARNED}[search]
            rc = lib().sba_aggregate_search(xy.data_ptr(), vptr, n, self._h, code,
                                            counts.data_ptr(), sptr, sp)
        _check(rc, "sba_aggregate")
        return counts[:self.n_polys], (sums[:self.n_polys] if values is not None else None)

    def learned_fallbacks(self, xy, stream=None):
        """Test support: (fallbacks, mismatches) of the learned run search over
        the cells of the points xy (int32 GPU tensor [2n])."""
        fb, mm = C.c_int64(0), C.c_int64(0)
        _check(lib().sba_debug_learned_fallbacks(self._h, xy.data_ptr(), xy.numel() // 2,
                                                 C.byref(fb), C.byref(mm), _stream_ptr(stream)),
               "sba_debug_learned_fallbacks")
        return int(fb.value), int(mm.value)

    def aggregate_partitioned(self, xy, values=None, counts=None, sums=None,
                              search: str | None = None, scratch=None, stream=None):
        """aggregate() for points in no spatial order: points partitioned by
        coarse region first (``sba_aggregate_partitioned``).  scratch: a uint8
        GPU tensor of scratch_bytes(n) bytes, allocated here if None."""
        torch = _torch()
        n = xy.numel() // 2
        if counts is None:
            counts = torch.empty(max(self.n_polys, 1), dtype=torch.int64, device=xy.device)
        if values is not None and sums is None:
            sums = torch.empty(max(self.n_polys, 1), dtype=torch.int64, device=xy.device)
        need = int(lib().sba_partition_scratch_bytes(n, 1 if values is not None else 0))
        if scratch is None:
            scratch = torch.empty(need, dtype=torch.uint8, device=xy.device)
        code = {"binary": SEARCH_BINARY, "learned": SEARCH_LEARNED}[search or self.search]
        rc = lib().sba_aggregate_partitioned(
            xy.data_ptr(), values.data_ptr() if values is not None else None, n, self._h, code,
            scratch.data_ptr(), scratch.numel(), counts.data_ptr(),
            sums.data_ptr() if values is not None else None, _stream_ptr(stream))
        _check(rc, "sba_aggregate_partitioned")
        return counts[:self.n_polys], (sums[:self.n_polys] if values is not None else None)

    @staticmethod
    def scratch_bytes(n: int, with_values: bool = True) -> int:
        return int(lib().sba_partition_scratch_bytes(int(n), 1 if with_values else 0))

    def lookup(self, ij, stream=None):
        """Refs of cells (int64 GPU tensor [2n] of i,j): -1 none, p, or -2-set."""
        torch = _torch()
        ij = _dev(ij, torch.int64, self.device)
        n = ij.numel() // 2
        ref = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        _check(lib().sba_lookup_cells(self._h, ij.data_ptr(), n, ref.data_ptr(),
                                      _stream_ptr(stream)), "sba_lookup_cells")
        return ref[:n]

    def sets(self):
        """Multi-polygon sets: (off int64 [S+1], ids int32) numpy arrays."""
        ns, ni = C.c_int64(0), C.c_int64(0)
        _torch().cuda.synchronize(self.device)
        _check(lib().sba_get_sets(self._h, C.byref(ns), C.byref(ni), None, None), "sba_get_sets")
        off = np.zeros(ns.value + 1, np.int64)
        ids = np.zeros(max(ni.value, 1), np.int32)
        _check(lib().sba_get_sets(self._h, C.byref(ns), C.byref(ni), off.ctypes.data,
                                  ids.ctypes.data), "sba_get_sets")
        return off, ids[:ni.value]

    def runs(self, stream=None):
        """Hilbert runs: (starts as int64 tensor, refs int32 tensor) on the GPU."""
        torch = _torch()
        n = self.info()["n_runs"]
        starts = torch.empty(max(n, 1), dtype=torch.int64, device=self.device)
        ids = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        _check(lib().sba_get_runs(self._h, starts.data_ptr(), ids.data_ptr(), _stream_ptr(stream)),
               "sba_get_runs")
        return starts[:n], ids[:n]

    def decode(self, refs) -> list:
        """Turn refs into sorted polygon-id tuples."""
        off, ids = self.sets()
        out = []
        for r in np.asarray(refs).tolist():
            if r == -1:
                out.append(())
            elif r >= 0:
                out.append((r,))
            else:
                k = -2 - r
                out.append(tuple(int(v) for v in ids[off[k]:off[k + 1]]))
        return out


def key_grid_for(eps: int, *polysets, device: str = "cuda", stream=None):
    """(level, i0, j0) of the Hilbert key grid covering the cell boxes of
    every given polygon set (objects with ring_off / vert_off / xy arrays) at
    distance bound eps (``sba_key_grid``), so that handles built on it can be
    joined (join_pairs)."""
    torch = _torch()
    dev = torch.device(device)
    keep, structs = [], []
    for p in polysets:
        ro = _dev(p.ring_off, torch.int32, dev)
        vo = _dev(p.vert_off, torch.int64, dev)
        pxy = _dev(p.xy, torch.int32, dev)
        keep += [ro, vo, pxy]
        structs.append(_Polys(int(ro.shape[0] - 1), ro.data_ptr(), vo.data_ptr(), pxy.data_ptr()))
    arr = (_Polys * max(len(structs), 1))(*structs)
    level, i0, j0 = C.c_int32(0), C.c_int64(0), C.c_int64(0)
    with torch.cuda.device(dev):
        _check(lib().sba_key_grid(arr, len(structs), int(eps), _stream_ptr(stream),
                                  C.byref(level), C.byref(i0), C.byref(j0)), "sba_key_grid")
    return (int(level.value), int(i0.value), int(j0.value))


def aggregate_range(alpha: "Approx", beta: "Approx", xy, values=None, stream=None):
    """Result range in one pass (``sba_aggregate_range``): (counts, sums,
    bcounts, bsums) as int64 GPU tensors, alpha from the full handle and beta
    from the boundary-only one (sums None for COUNT).  Build beta with
    alpha.info()'s tile_log2 and sub_log2 for the one-kernel path."""
    torch = _torch()
    if xy.dtype != torch.int32 or xy.device.type != "cuda" or not xy.is_contiguous():
        raise ValueError("xy must be a contiguous int32 GPU tensor")
    n = xy.numel() // 2
    np_ = max(alpha.n_polys, 1)
    mk = lambda: torch.empty(np_, dtype=torch.int64, device=xy.device)  # noqa: E731
    counts, bcounts = mk(), mk()
    sums, bsums = (mk(), mk()) if values is not None else (None, None)
    _check(lib().sba_aggregate_range(xy.data_ptr(), values.data_ptr() if values is not None else None,
                                     n, alpha._h, beta._h, counts.data_ptr(),
                                     sums.data_ptr() if sums is not None else None,
                                     bcounts.data_ptr(),
                                     bsums.data_ptr() if bsums is not None else None,
                                     _stream_ptr(stream)), "sba_aggregate_range")
    k = alpha.n_polys
    return (counts[:k], sums[:k] if sums is not None else None, bcounts[:k],
            bsums[:k] if bsums is not None else None)


def range_kernel(alpha: "Approx", beta: "Approx", with_values: bool = True) -> str:
    return lib().sba_range_kernel(alpha._h, beta._h, 1 if with_values else 0).decode()


def join_pairs(a: "Approx", b: "Approx", stream=None):
    """Polygon pairs (p of a, q of b) whose approximations share cells, with
    the shared cell counts (``sba_join_pairs``): (pa, pb, cells) int32/int32/
    int64 GPU tensors in (p, q) order.  a and b: Hilbert handles on one key
    grid with the same eps."""
    torch = _torch()
    dev = a.device
    cap = max(1024, a.info()["n_runs"] + b.info()["n_runs"])
    n = C.c_int64(0)
    while True:
        pa = torch.empty(cap, dtype=torch.int32, device=dev)
        pb = torch.empty(cap, dtype=torch.int32, device=dev)
        cells = torch.empty(cap, dtype=torch.int64, device=dev)
        _check(lib().sba_join_pairs(a._h, b._h, cap, pa.data_ptr(), pb.data_ptr(),
                                    cells.data_ptr(), C.byref(n), _stream_ptr(stream)),
               "sba_join_pairs")
        if n.value <= cap:
            k = n.value
            return pa[:k], pb[:k], cells[:k]
        cap = n.value


def _key_grid(g):
    if g is None:
        return (0, 0, 0)
    if isinstance(g, PointIndex):
        return g.key_grid()
    level, i0, j0 = g
    return (int(level), int(i0), int(j0))


class PointIndex:
    """Point-side pre-aggregation (``sba_pindex_build``): the points' cell keys
    on the Hilbert curve, sorted, with prefix sums of the values and a
    RadixSpline over the keys.  xy: int32 GPU tensor [2n]; values: int64 [n]
    or None.  A query (aggregate) takes a Hilbert Approx built with
    key_grid=this index and the same eps."""

    def __init__(self, xy, values, eps: int, radix_bits: int = 0, spline_err: int = 0,
                 device: str = "cuda", stream=None):
        torch = _torch()
        self._ix = C.c_void_p(None)
        self.device = torch.device(device)
        xy = _dev(xy, torch.int32, self.device)
        vals = _dev(values, torch.int64, self.device) if values is not None else None
        n = xy.numel() // 2
        opts = _PiOpts(int(radix_bits), int(spline_err))
        ix = C.c_void_p(None)
        with torch.cuda.device(self.device):
            rc = lib().sba_pindex_build(xy.data_ptr(), vals.data_ptr() if vals is not None else None,
                                        n, int(eps), C.byref(opts), _stream_ptr(stream),
                                        C.byref(ix))
        _check(rc, "sba_pindex_build")
        self._ix = ix
        self.eps = int(eps)
        self.has_values = values is not None

    def info(self) -> dict:
        inf = _PiInfo()
        _check(lib().sba_pindex_info(self._ix, C.byref(inf)), "sba_pindex_info")
        return {k: getattr(inf, k) for k, _ in _PiInfo._fields_}

    def key_grid(self):
        i = self.info()
        return (i["key_level"], i["key_i0"], i["key_j0"])

    def aggregate(self, approx: "Approx", search: str = "binary", counts=None, sums=None,
                  with_values: bool | None = None, stream=None):
        """Per-polygon (counts, sums) of the indexed points over approx's
        runs, as int64 GPU tensors (sums None for COUNT)."""
        torch = _torch()
        if with_values is None:
            with_values = self.has_values
        np_ = max(approx.n_polys, 1)
        if counts is None:
            counts = torch.empty(np_, dtype=torch.int64, device=self.device)
        if with_values and sums is None:
            sums = torch.empty(np_, dtype=torch.int64, device=self.device)
        code = {"binary": SEARCH_BINARY, "learned": SEARCH_LEARNED}[search]
        rc = lib().sba_pindex_aggregate(self._ix, approx._h, code, counts.data_ptr(),
                                        sums.data_ptr() if with_values else None,
                                        _stream_ptr(stream))
        _check(rc, "sba_pindex_aggregate")
        n = approx.n_polys
        return counts[:n], (sums[:n] if with_values else None)

    def lower_bounds(self, v, search: str = "learned", stream=None):
        """Test support: (number of indexed keys below each v as an int64 GPU
        tensor, RadixSpline windows that needed the full search)."""
        torch = _torch()
        v = _dev(v, torch.int64, self.device)
        n = v.numel()
        out = torch.empty(max(n, 1), dtype=torch.int64, device=self.device)
        fb = C.c_int64(0)
        code = {"binary": SEARCH_BINARY, "learned": SEARCH_LEARNED}[search]
        _check(lib().sba_debug_pindex_lb(self._ix, v.data_ptr(), n, code, out.data_ptr(),
                                         C.byref(fb), _stream_ptr(stream)), "sba_debug_pindex_lb")
        return out[:n], int(fb.value)

    def close(self, sync: bool = True):
        if self._ix:
            if sync:
                _torch().cuda.synchronize(self.device)
            lib().sba_pindex_free(self._ix)
            self._ix = C.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Task:
    """One task of ``aggregate_batch``: points [lo, hi) of (xy, values), a
    handle, an optional viewport (vx, vy, vw, vh) and output tensors."""

    def __init__(self, approx: "Approx", xy, values=None, lo: int = 0, hi: int | None = None,
                 viewport=None, counts=None, sums=None, search: str = "binary"):
        torch = _torch()
        self.approx = approx
        self.xy = xy
        self.values = values
        n = xy.numel() // 2
        self.lo = int(lo)
        self.hi = n if hi is None else int(hi)
        self.viewport = viewport
        self.search = search
        np_ = max(approx.n_polys, 1)
        self.counts = counts if counts is not None else torch.empty(np_, dtype=torch.int64,
                                                                    device=xy.device)
        if values is not None and sums is None:
            sums = torch.empty(np_, dtype=torch.int64, device=xy.device)
        self.sums = sums

    def _c(self) -> _Task:
        vx, vy, vw, vh = self.viewport if self.viewport is not None else (0, 0, 0, 0)
        return _Task(self.xy.data_ptr(), self.values.data_ptr() if self.values is not None else None,
                     self.lo, self.hi, self.approx._h,
                     {"binary": SEARCH_BINARY, "learned": SEARCH_LEARNED}[self.search],
                     int(vx), int(vy), int(vw), int(vh), self.counts.data_ptr(),
                     self.sums.data_ptr() if self.sums is not None else None)


def aggregate_batch(tasks, stream=None, no_alloc: bool = False):
    """Run ``sba_aggregate_batch`` over a list of Task objects (asynchronous);
    no_alloc: ``sba_aggregate_batch_noalloc`` (scratch in the library's fixed
    device array, no allocation)."""
    arr = (_Task * max(len(tasks), 1))(*[t._c() for t in tasks])
    fn = lib().sba_aggregate_batch_noalloc if no_alloc else lib().sba_aggregate_batch
    _check(fn(arr, len(tasks), _stream_ptr(stream)),
           "sba_aggregate_batch_noalloc" if no_alloc else "sba_aggregate_batch")
    return tasks


def batch_scratch_bytes(tasks) -> int:
    """Device scratch bytes the batch of Task objects needs."""
    arr = (_Task * max(len(tasks), 1))(*[t._c() for t in tasks])
    return int(lib().sba_batch_scratch_bytes(arr, len(tasks)))


def batch_noalloc_bytes() -> int:
    """Size of the no-allocation batch entry point's scratch array."""
    return int(lib().sba_batch_noalloc_bytes())


def bucket_points(xy, values, x0: int, y0: int, cell: int, G: int, stream=None):
    """``sba_bucket_points``: returns (xy, values, bucket_off) GPU tensors."""
    torch = _torch()
    n = xy.numel() // 2
    oxy = torch.empty_like(xy)
    ov = torch.empty_like(values) if values is not None else None
    off = torch.empty(G * G + 1, dtype=torch.int64, device=xy.device)
    _check(lib().sba_bucket_points(xy.data_ptr(), values.data_ptr() if values is not None else None,
                                   n, int(x0), int(y0), int(cell), int(G), oxy.data_ptr(),
                                   ov.data_ptr() if ov is not None else None, off.data_ptr(),
                                   _stream_ptr(stream)), "sba_bucket_points")
    return oxy, ov, off
