"""Python binding of the MI355X pair-count library (``libcute.so``).

Argument marshalling only: every step of the counting path runs in the HIP
kernels behind the C ABI declared in ``include/cute.h``. PyTorch is used only
for device memory and streams. Importing works without a GPU; the first call
that needs the library raises if it has not been built.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcute.so")

# enums of cute.h
OK, E_INVALID_ARG, E_UNSUPPORTED, E_OUT_OF_MEMORY, E_DEVICE, E_INTERNAL = range(6)
GEOM_BOX_PERIODIC, GEOM_BOX_OPEN, GEOM_SPHERE = range(3)
BIN_MONO, BIN_RMU, BIN_SIGMAPI, BIN_THETA = range(4)
LOS_Z, LOS_MIDPOINT = range(2)
PREC_FP64, PREC_FP32_EDGE, PREC_FP32_ONLY = range(3)
EST_NATURAL, EST_LS, EST_BOX = range(3)

BATCH_GRAPH, BATCH_EAGER = range(2)

EXPORTED = ["cute_build_grid", "cute_free_grid", "cute_get_grid_info", "cute_count_pairs",
            "cute_count_pairs_noalloc",
            "cute_tune_grid", "cute_batch_create", "cute_batch_run", "cute_batch_counts", "cute_batch_layout",
            "cute_batch_stats", "cute_batch_free", "cute_count_pairs_batched", "cute_count_jackknife",
            "cute_count_jackknife_cross",
            "cute_build_pixel_map", "cute_pixel_map_read", "cute_count_radial",
            "cute_xi_estimate", "cute_xi_multipoles", "cute_fp32_decision_tables",
            "cute_fp32_zlos_constants",
            "cute_status_string", "cute_last_error"]


class CuteError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("cute status %d: %s" % (status, msg))
        self.status = status


class GridParams(ctypes.Structure):
    _fields_ = [("geom", ctypes.c_int), ("box_size", ctypes.c_double),
                ("r_max", ctypes.c_double), ("cell_size", ctypes.c_double),
                ("device_ptrs", ctypes.c_int32), ("tile_points", ctypes.c_int32)]


class CBinning(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("los", ctypes.c_int),
                ("n1", ctypes.c_int32), ("edges1", ctypes.POINTER(ctypes.c_double)),
                ("n2", ctypes.c_int32), ("edges2", ctypes.POINTER(ctypes.c_double))]


class CountStats(ctypes.Structure):
    _fields_ = [("pair_evals", ctypes.c_uint64), ("pairs_in_range", ctypes.c_uint64),
                ("retests", ctypes.c_uint64), ("flips", ctypes.c_uint64),
                ("tiles", ctypes.c_uint64), ("ms_count", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class CBatchItem(ctypes.Structure):
    _fields_ = [("a", ctypes.c_void_p), ("b", ctypes.c_void_p), ("mask_a", ctypes.c_void_p),
                ("mask_b", ctypes.c_void_p), ("masks_on_device", ctypes.c_int32),
                ("bins", ctypes.POINTER(CBinning))]


class GridInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("dims", ctypes.c_int32 * 3),
                ("cell", ctypes.c_double * 3), ("origin", ctypes.c_double * 3),
                ("ms_build", ctypes.c_double)]


_lib = None


def library_path() -> str:
    return LIB_PATH


def load():
    """Load libcute.so; raises if it has not been built (no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libcute.so is not built: run paper_1210_1833_amd/build.py "
                           "(or __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    vp, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
    lib.cute_build_grid.restype = ctypes.c_int
    lib.cute_build_grid.argtypes = [vp, vp, vp, ctypes.c_int64, ctypes.POINTER(GridParams), vp,
                                    ctypes.POINTER(vp)]
    lib.cute_free_grid.restype = None
    lib.cute_free_grid.argtypes = [vp]
    lib.cute_get_grid_info.restype = ctypes.c_int
    lib.cute_get_grid_info.argtypes = [vp, ctypes.POINTER(GridInfo)]
    lib.cute_count_pairs.restype = ctypes.c_int
    lib.cute_count_pairs.argtypes = [vp, vp, ctypes.POINTER(CBinning), ctypes.c_int, vp,
                                     ctypes.c_int32, ctypes.POINTER(CountStats), vp]
    lib.cute_count_pairs_noalloc.restype = ctypes.c_int
    lib.cute_count_pairs_noalloc.argtypes = lib.cute_count_pairs.argtypes
    lib.cute_tune_grid.restype = ctypes.c_int
    lib.cute_tune_grid.argtypes = [vp, vp, vp, ctypes.c_int64, ctypes.POINTER(GridParams),
                                   ctypes.POINTER(CBinning), ctypes.c_int, ctypes.c_int32, dp,
                                   ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), vp, dp,
                                   ctypes.POINTER(ctypes.c_int32), dp]
    ip = ctypes.POINTER(ctypes.c_int64)
    lib.cute_batch_create.restype = ctypes.c_int
    lib.cute_batch_create.argtypes = [ctypes.POINTER(CBatchItem), ctypes.c_int32, ctypes.c_int, vp,
                                      ctypes.POINTER(vp)]
    lib.cute_batch_run.restype = ctypes.c_int
    lib.cute_batch_run.argtypes = [vp, ctypes.c_int32, vp]
    lib.cute_batch_counts.restype = ctypes.c_int
    lib.cute_batch_counts.argtypes = [vp, ctypes.c_int32, vp, ctypes.c_int32, vp]
    lib.cute_batch_layout.restype = ctypes.c_int
    lib.cute_batch_layout.argtypes = [vp, ctypes.c_int32, ip, ip]
    lib.cute_batch_stats.restype = ctypes.c_int
    lib.cute_batch_stats.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(CountStats), vp]
    lib.cute_batch_free.restype = None
    lib.cute_batch_free.argtypes = [vp]
    lib.cute_count_pairs_batched.restype = ctypes.c_int
    lib.cute_count_pairs_batched.argtypes = [ctypes.POINTER(CBatchItem), ctypes.c_int32,
                                             ctypes.c_int, ctypes.POINTER(vp), ctypes.c_int32,
                                             ctypes.POINTER(CountStats), vp]
    lib.cute_count_jackknife_cross.restype = ctypes.c_int
    lib.cute_count_jackknife_cross.argtypes = [vp, vp, vp, vp, ctypes.c_int32, ctypes.c_int32,
                                               ctypes.POINTER(CBinning), ctypes.c_int, vp, vp,
                                               ctypes.POINTER(CountStats), vp]
    lib.cute_count_jackknife.restype = ctypes.c_int
    lib.cute_count_jackknife.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.POINTER(CBinning), ctypes.c_int, vp, vp,
                                         ctypes.POINTER(CountStats), vp]
    lib.cute_build_pixel_map.restype = ctypes.c_int
    lib.cute_build_pixel_map.argtypes = [vp, vp, vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.POINTER(GridParams), vp, ctypes.POINTER(vp)]
    lib.cute_pixel_map_read.restype = ctypes.c_int
    lib.cute_pixel_map_read.argtypes = [vp, vp, vp, vp]
    lib.cute_count_radial.restype = ctypes.c_int
    lib.cute_count_radial.argtypes = [vp, vp, vp, vp, ctypes.c_int32, ctypes.c_double,
                                      ctypes.c_int32, dp, vp, ctypes.c_int32,
                                      ctypes.POINTER(CountStats), vp]
    lib.cute_xi_estimate.restype = ctypes.c_int
    lib.cute_xi_estimate.argtypes = [ctypes.c_int, vp, vp, vp, ctypes.c_int64, ctypes.c_int64,
                                     ctypes.POINTER(CBinning), ctypes.c_double, dp]
    lib.cute_xi_multipoles.restype = ctypes.c_int
    lib.cute_xi_multipoles.argtypes = [dp, ctypes.POINTER(CBinning), ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_int32), dp]
    lib.cute_fp32_decision_tables.restype = ctypes.c_int
    lib.cute_fp32_decision_tables.argtypes = [ctypes.POINTER(CBinning), dp, vp, vp, vp]
    lib.cute_fp32_zlos_constants.restype = ctypes.c_int
    lib.cute_fp32_zlos_constants.argtypes = [ctypes.POINTER(CBinning), dp, vp]
    lib.cute_status_string.restype = ctypes.c_char_p
    lib.cute_status_string.argtypes = [ctypes.c_int]
    lib.cute_last_error.restype = ctypes.c_char_p
    lib.cute_last_error.argtypes = []
    _lib = lib
    return lib


def _check(rc: int):
    if rc != OK:
        lib = load()
        raise CuteError(rc, "%s (%s)" % (lib.cute_status_string(rc).decode(),
                                         lib.cute_last_error().decode()))


_torch_gpu = None


def _stream_handle(stream):
    """The HIP stream to run on: the given one, or torch's current stream."""
    global _torch_gpu
    if stream is None:
        if _torch_gpu is None:
            try:
                import torch
                _torch_gpu = torch if torch.cuda.is_available() else False
            except Exception:  # pragma: no cover - torch without ROCm
                _torch_gpu = False
        if _torch_gpu:
            return _torch_gpu.cuda.current_stream().cuda_stream
        return None
    if isinstance(stream, int):
        return stream
    return getattr(stream, "cuda_stream", stream)


@dataclass
class Binning:
    """Edges of a binning (cute_binning). edges2 is None for MONO and THETA."""
    kind: int
    edges1: np.ndarray
    edges2: np.ndarray | None = None
    los: int = LOS_Z

    def __setattr__(self, name, value):
        if name != "_c":
            object.__setattr__(self, "_c", None)  # the C struct is rebuilt on next use
        object.__setattr__(self, name, value)

    def __post_init__(self):
        self.edges1 = np.ascontiguousarray(self.edges1, dtype=np.float64)
        if self.edges2 is not None:
            self.edges2 = np.ascontiguousarray(self.edges2, dtype=np.float64)

    @property
    def shape(self):
        n1 = len(self.edges1) - 1
        return (n1,) if self.edges2 is None else (n1, len(self.edges2) - 1)

    @property
    def nbins(self):
        return int(np.prod(self.shape))

    def c(self) -> CBinning:
        """The C struct (kept: it points into edges1/edges2, which must not be
        replaced afterwards)."""
        cached = getattr(self, "_c", None)
        if cached is not None:
            return cached
        b = CBinning()
        b.kind, b.los = int(self.kind), int(self.los)
        b.n1 = len(self.edges1) - 1
        b.edges1 = self.edges1.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        if self.edges2 is None:
            b.n2 = 0
            b.edges2 = ctypes.POINTER(ctypes.c_double)()
        else:
            b.n2 = len(self.edges2) - 1
            b.edges2 = self.edges2.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        self._c = b
        return b


class Grid:
    """A cell list built on the device (cute_build_grid); freed on deletion."""

    def __init__(self, handle, n, keep=None):
        self._h = handle
        self.n = n
        self._keep = keep

    @property
    def handle(self):
        return self._h

    def info(self) -> GridInfo:
        gi = GridInfo()
        _check(load().cute_get_grid_info(self._h, ctypes.byref(gi)))
        return gi

    def close(self):
        if self._h:
            load().cute_free_grid(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _coords(pos):
    """(x, y, z, n, device_ptrs, keepalive) from torch tensors or numpy data."""
    try:
        import torch
    except Exception:  # pragma: no cover
        torch = None
    if torch is not None and isinstance(pos, torch.Tensor):
        t = pos.contiguous()
        if t.dtype != torch.float64 or t.dim() != 2 or t.shape[1] != 3:
            raise ValueError("positions must be a float64 tensor of shape (n, 3)")
        cols = [t[:, k].contiguous() for k in range(3)]
        dev = 1 if t.is_cuda else 0
        return cols[0].data_ptr(), cols[1].data_ptr(), cols[2].data_ptr(), t.shape[0], dev, cols
    if isinstance(pos, (tuple, list)) and len(pos) == 3 and torch is not None and \
            isinstance(pos[0], torch.Tensor):
        cols = [c.contiguous() for c in pos]
        if any(c.dtype != torch.float64 for c in cols):
            raise ValueError("coordinates must be float64")
        dev = 1 if cols[0].is_cuda else 0
        return cols[0].data_ptr(), cols[1].data_ptr(), cols[2].data_ptr(), cols[0].shape[0], dev, cols
    if hasattr(pos, "x") and hasattr(pos, "y") and hasattr(pos, "z"):
        cols = [np.ascontiguousarray(getattr(pos, k), dtype=np.float64) for k in "xyz"]
    else:
        a = np.asarray(pos, dtype=np.float64)
        cols = [np.ascontiguousarray(a[:, k]) for k in range(3)]
    return (cols[0].ctypes.data, cols[1].ctypes.data, cols[2].ctypes.data, len(cols[0]), 0, cols)


def build_grid(pos, geom: int, box_size: float = 0.0, r_max: float = 0.0,
               cell_size: float = 0.0, stream=None, tile_points: int = 0) -> Grid:
    """cute_build_grid. ``pos``: (n, 3) float64 numpy/torch (host or device),
    a (x, y, z) triple of tensors, or an object with x, y, z arrays."""
    lib = load()
    x, y, z, n, dev, keep = _coords(pos)
    p = GridParams(int(geom), float(box_size), float(r_max), float(cell_size), int(dev),
                   int(tile_points))
    h = ctypes.c_void_p()
    _check(lib.cute_build_grid(x, y, z, int(n), ctypes.byref(p), _stream_handle(stream),
                               ctypes.byref(h)))
    return Grid(h, int(n), keep if dev else None)


class PixelMap(Grid):
    """A pixel map (cute_build_pixel_map): one point per non-empty pixel, at
    its centre, weighted by its occupancy. Counted like a SPHERE grid, against
    another pixel map, with a THETA binning."""

    def __init__(self, handle, n, n_cth, n_phi):
        super().__init__(handle, n)
        self.n_cth, self.n_phi = n_cth, n_phi

    def read(self, stream=None):
        """(ids, counts): the non-empty pixels in ascending id order (ring *
        n_phi + sector) and their occupancies, as uint32 numpy arrays."""
        ids = np.zeros(self.n, dtype=np.uint32)
        cnt = np.zeros(self.n, dtype=np.uint32)
        _check(load().cute_pixel_map_read(self._h, ids.ctypes.data, cnt.ctypes.data,
                                          _stream_handle(stream)))
        return ids, cnt


def build_pixel_map(pos, n_cth: int, n_phi: int, r_max: float = 0.0, cell_size: float = 0.0,
                    stream=None, tile_points: int = 0) -> PixelMap:
    """cute_build_pixel_map: the pixel map of the unit vectors ``pos`` with
    ``n_cth`` rings in cos(theta) and ``n_phi`` sectors in phi, gridded for
    angular counts to ``r_max`` radians."""
    lib = load()
    x, y, z, n, dev, keep = _coords(pos)
    p = GridParams(int(GEOM_SPHERE), 0.0, float(r_max), float(cell_size), int(dev), int(tile_points))
    h = ctypes.c_void_p()
    _check(lib.cute_build_pixel_map(x, y, z, int(n), int(n_cth), int(n_phi), ctypes.byref(p),
                                    _stream_handle(stream), ctypes.byref(h)))
    g = PixelMap(h, 0, int(n_cth), int(n_phi))
    g.n = int(g.info().n)
    return g


def _values(v):
    """(pointer, on_device, keepalive) of a float64 array: a torch device
    tensor or anything numpy takes."""
    if hasattr(v, "is_cuda") and v.is_cuda:
        import torch
        t = v.to(torch.float64).contiguous()
        return t.data_ptr(), 1, t
    a = np.ascontiguousarray(v, dtype=np.float64)
    return a.ctypes.data, 0, a


def count_radial(a: Grid, ra, b: Grid | None, rb, aperture: float, edges, out=None, stream=None,
                 with_stats: bool = False):
    """cute_count_radial: pairs closer than ``aperture`` radians binned by the
    difference of their redshifts ``ra`` / ``rb`` (one per object, in each
    grid's input order; ``b is None``: autocorrelation). Returns uint64
    counts (numpy), or fills ``out`` (a torch 64-bit device tensor)."""
    lib = load()
    e = np.ascontiguousarray(edges, dtype=np.float64)
    pa, da, ka = _values(ra)
    pb, db, kb = (pa, da, ka) if b is None else _values(rb)
    if da != db:
        raise ValueError("ra and rb must both be on the host or both on the device")
    st = CountStats()
    if out is None:
        counts = np.zeros(len(e) - 1, dtype=np.uint64)
        ptr, on_dev = counts.ctypes.data, 0
    else:
        counts, ptr, on_dev = out, out.data_ptr(), 1
    _check(lib.cute_count_radial(a.handle, pa, None if b is None else b.handle, pb, da,
                                 float(aperture), len(e) - 1,
                                 e.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ptr, on_dev,
                                 ctypes.byref(st), _stream_handle(stream)))
    return (counts, st.as_dict()) if with_stats else counts


def tune_grid(pos, geom: int, binning: Binning, box_size: float = 0.0, r_max: float = 0.0,
              prec: int = PREC_FP32_EDGE, cells=None, tiles=None, stream=None):
    """cute_tune_grid: (best cell side, best tile size, {(cell, tile): ms}) for
    the autocorrelation of ``pos`` under ``binning`` (cell 0 = the library's
    density rule). Build the grid with ``cell_size`` and ``tile_points`` set
    to the returned values."""
    lib = load()
    x, y, z, n, dev, keep = _coords(pos)
    p = GridParams(int(geom), float(box_size), float(r_max), 0.0, int(dev), 0)
    cb = binning.c()
    dp = ctypes.POINTER(ctypes.c_double)
    if cells is None:
        r = binning.edges1[-1] if binning.kind == BIN_THETA else (
            float(np.hypot(binning.edges1[-1], binning.edges2[-1])) if binning.kind == BIN_SIGMAPI
            else float(binning.edges1[-1]))
        cl, ca = [0.0] + [r / k for k in (2, 3, 4, 5, 6)], None
    else:
        ca = np.ascontiguousarray(cells, dtype=np.float64)
        cl = [float(c) for c in ca]
    if tiles is None:
        tl, ta = [32, 64], None
    else:
        ta = np.ascontiguousarray(tiles, dtype=np.int32)
        tl = [int(t) for t in ta]
    ms = np.full(len(cl) * len(tl), np.nan)
    bc, bt = ctypes.c_double(), ctypes.c_int32()
    _check(lib.cute_tune_grid(x, y, z, int(n), ctypes.byref(p), ctypes.byref(cb), int(prec),
                              0 if ca is None else len(ca),
                              None if ca is None else ca.ctypes.data_as(dp),
                              0 if ta is None else len(ta),
                              None if ta is None else ta.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                              _stream_handle(stream), ctypes.byref(bc), ctypes.byref(bt),
                              ms.ctypes.data_as(dp)))
    times = {(c, t): float(ms[i * len(tl) + j]) for i, c in enumerate(cl) for j, t in enumerate(tl)}
    return bc.value, bt.value, times


def count_pairs(a: Grid, b: Grid | None, binning: Binning, prec: int = PREC_FP32_EDGE,
                out=None, stream=None, with_stats: bool = False):
    """cute_count_pairs. Returns uint64 counts shaped like the binning (numpy),
    or fills ``out`` (a torch uint64/int64 device tensor of nbins) in place."""
    lib = load()
    cb = binning.c()
    st = CountStats()
    if out is None:
        counts = np.zeros(binning.nbins, dtype=np.uint64)
        ptr, on_dev = counts.ctypes.data, 0
    else:
        counts = out
        ptr, on_dev = out.data_ptr(), 1
    rc = lib.cute_count_pairs(a.handle, None if b is None else b.handle, ctypes.byref(cb),
                              int(prec), ptr, on_dev, ctypes.byref(st), _stream_handle(stream))
    _check(rc)
    res = counts.reshape(binning.shape) if out is None else counts
    return (res, st.as_dict()) if with_stats else res


# bytes of the per-GPU scratch array of count_pairs_noalloc (cute.h)
NOALLOC_SCRATCH_BYTES = 32 << 20


def count_pairs_noalloc(a: Grid, b: Grid | None, binning: Binning, prec: int = PREC_FP32_EDGE,
                        out=None, stream=None, with_stats: bool = False):
    """cute_count_pairs_noalloc: the count of ``count_pairs`` with every
    device temporary in the library's fixed per-GPU scratch array (no device
    allocation). Same arguments and results as ``count_pairs``."""
    lib = load()
    cb = binning.c()
    st = CountStats()
    if out is None:
        counts = np.zeros(binning.nbins, dtype=np.uint64)
        ptr, on_dev = counts.ctypes.data, 0
    else:
        counts = out
        ptr, on_dev = out.data_ptr(), 1
    _check(lib.cute_count_pairs_noalloc(a.handle, None if b is None else b.handle,
                                        ctypes.byref(cb), int(prec), ptr, on_dev,
                                        ctypes.byref(st), _stream_handle(stream)))
    res = counts.reshape(binning.shape) if out is None else counts
    return (res, st.as_dict()) if with_stats else res


@dataclass
class BatchItem:
    """One item of a batched count (cute_batch_item): the pairs of grids a and
    b (None: autocorrelation of a) with no masked point. Masks are uint8 arrays
    in the grid's input order (numpy on the host or torch on the device); a
    nonzero entry leaves the point out."""
    a: Grid
    b: Grid | None
    binning: Binning
    mask_a: object = None
    mask_b: object = None


def _mask_ptr(m, n):
    if m is None:
        return None, None
    try:
        import torch
        if isinstance(m, torch.Tensor):
            t = m.contiguous()
            if t.dtype not in (torch.uint8, torch.bool) or t.numel() != n:
                raise ValueError("a mask must be uint8/bool with one entry per point")
            return t, bool(t.is_cuda)
    except ImportError:  # pragma: no cover
        pass
    a = np.ascontiguousarray(m, dtype=np.uint8)
    if a.size != n:
        raise ValueError("a mask must have one entry per point")
    return a, False


def _c_items(items):
    """ctypes array of cute_batch_item plus the objects it points into."""
    keep = []
    arr = (CBatchItem * len(items))()
    for k, it in enumerate(items):
        cb = it.binning.c()
        keep.append((it.binning, cb))
        ma, da = _mask_ptr(it.mask_a, it.a.n)
        mb, db = _mask_ptr(it.mask_b, (it.b or it.a).n)
        if ma is not None and mb is not None and da != db:
            raise ValueError("both masks of an item must be on the host or both on the device")
        on_dev = bool(da) if ma is not None else bool(db)
        keep.extend([ma, mb])

        def addr(m):
            if m is None:
                return None
            return m.data_ptr() if hasattr(m, "data_ptr") else m.ctypes.data

        arr[k] = CBatchItem(it.a.handle, None if it.b is None else it.b.handle, addr(ma), addr(mb),
                            1 if on_dev else 0, ctypes.pointer(cb))
    return arr, keep


class Batch:
    """cute_batch: many pair counts planned once, run as one graph launch."""

    def __init__(self, items, prec: int = PREC_FP32_EDGE, stream=None):
        lib = load()
        self.items = list(items)
        arr, keep = _c_items(self.items)
        h = ctypes.c_void_p()
        _check(lib.cute_batch_create(arr, len(self.items), int(prec), _stream_handle(stream),
                                     ctypes.byref(h)))
        self._h = h
        self._grids = [(it.a, it.b) for it in self.items]   # grids must outlive the batch

    def run(self, stream=None, eager: bool = False):
        _check(load().cute_batch_run(self._h, BATCH_EAGER if eager else BATCH_GRAPH,
                                     _stream_handle(stream)))

    def layout(self, item: int = -1):
        w, o = ctypes.c_int64(), ctypes.c_int64()
        _check(load().cute_batch_layout(self._h, int(item), ctypes.byref(w), ctypes.byref(o)))
        return w.value, o.value

    def counts(self, item: int = -1, out=None, stream=None):
        """Counts of item (shaped like its binning), or all items concatenated
        (item=-1), as numpy; or copied into the device tensor ``out``."""
        w, _ = self.layout(item)
        if out is not None:
            _check(load().cute_batch_counts(self._h, int(item), out.data_ptr(), 1,
                                            _stream_handle(stream)))
            return out
        c = np.zeros(w, dtype=np.uint64)
        _check(load().cute_batch_counts(self._h, int(item), c.ctypes.data, 0,
                                        _stream_handle(stream)))
        return c.reshape(self.items[item].binning.shape) if item >= 0 else c

    def stats(self, item: int = -1, stream=None):
        st = CountStats()
        _check(load().cute_batch_stats(self._h, int(item), ctypes.byref(st), _stream_handle(stream)))
        return st.as_dict()

    def close(self):
        if self._h:
            load().cute_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def count_pairs_batched(items, prec: int = PREC_FP32_EDGE, stream=None, with_stats: bool = False):
    """cute_count_pairs_batched: a list of numpy uint64 counts, one per item."""
    lib = load()
    items = list(items)
    arr, keep = _c_items(items)
    outs = [np.zeros(it.binning.nbins, dtype=np.uint64) for it in items]
    ptrs = (ctypes.c_void_p * len(items))(*[o.ctypes.data for o in outs])
    st = CountStats()
    _check(lib.cute_count_pairs_batched(arr, len(items), int(prec), ptrs, 0, ctypes.byref(st),
                                        _stream_handle(stream)))
    res = [o.reshape(it.binning.shape) for o, it in zip(outs, items)]
    return (res, st.as_dict()) if with_stats else res


def _labels(region, n):
    """(pointer, on_device, keepalive) of int32 region labels, one per point."""
    try:
        import torch
        is_t = isinstance(region, torch.Tensor)
    except ImportError:  # pragma: no cover
        is_t = False
    if is_t:
        reg = region.contiguous()
        if reg.dtype != torch.int32 or reg.numel() != n:
            raise ValueError("region must be int32 with one label per point")
        return reg.data_ptr(), int(reg.is_cuda), reg
    reg = np.ascontiguousarray(region, dtype=np.int32)
    if reg.size != n:
        raise ValueError("region must have one label per point")
    return reg.ctypes.data, 0, reg


def count_jackknife_cross(a: Grid, region_a, b: Grid, region_b, n_regions: int,
                          binning: Binning, prec: int = PREC_FP32_EDGE, stream=None,
                          with_stats: bool = False):
    """cute_count_jackknife_cross: (total, jack) with jack[k] the cross count
    of a and b, both without their region-k points. Labels as for
    count_jackknife, both on the host or both on the device."""
    lib = load()
    pa, da, ka = _labels(region_a, a.n)
    pb, db, kb = _labels(region_b, b.n)
    if da != db:
        raise ValueError("region_a and region_b must both be on the host or both on the device")
    total = np.zeros(binning.nbins, dtype=np.uint64)
    jack = np.zeros((int(n_regions), binning.nbins), dtype=np.uint64)
    st = CountStats()
    _check(lib.cute_count_jackknife_cross(a.handle, pa, b.handle, pb, da, int(n_regions),
                                          ctypes.byref(binning.c()), int(prec), total.ctypes.data,
                                          jack.ctypes.data, ctypes.byref(st), _stream_handle(stream)))
    res = (total.reshape(binning.shape), jack.reshape((int(n_regions),) + binning.shape))
    return (res + (st.as_dict(),)) if with_stats else res


def count_jackknife(grid: Grid, region, n_regions: int, binning: Binning,
                    prec: int = PREC_FP32_EDGE, stream=None, with_stats: bool = False):
    """cute_count_jackknife: (total, jack) with jack[k] the autocorrelation of
    the grid's catalog without the points of region k. ``region``: one label
    in [0, n_regions) per point, in the grid's input order (numpy int32 on
    the host or a torch int32 tensor on the device)."""
    lib = load()
    ptr, on_dev, reg = _labels(region, grid.n)
    total = np.zeros(binning.nbins, dtype=np.uint64)
    jack = np.zeros((int(n_regions), binning.nbins), dtype=np.uint64)
    st = CountStats()
    _check(lib.cute_count_jackknife(grid.handle, ptr, on_dev, int(n_regions), ctypes.byref(binning.c()),
                                    int(prec), total.ctypes.data, jack.ctypes.data, ctypes.byref(st),
                                    _stream_handle(stream)))
    res = (total.reshape(binning.shape), jack.reshape((int(n_regions),) + binning.shape))
    return (res + (st.as_dict(),)) if with_stats else res


def xi_estimate(estimator: int, dd, dr, rr, nd: int, nr: int, binning: Binning,
                box_size: float = 0.0):
    """cute_xi_estimate (host arithmetic in the library)."""
    lib = load()
    cb = binning.c()

    def u64(v):
        return None if v is None else np.ascontiguousarray(v, dtype=np.uint64).reshape(-1)

    ddd, drr, rrr = u64(dd), u64(dr), u64(rr)
    xi = np.empty(binning.nbins, dtype=np.float64)
    _check(lib.cute_xi_estimate(int(estimator), ddd.ctypes.data,
                                None if drr is None else drr.ctypes.data,
                                None if rrr is None else rrr.ctypes.data,
                                int(nd), int(nr), ctypes.byref(cb), float(box_size),
                                xi.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return xi.reshape(binning.shape)


def xi_multipoles(xi_rmu, binning: Binning, ells=(0, 2, 4)):
    """cute_xi_multipoles: xi_l(r) for even l from an RMU xi(r, mu) table."""
    lib = load()
    cb = binning.c()
    x = np.ascontiguousarray(xi_rmu, dtype=np.float64).reshape(-1)
    e = np.ascontiguousarray(ells, dtype=np.int32)
    out = np.empty((len(e), binning.shape[0]), dtype=np.float64)
    _check(lib.cute_xi_multipoles(x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  ctypes.byref(cb), len(e),
                                  e.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                  out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out


DECISION_CONSTS = ("skip32", "llg", "K1", "K0", "w_sigma_top", "w_pi_top", "w_sigma_bottom",
                   "w_pi_bottom", "low", "A0", "A1", "A2", "B0", "B1", "B2", "C2", "C0")


def fp32_decision_tables(binning: Binning, ec: float, ec64: float, el: float, el64: float):
    """cute_fp32_decision_tables (host only): the FP32 thresholds of the
    midpoint predicates for a given error model, as (band1 [n1, 2],
    band2 [n2, 2], dict of constants)."""
    lib = load()
    cb = binning.c()
    err = np.array([ec, ec64, el, el64], dtype=np.float64)
    n1, n2 = binning.shape[0], binning.shape[1] if len(binning.shape) > 1 else 0
    b1 = np.zeros((n1, 2), dtype=np.float32)
    b2 = np.zeros((max(n2, 1), 2), dtype=np.float32)
    c = np.zeros(len(DECISION_CONSTS), dtype=np.float32)
    _check(lib.cute_fp32_decision_tables(ctypes.byref(cb),
                                         err.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                         b1.ctypes.data, b2.ctypes.data, c.ctypes.data))
    return b1, b2[:n2], dict(zip(DECISION_CONSTS, c.tolist()))


ZLOS_CONSTS = ("e1a", "s1", "e2a", "s2", "rB0", "muB1", "muB0", "out_hi", "path")


def fp32_zlos_constants(binning: Binning, ec: float, ec64: float):
    """cute_fp32_zlos_constants (host only): the FP32 decision constants of
    an RMU count with the z line of sight for a given error model, as a dict
    (float32 values; "path" 2: r and mu in bin units, 3: mu only, 0 or 1:
    band tables)."""
    lib = load()
    cb = binning.c()
    err = np.array([ec, ec64], dtype=np.float64)
    c = np.zeros(len(ZLOS_CONSTS), dtype=np.float32)
    _check(lib.cute_fp32_zlos_constants(ctypes.byref(cb),
                                        err.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                        c.ctypes.data))
    return dict(zip(ZLOS_CONSTS, c.tolist()))
